"""Seeded synthetic charge model for the XL-BOMD kernel (Section III).

The paper propagates net Mulliken charges ``n`` (one per atom) of an
SCC-DFTB model; its Hamiltonian depends on them through a charge-coupling
matrix.  Those models are not available here, so the water box of
``hamiltonians.water_box_hamiltonian`` gets a minimal stand-in:

* atoms O, H1, H2 per molecule own the orbitals (O s, px, py, pz), (H1 s),
  (H2 s); valence charges ``Z`` are 6, 1, 1 (eight electrons, four doubly
  occupied states per molecule, so the neutral box has ``n_occ = 4 M``);
* the coupling ``gamma`` is a screened Coulomb form: ``U_I`` on the diagonal
  (0.5 for O, 0.4 for H) and ``kappa / sqrt(r^2 + a^2)`` (``kappa`` 0.3,
  ``a`` 1 Angstrom) between atoms closer than 6 Angstrom (minimum image);
* the charge-dependent Hamiltonian shifts every orbital of atom ``I`` by
  ``(gamma n)_I``: ``H(n) = H0 + diag(B gamma n)`` with ``B`` the orbital-to-
  atom incidence.

Orbitals of one atom are contiguous, given as ``atom_ptr`` (atom ``I`` owns
orbitals ``atom_ptr[I] .. atom_ptr[I+1]-1``); padding orbitals belong to no
atom.  Nothing here computes a density matrix or a response.
"""

from __future__ import annotations

import numpy as np

from .hamiltonians import _min_image, water_box_hamiltonian

WATER_VALENCE = np.array([6.0, 1.0, 1.0])      # O, H1, H2
WATER_HUBBARD = np.array([0.5, 0.4, 0.4])
COULOMB_KAPPA = 0.3
COULOMB_SCREEN = 1.0   # Angstrom
COULOMB_CUTOFF = 6.0   # Angstrom


def water_charge_model(n_molecules, seed=0, n_pad=None, kappa=COULOMB_KAPPA,
                       screen=COULOMB_SCREEN, cutoff=COULOMB_CUTOFF):
    """The water box Hamiltonian ``h0`` (FP64, padded to ``n_pad``) with its
    charge model: ``atom_ptr`` (int64, ``3M + 1``), valence charges ``z``
    and the ``3M x 3M`` coupling ``gamma`` (FP64, symmetric)."""
    h0, atoms, box = water_box_hamiltonian(n_molecules, seed=seed, n_pad=n_pad,
                                           return_geometry=True)
    n_atoms = atoms.shape[0]
    per_atom = np.tile(np.array([4, 1, 1]), n_molecules)
    atom_ptr = np.concatenate([[0], np.cumsum(per_atom)]).astype(np.int64)
    z = np.tile(WATER_VALENCE, n_molecules)
    gamma = np.empty((n_atoms, n_atoms))
    chunk = 1024
    for a0 in range(0, n_atoms, chunk):
        a1 = min(a0 + chunk, n_atoms)
        d = _min_image(atoms[a0:a1, None, :] - atoms[None, :, :], box)
        r2 = np.einsum("ijk,ijk->ij", d, d)
        gamma[a0:a1] = np.where(r2 < cutoff * cutoff, kappa / np.sqrt(r2 + screen * screen), 0.0)
    gamma[np.arange(n_atoms), np.arange(n_atoms)] = np.tile(WATER_HUBBARD, n_molecules)
    return {"h0": h0, "atom_ptr": atom_ptr, "z": z, "gamma": gamma, "atoms": atoms,
            "box": box, "n_occ": 4 * n_molecules}


def random_charges(n_atoms, seed, scale=0.05):
    """Seeded net charges ``scale * N(0,1)`` shifted to sum to zero."""
    q = np.random.default_rng(seed).standard_normal(n_atoms) * scale
    return q - q.mean()


def charge_shifted_hamiltonian(h0, atom_ptr, gamma, charges):
    """``H(n) = H0 + diag(B gamma n)``: each orbital of atom ``I`` is shifted
    by ``(gamma n)_I``.  Padding orbitals are not shifted."""
    shift = np.asarray(gamma) @ np.asarray(charges, dtype=np.float64)
    h = np.array(h0, dtype=np.float64, copy=True)
    ptr = np.asarray(atom_ptr)
    counts = np.diff(ptr)
    orb = np.arange(ptr[0], ptr[-1])
    h[orb, orb] += np.repeat(shift, counts)
    return h
