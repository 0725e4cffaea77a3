"""Seeded synthetic Hamiltonians and operands.

The paper benchmarks the density-matrix solver on SCC-DFTB Hamiltonians of
periodic water boxes with six basis orbitals per molecule (Section II.E).
Those matrices are not available here, so two seeded stand-ins are drawn:

* ``random_orthogonal_hamiltonian``: ``H = Q diag(e) Q^T`` with a Haar-like
  orthogonal ``Q`` and a chosen, gapped spectrum ``e``.  The exact density
  matrix is known by construction (``Q_occ Q_occ^T``).
* ``water_box_hamiltonian``: a minimal tight-binding model of liquid water
  (O s, px, py, pz and one s orbital per H) at 1 g/cm^3 with random molecular
  orientations, an exponential, angle-free hopping and a 6 Angstrom cutoff.
  It has the size, sparsity profile and spectral gap structure of the paper's
  water workloads.

All random numbers come from ``numpy.random.default_rng(seed)``.  Nothing in
this module computes a density matrix.
"""

from __future__ import annotations

import math

import numpy as np

AVOGADRO = 6.02214076e23
WATER_MOLAR_MASS = 18.015  # g/mol
OH_BOND = 0.96  # Angstrom
HOH_ANGLE_DEG = 104.5
MIN_OO_DISTANCE = 2.5  # Angstrom, random sequential addition exclusion radius
HOPPING_DECAY = 1.0  # Angstrom
HOPPING_CUTOFF = 6.0  # Angstrom

# On-site energies per molecule in orbital order: O s, O px, O py, O pz, H1 s, H2 s.
WATER_ONSITE = np.array([-1.0, -0.5, -0.5, -0.5, -0.3, -0.3])
# Atom index (within the molecule: 0 = O, 1 = H1, 2 = H2) of each orbital.
_ORBITAL_ATOM = np.array([0, 0, 0, 0, 1, 2])


def random_orthogonal_hamiltonian(n, n_occ, occ_range=(-2.0, -0.5), virt_range=(0.5, 2.0),
                                  seed=0, return_factors=False):
    """``H = Q diag(e) Q^T`` with ``Q`` from the QR factorisation of a seeded
    standard-normal ``n x n`` matrix (columns sign-fixed by ``diag(R)``).

    ``e`` holds ``n_occ`` occupied levels drawn uniformly from ``occ_range``
    followed by ``n - n_occ`` virtual levels uniform in ``virt_range``; they
    are drawn after the normal matrix.  ``H`` is returned in FP64 and exactly
    symmetric.  With ``return_factors`` the tuple ``(H, Q, e)`` is returned.
    """
    if not 0 <= n_occ <= n:
        raise ValueError("n_occ must lie in [0, n]")
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    e = np.concatenate([rng.uniform(occ_range[0], occ_range[1], n_occ),
                        rng.uniform(virt_range[0], virt_range[1], n - n_occ)])
    h = (q * e[None, :]) @ q.T
    h = 0.5 * (h + h.T)
    if return_factors:
        return h, q, e
    return h


def water_box_length(n_molecules, density_g_cm3=1.0):
    """Edge (Angstrom) of the cube that holds ``n_molecules`` waters at the
    given mass density (29.915 cubic Angstrom per molecule at 1 g/cm^3)."""
    volume_cm3 = n_molecules * WATER_MOLAR_MASS / AVOGADRO / density_g_cm3
    return (volume_cm3 * 1e24) ** (1.0 / 3.0)


def _min_image(d, box):
    return d - box * np.round(d / box)


def _random_rotations(rng, count):
    """Uniform random rotation matrices from normalised N(0,1)^4 quaternions."""
    q = rng.standard_normal((count, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    rot = np.empty((count, 3, 3))
    rot[:, 0, 0] = 1 - 2 * (y * y + z * z)
    rot[:, 0, 1] = 2 * (x * y - z * w)
    rot[:, 0, 2] = 2 * (x * z + y * w)
    rot[:, 1, 0] = 2 * (x * y + z * w)
    rot[:, 1, 1] = 1 - 2 * (x * x + z * z)
    rot[:, 1, 2] = 2 * (y * z - x * w)
    rot[:, 2, 0] = 2 * (x * z - y * w)
    rot[:, 2, 1] = 2 * (y * z + x * w)
    rot[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return rot


def water_box_positions(n_molecules, seed=0, density_g_cm3=1.0, max_attempts=10_000_000):
    """Atom positions (``3M x 3``, Angstrom, order O, H1, H2 per molecule) and
    the box edge.  O centres are placed by random sequential addition with a
    minimum-image O-O distance of at least 2.5 Angstrom; each molecule (O-H
    0.96 Angstrom, H-O-H 104.5 degrees) gets a uniformly random orientation."""
    rng = np.random.default_rng(seed)
    box = water_box_length(n_molecules, density_g_cm3)
    centres = np.empty((n_molecules, 3))
    placed = 0
    attempts = 0
    min_d2 = MIN_OO_DISTANCE ** 2
    while placed < n_molecules:
        cand = rng.uniform(0.0, box, size=3)
        attempts += 1
        if attempts > max_attempts:
            raise RuntimeError("random sequential addition did not place all molecules")
        if placed:
            d = _min_image(centres[:placed] - cand[None, :], box)
            if np.min(np.einsum("ij,ij->i", d, d)) < min_d2:
                continue
        centres[placed] = cand
        placed += 1
    half = math.radians(HOH_ANGLE_DEG) / 2.0
    local = np.array([[0.0, 0.0, 0.0],
                      [OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)],
                      [-OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)]])
    rot = _random_rotations(rng, n_molecules)
    atoms = centres[:, None, :] + np.einsum("mij,aj->mai", rot, local)
    return atoms.reshape(3 * n_molecules, 3), box


def water_box_hamiltonian(n_molecules, seed=0, n_pad=None, dtype=np.float64,
                          density_g_cm3=1.0, block_diagonal=False, return_geometry=False):
    """Dense tight-binding Hamiltonian of a periodic water box.

    Six orbitals per molecule (O s, px, py, pz; H1 s; H2 s) with the on-site
    energies in ``WATER_ONSITE``.  Every pair of orbitals on two different
    atoms whose minimum-image distance ``r`` is below 6 Angstrom couples with
    ``-exp(-r / 1 Angstrom)``, independent of orbital type and direction;
    orbitals on the same atom do not couple.  ``block_diagonal=True`` keeps
    only intramolecular hopping.  The matrix is zero-padded to ``n_pad`` if
    given (padding rows and columns are all zero).
    """
    atoms, box = water_box_positions(n_molecules, seed, density_g_cm3)
    n_atoms = atoms.shape[0]
    n = 6 * n_molecules
    n_out = n if n_pad is None else int(n_pad)
    if n_out < n:
        raise ValueError("n_pad is smaller than 6 * n_molecules")
    atom_of = (3 * np.arange(n_molecules)[:, None] + _ORBITAL_ATOM[None, :]).reshape(-1)
    mol_of_atom = np.arange(n_atoms) // 3
    h = np.zeros((n_out, n_out), dtype=dtype)
    chunk = 1024
    # Orbital rows grouped by atom chunk keep the distance matrix small.
    for a0 in range(0, n_atoms, chunk):
        a1 = min(a0 + chunk, n_atoms)
        d = _min_image(atoms[a0:a1, None, :] - atoms[None, :, :], box)
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        hop = np.where(r < HOPPING_CUTOFF, -np.exp(-r / HOPPING_DECAY), 0.0)
        idx = np.arange(a0, a1)
        hop[idx - a0, idx] = 0.0  # no same-atom coupling
        if block_diagonal:
            hop[mol_of_atom[a0:a1, None] != mol_of_atom[None, :]] = 0.0
        rows = np.nonzero((atom_of >= a0) & (atom_of < a1))[0]
        h[rows[:, None], np.arange(n)[None, :]] = hop[atom_of[rows] - a0][:, atom_of].astype(dtype)
    diag = np.tile(WATER_ONSITE, n_molecules).astype(dtype)
    h[np.arange(n), np.arange(n)] = diag
    if return_geometry:
        return h, atoms, box
    return h


def symmetric_normal(n, seed, std=1.0, n_real=None, dtype=np.float64):
    """Symmetric ``n x n`` matrix whose upper triangle (diagonal included) is
    iid ``N(0, std^2)`` and whose lower triangle mirrors it.  Rows and
    columns at or beyond ``n_real`` are zero (padding)."""
    m = n if n_real is None else int(n_real)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, m)) * std
    up = np.triu(a)
    s = up + np.triu(up, 1).T
    out = np.zeros((n, n), dtype=dtype)
    out[:m, :m] = s
    return out


def trajectory_perturbation(n, seed, n_real=None, dtype=np.float64):
    """``H_p = (A + A^T) / (2 sqrt(2 m))`` with ``A`` iid ``N(0,1)`` of size
    ``m = n_real``, so that its spectral norm is about 1; zero on padding."""
    m = n if n_real is None else int(n_real)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, m))
    out = np.zeros((n, n), dtype=dtype)
    out[:m, :m] = (a + a.T) / (2.0 * math.sqrt(2.0 * m))
    return out


def trajectory_hamiltonian(h0, hp, t, amplitude=0.01, omega=0.1):
    """``H(t) = H0 + amplitude * sin(omega * t) * H_p``."""
    return h0 + (amplitude * math.sin(omega * t)) * hp


def pad_matrix(h, n_pad):
    """Zero-pad a square matrix to ``n_pad x n_pad``."""
    n = h.shape[0]
    if n_pad < n:
        raise ValueError("n_pad is smaller than the matrix")
    out = np.zeros((n_pad, n_pad), dtype=h.dtype)
    out[:n, :n] = h
    return out
