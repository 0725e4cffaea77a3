"""XL-BOMD kernel building block -- TEST INFRASTRUCTURE ONLY.

Section III propagates net Mulliken charges ``n`` and drives them towards
the ground-state charges ``q0[n]`` through the kernel ``K = J^-1``, with
``J`` the Jacobian of ``f(n) = q0[n] - n`` (Eq. 27-28); the action
``K f`` is to be approximated in a preconditioned Krylov subspace.  This
module is the plain FP64 reference of that building block on the synthetic
charge model of ``workloads.charges``:

* ``mulliken_charges``: ``q_I = Z_I - 2 sum_{mu in I} P_mu,mu`` (orthogonal
  basis, doubly occupied states);
* ``charge_response``: ``dq0/dn v = -2 B^T diag(P1)`` with ``P1`` the
  density-matrix response to ``H1 = diag(B gamma v)`` (any JVP of ``P``);
* ``jacobian``: ``J = dq0/dn - I`` column by column;
* ``krylov_kernel``: with a preconditioner ``K0`` (``-I`` by default), the
  Krylov basis ``v_1 = K0 f / ||K0 f||``, ``v_{k+1}`` = ``K0 J v_k``
  orthonormalised against ``v_1 .. v_k``; then ``K f ~ V c`` with ``c``
  minimising ``||K0 J V c - K0 f||`` (the preconditioned minimal-residual,
  i.e. GMRES, form of the Krylov approximation).

Pins (tests/test_oracle_xlbomd.py): at full rank the approximation equals
``J^{-1} f`` from a dense solve; with ``K0 = J^{-1}`` rank 1 is exact; the
minimal residual never grows with the rank; on a diagonal ``J`` the basis
terminates after as many vectors as distinct eigenvalues; the response
columns agree with central finite differences of ``q0`` and conserve the
total charge; Mulliken charges of the block-diagonal water box match
per-molecule 6x6 diagonalisations and sum to zero.
"""

from __future__ import annotations

import numpy as np

from .sp2_oracle import density_matrix_eigh, dmpt_response


def mulliken_charges(p, atom_ptr, z):
    """Net charges ``Z_I - 2 sum_{mu in I} P_mu,mu`` (atom ``I`` owns the
    orbitals ``atom_ptr[I] .. atom_ptr[I+1]-1``)."""
    d = np.diag(np.asarray(p, dtype=np.float64))
    ptr = np.asarray(atom_ptr)
    pop = np.array([d[ptr[i]:ptr[i + 1]].sum() for i in range(ptr.size - 1)])
    return np.asarray(z, dtype=np.float64) - 2.0 * pop


def potential_direction(n, atom_ptr, gamma, v):
    """``H1 = diag(B gamma v)`` (n x n): the derivative of ``H(n)`` in the
    charge direction ``v``."""
    shift = np.asarray(gamma, dtype=np.float64) @ np.asarray(v, dtype=np.float64)
    ptr = np.asarray(atom_ptr)
    d = np.zeros(n)
    for i in range(ptr.size - 1):
        d[ptr[i]:ptr[i + 1]] = shift[i]
    return np.diag(d)


def charge_response(n, atom_ptr, gamma, v, jvp):
    """``dq0/dn v = -2 B^T diag(P1)`` with ``P1 = jvp(H1)`` the density-matrix
    response to ``H1 = diag(B gamma v)``."""
    p1 = jvp(potential_direction(n, atom_ptr, gamma, v))
    ptr = np.asarray(atom_ptr)
    d = np.diag(p1)
    return np.array([-2.0 * d[ptr[i]:ptr[i + 1]].sum() for i in range(ptr.size - 1)])


def dmpt_jvp(h, n_occ):
    """JVP of the exact ``theta(mu I - H)`` at ``h`` (first-order density-matrix
    perturbation theory, one eigendecomposition reused)."""
    eig = np.linalg.eigh(np.asarray(h, dtype=np.float64))
    return lambda h1: dmpt_response(h, n_occ, h1, eig=eig)


def jacobian(n, atom_ptr, gamma, jvp):
    """``J = dq0/dn - I``, one response per column."""
    na = np.asarray(atom_ptr).size - 1
    j = np.empty((na, na))
    for c in range(na):
        e = np.zeros(na)
        e[c] = 1.0
        j[:, c] = charge_response(n, atom_ptr, gamma, e, jvp) - e
    return j


def residual(h0, n_occ, atom_ptr, z, gamma, charges, shifted_hamiltonian):
    """``f(n) = q0[n] - n`` with ``q0`` the Mulliken charges of the exact density
    of ``H(n) = shifted_hamiltonian(h0, atom_ptr, gamma, n)``."""
    h = shifted_hamiltonian(h0, atom_ptr, gamma, charges)
    p = density_matrix_eigh(h, n_occ)[0]
    return mulliken_charges(p, atom_ptr, z) - np.asarray(charges, dtype=np.float64)


def krylov_kernel(f, apply_j, rank, k0=None, breakdown=1e-12):
    """Rank-``rank`` Krylov approximation of ``K f = J^{-1} f``.  ``apply_j(v)``
    returns ``J v``; ``k0`` is the preconditioner (``-I`` if None).  Returns
    ``(kf, rho, V)``: the approximation, the minimal residuals
    ``rho[k] = min_c ||K0 J V_k c - K0 f||`` for ``k = 0 .. m`` (``rho[0] =
    ||K0 f||``) and the orthonormal basis ``V`` (``N_a x m``).  The basis
    stops early when a new direction vanishes (``||w|| <= breakdown *
    ||K0 J v_k||``): the subspace is then invariant and the result exact."""
    f = np.asarray(f, dtype=np.float64)
    pre = (lambda x: -x) if k0 is None else (lambda x: np.asarray(k0) @ x)
    r0 = pre(f)
    beta0 = float(np.linalg.norm(r0))
    if beta0 == 0.0:
        return np.zeros_like(f), np.zeros(1), np.zeros((f.size, 0))
    vs = [r0 / beta0]
    fs = []
    for k in range(rank):
        fk = pre(apply_j(vs[k]))
        fs.append(fk)
        if k + 1 == rank:
            break
        basis = np.array(vs).T
        w = fk - basis @ (basis.T @ fk)
        w = w - basis @ (basis.T @ w)
        b = float(np.linalg.norm(w))
        if not b > breakdown * float(np.linalg.norm(fk)):
            break
        vs.append(w / b)
    m = len(fs)
    vmat = np.array(vs[:m]).T
    fmat = np.array(fs).T
    rho = [beta0]
    c = None
    for k in range(1, m + 1):
        c, *_ = np.linalg.lstsq(fmat[:, :k], r0, rcond=None)
        rho.append(float(np.linalg.norm(fmat[:, :k] @ c - r0)))
    return vmat @ c, np.array(rho), vmat
