"""Pins of the XL-BOMD kernel oracle (oracle/xlbomd.py) against results that
do not come from the oracle itself: brute-force Mulliken sums, central finite
differences of the ground-state charges, dense linear solves and the
definition of the minimal-residual Krylov approximation over an explicitly
built power basis."""

import numpy as np
import pytest

import oracle
from oracle import xlbomd
from workloads import charge_shifted_hamiltonian, random_charges, water_charge_model


def _model(m=4, seed=0):
    mod = water_charge_model(m, seed=seed)
    charges = random_charges(3 * m, seed=5)
    h = charge_shifted_hamiltonian(mod["h0"], mod["atom_ptr"], mod["gamma"], charges)
    return mod, charges, h


def test_mulliken_brute_force():
    p = np.array([[0.5, 0.1, 0.0], [0.1, 1.0, 0.2], [0.0, 0.2, 0.25]])
    q = xlbomd.mulliken_charges(p, [0, 2, 3], [3.0, 1.0])
    assert q == pytest.approx([3.0 - 2.0 * 1.5, 1.0 - 2.0 * 0.25], abs=0)


def test_neutral_box_and_molecule_blocks():
    # no intermolecular hopping: every molecule is its own 6x6 problem with
    # four doubly occupied states at n_occ = 4M
    mod = water_charge_model(3, seed=1)
    from workloads import water_box_hamiltonian
    h = water_box_hamiltonian(3, seed=1, block_diagonal=True)
    p = oracle.density_matrix_eigh(h, mod["n_occ"])[0]
    q = xlbomd.mulliken_charges(p, mod["atom_ptr"], mod["z"])
    for m in range(3):
        blk = h[6 * m:6 * m + 6, 6 * m:6 * m + 6]
        w, v = np.linalg.eigh(blk)
        pm = v[:, :4] @ v[:, :4].T
        qm = np.array([6.0 - 2.0 * np.trace(pm[:4, :4]), 1.0 - 2.0 * pm[4, 4], 1.0 - 2.0 * pm[5, 5]])
        assert q[3 * m:3 * m + 3] == pytest.approx(qm, abs=1e-12)
    assert abs(q.sum()) < 1e-12


def test_response_matches_finite_differences():
    mod, charges, h = _model()
    n = h.shape[0]
    v = np.random.default_rng(3).standard_normal(charges.size)
    jvp = xlbomd.dmpt_jvp(h, mod["n_occ"])
    dq = xlbomd.charge_response(n, mod["atom_ptr"], mod["gamma"], v, jvp)
    step = 1e-5

    def q0(c):
        hh = charge_shifted_hamiltonian(mod["h0"], mod["atom_ptr"], mod["gamma"], c)
        p = oracle.density_matrix_eigh(hh, mod["n_occ"])[0]
        return xlbomd.mulliken_charges(p, mod["atom_ptr"], mod["z"])

    fd = (q0(charges + step * v) - q0(charges - step * v)) / (2 * step)
    assert np.abs(dq - fd).max() <= 1e-7 * np.abs(fd).max()
    # the response moves charge between atoms but never creates any
    assert abs(dq.sum()) <= 1e-12 * np.abs(dq).max()


def test_jacobian_is_the_derivative_of_the_residual():
    # J = d f / d n for f(n) = q0[n] - n, against central differences of f
    mod, charges, h = _model()
    n = h.shape[0]
    jmat = xlbomd.jacobian(n, mod["atom_ptr"], mod["gamma"], xlbomd.dmpt_jvp(h, mod["n_occ"]))
    v = np.random.default_rng(12).standard_normal(charges.size)
    step = 1e-5

    def f(c):
        return xlbomd.residual(mod["h0"], mod["n_occ"], mod["atom_ptr"], mod["z"], mod["gamma"], c,
                               charge_shifted_hamiltonian)

    fd = (f(charges + step * v) - f(charges - step * v)) / (2 * step)
    assert np.abs(jmat @ v - fd).max() <= 1e-7 * np.abs(fd).max()


def test_full_rank_equals_dense_solve():
    mod, charges, h = _model()
    n = h.shape[0]
    jvp = xlbomd.dmpt_jvp(h, mod["n_occ"])
    jmat = xlbomd.jacobian(n, mod["atom_ptr"], mod["gamma"], jvp)
    f = xlbomd.residual(mod["h0"], mod["n_occ"], mod["atom_ptr"], mod["z"], mod["gamma"], charges,
                        charge_shifted_hamiltonian)
    exact = np.linalg.solve(jmat, f)
    kf, rho, vmat = xlbomd.krylov_kernel(f, lambda x: jmat @ x, rank=f.size)
    assert np.linalg.norm(kf - exact) <= 1e-9 * np.linalg.norm(exact)
    assert rho[-1] <= 1e-9 * rho[0]
    assert np.allclose(vmat.T @ vmat, np.eye(vmat.shape[1]), atol=1e-10)
    # the residual of a minimal-residual method never grows with the rank
    assert np.all(np.diff(rho) <= 1e-12 * rho[0])


def test_exact_preconditioner_needs_rank_one():
    mod, charges, h = _model()
    n = h.shape[0]
    jmat = xlbomd.jacobian(n, mod["atom_ptr"], mod["gamma"], xlbomd.dmpt_jvp(h, mod["n_occ"]))
    f = np.random.default_rng(7).standard_normal(charges.size)
    kf, rho, _ = xlbomd.krylov_kernel(f, lambda x: jmat @ x, rank=1, k0=np.linalg.inv(jmat))
    assert np.linalg.norm(kf - np.linalg.solve(jmat, f)) <= 1e-10 * np.linalg.norm(kf)
    assert rho[1] <= 1e-10 * rho[0]


def test_diagonal_jacobian_terminates():
    d = np.repeat([-0.5, -1.0, -2.0], 5)
    f = np.random.default_rng(2).standard_normal(d.size)
    kf, rho, vmat = xlbomd.krylov_kernel(f, lambda x: d * x, rank=10)
    assert vmat.shape[1] == 3          # three distinct eigenvalues
    assert np.allclose(kf, f / d, rtol=1e-10)


def test_matches_power_basis_minimisation():
    # the same subspace built from explicit powers (K0 J)^k K0 f, minimised
    # by a least-squares solve in that basis
    rng = np.random.default_rng(4)
    a = rng.standard_normal((12, 12))
    jmat = -np.eye(12) + 0.3 * a
    f = rng.standard_normal(12)
    k0 = np.diag(rng.uniform(-1.5, -0.5, 12))
    for rank in (1, 2, 4):
        kf, rho, _ = xlbomd.krylov_kernel(f, lambda x: jmat @ x, rank=rank, k0=k0)
        r0 = k0 @ f
        powers = [r0]
        for _ in range(rank - 1):
            powers.append(k0 @ jmat @ powers[-1])
        pb = np.array(powers).T
        c, *_ = np.linalg.lstsq(k0 @ jmat @ pb, r0, rcond=None)
        ref = pb @ c
        assert np.linalg.norm(kf - ref) <= 1e-9 * np.linalg.norm(ref)
        assert rho[-1] == pytest.approx(np.linalg.norm(k0 @ jmat @ ref - r0), rel=1e-8, abs=1e-13)
