"""Pins of the oracle's Lanczos bound refinement against facts fixed outside
it: the generator's published outputs, the Lanczos relation, exactness at
k = N, the residual formula, and enclosure of the spectrum."""

import numpy as np
import pytest

import oracle
from oracle import lanczos as lz
from workloads import random_orthogonal_hamiltonian, water_box_hamiltonian


def test_splitmix64_published_outputs():
    # first outputs of SplitMix64 with state 0, as published with the
    # reference implementation
    assert lz.splitmix64(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_start_vector_is_uniform_and_normalised():
    v = lz.start_vector(4096, seed=7)
    assert abs(np.linalg.norm(v) - 1.0) < 1e-14
    u = v * np.linalg.norm([(z >> 11) * 2.0 ** -53 - 0.5 for z in lz.splitmix64(7, 4096)])
    assert -0.5 <= u.min() and u.max() < 0.5
    assert abs(np.mean(u)) < 0.02 and abs(np.var(u) - 1 / 12) < 0.005


def test_lanczos_relation_and_orthonormality():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((60, 60))
    h = a + a.T
    k = 12
    alpha, beta, v = lz.lanczos(h, k, seed=1, return_vectors=True)
    vk = v[:, :k]
    t = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    lhs = h @ vk
    rhs = vk @ t + np.outer(beta[-1] * v[:, k], np.eye(k)[-1])
    assert np.max(np.abs(lhs - rhs)) < 1e-12
    assert np.max(np.abs(vk.T @ vk - np.eye(k))) < 1e-10
    # alpha_j is the Rayleigh quotient of v_j
    assert np.allclose(alpha, np.einsum("ij,ij->j", vk, h @ vk), atol=1e-12)


def test_full_krylov_space_gives_the_eigenvalues():
    d = np.linspace(-3.0, 2.0, 24) + 0.01 * np.arange(24) ** 2
    q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((24, 24)))
    h = q @ np.diag(d) @ q.T
    alpha, beta = lz.lanczos(h, 24, seed=2)
    th = np.linalg.eigvalsh(np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1))
    assert np.max(np.abs(th - np.sort(d))) < 1e-9


def test_residual_formula_matches_explicit_residual():
    h = water_box_hamiltonian(40, seed=1)
    k = 20
    alpha, beta, v = lz.lanczos(h, k, seed=0, return_vectors=True)
    t = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    th, s = np.linalg.eigh(t)
    th_lo, r_lo, th_hi, r_hi = lz.ritz_extremes(alpha, beta)
    for idx, theta, r in ((0, th_lo, r_lo), (-1, th_hi, r_hi)):
        y = v[:, :k] @ s[:, idx]
        assert theta == pytest.approx(th[idx], abs=1e-13)
        assert np.linalg.norm(h @ y - theta * y) == pytest.approx(r, rel=1e-6, abs=1e-12)


@pytest.mark.parametrize("case", ["c1", "water", "random"])
@pytest.mark.parametrize("steps", [8, 32])
def test_bounds_enclose_the_spectrum_and_tighten_gershgorin(case, steps):
    if case == "c1":
        h = random_orthogonal_hamiltonian(256, 128, seed=0)
    elif case == "water":
        h = water_box_hamiltonian(100, seed=5).astype(np.float32).astype(np.float64)
    else:
        a = np.random.default_rng(9).standard_normal((200, 200))
        h = (a + a.T) / 20.0
    w = np.linalg.eigvalsh(h)
    lo, hi = lz.lanczos_bounds(h, steps)
    g_lo, g_hi = oracle.gershgorin_bounds(h)
    assert g_lo <= lo <= w[0] and w[-1] <= hi <= g_hi
    if steps == 32:
        assert hi - lo < 0.6 * (g_hi - g_lo)


def test_full_reorthogonalisation_keeps_the_basis_orthonormal():
    # 64 steps (the most the solver takes): with one Gram-Schmidt pass the
    # basis drifts to ~1e-9 here as Ritz values converge; two passes stay
    # orthonormal to rounding
    h = random_orthogonal_hamiltonian(256, 128, seed=0)
    _, _, v = lz.lanczos(h, 64, return_vectors=True)
    assert np.abs(v.T @ v - np.eye(v.shape[1])).max() <= 1e-13


def test_exact_gershgorin_interval_is_kept():
    # diagonal H: the Gershgorin interval is the exact spectral range, so the
    # widened Ritz interval is clipped back to it exactly
    d = np.linspace(-2.0, 3.0, 200)
    h = np.diag(np.random.default_rng(2).permutation(d))
    assert lz.lanczos_bounds(h, 32) == oracle.gershgorin_bounds(h) == (-2.0, 3.0)


def test_zero_steps_is_gershgorin():
    h = water_box_hamiltonian(20, seed=2)
    assert lz.lanczos_bounds(h, 0) == oracle.gershgorin_bounds(h)


def test_tighter_bounds_need_fewer_layers_same_result():
    h = water_box_hamiltonian(100, seed=5).astype(np.float32).astype(np.float64)
    p_g, rec_g = oracle.sp2(h, 400, tol=1e-10)
    p_l, rec_l = oracle.sp2(h, 400, tol=1e-10, bounds=lz.lanczos_bounds(h, 32))
    p_ref = oracle.density_matrix_eigh(h, 400)[0]
    assert rec_l.n_iter < rec_g.n_iter
    assert np.max(np.abs(p_l - p_ref)) < 1e-8 and np.max(np.abs(p_g - p_ref)) < 1e-8


# --- HOMO/LUMO estimates from a density matrix -------------------------------

def test_projected_lanczos_is_exact_on_the_projected_subspace():
    """With k equal to the dimension of the range of Q and distinct
    eigenvalues there, the Ritz values are exactly those eigenvalues of H
    (minus the shift): the recurrence stays in the occupied (virtual)
    eigenspace of H."""
    h, q, e = random_orthogonal_hamiltonian(24, 10, seed=4, return_factors=True)
    order = np.argsort(e)
    p = q[:, order[:10]] @ q[:, order[:10]].T
    for side, idx, shift in (("occupied", order[:10], -3.0), ("virtual", order[10:], 3.0)):
        k = len(idx)
        a, b = lz.projected_lanczos(h, p, side, k + 1, shift)
        t = np.diag(a[:k]) + np.diag(b[:k - 1], 1) + np.diag(b[:k - 1], -1)
        np.testing.assert_allclose(np.linalg.eigvalsh(t), np.sort(e[idx]) - shift, atol=1e-10)
        assert abs(b[k]) < 1e-12   # one step more: the Krylov space is exhausted


@pytest.mark.parametrize("m,seed", [(32, 0), (64, 0), (32, 3)])
def test_homo_lumo_estimates_lie_inside_the_gap(m, seed):
    """The estimates bracket a sub-interval of the true HOMO-LUMO gap (the
    side the accelerated network needs) and keep most of its width."""
    h = water_box_hamiltonian(m, seed=seed)
    n_occ = 4 * m
    p, w, _ = oracle.density_matrix_eigh(h, n_occ)
    for steps in (16, 24):
        homo, lumo = lz.homo_lumo_estimates(h, p, steps)
        assert w[n_occ - 1] <= homo < lumo <= w[n_occ]
        assert lumo - homo >= 0.6 * (w[n_occ] - w[n_occ - 1])


def test_homo_lumo_estimates_c1():
    h, q, e = random_orthogonal_hamiltonian(256, 128, seed=0, return_factors=True)
    p = oracle.density_matrix_eigh(h, 128)[0]
    homo, lumo = lz.homo_lumo_estimates(h, p, 24, margin=0.0)
    assert e[:128].max() <= homo < lumo <= e[128:].min()
    assert lumo - homo >= 0.5 * (e[128:].min() - e[:128].max())


def test_homo_lumo_estimates_margin_shrinks_symmetrically():
    h = water_box_hamiltonian(32, seed=0)
    p = oracle.density_matrix_eigh(h, 128)[0]
    h0, l0 = lz.homo_lumo_estimates(h, p, 16, margin=0.0)
    h1, l1 = lz.homo_lumo_estimates(h, p, 16, margin=0.1)
    assert h1 - h0 == pytest.approx(0.1 * (l0 - h0), rel=1e-12)
    assert l0 - l1 == pytest.approx(0.1 * (l0 - h0), rel=1e-12)
