"""Pins of the accelerated DNN-SP2 oracle (oracle/accelerated.py) and of the
layer-coefficient form of the derivative oracle, against what mathematics
fixes independently of the code: the diagonalisation, the spectral theorem
(scalar recursion on the eigenvalues), the defining values of each layer
polynomial, closed forms, perturbation theory and finite differences."""

import numpy as np
import pytest

import oracle
from oracle import accelerated as acc
from workloads import random_orthogonal_hamiltonian, symmetric_normal, water_box_hamiltonian


def _poly(coef, x):
    a, b, c = coef
    return a * x * x + b * x + c


@pytest.mark.parametrize("shift", [0.0, 0.05, 0.2, 0.37, 0.5])
def test_layer_polynomials_have_their_defining_values(shift):
    """p+(x) = ((x - s)/(1 - s))^2 vanishes with zero slope at s and is 1 at
    1; p-(x) = 1 - p+(1 - x) is 1 with zero slope at 1 - s and 0 at 0."""
    a, b, c = acc.layer_polynomial(1, shift)
    assert abs(_poly((a, b, c), shift)) < 1e-15
    assert _poly((a, b, c), 1.0) == pytest.approx(1.0, abs=1e-15)
    assert abs(2 * a * shift + b) < 1e-14
    assert a > 0
    a, b, c = acc.layer_polynomial(-1, shift)
    assert _poly((a, b, c), 1.0 - shift) == pytest.approx(1.0, abs=1e-15)
    assert abs(_poly((a, b, c), 0.0)) < 1e-15
    assert abs(2 * a * (1.0 - shift) + b) < 1e-14
    assert a < 0
    # s = 0: the plain SP2 layers x^2 and 2x - x^2
    if shift == 0.0:
        assert acc.layer_polynomial(1, 0.0) == (1.0, 0.0, 0.0)
        assert acc.layer_polynomial(-1, 0.0) == (-1.0, 2.0, 0.0)


def test_every_layer_maps_the_unit_interval_into_itself():
    x = np.linspace(0.0, 1.0, 2001)
    for shift in np.linspace(0.0, 0.5, 51):
        for sign in (1, -1):
            y = _poly(acc.layer_polynomial(sign, shift), x)
            assert y.min() >= -1e-14 and y.max() <= 1.0 + 1e-14


@pytest.mark.parametrize("l,h", [(0.157, 0.212), (0.4989, 0.5011), (0.1, 0.9), (0.7, 0.95),
                                 (0.0, 0.3), (0.45, 1.0)])
def test_schedule_follows_eigenvalues_at_the_interval_ends(l, h):
    """Eigenvalues placed exactly at 0, l, h and 1 under the schedule's layer
    polynomials: those at l and h are the largest virtual and smallest
    occupied eigenvalue after every layer (the ends it records), the
    ordering is kept, and everything ends within 1e-12 of 0 or 1."""
    sched = acc.acceleration_schedule(l, h)
    assert sched
    virt = np.concatenate([np.linspace(0.0, l, 41)])
    occ = np.linspace(h, 1.0, 41)
    for sign, shift, l_after, h_after in sched:
        coef = acc.layer_polynomial(sign, shift)
        virt, occ = _poly(coef, virt), _poly(coef, occ)
        assert virt.max() == pytest.approx(l_after, abs=1e-13)
        assert occ.min() == pytest.approx(h_after, abs=1e-13)
        assert virt.max() < occ.min()
    assert virt.max() < 1e-12 and occ.min() > 1.0 - 1e-12


def test_schedule_branches_toward_the_wider_interval():
    sched = acc.acceleration_schedule(0.157, 0.212)
    l, h = 0.157, 0.212
    for sign, shift, l_after, h_after in sched:
        assert sign == (1 if l >= 1.0 - h else -1)
        assert shift == pytest.approx(0.4 * (l if sign > 0 else 1.0 - h), rel=1e-15)
        l, h = l_after, h_after


def test_no_gap_gives_no_schedule():
    assert acc.acceleration_schedule(0.5, 0.5) == []
    assert acc.acceleration_schedule(0.6, 0.4) == []


def test_fewer_layers_than_plain_sp2():
    """The c1 input and a water box: about a third fewer layers with exact
    estimates and Gershgorin bounds."""
    h, q, e = random_orthogonal_hamiltonian(256, 128, seed=0, return_factors=True)
    _, rec = oracle.sp2(h, 128)
    p, rec_a = acc.sp2_accelerated(h, 128, e[:128].max(), e[128:].min())
    assert rec.converged and rec_a.converged
    assert rec.n_iter == 26
    assert rec_a.n_iter <= 18
    hw = water_box_hamiltonian(32, seed=0)
    w = np.linalg.eigvalsh(hw)
    _, recw = oracle.sp2(hw, 128)
    _, recw_a = acc.sp2_accelerated(hw, 128, w[127], w[128])
    assert recw_a.n_iter <= recw.n_iter - 8


def test_accelerated_matches_diagonalisation_c1():
    h, q, e = random_orthogonal_hamiltonian(256, 128, seed=0, return_factors=True)
    p_ref = q[:, e.argsort()[:128]] @ q[:, e.argsort()[:128]].T
    p, rec = acc.sp2_accelerated(h, 128, e[:128].max(), e[128:].min())
    assert rec.converged
    assert np.linalg.norm(p - p_ref) / 16.0 < 1e-10
    assert abs(np.trace(p) - 128) < 1e-9


@pytest.mark.parametrize("margin", [0.0, 0.1, 0.45])
def test_accelerated_matches_diagonalisation_water(margin):
    """Water box (N = 192) with estimates inside the true gap by a fraction
    `margin` of it on each side."""
    hw = water_box_hamiltonian(32, seed=1)
    n_occ = 128
    p_ref, w, _ = oracle.density_matrix_eigh(hw, n_occ)
    gap = w[n_occ] - w[n_occ - 1]
    p, rec = acc.sp2_accelerated(hw, n_occ, w[n_occ - 1] + margin * gap, w[n_occ] - margin * gap)
    assert rec.converged
    assert np.linalg.norm(p - p_ref) / np.sqrt(192) < 1e-10
    assert all(s == (1 if a > 0 else -1) for s, (a, _, _) in zip(rec.branches, rec.coefs))


def test_two_by_two_closed_form():
    """n = 2, n_occ = 1: P = (I - (H - tr(H)/2 I) / r) / 2 with
    r = sqrt(((a - c)/2)^2 + b^2)."""
    h = np.array([[0.3, -0.7], [-0.7, -0.4]])
    r = np.sqrt(((0.3 + 0.4) / 2) ** 2 + 0.49)
    p_ref = 0.5 * (np.eye(2) - (h - 0.5 * np.trace(h) * np.eye(2)) / r)
    w = np.linalg.eigvalsh(h)
    p, rec = acc.sp2_accelerated(h, 1, w[0] + 0.2, w[1] - 0.2)
    assert rec.converged
    assert np.abs(p - p_ref).max() < 1e-12


def test_scalar_recursion_reproduces_the_matrix_network():
    """Every layer is a polynomial of S_0: the eigenvalue recursion gives the
    same traces, branches and coefficients, and V p(x) V^T = P."""
    h, q, e = random_orthogonal_hamiltonian(128, 50, occ_range=(-2.0, -0.1), virt_range=(0.1, 2.0),
                                            seed=3, return_factors=True)
    homo, lumo = e[:50].max() + 0.05, e[50:].min() - 0.05
    p, rec = acc.sp2_accelerated(h, 50, homo, lumo)
    w, v = np.linalg.eigh(h)
    x, rec_s = acc.sp2_accelerated_scalar(w, 50, rec.eps_min, rec.eps_max, homo, lumo)
    assert rec.branches == rec_s.branches
    assert rec.coefs == rec_s.coefs
    np.testing.assert_allclose(rec.t1, rec_s.t1, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(rec.t2, rec_s.t2, rtol=1e-10, atol=1e-10)
    assert np.abs(v @ np.diag(x) @ v.T - p).max() < 1e-11


def test_estimates_outside_the_spectrum_reduce_to_plain_sp2():
    """Both estimates above eps_max map to l = h = 0: no schedule, and the
    network is plain DNN-SP2 bit for bit."""
    h = random_orthogonal_hamiltonian(96, 40, seed=5)
    eps_min, eps_max = oracle.gershgorin_bounds(h)
    p0, rec0 = oracle.sp2(h, 40)
    p1, rec1 = acc.sp2_accelerated(h, 40, eps_max + 1.0, eps_max + 2.0)
    assert rec1.branches == rec0.branches
    assert np.array_equal(p0, p1)


@pytest.mark.parametrize("shift_into", ["occupied", "virtual"])
def test_estimates_that_miss_the_gap_fall_back_to_the_plain_network(shift_into):
    """Estimates whose 'gap' lies inside the occupied band (below the 64-fold
    degenerate HOMO level of this box) or the virtual band: the schedule
    drives 20 or more states to the wrong side, the trace at its end is off,
    and the plain network runs instead -- the same P and record as the
    oracle's plain network with the same bounds."""
    hw = water_box_hamiltonian(32, seed=2)
    n_occ = 128
    p_ref, w, _ = oracle.density_matrix_eigh(hw, n_occ)
    if shift_into == "occupied":
        homo, lumo = w[n_occ - 100], w[n_occ - 80]
        assert lumo < w[n_occ - 65] < w[n_occ - 1] - 0.1
    else:
        homo, lumo = w[n_occ + 10], w[n_occ + 30]
    p, rec = acc.sp2_accelerated(hw, n_occ, homo, lumo, max_iter=100)
    assert rec.fallback and rec.converged
    p0, rec0 = oracle.sp2(hw, n_occ)
    assert rec.branches == rec0.branches and np.array_equal(p, p0)
    assert np.linalg.norm(p - p_ref) / np.sqrt(192) < 1e-8
    ws = np.linalg.eigvalsh(hw)
    x, rs = acc.sp2_accelerated_scalar(ws, n_occ, rec.eps_min, rec.eps_max, homo, lumo)
    assert rs.fallback and rs.branches == rec0.branches


def test_estimates_inside_the_gap_do_not_fall_back():
    hw = water_box_hamiltonian(32, seed=2)
    w = np.linalg.eigvalsh(hw)
    for frac in (0.0, 0.2, 0.45):
        g = w[128] - w[127]
        _, rec = acc.sp2_accelerated(hw, 128, w[127] + frac * g, w[128] - frac * g)
        assert rec.converged and not rec.fallback


def test_derivatives_of_the_accelerated_network():
    """JVP of the recorded accelerated network: the layer-coefficient
    Daleckii-Krein formula, perturbation theory at convergence and central
    finite differences of the network with fixed estimates; VJP by the dot
    test and VJP(W) = JVP(W) (self-adjoint, commuting layer maps)."""
    h, q, e = random_orthogonal_hamiltonian(64, 24, occ_range=(-2.0, -0.3), virt_range=(0.3, 2.0),
                                            seed=7, return_factors=True)
    homo, lumo = e[:24].max() + 0.05, e[24:].min() - 0.05
    p, rec = acc.sp2_accelerated(h, 24, homo, lumo)
    assert rec.converged and any(c != 0.0 for _, _, c in rec.coefs)
    h1 = symmetric_normal(64, 2, std=1e-3)
    wm = symmetric_normal(64, 1)
    j = oracle.sp2_jvp(h, h1, rec)
    dk = oracle.daleckii_krein_jvp(h, h1, rec)
    assert np.abs(j - dk).max() < 1e-12 * max(1.0, np.abs(dk).max()) + 1e-14
    dm = oracle.dmpt_response(h, 24, h1)
    assert np.linalg.norm(j - dm) / np.linalg.norm(dm) < 1e-8
    step = 1e-4
    pp, _ = acc.sp2_accelerated(h + step * h1, 24, homo, lumo, bounds=(rec.eps_min, rec.eps_max))
    pm, _ = acc.sp2_accelerated(h - step * h1, 24, homo, lumo, bounds=(rec.eps_min, rec.eps_max))
    fd = (pp - pm) / (2 * step)
    assert np.linalg.norm(j - fd) / np.linalg.norm(fd) < 1e-6
    g = oracle.sp2_vjp(h, wm, rec)
    assert np.sum(wm * j) == pytest.approx(np.sum(g * h1), rel=1e-10)
    assert np.abs(g - oracle.sp2_jvp(h, wm, rec)).max() < 1e-10 * np.abs(g).max()
