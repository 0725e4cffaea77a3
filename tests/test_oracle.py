"""Pins for the FP64 oracle: each test fixes a part of the oracle against
something other than the oracle itself (a closed form, a construction, brute
force, an invariant, an independent spectral formula or a library routine in
a special case).  CPU only."""

import math

import numpy as np
import pytest

import oracle
from oracle import sp2_oracle as orc
from workloads import (random_orthogonal_hamiltonian, symmetric_normal,
                       water_box_hamiltonian)


def _c1(n=256, n_occ=128, seed=0):
    return random_orthogonal_hamiltonian(n, n_occ, seed=seed, return_factors=True)


# --------------------------------------------------------------------------
# density_matrix_eigh
# --------------------------------------------------------------------------

def test_eigh_density_matches_construction():
    h, q, _ = _c1()
    p, _, _ = oracle.density_matrix_eigh(h, 128)
    ref = q[:, :128] @ q[:, :128].T
    assert np.max(np.abs(p - ref)) < 1e-12


def test_two_by_two_closed_form():
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, b, c = rng.uniform(-2, 2, 3)
        h = np.array([[a, b], [b, c]])
        rad = math.sqrt(((a - c) / 2) ** 2 + b * b)
        closed = 0.5 * (np.eye(2) - (h - 0.5 * (a + c) * np.eye(2)) / rad)
        p_e, _, _ = oracle.density_matrix_eigh(h, 1)
        p_s, rec = oracle.sp2(h, 1, tol=1e-14)
        assert np.max(np.abs(p_e - closed)) < 1e-12
        assert np.max(np.abs(p_s - closed)) < 1e-10
        assert rec.converged


def test_diagonal_hamiltonian_gives_indicator_of_lowest_levels():
    rng = np.random.default_rng(3)
    d = rng.permutation(np.linspace(-3.0, 2.0, 40))
    h = np.diag(d)
    n_occ = 17
    expected = np.diag((d <= np.sort(d)[n_occ - 1]).astype(float))
    p_e, _, _ = oracle.density_matrix_eigh(h, n_occ)
    p_s, _ = oracle.sp2(h, n_occ, tol=1e-12)
    assert np.max(np.abs(p_e - expected)) < 1e-12
    assert np.max(np.abs(p_s - expected)) < 1e-10


@pytest.mark.parametrize("n_occ", [0, 64])
def test_empty_and_full_occupation(n_occ):
    h, _, _ = _c1(64, 32)
    p, rec = oracle.sp2(h, n_occ)
    expected = np.zeros((64, 64)) if n_occ == 0 else np.eye(64)
    assert np.array_equal(p, expected) and rec.n_iter == 0 and rec.converged
    assert np.max(np.abs(oracle.density_matrix_eigh(h, n_occ)[0] - expected)) < 1e-12


def test_block_diagonal_water_equals_per_molecule_diagonalisation():
    m = 12
    h = water_box_hamiltonian(m, seed=4, block_diagonal=True)
    n_occ = 4 * m
    blocks = np.zeros_like(h)
    for k in range(m):
        sl = slice(6 * k, 6 * k + 6)
        w, v = np.linalg.eigh(h[sl, sl])
        blocks[sl, sl] = v[:, :4] @ v[:, :4].T
    p_e, _, _ = oracle.density_matrix_eigh(h, n_occ)
    p_s, rec = oracle.sp2(h, n_occ, tol=1e-12)
    assert np.max(np.abs(p_e - blocks)) < 1e-11
    assert np.max(np.abs(p_s - blocks)) < 1e-10


# --------------------------------------------------------------------------
# gershgorin_bounds
# --------------------------------------------------------------------------

def test_gershgorin_brute_force_and_enclosure():
    rng = np.random.default_rng(11)
    a = rng.standard_normal((7, 7))
    h = a + a.T
    lo, hi = math.inf, -math.inf
    for i in range(7):
        r = 0.0
        for j in range(7):
            if j != i:
                r += abs(h[i, j])
        lo = min(lo, h[i, i] - r)
        hi = max(hi, h[i, i] + r)
    g = oracle.gershgorin_bounds(h)
    assert g == pytest.approx((lo, hi), rel=0, abs=1e-13)
    w = np.linalg.eigvalsh(h)
    assert g[0] <= w[0] and w[-1] <= g[1]


def test_input_layer_maps_spectrum_into_unit_interval_reversed():
    h, _, e = _c1(64, 32)
    lo, hi = oracle.gershgorin_bounds(h)
    s0 = oracle.input_layer(h, lo, hi)
    x = np.linalg.eigvalsh(s0)
    assert x.min() >= -1e-14 and x.max() <= 1 + 1e-14
    # lowest energy -> largest mapped value
    assert np.allclose(np.sort(x)[::-1], (hi - np.sort(e)) / (hi - lo), atol=1e-13)


# --------------------------------------------------------------------------
# sp2
# --------------------------------------------------------------------------

def test_sp2_matches_diagonalisation_config1():
    h, q, _ = _c1()
    p, rec = oracle.sp2(h, 128, tol=1e-10)
    ref = q[:, :128] @ q[:, :128].T
    assert rec.converged
    assert 20 <= rec.n_iter <= 40          # "~30 layers" for this workload
    assert np.linalg.norm(p - ref) / math.sqrt(256) < 1e-12


def test_sp2_invariants_on_water():
    m = 32
    h = water_box_hamiltonian(m, seed=1)
    n_occ = 4 * m
    p, rec = oracle.sp2(h, n_occ, tol=1e-12)
    n = h.shape[0]
    assert rec.converged
    assert np.array_equal(p, p.T) or np.max(np.abs(p - p.T)) < 1e-14
    assert np.linalg.norm(p @ p - p) / math.sqrt(n) < 1e-11
    assert abs(np.trace(p) - n_occ) < 1e-9
    assert np.linalg.norm(h @ p - p @ h) / math.sqrt(n) < 1e-11
    p_e, _, _ = oracle.density_matrix_eigh(h, n_occ)
    assert np.max(np.abs(p - p_e)) < 1e-10


def test_scalar_recursion_reproduces_matrix_run():
    """All traces are spectral sums, so running the layers on the eigenvalues
    must give the same branches, traces and errors, and V p(x) V^T = P."""
    for h, n_occ in [(_c1()[0], 128), (water_box_hamiltonian(24, seed=2), 96)]:
        p, rec = oracle.sp2(h, n_occ, tol=1e-10)
        w, v = np.linalg.eigh(h)
        x, rs = oracle.sp2_scalar(w, n_occ, rec.eps_min, rec.eps_max, tol=1e-10)
        assert rs.branches == rec.branches
        assert np.allclose(rs.t1, rec.t1, rtol=0, atol=1e-10)
        assert np.allclose(rs.t2, rec.t2, rtol=0, atol=1e-10)
        assert np.allclose(rs.err, rec.err, rtol=1e-6, atol=1e-11)
        assert np.max(np.abs((v * x[None, :]) @ v.T - p)) < 1e-12


def test_permutation_equivariance():
    h, _, _ = _c1(96, 40, seed=4)
    perm = np.random.default_rng(0).permutation(96)
    hp = h[np.ix_(perm, perm)]
    p, rec = oracle.sp2(h, 40, tol=1e-10)
    pp, recp = oracle.sp2(hp, 40, tol=1e-10)
    assert rec.branches == recp.branches
    assert np.max(np.abs(pp - p[np.ix_(perm, perm)])) < 1e-12


def test_affine_invariance():
    h, _, _ = _c1(96, 40, seed=6)
    p, rec = oracle.sp2(h, 40, tol=1e-10)
    for alpha, beta in [(2.0, 0.0), (0.5, 0.25), (3.0, -1.5)]:
        pa, reca = oracle.sp2(alpha * h + beta * np.eye(96), 40, tol=1e-10)
        assert reca.branches == rec.branches
        assert np.max(np.abs(pa - p)) < 1e-11


def test_stagnation_rule_stops_at_rounding_floor():
    """With an unreachable tolerance, rule 0 runs to max_iter while rule 1
    stops at the floor with the same density matrix."""
    h, q, _ = _c1(128, 64, seed=9)
    p0, r0 = oracle.sp2(h, 64, tol=0.0, max_iter=80, stop_rule=0)
    p1, r1 = oracle.sp2(h, 64, tol=0.0, max_iter=80, stop_rule=1)
    assert not r0.converged and r0.n_iter == 80
    assert r1.converged and r1.n_iter < 60
    ref = q[:, :64] @ q[:, :64].T
    assert np.max(np.abs(p1 - ref)) < 1e-12


@pytest.mark.parametrize("n_occ", [1, 2, 5, 299])
def test_stop_rule_at_extreme_occupations(n_occ):
    """With few eigenvalues on one side of the gap, the error estimate drops
    below the stagnation gate while an occupied eigenvalue is still close to
    0 (or a virtual one close to 1).  The trace condition keeps the network
    running; the result is the projector onto the n_occ lowest states."""
    h = random_orthogonal_hamiltonian(300, n_occ, seed=11)
    w, v = np.linalg.eigh(h)
    ref = v[:, :n_occ] @ v[:, :n_occ].T
    p, rec = oracle.sp2(h, n_occ, tol=1e-5, stop_rule=1)
    assert rec.converged
    assert np.max(np.abs(p - ref)) < 1e-5
    # the guard was needed: some earlier approximation met the stagnation
    # condition with the trace still at least 1/2 away from n_occ (for
    # n_occ = 5 the trace is right but the error estimate is above the gate)
    hit = [k for k in range(2, rec.n_iter)
           if rec.err[k] < 1.0 and rec.err[k] >= rec.err[k - 2]
           and (abs(rec.t1[k] - n_occ) >= 0.5 or rec.err[k] >= oracle.STALL_GATE)]
    assert hit


def test_single_layer_rise_does_not_stop_the_network():
    """Few occupied states: the error estimate of the exact-arithmetic
    network rises for one layer inside the stagnation gate while the run is
    still far from converged (0.1775, 0.0748, 0.0752, then falling), so a
    stagnation test that compared one layer back would stop there; the rule
    compares two layers back and runs on to the floor."""
    w = np.concatenate([np.linspace(-3.0, -0.5, 5), np.linspace(0.5, 3.0, 95)])
    _, rec = oracle.sp2_scalar(w, 5, -4.0, 4.0, tol=0.0, max_iter=80)
    k = 15
    assert rec.err[k - 1] < rec.err[k] < min(rec.err[k - 2], oracle.STALL_GATE)
    assert abs(rec.t1[k] - 5) < 0.5
    assert not oracle.should_stop(k, rec.err, abs(rec.t1[k] - 5), 0.0, 1, oracle.STALL_GATE)
    _, r1 = oracle.sp2_scalar(w, 5, -4.0, 4.0, tol=1e-12, max_iter=80, stop_rule=1)
    assert r1.converged and r1.err[-1] < 1e-12


def test_quadratic_stall_threshold():
    """Rule 1 compares e_k with min(e_{k-2}, 16 e_{k-2}^2): at e_{k-2} = 0.01
    the threshold is 1.6e-3 (not 1e-2, the plain comparison, nor 4e-4);
    above e_{k-2} = 1/16 the plain comparison is the smaller one; the gate,
    the trace guard and stall_from still apply."""
    g = oracle.STALL_GATE
    assert oracle.QUAD_FACTOR == 16.0
    stop = lambda errs, gap=0.0, sf=0: oracle.should_stop(len(errs) - 1, errs, gap, 0.0, 1, g, sf)
    assert stop([0.01, 0.5, 1.6e-3])
    assert not stop([0.01, 0.5, 1.59e-3])
    assert not stop([0.01, 0.5, 1.6e-3], gap=0.5)
    assert not stop([0.5, 0.01, 0.5, 1.6e-3], sf=2)
    assert stop([0.5, 0.01, 0.5, 1.6e-3], sf=1)
    assert stop([0.1, 0.5, 0.1]) and not stop([0.1, 0.5, 0.0999])      # min is e_{k-2}
    assert not stop([0.1, 0.5, 0.1], gap=0.6)
    assert not stop([0.3, 0.5, 0.2])                                   # above the gate
    assert not oracle.should_stop(2, [0.01, 0.5, 1.0], 0.0, 0.0, 0, g)  # rule 0


def _random_spectrum(rng, trial):
    n = int(rng.integers(3, 300))
    kind = trial % 4
    if kind == 0:
        w = rng.normal(size=n)
    elif kind == 1:
        w = rng.uniform(-1.0, 1.0, size=n)
    elif kind == 2:
        w = np.concatenate([rng.normal(-1.0, 0.3, n // 2), rng.normal(1.0, 0.3, n - n // 2)])
    else:
        w = np.round(rng.normal(size=n), 1)       # many degenerate levels
    w = np.sort(w)
    n_occ = int(rng.integers(1, n))
    lo = w[0] - rng.uniform(0.0, 0.5) * (w[-1] - w[0]) - 1e-3
    hi = w[-1] + rng.uniform(0.0, 0.5) * (w[-1] - w[0]) + 1e-3
    return w, n_occ, lo, hi


def test_quadratic_stall_rule_never_stops_an_exact_network_early():
    """In exact (FP64 scalar) arithmetic rule 1 with tol = 0 runs every plain
    and accelerated network on random spectra (normal, uniform, two bands,
    degenerate levels; occupations 1 .. N-1; loose and tight bounds) until
    e_k < 1e-6 with every eigenvalue within 1e-6 of its side.  (The bound
    e_k <= 4 e_{k-2}^2 can fail by itself only once e is tiny and carried by
    one or two eigenvalues: over 2232 such runs the earliest stop was at
    2.9e-7.)  A comparison that fired on a quadratically falling e (a
    smaller factor, the wrong lag, or no stall_from in the schedule) stops
    with e_k of order 1e-2 .. 1e-1 on some of them."""
    rng = np.random.default_rng(7)
    runs = 0
    for trial in range(160):
        w, n_occ, lo, hi = _random_spectrum(rng, trial)
        gap = w[n_occ] - w[n_occ - 1]
        if gap < 1e-3 * (hi - lo):
            continue
        target = np.arange(w.size) < n_occ
        x, rec = oracle.sp2_scalar(w, n_occ, lo, hi, tol=0.0, max_iter=200, stop_rule=1)
        nets = [(x, rec)]
        for m in (0.0, 0.3):
            nets.append(oracle.accelerated.sp2_accelerated_scalar(
                w, n_occ, lo, hi, w[n_occ - 1] + m * gap, w[n_occ] - m * gap, tol=0.0,
                max_iter=200, stop_rule=1))
        for x, rec in nets:
            runs += 1
            assert rec.converged
            assert rec.err[-1] < 1e-6, (trial, rec.err[-4:])
            assert np.max(np.abs(x - target)) < 1e-6, trial
    assert runs > 250


def test_quadratic_stall_rule_ends_a_slowly_falling_floor():
    """A rounding floor that still drifts down by 1% per layer: the plain
    comparison e_k >= e_{k-2} never fires on it, the quadratic one fires as
    soon as e_k is mostly floor (the exact part below a tenth of it), and
    never while e_{k-2} is still large."""
    w = np.concatenate([np.linspace(-2.0, -0.5, 40), np.linspace(0.5, 2.0, 60)])
    _, rec = oracle.sp2_scalar(w, 40, -3.0, 3.0, tol=1e-12, max_iter=80, stop_rule=0)
    floor = 2e-3 * 0.99 ** np.arange(len(rec.err))
    errs = list(np.array(rec.err) + floor)
    first = next(k for k in range(len(errs)) if rec.err[k] < 0.1 * floor[k])
    fired = [k for k in range(2, len(errs))
             if oracle.should_stop(k, errs, 0.0, 0.0, 1, oracle.STALL_GATE)]
    assert fired and first <= fired[0] <= first + 2
    assert all(rec.err[k - 2] < 1e-2 for k in fired)
    assert not any(errs[k] >= errs[k - 2] for k in range(first, len(errs)))


def test_vjp_of_nonsymmetric_weight_is_the_symmetric_gradient():
    """The gradient of Tr(W P) over symmetric perturbations of H is symmetric
    and depends on W only through sym(W)."""
    h, _, _ = _c1(64, 32, seed=3)
    _, rec = oracle.sp2(h, 32, tol=1e-12, refine=True)
    wm = np.random.default_rng(8).standard_normal((64, 64))
    g = oracle.sp2_vjp(h, wm, rec)
    scale = np.abs(g).max()
    assert np.allclose(g, g.T, rtol=0, atol=1e-13 * scale)
    assert np.allclose(g, oracle.sp2_vjp(h, 0.5 * (wm + wm.T), rec), rtol=0, atol=1e-13 * scale)


def test_mcweeny_acts_as_cubic_on_eigenvalues():
    rng = np.random.default_rng(2)
    q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    x = rng.uniform(-0.1, 1.1, 30)
    s = (q * x) @ q.T
    got = np.sort(np.linalg.eigvalsh(oracle.mcweeny(s)))
    assert np.allclose(got, np.sort(3 * x ** 2 - 2 * x ** 3), atol=1e-13)


def test_refinement_improves_idempotency_of_truncated_run():
    h, q, _ = _c1(128, 64, seed=1)
    p, rec = oracle.sp2(h, 64, tol=1e-3)
    pr, recr = oracle.sp2(h, 64, tol=1e-3, refine=True)
    i0 = np.linalg.norm(p @ p - p)
    i1 = np.linalg.norm(pr @ pr - pr)
    assert i1 < 0.1 * i0 and recr.branches == rec.branches


# --------------------------------------------------------------------------
# derivatives
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_case():
    h, _, _ = _c1(160, 80, seed=7)
    h1 = symmetric_normal(160, 2, std=1e-3)
    w = symmetric_normal(160, 1)
    p, rec = oracle.sp2(h, 80, tol=1e-10)
    return h, h1, w, p, rec


def test_jvp_matches_spectral_divided_differences(small_case):
    h, h1, _, _, rec = small_case
    j = oracle.sp2_jvp(h, h1, rec)
    dk = oracle.daleckii_krein_jvp(h, h1, rec)
    assert np.linalg.norm(j - dk) / np.linalg.norm(dk) < 1e-12


def test_jvp_matches_perturbation_theory_and_finite_differences(small_case):
    h, h1, _, p, rec = small_case
    j = oracle.sp2_jvp(h, h1, rec)
    dm = oracle.dmpt_response(h, 80, h1)
    fd = oracle.finite_difference_jvp(h, 80, h1, step=1e-4, tol=1e-10)
    nrm = np.linalg.norm(dm)
    assert np.linalg.norm(j - dm) / nrm < 1e-9
    assert np.linalg.norm(j - fd) / nrm < 1e-6


def test_jvp_invariants(small_case):
    h, h1, _, p, rec = small_case
    j = oracle.sp2_jvp(h, h1, rec)
    scale = np.linalg.norm(j)
    assert abs(np.trace(j)) < 1e-10 * scale + 1e-14
    assert np.linalg.norm(p @ j + j @ p - j) < 1e-9 * scale
    assert np.linalg.norm(h @ j - j @ h + h1 @ p - p @ h1) < 1e-9 * scale


@pytest.mark.parametrize("refine", [False, True])
def test_vjp_dot_test_and_self_adjointness(small_case, refine):
    h, h1, w, _, _ = small_case
    _, rec = oracle.sp2(h, 80, tol=1e-6, refine=refine)
    j = oracle.sp2_jvp(h, h1, rec)
    g = oracle.sp2_vjp(h, w, rec)
    lhs = float(np.sum(w * j))
    rhs = float(np.sum(g * h1))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + np.linalg.norm(w) * np.linalg.norm(j))
    assert np.linalg.norm(g - oracle.sp2_jvp(h, w, rec)) < 1e-12 * np.linalg.norm(g)
    dk = oracle.daleckii_krein_jvp(h, h1, rec)
    assert np.linalg.norm(j - dk) < 1e-11 * np.linalg.norm(dk)


# --------------------------------------------------------------------------
# 16-bit rounding of the dual representation
# --------------------------------------------------------------------------

def _rounding_inputs():
    rng = np.random.default_rng(0)
    vals = [rng.standard_normal(4096).astype(np.float32),
            (rng.standard_normal(4096) * 1e-6).astype(np.float32),
            np.array([0.0, -0.0, 1.0, -1.0, 65504.0, 1e-8, -3e-41, 6e-5], np.float32)]
    # exact ties for bf16: low 16 bits = 0x8000 with both parities of bit 16
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x40490000 | 0x8000], np.uint32)
    vals.append(ties.view(np.float32))
    return np.concatenate(vals)


def test_bf16_rounding_matches_torch_bitwise():
    torch = pytest.importorskip("torch")
    x = _rounding_inputs()
    mine = oracle.round_to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mine.view(np.uint32), ref.view(np.uint32))


def test_fp16_rounding_matches_torch_bitwise():
    torch = pytest.importorskip("torch")
    x = _rounding_inputs()
    mine = oracle.round_to_fp16(x)
    ref = torch.from_numpy(x).to(torch.float16).to(torch.float32).numpy()
    assert np.array_equal(mine.view(np.uint32), ref.view(np.uint32))


def test_split_pairs_reconstruct_to_working_precision():
    x = np.random.default_rng(1).uniform(-1, 1, 10000).astype(np.float32)
    hi, lo = oracle.split_bf16(x)
    assert np.all(np.abs((hi.astype(np.float64) + lo) - x) <= 2.0 ** -16 * np.abs(x) + 1e-45)
    s = 2.0 ** oracle.FP16_SPLIT_SCALE_LOG2
    hi, lo = oracle.split_fp16_scaled(x)
    rec = (hi.astype(np.float64) + lo) / s
    assert np.all(np.abs(rec - x) <= 2.0 ** -21 * np.abs(x) + 2.0 ** -38)


# --------------------------------------------------------------------------
# The pins catch planted mistakes (mutations applied to the oracle, on CPU)
# --------------------------------------------------------------------------

def test_pins_catch_a_flipped_branch_rule(monkeypatch):
    h, q, _ = _c1(128, 64, seed=2)
    monkeypatch.setattr(orc, "choose_branch", lambda t1, t2, n: -1 if abs(t2 - n) <= abs(2 * t1 - t2 - n) else 1)
    p, rec = orc.sp2(h, 64, tol=1e-10, max_iter=60)
    ref = q[:, :64] @ q[:, :64].T
    assert np.max(np.abs(p - ref)) > 1e-3


def test_pins_catch_a_non_reversed_input_map(monkeypatch):
    h, q, _ = _c1(128, 64, seed=2)
    monkeypatch.setattr(orc, "input_layer",
                        lambda hh, lo, hi: (np.asarray(hh) - lo * np.eye(hh.shape[0])) / (hi - lo))
    p, rec = orc.sp2(h, 64, tol=1e-10, max_iter=60)
    ref = q[:, :64] @ q[:, :64].T
    assert np.max(np.abs(p - ref)) > 1e-3


def test_pins_catch_a_one_sided_jvp_layer(small_case):
    """Mutant layer derivative ``2 S dS`` instead of ``S dS + dS S``: the
    spectral divided-difference pin must reject it."""
    h, h1, _, _, rec = small_case
    iters = orc._replay(h, rec)
    y = -h1 / (rec.eps_max - rec.eps_min)
    for sign, s in zip(rec.branches, iters[:-1]):
        sy = 2.0 * (s @ y)
        y = sy if sign > 0 else 2.0 * y - sy
    dk = orc.daleckii_krein_jvp(h, h1, rec)
    assert np.linalg.norm(y - dk) > 1e-3 * np.linalg.norm(dk)
