"""Pins for the rounding-level emulation of the GPU precision modes
(``oracle/precision_emulation.py``) and for the error report
(``oracle.error_metrics``).  CPU only.

The emulation sets the tolerance of most end-to-end GPU tests, so each of its
parts is fixed here against something other than itself: products of operands
that are exactly representable in the mode (the split must return those
operands, and the FP32 sums of their products are exact, so the result must
equal the FP64 sum of the three products of Eq. (22) exactly), closed forms of
the stagnation gate, and a plain FP32 SP2 loop written out below.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import precision_emulation as emu
from oracle import sp2_oracle as orc
from workloads import random_orthogonal_hamiltonian


def _sym(a):
    return np.triu(a) + np.triu(a, 1).T


def _exact_pair_bf16(n, seed):
    """Symmetric X = X0 + X1 with X0 bfloat16 integers in 5..7 and X1 = k / 1024,
    |k| <= 15: |X| stays in [4, 8), where the BF16 ulp is 2^-5, and X1 is
    below half of it, so BF16 rounding of X returns X0 and X - X0 = X1."""
    rng = np.random.default_rng(seed)
    hi = _sym(rng.integers(5, 8, (n, n)) * rng.choice([-1.0, 1.0], (n, n)))
    lo = _sym(rng.integers(-15, 16, (n, n)) / 1024.0)
    return hi, lo


def _exact_pair_fp16(n, seed):
    """Symmetric X = 2^-14 (X0 + X1) with X0 half-precision integers in 9..15
    and X1 = k 2^-12, |k| <= 15: |2^14 X| stays in [8, 16), where the FP16 ulp
    is 2^-7, and X1 is below half of it, so the scaled FP16 split of X returns
    X0 and X1 exactly."""
    rng = np.random.default_rng(seed)
    hi = _sym(rng.integers(9, 16, (n, n)) * rng.choice([-1.0, 1.0], (n, n)))
    lo = _sym(rng.integers(-15, 16, (n, n)) * 2.0 ** -12)
    return hi, lo


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bf16_modes_equal_exact_products_of_representable_operands(seed):
    n = 16   # every partial sum below stays within 24 significant bits
    hi, lo = _exact_pair_bf16(n, seed)
    x = (hi + lo).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), hi + lo)          # X itself is exact
    h64, l64 = hi.astype(np.float64), lo.astype(np.float64)
    three = h64 @ h64 + h64 @ l64 + l64 @ h64                      # Eq. (22), X1 X1 dropped
    got3 = emu.square_emulated(x, "bf16x3").astype(np.float64)
    assert np.array_equal(got3, three)
    got1 = emu.square_emulated(x, "bf16x1").astype(np.float64)
    assert np.array_equal(got1, h64 @ h64)                         # single pass: X0 X0 only
    # the dropped X1 X1 term is not zero here, so "X^2 of FP32 X" is a different answer
    assert not np.array_equal(got3, (hi + lo) @ (hi + lo))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp16x3_equals_exact_rescaled_products_of_representable_operands(seed):
    n = 8
    hi, lo = _exact_pair_fp16(n, seed)
    x = ((hi + lo) * 2.0 ** -14).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), (hi + lo) * 2.0 ** -14)
    three = (hi @ hi + hi @ lo + lo @ hi) * 2.0 ** -28              # products carry 2^28
    got = emu.square_emulated(x, "fp16x3").astype(np.float64)
    assert np.array_equal(got, three)


def test_fp32_mode_is_the_plain_product():
    rng = np.random.default_rng(4)
    x = _sym(rng.integers(-50, 51, (24, 24)).astype(np.float64))
    got = emu.square_emulated(x.astype(np.float32), "fp32")
    assert got.dtype == np.float32
    assert np.array_equal(got.astype(np.float64), x @ x)          # integer sums: exact


@pytest.mark.parametrize("mode", emu.MODES)
@pytest.mark.parametrize("abc", [(1.0, 0.0, 0.0), (-1.0, 2.0, 0.0), (1.5625, -0.625, 0.0625),
                                 (-1.5625, 2.5, 0.0)])
def test_centred_layer_is_the_exact_layer(mode, abc):
    """An iterate with entries k/64 (|k| <= 32): its centred matrix S - I/2
    is exact in every 16-bit format, every product of two entries is
    exact and the sums stay far inside FP32, so the emulated layer (split
    modes: square of the centred matrix plus the FP32 restoration) equals
    the exact a S^2 + b S + c I for the plain layers and shifted ones
    (coefficients with few bits).  A wrong restoration (b + a, c - a/4 as
    other multiples of the centre) fails."""
    a, b, c = abc
    rng = np.random.default_rng(12)
    s = _sym(rng.integers(-32, 33, (32, 32)).astype(np.float64)) / 64.0
    s = np.triu(s) + np.triu(s, 1).T
    exact = a * (s @ s) + b * s + c * np.eye(32)
    got = emu.layer_emulated(s.astype(np.float32), mode, a, b, c)
    assert got.dtype == np.float32
    if mode == "bf16x1":        # one plane: the square of the rounded centred matrix
        t = s - 0.5 * np.eye(32)
        hi, _ = orc.split_bf16(t.astype(np.float32))
        assert np.array_equal(hi.astype(np.float64), t)   # representable: no rounding
    assert np.array_equal(got.astype(np.float64), exact)


def test_unknown_mode_is_refused():
    with pytest.raises(ValueError):
        emu.square_emulated(np.eye(2, dtype=np.float32), "fp8")


def test_automatic_stall_gate_closed_forms():
    assert emu.automatic_stall_gate(256, "fp32") == 3.0 / 16.0
    assert emu.automatic_stall_gate(6144, "bf16x1") == 6144 / 256 / 16    # 1.5
    assert emu.automatic_stall_gate(6144, "bf16x3") == 3.0 / 16.0         # 6144 / 2^16 / 16 < 3/16
    assert emu.automatic_stall_gate(2 ** 20, "bf16x3") == 1.0
    assert emu.automatic_stall_gate(2 ** 26, "fp16x3") == 1.0
    assert emu.automatic_stall_gate(2 ** 28, "fp32") == 1.0


def _plain_fp32_sp2(h, n_occ, tol, stall_gate, refine, coefs=()):
    """FP32-stored SP2 written out step by step: FP64 Gershgorin discs, the
    reversed linear map rounded to FP32, then per layer FP64 traces of the
    FP32 iterate, the stop test and branch rule of the FP64 oracle, an FP32
    square, FP32 S^2 or 2S - S^2 and the upper triangle mirrored; FP32 McWeeny
    at the end."""
    h64 = np.asarray(h, dtype=np.float32).astype(np.float64)
    n = h64.shape[0]
    rows = [(h64[i, i] - (np.sum(np.abs(h64[i])) - abs(h64[i, i])),
             h64[i, i] + (np.sum(np.abs(h64[i])) - abs(h64[i, i]))) for i in range(n)]
    lo_b = min(r[0] for r in rows)
    hi_b = max(r[1] for r in rows)
    s = ((hi_b * np.eye(n) - h64) / (hi_b - lo_b)).astype(np.float32)
    errs, layers = [], 0
    for k in range(101):
        t1 = float(np.trace(s.astype(np.float64)))
        t2 = float(np.sum(s.astype(np.float64) ** 2))
        errs.append(abs(t1 - t2))
        if orc.should_stop(k, errs, abs(t1 - n_occ), tol, 1, stall_gate) or k == 100:
            break
        sq = np.matmul(s, s, dtype=np.float32)
        if k < len(coefs):     # accelerated layer: a S^2 + b S, then c on the diagonal
            a, b, c = coefs[k]
            s = np.float32(a) * sq + np.float32(b) * s
            for i in range(n):
                s[i, i] = s[i, i] + np.float32(c)
        else:
            plus = abs(t2 - n_occ) <= abs(2.0 * t1 - t2 - n_occ)
            s = sq if plus else np.float32(2.0) * s - sq
        s = np.triu(s) + np.triu(s, 1).T
        layers += 1
    if refine:
        s2 = np.matmul(s, s, dtype=np.float32)
        s = np.float32(3.0) * s2 - np.float32(2.0) * np.matmul(s, s2, dtype=np.float32)
    return s, layers


@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("n_occ", [20, 30])     # first layer S^2 (20) or 2S - S^2 (30)
def test_fp32_emulation_equals_a_plain_fp32_loop(refine, n_occ):
    h = random_orthogonal_hamiltonian(48, n_occ, seed=3).astype(np.float32)
    p, nl = emu.sp2_emulated(h, n_occ, "fp32", tol=1e-5, refine=refine)
    q, ml = _plain_fp32_sp2(h, n_occ, 1e-5, emu.automatic_stall_gate(48, "fp32"), refine)
    assert nl == ml and nl > 10
    assert p.dtype == np.float32
    assert np.array_equal(p, q)       # the same FP32 operations in the same order


def test_accelerated_fp32_emulation_equals_a_plain_fp32_loop():
    from oracle import accelerated as acc
    h, q, e = random_orthogonal_hamiltonian(48, 20, seed=3, return_factors=True)
    h = h.astype(np.float32)
    homo, lumo = e[:20].max() + 0.02, e[20:].min() - 0.02
    lo_b, hi_b = orc.gershgorin_bounds(h.astype(np.float64))
    l, hh = acc.mapped_interval(lo_b, hi_b, homo, lumo)
    coefs = [acc.layer_polynomial(sg, sh) for sg, sh, _, _ in acc.acceleration_schedule(l, hh)]
    p, nl = emu.sp2_emulated(h, 20, "fp32", tol=1e-5, refine=True, homo=homo, lumo=lumo)
    q2, ml = _plain_fp32_sp2(h, 20, 1e-5, emu.automatic_stall_gate(48, "fp32"), True, coefs)
    assert nl == ml and 5 < nl < 15
    assert np.array_equal(p, q2)


def test_emulation_with_estimates_outside_the_spectrum_is_the_plain_network():
    h = random_orthogonal_hamiltonian(48, 20, seed=5).astype(np.float32)
    _, hi_b = orc.gershgorin_bounds(h.astype(np.float64))
    for mode in ("fp32", "bf16x3"):
        p0, n0 = emu.sp2_emulated(h, 20, mode)
        p1, n1 = emu.sp2_emulated(h, 20, mode, homo=hi_b + 1.0, lumo=hi_b + 2.0)
        assert n0 == n1 and np.array_equal(p0, p1)


@pytest.mark.parametrize("mode,bits", [("fp32", 24), ("fp16x3", 22), ("bf16x3", 16), ("bf16x1", 8)])
def test_accelerated_emulated_error_follows_operand_precision(mode, bits):
    """The accelerated network lands in the same band, [1/256, 2] of u times
    the Gershgorin width, with fewer layers."""
    for seed in (6, 7):
        h, q, e = random_orthogonal_hamiltonian(96, 48, seed=seed, return_factors=True)
        h = h.astype(np.float32)
        p_ref = oracle.density_matrix_eigh(h.astype(np.float64), 48)[0]
        lo_b, hi_b = orc.gershgorin_bounds(h.astype(np.float64))
        homo, lumo = e[:48].max(), e[48:].min()
        p, nl = emu.sp2_emulated(h, 48, mode, tol=1e-7, homo=homo, lumo=lumo)
        _, nl0 = emu.sp2_emulated(h, 48, mode, tol=1e-7)
        err = oracle.error_metrics(p, p_ref)["fro_over_sqrt_n"]
        scale = 2.0 ** -bits * (hi_b - lo_b)
        assert scale / 256 < err < 2 * scale
        assert nl < nl0


@pytest.mark.parametrize("mode,bits", [("fp32", 24), ("fp16x3", 22), ("bf16x3", 16), ("bf16x1", 8)])
def test_emulated_error_follows_operand_precision(mode, bits):
    """Against the exact density matrix each mode lands near its operand
    roundoff ``u`` times the width of the Gershgorin interval (the inverse of
    the mapped gap, the levels being at least 0.5 from mu): measured
    0.007-0.55 of ``u * width`` for every mode (the centred planes of the
    split modes keep them at the low end).  A dropped lo term or a missing
    rescale moves a mode by orders of magnitude."""
    for seed in (6, 7):
        h = random_orthogonal_hamiltonian(96, 48, seed=seed).astype(np.float32)
        p_ref = oracle.density_matrix_eigh(h.astype(np.float64), 48)[0]
        lo_b, hi_b = orc.gershgorin_bounds(h.astype(np.float64))
        p, _ = emu.sp2_emulated(h, 48, mode, tol=1e-7)
        err = oracle.error_metrics(p, p_ref)["fro_over_sqrt_n"]
        scale = 2.0 ** -bits * (hi_b - lo_b)
        assert scale / 256 < err < 2 * scale


def test_single_pass_bf16_is_worse_than_the_pairs():
    """Operand bits set the order: BF16 (8) far behind the BF16 pair (16),
    which trails the FP16 pair (22); the last gap is narrower than 2^6
    because the FP16 pair's error already sits near the FP32 accumulation
    and storage level."""
    h = random_orthogonal_hamiltonian(96, 48, seed=7).astype(np.float32)
    p_ref = oracle.density_matrix_eigh(h.astype(np.float64), 48)[0]
    errs = {m: oracle.error_metrics(emu.sp2_emulated(h, 48, m)[0], p_ref)["fro_over_sqrt_n"]
            for m in ("bf16x1", "bf16x3", "fp16x3")}
    assert errs["bf16x1"] > 100 * errs["bf16x3"]
    assert errs["bf16x3"] > 4 * errs["fp16x3"]


# --------------------------------------------------------------------------
# error_metrics
# --------------------------------------------------------------------------

def test_error_metrics_diagonal_closed_form():
    p = np.diag([1.0, 1.0, 0.5, 0.0])
    p_ref = np.diag([1.0, 1.0, 0.0, 0.0])
    m = oracle.error_metrics(p, p_ref, h=np.diag([-2.0, -1.0, 1.0, 2.0]), n_occ=2)
    assert m["fro_over_sqrt_n"] == 0.25       # 0.5 / sqrt(4)
    assert m["fro_over_n"] == 0.125           # 0.5 / 4
    assert m["max_abs"] == 0.5
    assert m["idempotency"] == 0.125          # |0.25 - 0.5| / sqrt(4)
    assert m["trace_err"] == 0.5
    assert m["commutator"] == 0.0             # diagonal H and P commute
    # the largest difference negative: max-abs is still its magnitude
    assert oracle.error_metrics(p_ref, p)["max_abs"] == 0.5


def test_error_metrics_two_by_two_closed_form():
    p = np.array([[1.0, 0.5], [0.5, 0.0]])
    p_ref = np.array([[1.0, 0.0], [0.0, 0.0]])
    h = np.diag([1.0, -1.0])
    m = oracle.error_metrics(p, p_ref, h=h, n_occ=1)
    # difference [[0, .5], [.5, 0]]: Frobenius sqrt(0.5)
    assert math.isclose(m["fro_over_sqrt_n"], math.sqrt(0.5) / math.sqrt(2), rel_tol=1e-15)
    assert math.isclose(m["fro_over_n"], math.sqrt(0.5) / 2, rel_tol=1e-15)
    assert m["max_abs"] == 0.5
    # P^2 - P = [[0.25, 0], [0, 0.25]]: Frobenius sqrt(0.125)
    assert math.isclose(m["idempotency"], math.sqrt(0.125) / math.sqrt(2), rel_tol=1e-15)
    assert m["trace_err"] == 0.0
    # H P - P H = [[0, 1], [-1, 0]]: Frobenius sqrt(2)
    assert math.isclose(m["commutator"], 1.0, rel_tol=1e-15)


def test_error_metrics_zero_for_the_exact_answer():
    h = random_orthogonal_hamiltonian(32, 10, seed=9)
    p_ref = oracle.density_matrix_eigh(h, 10)[0]
    m = oracle.error_metrics(p_ref, p_ref, h=h, n_occ=10)
    assert m["fro_over_sqrt_n"] == 0.0 and m["max_abs"] == 0.0
    assert m["idempotency"] < 1e-14 and m["trace_err"] < 1e-12 and m["commutator"] < 1e-13
