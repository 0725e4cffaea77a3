"""Kernel-level parity of the HIP path against the FP64 oracle, through the
C ABI: Gershgorin bounds, the 16-bit dual representation (bit-exact) and
single expansion layers computed by the symmetric MFMA kernels."""

import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev, to_host
from workloads import random_orthogonal_hamiltonian

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24   # unit roundoff of FP32


@pytest.fixture(scope="module")
def pk():
    import paper_2107_02737_amd as pk
    pk.load_library()
    return pk


@pytest.mark.parametrize("n,ld", [(256, 256), (300, 307), (302, 308), (1000, 1000), (1100, 1100)])
def test_bounds_match_oracle(pk, n, ld):
    banner(f"bounds n={n} ld={ld}")
    h32 = random_orthogonal_hamiltonian(n, n // 2, seed=n).astype(np.float32)
    ws = pk.allocate_workspace(n)
    lo, hi = pk.sp2_bounds(to_dev(h32, ld), ws)
    rlo, rhi = oracle.gershgorin_bounds(h32.astype(np.float64))
    scale = max(abs(rlo), abs(rhi))
    assert abs(lo - rlo) <= 1e-13 * scale and abs(hi - rhi) <= 1e-13 * scale


@pytest.mark.parametrize("n,ld,i,j,val", [
    (64, 64, 3, 5, np.nan),        # off the diagonal, inside the 16-byte loop
    (64, 64, 7, 7, np.nan),        # on the diagonal
    (64, 64, 10, 40, np.inf),
    (64, 64, 12, 12, -np.inf),     # the diagonal term taken off the row sum: inf - inf
    (1100, 1100, 600, 1031, np.nan),   # a later batch of four loads per lane
    (67, 72, 66, 65, np.inf),      # ragged: the scalar tail of the row
    (67, 72, 66, 66, np.nan),      # ragged: the diagonal in the scalar tail
])
def test_bounds_reject_nonfinite(pk, n, ld, i, j, val):
    banner(f"bounds non-finite n={n} ld={ld} H[{i},{j}]={val}")
    h = random_orthogonal_hamiltonian(n, n // 2, seed=1).astype(np.float32)
    h[i, j] = h[j, i] = val
    ws = pk.allocate_workspace(n)
    with pytest.raises(pk.SP2Error) as ei:
        pk.sp2_bounds(to_dev(h, ld), ws)
    assert ei.value.status == 2


def _bits_bf16(x32):
    return (np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


def _bits_fp16(x32):
    return np.asarray(x32, dtype=np.float32).astype(np.float16).view(np.uint16)


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
def test_split_bit_exact(pk, precision):
    import torch
    banner(f"split {precision}")
    rng = np.random.default_rng(7)
    n, ld = 67, 70
    x = rng.uniform(-2.0, 2.0, (n, n)).astype(np.float32)
    specials = np.array([0.0, -0.0, 1.0, -1.0, 1e-8, -3e-41, 6e-5, 2.0 ** -20, 0.1, 1.0 / 3.0],
                        np.float32)
    x.flat[:specials.size] = specials
    # exact bf16 rounding ties (low 16 bits 0x8000)
    ties = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x3E4C8000], np.uint32).view(np.float32)
    x.flat[specials.size:specials.size + ties.size] = ties
    hi = torch.empty((n, n), dtype=torch.int16, device="cuda")
    lo = torch.empty((n, n), dtype=torch.int16, device="cuda")
    pk.sp2_split(to_dev(x, ld), precision, hi, lo)
    ghi = hi.cpu().numpy().view(np.uint16)
    glo = lo.cpu().numpy().view(np.uint16)
    if precision == "bf16x3":
        rhi, rlo = oracle.split_bf16(x)
        assert np.array_equal(ghi, _bits_bf16(rhi))
        assert np.array_equal(glo, _bits_bf16(rlo))
    else:
        rhi, rlo = oracle.split_fp16_scaled(x)
        assert np.array_equal(ghi, _bits_fp16(rhi))
        assert np.array_equal(glo, _bits_fp16(rlo))


def _layer_reference(x32, precision, sign):
    """FP64 value of exactly what the kernel computes, and the elementwise
    FP32-accumulation error bound gamma * (|A||B| summed) plus the FP32
    roundings of the epilogue.  FP32: X^2 (or 2X - X^2) of the FP32 operand.
    Split modes square the centred matrix T = X - I/2 (rounded to FP32, then
    split; the operands are its planes) and restore the layer as
    a T^2 + (b + a) X + (-a/4) I, with (a, b) = (1, 0) or (-1, 2)."""
    x = x32.astype(np.float64)
    n = x.shape[0]
    a, b = (1.0, 0.0) if sign > 0 else (-1.0, 2.0)
    if precision == "fp32":
        r = x @ x
        acc = np.abs(x) @ np.abs(x)
        nterms = n
        y = a * r + b * x
        bound = (nterms + 4) * U32 * acc + 2 * U32 * np.abs(r)
        if sign < 0:
            bound = bound + 4 * U32 * np.abs(x) + 2 * U32 * np.abs(y)
        return y, bound
    t32 = x32.copy()
    t32[np.diag_indices(n)] -= np.float32(0.5)
    if precision == "fp16x3":
        hi, lo = oracle.split_fp16_scaled(t32)
        s = 2.0 ** (-2 * oracle.FP16_SPLIT_SCALE_LOG2)
    else:
        hi, lo = oracle.split_bf16(t32)
        s = 1.0
    hi = hi.astype(np.float64)
    lo = lo.astype(np.float64)
    if precision == "bf16x1":
        r = hi @ hi
        acc = np.abs(hi) @ np.abs(hi)
        nterms = n
    else:
        r = (hi @ hi + hi @ lo + lo @ hi) * s
        acc = (np.abs(hi) @ np.abs(hi) + np.abs(hi) @ np.abs(lo) + np.abs(lo) @ np.abs(hi)) * s
        nterms = 3 * n
    y = a * r + (b + a) * x - 0.25 * a * np.eye(n)
    bound = ((nterms + 4) * U32 * acc + 2 * U32 * np.abs(r) + 4 * U32 * np.abs(x)
             + 4 * U32 * np.abs(y))
    return y, bound


# (n, ld, split-K): at these sizes the 256x256 tiles do not fill the machine,
# so by default every tile is split along K into pieces that the strip tail
# kernel sums; split-K off (SP2_NO_SPLITK) forces whole-tile work-groups only.
CASES = [(256, 256, True), (300, 300, True), (1000, 1003, True), (520, 520, True),
         (1000, 1000, False), (768, 768, False)]


@pytest.mark.parametrize("precision", ["fp32", "bf16x1", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("n,ld,splitk", CASES)
@pytest.mark.parametrize("sign", [1, -1])
def test_layer_matches_oracle_product(pk, precision, n, ld, splitk, sign, monkeypatch):
    import torch
    banner(f"layer {precision} n={n} ld={ld} splitk={splitk} sign={sign}")
    if not splitk:
        monkeypatch.setenv("SP2_NO_SPLITK", "1")
    rng = np.random.default_rng(n + 3)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    x = (q * rng.uniform(0.0, 1.0, n)) @ q.T
    x32 = x.astype(np.float32)
    x32 = np.triu(x32) + np.triu(x32, 1).T            # exactly symmetric FP32
    X = to_dev(x32, ld)
    Y = to_dev(np.zeros((n, n)), ld)
    ws = pk.allocate_workspace(n)
    pk.sp2_layer(X, precision, sign, Y, ws)
    y = to_host(Y)
    r, bound = _layer_reference(x32, precision, sign)
    err = np.abs(y - r)
    print(f"  max|err| {err.max():.3e}  max err/bound {np.max(err / bound):.3f}", flush=True)
    assert np.all(err <= bound)
    assert np.array_equal(y, y.T)                      # mirror write is exact
    if ld > n:                                         # padding columns untouched
        full = Y.as_strided((n, ld), (ld, 1))
        assert torch.isnan(full[:, n:]).all()
