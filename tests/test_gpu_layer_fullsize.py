"""Element-wise parity of one expansion layer (sp2_layer: the same product
kernels, work decomposition and epilogue as the solver's layers) at the
benchmark's order N = 6144 and at the trajectory's N = 16384.

At these sizes there are more 256 x 256 upper-triangle tiles than the
machine runs at once, so a launch mixes whole-tile work-groups with tiles
split along K whose pieces are summed by a second kernel.  Every output
entry at N = 6144, and whole sampled rows at N = 16384 (every tile row that
holds a split tile among them), are compared with the FP64 product of exactly
the operands the kernel multiplies (the oracle's 16-bit rounding of the
centred matrix X - I/2), within the FP32 accumulation bound
(3n + 4) u sum|a||b| plus the rounding of the epilogue that restores the
layer."""

import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def pk():
    import paper_2107_02737_amd as pk
    pk.load_library()
    return pk


def _operands(x32, precision):
    """Hi/lo operands (FP64) of the centred matrix X - I/2 (rounded to FP32,
    then split, as the kernel's planes) and the scale of their products."""
    t32 = x32.copy()
    t32[np.diag_indices(t32.shape[0])] -= np.float32(0.5)
    if precision == "fp16x3":
        hi, lo = oracle.split_fp16_scaled(t32)
        return hi.astype(np.float64), lo.astype(np.float64), 2.0 ** (-2 * oracle.FP16_SPLIT_SCALE_LOG2)
    hi, lo = oracle.split_bf16(t32)
    return hi.astype(np.float64), lo.astype(np.float64), 1.0


def _rows_reference(x32, rows, precision):
    """Rows `rows` of the FP64 product of the split operands and of the
    accumulation bound (both signs share the product)."""
    hi, lo, s = _operands(x32, precision)
    ahi, alo = np.abs(hi), np.abs(lo)
    r = (hi[rows] @ hi + hi[rows] @ lo + lo[rows] @ hi) * s
    a = (ahi[rows] @ ahi + ahi[rows] @ alo + alo[rows] @ ahi) * s
    n = x32.shape[0]
    return r, (3 * n + 4) * U32 * a + 2 * U32 * np.abs(r)


def _check(y_rows, x_rows, rows, r, bound, sign):
    """The layer restored from the centred square: a T^2 + (b + a) X - (a/4) I
    with (a, b) = (1, 0) for X^2 and (-1, 2) for 2X - X^2."""
    x = x_rows.astype(np.float64)
    a, b = (1.0, 0.0) if sign > 0 else (-1.0, 2.0)
    ref = a * r + (b + a) * x
    ref[np.arange(len(rows)), rows] -= 0.25 * a
    bnd = bound + 4 * U32 * np.abs(x) + 4 * U32 * np.abs(ref)
    err = np.abs(y_rows - ref)
    worst = float(np.max(err / bnd))
    print(f"  sign={sign:+d} max|err| {err.max():.3e}  max err/bound {worst:.3f}", flush=True)
    assert np.all(err <= bnd)


def _water_input_layer():
    """S_0 of the benchmark's water box (1024 molecules, N = 6144): the
    spectrum of H mapped onto [0, 1] in reverse order, rounded to FP32."""
    from workloads import water_box_hamiltonian
    h = water_box_hamiltonian(1024, seed=0).astype(np.float32).astype(np.float64)
    lo, hi = oracle.gershgorin_bounds(h)
    x32 = oracle.input_layer(h, lo, hi).astype(np.float32)
    return np.triu(x32) + np.triu(x32, 1).T


@pytest.fixture(scope="module")
def water6144():
    return _water_input_layer()


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
def test_layer_every_entry_n6144(pk, water6144, precision):
    import torch
    x32 = water6144
    n = x32.shape[0]
    X = to_dev(x32)
    ws = pk.allocate_workspace(n)
    rows = np.arange(n)
    r, bound = _rows_reference(x32, rows, precision)
    for sign in (1, -1):
        banner(f"layer {precision} N={n} sign={sign} (every entry)")
        Y = torch.empty_like(X)
        pk.sp2_layer(X, precision, sign, Y, ws)
        y = to_host(Y)
        assert np.array_equal(y, y.T)
        _check(y, x32, rows, r, bound, sign)


def _tile_rows_of_tail(n, cus=256, band=4):
    """Tile rows that hold the tiles split along K: the library runs whole
    rounds of the machine unsplit and splits the tiles of the last partial
    round; logical tiles walk bands of `band` tile rows column by column."""
    nb = n // 256
    order = []
    for r0 in range(0, nb, band):
        r1 = min(r0 + band, nb) - 1
        for j in range(r0, nb):
            for i in range(r0, min(r1, j) + 1):
                order.append((i, j))
    rem = len(order) % cus
    tail = order[len(order) - rem:] if rem else []
    return sorted({i for i, _ in tail} | {j for _, j in tail})


def test_layer_sampled_rows_n16384(pk):
    import torch
    n = 16384
    rng = np.random.default_rng(11)
    a = rng.standard_normal((n, n), dtype=np.float32) * np.float32(0.01)
    x32 = (a + a.T) * np.float32(0.5)
    del a
    x32[np.diag_indices(n)] = rng.uniform(0.0, 1.0, n).astype(np.float32)
    tail_rows = _tile_rows_of_tail(n)
    assert tail_rows, "expected split tiles at N = 16384"
    # 8 rows from each tile row of a split tile, and from whole-tile rows
    picks = sorted(set(tail_rows) | {0, 17, 33, 50})
    rows = np.concatenate([256 * t + rng.choice(256, 8, replace=False) for t in picks])
    X = torch.from_numpy(x32).to("cuda")
    ws = pk.allocate_workspace(n)
    for precision in ("bf16x3", "fp16x3"):
        r, bound = _rows_reference(x32, rows, precision)
        for sign in (1, -1):
            banner(f"layer {precision} N={n} sign={sign} ({rows.size} sampled rows, tile rows {picks})")
            Y = torch.empty_like(X)
            pk.sp2_layer(X, precision, sign, Y, ws)
            ri = torch.from_numpy(rows).to("cuda")
            y_rows = Y.index_select(0, ri).double().cpu().numpy()
            yt_rows = Y.index_select(1, ri).t().double().cpu().numpy()
            assert np.array_equal(y_rows, yt_rows)          # the mirror write is exact
            _check(y_rows, x32[rows], rows, r, bound, sign)
            del Y
