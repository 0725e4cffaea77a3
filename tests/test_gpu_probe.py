"""The matrix-core rate probe (include/sp2_probe.h) that bench.py runs beside
the layer kernel's roofline: on zero planes its products are exactly zero,
its clock counters advance, and the shader clock it reports lies in the
GPU's range."""

import ctypes

import numpy as np
import pytest

from gpu_util import banner

pytestmark = pytest.mark.gpu


def test_probe_runs_and_reports_clocks():
    import torch

    import paper_2107_02737_amd as pk
    from paper_2107_02737_amd.build import PROBE_PATH
    pk.load_library()
    lib = ctypes.CDLL(PROBE_PATH)
    f = lib.sp2_probe_mfma
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                  ctypes.c_void_p]
    n, nblocks, iters = 512, 8, 200
    banner(f"mfma probe n={n} blocks={nblocks} iters={iters}")
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.5, 0.5, (n, n)).astype(np.float32)
    X = torch.from_numpy((x + x.T) / 2).cuda()
    hi = torch.empty((n, n), dtype=torch.int16, device="cuda")
    lo = torch.empty_like(hi)
    sink = torch.full((nblocks * 256,), float("nan"), device="cuda")
    clocks = torch.zeros(4 * nblocks, dtype=torch.int64, device="cuda")
    hz = ctypes.c_double()
    for precision, code in (("fp16x3", 3), ("bf16x3", 2)):
        pk.sp2_split(X, precision, hi, lo)
        assert f(hi.data_ptr(), lo.data_ptr(), n, code, iters, nblocks, sink.data_ptr(),
                 clocks.data_ptr(), ctypes.byref(hz), None) == 0
        torch.cuda.synchronize()
        assert torch.isfinite(sink).all()
        c = clocks.view(nblocks, 4).cpu().numpy().astype(np.float64)
        assert (c[:, 2] > c[:, 0]).all() and (c[:, 3] > c[:, 1]).all()
        ghz = (c[:, 2] - c[:, 0]) / (c[:, 3] - c[:, 1]) * hz.value / 1e9
        print(f"  {precision}: shader clock {ghz.min():.2f}-{ghz.max():.2f} GHz "
              f"(wall clock {hz.value / 1e6:.0f} MHz)", flush=True)
        assert hz.value > 0 and (ghz > 0.3).all() and (ghz < 3.0).all()
    hi.zero_()
    lo.zero_()
    assert f(hi.data_ptr(), lo.data_ptr(), n, 3, iters, nblocks, sink.data_ptr(), clocks.data_ptr(),
             None, None) == 0
    torch.cuda.synchronize()
    assert (sink == 0).all()
