"""The C-ABI library loads and exports every symbol include/sp2.h declares;
host-only argument checks behave as documented.  No GPU work is issued."""

import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sp2.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sp2_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2107_02737_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsp2.so is not built; run paper_2107_02737_amd.build.build()")
    return _lib.load_library()


def test_header_declares_expected_entry_points():
    from paper_2107_02737_amd import _lib
    assert _declared_functions() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    from paper_2107_02737_amd import _lib
    assert ctypes.sizeof(_lib.sp2_options) == 8 * 4 + 4 * 8
    assert ctypes.sizeof(_lib.sp2_info) == 4 * 4 + 6 * 8


def test_default_options(lib):
    from paper_2107_02737_amd import _lib
    o = _lib.sp2_default_options()
    assert (o.precision, o.refine, o.max_iter, o.stop_rule, o.checkpoint_every) == (2, 1, 100, 1, 0)
    assert o.tol == 1e-5 and o.stall_gate == -1.0
    assert (o.bound_steps, o.bound_seed, o.flags) == (0, 0, 0)
    assert (o.homo, o.lumo) == (0.0, 0.0)


def test_workspace_bytes(lib):
    from paper_2107_02737_amd import _lib
    o = _lib.sp2_default_options()
    n = 6144
    b = _lib.sp2_workspace_bytes(n, o)
    assert b >= 4 * n * n * 4                   # four padded FP32 slots
    # + split-K partial accumulators and two sets (the estimator's two sides)
    # of 67 Lanczos vectors of n doubles
    assert b < 4 * n * n * 4 + (65 << 20) + 2 * 67 * n * 8 + (1 << 20)
    o.checkpoint_every = 4
    bt = _lib.sp2_workspace_bytes(n, o)
    assert bt - b == (4 + 4 + 100 // 4 + 1) * n * n * 4
    assert _lib.sp2_workspace_bytes(1000, None) >= 4 * 1024 * 1024 * 4   # padded to 1024
    assert _lib.sp2_workspace_bytes(0, o) == 0
    o.max_iter = 0
    assert _lib.sp2_workspace_bytes(256, o) == 0
    o = _lib.sp2_default_options()
    o.bound_steps = 65
    assert _lib.sp2_workspace_bytes(256, o) == 0
    o.bound_steps = 7
    assert _lib.sp2_workspace_bytes(256, o) == 0
    for k in (8, 64):
        o.bound_steps = k
        assert _lib.sp2_workspace_bytes(256, o) > 0


def test_invalid_arguments_rejected_before_device_work(lib):
    from paper_2107_02737_amd import _lib
    fake = ctypes.c_void_p(0x1000)
    info = _lib.sp2_info()
    opt = _lib.sp2_default_options()
    br = (ctypes.c_uint8 * 4)()
    ws = ctypes.c_void_p(0x100000)
    # n_occ out of range
    st = lib.sp2_density_ex(fake, 8, 8, 9, ctypes.byref(opt), fake, ctypes.byref(info), br, 4,
                            ws, 1 << 30, None)
    assert st == _lib.SP2_ERR_INVALID_ARG and "n_occ" in _lib.sp2_last_error()
    # ld < n
    st = lib.sp2_density_ex(fake, 8, 4, 2, ctypes.byref(opt), fake, ctypes.byref(info), br, 4,
                            ws, 1 << 30, None)
    assert st == _lib.SP2_ERR_INVALID_ARG
    # bad option
    opt.precision = 7
    st = lib.sp2_density_ex(fake, 8, 8, 2, ctypes.byref(opt), fake, ctypes.byref(info), br, 4,
                            ws, 1 << 30, None)
    assert st == _lib.SP2_ERR_INVALID_ARG
    opt = _lib.sp2_default_options()
    opt.stall_gate = float("nan")           # a negative gate is the automatic one; NaN is not
    st = lib.sp2_density_ex(fake, 8, 8, 2, ctypes.byref(opt), fake, ctypes.byref(info), br, 4,
                            ws, 1 << 30, None)
    assert st == _lib.SP2_ERR_INVALID_ARG and "options" in _lib.sp2_last_error()
    opt = _lib.sp2_default_options()
    # workspace too small / misaligned / missing
    st = lib.sp2_density_ex(fake, 8, 8, 2, ctypes.byref(opt), fake, ctypes.byref(info), br, 4,
                            ws, 1024, None)
    assert st == _lib.SP2_ERR_WORKSPACE and "too small" in _lib.sp2_last_error()
    st = lib.sp2_density_ex(fake, 8, 8, 2, ctypes.byref(opt), fake, ctypes.byref(info), br, 4,
                            ctypes.c_void_p(0x100010), 1 << 30, None)
    assert st == _lib.SP2_ERR_WORKSPACE
    st = lib.sp2_density_ex(fake, 8, 8, 2, ctypes.byref(opt), fake, ctypes.byref(info), br, 4,
                            None, 1 << 30, None)
    assert st == _lib.SP2_ERR_WORKSPACE
    # NULL matrices, bad sign
    st = lib.sp2_density_ex(None, 8, 8, 2, ctypes.byref(opt), fake, ctypes.byref(info), br, 4,
                            ws, 1 << 30, None)
    assert st == _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_layer(fake, 8, 8, 2, 0, ctypes.c_void_p(0x2000), ws, 1 << 30, None) == \
        _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_split(fake, 8, 8, 0, fake, fake, None) == _lib.SP2_ERR_INVALID_ARG
    lo, hi = ctypes.c_double(), ctypes.c_double()
    for steps in (0, 7, 65):
        assert lib.sp2_spectral_bounds(fake, 8, 8, steps, 0, ctypes.byref(lo), ctypes.byref(hi),
                                       ws, 1 << 30, None) == _lib.SP2_ERR_INVALID_ARG


def test_history_rejects_bad_arguments(lib):
    from paper_2107_02737_amd import _lib
    buf = (ctypes.c_double * 4)()
    cnt = ctypes.c_int32(0)
    ws = ctypes.c_void_p(0x100000)
    assert lib.sp2_history(ws, 1 << 30, -1, buf, None, None, None, ctypes.byref(cnt), None) == \
        _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_history(ws, 1 << 30, 4, None, None, None, None, ctypes.byref(cnt), None) == \
        _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_history(None, 1 << 30, 4, buf, None, None, None, ctypes.byref(cnt), None) == \
        _lib.SP2_ERR_WORKSPACE
    assert lib.sp2_history(None, 1 << 30, 4, None, None, None, buf, ctypes.byref(cnt), None) == \
        _lib.SP2_ERR_WORKSPACE       # coefficients alone are a valid request
    assert lib.sp2_history(ctypes.c_void_p(0x100010), 1 << 30, 4, buf, None, None, None, None,
                           None) == _lib.SP2_ERR_WORKSPACE
    assert lib.sp2_history(ws, 64, 4, buf, None, None, None, None, None) == _lib.SP2_ERR_WORKSPACE


def test_xl_entry_points_reject_bad_arguments(lib):
    from paper_2107_02737_amd import _lib
    fake = ctypes.c_void_p(0x1000)
    assert lib.sp2_xl_scratch_bytes(0, 10, 4) == 0
    assert lib.sp2_xl_scratch_bytes(64, 10, 0) == 0
    assert lib.sp2_xl_scratch_bytes(64, 10, _lib.SP2_XL_MAX_RANK + 1) == 0
    small = lib.sp2_xl_scratch_bytes(64, 10, 1)
    # two n x n FP32 matrices, 2 rank + 5 charge vectors and the Krylov state
    assert small >= 2 * 64 * 64 * 4 + 7 * 10 * 8
    assert lib.sp2_xl_scratch_bytes(64, 10, 8) > small
    assert lib.sp2_mulliken(None, 8, 8, 2, fake, fake, None, fake, None) == _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_mulliken(fake, 8, 4, 2, fake, fake, None, fake, None) == _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_mulliken(fake, 8, 8, 0, fake, fake, None, fake, None) == _lib.SP2_ERR_INVALID_ARG
    rho = (ctypes.c_double * 40)()
    used = ctypes.c_int32()
    for rank in (0, _lib.SP2_XL_MAX_RANK + 1):
        st = lib.sp2_xl_kernel(fake, 1 << 30, 4, fake, fake, None, fake, rank, fake, rho,
                               ctypes.byref(used), fake, 1 << 30, None)
        assert st == _lib.SP2_ERR_INVALID_ARG and "rank" in _lib.sp2_last_error()
    st = lib.sp2_xl_kernel(fake, 1 << 30, 4, fake, fake, None, None, 2, fake, rho,
                           ctypes.byref(used), fake, 1 << 30, None)
    assert st == _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_xl_response(fake, 1 << 30, 4, fake, fake, None, fake, fake, 1 << 30, None) == \
        _lib.SP2_ERR_INVALID_ARG
    # checks that precede the tape read: missing charge model, misaligned scratch
    assert lib.sp2_xl_response(fake, 1 << 30, 4, None, fake, fake, fake, fake, 1 << 30, None) == \
        _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_xl_response(fake, 1 << 30, 4, fake, fake, fake, fake,
                               ctypes.c_void_p(0x1010), 1 << 30, None) == _lib.SP2_ERR_INVALID_ARG


def test_nvt_entry_points_reject_bad_arguments(lib):
    from paper_2107_02737_amd import _lib
    assert ctypes.sizeof(_lib.sp2_nvt_params) == 4 * 8 + 2 * 4
    fake = ctypes.c_void_p(0x1000)
    # Eq. 33: gamma_tc = sigma^2 dt / (2 kT); NaN outside the domain
    assert _lib.sp2_nvt_gamma_tc(0.3, 0.04, 0.5) == 0.3 * 0.3 * 0.5 / (2.0 * 0.04)
    for bad in ((-0.1, 0.04, 0.5), (0.1, 0.0, 0.5), (0.1, 0.04, 0.0), (float("nan"), 0.04, 0.5)):
        assert math.isnan(_lib.sp2_nvt_gamma_tc(*bad))

    def first(p, n=8, eta=fake):
        return lib.sp2_nvt_first_half(fake, fake, fake, eta, fake, n,
                                      ctypes.byref(p) if p is not None else None, None)

    good = _lib.nvt_params(0.5, 0.04, 0.1, 1e-3, 0)
    assert first(good, n=0) == _lib.SP2_OK                       # nothing to do, no launch
    assert first(None) == _lib.SP2_ERR_INVALID_ARG
    assert first(good, n=-1) == _lib.SP2_ERR_INVALID_ARG
    assert first(good, eta=None) == _lib.SP2_ERR_INVALID_ARG     # gamma_l > 0 needs eta
    assert "eta" in _lib.sp2_last_error()
    for p in (_lib.nvt_params(0.0, 0.04), _lib.nvt_params(0.5, -1.0), _lib.nvt_params(0.5, 0.04, -1),
              _lib.nvt_params(0.5, 0.04, 0.0, float("inf")), _lib.nvt_params(0.5, 0.04, scheme=2),
              _lib.nvt_params(float("nan"), 0.04)):
        assert first(p) == _lib.SP2_ERR_INVALID_ARG
        assert lib.sp2_nvt_second_half(fake, fake, fake, 8, ctypes.byref(p), None) == \
            _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_nvt_second_half(None, fake, fake, 8, ctypes.byref(good), None) == \
        _lib.SP2_ERR_INVALID_ARG


def test_noalloc_limits_rejected_before_device_work(lib):
    """sp2_density_noalloc refuses a tape, layer timing and orders whose
    workspace exceeds the static scratch, before any HIP call."""
    from paper_2107_02737_amd import _lib
    limit = 136 << 20
    o = _lib.sp2_default_options()
    assert _lib.sp2_workspace_bytes(2048, o) <= limit < _lib.sp2_workspace_bytes(2049, o)
    info = _lib.sp2_info()
    dummy = ctypes.c_void_p(256)

    def call(n, opt):
        return lib.sp2_density_noalloc(dummy, n, n, n // 2, ctypes.byref(opt), dummy,
                                       ctypes.byref(info), None, 0, None)
    assert call(2049, o) == _lib.SP2_ERR_INVALID_ARG
    assert "static scratch" in _lib.sp2_last_error()
    o.checkpoint_every = 4
    assert call(256, o) == _lib.SP2_ERR_INVALID_ARG
    o = _lib.sp2_default_options()
    o.flags = _lib.SP2_FLAG_TIME_LAYERS
    assert call(256, o) == _lib.SP2_ERR_INVALID_ARG
    o = _lib.sp2_default_options()
    assert call(0, o) == _lib.SP2_ERR_INVALID_ARG


def test_accelerate_option_checks(lib):
    """SP2_FLAG_ACCELERATE needs finite estimates with homo < lumo."""
    from paper_2107_02737_amd import _lib
    o = _lib.make_options("fp16x3", "split", homo=-0.5, lumo=-0.2)
    assert o.flags & _lib.SP2_FLAG_ACCELERATE
    assert _lib.sp2_workspace_bytes(512, o) > 0
    for h, l in ((-0.2, -0.5), (0.1, 0.1), (float("nan"), 0.0), (-float("inf"), 0.0)):
        o.homo, o.lumo = h, l
        assert _lib.sp2_workspace_bytes(512, o) == 0
    with pytest.raises(ValueError):
        _lib.make_options(homo=-0.5)


def test_homo_lumo_argument_checks(lib):
    """sp2_homo_lumo rejects bad arguments before any device work."""
    from paper_2107_02737_amd import _lib
    a, b = ctypes.c_double(), ctypes.c_double()
    dummy = ctypes.c_void_p(256)
    ws = ctypes.c_void_p(1 << 20)

    def call(n, ld, steps, margin):
        return lib.sp2_homo_lumo(dummy, dummy, n, ld, steps, 0, margin, ctypes.byref(a),
                                 ctypes.byref(b), ws, 1 << 40, None)
    assert call(0, 0, 16, 0.0) == _lib.SP2_ERR_INVALID_ARG
    assert call(64, 32, 16, 0.0) == _lib.SP2_ERR_INVALID_ARG
    assert call(64, 64, 7, 0.0) == _lib.SP2_ERR_INVALID_ARG
    assert call(64, 64, 65, 0.0) == _lib.SP2_ERR_INVALID_ARG
    assert call(64, 64, 16, 0.5) == _lib.SP2_ERR_INVALID_ARG
    assert call(64, 64, 16, -0.1) == _lib.SP2_ERR_INVALID_ARG
    assert lib.sp2_homo_lumo(None, dummy, 64, 64, 16, 0, 0.0, ctypes.byref(a), ctypes.byref(b), ws,
                             1 << 40, None) == _lib.SP2_ERR_INVALID_ARG



def test_probe_library_exports_and_rejects_bad_arguments():
    """The matrix-core rate probe beside the library (include/sp2_probe.h):
    every declared symbol is exported, and invalid arguments return 1 before
    anything is launched."""
    from paper_2107_02737_amd.build import PROBE_PATH
    if not os.path.exists(PROBE_PATH):
        pytest.fail("libsp2_probe.so is not built; run paper_2107_02737_amd.build.build()")
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "sp2_probe.h")).read(),
                  flags=re.S)
    names = sorted(set(re.findall(r"\b(sp2_[a-z_]+)\s*\(", text)))
    assert names == ["sp2_probe_mfma"]
    plib = ctypes.CDLL(PROBE_PATH)
    f = plib.sp2_probe_mfma
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                  ctypes.c_void_p]
    p = ctypes.c_void_p(256)   # never dereferenced: every call below fails its checks first
    ok = dict(hi=p, lo=p, np=512, precision=3, iters=10, nblocks=4, sink=p, clocks=p)
    bad = [dict(hi=None), dict(lo=None), dict(sink=None), dict(clocks=None), dict(np=300),
           dict(np=0), dict(precision=0), dict(precision=1), dict(iters=0), dict(nblocks=0),
           dict(nblocks=70000)]
    for b in bad:
        a = {**ok, **b}
        assert f(a["hi"], a["lo"], a["np"], a["precision"], a["iters"], a["nblocks"], a["sink"],
                 a["clocks"], None, None) == 1, b
