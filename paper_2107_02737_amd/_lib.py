"""ctypes binding of the C ABI in ``include/sp2.h`` (argument marshalling only).

Every function here has the name of the C entry point it calls and takes
torch tensors where the C side takes device pointers.  torch supplies device
memory and the current HIP stream; all computation runs in the library's
HIP kernels.  torch is imported before the library is loaded so that both
share one HIP runtime.
"""

from __future__ import annotations

import ctypes
import os

import torch

from .build import LIB_PATH

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p

SP2_OK = 0
SP2_ERR_INVALID_ARG = 1
SP2_ERR_NONFINITE = 2
SP2_ERR_NOT_CONVERGED = 3
SP2_ERR_WORKSPACE = 4
SP2_ERR_DEVICE = 5
SP2_ERR_TAPE = 6
STATUS_NAMES = {0: "SP2_OK", 1: "SP2_ERR_INVALID_ARG", 2: "SP2_ERR_NONFINITE",
                3: "SP2_ERR_NOT_CONVERGED", 4: "SP2_ERR_WORKSPACE", 5: "SP2_ERR_DEVICE",
                6: "SP2_ERR_TAPE"}

PRECISIONS = {"fp32": 0, "bf16x1": 1, "bf16x3": 2, "fp16x3": 3}
REFINES = {"none": 0, None: 0, False: 0, "fp32": 1, True: 1, "split": 2}
SP2_MAX_ITER = 256

# Every symbol include/sp2.h declares.
EXPORTED = ["sp2_default_options", "sp2_workspace_bytes", "sp2_density", "sp2_density_ex",
            "sp2_jvp", "sp2_vjp", "sp2_bounds", "sp2_spectral_bounds", "sp2_split", "sp2_layer",
            "sp2_mulliken", "sp2_xl_scratch_bytes", "sp2_xl_response", "sp2_xl_kernel",
            "sp2_nvt_gamma_tc", "sp2_nvt_first_half", "sp2_nvt_second_half", "sp2_last_error",
            "sp2_history", "sp2_density_noalloc", "sp2_homo_lumo"]
SP2_XL_MAX_RANK = 32


class sp2_options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("refine", c_int32), ("max_iter", c_int32),
                ("stop_rule", c_int32), ("checkpoint_every", c_int32), ("flags", c_int32),
                ("bound_steps", c_int32), ("bound_seed", c_int32),
                ("tol", c_double), ("stall_gate", c_double), ("homo", c_double),
                ("lumo", c_double)]


class sp2_info(ctypes.Structure):
    _fields_ = [("n_iter", c_int32), ("converged", c_int32), ("status", c_int32),
                ("fallback", c_int32), ("eps_min", c_double), ("eps_max", c_double),
                ("trace", c_double), ("idem_err", c_double), ("layer_ms", c_double),
                ("refine_ms", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class sp2_nvt_params(ctypes.Structure):
    _fields_ = [("dt", c_double), ("kt", c_double), ("gamma_tc", c_double),
                ("gamma_l", c_double), ("scheme", c_int32), ("reserved", c_int32)]


class SP2Error(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_LIB = None


def load_library(path=None):
    """Load ``libsp2.so`` (built in-tree by ``paper_2107_02737_amd.build.build()``).
    Fails loudly when it is missing: there is no fallback path."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2107_02737_amd.build.build() first")
    lib = ctypes.CDLL(path)
    vp = c_void_p
    lib.sp2_default_options.argtypes = [ctypes.POINTER(sp2_options)]
    lib.sp2_default_options.restype = None
    lib.sp2_workspace_bytes.argtypes = [c_int64, ctypes.POINTER(sp2_options)]
    lib.sp2_workspace_bytes.restype = c_size_t
    lib.sp2_density.argtypes = [vp, c_int64, c_int64, c_double, vp, ctypes.POINTER(c_int32), vp,
                                c_int32, vp, c_size_t, vp]
    lib.sp2_density.restype = c_int32
    lib.sp2_density_ex.argtypes = [vp, c_int64, c_int64, c_int64, ctypes.POINTER(sp2_options), vp,
                                   ctypes.POINTER(sp2_info), vp, c_int32, vp, c_size_t, vp]
    lib.sp2_density_ex.restype = c_int32
    lib.sp2_density_noalloc.argtypes = [vp, c_int64, c_int64, c_int64, ctypes.POINTER(sp2_options),
                                        vp, ctypes.POINTER(sp2_info), vp, c_int32, vp]
    lib.sp2_density_noalloc.restype = c_int32
    lib.sp2_jvp.argtypes = [vp, c_size_t, vp, c_int64, vp, vp]
    lib.sp2_jvp.restype = c_int32
    lib.sp2_vjp.argtypes = [vp, c_size_t, vp, c_int64, vp, vp]
    lib.sp2_vjp.restype = c_int32
    lib.sp2_bounds.argtypes = [vp, c_int64, c_int64, ctypes.POINTER(c_double),
                               ctypes.POINTER(c_double), vp, c_size_t, vp]
    lib.sp2_bounds.restype = c_int32
    lib.sp2_spectral_bounds.argtypes = [vp, c_int64, c_int64, c_int32, c_int32,
                                        ctypes.POINTER(c_double), ctypes.POINTER(c_double), vp,
                                        c_size_t, vp]
    lib.sp2_spectral_bounds.restype = c_int32
    lib.sp2_homo_lumo.argtypes = [vp, vp, c_int64, c_int64, c_int32, c_int32, c_double,
                                  ctypes.POINTER(c_double), ctypes.POINTER(c_double), vp, c_size_t, vp]
    lib.sp2_homo_lumo.restype = c_int32
    lib.sp2_split.argtypes = [vp, c_int64, c_int64, c_int32, vp, vp, vp]
    lib.sp2_split.restype = c_int32
    lib.sp2_layer.argtypes = [vp, c_int64, c_int64, c_int32, c_int32, vp, vp, c_size_t, vp]
    lib.sp2_layer.restype = c_int32
    lib.sp2_mulliken.argtypes = [vp, c_int64, c_int64, c_int64, vp, vp, vp, vp, vp]
    lib.sp2_mulliken.restype = c_int32
    lib.sp2_xl_scratch_bytes.argtypes = [c_int64, c_int64, c_int32]
    lib.sp2_xl_scratch_bytes.restype = c_size_t
    lib.sp2_xl_response.argtypes = [vp, c_size_t, c_int64, vp, vp, vp, vp, vp, c_size_t, vp]
    lib.sp2_xl_response.restype = c_int32
    lib.sp2_xl_kernel.argtypes = [vp, c_size_t, c_int64, vp, vp, vp, vp, c_int32, vp,
                                  ctypes.POINTER(c_double), ctypes.POINTER(c_int32), vp, c_size_t, vp]
    lib.sp2_xl_kernel.restype = c_int32
    lib.sp2_nvt_gamma_tc.argtypes = [c_double, c_double, c_double]
    lib.sp2_nvt_gamma_tc.restype = c_double
    lib.sp2_nvt_first_half.argtypes = [vp, vp, vp, vp, vp, c_int64,
                                       ctypes.POINTER(sp2_nvt_params), vp]
    lib.sp2_nvt_first_half.restype = c_int32
    lib.sp2_nvt_second_half.argtypes = [vp, vp, vp, c_int64, ctypes.POINTER(sp2_nvt_params), vp]
    lib.sp2_nvt_second_half.restype = c_int32
    lib.sp2_history.argtypes = [vp, c_size_t, c_int32, vp, vp, vp, vp, ctypes.POINTER(c_int32), vp]
    lib.sp2_history.restype = c_int32
    lib.sp2_last_error.argtypes = []
    lib.sp2_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _check(status, allow=()):
    if status != SP2_OK and status not in allow:
        msg = load_library().sp2_last_error().decode(errors="replace")
        raise SP2Error(status, msg)
    return status


def _dev_ptr(t, dtype=torch.float32, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major tensor")
    return c_void_p(t.data_ptr())


def _stream(device):
    return c_void_p(torch.cuda.current_stream(device).cuda_stream)


SP2_FLAG_TIME_LAYERS = 1
SP2_FLAG_SPLIT_DERIVATIVES = 2
SP2_FLAG_ACCELERATE = 4


def make_options(precision="bf16x3", refine="fp32", max_iter=100, stop_rule=1,
                 checkpoint_every=0, tol=1e-5, stall_gate=-1.0, time_layers=False,
                 bound_steps=0, bound_seed=0, split_derivatives=False, homo=None, lumo=None):
    """sp2_options; ``stall_gate`` < 0 selects the library's automatic gate.
    ``homo`` and ``lumo`` (both or neither) select the accelerated network
    (SP2_FLAG_ACCELERATE) with these eigenvalue estimates."""
    lib = load_library()
    o = sp2_options()
    lib.sp2_default_options(ctypes.byref(o))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.refine = REFINES[refine] if not isinstance(refine, int) or isinstance(refine, bool) else int(refine)
    o.max_iter = int(max_iter)
    o.stop_rule = int(stop_rule)
    o.checkpoint_every = int(checkpoint_every)
    o.tol = float(tol)
    o.stall_gate = float(stall_gate)
    o.flags = (SP2_FLAG_TIME_LAYERS if time_layers else 0) | \
        (SP2_FLAG_SPLIT_DERIVATIVES if split_derivatives else 0)
    o.bound_steps = int(bound_steps)
    o.bound_seed = int(bound_seed)
    if (homo is None) != (lumo is None):
        raise ValueError("give both homo and lumo, or neither")
    if homo is not None:
        o.flags |= SP2_FLAG_ACCELERATE
        o.homo = float(homo)
        o.lumo = float(lumo)
    return o


def sp2_default_options():
    o = sp2_options()
    load_library().sp2_default_options(ctypes.byref(o))
    return o


def sp2_workspace_bytes(n, opt=None):
    lib = load_library()
    return int(lib.sp2_workspace_bytes(int(n), ctypes.byref(opt) if opt is not None else None))


def allocate_workspace(n, opt=None, device=None):
    """Caller-owned device workspace (a torch uint8 tensor, 256-byte aligned)."""
    nbytes = sp2_workspace_bytes(n, opt)
    if nbytes == 0:
        raise SP2Error(SP2_ERR_INVALID_ARG, "invalid size or options")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def sp2_density(H, n_occ, tol, P, workspace, branches_cap=SP2_MAX_ITER):
    """Minimal form.  Returns ``(status, n_iter, branches)`` with ``branches`` a
    host ``bytes`` object (1 = S^2, 0 = 2S - S^2)."""
    lib = load_library()
    n = H.shape[0]
    n_iter = c_int32(0)
    br = (ctypes.c_uint8 * max(1, branches_cap))()
    st = lib.sp2_density(_dev_ptr(H, name="H"), n, int(n_occ), float(tol), _dev_ptr(P, name="P"),
                         ctypes.byref(n_iter), br, branches_cap,
                         c_void_p(workspace.data_ptr()), workspace.numel(), _stream(H.device))
    _check(st, allow=(SP2_ERR_NOT_CONVERGED,))
    return st, n_iter.value, bytes(br[:min(n_iter.value, branches_cap)])


def sp2_density_ex(H, n_occ, opt, P, workspace, branches_cap=SP2_MAX_ITER, check=True):
    """Full form.  ``H`` and ``P`` share the leading dimension ``H.stride(0)``.
    Returns ``(status, info, branches)``."""
    lib = load_library()
    n = H.shape[0]
    if P.stride(0) != H.stride(0):
        raise ValueError("H and P must have the same leading dimension")
    info = sp2_info()
    br = (ctypes.c_uint8 * max(1, branches_cap))()
    st = lib.sp2_density_ex(_dev_ptr(H, name="H"), n, H.stride(0), int(n_occ), ctypes.byref(opt),
                            _dev_ptr(P, name="P"), ctypes.byref(info), br, branches_cap,
                            c_void_p(workspace.data_ptr()), workspace.numel(), _stream(H.device))
    if check:
        _check(st, allow=(SP2_ERR_NOT_CONVERGED,))
    return st, info, bytes(br[:min(info.n_iter, branches_cap)])


def sp2_density_noalloc(H, n_occ, opt, P, branches_cap=SP2_MAX_ITER, check=True):
    """``sp2_density_ex`` on the library's static scratch (no workspace).
    Returns ``(status, info, branches)``."""
    lib = load_library()
    n = H.shape[0]
    if P.stride(0) != H.stride(0):
        raise ValueError("H and P must have the same leading dimension")
    info = sp2_info()
    br = (ctypes.c_uint8 * max(1, branches_cap))()
    st = lib.sp2_density_noalloc(_dev_ptr(H, name="H"), n, H.stride(0), int(n_occ),
                                 ctypes.byref(opt), _dev_ptr(P, name="P"), ctypes.byref(info), br,
                                 branches_cap, _stream(H.device))
    if check:
        _check(st, allow=(SP2_ERR_NOT_CONVERGED,))
    return st, info, bytes(br[:min(info.n_iter, branches_cap)])


def sp2_jvp(workspace, H1, P1):
    lib = load_library()
    _check(lib.sp2_jvp(c_void_p(workspace.data_ptr()), workspace.numel(), _dev_ptr(H1, name="H1"),
                       H1.stride(0), _dev_ptr(P1, name="P1"), _stream(H1.device)))
    return P1


def sp2_vjp(workspace, W, G):
    lib = load_library()
    _check(lib.sp2_vjp(c_void_p(workspace.data_ptr()), workspace.numel(), _dev_ptr(W, name="W"),
                       W.stride(0), _dev_ptr(G, name="G"), _stream(W.device)))
    return G


def sp2_bounds(H, workspace):
    lib = load_library()
    lo, hi = c_double(), c_double()
    _check(lib.sp2_bounds(_dev_ptr(H, name="H"), H.shape[0], H.stride(0), ctypes.byref(lo),
                          ctypes.byref(hi), c_void_p(workspace.data_ptr()), workspace.numel(),
                          _stream(H.device)))
    return lo.value, hi.value


def sp2_spectral_bounds(H, steps, workspace, seed=0):
    lib = load_library()
    lo, hi = c_double(), c_double()
    _check(lib.sp2_spectral_bounds(_dev_ptr(H, name="H"), H.shape[0], H.stride(0), int(steps),
                                   int(seed), ctypes.byref(lo), ctypes.byref(hi),
                                   c_void_p(workspace.data_ptr()), workspace.numel(),
                                   _stream(H.device)))
    return lo.value, hi.value


def sp2_split(X, precision, hi, lo):
    lib = load_library()
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib.sp2_split(_dev_ptr(X, name="X"), X.shape[0], X.stride(0), p,
                         _dev_ptr(hi, torch.int16, "hi"), _dev_ptr(lo, torch.int16, "lo"),
                         _stream(X.device)))
    return hi, lo


def sp2_layer(X, precision, sign, Y, workspace):
    lib = load_library()
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if Y.stride(0) != X.stride(0):
        raise ValueError("X and Y must have the same leading dimension")
    _check(lib.sp2_layer(_dev_ptr(X, name="X"), X.shape[0], X.stride(0), p, int(sign),
                         _dev_ptr(Y, name="Y"), c_void_p(workspace.data_ptr()), workspace.numel(),
                         _stream(X.device)))
    return Y


def sp2_history(workspace, cap=SP2_MAX_ITER + 1):
    """Per-layer record of the last solve on ``workspace``: a dict of lists
    ``t1`` (Tr S_k), ``t2`` (||S_k||_F^2) and ``err`` (|t1 - t2|) for
    k = 0 .. n_iter, and ``coef``, the ``(a, b, c)`` of every applied layer
    ``S_{k+1} = a S_k^2 + b S_k + c I``."""
    lib = load_library()
    t1, t2, err = (c_double * cap)(), (c_double * cap)(), (c_double * cap)()
    coef = (c_double * (3 * cap))()
    cnt = c_int32(0)
    _check(lib.sp2_history(c_void_p(workspace.data_ptr()), workspace.numel(), int(cap), t1, t2,
                           err, coef, ctypes.byref(cnt), _stream(workspace.device)))
    m = min(cnt.value, cap)
    nl = min(cnt.value - 1, cap)
    return {"t1": list(t1[:m]), "t2": list(t2[:m]), "err": list(err[:m]),
            "coef": [tuple(coef[3 * k:3 * k + 3]) for k in range(max(nl, 0))]}


def sp2_homo_lumo(H, P, workspace, steps=24, seed=0, margin=0.05):
    """Estimates ``(homo, lumo)`` of the highest occupied and lowest
    unoccupied eigenvalue of ``H`` from its density matrix ``P``."""
    lib = load_library()
    if P.stride(0) != H.stride(0) or P.shape != H.shape:
        raise ValueError("H and P must have the same shape and leading dimension")
    homo, lumo = c_double(), c_double()
    _check(lib.sp2_homo_lumo(_dev_ptr(H, name="H"), _dev_ptr(P, name="P"), H.shape[0], H.stride(0),
                             int(steps), int(seed), float(margin), ctypes.byref(homo),
                             ctypes.byref(lumo), c_void_p(workspace.data_ptr()), workspace.numel(),
                             _stream(H.device)))
    return homo.value, lumo.value


def sp2_last_error():
    return load_library().sp2_last_error().decode(errors="replace")


def _dev_vec(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D {dtype} tensor")
    return c_void_p(t.data_ptr())


def _charge_model_args(atom_ptr, gamma):
    na = atom_ptr.numel() - 1
    if na < 1:
        raise ValueError("atom_ptr needs n_atoms + 1 entries")
    if gamma.shape != (na, na) or gamma.dtype != torch.float64 or not gamma.is_contiguous():
        raise ValueError("gamma must be a contiguous n_atoms x n_atoms float64 device tensor")
    return na, _dev_vec(atom_ptr, torch.int64, "atom_ptr"), c_void_p(gamma.data_ptr())


def sp2_mulliken(P, atom_ptr, z, sub=None, q=None):
    """``q_I = z_I - 2 sum_{mu in I} P_mu,mu`` (minus ``sub`` if given)."""
    lib = load_library()
    na = atom_ptr.numel() - 1
    if q is None:
        q = torch.empty(na, dtype=torch.float64, device=P.device)
    _check(lib.sp2_mulliken(_dev_ptr(P, name="P"), P.shape[0], P.stride(0), na,
                            _dev_vec(atom_ptr, torch.int64, "atom_ptr"),
                            _dev_vec(z, torch.float64, "z"),
                            _dev_vec(sub, torch.float64, "sub") if sub is not None else None,
                            _dev_vec(q, torch.float64, "q"), _stream(P.device)))
    return q


def sp2_xl_scratch_bytes(n, n_atoms, rank):
    return int(load_library().sp2_xl_scratch_bytes(int(n), int(n_atoms), int(rank)))


def allocate_xl_scratch(n, n_atoms, rank, device=None):
    """Caller-owned device scratch of sp2_xl_response / sp2_xl_kernel."""
    nbytes = sp2_xl_scratch_bytes(n, n_atoms, rank)
    if nbytes == 0:
        raise SP2Error(SP2_ERR_INVALID_ARG, "invalid size or rank")
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def sp2_xl_response(workspace, atom_ptr, gamma, v, scratch, jv=None):
    """``J v = dq0/dn v - v`` at the taped H."""
    lib = load_library()
    na, ptr, g = _charge_model_args(atom_ptr, gamma)
    if jv is None:
        jv = torch.empty(na, dtype=torch.float64, device=v.device)
    _check(lib.sp2_xl_response(c_void_p(workspace.data_ptr()), workspace.numel(), na, ptr, g,
                               _dev_vec(v, torch.float64, "v"), _dev_vec(jv, torch.float64, "jv"),
                               c_void_p(scratch.data_ptr()), scratch.numel(), _stream(v.device)))
    return jv


def sp2_xl_kernel(workspace, atom_ptr, gamma, f, rank, scratch, k0=None, kf=None):
    """Rank-``rank`` Krylov approximation of ``K f = J^-1 f`` at the taped H.
    Returns ``(kf, rho, rank_used)`` (``rho`` a list of ``rank + 1`` floats)."""
    lib = load_library()
    na, ptr, g = _charge_model_args(atom_ptr, gamma)
    if kf is None:
        kf = torch.empty(na, dtype=torch.float64, device=f.device)
    if k0 is not None and (k0.shape != (na, na) or k0.dtype != torch.float64
                           or not k0.is_contiguous() or not k0.is_cuda):
        raise ValueError("k0 must be a contiguous n_atoms x n_atoms float64 device tensor")
    rank = int(rank)
    rho = (c_double * (max(rank, 0) + 1))()
    used = c_int32(0)
    _check(lib.sp2_xl_kernel(c_void_p(workspace.data_ptr()), workspace.numel(), na, ptr, g,
                             c_void_p(k0.data_ptr()) if k0 is not None else None,
                             _dev_vec(f, torch.float64, "f"), rank, _dev_vec(kf, torch.float64, "kf"),
                             rho, ctypes.byref(used), c_void_p(scratch.data_ptr()), scratch.numel(),
                             _stream(f.device)))
    return kf, list(rho), used.value


def nvt_params(dt, kt, gamma_tc=0.0, gamma_l=0.0, scheme=0):
    """sp2_nvt_params of one canonical integration step (Section IV)."""
    return sp2_nvt_params(float(dt), float(kt), float(gamma_tc), float(gamma_l), int(scheme), 0)


def sp2_nvt_gamma_tc(sigma_tc, kt, dt):
    """Friction balancing force noise of standard deviation sigma_tc (Eq. 33)."""
    return float(load_library().sp2_nvt_gamma_tc(float(sigma_tc), float(kt), float(dt)))


def _nvt_vec(t, n, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
            or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous float64 device tensor of {n} entries")
    return c_void_p(t.data_ptr())


def sp2_nvt_first_half(R, V, F, eta, mass, params):
    """In place: R <- R_{k+1}, V <- the velocity before the last half kick.
    ``eta`` may be None when the Langevin friction is 0."""
    n = R.numel()
    _check(load_library().sp2_nvt_first_half(
        _nvt_vec(R, n, "R"), _nvt_vec(V, n, "V"), _nvt_vec(F, n, "F"),
        _nvt_vec(eta, n, "eta") if eta is not None else None, _nvt_vec(mass, n, "mass"), n,
        ctypes.byref(params), _stream(R.device)))
    return R, V


def sp2_nvt_second_half(V, F, mass, params):
    """In place: V <- V_{k+1} from the intermediate velocity and F_{k+1}."""
    n = V.numel()
    _check(load_library().sp2_nvt_second_half(
        _nvt_vec(V, n, "V"), _nvt_vec(F, n, "F"), _nvt_vec(mass, n, "mass"), n,
        ctypes.byref(params), _stream(V.device)))
    return V
