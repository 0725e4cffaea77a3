"""FP64 oracle for the recursive Fermi-operator expansion (DNN-SP2).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.

Paper: Finkelstein et al., "Quantum-based molecular dynamics simulations using
tensor cores" (arXiv 2107.02737).  Notation follows Section II.C-D:
``H`` is the (orthogonalised) Hamiltonian, ``D = theta(mu I - H)`` the density
matrix (Eq. 18), ``S_n`` the n-th density-matrix approximation of the network
``D = f(... f(W_1 f(W_0 X_0 + B_0) + B_1) ...)`` (Eq. 19) with activation
``f(X) = X^2``, ``X_n = f(S_{n-1})`` and ``S_n = W_n X_n + B_n``.

Everything here runs in FP64 except the explicit 16-bit rounding emulation.

Parity pins (what fixes each function other than itself; see tests/):

* ``density_matrix_eigh``   -- by-construction ``Q_occ Q_occ^T``; 2x2 closed
  form; diagonal H; n_occ in {0, N}; block-diagonal water vs 6x6 blocks.
* ``gershgorin_bounds``     -- brute-force loop on tiny matrices; enclosure of
  the spectrum; permutation and affine transformation rules.
* ``sp2``                   -- agreement with ``density_matrix_eigh``; scalar
  recursion on the eigenvalues (``sp2_scalar``) reproduces branches, traces
  and idempotency errors; invariants P^2 = P, Tr P = n_occ, [H, P] = 0;
  permutation equivariance; affine invariance with identical branches.
* ``sp2_jvp``               -- spectral divided-difference formula
  (``daleckii_krein_jvp``), first-order perturbation theory (``dmpt_response``)
  at convergence, central finite differences, Tr P1 = 0,
  P P1 + P1 P = P1, [H, P1] + [H1, P] = 0.
* ``sp2_vjp``               -- dot test against ``sp2_jvp`` and the identity
  VJP(W) = JVP(W) (the layer maps are self-adjoint and commute).
* ``split_*`` rounding      -- bit-exact against torch's CPU casts.
* ``mcweeny``               -- scalar closed form 3x^2 - 2x^3 on eigenvalues.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "density_matrix_eigh",
    "gershgorin_bounds",
    "input_layer",
    "choose_branch",
    "should_stop",
    "STALL_GATE",
    "QUAD_FACTOR",
    "sp2",
    "sp2_scalar",
    "mcweeny",
    "SP2Record",
    "apply_layer",
    "sp2_jvp",
    "sp2_vjp",
    "daleckii_krein_jvp",
    "dmpt_response",
    "finite_difference_jvp",
    "round_to_bf16",
    "round_to_fp16",
    "split_bf16",
    "split_fp16_scaled",
    "FP16_SPLIT_SCALE_LOG2",
    "error_metrics",
]

# Exponent of the power-of-two scale applied before the FP16 hi/lo split
# (keeps small matrix entries and their residuals out of the FP16 subnormal
# range).
FP16_SPLIT_SCALE_LOG2 = 14


# ---------------------------------------------------------------------------
# Plain definition of the result
# ---------------------------------------------------------------------------

def density_matrix_eigh(h, n_occ):
    """Density matrix by diagonalisation, Eq. (17) with occupation ``f_k = 1``
    for the ``n_occ`` lowest eigenstates and 0 otherwise, i.e. the matrix step
    function of Eq. (18) with the step between states ``n_occ`` and
    ``n_occ + 1``.  Returns ``(D, w, V)`` with ascending eigenvalues ``w``."""
    h = np.asarray(h, dtype=np.float64)
    w, v = np.linalg.eigh(h)
    vo = v[:, :n_occ]
    return vo @ vo.T, w, v


def gershgorin_bounds(h):
    """Gershgorin enclosure of the spectrum of a symmetric matrix:
    ``eps_min = min_i (H_ii - sum_{j != i} |H_ij|)`` and
    ``eps_max = max_i (H_ii + sum_{j != i} |H_ij|)``.  The paper maps the
    spectrum onto [0, 1] (Section II.D) without naming the bound estimate;
    Gershgorin discs are used here."""
    h = np.asarray(h, dtype=np.float64)
    d = np.diag(h).copy()
    off = np.abs(h)
    np.fill_diagonal(off, 0.0)
    r = off.sum(axis=1)
    return float(np.min(d - r)), float(np.max(d + r))


def input_layer(h, eps_min, eps_max):
    """First layer ``S_0 = W_0 X_0 + B_0`` with ``X_0 = H``,
    ``W_0 = -I / (eps_max - eps_min)`` and ``B_0 = eps_max I / (eps_max - eps_min)``:
    the spectrum is mapped linearly onto [0, 1] in reverse order (Section II.D)."""
    n = h.shape[0]
    w0 = -1.0 / (eps_max - eps_min)
    b0 = eps_max / (eps_max - eps_min)
    return w0 * np.asarray(h, dtype=np.float64) + b0 * np.eye(n)


def choose_branch(t1, t2, n_occ):
    """Sign of ``W_n`` (Section II.D, Fig. 1): ``+1`` gives ``S_n = S_{n-1}^2``,
    ``-1`` gives ``S_n = 2 S_{n-1} - S_{n-1}^2``.  The sign is chosen so that
    the trace of the next approximation lands closer to the occupation:
    ``Tr S^2 = t2`` versus ``Tr(2S - S^2) = 2 t1 - t2`` (ties take ``+``)."""
    return 1 if abs(t2 - n_occ) <= abs(2.0 * t1 - t2 - n_occ) else -1


def should_stop(k, errs, trace_gap, tol, stop_rule, stall_gate, stall_from=0):
    """Convergence test on the idempotency estimate ``e_k = |Tr S_k - Tr S_k^2|``
    (Section II.E: idempotency estimated from traces).

    No stop while ``trace_gap = |Tr S_k - n_occ| >= 1/2``: the approximation
    does not yet hold ``n_occ`` eigenvalues near 1 (an occupied eigenvalue can
    be driven close to 0 on the way, which makes ``e_k`` small long before
    convergence).  Otherwise rule 0 stops when ``e_k < tol``; rule 1 also
    stops once ``e_k < stall_gate`` when the last two layers no longer
    reduced the error as exact arithmetic would: ``e_k >= e_{k-2}`` or
    ``e_k >= QUAD_FACTOR e_{k-2}^2``.  With every eigenvalue in [0, 1],
    ``e_k < 3/16`` puts each within 1/4 of 0 or 1; together with the trace
    gap this also fixes which eigenvalues sit near 1.  There, with
    ``m = x (1 - x)`` an eigenvalue's share of ``e`` and its deviation from
    0 or 1 at most 1/4, a pair of layers of opposite sign maps ``m`` to at
    most ``(64/9) m^2`` (``4 m^2`` in the limit: ``2 d^2`` for a deviation
    ``d`` from 0 after ``+ -``, ``4 d^2`` after ``- +``, the mirror for
    deviations from 1), and the trace-closest rule squares the deviations of
    the side that dominates the trace, so ``e_k <= (64/9) e_{k-2}^2``: an
    ``e_k`` of ``16 e_{k-2}^2`` or more is mostly rounding, and the layers
    after it would only add more.
    ``stall_from``: the comparisons use only ``e_{k-2}`` with
    ``k - 2 >= stall_from`` (an accelerated schedule can raise ``e`` by
    itself before that, see ``oracle.accelerated``)."""
    if not trace_gap < 0.5:
        return False
    e = errs[k]
    if e < tol:
        return True
    if stop_rule == 1 and k >= 2 and k - 2 >= stall_from and e < stall_gate:
        ep = errs[k - 2]
        return e >= min(ep, QUAD_FACTOR * ep * ep)
    return False


STALL_GATE = 3.0 / 16.0
# Rule 1 stops when e_k >= QUAD_FACTOR e_{k-2}^2: above the exact-arithmetic bound
# e_k <= (64/9) e_{k-2}^2 below the gate (4 e_{k-2}^2 in the limit; see should_stop).
QUAD_FACTOR = 16.0


@dataclass
class SP2Record:
    """What one SP2 run recorded: bounds, branch signs (+1/-1 per applied layer),
    traces ``t1 = Tr S_k``, ``t2 = ||S_k||_F^2`` and ``e_k = |t1 - t2|`` for
    every examined approximation ``S_k`` (k = 0 .. n_iter), and whether the
    stop test passed."""
    eps_min: float
    eps_max: float
    branches: list = field(default_factory=list)
    t1: list = field(default_factory=list)
    t2: list = field(default_factory=list)
    err: list = field(default_factory=list)
    converged: bool = False
    refine: bool = False
    trivial: bool = False     # n_occ in {0, N}: P = 0 or I, independent of H
    coefs: list = field(default_factory=list)   # (a, b, c) per layer when not plain
    fallback: bool = False    # an accelerated network failed its end-of-schedule check

    @property
    def n_iter(self):
        return len(self.branches)

    @property
    def layer_coefs(self):
        """``(a, b, c)`` of every applied layer ``S_{k+1} = a S_k^2 + b S_k + c I``:
        the recorded ones, or ``(1, 0, 0)`` / ``(-1, 2, 0)`` from the signs of
        plain SP2 layers."""
        if len(self.coefs) == len(self.branches):
            return list(self.coefs)
        return [(1.0, 0.0, 0.0) if s > 0 else (-1.0, 2.0, 0.0) for s in self.branches]

    @property
    def branch_bits(self):
        """Branches as bytes: 1 for ``S^2`` and 0 for ``2S - S^2``."""
        return np.array([1 if s > 0 else 0 for s in self.branches], dtype=np.uint8)


def sp2(h, n_occ, tol=1e-10, max_iter=100, stop_rule=0, stall_gate=STALL_GATE,
        bounds=None, refine=False, return_iterates=False):
    """DNN-SP2 in FP64 (Eq. 19 and Fig. 1 of Section II.D).

    ``S_0`` maps the spectrum of ``H`` onto [0, 1] in reverse order; each
    following layer forms ``X_n = f(S_{n-1}) = S_{n-1}^2`` and
    ``S_n = W_n X_n + B_n`` with ``W_n = +-I`` and ``B_n = (I - W_n) S_{n-1}``.
    Before each layer the traces of the current approximation decide whether
    to stop (``should_stop``) and which sign to take (``choose_branch``).
    With ``refine`` one McWeeny purification ``3 S^2 - 2 S^3`` follows (the
    refinement step at the end of Section II.D).

    Returns ``(D, record)``; with ``return_iterates`` also the list of all
    ``S_k`` (k = 0 .. n_iter).
    """
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    if not 0 <= n_occ <= n:
        raise ValueError("n_occ out of range")
    eps_min, eps_max = gershgorin_bounds(h) if bounds is None else bounds
    rec = SP2Record(eps_min=eps_min, eps_max=eps_max, refine=refine)
    if n_occ == 0 or n_occ == n:
        rec.converged = True
        rec.trivial = True
        d = np.zeros((n, n)) if n_occ == 0 else np.eye(n)
        return (d, rec, [d]) if return_iterates else (d, rec)
    if not eps_max > eps_min:
        raise ValueError("degenerate spectrum: no gap to place the step in")
    s = input_layer(h, eps_min, eps_max)
    iterates = [s]
    for k in range(max_iter + 1):
        t1 = float(np.trace(s))
        t2 = float(np.sum(s * s))
        rec.t1.append(t1)
        rec.t2.append(t2)
        rec.err.append(abs(t1 - t2))
        if should_stop(k, rec.err, abs(t1 - n_occ), tol, stop_rule, stall_gate):
            rec.converged = True
            break
        if k == max_iter:
            break
        sign = choose_branch(t1, t2, n_occ)
        x = s @ s                                  # X_{k+1} = f(S_k)
        w = float(sign)                            # W_{k+1} = sign * I
        b = (1.0 - w) * s                          # B_{k+1} = (I - W_{k+1}) S_k
        s = w * x + b                              # S_{k+1}
        rec.branches.append(sign)
        if return_iterates:
            iterates.append(s)
    if refine:
        s = mcweeny(s)
    if return_iterates:
        return s, rec, iterates
    return s, rec


def sp2_scalar(w, n_occ, eps_min, eps_max, tol=1e-10, max_iter=100, stop_rule=0,
               stall_gate=STALL_GATE):
    """The same recursion applied to the eigenvalues ``w`` of ``H`` instead of
    the matrix: every layer acts on the spectrum only (the eigenvectors stay
    the same, Section II.C-D), so traces are plain sums over the mapped
    eigenvalues.  Returns ``(x_final, record)`` where ``x_final`` holds the
    polynomial ``p(x_i)`` for each mapped eigenvalue."""
    x = (eps_max - np.asarray(w, dtype=np.float64)) / (eps_max - eps_min)
    rec = SP2Record(eps_min=eps_min, eps_max=eps_max)
    for k in range(max_iter + 1):
        t1 = float(np.sum(x))
        t2 = float(np.sum(x * x))
        rec.t1.append(t1)
        rec.t2.append(t2)
        rec.err.append(abs(t1 - t2))
        if should_stop(k, rec.err, abs(t1 - n_occ), tol, stop_rule, stall_gate):
            rec.converged = True
            break
        if k == max_iter:
            break
        sign = choose_branch(t1, t2, n_occ)
        x = x * x if sign > 0 else 2.0 * x - x * x
        rec.branches.append(sign)
    return x, rec


def mcweeny(s):
    """McWeeny purification ``3 S^2 - 2 S^3`` (the refinement step cited in
    Section II.D): pushes eigenvalues near 0 and 1 closer to 0 and 1."""
    s2 = s @ s
    return 3.0 * s2 - 2.0 * (s @ s2)


# ---------------------------------------------------------------------------
# Derivatives with branches and bounds held fixed
# ---------------------------------------------------------------------------

def apply_layer(s, x, coef):
    """``S_{k+1} = a X + b S_k + c I`` with ``X = S_k^2`` (Eq. 19 with
    ``W = a I`` and ``B = b S_k + c I``; plain SP2 has ``(1, 0, 0)`` and
    ``(-1, 2, 0)``)."""
    a, b, c = coef
    out = a * x + b * s
    if c:
        out[np.diag_indices(s.shape[0])] += c
    return out


def _replay(h, rec):
    """All approximations ``S_0 .. S_L`` for the recorded bounds and layers."""
    s = input_layer(h, rec.eps_min, rec.eps_max)
    out = [s]
    for coef in rec.layer_coefs:
        s = apply_layer(s, s @ s, coef)
        out.append(s)
    return out


def sp2_jvp(h, h1, rec):
    """Forward derivative ``P_1 = dP/dH [H_1]`` of the recorded network (the
    density-matrix response needed by the XL-BOMD kernel of Section III).
    With the bounds fixed, ``dS_0 = -H_1 / (eps_max - eps_min)``; each layer
    differentiates to ``dS_n = S dS + dS S`` (sign +) or
    ``2 dS - (S dS + dS S)`` (sign -), in general ``a (S dS + dS S) + b dS``
    for the layer ``a S^2 + b S + c I``; the refinement contributes
    ``3 (S dS + dS S) - 2 (S^2 dS + S dS S + dS S^2)``."""
    h1 = np.asarray(h1, dtype=np.float64)
    n = h.shape[0]
    if rec.trivial:               # P does not depend on H
        return np.zeros((n, n))
    iters = _replay(h, rec)
    y = -h1 / (rec.eps_max - rec.eps_min)
    for (a, b, _), s in zip(rec.layer_coefs, iters[:-1]):
        sy = s @ y + y @ s
        y = a * sy + b * y
    if rec.refine:
        s = iters[-1]
        s2 = s @ s
        y = 3.0 * (s @ y + y @ s) - 2.0 * (s2 @ y + s @ y @ s + y @ s2)
    return y


def sp2_vjp(h, wmat, rec):
    """Reverse derivative: the symmetric ``G`` with
    ``Tr(G H_1) = Tr(W P_1)`` for every symmetric ``H_1``, i.e. the gradient of
    ``Tr(W P)`` with respect to ``H`` (bounds and branches fixed).  ``W`` is
    symmetrised first.  Walks the layers backwards: the adjoint of
    ``dS -> S dS + dS S`` is the same map, so ``G <- S G + G S`` (sign +) or
    ``2 G - (S G + G S)`` (sign -), in general ``a (S G + G S) + b G``,
    ending with ``-G / (eps_max - eps_min)``."""
    n = h.shape[0]
    if rec.trivial:               # P does not depend on H
        return np.zeros((n, n))
    g = 0.5 * (np.asarray(wmat, dtype=np.float64) + np.asarray(wmat, dtype=np.float64).T)
    iters = _replay(h, rec)
    if rec.refine:
        s = iters[-1]
        s2 = s @ s
        g = 3.0 * (s @ g + g @ s) - 2.0 * (s2 @ g + s @ g @ s + g @ s2)
    for (a, b, _), s in zip(reversed(rec.layer_coefs), reversed(iters[:-1])):
        sg = s @ g + g @ s
        g = a * sg + b * g
    return -g / (rec.eps_max - rec.eps_min)


def daleckii_krein_jvp(h, h1, rec):
    """Spectral form of the same derivative.  The network is a polynomial
    ``p`` of ``S_0``, which shares eigenvectors ``V`` with ``H``; the Frechet
    derivative of ``V p(x) V^T`` in direction ``X_1`` is
    ``V [Gamma o (V^T X_1 V)] V^T`` with the divided differences
    ``Gamma_ij = p[x_i, x_j]``.  Each divided difference is built layer by
    layer from the chain rule ``(g o f)[x, y] = g[f(x), f(y)] f[x, y]`` with
    ``[x, y] -> x + y`` for ``x^2`` and ``2 - x - y`` for ``2x - x^2``, in
    general ``a (x + y) + b`` for ``a x^2 + b x + c`` (and
    ``3(x+y) - 2(x^2 + x y + y^2)`` for the McWeeny step), which stays exact
    for close or equal eigenvalues."""
    w, v = np.linalg.eigh(np.asarray(h, dtype=np.float64))
    x = (rec.eps_max - w) / (rec.eps_max - rec.eps_min)
    gam = np.ones((x.size, x.size))
    u = x.copy()
    for a, b, c in rec.layer_coefs:
        uu = u[:, None] + u[None, :]
        gam *= a * uu + b
        u = a * (u * u) + (b * u + c)
    if rec.refine:
        a, b = u[:, None], u[None, :]
        gam *= 3.0 * (a + b) - 2.0 * (a * a + a * b + b * b)
    x1 = -np.asarray(h1, dtype=np.float64) / (rec.eps_max - rec.eps_min)
    return v @ (gam * (v.T @ x1 @ v)) @ v.T


def dmpt_response(h, n_occ, h1, eig=None):
    """First-order density-matrix perturbation theory at the exact step
    function: in the eigenbasis of ``H`` the response couples occupied ``i``
    and virtual ``a`` states only, ``(V^T P_1 V)_ia = (V^T H_1 V)_ia / (w_i - w_a)``.
    The map is self-adjoint, so for a symmetric ``W`` the same call gives the
    gradient of ``Tr(W P)`` with respect to ``H``.  ``eig = (w, V)`` reuses an
    eigendecomposition of ``H`` (ascending ``w``) instead of computing one."""
    if eig is None:
        w, v = np.linalg.eigh(np.asarray(h, dtype=np.float64))
    else:
        w, v = eig
    hv = v.T @ np.asarray(h1, dtype=np.float64) @ v
    m = np.zeros_like(hv)
    occ = slice(0, n_occ)
    vir = slice(n_occ, w.size)
    denom = w[occ][:, None] - w[vir][None, :]
    m[occ, vir] = hv[occ, vir] / denom
    m[vir, occ] = m[occ, vir].T
    return v @ m @ v.T


def finite_difference_jvp(h, n_occ, h1, step=1e-4, **sp2_kwargs):
    """Central difference ``(P(H + h H_1) - P(H - h H_1)) / 2h`` of the full
    FP64 ``sp2`` (bounds and branches free to change)."""
    pp, _ = sp2(np.asarray(h) + step * h1, n_occ, **sp2_kwargs)
    pm, _ = sp2(np.asarray(h) - step * h1, n_occ, **sp2_kwargs)
    return (pp - pm) / (2.0 * step)


# ---------------------------------------------------------------------------
# Dual (hi/lo) 16-bit representation, Eq. (20)-(21)
# ---------------------------------------------------------------------------

def round_to_bf16(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as
    FP32.  Works on the IEEE bit pattern: add ``0x7FFF`` plus the lowest kept
    bit, then clear the 16 low bits."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def round_to_fp16(x):
    """Round FP32 values to the nearest IEEE half (ties to even), as FP32."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def split_bf16(x):
    """Eq. (20)-(21) with bfloat16: ``X0 = BF16[X]``, ``X1 = BF16[X - X0]``
    (the difference is exact in FP32).  Returns FP32 arrays holding the
    bfloat16 values."""
    x = np.asarray(x, dtype=np.float32)
    hi = round_to_bf16(x)
    lo = round_to_bf16(x - hi)
    return hi, lo


def split_fp16_scaled(x, scale_log2=FP16_SPLIT_SCALE_LOG2):
    """Eq. (20)-(21) with IEEE half on the matrix scaled by ``2^scale_log2``:
    ``X0 = FP16[2^s X]``, ``X1 = FP16[2^s X - X0]``.  The power-of-two scale
    is exact and keeps small entries out of the half-precision subnormal
    range; products of the pair carry a factor ``2^(2s)``."""
    xs = np.asarray(x, dtype=np.float32) * np.float32(2.0 ** scale_log2)
    hi = round_to_fp16(xs)
    lo = round_to_fp16(xs - hi)
    return hi, lo


# ---------------------------------------------------------------------------
# Error report against the exact density matrix
# ---------------------------------------------------------------------------

def error_metrics(p, p_ref, h=None, n_occ=None):
    """Per-result accuracy figures: ``||P - P_ref||_F / sqrt(N)``,
    ``||P - P_ref||_F / N``, max-abs difference, ``||P^2 - P||_F / sqrt(N)``,
    ``|Tr P - n_occ|`` and ``||[H, P]||_F / sqrt(N)``."""
    p = np.asarray(p, dtype=np.float64)
    p_ref = np.asarray(p_ref, dtype=np.float64)
    n = p.shape[0]
    d = p - p_ref
    fro = float(np.linalg.norm(d))
    out = {
        "fro_over_sqrt_n": fro / math.sqrt(n),
        "fro_over_n": fro / n,
        "max_abs": float(np.max(np.abs(d))) if n else 0.0,
        "idempotency": float(np.linalg.norm(p @ p - p)) / math.sqrt(n),
    }
    if n_occ is not None:
        out["trace_err"] = abs(float(np.trace(p)) - n_occ)
    if h is not None:
        hh = np.asarray(h, dtype=np.float64)
        out["commutator"] = float(np.linalg.norm(hh @ p - p @ hh)) / math.sqrt(n)
    return out
