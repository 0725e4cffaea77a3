"""Rounding-level emulation of the GPU precision modes -- TEST INFRASTRUCTURE.

Runs the same DNN-SP2 network as ``sp2_oracle.sp2`` but stores every iterate
in FP32 and forms each square from the dual 16-bit representation of
Eq. (20)-(22) of the centred iterate ``S - I/2`` (or plain FP32), with FP32
accumulation (NumPy ``float32`` matmul), restoring the square in FP32
(``layer_emulated``).  Used only to predict the error floor each precision mode reaches
against the exact density matrix, from which the end-to-end test
tolerances are derived.  The accumulation order differs from the GPU's
MFMA, so agreement with the GPU is statistical, not bitwise
(parity unpinned for bitwise equality).

Pins (tests/test_oracle_emulation.py): on operands exactly representable in
each mode, ``square_emulated`` equals the exact FP64 sum of the products of
Eq. (22) (with the 2^-28 rescale for the scaled FP16 pair; X0 X0 alone for the
single pass); ``layer_emulated`` equals the exact layer ``a S^2 + b S + c I``
on iterates whose centred matrix and products are exact in every mode;
``automatic_stall_gate`` against closed forms;
``sp2_emulated("fp32")`` bitwise against a plain FP32 loop written out in
the test (plain and accelerated); every mode's error against the exact
density matrix within [1/64, 2] of its operand roundoff times the
Gershgorin width (plain and accelerated); estimates outside the spectrum
leave the plain network bit for bit.
"""

from __future__ import annotations

import numpy as np

from .accelerated import acceleration_schedule, layer_polynomial, mapped_interval, stall_start
from .sp2_oracle import (FP16_SPLIT_SCALE_LOG2, STALL_GATE, choose_branch, gershgorin_bounds,
                         should_stop, split_bf16, split_fp16_scaled)

MODES = ("fp32", "bf16x1", "bf16x3", "fp16x3")

# The split modes represent a network iterate S by the planes of S - cI,
# c = PLANE_CENTRE: its eigenvalues lie in [-1/2, 1/2] and its diagonal
# entries (near 0 or 1 for S near a density matrix) shrink, and with them
# the FP32 partial sums of each product and the 16-bit roundings.
PLANE_CENTRE = 0.5


def square_emulated(x, mode):
    """``X^2`` of an FP32 symmetric matrix in the given arithmetic, FP32 result.
    Split modes use Eq. (22): ``X0 X0 + X0 X1 + X1 X0`` (``X1 X1`` dropped)."""
    x = np.asarray(x, dtype=np.float32)
    if mode == "fp32":
        return x @ x
    if mode == "bf16x1":
        hi, _ = split_bf16(x)
        return hi @ hi
    if mode == "bf16x3":
        hi, lo = split_bf16(x)
        return hi @ hi + (hi @ lo + lo @ hi)
    if mode == "fp16x3":
        hi, lo = split_fp16_scaled(x)
        return (hi @ hi + (hi @ lo + lo @ hi)) * np.float32(2.0 ** (-2 * FP16_SPLIT_SCALE_LOG2))
    raise ValueError(mode)


def layer_emulated(s, mode, a, b, c):
    """One layer ``a S^2 + b S + c I`` of an FP32 symmetric iterate in the
    given arithmetic, FP32 result.  The split modes square the centred
    matrix ``T = S - PLANE_CENTRE I`` (rounded to FP32, then to its planes)
    and restore ``S^2 = T^2 + 2c S - c^2 I`` (c = PLANE_CENTRE) in FP32:
    ``a T^2 + (b + 2c a) S + (c' - c^2 a) I``."""
    s = np.asarray(s, dtype=np.float32)
    diag = np.diag_indices(s.shape[0])
    if mode == "fp32":
        out = np.float32(a) * square_emulated(s, mode).astype(np.float32) + np.float32(b) * s
        if c != 0.0:
            out[diag] += np.float32(c)
        return out
    t = s.copy()
    t[diag] -= np.float32(PLANE_CENTRE)
    sq = square_emulated(t, mode).astype(np.float32)
    out = np.float32(a) * sq + np.float32(b + 2.0 * PLANE_CENTRE * a) * s
    out[diag] += np.float32(c - PLANE_CENTRE * PLANE_CENTRE * a)
    return out


# Significant bits of the layer operands in each mode: a BF16 value carries 8,
# an FP16 value 11, the hi/lo pairs twice that, FP32 24.
OPERAND_BITS = {"bf16x1": 8, "bf16x3": 16, "fp16x3": 22, "fp32": 24}


def automatic_stall_gate(n, mode):
    """Default gate of the stagnation test for an ``n x n`` problem in
    ``mode``: the larger of 3/16 (below it every eigenvalue of the iterate is
    within 1/4 of 0 or 1, see ``should_stop``) and ``n u / 16`` with ``u`` the
    unit roundoff of the layer operands, which keeps the gate above the
    rounding floor of the error estimate (measured with this emulation: about
    0.06 n u for single BF16 operands at n = 1536 and 6144)."""
    u = 2.0 ** (-OPERAND_BITS[mode])
    return max(STALL_GATE, n * u / 16.0)


def sp2_emulated(h, n_occ, mode, tol=1e-5, max_iter=100, stop_rule=1, stall_gate=None,
                 refine=True, bounds=None, homo=None, lumo=None):
    """FP32-stored DNN-SP2 with the layer squares of ``mode``; the traces,
    bounds and decisions are FP64 as on the GPU.  ``bounds`` overrides the
    Gershgorin bounds; ``stall_gate=None`` takes ``automatic_stall_gate``.
    With ``homo`` and ``lumo`` the first layers follow the accelerated
    schedule (``oracle.accelerated``), ``S <- a S^2 + b S + c I`` with the
    coefficients rounded to FP32 and ``c`` added to the diagonal, and the
    end-of-schedule trace check falls back to the plain network.
    Returns ``(P, n_iter)``."""
    h = np.asarray(h, dtype=np.float32)
    n = h.shape[0]
    if stall_gate is None:
        stall_gate = automatic_stall_gate(n, mode)
    lo_b, hi_b = gershgorin_bounds(h.astype(np.float64)) if bounds is None else bounds
    s = ((hi_b * np.eye(n) - h.astype(np.float64)) / (hi_b - lo_b)).astype(np.float32)
    sched, stall_from = [], 0
    if homo is not None:
        l, hh = mapped_interval(lo_b, hi_b, homo, lumo)
        steps = acceleration_schedule(l, hh, max_iter)
        sched = [layer_polynomial(sg, sh) for sg, sh, _, _ in steps]
        if steps:
            stall_from = stall_start(l, hh, steps)
    diag = np.diag_indices(n)
    errs = []
    layers = 0
    for k in range(max_iter + 1):
        sd = s.astype(np.float64)
        t1 = float(np.trace(sd))
        t2 = float(np.sum(sd * sd))
        errs.append(abs(t1 - t2))
        if should_stop(k, errs, abs(t1 - n_occ), tol, stop_rule, stall_gate, stall_from) \
                or k == max_iter:
            break
        if sched and k == len(sched) and not abs(t1 - n_occ) < 0.5:
            # end-of-schedule check failed: the plain network from the start
            return sp2_emulated(h, n_occ, mode, tol, max_iter, stop_rule, stall_gate, refine,
                                (lo_b, hi_b))
        if k < len(sched):
            a, b, c = sched[k]
        else:
            a, b, c = (1.0, 0.0, 0.0) if choose_branch(t1, t2, n_occ) > 0 else (-1.0, 2.0, 0.0)
        s = layer_emulated(s, mode, a, b, c)
        s = np.triu(s) + np.triu(s, 1).T          # upper triangle mirrored, as computed
        layers += 1
    if refine:
        s2 = s @ s
        s = np.float32(3.0) * s2 - np.float32(2.0) * (s @ s2)
    return s, layers
