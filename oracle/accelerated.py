"""Accelerated DNN-SP2 with HOMO/LUMO estimates -- TEST INFRASTRUCTURE ONLY.

Imported by tests, the smoke check and the benchmark's CPU-baseline leg;
never by the product path.

Section II.E notes that the layer count of DNN-SP2 can be cut further (by up
to half) when estimates of the highest occupied and lowest unoccupied
eigenvalues are known beforehand, citing the accelerated (scaled and
shifted, nonmonotonic) recursive expansions of Rubensson and co-workers.
The paper gives no formulas.  Reading used here, derived from the spectral
picture of Section II.D:

* With the input layer of Eq. (19) the occupied eigenvalues of ``S_0`` lie
  in ``[h, 1]`` and the virtual ones in ``[0, l]``, where
  ``h = (eps_max - homo) / (eps_max - eps_min)`` and
  ``l = (eps_max - lumo) / (eps_max - eps_min)``, ``l < h`` (estimates:
  ``homo`` at or above the true HOMO, ``lumo`` at or below the true LUMO).
* A layer keeps the DNN form ``S_n = W_n X_n + B_n``, ``X_n = S_{n-1}^2``,
  now with ``W_n = a I`` and ``B_n = b S_{n-1} + c I``, i.e. the quadratic
  ``p(x) = a x^2 + b x + c`` on every eigenvalue.  The two families are
  ``p+(x) = ((x - s) / (1 - s))^2`` (pushes the virtual interval to 0,
  folding ``[0, l]`` about ``s``) and its mirror
  ``p-(x) = 1 - p+(1 - x)`` (pushes the occupied interval to 1), with shift
  ``0 <= s <= 1/2``.  ``s = 0`` gives the plain SP2 layers ``x^2`` and
  ``2x - x^2``; every such map sends [0, 1] into [0, 1].
* Schedule: ``+`` when the virtual interval is the wider one
  (``l >= 1 - h``), else ``-``; the shift is the fraction ``FOLD = 0.4`` of
  the width of the interval being folded (``s = 0.4 l`` for ``+``,
  ``0.4 (1 - h)`` for ``-``).  Half the width would minimise the folded
  interval's image (fewest layers), but each shift also widens the other
  side's distance from its target by ``1/(1 - s)``, which slows the growth
  of the gap between the two intervals and so amplifies early rounding
  more: in the FP32-storage emulation (water N = 1536 and a c2-type
  N = 1024, Gershgorin and Lanczos bounds, FP16 pairs) 0.5 cost up to 1.7x
  the plain network's error, 0.4 stayed within 0.8-1.4x of it at 15-24
  layers instead of 23-42.  The interval ends follow the
  same maps exactly, so the whole schedule is fixed by ``(l, h)`` before
  the first product.  It runs while ``max(l, 1 - h) >= ACC_END``; after it
  the trace-driven branch rule of plain DNN-SP2 takes over.
* Check at the end of the schedule: with estimates that bracket part of the
  gap, every eigenvalue has been driven to its side by then, so
  ``|Tr S - n_occ| < 1/2``.  If not, the estimates were wrong; the
  eigenvalues they put on the wrong side sit next to those of the right
  one (in finite precision they can no longer be told apart), so the
  iterate is dropped and the plain network runs from the start
  (``record.fallback``).
* The stop test and refinement are those of ``sp2_oracle.sp2``, with one
  change for rule 1 (comparisons of ``e_k`` with ``e_{k-2}``): inside the
  schedule ``e_k`` can rise by itself, or fall less than quadratically (two
  layers of the same sign, and each shift scales the other side's distance
  from its target by up to ``1/(1 - s)``), so the comparisons are allowed
  only from the iterate whose tracked width ``max(l_k, 1 - h_k)`` is below
  ``STALL_WIDTH`` (the remaining shifts are then below ``0.4 STALL_WIDTH``
  and the layers act as plain ones), or from the end of the schedule.

Pins (tests/test_oracle_accelerated.py): agreement with the diagonalisation
(``density_matrix_eigh``); the scalar recursion on the eigenvalues
(``sp2_accelerated_scalar``) reproduces traces and, through the spectral
theorem, P; each layer polynomial against its defining values (``p+(s) =
0``, ``p+(1) = 1``, ``p+'(s) = 0`` and the mirror); the interval ends are
images of eigenvalues placed exactly at them; [0, 1] maps into itself for
every shift; zero-width intervals give no schedule (plain SP2 bit for bit);
fewer layers than plain SP2 on the c1/water workloads (scalar probe: 26 ->
16, 28 -> 16 with Gershgorin bounds); estimates that miss the gap fail the
end-of-schedule check and end in the plain network's P.
"""

from __future__ import annotations

import numpy as np

from .sp2_oracle import (SP2Record, STALL_GATE, apply_layer, choose_branch, gershgorin_bounds,
                         input_layer, mcweeny, should_stop, sp2, sp2_scalar)

# The schedule stops once both mapped intervals are this close to 0 and 1.
ACC_END = 1e-14
# Shift of a layer as a fraction of the width of the interval it folds.
FOLD = 0.4
# Tracked width below which the stop rule may compare errors two layers apart.
STALL_WIDTH = 1e-4


def mapped_interval(eps_min, eps_max, homo, lumo):
    """``(l, h)``: upper end of the virtual and lower end of the occupied
    interval of ``S_0``, clipped to [0, 1]."""
    r = eps_max - eps_min
    lo = (eps_max - lumo) / r
    hi = (eps_max - homo) / r
    return min(max(lo, 0.0), 1.0), min(max(hi, 0.0), 1.0)


def layer_polynomial(sign, shift):
    """Coefficients ``(a, b, c)`` of ``p(x) = a x^2 + b x + c``:
    ``sign = +1``: ``((x - s)/(1 - s))^2``; ``sign = -1``:
    ``1 - ((1 - x - s)/(1 - s))^2``."""
    d = 1.0 - shift
    if sign > 0:
        return 1.0 / (d * d), -2.0 * shift / (d * d), shift * shift / (d * d)
    return -1.0 / (d * d), 2.0 / d, 0.0


def acceleration_schedule(l, h, max_len=100, end=ACC_END):
    """Signs and shifts of the accelerated layers for mapped interval ends
    ``(l, h)``, with the interval ends after each layer.  Returns a list of
    ``(sign, shift, l_after, h_after)``; empty when ``l >= h``."""
    out = []
    if not l < h:
        return out
    while len(out) < max_len and max(l, 1.0 - h) >= end:
        if l >= 1.0 - h:
            s = FOLD * l
            d = 1.0 - s
            q, r = max(s, l - s) / d, (h - s) / d
            l, h = q * q, r * r
            out.append((1, s, l, h))
        else:
            s = FOLD * (1.0 - h)
            d = 1.0 - s
            q, r = (1.0 - l - s) / d, max(s, 1.0 - h - s) / d
            l, h = 1.0 - q * q, 1.0 - r * r
            out.append((-1, s, l, h))
    return out


def stall_start(l, h, sched, width=STALL_WIDTH):
    """First iterate index whose tracked width ``max(l_k, 1 - h_k)`` is below
    ``width`` (``len(sched)`` if none is): from there the stagnation rule may
    compare errors."""
    w = max(l, 1.0 - h)
    for k, (_, _, lk, hk) in enumerate(sched):
        if w < width:
            return k
        w = max(lk, 1.0 - hk)
    return len(sched)


def _schedule(rec, homo, lumo, max_iter):
    l, h = mapped_interval(rec.eps_min, rec.eps_max, homo, lumo)
    sched = acceleration_schedule(l, h, max_iter)
    return ([layer_polynomial(sg, s) for sg, s, _, _ in sched],
            stall_start(l, h, sched) if sched else 0)


def sp2_accelerated(h, n_occ, homo, lumo, tol=1e-10, max_iter=100, stop_rule=0,
                    stall_gate=STALL_GATE, bounds=None, refine=False, return_iterates=False):
    """DNN-SP2 whose first layers follow the accelerated schedule of the
    estimates ``homo < lumo`` (energies), then the trace-driven rule.

    Returns ``(D, record)``; ``record.coefs`` holds ``(a, b, c)`` of every
    applied layer (``record.branches`` its sign)."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    if not 0 <= n_occ <= n:
        raise ValueError("n_occ out of range")
    if not homo < lumo:
        raise ValueError("need homo < lumo")
    eps_min, eps_max = gershgorin_bounds(h) if bounds is None else bounds
    rec = SP2Record(eps_min=eps_min, eps_max=eps_max, refine=refine)
    if n_occ == 0 or n_occ == n:
        rec.converged = True
        rec.trivial = True
        d = np.zeros((n, n)) if n_occ == 0 else np.eye(n)
        return (d, rec, [d]) if return_iterates else (d, rec)
    if not eps_max > eps_min:
        raise ValueError("degenerate spectrum: no gap to place the step in")
    sched, stall_from = _schedule(rec, homo, lumo, max_iter)
    s = input_layer(h, eps_min, eps_max)
    iterates = [s]
    for k in range(max_iter + 1):
        t1 = float(np.trace(s))
        t2 = float(np.sum(s * s))
        rec.t1.append(t1)
        rec.t2.append(t2)
        rec.err.append(abs(t1 - t2))
        if should_stop(k, rec.err, abs(t1 - n_occ), tol, stop_rule, stall_gate, stall_from):
            rec.converged = True
            break
        if k == max_iter:
            break
        if sched and k == len(sched) and not abs(t1 - n_occ) < 0.5:
            d, rec0 = sp2(h, n_occ, tol, max_iter, stop_rule, stall_gate, (eps_min, eps_max), refine)
            rec0.fallback = True
            return (d, rec0, None) if return_iterates else (d, rec0)
        if k < len(sched):
            a, b, c = sched[k]
        else:
            a, b, c = (1.0, 0.0, 0.0) if choose_branch(t1, t2, n_occ) > 0 else (-1.0, 2.0, 0.0)
        s = apply_layer(s, s @ s, (a, b, c))       # S_{k+1} = W f(S_k) + B
        rec.branches.append(1 if a > 0 else -1)
        rec.coefs.append((a, b, c))
        if return_iterates:
            iterates.append(s)
    if refine:
        s = mcweeny(s)
    if return_iterates:
        return s, rec, iterates
    return s, rec


def sp2_accelerated_scalar(w, n_occ, eps_min, eps_max, homo, lumo, tol=1e-10, max_iter=100,
                           stop_rule=0, stall_gate=STALL_GATE):
    """The same network on the eigenvalues ``w`` of ``H`` (every layer is a
    polynomial of ``S_0``, which shares the eigenvectors of ``H``).
    Returns ``(p(x), record)``."""
    x = (eps_max - np.asarray(w, dtype=np.float64)) / (eps_max - eps_min)
    rec = SP2Record(eps_min=eps_min, eps_max=eps_max)
    sched, stall_from = _schedule(rec, homo, lumo, max_iter)
    for k in range(max_iter + 1):
        t1 = float(np.sum(x))
        t2 = float(np.sum(x * x))
        rec.t1.append(t1)
        rec.t2.append(t2)
        rec.err.append(abs(t1 - t2))
        if should_stop(k, rec.err, abs(t1 - n_occ), tol, stop_rule, stall_gate, stall_from):
            rec.converged = True
            break
        if k == max_iter:
            break
        if sched and k == len(sched) and not abs(t1 - n_occ) < 0.5:
            x0, rec0 = sp2_scalar(w, n_occ, eps_min, eps_max, tol, max_iter, stop_rule, stall_gate)
            rec0.fallback = True
            return x0, rec0
        if k < len(sched):
            a, b, c = sched[k]
        else:
            a, b, c = (1.0, 0.0, 0.0) if choose_branch(t1, t2, n_occ) > 0 else (-1.0, 2.0, 0.0)
        x = a * (x * x) + b * x + c
        rec.branches.append(1 if a > 0 else -1)
        rec.coefs.append((a, b, c))
    return x, rec
