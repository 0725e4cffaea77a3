"""Lanczos refinement of the spectral bounds -- TEST INFRASTRUCTURE ONLY.

The paper maps the spectrum of H onto [0, 1] before the first layer
(Section II.D) without saying how the bounds are estimated.  Gershgorin discs
(``sp2_oracle.gershgorin_bounds``) are always valid but loose; the tighter
the interval, the larger the mapped HOMO-LUMO gap and the fewer layers the
network needs.  This module is the plain FP64 reference of the optional
tightening step: ``k`` steps of the symmetric Lanczos recurrence with full
reorthogonalisation (Golub and Van Loan, Matrix Computations, Sections 10.1
and 10.3) from a pseudo-random start vector, the extreme Ritz values of the
tridiagonal matrix, each widened by
its Ritz residual norm ``|beta_k s_k|`` and a relative safety margin, then
clipped to the Gershgorin interval.

Start vector: ``u_i = (z_i >> 11) * 2^-53 - 1/2`` with ``z_i`` the
SplitMix64 output (Steele, Lea and Flood, OOPSLA 2014) of state
``seed + (i + 1) * 0x9E3779B97F4A7C15``, normalised; both sides of the
comparison implement this generator from its published definition.

Pins (tests/test_oracle_lanczos.py): SplitMix64's published first outputs
for seed 0; the Lanczos relation ``H V = V T + beta_k v_{k+1} e_k^T`` and
orthonormality of ``V`` on small inputs; Ritz values equal to the
eigenvalues when ``k = N`` on a matrix with N distinct eigenvalues; the
residual formula against ``||H y - theta y||`` computed explicitly; and
enclosure of the spectrum (``numpy.linalg.eigvalsh``) on every workload.
"""

from __future__ import annotations

import numpy as np

from .sp2_oracle import gershgorin_bounds

SPLITMIX_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(seed, count):
    """The first ``count`` SplitMix64 outputs of state ``seed`` (Python ints)."""
    out = []
    for i in range(count):
        z = (seed + (i + 1) * SPLITMIX_GAMMA) & _M64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out.append(z ^ (z >> 31))
    return out


def start_vector(n, seed=0):
    """Normalised start vector ``u / ||u||`` with ``u_i`` uniform in [-1/2, 1/2)."""
    u = np.array([(z >> 11) * 2.0 ** -53 - 0.5 for z in splitmix64(seed, n)])
    return u / np.linalg.norm(u)


def lanczos(h, steps, seed=0, return_vectors=False):
    """``steps`` steps of the Lanczos recurrence on the symmetric ``h`` (FP64)
    with full reorthogonalisation (Golub and Van Loan Section 10.3): for
    ``w = H v_j``, two passes of classical Gram-Schmidt against
    ``V = [v_0 .. v_j]`` (``c = V^T w``, ``w -= V c``), the first pass giving
    ``alpha_j = c_j = v_j . H v_j`` (in exact arithmetic the same numbers as
    the three-term recurrence); ``beta_j = ||w||``,
    ``v_{j+1} = w * (1 / beta_j)``.  Stops early when ``beta_j`` vanishes
    (an invariant subspace was found).  Returns ``(alpha, beta)``
    (``beta[-1]`` couples to the next, unused vector), plus the Lanczos
    vectors ``V`` (N x (k+1)) if asked."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    vecs = [start_vector(n, seed)]
    alpha, beta = [], []
    for j in range(min(steps, n)):
        w = h @ vecs[j]
        basis = np.array(vecs).T
        c = basis.T @ w
        w = w - basis @ c
        w = w - basis @ (basis.T @ w)
        b = float(np.linalg.norm(w))
        alpha.append(float(c[j]))
        beta.append(b)
        if not b > 1e-300:
            break
        vecs.append(w * (1.0 / b))
    if return_vectors:
        return np.array(alpha), np.array(beta), np.array(vecs).T
    return np.array(alpha), np.array(beta)


def ritz_extremes(alpha, beta):
    """Smallest and largest eigenvalue of the Lanczos tridiagonal matrix and
    the residual norm ``|beta_k s_k|`` of each Ritz pair (``s_k``: last entry
    of the normalised eigenvector).  Returns ``(th_min, r_min, th_max, r_max)``."""
    k = len(alpha)
    t = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    th, s = np.linalg.eigh(t)
    r = np.abs(beta[k - 1] * s[-1, :])
    return float(th[0]), float(r[0]), float(th[-1]), float(r[-1])


def lanczos_bounds(h, steps, seed=0, margin=0.01):
    """Refined spectral bounds: ``[th_min - r_min - m, th_max + r_max + m]``
    with ``m = margin * (th_max - th_min)``, clipped to the Gershgorin
    interval (which stays the answer when ``steps`` is 0)."""
    g_lo, g_hi = gershgorin_bounds(h)
    if steps <= 0 or not g_hi > g_lo:
        return g_lo, g_hi
    alpha, beta = lanczos(h, steps, seed)
    th_lo, r_lo, th_hi, r_hi = ritz_extremes(alpha, beta)
    m = margin * (th_hi - th_lo)
    return max(g_lo, th_lo - r_lo - m), min(g_hi, th_hi + r_hi + m)


# ---------------------------------------------------------------------------
# HOMO/LUMO estimates from a density matrix (input of the accelerated
# network, Section II.E)
# ---------------------------------------------------------------------------

def projected_lanczos(h, p, side, steps, shift, seed=0):
    """Lanczos recurrence (as ``lanczos``) on the operator
    ``A v = Q ((H - shift I) v)`` with ``Q = P`` (``side = "occupied"``) or
    ``Q = I - P`` (``side = "virtual"``), started from ``Q u / ||Q u||``
    (``u`` the SplitMix64 start vector).  For a projector ``P`` commuting
    with ``H`` the vectors stay in the range of ``Q``, where ``A`` is
    ``H - shift I`` restricted to the occupied (virtual) eigenstates.
    Returns ``(alpha, beta)``."""
    h = np.asarray(h, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    n = h.shape[0]

    def q_of(y):
        py = p @ y
        return py if side == "occupied" else y - py

    u = q_of(start_vector(n, seed))
    vecs = [u * (1.0 / float(np.linalg.norm(u)))]
    alpha, beta = [], []
    for j in range(min(steps, n)):
        w = q_of(h @ vecs[j] - shift * vecs[j])
        basis = np.array(vecs).T
        c = basis.T @ w
        w = w - basis @ c
        w = w - basis @ (basis.T @ w)
        b = float(np.linalg.norm(w))
        alpha.append(float(c[j]))
        beta.append(b)
        if not b > 1e-300:
            break
        vecs.append(w * (1.0 / b))
    return np.array(alpha), np.array(beta)


def homo_lumo_estimates(h, p, steps=24, seed=0, margin=0.05, bounds=None):
    """Estimates of the highest occupied and lowest unoccupied eigenvalue of
    ``H`` from a density matrix ``P`` of it: the largest eigenvalue of
    ``H`` on the range of ``P`` and the smallest on the range of ``I - P``,
    each from ``steps`` Lanczos steps (``projected_lanczos``; shifts
    ``eps_min`` and ``eps_max``, the spectral bounds, so that the zero
    eigenvalue of the complement stays on the inner side), widened outwards
    by its Ritz residual norm (HOMO up, LUMO down), then the interval
    between them shrunk by ``margin`` of its width on each side.  Returns
    ``(homo, lumo)``, or ``None`` when no gap remains."""
    eps_min, eps_max = gershgorin_bounds(h) if bounds is None else bounds
    a, b = projected_lanczos(h, p, "occupied", steps, eps_min, seed)
    _, _, th_hi, r_hi = ritz_extremes(a, b)
    a, b = projected_lanczos(h, p, "virtual", steps, eps_max, seed)
    th_lo, r_lo, _, _ = ritz_extremes(a, b)
    homo = th_hi + eps_min + r_hi
    lumo = th_lo + eps_max - r_lo
    gap = lumo - homo
    if not gap > 0.0:
        return None
    return homo + margin * gap, lumo - margin * gap
