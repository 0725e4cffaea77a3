"""Writes the stored expected values used by the full-size GPU tests and the
benchmark's error report.  Calls only the seeded generators and the FP64
oracle (``oracle.density_matrix_eigh``, ``oracle.gershgorin_bounds``,
``oracle.dmpt_response``).

water_m1024_seed0.npz -- tight-binding water box, 1024 molecules, seed 0,
N = 6144, n_occ = 4096, H cast to FP32 (the matrix the GPU receives).
Holds sampled entries of the exact density matrix P_ref = theta(mu I - H)
(Eq. 17-18): every diagonal entry and 8192 uniformly drawn (i, j) pairs
(rng seed 1234), plus the Gershgorin bounds, the HOMO/LUMO levels, the
ends of the spectrum and checksums of H that detect generator drift.

water_m682_n4096_deriv.npz -- derivative workload: 682 molecules (4092
orbitals) zero-padded to N = 4096, n_occ = 2728 (four doubly occupied states
per molecule), H cast to FP32; H1 = symmetric N(0, 1e-3^2) (seed 2) and
W = symmetric N(0, 1) (seed 1), both zero on the padding and cast to FP32.
Samples (diagonal + 8192 pairs) of P_ref, of the perturbation-theory
response P1 = dP/dH [H1] and of the gradient G = d Tr(W P)/dH (the same
self-adjoint map applied to W); the full inner product <W, P1>; and the
central finite difference of Tr(W P(H + h H1)) with h = 1e-4, every P from
FP64 diagonalisation.

water_m2730_n16384_traj.npz -- trajectory workload: 2730 molecules (16380
orbitals) zero-padded to N = 16384, n_occ = 10920, H0 cast to FP32,
H_p = (A + A^T)/(2 sqrt(2m)) (seed 3) cast to FP32, and
H(t) = H0 + fl32(a_t * H_p) with a_t = fl32(0.01 sin(0.1 t)) rounded
elementwise in FP32 (one product, one sum).  Samples of P_ref at t = 0 and
t = 99, and of G = d Tr(W P)/dH at t = 99 (W seed 1).

Run:  python tests/golden/make_golden.py [water6144|deriv4096|traj16384|all]
      (about 1, 1 and 15 minutes on 8 cores)
"""

import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import (symmetric_normal, trajectory_perturbation,  # noqa: E402
                       water_box_hamiltonian)

N_PAIRS = 8192


def _pairs(n, seed=1234):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, N_PAIRS), rng.integers(0, n, N_PAIRS)


def _samples(prefix, m, ri, rj):
    return {f"{prefix}_diag": np.diag(m).copy(), f"{prefix}_pair": m[ri, rj].copy()}


def water6144():
    m, seed, n_occ = 1024, 0, 4096
    h32 = water_box_hamiltonian(m, seed=seed).astype(np.float32)
    n = h32.shape[0]
    h = h32.astype(np.float64)
    p_ref, w, _ = oracle.density_matrix_eigh(h, n_occ)
    lo, hi = oracle.gershgorin_bounds(h)
    ri, rj = _pairs(n)
    np.savez_compressed(
        os.path.join(HERE, "water_m1024_seed0.npz"),
        n=n, n_occ=n_occ, molecules=m, seed=seed,
        diag=np.diag(p_ref).copy(),
        pair_i=ri.astype(np.uint16), pair_j=rj.astype(np.uint16), pair_val=p_ref[ri, rj],
        eps_min=lo, eps_max=hi, homo=w[n_occ - 1], lumo=w[n_occ], lam_min=w[0], lam_max=w[-1],
        h_sum=float(h.sum()), h_sumsq=float((h * h).sum()))
    print(f"wrote water_m1024_seed0.npz: gap={w[n_occ] - w[n_occ - 1]:.4f} bounds=({lo:.4f}, {hi:.4f})")


def deriv4096():
    m, n, n_occ, fd_step = 682, 4096, 2728, 1e-4
    h = water_box_hamiltonian(m, seed=0, n_pad=n).astype(np.float32).astype(np.float64)
    h1 = symmetric_normal(n, 2, std=1e-3, n_real=6 * m).astype(np.float32).astype(np.float64)
    wm = symmetric_normal(n, 1, n_real=6 * m).astype(np.float32).astype(np.float64)
    p_ref, w, v = oracle.density_matrix_eigh(h, n_occ)
    p1 = oracle.dmpt_response(h, n_occ, h1, eig=(w, v))
    g = oracle.dmpt_response(h, n_occ, wm, eig=(w, v))
    pp, _, _ = oracle.density_matrix_eigh(h + fd_step * h1, n_occ)
    pm, _, _ = oracle.density_matrix_eigh(h - fd_step * h1, n_occ)
    fd = (float(np.sum(wm * pp)) - float(np.sum(wm * pm))) / (2.0 * fd_step)
    lo, hi = oracle.gershgorin_bounds(h)
    ri, rj = _pairs(n)
    out = dict(n=n, n_occ=n_occ, molecules=m, seed=0, seed_w=1, seed_h1=2, h1_std=1e-3,
               fd_step=fd_step, pair_i=ri.astype(np.uint16), pair_j=rj.astype(np.uint16),
               eps_min=lo, eps_max=hi, homo=w[n_occ - 1], lumo=w[n_occ], lam_min=w[0], lam_max=w[-1],
               h_sum=float(h.sum()), h1_sum=float(h1.sum()), w_sum=float(wm.sum()),
               w_dot_p1=float(np.sum(wm * p1)), w_dot_p1_fd=fd,
               trace_p1=float(np.trace(p1)), p1_fro=float(np.linalg.norm(p1)),
               g_fro=float(np.linalg.norm(g)), w_dot_p=float(np.sum(wm * p_ref)))
    out.update(_samples("p", p_ref, ri, rj))
    out.update(_samples("p1", p1, ri, rj))
    out.update(_samples("g", g, ri, rj))
    np.savez_compressed(os.path.join(HERE, "water_m682_n4096_deriv.npz"), **out)
    print(f"wrote water_m682_n4096_deriv.npz: gap={w[n_occ] - w[n_occ - 1]:.4f} "
          f"<W,P1>={out['w_dot_p1']:.10e} fd={fd:.10e}")


def trajectory_coefficient(t):
    """``a_t`` of H(t) = H0 + a_t H_p, rounded to FP32."""
    return np.float32(0.01 * math.sin(0.1 * t))


def traj16384():
    m, n, n_occ = 2730, 16384, 10920
    t0 = time.time()
    h0 = water_box_hamiltonian(m, seed=0, n_pad=n, dtype=np.float32)
    hp = trajectory_perturbation(n, 3, n_real=6 * m, dtype=np.float32)
    ri, rj = _pairs(n)
    out = dict(n=n, n_occ=n_occ, molecules=m, seed=0, seed_hp=3, seed_w=1, times=np.array([0, 99]),
               pair_i=ri.astype(np.uint16), pair_j=rj.astype(np.uint16),
               h0_sum=float(h0.astype(np.float64).sum()), hp_sum=float(hp.astype(np.float64).sum()))
    print(f"generated H0, H_p ({time.time() - t0:.0f} s)", flush=True)
    for t in (0, 99):
        ht = (h0 + trajectory_coefficient(t) * hp).astype(np.float32)   # FP32 product, FP32 sum
        h = ht.astype(np.float64)
        del ht
        p_ref, w, v = oracle.density_matrix_eigh(h, n_occ)
        lo, hi = oracle.gershgorin_bounds(h)
        out.update({f"t{t}_eps_min": lo, f"t{t}_eps_max": hi, f"t{t}_homo": w[n_occ - 1],
                    f"t{t}_lumo": w[n_occ], f"t{t}_h_sum": float(h.sum())})
        out.update(_samples(f"t{t}_p", p_ref, ri, rj))
        del p_ref
        print(f"t={t}: eigh done ({time.time() - t0:.0f} s), gap={w[n_occ] - w[n_occ - 1]:.4f}",
              flush=True)
        if t == 99:
            wm = symmetric_normal(n, 1, n_real=6 * m, dtype=np.float32).astype(np.float64)
            g = oracle.dmpt_response(h, n_occ, wm, eig=(w, v))
            out.update(_samples("t99_g", g, ri, rj))
            out["t99_g_fro"] = float(np.linalg.norm(g))
            out["w_sum"] = float(wm.sum())
            del g, wm
        del v, h
    np.savez_compressed(os.path.join(HERE, "water_m2730_n16384_traj.npz"), **out)
    print(f"wrote water_m2730_n16384_traj.npz ({time.time() - t0:.0f} s)")


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    jobs = {"water6144": water6144, "deriv4096": deriv4096, "traj16384": traj16384}
    for name, fn in jobs.items():
        if which in (name, "all"):
            fn()


if __name__ == "__main__":
    main()
