"""Writes the stored expected values used by the full-size GPU tests and the
benchmark's error report.  Calls only the seeded generators and the FP64
oracle (``oracle.density_matrix_eigh``, ``oracle.gershgorin_bounds``).

water_m1024_seed0.npz -- tight-binding water box, 1024 molecules, seed 0,
N = 6144, n_occ = 4096, H cast to FP32 (the matrix the GPU receives).
Holds sampled entries of the exact density matrix P_ref = theta(mu I - H)
(Eq. 17-18): every diagonal entry and 8192 uniformly drawn (i, j) pairs
(rng seed 1234), plus the Gershgorin bounds, the HOMO/LUMO gap and
checksums of H that detect generator drift.

Run:  python tests/golden/make_golden.py   (about a minute on 8 cores)
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import water_box_hamiltonian  # noqa: E402


def main():
    m, seed, n_occ = 1024, 0, 4096
    h32 = water_box_hamiltonian(m, seed=seed).astype(np.float32)
    n = h32.shape[0]
    h = h32.astype(np.float64)
    p_ref, w, _ = oracle.density_matrix_eigh(h, n_occ)
    lo, hi = oracle.gershgorin_bounds(h)
    rng = np.random.default_rng(1234)
    ri = rng.integers(0, n, 8192)
    rj = rng.integers(0, n, 8192)
    np.savez_compressed(
        os.path.join(HERE, "water_m1024_seed0.npz"),
        n=n, n_occ=n_occ, molecules=m, seed=seed,
        diag=np.diag(p_ref).copy(),
        pair_i=ri.astype(np.uint16), pair_j=rj.astype(np.uint16), pair_val=p_ref[ri, rj],
        eps_min=lo, eps_max=hi, homo=w[n_occ - 1], lumo=w[n_occ],
        h_sum=float(h.sum()), h_sumsq=float((h * h).sum()))
    print(f"wrote water_m1024_seed0.npz: gap={w[n_occ] - w[n_occ - 1]:.4f} bounds=({lo:.4f}, {hi:.4f})")


if __name__ == "__main__":
    main()
