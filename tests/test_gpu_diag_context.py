"""The GPU diagonalisation that bench.py times beside the SP2 solver for
context (the comparison of Fig. 2: a dense eigensolver plus the occupied
outer product of Eq. 17) gives the oracle's density matrix: FP64 to
rounding, FP32 to the single-precision eigenvector accuracy."""

import os
import sys

import numpy as np
import pytest

import oracle
from gpu_util import banner
from workloads import water_box_hamiltonian

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def test_diagonalization_context_matches_the_oracle():
    import torch

    import bench
    h32 = water_box_hamiltonian(128, seed=3).astype(np.float32)   # N = 768
    n = h32.shape[0]
    n_occ = 2 * n // 3
    banner(f"diagonalisation context water N={n}")
    p_ref, _, _ = oracle.density_matrix_eigh(h32.astype(np.float64), n_occ)
    out = bench.diagonalization_baseline(torch.from_numpy(h32).to("cuda"), n_occ, p_ref)
    print(f"  float32 {out['float32']['fro_over_sqrt_n']:.3e} "
          f"float64 {out['float64']['fro_over_sqrt_n']:.3e}", flush=True)
    assert out["float64"]["fro_over_sqrt_n"] <= 1e-12
    assert out["float32"]["fro_over_sqrt_n"] <= 1e-4
    assert out["float32"]["seconds"] > 0.0 and out["float64"]["seconds"] > 0.0
