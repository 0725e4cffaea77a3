"""The allocation-free solve (sp2_density_noalloc, the library's static
scratch in place of a caller workspace) against sp2_density_ex with a
caller workspace, through the C ABI: same kernels and the same work
decomposition, so P, the branch string and the info record agree bitwise.
Two calls in a row on the shared scratch, the second smaller and ragged
(leading dimension > n), so stale scratch contents from the first call
cannot leak into the second."""

import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev
from workloads import random_orthogonal_hamiltonian

pytestmark = pytest.mark.gpu

# (n, n_occ, precision, refine, bound_steps, ld, tolerance vs the FP64 oracle)
CASES = [(2048, 1024, "bf16x3", "fp32", 0, 2048, 3e-4),
         (1000, 300, "fp16x3", "split", 16, 1008, 3e-5)]


def test_noalloc_matches_workspace_entry_point():
    import torch

    import paper_2107_02737_amd as pk
    pk.load_library()
    for n, n_occ, precision, refine, bound_steps, ld, tol in CASES:
        banner(f"noalloc n={n} n_occ={n_occ} {precision} refine={refine} bound_steps={bound_steps} ld={ld}")
        h = random_orthogonal_hamiltonian(n, n_occ, occ_range=(-2.0, -0.1), virt_range=(0.1, 2.0),
                                          seed=n).astype(np.float32)
        H = to_dev(h, ld)
        opt = pk.make_options(precision, refine, bound_steps=bound_steps)
        ws = pk.allocate_workspace(n, opt)
        P_ws = to_dev(np.zeros((n, n), np.float32), ld)
        P_na = to_dev(np.full((n, n), np.nan, np.float32), ld)
        st1, info1, br1 = pk.sp2_density_ex(H, n_occ, opt, P_ws, ws)
        st2, info2, br2 = pk.sp2_density_noalloc(H, n_occ, opt, P_na)
        torch.cuda.synchronize()
        assert st1 == st2 == 0
        assert info1.converged == info2.converged == 1
        assert br1 == br2 and len(br2) == info2.n_iter > 0
        for f in ("n_iter", "eps_min", "eps_max", "trace", "idem_err"):
            assert getattr(info1, f) == getattr(info2, f), f
        assert torch.equal(P_ws, P_na)
        # padding columns of the caller's buffer stay untouched
        if ld > n:
            base = P_na.as_strided((n, ld), (ld, 1))
            assert torch.isnan(base[:, n:]).all()
        p_ref = oracle.density_matrix_eigh(h.astype(np.float64), n_occ)[0]
        err = oracle.error_metrics(P_na.double().cpu().numpy(), p_ref)["fro_over_sqrt_n"]
        print(f"  n_iter={info2.n_iter} ||P-P_ref||_F/sqrt(N)={err:.3e}", flush=True)
        assert err <= tol
