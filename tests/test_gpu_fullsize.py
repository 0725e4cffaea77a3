"""Full-size parity at the benchmark's workload (water box, N = 6144,
n_occ = 4096) in the launch configuration bench.py times.  The exact density
matrix P_ref = theta(mu I - H) of the FP32 H the GPU receives comes from the
FP64 oracle's diagonalisation at test time, and every entry of the GPU's P
is compared with it: ||P - P_ref||_F / sqrt(N) and max |P - P_ref|, plus
properties that hold at any size.  Stored checksums detect generator drift."""

import math
import os

import numpy as np
import pytest

import oracle
from gpu_util import banner

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "water_m1024_seed0.npz")

# ||P - P_ref||_F / sqrt(N): 3x the FP32-storage emulation of a 256-molecule
# box of the same model (the error is set by the mapped gap, which the larger
# box shares).
TOL = {"bf16x3": 5e-5, "fp16x3": 3e-6, "fp32": 3e-6}
# The stated bound for the FP32-equivalent mode (split hi/lo layers with the
# refinement): ||P - P_ref||_F / sqrt(N) <= 1e-6.  FP16x3 layers with the
# refinement in the same FP16x3 arithmetic reach it once the Lanczos bounds
# widen the mapped gap (8, 16, 32 and 64 steps).  An FP32
# refinement adds its own FP32 MFMA rounding (1.2e-6), so it is held to the
# FP16x3 tolerance only.
FP32_EQUIVALENT = [("fp16x3", 8, "split"), ("fp16x3", 16, "split"), ("fp16x3", 32, "split"),
                   ("fp16x3", 64, "split")]
# Lanczos steps of the benchmark's bounds (bench.py --bound-steps): on this
# box they enclose the spectrum [-4.867, 0.615] as (-5.090, 0.666).
BENCH_BOUND_STEPS = 8
FP32_EQUIVALENT_TOL = 1e-6
# max |P - P_ref| is about 3x ||P - P_ref||_F / sqrt(N) in the emulation
# (N = 1536, every mode); allowed: 6x the Frobenius tolerance.
MAX_ABS_FACTOR = 6.0


@pytest.fixture(scope="module")
def setup():
    import torch

    import paper_2107_02737_amd as pk
    from workloads import water_box_hamiltonian
    gold = np.load(GOLDEN)
    h32 = water_box_hamiltonian(int(gold["molecules"]), seed=int(gold["seed"])).astype(np.float32)
    assert abs(float(h32.astype(np.float64).sum()) - float(gold["h_sum"])) < 1e-6 * abs(float(gold["h_sum"]))
    n_occ = int(gold["n_occ"])
    p_ref, w, _ = oracle.density_matrix_eigh(h32.astype(np.float64), n_occ)
    pk.load_library()
    return pk, gold, torch.from_numpy(h32).to("cuda"), p_ref, w


@pytest.mark.parametrize("precision,bound_steps,refine",
                         [("bf16x3", 0, "fp32"), ("fp16x3", 0, "fp32"), ("fp32", 0, "fp32"),
                          ("bf16x3", 32, "fp32"), ("fp32", 32, "fp32"), ("fp16x3", 32, "fp32")]
                         + FP32_EQUIVALENT)
def test_water_6144(setup, precision, bound_steps, refine):
    import torch
    pk, gold, H, p_ref, w = setup
    n, n_occ = int(gold["n"]), int(gold["n_occ"])
    banner(f"water N={n} {precision} refine={refine} bound_steps={bound_steps}")
    P, info = pk.density(H, n_occ, precision=precision, refine=refine, bound_steps=bound_steps,
                         return_info=True)
    assert info["converged"] == 1
    if bound_steps == 0:
        assert info["eps_min"] == pytest.approx(float(gold["eps_min"]), rel=1e-12)
        assert info["eps_max"] == pytest.approx(float(gold["eps_max"]), rel=1e-12)
    else:   # tighter than Gershgorin, still enclosing the whole spectrum
        assert float(gold["eps_min"]) < info["eps_min"] <= w[0]
        assert w[-1] <= info["eps_max"] < float(gold["eps_max"])
    d = P.double().cpu().numpy() - p_ref
    fro = float(np.linalg.norm(d)) / math.sqrt(n)
    mabs = float(np.max(np.abs(d)))
    pp = P @ P
    idem = float(torch.linalg.norm((pp - P).double()).item()) / math.sqrt(n)
    tol = FP32_EQUIVALENT_TOL if (precision, bound_steps, refine) in FP32_EQUIVALENT \
        else TOL[precision]
    print(f"  n_iter={info['n_iter']} ||P-P_ref||_F/sqrt(N)={fro:.3e} (tol {tol:.0e}) "
          f"max|P-P_ref|={mabs:.3e} idem={idem:.2e} trace_err={abs(info['trace'] - n_occ):.2e}",
          flush=True)
    assert torch.equal(P, P.T)
    assert fro <= tol
    assert mabs <= MAX_ABS_FACTOR * tol
    assert abs(info["trace"] - n_occ) < 0.05
    assert idem < 1e-4


def test_lanczos_bounds_enclose_the_spectrum(setup):
    """The Lanczos-tightened interval at full size encloses both ends of the
    exact spectrum (not only the HOMO-LUMO gap)."""
    pk, gold, H, _, w = setup
    banner("lanczos bounds N=6144, 16 and 32 steps")
    ws = pk.allocate_workspace(H.shape[0])
    for steps in (16, 32):
        lo, hi = pk.sp2_spectral_bounds(H, steps, ws)
        print(f"  steps={steps} ({lo:.6f}, {hi:.6f}) vs spectrum ({w[0]:.6f}, {w[-1]:.6f})",
              flush=True)
        assert float(gold["eps_min"]) <= lo <= w[0]
        assert w[-1] <= hi <= float(gold["eps_max"])
        assert np.isclose(w[0], float(gold["lam_min"]), rtol=1e-12)


def test_accelerated_fp32_equivalent_mode(setup):
    """The accelerated network at full size, with HOMO/LUMO estimates from
    the previous solve's P (sp2_homo_lumo), as the benchmark's accelerated
    leg runs it: every entry within the stated 1e-6, far fewer layers."""
    import torch
    pk, gold, H, p_ref, w = setup
    n, n_occ = int(gold["n"]), int(gold["n_occ"])
    banner(f"accelerated water N={n} fp16x3 refine=split bound_steps=32")
    P0, info0 = pk.density(H, n_occ, precision="fp16x3", refine="split", bound_steps=32,
                           return_info=True)
    homo, lumo = pk.homo_lumo(H, P0)
    assert w[n_occ - 1] <= homo < lumo <= w[n_occ]
    P, info = pk.density(H, n_occ, precision="fp16x3", refine="split", bound_steps=32, homo=homo,
                         lumo=lumo, return_info=True)
    d = P.double().cpu().numpy() - p_ref
    fro = float(np.linalg.norm(d)) / math.sqrt(n)
    mabs = float(np.max(np.abs(d)))
    print(f"  estimates ({homo:.5f}, {lumo:.5f}) vs ({w[n_occ - 1]:.5f}, {w[n_occ]:.5f}); "
          f"n_iter={info['n_iter']} (plain {info0['n_iter']}) fro={fro:.3e} max={mabs:.3e}",
          flush=True)
    assert info["converged"] == 1
    assert info["n_iter"] <= info0["n_iter"] - 4
    assert torch.equal(P, P.T)
    assert fro <= FP32_EQUIVALENT_TOL
    assert mabs <= MAX_ABS_FACTOR * FP32_EQUIVALENT_TOL


def test_benchmark_configuration(setup):
    """The benchmark's configuration: FP32-equivalent mode with the stop
    tolerance 2e-3 (the McWeeny refinement that follows maps a deviation d
    of an eigenvalue from 0 or 1 to 3d^2 - 2d^3, so e_n < 2e-3 leaves at
    most 3 tol^2 / sqrt(N) = 1.5e-7 in ||P - P_ref||_F / sqrt(N); the layers
    that would drive e_n down to its rounding floor only add rounding),
    plain and accelerated (estimates from 8 Lanczos steps per side, as the
    benchmark takes them): every entry within the stated 1e-6, no more layers
    than with tol 1e-5 (where the stop rule ends at the rounding floor)."""
    import torch
    pk, gold, H, p_ref, w = setup
    n, n_occ = int(gold["n"]), int(gold["n_occ"])
    b = BENCH_BOUND_STEPS
    banner(f"benchmark configuration water N={n} fp16x3 refine=split bound_steps={b} tol=2e-3")
    P5, info5 = pk.density(H, n_occ, precision="fp16x3", refine="split", bound_steps=b,
                           return_info=True)
    P, info = pk.density(H, n_occ, precision="fp16x3", refine="split", bound_steps=b, tol=2e-3,
                         return_info=True)
    homo, lumo = pk.homo_lumo(H, P, steps=8)
    Pa, infoa = pk.density(H, n_occ, precision="fp16x3", refine="split", bound_steps=b, tol=2e-3,
                           homo=homo, lumo=lumo, return_info=True)
    for name, Q, inf in (("plain", P, info), ("accelerated", Pa, infoa)):
        d = Q.double().cpu().numpy() - p_ref
        fro = float(np.linalg.norm(d)) / math.sqrt(n)
        mabs = float(np.max(np.abs(d)))
        idem = float(torch.linalg.norm((Q @ Q - Q).double()).item()) / math.sqrt(n)
        print(f"  {name}: n_iter={inf['n_iter']} (tol 1e-5: {info5['n_iter']}) fro={fro:.3e} "
              f"max={mabs:.3e} idem={idem:.2e}", flush=True)
        assert inf["converged"] == 1 and inf["fallback"] == 0
        assert fro <= FP32_EQUIVALENT_TOL
        assert mabs <= MAX_ABS_FACTOR * FP32_EQUIVALENT_TOL
        assert idem < 1e-5
        assert torch.equal(Q, Q.T)
    assert info["n_iter"] <= info5["n_iter"]
    assert infoa["n_iter"] < info["n_iter"]



def test_single_pass_bf16_meets_its_bound(setup):
    """Single-pass BF16 (one BF16 product per layer, FP16-pair refinement, the
    benchmark's Lanczos bound steps), as its single-pass leg runs it: every
    entry of P within the stated 1e-3 of the diagonalisation.  The late
    layers round an iterate close to a projector to 8 significant bits;
    with the planes centred at I/2 that rounding acts on entries that are
    mostly far smaller than those of the iterate itself (uncentred:
    3.9e-3)."""
    pk, gold, H, p_ref, w = setup
    n, n_occ = int(gold["n"]), int(gold["n_occ"])
    b = BENCH_BOUND_STEPS
    banner(f"single-pass bf16 water N={n} refine=split bound_steps={b} tol=2e-3")
    P, info = pk.density(H, n_occ, precision="bf16x1", refine="split", bound_steps=b, tol=2e-3,
                         return_info=True)
    d = P.double().cpu().numpy() - p_ref
    fro = float(np.linalg.norm(d)) / math.sqrt(n)
    mabs = float(np.max(np.abs(d)))
    print(f"  n_iter={info['n_iter']} fro={fro:.3e} max={mabs:.3e}", flush=True)
    assert info["converged"] == 1
    assert fro <= 1e-3
    assert mabs <= MAX_ABS_FACTOR * 1e-3
