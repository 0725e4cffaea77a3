"""Lanczos-tightened spectral bounds on the GPU against the oracle's FP64
Lanczos (same SplitMix64 start vector, same widening), and solves that use
them: the same density matrix as with Gershgorin bounds, in fewer layers."""

import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev, to_host
from oracle.precision_emulation import sp2_emulated
from workloads import random_orthogonal_hamiltonian, water_box_hamiltonian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_2107_02737_amd as pk
    pk.load_library()
    return pk


def _case(name):
    if name == "c1":
        return random_orthogonal_hamiltonian(256, 128, seed=0).astype(np.float32), 128, None
    if name == "water-ragged":
        return water_box_hamiltonian(50, seed=3).astype(np.float32), 200, 305
    if name == "water":
        return water_box_hamiltonian(100, seed=5).astype(np.float32), 400, None
    if name == "random4099":   # ragged, many matrix-vector work-groups and chunks
        a = np.random.default_rng(4).standard_normal((4099, 4099))
        return ((a + a.T) / 120.0).astype(np.float32), 2000, 4100
    a = np.random.default_rng(9).standard_normal((777, 777))
    return ((a + a.T) / 40.0).astype(np.float32), 300, None


@pytest.mark.parametrize("name", ["c1", "water-ragged", "water", "random777", "random4099"])
@pytest.mark.parametrize("steps", [8, 16, 32, 64])
def test_bounds_match_oracle(pk, name, steps):
    h32, _, ld = _case(name)
    n = h32.shape[0]
    banner(f"lanczos bounds {name} N={n} steps={steps}")
    h64 = h32.astype(np.float64)
    ws = pk.allocate_workspace(n)
    lo, hi = pk.sp2_spectral_bounds(to_dev(h32, ld), steps, ws, seed=0)
    rlo, rhi = oracle.lanczos_bounds(h64, steps, seed=0)
    w = np.linalg.eigvalsh(h64)
    print(f"  gpu ({lo:.15f}, {hi:.15f}) oracle ({rlo:.15f}, {rhi:.15f}) "
          f"spectrum ({w[0]:.6f}, {w[-1]:.6f})", flush=True)
    span = rhi - rlo
    # FP64 recurrences with different summation orders: agreement to rounding
    assert abs(lo - rlo) <= 1e-9 * span and abs(hi - rhi) <= 1e-9 * span
    assert lo <= w[0] and w[-1] <= hi


def test_seed_changes_start_vector_only(pk):
    h32, _, _ = _case("water")
    banner("lanczos seeds")
    ws = pk.allocate_workspace(600)
    H = to_dev(h32)
    for seed in (1, 12345):
        lo, hi = pk.sp2_spectral_bounds(H, 32, ws, seed=seed)
        rlo, rhi = oracle.lanczos_bounds(h32.astype(np.float64), 32, seed=seed)
        assert abs(lo - rlo) <= 1e-9 * (rhi - rlo) and abs(hi - rhi) <= 1e-9 * (rhi - rlo)


def test_degenerate_and_nonfinite(pk):
    banner("lanczos degenerate / NaN")
    ws = pk.allocate_workspace(64)
    lo, hi = pk.sp2_spectral_bounds(to_dev(0.7 * np.eye(64)), 16, ws)
    assert lo == hi == pytest.approx(0.7)
    h = random_orthogonal_hamiltonian(64, 32, seed=1).astype(np.float32)
    h[3, 5] = h[5, 3] = np.nan
    with pytest.raises(pk.SP2Error) as ei:
        pk.sp2_spectral_bounds(to_dev(h), 16, ws)
    assert ei.value.status == 2


@pytest.mark.parametrize("name", ["c1", "water-ragged", "water"])
@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "fp16x3"])
def test_solve_with_lanczos_bounds(pk, name, mode):
    h32, n_occ, ld = _case(name)
    n = h32.shape[0]
    banner(f"solve {name} N={n} {mode} bound_steps=32")
    h64 = h32.astype(np.float64)
    p_ref = oracle.density_matrix_eigh(h64, n_occ)[0]
    H = to_dev(h32, ld)
    P, info = pk.density(H, n_occ, precision=mode, refine="fp32", bound_steps=32, return_info=True)
    _, info_g = pk.density(H, n_occ, precision=mode, refine="fp32", return_info=True)
    bounds = oracle.lanczos_bounds(h64, 32)
    pe, le = sp2_emulated(h32, n_occ, mode, bounds=bounds)
    emul = oracle.error_metrics(pe, p_ref)["fro_over_sqrt_n"]
    err = oracle.error_metrics(to_host(P), p_ref)["fro_over_sqrt_n"]
    print(f"  layers {info['n_iter']} (Gershgorin {info_g['n_iter']}, emulated {le}) err={err:.3e} "
          f"(emulated {emul:.3e})", flush=True)
    assert info["converged"] == 1
    assert info["eps_min"] == pytest.approx(bounds[0], abs=1e-9 * (bounds[1] - bounds[0]))
    assert info["eps_max"] == pytest.approx(bounds[1], abs=1e-9 * (bounds[1] - bounds[0]))
    assert info["n_iter"] < info_g["n_iter"]
    assert err <= 3.0 * emul + 1e-7
