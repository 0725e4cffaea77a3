"""The accelerated network (SP2_FLAG_ACCELERATE: HOMO/LUMO estimates let
the first layers follow a shifted-and-scaled schedule, Section II.E) and the
HOMO/LUMO estimator (sp2_homo_lumo) on the GPU, through the C ABI, against
the FP64 oracle: the recorded schedule against the oracle's, P against the
diagonalisation in every mode (tolerance from the FP32-storage emulation of
the same accelerated network), traces against the oracle's FP64 network,
padding, estimates that miss the gap, the derivatives of the accelerated
network, and the estimator against the oracle's projected Lanczos on the
same inputs."""

import math

import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev, to_host
from oracle import accelerated as acc
from oracle import lanczos as lz
from oracle.precision_emulation import sp2_emulated
from workloads import random_orthogonal_hamiltonian, symmetric_normal, water_box_hamiltonian

pytestmark = pytest.mark.gpu

MODES = ["fp32", "bf16x1", "bf16x3", "fp16x3"]


@pytest.fixture(scope="module")
def pk():
    import paper_2107_02737_amd as pk
    pk.load_library()
    return pk


@pytest.fixture(scope="module")
def c1():
    h, _, e = random_orthogonal_hamiltonian(256, 128, seed=0, return_factors=True)
    h32 = h.astype(np.float32)
    p_ref, w, _ = oracle.density_matrix_eigh(h32.astype(np.float64), 128)
    return h32, 128, p_ref, w


def _oracle_schedule(h32, homo, lumo):
    lo, hi = oracle.gershgorin_bounds(h32.astype(np.float64))
    l, h = acc.mapped_interval(lo, hi, homo, lumo)
    return lo, hi, [acc.layer_polynomial(sg, s) for sg, s, _, _ in acc.acceleration_schedule(l, h)]


def test_schedule_and_traces_follow_the_oracle(pk, c1):
    """The coefficients the layers recorded are the oracle's schedule for the
    same bounds (the FP64 Gershgorin sums differ from the oracle's only in
    rounding order), the branch bytes their signs, and the traces of every
    examined iterate those of the oracle's FP64 accelerated network to FP32
    accuracy; the network needs far fewer layers than the plain one."""
    h32, n_occ, p_ref, w = c1
    homo, lumo = w[n_occ - 1] + 0.01, w[n_occ] - 0.01
    banner("accelerated schedule c1 fp32")
    H = to_dev(h32)
    P, info = pk.density(H, n_occ, precision="fp32", refine="none", homo=homo, lumo=lumo,
                         return_info=True)
    lo, hi, coefs = _oracle_schedule(h32, homo, lumo)
    assert info["eps_min"] == pytest.approx(lo, rel=1e-12)
    assert info["eps_max"] == pytest.approx(hi, rel=1e-12)
    nl = info["n_iter"]
    hist = pk.sp2_history(info["workspace"])
    assert info["converged"] and not info["fallback"] and 0 < nl < len(coefs)
    for k in range(nl):
        np.testing.assert_allclose(hist["coef"][k], coefs[k], rtol=1e-12, atol=1e-14)
        assert info["branches"][k] == (1 if coefs[k][0] > 0 else 0)
    _, rec = acc.sp2_accelerated(h32.astype(np.float64), n_occ, homo, lumo, bounds=(lo, hi),
                                 max_iter=nl)
    for k in range(nl + 1):
        assert abs(hist["t1"][k] - rec.t1[k]) < 1e-4 and abs(hist["t2"][k] - rec.t2[k]) < 1e-4, k
    _, info0 = pk.density(H, n_occ, precision="fp32", refine="none", return_info=True)
    print(f"  layers: accelerated {nl}, plain {info0['n_iter']}", flush=True)
    assert nl <= info0["n_iter"] - 5
    err = oracle.error_metrics(to_host(P), p_ref)["fro_over_sqrt_n"]
    assert err < 1e-5


@pytest.mark.parametrize("mode", MODES)
def test_every_mode_on_a_ragged_water_box(pk, mode):
    """Water box N = 1020 (padded to 1024 inside), ld = 1030, estimates 5% of
    the gap inside it: P within 3x of the emulated error of the same
    accelerated network, fewer layers than the plain network, the caller's
    padding columns untouched (the c I term reaches real rows only, or the
    traces and P would be off)."""
    import torch
    h32 = water_box_hamiltonian(170, seed=4).astype(np.float32)
    n, n_occ, ld = 1020, 680, 1030
    p_ref, w, _ = oracle.density_matrix_eigh(h32.astype(np.float64), n_occ)
    gap = w[n_occ] - w[n_occ - 1]
    homo, lumo = w[n_occ - 1] + 0.05 * gap, w[n_occ] - 0.05 * gap
    banner(f"accelerated water N={n} ld={ld} {mode}")
    pe, nle = sp2_emulated(h32, n_occ, mode, homo=homo, lumo=lumo)
    m = oracle.error_metrics(pe, p_ref, n_occ=n_occ)
    tol = 3.0 * m["fro_over_sqrt_n"] + 1e-7
    H = to_dev(h32, ld)
    P = to_dev(np.full((n, n), np.nan, np.float32), ld)
    opt = pk.make_options(mode, "fp32", homo=homo, lumo=lumo)
    ws = pk.allocate_workspace(n, opt)
    st, info, br = pk.sp2_density_ex(H, n_occ, opt, P, ws)
    err = oracle.error_metrics(to_host(P), p_ref)["fro_over_sqrt_n"]
    opt0 = pk.make_options(mode, "fp32")
    P0 = to_dev(np.zeros((n, n), np.float32), ld)
    st0, info0, _ = pk.sp2_density_ex(H, n_occ, opt0, P0, ws)
    print(f"  n_iter={info.n_iter} (plain {info0.n_iter}, emulated {nle}) err={err:.3e} "
          f"(emulated {m['fro_over_sqrt_n']:.3e})", flush=True)
    assert st == 0 and info.converged == 1
    assert err <= tol
    assert info.n_iter < info0.n_iter
    assert torch.isnan(P.as_strided((n, ld), (ld, 1))[:, n:]).all()


@pytest.mark.parametrize("where", ["occupied", "virtual"])
def test_estimates_that_miss_the_gap_fall_back(pk, where):
    """A 'gap' inside the occupied band (below this box's 128-fold degenerate
    HOMO level) or the virtual band: the schedule drives tens of states to
    the wrong side, where FP32 can no longer tell them apart, so the trace
    check at its end fails and the plain network runs instead
    (info.fallback): converged, with the plain network's P."""
    import torch
    h32 = water_box_hamiltonian(64, seed=2).astype(np.float32)
    n_occ = 256
    p_ref, w, _ = oracle.density_matrix_eigh(h32.astype(np.float64), n_occ)
    homo, lumo = (w[n_occ - 200], w[n_occ - 170]) if where == "occupied" else (w[n_occ + 20], w[n_occ + 50])
    assert homo < lumo and (lumo < w[n_occ - 1] - 0.05 or homo > w[n_occ] + 0.005)
    banner(f"accelerated with estimates in the {where} band")
    H = to_dev(h32)
    P, info = pk.density(H, n_occ, precision="fp32", refine="fp32", homo=homo, lumo=lumo,
                         return_info=True)
    P0, info0 = pk.density(H, n_occ, precision="fp32", refine="fp32", return_info=True)
    err = oracle.error_metrics(to_host(P), p_ref)["fro_over_sqrt_n"]
    print(f"  fallback={info['fallback']} converged={info['converged']} n_iter={info['n_iter']} "
          f"err={err:.3e}", flush=True)
    assert info["fallback"] == 1 and info["converged"] == 1
    assert info["n_iter"] == info0["n_iter"] and info["branches"] == info0["branches"]
    assert torch.equal(P, P0)
    assert err < 3e-5


def test_two_by_two_closed_form(pk):
    h = np.array([[0.3, -0.7], [-0.7, -0.4]], np.float32)
    hd = h.astype(np.float64)
    r = math.sqrt(((hd[0, 0] - hd[1, 1]) / 2) ** 2 + hd[0, 1] ** 2)
    p_ref = 0.5 * (np.eye(2) - (hd - 0.5 * np.trace(hd) * np.eye(2)) / r)
    w = np.linalg.eigvalsh(hd)
    banner("accelerated 2x2")
    for mode in MODES:
        P, info = pk.density(to_dev(h), 1, precision=mode, refine="fp32", homo=w[0] + 0.2,
                             lumo=w[1] - 0.2, return_info=True)
        assert info["converged"]
        tol = 2e-2 if mode == "bf16x1" else 1e-5
        assert np.abs(to_host(P) - p_ref).max() < tol, mode


def test_derivatives_of_the_accelerated_network(pk, c1):
    """JVP and VJP of the taped accelerated network (FP32 derivative
    products) against the oracle's derivatives of its own FP64 accelerated
    network with the same bounds, estimates and layer count, and against
    perturbation theory; dot test between the two."""
    import torch
    h32, n_occ, _, w = c1
    homo, lumo = w[n_occ - 1] + 0.01, w[n_occ] - 0.01
    banner("accelerated JVP/VJP c1 fp32")
    H = to_dev(h32)
    P, info = pk.density(H, n_occ, precision="fp32", refine="fp32", homo=homo, lumo=lumo,
                         checkpoint_every=3, return_info=True)
    nl = info["n_iter"]
    h1 = symmetric_normal(256, 2, std=1e-3).astype(np.float32)
    wm = symmetric_normal(256, 1).astype(np.float32)
    P1 = torch.empty_like(H)
    G = torch.empty_like(H)
    pk.sp2_jvp(info["workspace"], to_dev(h1), P1)
    pk.sp2_vjp(info["workspace"], to_dev(wm), G)
    lo, hi, _ = _oracle_schedule(h32, homo, lumo)
    h64 = h32.astype(np.float64)
    _, rec = acc.sp2_accelerated(h64, n_occ, homo, lumo, bounds=(lo, hi), max_iter=nl, refine=True)
    j_ref = oracle.sp2_jvp(h64, h1.astype(np.float64), rec)
    g_ref = oracle.sp2_vjp(h64, wm.astype(np.float64), rec)
    j, g = to_host(P1), to_host(G)
    rel_j = np.linalg.norm(j - j_ref) / np.linalg.norm(j_ref)
    rel_g = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    dm = oracle.dmpt_response(h64, n_occ, h1.astype(np.float64))
    rel_dm = np.linalg.norm(j - dm) / np.linalg.norm(dm)
    print(f"  n_iter={nl} jvp {rel_j:.2e} vjp {rel_g:.2e} vs DMPT {rel_dm:.2e}", flush=True)
    assert rel_j < 1e-4 and rel_g < 1e-4
    assert rel_dm < 1e-4
    lhs = float(np.sum(wm.astype(np.float64) * j))
    rhs = float(np.sum(g * h1.astype(np.float64)))
    assert lhs == pytest.approx(rhs, rel=1e-4)


def test_split_derivatives_of_the_accelerated_network(pk, c1):
    """The same with BF16x3 layers and split derivatives (SP2_FLAG_SPLIT_
    DERIVATIVES): the replayed scheduled layers, the derivative maps and the
    refinement's derivative all run on the centred planes of the iterates
    with their correction terms.  Against the oracle's derivatives of its
    FP64 accelerated network and perturbation theory, within the BF16x3
    tolerance of the plain network's split derivatives (1e-3), dot test
    between JVP and VJP."""
    import torch
    h32, n_occ, _, w = c1
    homo, lumo = w[n_occ - 1] + 0.01, w[n_occ] - 0.01
    banner("accelerated JVP/VJP c1 bf16x3 split derivatives")
    H = to_dev(h32)
    P, info = pk.density(H, n_occ, precision="bf16x3", refine="fp32", homo=homo, lumo=lumo,
                         checkpoint_every=3, split_derivatives=True, return_info=True)
    nl = info["n_iter"]
    assert info["converged"] and not info["fallback"]
    h1 = symmetric_normal(256, 2, std=1e-3).astype(np.float32)
    wm = symmetric_normal(256, 1).astype(np.float32)
    P1 = torch.empty_like(H)
    G = torch.empty_like(H)
    pk.sp2_jvp(info["workspace"], to_dev(h1), P1)
    pk.sp2_vjp(info["workspace"], to_dev(wm), G)
    lo, hi, coefs = _oracle_schedule(h32, homo, lumo)
    h64 = h32.astype(np.float64)
    hist = pk.sp2_history(info["workspace"])
    # the scheduled layers are the oracle's; the network differentiated is
    # the one the GPU recorded (its trace-driven signs after the schedule)
    for k in range(min(nl, len(coefs))):
        np.testing.assert_allclose(hist["coef"][k], coefs[k], rtol=1e-12, atol=1e-14)
    rec = oracle.SP2Record(eps_min=info["eps_min"], eps_max=info["eps_max"], refine=True,
                           branches=[1 if c[0] > 0 else -1 for c in hist["coef"][:nl]],
                           coefs=[tuple(c) for c in hist["coef"][:nl]])
    j_ref = oracle.sp2_jvp(h64, h1.astype(np.float64), rec)
    g_ref = oracle.sp2_vjp(h64, wm.astype(np.float64), rec)
    j, g = to_host(P1), to_host(G)
    rel_j = np.linalg.norm(j - j_ref) / np.linalg.norm(j_ref)
    rel_g = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    dm = oracle.dmpt_response(h64, n_occ, h1.astype(np.float64))
    rel_dm = np.linalg.norm(j - dm) / np.linalg.norm(dm)
    print(f"  n_iter={nl} jvp {rel_j:.2e} vjp {rel_g:.2e} vs DMPT {rel_dm:.2e}", flush=True)
    assert rel_j < 1e-3 and rel_g < 1e-3
    assert rel_dm < 2e-3
    lhs = float(np.sum(wm.astype(np.float64) * j))
    rhs = float(np.sum(g * h1.astype(np.float64)))
    assert lhs == pytest.approx(rhs, rel=1e-3)


@pytest.mark.parametrize("m,steps", [(170, 24), (64, 16)])
def test_homo_lumo_estimator_matches_the_oracle(pk, m, steps):
    """sp2_homo_lumo on the FP32 H and the FP32 cast of the exact P against
    the oracle's projected Lanczos on the same two matrices: the same
    estimates to 1e-8 (FP64 recurrences, summation orders differ), both
    inside the true gap."""
    h32 = water_box_hamiltonian(m, seed=0).astype(np.float32)
    n, n_occ = h32.shape[0], 4 * m
    p_ref, w, _ = oracle.density_matrix_eigh(h32.astype(np.float64), n_occ)
    p32 = p_ref.astype(np.float32)
    banner(f"homo/lumo estimator N={n} steps={steps}")
    ws = pk.allocate_workspace(n)
    got = pk.sp2_homo_lumo(to_dev(h32), to_dev(p32), ws, steps=steps, margin=0.05)
    ref = lz.homo_lumo_estimates(h32.astype(np.float64), p32.astype(np.float64), steps, margin=0.05)
    print(f"  gpu {got} oracle {ref} true ({w[n_occ - 1]:.6f}, {w[n_occ]:.6f})", flush=True)
    assert abs(got[0] - ref[0]) < 1e-8 and abs(got[1] - ref[1]) < 1e-8
    assert w[n_occ - 1] <= got[0] < got[1] <= w[n_occ]


def test_homo_lumo_estimator_from_a_gpu_solve_drives_the_accelerated_network(pk):
    """The molecular-dynamics use: estimates from the previous solve's P
    (here the same H) accelerate the next solve, which keeps its accuracy."""
    h32 = water_box_hamiltonian(170, seed=0).astype(np.float32)
    n, n_occ = 1020, 680
    p_ref, w, _ = oracle.density_matrix_eigh(h32.astype(np.float64), n_occ)
    banner("homo/lumo from a GPU solve, then an accelerated solve, fp16x3")
    H = to_dev(h32)
    P0, info0 = pk.density(H, n_occ, precision="fp16x3", refine="split", bound_steps=32,
                           return_info=True)
    homo, lumo = pk.homo_lumo(H, P0)
    assert w[n_occ - 1] <= homo < lumo <= w[n_occ]
    P1, info1 = pk.density(H, n_occ, precision="fp16x3", refine="split", bound_steps=32,
                           homo=homo, lumo=lumo, return_info=True)
    e0 = oracle.error_metrics(to_host(P0), p_ref)["fro_over_sqrt_n"]
    e1 = oracle.error_metrics(to_host(P1), p_ref)["fro_over_sqrt_n"]
    print(f"  plain {info0['n_iter']} layers {e0:.3e}; accelerated {info1['n_iter']} layers "
          f"{e1:.3e}", flush=True)
    assert info1["n_iter"] <= info0["n_iter"] - 5
    assert e1 <= 1.5 * e0 + 1e-7
