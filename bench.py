"""Benchmark: DNN-SP2 density-matrix solves/s at N = 6144 on one MI355X.

One step = one full ``sp2_density_ex`` call on a device-resident FP32
Hamiltonian in the FP32-equivalent mode: Gershgorin discs tightened by 8
Lanczos steps, the input layer, every SP2 layer as an FP16 hi/lo split
product of the centred iterate S - I/2 on MFMA (Eq. 20-22; FP64
trace-driven branch and stop decided on the device) and the McWeeny
refinement in the same FP16 hi/lo arithmetic, ending with P in a caller
buffer.  This mode meets the stated ||P - P_ref||_F / sqrt(N) <= 1e-6 over
every entry with a margin (an FP32 refinement meets it too, closer to the
bound: on this GPU its FP32 MFMA products round more coarsely than the FP16
pair).  The stop tolerance is 2e-3 on e_n = |Tr S - ||S||_F^2|: the
refinement maps an eigenvalue's deviation d from 0 or 1 to 3d^2 - 2d^3, so
what is left is at most 3 tol^2 / sqrt(N) = 1.5e-7 in ||P - P_ref||_F /
sqrt(N), and the layers that would drive e_n further down to its rounding
floor only add rounding.

Workload: seeded tight-binding water box, 1024 molecules, N = 6144,
n_occ = 4096, H in FP32 (synthetic stand-in for the paper's SCC-DFTB water).

Prints ONE JSON line.  Also reported: effective TFLOPS (3 products of
2 N^3 per split layer + 2 N^3 per refinement product), the error of every
entry against the FP64 oracle's diagonalisation, the roofline of the layer
kernel (HIP events around every layer launch on the solve's stream, in a
second timed pass of the same solves), side legs in the other arithmetics
(BF16 pair, single-pass BF16, plain FP32 MFMA SP2) timed over as many
steps, the accelerated network (Section II.E) with HOMO/LUMO estimates
taken from the previous solve, the FP64 oracle timed on the host cores and,
outside the timed steps, the XL-BOMD kernel building block and the
canonical integration step of Section IV on a large batch of coordinates,
and, for context (the comparison of the paper's Fig. 2), the density matrix
from the GPU's dense eigensolver library in FP32 and FP64.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SP2 density-matrix solves/s + effective TFLOPS at N=6144; error vs FP64 oracle"
PEAK_TFLOPS = {"bf16x3": 2500.0, "fp16x3": 2500.0, "bf16x1": 2500.0, "fp32": 157.3}
PRODUCTS = {"bf16x3": 3, "fp16x3": 3, "bf16x1": 1, "fp32": 1}
GOLDEN = os.path.join(ROOT, "tests", "golden", "water_m1024_seed0.npz")
TRAFFIC_PROFILES = {p: os.path.join(ROOT, "profiles", f"k_sym_split_{p}_water6144_traffic.md")
                    for p in ("bf16x3", "fp16x3")}
# Stated bounds on ||P - P_ref||_F / sqrt(N): FP32-equivalent mode and
# single-pass BF16.
TOL_FP32_EQUIVALENT = 1e-6
TOL_SINGLE_PASS_BF16 = 1e-3
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2107_02737_amd", "csrc", f)
                  for f in ("sp2_common.hpp", "sp2_gemm.hpp")]
NVT_PROFILE = os.path.join(ROOT, "profiles", "k_nvt_step_3x2e24coords.md")
NVT_SOURCES = [os.path.join(ROOT, "paper_2107_02737_amd", "csrc", "sp2_nvt.hpp")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp16x3", choices=list(PRODUCTS))
    ap.add_argument("--refine", default="split", choices=["none", "fp32", "split"])
    ap.add_argument("--tol", type=float, default=2e-3,
                    help="stop tolerance on e_n = |Tr S - ||S||_F^2| (every configuration here "
                         "refines: one McWeeny step maps an eigenvalue's deviation d to "
                         "3d^2 - 2d^3, which leaves at most 3 tol^2 / sqrt(N) = 1.5e-7 in "
                         "||P - P_ref||_F / sqrt(N) at N = 6144, 15%% of the 1e-6 budget)")
    ap.add_argument("--bound-steps", type=int, default=8,
                    help="Lanczos steps tightening the Gershgorin bounds (0: Gershgorin only)")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the side legs in other arithmetics")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--est-steps", type=int, default=8,
                    help="Lanczos steps per side of the HOMO/LUMO estimator (accelerated leg and "
                         "trajectory); on the water box 8 give the same accelerated layer count "
                         "as 24 at a third of the cost")
    ap.add_argument("--no-accelerated", action="store_true",
                    help="skip the accelerated leg (HOMO/LUMO estimates from the previous solve)")
    ap.add_argument("--cpu-layers", type=int, default=4,
                    help="FP64 oracle layers timed for the CPU baseline sample")
    ap.add_argument("--trajectory", type=int, default=0, metavar="STEPS",
                    help="instead of the benchmark: run STEPS steps of the N=16384 trajectory "
                         "workload H(t) = H0 + 0.01 sin(0.1 t) H_p (adjoint on the last step) "
                         "and print per-step times and the drift of Tr P and idempotency")
    ap.add_argument("--traj-precision", default="bf16x3", choices=list(PRODUCTS),
                    help="layer arithmetic of the trajectory run")
    ap.add_argument("--traj-refine", default="fp32", choices=["none", "fp32", "split"],
                    help="refinement of the trajectory run")
    ap.add_argument("--traj-accelerate", action="store_true",
                    help="trajectory: every step after the first runs the accelerated network "
                         "with HOMO/LUMO estimates from the previous step's P (timed apart)")
    ap.add_argument("--xl-rank", type=int, default=4,
                    help="also time the XL-BOMD kernel building block (Krylov approximation of "
                         "K f of this rank on the water box's charge model; 0: skip)")
    ap.add_argument("--nvt-coords", type=int, default=3 * 2 ** 24,
                    help="also time the canonical integration step on this many FP64 "
                         "coordinates (0: skip)")
    ap.add_argument("--no-mfma-probe", action="store_true",
                    help="skip the matrix-core rate probe (no memory traffic) beside the roofline")
    ap.add_argument("--no-diag", action="store_true",
                    help="skip the GPU diagonalisation context (library eigh + outer product)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM traffic counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device copy of known size: 1 GiB read + 1 GiB written per launch.
    Its FETCH_SIZE / WRITE_SIZE counter readings calibrate the traffic figures
    reported for the layer kernel."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": 4 * n, "launches": 3}), flush=True)


def measured_traffic(precision, profile=None, sources=KERNEL_SOURCES,
                     key="traffic_bytes_per_launch"):
    """HBM bytes per launch from a committed counter summary (FETCH_SIZE +
    WRITE_SIZE, calibrated against a plain copy), or None when there is no
    summary for this precision or the kernel source has changed since the
    counters were taken."""
    import hashlib
    profile = profile or TRAFFIC_PROFILES.get(precision)
    if profile is None or not os.path.exists(profile):
        return None
    sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in sources)).hexdigest()
    fields = {}
    for line in open(profile):
        if ":" in line and not line.startswith(("|", " ", "#")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != sha or key not in fields:
        return None
    return float(fields[key])


def trajectory(steps, precision, refine, accelerate=False, est_steps=8):
    """Trajectory workload: water box of 2730 molecules zero-padded to
    N = 16384, n_occ = 10920; H(t) = H0 + fl32(a_t H_p), a_t = 0.01 sin(0.1 t),
    formed on the device; every step an independent split-precision solve,
    the last one with the tape (checkpoint every 4th iterate) and the adjoint
    d Tr(W P)/dH, with FP32 and (BF16X3 layers) with split derivative
    products.  Solve times from HIP events on the solve's stream."""
    import torch

    import paper_2107_02737_amd as pk
    from workloads import symmetric_normal, trajectory_perturbation, water_box_hamiltonian
    m, n, n_occ = 2730, 16384, 10920
    t0 = time.perf_counter()
    H0 = torch.from_numpy(water_box_hamiltonian(m, seed=0, n_pad=n, dtype=np.float32)).cuda()
    Hp = torch.from_numpy(trajectory_perturbation(n, 3, n_real=6 * m, dtype=np.float32)).cuda()
    W = torch.from_numpy(symmetric_normal(n, 1, n_real=6 * m, dtype=np.float32)).cuda()
    print(f"# trajectory inputs ready ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    pk.load_library()
    opt = pk.make_options(precision, refine)
    opt_tape = pk.make_options(precision, refine, checkpoint_every=4)
    ws = pk.allocate_workspace(n, opt_tape)
    P = torch.empty_like(H0)
    times, drift_tr, drift_idem, layers, est_times, fallbacks = [], [], [], [], [], 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    adj_ms = adj_split_ms = adj_split_rel = None
    est = None
    for t in range(steps):
        H = torch.add(H0, torch.mul(Hp, float(np.float32(0.01 * math.sin(0.1 * t)))))
        last = t == steps - 1
        o = opt_tape if last else opt
        if accelerate and est is not None:
            o = pk.make_options(precision, refine, checkpoint_every=4 if last else 0,
                                homo=est[0], lumo=est[1])
        torch.cuda.synchronize()
        ev0.record()
        st, info, _ = pk.sp2_density_ex(H, n_occ, o, P, ws)
        ev1.record()
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1))
        layers.append(info.n_iter)
        fallbacks += info.fallback
        if accelerate and not last:
            ev0.record()
            est = pk.sp2_homo_lumo(H, P, ws, steps=est_steps)
            ev1.record()
            torch.cuda.synchronize()
            est_times.append(ev0.elapsed_time(ev1))
        drift_tr.append(info.trace - n_occ)
        drift_idem.append(float(torch.linalg.norm((P @ P - P).double()).item()) / math.sqrt(n))
        if last:
            G = torch.empty_like(P)
            ev0.record()
            pk.sp2_vjp(ws, W, G)
            ev1.record()
            torch.cuda.synchronize()
            adj_ms = ev0.elapsed_time(ev1)
            if precision == "bf16x3" and not accelerate:
                # the same adjoint with the layer maps in BF16X3 (taped again with the option)
                pk.sp2_density_ex(H, n_occ, pk.make_options(precision, refine, checkpoint_every=4,
                                                            split_derivatives=True), P, ws)
                G2 = torch.empty_like(P)
                ev0.record()
                pk.sp2_vjp(ws, W, G2)
                ev1.record()
                torch.cuda.synchronize()
                adj_split_ms = ev0.elapsed_time(ev1)
                adj_split_rel = float(torch.linalg.norm((G2 - G).double()).item()
                                      / torch.linalg.norm(G.double()).item())
                del G2
        if t % 10 == 0 or last:
            print(f"# t={t} status={st} n_iter={info.n_iter} {times[-1]:.1f} ms "
                  f"TrP-n={drift_tr[-1]:.2e} idem={drift_idem[-1]:.2e}", file=sys.stderr, flush=True)
        del H
    tt = np.array(times)
    print(json.dumps({
        "workload": f"trajectory: water box {m} molecules zero-padded to N={n}, n_occ={n_occ}, "
                    f"H(t)=H0+0.01 sin(0.1t) H_p, {steps} steps, {precision} + {refine} refinement"
                    + (", accelerated from the previous step's HOMO/LUMO" if accelerate else ""),
        "steps": steps, "ms_per_step_mean": float(tt.mean()), "ms_p10": float(np.percentile(tt, 10)),
        "ms_p90": float(np.percentile(tt, 90)), "layers": [min(layers), max(layers)],
        "trace_drift": [float(min(drift_tr)), float(max(drift_tr))],
        "idempotency": [float(min(drift_idem)), float(max(drift_idem))],
        "adjoint_ms_last_step": adj_ms,
        "adjoint_ms_last_step_split_derivatives": adj_split_ms,
        "adjoint_split_vs_fp32_rel": adj_split_rel,
        "solve_ms_last_step_with_tape": float(tt[-1]),
        "accelerated": accelerate,
        "estimator_ms_mean": float(np.mean(est_times)) if est_times else None,
        "estimator_steps": est_steps if accelerate else None,
        "ms_per_md_step_mean": float(tt[1:].mean() + np.mean(est_times)) if est_times else None,
        "fallbacks": fallbacks}), flush=True)


def timed_solves(pk, H, n_occ, precision, refine, steps, warmup, time_layers, bound_steps=0,
                 homo=None, lumo=None, tol=1e-5):
    import torch
    opt = pk.make_options(precision, refine, time_layers=time_layers, bound_steps=bound_steps,
                          homo=homo, lumo=lumo, tol=tol)
    ws = pk.allocate_workspace(H.shape[0], opt, H.device)
    P = torch.empty_like(H)
    for _ in range(warmup):
        pk.sp2_density_ex(H, n_occ, opt, P, ws)
    torch.cuda.synchronize()
    infos = []
    stream = torch.cuda.current_stream()
    events = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    events[0].record(stream)
    for k in range(steps):
        st, info, br = pk.sp2_density_ex(H, n_occ, opt, P, ws)
        events[k + 1].record(stream)
        infos.append(info.as_dict())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-solve durations between consecutive events on the solve stream
    per = np.array([events[k].elapsed_time(events[k + 1]) for k in range(steps)])
    for d, ms in zip(infos, per):
        d["solve_ms"] = float(ms)
    return P, infos, (t1 - t0) / steps


def full_error(P, p_ref):
    """Every entry of P against the exact P_ref (FP64, host):
    ||P - P_ref||_F / sqrt(N), ||P - P_ref||_F / N and max |P - P_ref|."""
    d = P.detach().double().cpu().numpy() - p_ref
    n = d.shape[0]
    fro = float(np.linalg.norm(d))
    return {"fro_over_sqrt_n": fro / math.sqrt(n), "fro_over_n": fro / n,
            "max_abs": float(np.max(np.abs(d))), "entries": "all"}


def sampled_error(P, gold):
    """||P - P_ref||_F / sqrt(N) estimated from uniformly sampled entries of the
    exact P_ref, plus the exact diagonal error (used when the CPU leg, which
    computes the exact P_ref, is skipped)."""
    n = int(gold["n"])
    p = P.detach()
    pi = np.asarray(gold["pair_i"], dtype=np.int64)
    pj = np.asarray(gold["pair_j"], dtype=np.int64)
    import torch
    got = p[torch.from_numpy(pi).to(p.device), torch.from_numpy(pj).to(p.device)]
    d = got.double().cpu().numpy() - gold["pair_val"]
    diag = torch.diagonal(p).double().cpu().numpy() - gold["diag"]
    return {
        "fro_over_sqrt_n": math.sqrt(n * float(np.mean(d * d))),
        "max_abs": float(np.max(np.abs(d))),
        "diag_rms": float(np.sqrt(np.mean(diag * diag))),
        "entries": f"{int(d.size)} sampled + diagonal",
    }


def device_checks(P, n_occ):
    import torch
    p = P.detach()
    n = p.shape[0]
    pp = p @ p
    return {
        "idempotency": float(torch.linalg.norm((pp - p).double()).item() / math.sqrt(n)),
        "trace_err": float(abs(torch.trace(p.double()).item() - n_occ)),
        "symmetric": bool(torch.equal(p, p.T)),
    }


def diagonalization_baseline(H, n_occ, p_ref=None, dtypes=("float32", "float64"), reps=1):
    """Context for the paper's Fig. 2 comparison: the density matrix from a
    dense GPU eigensolver (the vendor library behind ``torch.linalg.eigh``,
    the symmetric divide-and-conquer ``syevd`` path) and the outer product of
    the occupied eigenvectors, P = V_occ V_occ^T (Eq. 17), timed on the GPU
    in single and double precision.  A library baseline beside the SP2
    solver, not part of it."""
    import torch
    out = {"library": str(torch.backends.cuda.preferred_linalg_library()),
           "method": "torch.linalg.eigh on the GPU + occupied outer product"}
    for name in dtypes:
        dt = getattr(torch, name)
        A = H.to(dt)

        def build():
            w, v = torch.linalg.eigh(A)
            vo = v[:, :n_occ].contiguous()
            return vo @ vo.T

        P = build()   # warm-up: library set-up and workspace
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            P = build()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        rec = {"seconds": float(min(times)), "reps": reps}
        if p_ref is not None:
            rec.update(full_error(P, p_ref))
        out[name] = rec
        del P, A
    return out


def xl_kernel(pk, seed, rank, precision, refine, split_derivatives=False):
    """The XL-BOMD kernel building block at N = 6144: H(n) of the water box's
    synthetic charge model at seeded charges n, one taped solve, then one
    charge-space response J v and one rank-``rank`` Krylov approximation of
    K f (f = q0[n] - n), each timed with HIP events; the minimal residual the
    Krylov call reports is checked against |f - J kf| from a further response."""
    import torch
    from workloads import charge_shifted_hamiltonian, random_charges, water_charge_model

    mod = water_charge_model(1024, seed=seed)
    na = mod["z"].size
    charges = random_charges(na, seed=5)
    h = charge_shifted_hamiltonian(mod["h0"], mod["atom_ptr"], mod["gamma"], charges)
    H = torch.from_numpy(h.astype(np.float32)).to("cuda")
    dev = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    ptr, z, gamma, nvec = dev(mod["atom_ptr"], torch.int64), dev(mod["z"]), dev(mod["gamma"]), dev(charges)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record()
    P, info = pk.density(H, mod["n_occ"], precision=precision, refine=refine, checkpoint_every=4,
                         return_info=True, split_derivatives=split_derivatives)
    ev[1].record()
    ws = info["workspace"]
    f = pk.sp2_mulliken(P, ptr, z, sub=nvec)
    scratch = pk.allocate_xl_scratch(H.shape[0], na, rank)
    v = dev(np.random.default_rng(3).standard_normal(na))
    ev[2].record()
    pk.sp2_xl_response(ws, ptr, gamma, v, scratch)
    ev[3].record()
    kf, rho, used = pk.sp2_xl_kernel(ws, ptr, gamma, f, rank, scratch)
    ev[4].record()
    jkf = pk.sp2_xl_response(ws, ptr, gamma, kf, scratch)
    torch.cuda.synchronize()
    direct = float(np.linalg.norm(f.cpu().numpy() - jkf.cpu().numpy()))
    return {"n_atoms": na, "rank": rank, "rank_used": used, "precision": precision,
            "derivative_products": "bf16x3" if split_derivatives and precision == "bf16x3" else "fp32",
            "taped_solve_ms": ev[0].elapsed_time(ev[1]),
            "response_ms": ev[2].elapsed_time(ev[3]), "krylov_ms": ev[3].elapsed_time(ev[4]),
            "rho_over_rho0": [r / rho[0] for r in rho],
            "check_residual_over_rho0": direct / rho[0],
            "workload": "water box 1024 molecules, synthetic charge model (screened Coulomb "
                        "gamma), seeded charges"}


def cpu_baseline(h32, n_occ, layers, n_iter_ref):
    """The FP64 oracle as it stands on the host cores, on a bounded sample:
    bounds + input layer + ``layers`` SP2 layers at full N, extrapolated to a
    full solve of ``n_iter_ref`` layers."""
    import oracle
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        infos = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        threads = max([d.get("num_threads", 1) for d in infos] or [os.cpu_count() or 1])
        if infos:
            blas = f"{infos[0].get('internal_api', '?')} {infos[0].get('version', '')}".strip()
    except Exception:
        threads = os.cpu_count() or 1
    h = h32.astype(np.float64)
    t0 = time.perf_counter()
    oracle.sp2(h, n_occ, tol=0.0, max_iter=0)
    t1 = time.perf_counter()
    oracle.sp2(h, n_occ, tol=0.0, max_iter=layers)
    t2 = time.perf_counter()
    setup = t1 - t0
    per_layer = max(0.0, (t2 - t1) - setup) / layers
    t_solve = setup + n_iter_ref * per_layer
    # the plain definition: FP64 diagonalisation and the occupied outer product
    # (its result is also the reference for the GPU's error report)
    t3 = time.perf_counter()
    p_ref, _, _ = oracle.density_matrix_eigh(h, n_occ)
    t_eigh = time.perf_counter() - t3
    # sanity line: plain FP32 NumPy layers (SGEMM square, traces summed in FP64)
    lo, hi = oracle.gershgorin_bounds(h)
    x = ((hi * np.eye(h.shape[0]) - h) / (hi - lo)).astype(np.float32)
    t4 = time.perf_counter()
    for _ in range(layers):
        t1_ = float(np.trace(x, dtype=np.float64))
        t2_ = float(np.sum(x * x, dtype=np.float64))
        x2 = x @ x
        x = x2 if oracle.choose_branch(t1_, t2_, n_occ) > 0 else np.float32(2.0) * x - x2
    t_fp32 = (time.perf_counter() - t4) / layers * n_iter_ref
    return p_ref, {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"FP64 oracle sp2(): bounds + input layer + {layers} layers at N={h.shape[0]} "
                  f"({t2 - t1:.1f} s), extrapolated to {n_iter_ref} layers",
        "seconds_per_solve": t_solve,
        "blas": blas,
        "host_cpus": os.cpu_count(),
        "eigh_seconds": t_eigh,
        "fp32_numpy_sp2_seconds_per_solve": t_fp32,
    }


def mfma_probe(pk, H, n_occ, precision, iters=2500, warm=20, reps=10):
    """What the matrix cores reach on this GPU under its power limit with no
    memory traffic: the layer kernel's 96-instruction K-step pair on
    register-resident fragments (libsp2_probe.so, one work-group per CU),
    for operand planes of the same water box at several points of a solve:
    the centred input layer S_0 - I/2 (sparse), the iterates after 4 and 8
    layers, the converged P - I/2, and all-zero planes.  Rate from HIP
    events on the launch stream; shader clock from the kernel's own clock
    and wall-clock counters."""
    import ctypes

    import torch
    from paper_2107_02737_amd.build import PROBE_PATH
    lib = ctypes.CDLL(PROBE_PATH)
    lib.sp2_probe_mfma.restype = ctypes.c_int32
    lib.sp2_probe_mfma.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    n = H.shape[0]
    dev = H.device
    nblocks = torch.cuda.get_device_properties(dev).multi_processor_count
    code = {"bf16x3": 2, "fp16x3": 3}[precision]
    eye = torch.eye(n, device=dev)
    ws = pk.allocate_workspace(n, None, dev)
    P = torch.empty_like(H)
    iterates = {}
    for k in (0, 4, 8):
        # the iterate after k layers (max_iter = k stops there; k = 0: the input layer)
        opt = pk.make_options(precision, "none", max_iter=max(k, 1), tol=0.0)
        if k == 0:
            lo_hi = pk.sp2_bounds(H, ws)
            iterates["input layer"] = (lo_hi[1] * eye - H) / (lo_hi[1] - lo_hi[0])
            continue
        st, info, _ = pk.sp2_density_ex(H, n_occ, opt, P, ws, check=False)
        if st not in (0, 3):
            raise RuntimeError(f"probe input solve failed with status {st}")
        iterates[f"after {k} layers"] = P.clone()
    st, info, _ = pk.sp2_density_ex(H, n_occ, pk.make_options(precision, "none", tol=2e-3), P, ws,
                                    check=False)
    iterates["converged"] = P.clone()
    hi = torch.empty((n, n), dtype=torch.int16, device=dev)
    lo = torch.empty_like(hi)
    sink = torch.empty(nblocks * 256, dtype=torch.float32, device=dev)
    clocks = torch.zeros(4 * nblocks, dtype=torch.int64, device=dev)
    wall_hz = ctypes.c_double()
    stream = torch.cuda.current_stream(dev)
    flop = nblocks * 4 * iters * 96 * 32768.0
    out = {"precision": precision, "work_groups": nblocks, "iters": iters,
           "flop_per_launch": flop, "peak_tflops": PEAK_TFLOPS[precision], "operands": {}}
    kinds = list(iterates.items()) + [("zeros", None)]
    for name, S in kinds:
        if S is None:
            hi.zero_()
            lo.zero_()
        else:
            pk.sp2_split((S - 0.5 * eye).contiguous(), precision, hi, lo)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

        def launch():
            r = lib.sp2_probe_mfma(ctypes.c_void_p(hi.data_ptr()), ctypes.c_void_p(lo.data_ptr()), n,
                                   code, iters, nblocks, ctypes.c_void_p(sink.data_ptr()),
                                   ctypes.c_void_p(clocks.data_ptr()), ctypes.byref(wall_hz),
                                   ctypes.c_void_p(stream.cuda_stream))
            if r != 0:
                raise RuntimeError(f"sp2_probe_mfma returned {r}")

        for _ in range(warm):
            launch()
        ev[0].record(stream)
        for _ in range(reps):
            launch()
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        c = clocks.view(nblocks, 4).cpu().numpy().astype(np.float64)
        ghz = float(np.mean((c[:, 2] - c[:, 0]) / (c[:, 3] - c[:, 1]))) * wall_hz.value / 1e9
        tf = flop / (ms * 1e-3) / 1e12
        out["operands"][name] = {"ms_per_launch": ms, "tflops": tf,
                                 "frac_of_peak": tf / PEAK_TFLOPS[precision], "shader_ghz": ghz}
    del hi, lo, ws, P
    return out


def canonical_step(pk, n, reps=20):
    """Both halves of the canonical integration step (Section IV, Eq. 31) on
    ``n`` FP64 coordinates (seeded, device-resident), timed with HIP events
    on the stream they are launched on; algorithmic bytes per coordinate:
    first half reads R, V, F, eta, M and writes R, V (56 B), second half
    reads V, F, M and writes V (32 B).  Also the per-step time of the water
    box's 3072 atoms (9216 coordinates), where launch latency dominates."""
    import torch
    from workloads import AMU, KB_EV

    kt = 500.0 * KB_EV
    p = pk.nvt_params(0.5, kt, pk.sp2_nvt_gamma_tc(1.5e-4, kt, 0.5), 1e-3, 0)

    def run(count, iters):
        g = torch.Generator(device="cuda").manual_seed(7)
        rnd = lambda s: torch.randn(count, dtype=torch.float64, device="cuda", generator=g) * s
        R, V, F, eta = rnd(1.0), rnd(0.01), rnd(1.0), rnd(1.0)
        M = torch.full((count,), 16.0 * AMU, dtype=torch.float64, device="cuda")
        for _ in range(3):
            pk.sp2_nvt_first_half(R, V, F, eta, M, p)
            pk.sp2_nvt_second_half(V, F, M, p)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(iters):
            pk.sp2_nvt_first_half(R, V, F, eta, M, p)
        ev[1].record()
        for _ in range(iters):
            pk.sp2_nvt_second_half(V, F, M, p)
        ev[2].record()
        torch.cuda.synchronize()
        if not bool(torch.isfinite(R).all()):
            raise RuntimeError("canonical step produced non-finite positions")
        return ev[0].elapsed_time(ev[1]) / iters * 1e3, ev[1].elapsed_time(ev[2]) / iters * 1e3

    t1, t2 = run(n, reps)
    w1, w2 = run(9216, 200)
    gbps = 88.0 * n / ((t1 + t2) * 1e-6) / 1e9
    return {"workload": f"{n} independent coordinates (FP64 R, V, F, eta, M), scheme 0 with "
                        "both friction terms", "n_coords": n,
            "first_half_us": t1, "second_half_us": t2,
            "first_half_gbps": 56.0 * n / (t1 * 1e-6) / 1e9,
            "second_half_gbps": 32.0 * n / (t2 * 1e-6) / 1e9,
            "roofline": {"bound": "hbm", "achieved": gbps, "peak": 8000.0, "unit": "GB/s",
                         "frac": gbps / 8000.0,
                         "traffic": measured_traffic(None, NVT_PROFILE, NVT_SOURCES,
                                                     f"traffic_bytes_per_step_{n}")
                         if n == 3 * 2 ** 24 else None,
                         "kernel": "k_nvt_first + k_nvt_second"},
            "water_box_step_us": w1 + w2}


def accelerated_leg(pk, H, P, n_occ, n, args, p_ref, gold, n_iter, prods, nref, tol, headline):
    """The accelerated network of Section II.E: HOMO/LUMO estimates from the
    previous solve's P (the headline's last one, as a molecular-dynamics
    step would take them from the step before), then the same solves with
    the accelerated schedule.  The estimator is timed on its own."""
    import torch
    print("# accelerated leg", file=sys.stderr, flush=True)
    ws_est = pk.allocate_workspace(n, None, H.device)
    homo, lumo = pk.sp2_homo_lumo(H, P, ws_est, steps=args.est_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pk.sp2_homo_lumo(H, P, ws_est, steps=args.est_steps)
    torch.cuda.synchronize()
    est_ms = (time.perf_counter() - t0) / args.steps * 1e3
    del ws_est
    Pa, ainfos, asec = timed_solves(pk, H, n_occ, args.precision, args.refine, args.steps,
                                    args.warmup, False, args.bound_steps, homo, lumo, args.tol)
    aerr = full_error(Pa, p_ref) if p_ref is not None else sampled_error(Pa, gold)
    del Pa
    an = ainfos[-1]["n_iter"]
    return {
        "solves_per_s": 1.0 / asec, "ms_per_solve": asec * 1e3, "steps": args.steps,
        "n_iter": an, "n_iter_plain": n_iter, "converged": bool(ainfos[-1]["converged"]),
        "fallback": bool(ainfos[-1]["fallback"]),
        "homo_lumo_estimates": [homo, lumo], "estimator_ms": est_ms,
        "md_step_ms": asec * 1e3 + est_ms,
        "speedup_over_headline": (1.0 / asec) / headline,
        "effective_tflops": (an * prods + nref) * 2.0 * n ** 3 / asec / 1e12,
        "fro_over_sqrt_n": aerr["fro_over_sqrt_n"], "max_abs": aerr["max_abs"],
        "meets_tolerance": bool(aerr["fro_over_sqrt_n"] <= tol),
        "estimator_steps": args.est_steps,
        "note": f"estimates from the previous solve's P (sp2_homo_lumo, {args.est_steps} Lanczos steps per "
                "side, 5% margin); md_step_ms = estimator + accelerated solve, with the "
                "estimates refreshed every step"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.trajectory:
        trajectory(args.trajectory, args.traj_precision, args.traj_refine, args.traj_accelerate,
                   args.est_steps)
        return
    import torch

    import paper_2107_02737_amd as pk
    from workloads import water_box_hamiltonian

    gold = np.load(GOLDEN)
    m, n_occ = int(gold["molecules"]), int(gold["n_occ"])
    h32 = water_box_hamiltonian(m, seed=int(gold["seed"])).astype(np.float32)
    n = h32.shape[0]
    if abs(float(h32.astype(np.float64).sum()) - float(gold["h_sum"])) > 1e-6 * abs(float(gold["h_sum"])):
        raise RuntimeError("water-box generator drifted from the stored golden values")
    H = torch.from_numpy(h32).to("cuda")
    pk.load_library()
    print(f"# bench: water N={n} {args.precision} refine={args.refine} "
          f"bound_steps={args.bound_steps} tol={args.tol}", file=sys.stderr, flush=True)

    # the timed steps: solves only, no per-layer events
    P, infos, sec = timed_solves(pk, H, n_occ, args.precision, args.refine, args.steps,
                                 args.warmup, False, args.bound_steps, tol=args.tol)
    n_iter = infos[-1]["n_iter"]
    solve_ms = np.array([d["solve_ms"] for d in infos])
    prods = PRODUCTS[args.precision]
    nref = 2 if args.refine != "none" else 0
    eff_flop = (n_iter * prods + nref) * 2.0 * n ** 3
    # the same solves again with HIP events around every layer launch on the
    # solve's stream: the layer kernel's average launch duration
    _, tinfos, tsec = timed_solves(pk, H, n_occ, args.precision, args.refine, args.steps, 1,
                                   True, args.bound_steps, tol=args.tol)
    layer_ms = float(np.mean([d["layer_ms"] / max(1, d["n_iter"]) for d in tinfos]))
    # algorithmic work of one layer launch: upper-triangle tiles only, i.e.
    # prods * N^3 FMA = 2 * prods * N^3 / 2 flop
    layer_flop = prods * float(n) ** 3
    achieved = layer_flop / (layer_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    print(f"# headline {1.0 / sec:.2f} solves/s, layer {layer_ms:.3f} ms", file=sys.stderr,
          flush=True)

    if not args.no_mfma_probe and args.precision in ("bf16x3", "fp16x3"):
        print("# matrix-core rate probe", file=sys.stderr, flush=True)
        probe = mfma_probe(pk, H, n_occ, args.precision)
        mid = probe["operands"]["after 8 layers"]["tflops"]
        probe["layer_vs_probe_mid_solve"] = achieved / mid
        print(f"# probe: " + ", ".join(f"{k} {v['tflops']:.0f} TFLOP/s @ {v['shader_ghz']:.2f} GHz"
                                        for k, v in probe["operands"].items()),
              file=sys.stderr, flush=True)
    else:
        probe = None

    p_ref, cb = None, None
    if not args.no_cpu_baseline:
        print("# cpu baseline (FP64 oracle on the host cores)", file=sys.stderr, flush=True)
        p_ref, cb = cpu_baseline(h32, n_occ, args.cpu_layers, n_iter)
    err = full_error(P, p_ref) if p_ref is not None else sampled_error(P, gold)
    err.update(device_checks(P, n_occ))
    tol = TOL_FP32_EQUIVALENT if args.precision in ("fp16x3", "bf16x3", "fp32") else TOL_SINGLE_PASS_BF16
    err["stated_tolerance"] = tol
    err["meets_tolerance"] = bool(err["fro_over_sqrt_n"] <= tol)

    out = {
        "metric": METRIC,
        "value": 1.0 / sec,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16", "bf16x1": "bf16", "fp16x3": "fp16", "fp32": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"tight-binding water box, {m} molecules, N={n}, n_occ={n_occ}, "
                               f"seed {int(gold['seed'])}, H fp32 on device",
                   "n": n, "n_occ": n_occ, "precision": args.precision, "refine": args.refine,
                   "tol": args.tol,
                   "bounds": "gershgorin" if args.bound_steps == 0
                   else f"gershgorin + lanczos {args.bound_steps} steps",
                   "parallelism": "single GPU"},
        "n_iter": n_iter,
        "solve_ms": {"median": float(np.median(solve_ms)), "p10": float(np.percentile(solve_ms, 10)),
                     "p90": float(np.percentile(solve_ms, 90)), "source": "HIP events per solve"},
        "effective_tflops": eff_flop / sec / 1e12,
        "paper_context": {
            "effective_tera_fma_per_s": eff_flop / 2.0 / sec / 1e12,
            "paper": "more than 100 Tflops on one A100 counting an FMA as one flop, three "
                     "products per split layer, N = 19,008 (Section II.E); other hardware and "
                     "inputs: context, not a target",
        },
        "error_vs_oracle": err,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(args.precision),
                     "kernel": f"k_sym_split<{args.precision}> + k_split_tail (layer product)"
                               if args.precision != "fp32" else "k_sym_f32 + k_split_tail",
                     "layer_ms": layer_ms,
                     "layer_flop": layer_flop,
                     "refine_ms": float(np.mean([d["refine_ms"] for d in tinfos])),
                     "timing": f"HIP events around every layer launch, {args.steps} solves "
                               "after the timed ones",
                     "solves_per_s_with_layer_events": 1.0 / tsec,
                     "mfma_only_probe": probe},
    }

    def leg(precision, refine, bound_steps, label):
        print(f"# leg {label}", file=sys.stderr, flush=True)
        Pl, linfo, lsec = timed_solves(pk, H, n_occ, precision, refine, args.steps, args.warmup,
                                       False, bound_steps, tol=args.tol)
        lerr = full_error(Pl, p_ref) if p_ref is not None else sampled_error(Pl, gold)
        del Pl
        return {"precision": precision, "refine": refine, "bound_steps": bound_steps,
                "solves_per_s": 1.0 / lsec, "steps": args.steps, "n_iter": linfo[-1]["n_iter"],
                "converged": bool(linfo[-1]["converged"]),
                "fro_over_sqrt_n": lerr["fro_over_sqrt_n"], "max_abs": lerr["max_abs"]}

    # The accelerated network of Section II.E: HOMO/LUMO estimates from the
    # previous solve's P (the headline's last one, as a molecular-dynamics
    # step would take them from the step before), then the same solves with
    # the accelerated schedule.  The estimator is timed on its own.
    if not args.no_accelerated:
        out["accelerated"] = accelerated_leg(pk, H, P, n_occ, n, args, p_ref, gold, n_iter, prods,
                                             nref, tol, out["value"])

    if not args.no_legs:
        legs = {}
        legs["fp16x3_fp32_refine"] = leg("fp16x3", "fp32", args.bound_steps,
                                         "FP16 pair, FP32 refinement")
        legs["bf16x3_gershgorin"] = leg("bf16x3", "fp32", 0, "BF16 pair, Gershgorin bounds")
        legs["bf16x3_lanczos"] = leg("bf16x3", "fp32", args.bound_steps,
                                     "BF16 pair, Lanczos bounds")
        sp = leg("bf16x1", "split", args.bound_steps, "single-pass BF16")
        sp["stated_tolerance"] = TOL_SINGLE_PASS_BF16
        sp["meets_tolerance"] = bool(sp["fro_over_sqrt_n"] <= TOL_SINGLE_PASS_BF16)
        if not sp["meets_tolerance"]:
            sp["note"] = ("single-pass BF16 misses its stated 1e-3 here: every BF16 rounding "
                          "of the centred iterate near convergence leaves an occupied-virtual "
                          "error that later layers keep")
        legs["bf16x1_single_pass"] = sp
        f32 = leg("fp32", "fp32", args.bound_steps, "plain FP32 MFMA SP2")
        f32["speedup_of_headline"] = out["value"] / f32["solves_per_s"]
        legs["fp32_sp2"] = f32
        out["legs"] = legs
    if args.xl_rank > 0:
        print("# XL-BOMD kernel block", file=sys.stderr, flush=True)
        out["xl_kernel"] = xl_kernel(pk, int(gold["seed"]), args.xl_rank, "bf16x3", args.refine)
        out["xl_kernel_split_derivatives"] = xl_kernel(pk, int(gold["seed"]), args.xl_rank,
                                                       "bf16x3", args.refine, True)
    if args.nvt_coords > 0:
        print("# canonical step", file=sys.stderr, flush=True)
        out["canonical_step"] = canonical_step(pk, args.nvt_coords)
    if not args.no_diag:
        print("# GPU diagonalisation context (library eigh)", file=sys.stderr, flush=True)
        try:
            dg = diagonalization_baseline(H, n_occ, p_ref)
            for name in ("float32", "float64"):
                dg[name]["headline_speedup"] = dg[name]["seconds"] * out["value"]
            out["gpu_diagonalization"] = dg
        except RuntimeError as e:   # a missing or failing solver library: report, go on
            out["gpu_diagonalization"] = {"error": str(e)[:300]}
    if cb is not None:
        cb["gpu_speedup_vs_oracle_sp2"] = out["value"] / cb["value"]
        cb["gpu_speedup_vs_oracle_eigh"] = cb["eigh_seconds"] * out["value"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
