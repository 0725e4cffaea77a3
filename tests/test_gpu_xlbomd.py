"""XL-BOMD kernel building block on the GPU (sp2_mulliken, sp2_xl_response,
sp2_xl_kernel) against the FP64 oracle (oracle/xlbomd.py).

The charge-space Jacobian is built from density-matrix responses, so the
same rule as for the JVP applies: the GPU's branch string is validated
against FP64 decisions first, and the oracle then differentiates that same
network in FP64 (Daleckii-Krein form, no GPU-derived matrix); the exact
step-function response (perturbation theory) is checked too.  Tolerances
follow the JVP's: relative 1e-4 for the FP32 network, 1e-3 for the split
network; the Krylov bookkeeping adds only FP64 rounding.  At the 4096-orbital
size the minimal residual the GPU reports is checked against an independent
response of its result, J kf, computed through the C ABI."""

import numpy as np
import pytest

from gpu_util import banner, to_dev, to_host
from oracle import daleckii_krein_jvp, density_matrix_eigh, dmpt_response, xlbomd
from test_gpu_derivatives import validated_record
from workloads import charge_shifted_hamiltonian, random_charges, water_charge_model

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_2107_02737_amd as pk
    pk.load_library()
    return pk


def _dvec(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype or np.float64)).to("cuda")


def _setup(pk, m, precision, refine="fp32", n_pad=None, seed=0, n_occ=None, validate=True,
           split=False):
    mod = water_charge_model(m, seed=seed, n_pad=n_pad)
    charges = random_charges(3 * m, seed=5)
    h = charge_shifted_hamiltonian(mod["h0"], mod["atom_ptr"], mod["gamma"], charges)
    h32 = h.astype(np.float32)
    n_occ = mod["n_occ"] if n_occ is None else n_occ
    P, info = pk.density(to_dev(h32), n_occ, precision=precision, refine=refine,
                         checkpoint_every=4, return_info=True, split_derivatives=split)
    h64 = h32.astype(np.float64)
    rec = None
    if validate and 0 < n_occ < h.shape[0]:
        rec, _ = validated_record(h64, n_occ, info, precision, refine)
    dev = {"ptr": _dvec(mod["atom_ptr"], np.int64), "z": _dvec(mod["z"]),
           "gamma": _dvec(mod["gamma"]), "charges": _dvec(charges)}
    return mod, charges, h64, n_occ, P, info, rec, dev


def _dk_jacobian(mod, h64, rec):
    n = h64.shape[0]
    return xlbomd.jacobian(n, mod["atom_ptr"], mod["gamma"], lambda h1: daleckii_krein_jvp(h64, h1, rec))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n_pad", [None, 305])
def test_mulliken_residual_matches_oracle(pk, n_pad):
    banner(f"mulliken M=50 n_pad={n_pad}")
    mod, charges, h64, n_occ, P, info, rec, dev = _setup(pk, 50, "fp32", n_pad=n_pad)
    f = pk.sp2_mulliken(P, dev["ptr"], dev["z"], sub=dev["charges"])
    q = pk.sp2_mulliken(P, dev["ptr"], dev["z"])
    p_host = to_host(P)
    q_ref = xlbomd.mulliken_charges(p_host, mod["atom_ptr"], mod["z"])
    # the same FP32 diagonal summed in the same order in FP64
    assert np.abs(to_host(q) - q_ref).max() <= 1e-13
    assert np.abs(to_host(f) - (q_ref - charges)).max() <= 1e-13
    assert abs(float(to_host(q).sum())) <= 1e-3        # Tr P = n_occ: neutral box
    # against the exact charges of H(n)
    q_exact = xlbomd.mulliken_charges(density_matrix_eigh(h64, n_occ)[0],
                                      mod["atom_ptr"], mod["z"])
    assert np.abs(to_host(q) - q_exact).max() <= 1e-4


@pytest.mark.parametrize("precision,tol,split", [("fp32", 1e-4, False), ("bf16x3", 1e-3, False),
                                                 ("bf16x3", 1e-3, True)])
def test_response_matches_oracle(pk, precision, tol, split):
    banner(f"xl response M=50 {precision} split_derivatives={split}")
    mod, charges, h64, n_occ, P, info, rec, dev = _setup(pk, 50, precision, split=split)
    na = charges.size
    v = np.random.default_rng(11).standard_normal(na)
    scratch = pk.allocate_xl_scratch(h64.shape[0], na, 1)
    jv = to_host(pk.sp2_xl_response(info["workspace"], dev["ptr"], dev["gamma"], _dvec(v), scratch))
    n = h64.shape[0]
    ref = xlbomd.charge_response(n, mod["atom_ptr"], mod["gamma"], v,
                                 lambda h1: daleckii_krein_jvp(h64, h1, rec)) - v
    exact = xlbomd.charge_response(n, mod["atom_ptr"], mod["gamma"], v,
                                   lambda h1: dmpt_response(h64, n_occ, h1)) - v
    print(f"  rel vs network {_rel(jv, ref):.2e}  vs perturbation theory {_rel(jv, exact):.2e}",
          flush=True)
    assert _rel(jv, ref) <= tol
    assert _rel(jv, exact) <= max(tol, 1e-3)
    # dq0/dn v moves charge but creates none: sum(J v) = -sum(v)
    assert abs((jv + v).sum()) <= tol * np.abs(jv + v).sum()


@pytest.mark.parametrize("rank", [1, 4, 8])
def test_krylov_matches_oracle(pk, rank):
    banner(f"xl kernel M=50 fp32 rank={rank}")
    mod, charges, h64, n_occ, P, info, rec, dev = _setup(pk, 50, "fp32")
    na = charges.size
    f = pk.sp2_mulliken(P, dev["ptr"], dev["z"], sub=dev["charges"])
    scratch = pk.allocate_xl_scratch(h64.shape[0], na, rank)
    kf, rho, used = pk.sp2_xl_kernel(info["workspace"], dev["ptr"], dev["gamma"], f, rank, scratch)
    jmat = _dk_jacobian(mod, h64, rec)
    kf_ref, rho_ref, _ = xlbomd.krylov_kernel(to_host(f), lambda x: jmat @ x, rank)
    print(f"  used {used}  kf rel {_rel(to_host(kf), kf_ref):.2e}  rho {np.array(rho) / rho[0]}",
          flush=True)
    assert used == rank
    assert _rel(to_host(kf), kf_ref) <= 1e-4
    assert np.allclose(rho, rho_ref, rtol=0, atol=1e-4 * rho_ref[0])
    assert all(b <= a * (1 + 1e-12) for a, b in zip(rho, rho[1:]))
    # deterministic: a second call is bitwise identical
    kf2, rho2, _ = pk.sp2_xl_kernel(info["workspace"], dev["ptr"], dev["gamma"], f, rank, scratch)
    assert bool((kf2 == kf).all()) and rho2 == rho


def test_full_rank_and_exact_preconditioner(pk):
    banner("xl kernel M=4 full rank / exact K0")
    mod, charges, h64, n_occ, P, info, rec, dev = _setup(pk, 4, "fp32")
    na = charges.size
    jmat = _dk_jacobian(mod, h64, rec)
    f = np.random.default_rng(9).standard_normal(na)
    exact = np.linalg.solve(jmat, f)
    scratch = pk.allocate_xl_scratch(h64.shape[0], na, na)
    kf, rho, used = pk.sp2_xl_kernel(info["workspace"], dev["ptr"], dev["gamma"], _dvec(f), na,
                                     scratch)
    print(f"  full rank: used {used} rel {_rel(to_host(kf), exact):.2e} rho_end/rho_0 "
          f"{rho[-1] / rho[0]:.2e}", flush=True)
    assert _rel(to_host(kf), exact) <= 1e-4 and rho[-1] <= 1e-4 * rho[0]
    kf1, rho1, used1 = pk.sp2_xl_kernel(info["workspace"], dev["ptr"], dev["gamma"], _dvec(f), 1,
                                        scratch, k0=_dvec(np.linalg.inv(jmat)))
    assert used1 == 1 and _rel(to_host(kf1), exact) <= 1e-4 and rho1[1] <= 1e-4 * rho1[0]


def test_degenerate_cases(pk):
    banner("xl kernel zero residual / empty occupation")
    mod, charges, h64, n_occ, P, info, rec, dev = _setup(pk, 4, "fp32")
    na = charges.size
    scratch = pk.allocate_xl_scratch(h64.shape[0], na, 4)
    kf, rho, used = pk.sp2_xl_kernel(info["workspace"], dev["ptr"], dev["gamma"], _dvec(np.zeros(na)),
                                     4, scratch)
    assert used == 0 and rho == [0.0] * 5 and not bool(kf.any())
    # n_occ = 0: P does not depend on H, so J = -I and K f = -f
    mod, charges, h64, n_occ, P, info, rec, dev = _setup(pk, 4, "fp32", n_occ=0)
    f = np.random.default_rng(1).standard_normal(na)
    kf, rho, used = pk.sp2_xl_kernel(info["workspace"], dev["ptr"], dev["gamma"], _dvec(f), 4,
                                     scratch)
    assert used == 1 and np.allclose(to_host(kf), -f, rtol=1e-14, atol=0)


def test_residual_property_at_4096(pk):
    # water, 682 molecules + 4 padding orbitals (N = 4096, 2046 atoms)
    banner("xl kernel N=4096 bf16x3 (split derivatives) rank=4 + independent J kf")
    mod, charges, h64, n_occ, P, info, rec, dev = _setup(pk, 682, "bf16x3", n_pad=4096,
                                                          validate=False, split=True)
    na = charges.size
    f = pk.sp2_mulliken(P, dev["ptr"], dev["z"], sub=dev["charges"])
    scratch = pk.allocate_xl_scratch(4096, na, 4)
    kf, rho, used = pk.sp2_xl_kernel(info["workspace"], dev["ptr"], dev["gamma"], f, 4, scratch)
    jkf = pk.sp2_xl_response(info["workspace"], dev["ptr"], dev["gamma"], kf, scratch)
    # K0 = -I: the minimal residual is |-(J kf) + f|
    direct = float(np.linalg.norm(to_host(f) - to_host(jkf)))
    print(f"  used {used} rho/rho0 {np.array(rho) / rho[0]}  |f - J kf| {direct:.3e} vs rho_4 "
          f"{rho[4]:.3e}", flush=True)
    assert used == 4
    assert all(b <= a * (1 + 1e-12) for a, b in zip(rho, rho[1:]))
    assert rho[4] < 0.1 * rho[0]
    assert abs(direct - rho[4]) <= 1e-3 * rho[0]
