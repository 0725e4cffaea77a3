"""Concurrent solves from several host threads through the C ABI.

Every call's device state lives in its caller's workspace and the host
state in per-thread storage, so independent callers (each with its own
stream and workspace) must not interfere: results are bitwise those of the
same calls made one after another.  ctypes releases the interpreter lock
during library calls, so the threads do run inside the library together."""

import threading

import numpy as np
import pytest

from gpu_util import banner
from workloads import random_orthogonal_hamiltonian, symmetric_normal, water_box_hamiltonian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_2107_02737_amd as pk
    pk.load_library()
    return pk


def _cases():
    return [
        ("water N=1200", water_box_hamiltonian(200, seed=1).astype(np.float32), 800, "bf16x3", 0),
        ("c1 N=256", random_orthogonal_hamiltonian(256, 128, seed=0).astype(np.float32), 128, "fp32", 0),
        ("random N=777", random_orthogonal_hamiltonian(777, 300, seed=4).astype(np.float32), 300,
         "fp16x3", 16),
        ("water N=600", water_box_hamiltonian(100, seed=2).astype(np.float32), 400, "bf16x3", 24),
    ]


def _work(pk, h32, n_occ, precision, bound_steps, repeats=3):
    """Solves with a tape, then one JVP; returns host copies of everything."""
    import torch
    H = torch.from_numpy(h32).to("cuda")
    H1 = torch.from_numpy(symmetric_normal(h32.shape[0], seed=7, std=1e-3).astype(np.float32)).to("cuda")
    out = []
    for _ in range(repeats):
        P, info = pk.density(H, n_occ, precision=precision, bound_steps=bound_steps,
                             checkpoint_every=4, return_info=True)
        P1 = torch.empty_like(H1)
        pk.sp2_jvp(info["workspace"], H1, P1)
        torch.cuda.current_stream().synchronize()
        out.append((P.cpu().numpy(), P1.cpu().numpy(), info["n_iter"], info["branches"],
                    info["eps_min"], info["eps_max"]))
    return out


def test_threads_match_sequential_calls(pk):
    import torch
    cases = _cases()
    banner("concurrency: sequential reference")
    ref = [_work(pk, h, n_occ, prec, bs) for _, h, n_occ, prec, bs in cases]
    results = [None] * len(cases)
    errors = []

    def run(i):
        try:
            with torch.cuda.stream(torch.cuda.Stream()):
                _, h, n_occ, prec, bs = cases[i]
                results[i] = _work(pk, h, n_occ, prec, bs)
        except Exception as e:  # reported below
            errors.append((cases[i][0], repr(e)))

    banner(f"concurrency: {len(cases)} threads")
    threads = [threading.Thread(target=run, args=(i,)) for i in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=100)
    assert not any(t.is_alive() for t in threads), "a solver thread did not finish"
    assert not errors, errors
    for (name, *_), r, s in zip(cases, ref, results):
        for (p, p1, it, br, lo, hi), (q, q1, it2, br2, lo2, hi2) in zip(r, s):
            assert it == it2 and br == br2 and lo == lo2 and hi == hi2, name
            assert np.array_equal(p, q) and np.array_equal(p1, q1), name
        print(f"  {name}: {len(s)} solves + JVPs bitwise equal", flush=True)
