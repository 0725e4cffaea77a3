"""GPU solves of small and structured inputs whose density matrix is known
without the solver, through the C ABI.

* n = 1 (both occupations are trivial) and n = 2, 3 with every non-trivial
  occupation: the 2 x 2 closed form ``P = (I - (H - tr(H)/2 I) / r) / 2``
  with ``r = sqrt(((a - c)/2)^2 + b^2)`` for one occupied state, FP64
  ``eigh`` of the cast matrix otherwise.
* Diagonal ``H`` (N = 300, ragged): ``P`` is the indicator of the ``n_occ``
  smallest diagonal entries; every off-diagonal entry stays exactly zero
  under the layer products (sums of zero products), in every mode.
* Block-diagonal water (no intermolecular hopping, N = 300): each 6 x 6
  molecule block is its own problem with four occupied states; ``P`` is
  their per-block ``eigh`` projectors and is exactly zero between blocks.
* Extreme occupations ``n_occ = 1`` and ``n_occ = N - 1`` (N = 300).
* Exact invariances of the network (Section II.D): scaling ``H`` by a power
  of two scales the bounds exactly and leaves the input layer, every layer,
  the branch string and ``P`` bitwise unchanged (Gershgorin and Lanczos
  bounds); a symmetric permutation of ``H`` permutes ``P`` (within rounding,
  since the sums run in another order).

Tolerances follow the other solve tests: 3x the FP32-storage emulation of
the same network (``oracle.precision_emulation``) plus a floor of 2e-6 for
FP32 rounding that the emulation orders differently."""

import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev, to_host
from oracle.precision_emulation import sp2_emulated
from workloads import random_orthogonal_hamiltonian, water_box_hamiltonian

pytestmark = pytest.mark.gpu

MODES = ["fp32", "bf16x1", "bf16x3", "fp16x3"]


@pytest.fixture(scope="module")
def pk():
    import paper_2107_02737_amd as pk
    pk.load_library()
    return pk


def _fro(p, q):
    return float(np.linalg.norm(p - q) / np.sqrt(p.shape[0]))


def _tol(h32, n_occ, p_exact, mode, refine="fp32", floor=2e-6):
    pe, _ = sp2_emulated(h32, n_occ, mode, refine=refine != "none")
    return 3.0 * _fro(pe.astype(np.float64), p_exact) + floor


def _solve(pk, h32, n_occ, **kw):
    P, info = pk.density(to_dev(h32), n_occ, return_info=True, **kw)
    return to_host(P), info


@pytest.mark.parametrize("n_occ", [0, 1])
def test_single_orbital(pk, n_occ):
    banner(f"n=1 n_occ={n_occ}")
    p, info = _solve(pk, np.array([[0.3]], dtype=np.float32), n_occ)
    assert p.shape == (1, 1) and p[0, 0] == float(n_occ)
    assert info["n_iter"] == 0 and info["converged"] == 1


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("mode", MODES)
def test_two_by_two_closed_form(pk, seed, mode):
    banner(f"n=2 closed form seed={seed} mode={mode}")
    rng = np.random.default_rng(100 + seed)
    a, c = rng.uniform(-1.0, 1.0, 2)
    b = rng.uniform(0.1, 0.5)
    h32 = np.array([[a, b], [b, c]], dtype=np.float32)
    h = h32.astype(np.float64)
    r = np.sqrt(((h[0, 0] - h[1, 1]) / 2) ** 2 + h[0, 1] ** 2)
    p_exact = 0.5 * (np.eye(2) - (h - 0.5 * np.trace(h) * np.eye(2)) / r)
    p, info = _solve(pk, h32, 1, precision=mode)
    tol = _tol(h32, 1, p_exact, mode)
    print(f"  n_iter={info['n_iter']} err={_fro(p, p_exact):.2e} tol={tol:.2e}", flush=True)
    assert info["converged"] == 1
    assert _fro(p, p_exact) <= tol
    assert p[0, 1] == p[1, 0]


@pytest.mark.parametrize("n_occ", [1, 2])
def test_three_orbitals(pk, n_occ):
    banner(f"n=3 n_occ={n_occ}")
    h32 = np.array([[0.2, 0.3, -0.1], [0.3, -0.5, 0.2], [-0.1, 0.2, 0.9]], dtype=np.float32)
    p_exact = oracle.density_matrix_eigh(h32.astype(np.float64), n_occ)[0]
    for mode in ("fp32", "bf16x3", "fp16x3"):
        p, info = _solve(pk, h32, n_occ, precision=mode)
        assert info["converged"] == 1
        assert _fro(p, p_exact) <= _tol(h32, n_occ, p_exact, mode), mode
        assert abs(np.trace(p) - n_occ) <= 1e-5


@pytest.mark.parametrize("mode", MODES)
def test_diagonal_hamiltonian(pk, mode):
    banner(f"diagonal N=300 n_occ=120 mode={mode}")
    rng = np.random.default_rng(7)
    d = np.concatenate([rng.uniform(-2.0, -0.5, 120), rng.uniform(0.5, 2.0, 180)])
    d = rng.permutation(d)
    h32 = np.diag(d).astype(np.float32)
    p_exact = np.diag((d < 0).astype(np.float64))
    p, info = _solve(pk, h32, 120, precision=mode)
    err = _fro(p, p_exact)
    print(f"  n_iter={info['n_iter']} err={err:.2e}", flush=True)
    assert info["converged"] == 1
    assert not np.any(p - np.diag(np.diag(p)))            # off-diagonal exactly zero
    assert err <= _tol(h32, 120, p_exact, mode)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "fp16x3"])
def test_block_diagonal_water(pk, mode):
    banner(f"block-diagonal water N=300 mode={mode}")
    m = 50
    h32 = water_box_hamiltonian(m, seed=4, block_diagonal=True).astype(np.float32)
    h = h32.astype(np.float64)
    p_exact = np.zeros_like(h)
    for k in range(m):
        s = slice(6 * k, 6 * k + 6)
        _, v = np.linalg.eigh(h[s, s])
        p_exact[s, s] = v[:, :4] @ v[:, :4].T
    p, info = _solve(pk, h32, 4 * m, precision=mode)
    err = _fro(p, p_exact)
    print(f"  n_iter={info['n_iter']} err={err:.2e}", flush=True)
    assert info["converged"] == 1
    mask = np.kron(np.eye(m), np.ones((6, 6))) == 0
    assert not np.any(p[mask])                            # exactly zero between molecules
    assert err <= _tol(h32, 4 * m, p_exact, mode)


@pytest.mark.parametrize("n_occ", [1, 299])
@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_extreme_occupations(pk, n_occ, mode):
    banner(f"N=300 n_occ={n_occ} mode={mode}")
    h32 = random_orthogonal_hamiltonian(300, n_occ, seed=11).astype(np.float32)
    p_exact = oracle.density_matrix_eigh(h32.astype(np.float64), n_occ)[0]
    p, info = _solve(pk, h32, n_occ, precision=mode)
    err = _fro(p, p_exact)
    print(f"  n_iter={info['n_iter']} err={err:.2e}", flush=True)
    assert info["converged"] == 1
    assert err <= _tol(h32, n_occ, p_exact, mode)
    assert abs(info["trace"] - n_occ) <= 1e-3


@pytest.mark.parametrize("bound_steps", [0, 16])
@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "fp16x3"])
def test_power_of_two_scaling_is_exact(pk, mode, bound_steps):
    banner(f"scaling water N=300 mode={mode} bound_steps={bound_steps}")
    h32 = water_box_hamiltonian(50, seed=3).astype(np.float32)
    p0, i0 = _solve(pk, h32, 200, precision=mode, bound_steps=bound_steps)
    assert i0["converged"] == 1
    for scale in (4.0, 0.125):
        p, info = _solve(pk, (h32 * np.float32(scale)).astype(np.float32), 200, precision=mode,
                         bound_steps=bound_steps)
        assert info["eps_min"] == scale * i0["eps_min"]
        assert info["eps_max"] == scale * i0["eps_max"]
        assert info["branches"] == i0["branches"]
        assert np.array_equal(p, p0), f"scale {scale}"


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_permutation_equivariance(pk, mode):
    banner(f"permutation water N=300 mode={mode}")
    h32 = water_box_hamiltonian(50, seed=6).astype(np.float32)
    perm = np.random.default_rng(3).permutation(300)
    p_exact = oracle.density_matrix_eigh(h32.astype(np.float64), 200)[0]
    tol = _tol(h32, 200, p_exact, mode)
    p, _ = _solve(pk, h32, 200, precision=mode)
    pp, info = _solve(pk, np.ascontiguousarray(h32[np.ix_(perm, perm)]), 200, precision=mode)
    back = np.empty_like(pp)
    back[np.ix_(perm, perm)] = pp
    print(f"  err {_fro(p, p_exact):.2e} permuted {_fro(back, p_exact):.2e} "
          f"difference {_fro(back, p):.2e}", flush=True)
    assert info["converged"] == 1
    assert _fro(back, p_exact) <= tol
    assert _fro(back, p) <= 2 * tol
