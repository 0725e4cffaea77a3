"""Checks of the seeded input generators (shapes, seeds, geometry and the
spectral structure the water model has by construction).  CPU only."""

import math

import numpy as np

from workloads import (pad_matrix, random_orthogonal_hamiltonian, symmetric_normal,
                       trajectory_perturbation, water_box_hamiltonian, water_box_length,
                       water_box_positions)


def test_random_orthogonal_spectrum_and_seed():
    h, q, e = random_orthogonal_hamiltonian(64, 20, occ_range=(-2, -0.1), virt_range=(0.1, 2),
                                            seed=3, return_factors=True)
    assert np.array_equal(h, h.T)
    assert np.allclose(q.T @ q, np.eye(64), atol=1e-13)
    assert np.all(e[:20] <= -0.1) and np.all(e[20:] >= 0.1)
    assert np.allclose(np.sort(np.linalg.eigvalsh(h)), np.sort(e), atol=1e-12)
    assert np.array_equal(h, random_orthogonal_hamiltonian(64, 20, occ_range=(-2, -0.1),
                                                           virt_range=(0.1, 2), seed=3))


def test_water_box_edge_matches_density():
    # 1 g/cm^3: 18.015 g/mol / N_A = 29.915 cubic Angstrom per molecule
    assert abs(water_box_length(1024) - 31.289) < 1e-3
    assert abs(water_box_length(1) ** 3 - 29.915) < 1e-3


def test_water_geometry():
    atoms, box = water_box_positions(64, seed=0)
    o = atoms[0::3]
    d = o[:, None, :] - o[None, :, :]
    d -= box * np.round(d / box)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(64) * 1e9
    assert r.min() >= 2.5 - 1e-12
    for k in range(64):
        oh1 = atoms[3 * k + 1] - atoms[3 * k]
        oh2 = atoms[3 * k + 2] - atoms[3 * k]
        assert abs(np.linalg.norm(oh1) - 0.96) < 1e-12 and abs(np.linalg.norm(oh2) - 0.96) < 1e-12
        ang = math.degrees(math.acos(oh1 @ oh2 / 0.96 ** 2))
        assert abs(ang - 104.5) < 1e-9


def test_isolated_molecule_spectrum_closed_form():
    """Angle-free hopping: the two p combinations orthogonal to (1,1,1) and the
    antisymmetric H combination decouple; the rest is a 3x3 problem."""
    h = water_box_hamiltonian(5, seed=1, block_diagonal=True)
    t1 = -math.exp(-0.96)
    r_hh = 2 * 0.96 * math.sin(math.radians(104.5 / 2))
    t2 = -math.exp(-r_hh)
    red = np.array([[-1.0, 0.0, math.sqrt(2) * t1],
                    [0.0, -0.5, math.sqrt(6) * t1],
                    [math.sqrt(2) * t1, math.sqrt(6) * t1, -0.3 + t2]])
    expected = np.sort(np.concatenate([np.linalg.eigvalsh(red), [-0.5, -0.5, -0.3 - t2]]))
    for k in range(5):
        blk = h[6 * k:6 * k + 6, 6 * k:6 * k + 6]
        assert np.allclose(np.linalg.eigvalsh(blk), expected, atol=1e-12)


def test_water_box_structure():
    m = 64
    h = water_box_hamiltonian(m, seed=0)
    assert h.shape == (6 * m, 6 * m) and np.array_equal(h, h.T)
    w = np.linalg.eigvalsh(h)
    # exactly 2M-fold level at -0.5 (decoupled p combinations)
    assert np.sum(np.abs(w + 0.5) < 1e-9) == 2 * m
    # chemical filling (4 doubly occupied orbitals per molecule) sits below a gap
    assert w[4 * m] - w[4 * m - 1] > 0.25


def test_padding_and_operands():
    h = water_box_hamiltonian(10, seed=0, n_pad=64)
    assert h.shape == (64, 64) and not h[60:].any() and not h[:, 60:].any()
    assert np.array_equal(pad_matrix(h[:60, :60], 64), h)
    s = symmetric_normal(64, 2, std=1e-3, n_real=60)
    assert np.array_equal(s, s.T) and not s[60:].any()
    assert 0.5e-3 < s[:60, :60].std() < 2e-3
    hp = trajectory_perturbation(64, 3, n_real=60)
    assert np.array_equal(hp, hp.T) and not hp[:, 60:].any()
    assert 0.7 < np.linalg.norm(hp[:60, :60], 2) < 1.3


def test_water_charge_model():
    from workloads import charge_shifted_hamiltonian, random_charges, water_charge_model
    mod = water_charge_model(5, seed=2)
    ptr, g = mod["atom_ptr"], mod["gamma"]
    assert ptr.tolist()[:4] == [0, 4, 5, 6] and ptr[-1] == 30 and ptr.size == 16
    assert mod["z"].sum() == 2 * mod["n_occ"]            # neutral at n_occ = 4M
    assert np.array_equal(g, g.T) and np.all(np.diag(g)[:3] == [0.5, 0.4, 0.4])
    assert np.all(np.linalg.eigvalsh(g) > 0)
    c = random_charges(15, seed=1)
    assert abs(c.sum()) < 1e-15
    h = charge_shifted_hamiltonian(mod["h0"], ptr, g, c)
    shift = g @ c
    assert np.allclose(np.diag(h - mod["h0"]), np.repeat(shift, np.diff(ptr)))
    off = (h - mod["h0"]) - np.diag(np.diag(h - mod["h0"]))
    assert np.all(off == 0)
