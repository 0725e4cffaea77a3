"""Seeded inputs for the canonical integration scheme (Section IV).

Units: eV, Angstrom, fs; masses in eV fs^2 / Angstrom^2 (``AMU`` per atomic
mass unit).  The test well is a Morse potential
``U(r) = D (1 - exp(-a (r - r0)))^2`` (curvature ``2 D a^2`` at ``r0``);
the force noise is Laplace distributed with zero mean and unit variance
(the approximately double-sided exponential force errors of Section IV);
the Langevin noise is standard normal.  Nothing here advances a coordinate.
"""

from __future__ import annotations

import math

import numpy as np

AMU = 103.642697            # eV fs^2 / Angstrom^2 per atomic mass unit
KB_EV = 8.617333262e-5      # Boltzmann constant, eV / K

MORSE_D = 2.0               # eV (46 kT at 500 K: no escape over the plateau)
MORSE_A = 1.0               # 1 / Angstrom
MORSE_R0 = 1.0              # Angstrom


def morse_energy(r, d=MORSE_D, a=MORSE_A, r0=MORSE_R0):
    e = 1.0 - np.exp(-a * (np.asarray(r, dtype=np.float64) - r0))
    return d * e * e


def morse_force(r, d=MORSE_D, a=MORSE_A, r0=MORSE_R0):
    """``-dU/dr``."""
    x = np.exp(-a * (np.asarray(r, dtype=np.float64) - r0))
    return -2.0 * d * a * x * (1.0 - x)


def laplace_unit(rng, shape):
    """Laplace samples with zero mean and unit variance (scale 1/sqrt(2))."""
    return rng.laplace(0.0, 1.0 / math.sqrt(2.0), size=shape)


def canonical_noise(steps, n, seed):
    """``(eta, xi)``: ``steps x n`` standard normal Langevin noise and
    ``(steps + 1) x n`` unit-variance Laplace force noise (row 0 belongs to
    the force at the initial positions)."""
    rng = np.random.default_rng(seed)
    eta = rng.standard_normal((steps, n))
    xi = laplace_unit(rng, (steps + 1, n))
    return eta, xi


def water_atom_masses(n_molecules):
    """Per-coordinate masses (x, y, z of O, H, H per molecule), eV fs^2/A^2."""
    per_atom = np.tile(np.array([15.999, 1.008, 1.008]) * AMU, n_molecules)
    return np.repeat(per_atom, 3)
