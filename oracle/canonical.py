"""Canonical integration with force noise as the heat bath -- TEST
INFRASTRUCTURE ONLY.

Section IV treats the error of the low-precision forces as a random force
``sigma_TC xi`` (zero mean, unit variance, not necessarily Gaussian) and
balances it with a friction term; an optional ordinary Langevin thermostat
(friction ``gamma_L``, Gaussian noise ``eta``) can be added.  This module is
the plain FP64 reference of one time step for a set of independent scalar
coordinates (each with its own mass), in two forms:

* scheme 0, Eq. 31: half kick with the force and the friction
  ``gamma_TC V``; half drift; Langevin velocity update
  ``V <- c_L V + sigma_L eta``; half drift; half kick with the new force and
  the friction on the new velocity (solved for it: the last sub-step is
  implicit in ``V_{k+1}``);
* scheme 1, the alternative of the Supporting Information: plain half kicks,
  and the friction applied as the factor ``sqrt(c_TC)`` on both sides of
  the Langevin update.

Coefficients (Eq. 32-33): ``c_L = (1 - gamma_L dt/2) / (1 + gamma_L dt/2)``,
``sigma_L = sqrt(kT (1 - c_L^2) / M)``, ``sigma_TC^2 = 2 kT gamma_TC / dt``.

Reading of the units: in Eq. 31 ``gamma_TC`` multiplies a velocity inside a
force, so it is a force per unit velocity (mass per time); Eq. 33 then fixes
it from the noise level.  The Supporting Information writes its variant with
a per-time friction ``gamma`` and ``sigma_TC^2 = 2 kT gamma M / dt``, which
is the same relation for ``gamma = gamma_TC / M``; so
``c_TC = (1 - gamma_TC dt/(2M)) / (1 + gamma_TC dt/(2M))`` here.

A step is split where the force is evaluated: ``first_half`` takes
``R_k, V_k, F_k, eta_k`` to ``R_{k+1}`` and an intermediate velocity;
the caller evaluates ``F_{k+1}`` at ``R_{k+1}``; ``second_half`` finishes
``V_{k+1}``.

Pins (tests/test_oracle_canonical.py): without friction both schemes are
velocity Verlet; for a harmonic well the stationary covariance of the step
(from the discrete Lyapunov equation of its linear map) gives the exact
configurational temperature when only the Langevin term acts (the
Gronbech-Jensen--Farago property the paper cites for ``gamma_TC = 0``), and
the temperature to within the time-step error when only the force noise
acts; a long run in a Morse well with Laplace-distributed force noise
samples the Boltzmann distribution.
"""

from __future__ import annotations

import numpy as np


def langevin_coefficients(gamma_l, dt, kt, mass):
    """``(c_L, sigma_L)`` of the Langevin velocity update (Eq. 32)."""
    c_l = (1.0 - 0.5 * gamma_l * dt) / (1.0 + 0.5 * gamma_l * dt)
    sigma_l = np.sqrt(kt * (1.0 - c_l * c_l) / np.asarray(mass, dtype=np.float64))
    return c_l, sigma_l


def gamma_tc_from_noise(sigma_tc, kt, dt):
    """Friction that balances force noise of standard deviation ``sigma_tc``
    (Eq. 33): ``gamma_TC = sigma_TC^2 dt / (2 kT)`` (force per velocity)."""
    return sigma_tc * sigma_tc * dt / (2.0 * kt)


def first_half(r, v, f, eta, mass, dt, kt, gamma_tc, gamma_l, scheme=0):
    """``(R_{k+1}, W)`` from ``R_k, V_k, F_k, eta_k``; ``W`` is ``V_{k+3/4}``
    (scheme 0) or ``V_{k+4/5}`` (scheme 1)."""
    r = np.asarray(r, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64)
    c_l, sigma_l = langevin_coefficients(gamma_l, dt, kt, m)
    if scheme == 0:
        v1 = v + dt / (2.0 * m) * (f - gamma_tc * v)          # V_{k+1/4}
        r1 = r + 0.5 * dt * v1                                 # R_{k+1/2}
        w = c_l * v1 + sigma_l * eta                           # V_{k+3/4}
    else:
        c_tc = (1.0 - gamma_tc * dt / (2.0 * m)) / (1.0 + gamma_tc * dt / (2.0 * m))
        v1 = v + dt / (2.0 * m) * f                            # V_{k+1/5}
        r1 = r + 0.5 * dt * v1                                 # R_{k+1/2}
        v2 = np.sqrt(c_tc) * v1                                # V_{k+2/5}
        v3 = c_l * v2 + sigma_l * eta                          # V_{k+3/5}
        w = np.sqrt(c_tc) * v3                                 # V_{k+4/5}
    return r1 + 0.5 * dt * w, w                                # R_{k+1}


def second_half(w, f_new, mass, dt, gamma_tc, scheme=0):
    """``V_{k+1}`` from the intermediate velocity and ``F_{k+1}``.  Scheme 0
    solves ``V_{k+1} = W + dt/(2M) (F_{k+1} - gamma_TC V_{k+1})``."""
    w = np.asarray(w, dtype=np.float64)
    m = np.asarray(mass, dtype=np.float64)
    kick = w + dt / (2.0 * m) * np.asarray(f_new, dtype=np.float64)
    if scheme == 0:
        return kick / (1.0 + gamma_tc * dt / (2.0 * m))
    return kick


def integrate(r, v, force, mass, dt, kt, gamma_tc, gamma_l, steps, eta, xi, sigma_tc,
              scheme=0):
    """``steps`` full steps.  ``force(r)`` is the exact force; the noisy force
    is ``force(r) + sigma_tc xi[k]`` at the k-th evaluation (``xi`` has
    ``steps + 1`` rows, row 0 for the initial force); ``eta`` has ``steps``
    rows.  Returns ``(R, V)`` after the last step."""
    f = force(r) + sigma_tc * xi[0]
    for k in range(steps):
        r, w = first_half(r, v, f, eta[k], mass, dt, kt, gamma_tc, gamma_l, scheme)
        f = force(r) + sigma_tc * xi[k + 1]
        v = second_half(w, f, mass, dt, gamma_tc, scheme)
    return r, v
