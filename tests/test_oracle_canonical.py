"""Pins of the canonical-integration oracle (oracle/canonical.py, Section IV,
Eq. 31-33 and the alternative scheme of the Supporting Information) against
results that do not come from the oracle itself:

* without friction both schemes are velocity Verlet (written out here);
* harmonic well, exact stationary statistics: with a force linear in R, one
  step is a linear map of (R, V, current force noise) plus fresh noise, so
  the discrete Lyapunov equation gives the stationary covariance without
  sampling.  With only the Langevin term, kappa <R^2> = kT for every stable
  time step (the configurational exactness of this BAOAB-ordered splitting
  of Gronbech-Jensen--Farago for linear forces); with only the force noise
  balanced by Eq. 33, kappa <R^2> = kT / (1 - kappa dt^2 / (4M)), the
  velocity-Verlet harmonic factor, for any noise level.  A factor-2 slip in
  Eq. 33 gives 0.5 instead;
* force-free decay: without forces and noise one step multiplies V by the
  friction factors, which must approximate the continuous decay
  exp(-(gamma_L + gamma_TC / M) dt) to third order (they are its (1,1) Pade
  approximants, error below (g dt)^3 / 12 per factor); the stationary tests
  cannot see a wrong time scale, since c V + sqrt(kT (1 - c^2) / M) eta
  keeps the Maxwell distribution for any c;
* Morse well, Laplace-distributed force noise (the non-Gaussian case of
  Section IV), started at rest: after equilibration the sampled mean and
  variance of r and the kinetic temperature match the Boltzmann
  distribution (quadrature) within sampling error.
"""

import numpy as np
import pytest
from scipy.linalg import solve_discrete_lyapunov

from oracle import canonical as C
from workloads import AMU, KB_EV, laplace_unit, morse_energy, morse_force

M7 = 7.0 * AMU
KT500 = 500.0 * KB_EV


@pytest.mark.parametrize("scheme", [0, 1])
def test_without_friction_is_velocity_verlet(scheme):
    rng = np.random.default_rng(0)
    n = 64
    r0 = 1.0 + 0.3 * rng.standard_normal(n)
    v0 = 0.01 * rng.standard_normal(n)
    m = rng.uniform(1.0, 16.0, n) * AMU
    dt, steps = 0.5, 400
    zeros = np.zeros((steps + 1, n))
    r, v = C.integrate(r0, v0, morse_force, m, dt, KT500, 0.0, 0.0, steps, zeros, zeros, 0.0,
                       scheme)
    rr, vv = r0.copy(), v0.copy()
    f = morse_force(rr)
    for _ in range(steps):
        rr = rr + dt * vv + dt * dt / (2.0 * m) * f
        f1 = morse_force(rr)
        vv = vv + dt / (2.0 * m) * (f + f1)
        f = f1
    assert np.allclose(r, rr, rtol=0, atol=1e-11)
    assert np.allclose(v, vv, rtol=0, atol=1e-13)


def _stationary(kappa, m, dt, kt, gamma_tc, gamma_l, sigma_tc, scheme):
    """kappa <R^2> / kT and M <V^2> / kT of the stationary state."""
    def step(s, w):
        r, v, xi = s
        eta, xi1 = w
        rn, wv = C.first_half(r, v, -kappa * r + sigma_tc * xi, eta, m, dt, kt, gamma_tc,
                              gamma_l, scheme)
        vn = C.second_half(wv, -kappa * rn + sigma_tc * xi1, m, dt, gamma_tc, scheme)
        return np.array([rn, vn, xi1])
    a = np.column_stack([step(e, (0.0, 0.0)) for e in np.eye(3)])
    b = np.column_stack([step(np.zeros(3), e) for e in np.eye(2)])
    s = solve_discrete_lyapunov(a, b @ b.T)
    return kappa * s[0, 0] / kt, m * s[1, 1] / kt


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("dt", [0.5, 2.0, 10.0])
@pytest.mark.parametrize("gamma_l", [1e-3, 1e-2])
def test_langevin_term_samples_harmonic_well_exactly(scheme, dt, gamma_l):
    conf, kin = _stationary(1.0, M7, dt, KT500, 0.0, gamma_l, 0.0, scheme)
    assert conf == pytest.approx(1.0, abs=1e-10)
    assert 0.9 < kin <= 1.0 + 1e-12


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("dt", [0.5, 2.0])
@pytest.mark.parametrize("sigma_tc", [0.01, 0.1, 0.3])
def test_force_noise_balanced_by_eq33(scheme, dt, sigma_tc):
    kappa = 1.0
    gamma_tc = C.gamma_tc_from_noise(sigma_tc, KT500, dt)
    conf, kin = _stationary(kappa, M7, dt, KT500, gamma_tc, 0.0, sigma_tc, scheme)
    assert conf == pytest.approx(1.0 / (1.0 - kappa * dt * dt / (4.0 * M7)), rel=1e-9)
    assert kin == pytest.approx(1.0, abs=5e-3)
    # the same noise with twice the friction cools the well to half the temperature
    conf2, _ = _stationary(kappa, M7, dt, KT500, 2.0 * gamma_tc, 0.0, sigma_tc, scheme)
    assert conf2 == pytest.approx(0.5 * conf, rel=2e-3)


@pytest.mark.parametrize("scheme", [0, 1])
def test_both_channels_together(scheme):
    dt, sigma_tc = 0.5, 0.1
    conf, kin = _stationary(1.0, M7, dt, KT500, C.gamma_tc_from_noise(sigma_tc, KT500, dt), 1e-3,
                            sigma_tc, scheme)
    assert conf == pytest.approx(1.0, abs=2e-4) and kin == pytest.approx(1.0, abs=1e-3)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("gamma_l,gamma_tc", [(1e-3, 0.0), (2e-2, 0.0), (0.0, 5.0), (1e-2, 3.0)])
def test_force_free_decay_follows_the_friction_rates(scheme, gamma_l, gamma_tc):
    dt, m = 0.5, np.array([M7, 2.0 * AMU])
    zero = np.zeros(2)
    _, w = C.first_half(zero, np.ones(2), zero, zero, m, dt, KT500, gamma_tc, gamma_l, scheme)
    factor = C.second_half(w, zero, m, dt, gamma_tc, scheme)
    exact = np.exp(-(gamma_l + gamma_tc / m) * dt)
    bound = ((gamma_l * dt) ** 3 + (gamma_tc / m * dt) ** 3) / 12.0 + 1e-15
    assert np.all(np.abs(factor - exact) <= 1.01 * bound), (factor - exact, bound)
    assert np.all(factor < 1.0) if gamma_l + gamma_tc > 0 else True


def _boltzmann_moments(kt):
    r = np.linspace(0.2, 6.0, 200001)
    w = np.exp(-morse_energy(r) / kt)
    z = np.trapezoid(w, r)
    mean = np.trapezoid(r * w, r) / z
    return mean, np.trapezoid((r - mean) ** 2 * w, r) / z


@pytest.mark.parametrize("scheme", [0, 1])
def test_morse_well_with_laplace_noise_samples_boltzmann(scheme):
    rng = np.random.default_rng(11 + scheme)
    n, dt, sigma_tc = 4000, 0.5, 0.3
    gamma_tc = C.gamma_tc_from_noise(sigma_tc, KT500, dt)   # energy relaxes in M / gamma_TC ~ 1.4 ps
    m = np.full(n, M7)
    r = np.full(n, 1.0)
    v = np.zeros(n)
    f = morse_force(r) + sigma_tc * laplace_unit(rng, n)
    zero = np.zeros(n)
    rs, ks = [], []
    for k in range(24000):
        r, w = C.first_half(r, v, f, zero, m, dt, KT500, gamma_tc, 0.0, scheme)
        f = morse_force(r) + sigma_tc * laplace_unit(rng, n)
        v = C.second_half(w, f, m, dt, gamma_tc, scheme)
        if k >= 14000 and k % 10 == 0:
            rs.append(r.copy())
            ks.append(np.mean(m * v * v) / KT500)
    rs = np.array(rs)
    mean, var = _boltzmann_moments(KT500)
    assert abs(rs.mean() - mean) < 0.05 * np.sqrt(var)
    assert rs.var() == pytest.approx(var, rel=0.05)
    assert np.mean(ks) == pytest.approx(1.0, abs=0.03)
