"""Pins of the oracle's real-time steps with RENORM after every step (App. A
rescales after each time step of the propagation; opt-in here):
- the norm is 1 after every step (Eq. (DJ2)), and the magnetisation m too
  under Eq. (DJ);
- without nonlinearity, SO and Rabi coupling the real-time step is unitary,
  so the rescaling is the identity to rounding;
- a converged imaginary-time ground state is stationary in real time: its
  energy stays put far better with the rescaling than without when the
  explicit SO sub-step is on (the sample output of Sec. 3 holds E to five
  digits over 90,000 steps)."""
import numpy as np
import pytest

import oracle
from paper_2009_13507_amd import workloads as W


def norm2d(psi, dx):
    return float(np.sum(np.abs(psi) ** 2) * dx * dx)


def test_norm_is_one_after_every_step():
    nx, ny, dx = 40, 32, 0.25
    c = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, c0=3.0, c2=-0.4, gamma=0.9, omega=0.2,
                   dt=0.01, so=oracle.SO_PX_SX)
    psi = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5)
    for _ in range(5):
        psi = oracle.step_real_renorm(c, psi, 1)
        assert abs(norm2d(psi, dx) - 1.0) < 1e-14


def test_fixed_magnetisation_rule_in_real_time():
    nx, dx = 64, 0.2
    c = oracle.Cfg(dim=1, nx=nx, ny=1, dx=dx, dy=dx, imag=False, c0=10.0, c2=2.0, dt=0.01,
                   renorm=oracle.RENORM_FIXED_M, mag0=0.3)
    psi = W.gaussian(1, nx, 1, dx, dx, weights=(0.6, 0.1, 0.3), width=2.0)
    out = oracle.step_real_renorm(c, psi, 7)
    N = np.sum(np.abs(out) ** 2, axis=1) * dx
    assert abs(N.sum() - 1.0) < 1e-13
    assert abs((N[0] - N[2]) - 0.3) < 1e-13


def test_linear_unitary_step_is_left_alone():
    nx, ny, dx = 36, 28, 0.3
    # (the norm-only rule: the AUTO rule would pick Eq. (DJ) here and also fix M)
    c = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, dt=0.02, renorm=oracle.RENORM_NORM)
    psi = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5) * (1 + W.random_state((3, ny, nx), 3, 0.1))
    psi = psi / np.sqrt(norm2d(psi, dx))
    np.testing.assert_allclose(oracle.step_real_renorm(c, psi, 6), oracle.step(c, psi, 6), rtol=0, atol=1e-13)


def test_ground_state_stays_stationary_with_the_rescaling():
    nx, dx = 48, 0.3
    prm = dict(c0=20.0, c2=1.5, gamma=0.5, omega=0.0, so=oracle.SO_RASHBA)
    ci = oracle.Cfg(dim=2, nx=nx, ny=nx, dx=dx, dy=dx, imag=True, dt=2e-3, **prm)
    g = oracle.step(ci, W.vortex(nx, nx, dx, dx, (-1, 0, 1), width=1.5), 3000)
    cr = oracle.Cfg(dim=2, nx=nx, ny=nx, dx=dx, dy=dx, imag=False, dt=2e-3, **prm)
    e0 = oracle.observables(cr, g)["E"]
    with_r = oracle.observables(cr, oracle.step_real_renorm(cr, g, 400))["E"]
    without = oracle.observables(cr, oracle.step(cr, g, 400))["E"]
    assert abs(with_r - e0) < 0.1 * abs(without - e0)
    assert abs(with_r - e0) < 1e-4 * abs(e0)


def test_rejects_imaginary_time():
    c = oracle.Cfg(dim=1, nx=16, ny=1, dx=0.2, dy=0.2, imag=True, dt=0.01)
    with pytest.raises(ValueError):
        oracle.step_real_renorm(c, W.gaussian(1, 16, 1, 0.2, 0.2), 1)
