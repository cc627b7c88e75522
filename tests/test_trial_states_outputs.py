"""Host-side trial states (Sec. 3: vortex imprints (x +- iy)^L, stripes, the
OPT_ST rule) and output quantities (densities, radial density, phases,
winding numbers), checked against closed forms on the CPU."""
import numpy as np
import pytest

from paper_2009_13507_amd import outputs as O
from paper_2009_13507_amd import workloads as W


def norm2d(psi, dx, dy):
    return float(np.sum(np.abs(psi) ** 2) * dx * dy)


@pytest.mark.parametrize("lz", [(-1, 0, 1), (1, 0, -1), (0, 1, 2), (0, -1, -2), (3, -2, 0)])
def test_vortex_imprint_winding_and_norm(lz):
    n, h = 96, 0.125
    psi = W.vortex(n, n, h, h, lz, width=1.5)
    assert abs(norm2d(psi, h, h) - 1.0) < 1e-12
    for j in range(3):
        for half in (4, 11, 20):
            assert O.winding(psi[j], half) == lz[j], (j, half)


def test_vortex_profile_is_r_to_the_L_times_gaussian():
    n, h, w = 64, 0.1, 1.2
    psi = W.vortex(n, n, h, h, (0, 1, 2), weights=(1 / 3, 1 / 3, 1 / 3), width=w)
    x = W.coords(n, h)
    X, Y = np.meshgrid(x, x)
    r2 = X ** 2 + Y ** 2
    g = np.exp(-r2 / (2 * w ** 2))
    # ratios between components remove the common normalisation
    np.testing.assert_allclose(psi[1], psi[0] * (X + 1j * Y), rtol=0, atol=1e-14)
    np.testing.assert_allclose(psi[2], psi[0] * (X + 1j * Y) ** 2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(np.abs(psi[0]) / np.abs(psi[0]).max(), g, atol=1e-14)
    # (x - iy)^L for an anti-vortex is the complex conjugate of the vortex
    anti = W.vortex(n, n, h, h, (0, -1, -2), weights=(1 / 3, 1 / 3, 1 / 3), width=w)
    np.testing.assert_allclose(anti, np.conj(psi), atol=1e-15)


def test_stripes_are_the_polar_stripe_spinor():
    n, h, gam = 80, 0.1, 1.3
    psi = W.stripes(n, n, h, h, gam, width=2.0)
    assert abs(norm2d(psi, h, h) - 1.0) < 1e-12
    x = W.coords(n, h)
    s, c = np.sin(gam * x)[None, :], np.cos(gam * x)[None, :]
    # psi_+1 = psi_-1 = i sin / sqrt 2 * G and psi_0 = -cos * G for one G
    np.testing.assert_array_equal(psi[0], psi[2])
    np.testing.assert_allclose(psi[0] * c, -1j * s / np.sqrt(2.0) * psi[1], atol=1e-15)
    # the stripe spinor has unit length at every x: the local total density is G^2
    rho = O.density(psi)[3]
    g2 = np.abs(psi[1]) ** 2 + 2 * np.abs(psi[0]) ** 2
    np.testing.assert_allclose(rho, g2, rtol=1e-14)
    G2 = np.exp(-(x[None, :] ** 2 + x[:, None] ** 2) / 4.0)
    np.testing.assert_allclose(rho / rho.max(), G2 / G2.max(), rtol=1e-12)


RULE = [  # (so, gamma, c2, expected)
    (W.SO_RASHBA, 0.5, 15.0, ("vortex", (-1, 0, 1))),
    (W.SO_DRESSELHAUS, 0.5, 15.0, ("vortex", (1, 0, -1))),
    (W.SO_RASHBA, 0.5, -6.15, ("vortex", (0, 1, 2))),
    (W.SO_DRESSELHAUS, 0.5, -6.15, ("vortex", (0, -1, -2))),
    (W.SO_RASHBA, 1.0, 15.0, ("stripes", None)),
    (W.SO_DRESSELHAUS, 1.0, 15.0, ("stripes", None)),
    (W.SO_RASHBA, 1.0, -6.15, ("vortex", (0, 1, 2))),
    (W.SO_ERD, 0.5, 15.0, ("stripes", None)),
    (W.SO_ERD, 0.5, -6.15, ("gaussian", None)),
    (W.SO_PX_SX, 0.5, 15.0, ("gaussian", None)),
    (W.SO_RASHBA, 0.0, 15.0, ("gaussian", None)),
    (W.SO_NONE, 0.0, -1.0, ("gaussian", None)),
]


@pytest.mark.parametrize("so,gamma,c2,expected", RULE)
def test_opt_st_rule(so, gamma, c2, expected):
    assert W.so_trial_kind(so, gamma, c2) == expected
    psi = W.so_trial(32, 32, 0.2, 0.2, so, gamma, c2, width=1.0)
    assert psi.shape == (3, 32, 32)
    assert abs(norm2d(psi, 0.2, 0.2) - 1.0) < 1e-12


def test_opt_st_threshold_is_a_parameter():
    assert W.so_trial_kind(W.SO_RASHBA, 0.5, 15.0, opt_st=0.4) == ("stripes", None)
    assert W.so_trial_kind(W.SO_RASHBA, 0.8, 15.0, opt_st=1.0) == ("vortex", (-1, 0, 1))


def test_radial_density_of_a_gaussian():
    """A normalised Gaussian of width w has rho(r) = exp(-r^2/w^2) / (pi w^2).
    Each annulus value is the mean of that function over the grid points in
    the annulus (brute force here), and lies within the function's change
    across the annulus of its value at mid-radius."""
    n, h, w = 256, 0.05, 1.0
    psi = W.gaussian(2, n, n, h, h, weights=(0.25, 0.5, 0.25), width=w)
    r, rho = O.radial_density(psi, h, h)
    f = lambda rr: np.exp(-rr ** 2 / w ** 2) / (np.pi * w ** 2)
    x = W.coords(n, h)
    rp = np.hypot(x[None, :], x[:, None]).ravel()
    for k in (0, 1, 5, 17, 40, len(r) - 1):
        sel = (rp >= k * h) & (rp < (k + 1) * h)
        assert abs(rho[3][k] - f(rp[sel]).mean()) < 1e-12 * f(0.0), k
        assert f((k + 1) * h) - 1e-15 <= rho[3][k] <= f(k * h) + 1e-15, k
    np.testing.assert_allclose(rho[3], f(r), rtol=0, atol=1e-2 * f(0.0))
    np.testing.assert_allclose(rho[0] + rho[1] + rho[2], rho[3], rtol=1e-13)
    np.testing.assert_allclose(rho[1], 2 * rho[0], rtol=1e-12)
    # annulus means times the point counts give back the norm exactly (the
    # Gaussian has decayed far below 1e-13 at the largest inscribed circle);
    # the ring integral 2 pi r rho dr at the mid-radii approximates it
    cnt = np.bincount(np.floor(rp / h).astype(np.int64), minlength=len(r))[:len(r)]
    assert abs(np.sum(cnt * h * h * rho[3]) - 1.0) < 1e-13
    assert abs(np.sum(2 * np.pi * r * rho[3] * h) - 1.0) < 1e-2


def test_density_and_phase_of_a_random_state():
    psi = W.random_state((3, 7, 9), 3)
    rho = O.density(psi)
    assert rho.shape == (4, 7, 9)
    np.testing.assert_allclose(rho[:3], psi.real ** 2 + psi.imag ** 2, rtol=1e-14)
    np.testing.assert_allclose(rho[3], rho[:3].sum(0), rtol=1e-14)
    ph = O.phase(psi)
    np.testing.assert_allclose(np.abs(psi) * np.exp(1j * ph), psi, atol=1e-14)


def test_writers_layout(tmp_path):
    n, h = 16, 0.25
    psi = W.vortex(n, n, h, h, (-1, 0, 1), width=1.0)
    O.write_density(str(tmp_path / "den.txt"), psi, h, h)
    O.write_phase(str(tmp_path / "phase.txt"), psi, h, h)
    O.write_radial_density(str(tmp_path / "rad.txt"), psi, h, h)
    den = np.loadtxt(tmp_path / "den.txt")
    assert den.shape == (n * n, 6)
    np.testing.assert_allclose(den[:n, 0], W.coords(n, h))       # x fastest
    np.testing.assert_allclose(den[:n, 1], W.coords(n, h)[0])
    np.testing.assert_allclose(den[:, 5], den[:, 2] + den[:, 3] + den[:, 4], rtol=1e-9)
    ph = np.loadtxt(tmp_path / "phase.txt")
    assert ph.shape == (n * n, 5)
    rad = np.loadtxt(tmp_path / "rad.txt")
    assert rad.shape[1] == 5
    psi1 = W.gaussian(1, 40, 1, 0.1, 0.1)
    O.write_density(str(tmp_path / "den1.txt"), psi1, 0.1)
    assert np.loadtxt(tmp_path / "den1.txt").shape == (40, 5)


def test_winding_rejects_bad_loops():
    psi = W.vortex(16, 16, 0.25, 0.25, (1, 0, 0))
    with pytest.raises(ValueError):
        O.winding(psi[0], 9)
    with pytest.raises(ValueError):
        O.winding(np.zeros((16, 16), complex), 3)
