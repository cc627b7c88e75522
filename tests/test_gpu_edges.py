"""GPU against the CPU oracle at the method's edge cases, through the C ABI.

Each case is compared element by element: relative L2 over all components
and points <= 1e-10 (FP64), and beside it the largest pointwise difference
relative to the largest |psi| of the reference, so that an error confined to
a few points (a boundary, a tail) cannot hide below the L2 norm.

- Nonzero values next to the zero ghosts at the benchmarked shapes (rows and
  columns of 1024 points: the x-pass with 4 points per thread, no range
  checks, tabulated fix-ups, and the y-pass with chunks of 16 rows), for
  gamma p_x Sigma_x and the Rashba coupling, in real and imaginary time; the
  boundary bands are also compared on their own scale.
- Large dt phi and dt C on O(1) values: CALCNU's longer series and the library
  cos/sin, HERM's general series and library branch (App. A Eq. (eq11)), in
  real and imaginary time, forward and adjoint.
- The fall-back of Eq. (DJ) to Eq. (DJ2) (App. A): an empty -1 or +1
  component and |m| = 1, beside Eq. (DJ) itself close to its limit (m = 0.95),
  in 2D, 1D and the batch.  (The radicands 1 +- m - d_0^2 N_0 of Eq. (DJ) are
  never negative in exact arithmetic: d_0^2 N_0 <= 1 - |m|.)
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2009_13507_amd import api  # noqa: E402
from paper_2009_13507_amd import workloads as W  # noqa: E402

TOL = 1e-10
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check(got, ref, tol=TOL):
    e2, einf = rel(got, ref), maxrel(got, ref)
    assert e2 < tol and einf < tol, (e2, einf)


def bands(a, w=2):
    """The points within w of the box edges (2D state (3, ny, nx))."""
    return np.concatenate([a[:, :w, :].ravel(), a[:, -w:, :].ravel(), a[:, w:-w, :w].ravel(),
                           a[:, w:-w, -w:].ravel()])


def gpu_run(psi0, dx, dy, imag, nsteps, **p):
    t = torch.from_numpy(np.ascontiguousarray(psi0)).to(DEV)
    g = api.Grid(t, dx, dy)
    g.set_params(**p)
    (g.step_imag if imag else g.step_real)(nsteps)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    obs = g.observables()
    g.close()
    return out, obs


def noisy(dim, nx, ny, dx, dy, seed, amp=1e-3, width=1.5):
    """A Gaussian plus additive complex noise of size amp at every point, so
    that the edge rows and columns hold values of order amp."""
    base = W.gaussian(dim, nx, ny, dx, dy, phases=(0.3, 1.1, 2.0), width=width)
    return base + W.random_state(base.shape, seed, amp)


# ------------------------------------------------ nonzero box edges -------
@pytest.mark.parametrize("so", [api.SO_PX_SX, api.SO_RASHBA])
@pytest.mark.parametrize("imag", [False, True])
def test_nonzero_edges_at_1024(so, imag):
    """1024^2, dx = 0.05, dt = 1e-4 (the real-time workload's grid and step),
    three steps from a state with O(1e-3) values on every edge."""
    w = W.W2D_REAL
    n, dx = w.nx, w.dx
    p = dict(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=so)
    print(f"edges 1024^2 so={so} imag={imag}", flush=True)
    psi0 = noisy(2, n, n, dx, dx, seed=11 + so + 2 * imag)
    got, _ = gpu_run(psi0, dx, dx, imag, 3, **p)
    ref = oracle.step(oracle.Cfg(dim=2, nx=n, ny=n, dx=dx, dy=dx, imag=imag, **p), psi0, 3)
    check(got, ref)
    gb, rb = bands(got), bands(ref)
    assert np.abs(rb).max() > 1e-4  # the edges are populated
    assert maxrel(gb, rb) < TOL, maxrel(gb, rb)


@pytest.mark.parametrize("nx,ny", [(1024, 40), (40, 1024), (1000, 24), (24, 1000)])
@pytest.mark.parametrize("imag", [False, True])
def test_nonzero_edges_rows_and_columns(nx, ny, imag):
    """Rows (x-pass) and columns (y-pass) of 1024 and 1000 points with edge
    values, p_x Sigma_x with Rabi coupling, 6 steps."""
    dx = 0.05
    p = dict(c0=2.0, c2=0.1, gamma=0.8, omega=0.2, dt=1e-4, so=api.SO_PX_SX)
    psi0 = noisy(2, nx, ny, dx, dx, seed=nx + ny + imag, amp=3e-3, width=0.6)
    got, _ = gpu_run(psi0, dx, dx, imag, 6, **p)
    ref = oracle.step(oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=imag, **p), psi0, 6)
    check(got, ref)
    assert maxrel(bands(got), bands(ref)) < TOL


# ------------------------------------- large dt phi and dt C (series tiers)
# dt and Omega chosen so that, on O(1) values, the CALCNU angles dt phi reach
# the 6-term band (|dt phi| <= 0.16), the 10-term band (<= pi/4) and beyond
# (library), and HERM's u = dt C / 2 the general series (u <= pi/4) and the
# library branch.
TIER_CASES = [
    (0.012, 4.0, 20.0),    # CALCNU 6-term, HERM general series
    (0.05, 4.0, 20.0),     # CALCNU 10-term, HERM general series
    (0.05, 4.0, 60.0),     # HERM library branch
    (0.2, 4.0, 20.0),      # CALCNU and HERM library
    (0.03, 200.0, 60.0),   # large c0: CALCNU library on the dense region
]


def tier_state(nx, ny, dx, seed):
    """O(1) values at every point (no underflowed tails)."""
    g = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=2.0)
    return g + W.random_state(g.shape, seed, 0.15)


@pytest.mark.parametrize("dt,c0,omega", TIER_CASES)
@pytest.mark.parametrize("imag", [False, True])
def test_series_tiers_forward(dt, c0, omega, imag):
    nx, ny, dx = 300, 24, 0.05
    if imag and dt * omega > 2.0:
        pytest.skip("exp(dt C) beyond 1e3: the imaginary-time case is covered at smaller dt C")
    p = dict(c0=c0, c2=-0.7, gamma=0.3, omega=omega, dt=dt, so=api.SO_PX_SX)
    psi0 = tier_state(nx, ny, dx, seed=int(100 * dt) + int(omega))
    # the angles really span the bands
    x = W.coords(nx, dx)
    y = W.coords(ny, dx)
    V = 0.5 * (x[None, :] ** 2 + y[:, None] ** 2)
    rho = (np.abs(psi0) ** 2).sum(0)
    th = dt * (V + c0 * rho)
    assert th.max() > 0.1
    got, _ = gpu_run(psi0, dx, dx, imag, 3, **p)
    ref = oracle.step(oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=imag, **p), psi0, 3)
    check(got, ref)


@pytest.mark.parametrize("dt,c0,omega", TIER_CASES)
def test_series_tiers_1d(dt, c0, omega):
    nx, dx = 500, 0.02
    p = dict(c0=c0, c2=-0.7, gamma=0.3, omega=omega, dt=dt, so=api.SO_PX_SX)
    g = W.gaussian(1, nx, 1, dx, dx, phases=(0.3, 1.1, 2.0), width=2.0)
    psi0 = g + W.random_state(g.shape, 7, 0.15)
    got, _ = gpu_run(psi0, dx, dx, False, 3, **p)
    ref = oracle.step(oracle.Cfg(dim=1, nx=nx, dx=dx, imag=False, **p), psi0, 3)
    check(got, ref)


@pytest.mark.parametrize("dt,c0,omega", TIER_CASES)
@pytest.mark.parametrize("dim", [1, 2])
def test_series_tiers_adjoint(dt, c0, omega, dim):
    """Adjoint of two real-time steps against the oracle's dual-number
    adjoint: the transposed CALCNU and HERM Jacobians at large dt phi and
    dt C (the library sincos and the closed-form derivative of sinc)."""
    nx, ny, dx = (300, 24, 0.05) if dim == 2 else (500, 1, 0.02)
    base = dict(dim=dim, nx=nx, ny=ny, dx=dx, dy=dx, c0=c0, c2=-0.7, gamma=0.3, dt=dt, imag=False,
                so=api.SO_PX_SX, omega=omega)
    g0 = W.gaussian(dim, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=2.0)
    psi0 = g0 + W.random_state(g0.shape, 3, 0.15)
    cfg = oracle.Cfg(**base)
    s1 = oracle.step(cfg, psi0, 1)
    s2 = oracle.step(cfg, s1, 1)
    dA = dx * (dx if dim == 2 else 1.0)
    lam = np.zeros_like(s2)
    lam[0] = 2 * dA * s2[0]
    lam_ref, d1 = oracle.step_adjoint(cfg, s1, lam)
    lam_ref, d0 = oracle.step_adjoint(cfg, psi0, lam_ref)
    work = torch.from_numpy(psi0.copy()).to(DEV)
    g = api.Grid(work, dx, dx if dim == 2 else None)
    g.set_params(c0=c0, c2=-0.7, gamma=0.3, omega=omega, dt=dt, so=api.SO_PX_SX)
    g.omega_grad(reset=True)
    t_states = torch.from_numpy(np.stack([psi0, s1])).to(DEV)
    t_lam = torch.from_numpy(lam).to(DEV)
    g.step_index = 2
    g.step_real_adjoint(t_states, t_lam, 2)
    dom = g.omega_grad(reset=True)[0]
    got = t_lam.cpu().numpy()
    g.close()
    check(got, lam_ref)
    assert abs(dom - (d0 + d1)) <= TOL * max(abs(d0 + d1), 1e-300), (dom, d0 + d1)


# ------------------------------------------- (DJ) -> (DJ2) fall-back -----
def dj_cases():
    """(name, params, weights, falls back): the first three make Eq. (DJ)
    unusable at every step, the last keeps it at m = 0.95."""
    fm = api.RENORM_FIXED_M
    return [
        ("empty_minus", dict(c0=10.0, c2=0.0, renorm=fm, mag0=0.3), (0.6, 0.4, 0.0), 1),
        ("empty_plus", dict(c0=10.0, c2=0.0, renorm=fm, mag0=-0.2), (0.0, 0.7, 0.3), 1),
        ("m_one", dict(c0=10.0, c2=0.5, renorm=fm, mag0=1.0), (0.5, 0.3, 0.2), 1),
        ("m_095", dict(c0=10.0, c2=0.5, renorm=fm, mag0=0.95), (0.02, 0.96, 0.02), 0),
    ]


def dj_state(dim, nx, ny, dx, wts, seed):
    psi = W.gaussian(dim, nx, ny, dx, dx, weights=wts, phases=(0.3, 1.1, 2.0), width=1.5)
    noise = W.random_state(psi.shape, seed, 0.05)
    return psi * (1 + noise)


@pytest.mark.parametrize("name,prm,wts,falls", dj_cases())
@pytest.mark.parametrize("dim", [1, 2])
def test_dj_fallback(name, prm, wts, falls, dim):
    nx, ny, dx = (200, 1, 0.1) if dim == 1 else (64, 48, 0.3)
    p = dict(dt=2e-3, so=api.SO_NONE, **prm)
    psi0 = dj_state(dim, nx, ny, dx, wts, seed=21)
    cfg = oracle.Cfg(dim=dim, nx=nx, ny=ny, dx=dx, dy=dx, imag=True, **p)
    # the case does (or does not) fall back at the first step: the oracle's report
    first = oracle.herm(cfg, oracle.calcnu(cfg, psi0))
    first = oracle.cn_x(cfg, first)
    if dim == 2:
        first = oracle.cn_y(cfg, first)
    _, fb = oracle.renorm(cfg, first)
    assert fb == falls
    got, obs = gpu_run(psi0, dx, dx, True, 30, **p)
    ref = oracle.step(cfg, psi0, 30)
    check(got, ref)
    assert abs(obs["N"] - 1.0) < 1e-13
    if not falls:
        assert abs(obs["M"] - prm["mag0"]) < 1e-13


def test_dj_fallback_in_batch():
    """The fall-back cases and (DJ) at m = 0.95 and m = 0.3 in one batch."""
    dx = 0.3
    shapes = [(48, 64), (40, 33), (64, 70), (30, 30), (36, 52)]
    cases = dj_cases() + [("regular", dict(c0=10.0, c2=0.5, renorm=api.RENORM_FIXED_M, mag0=0.3),
                           (0.5, 0.3, 0.2), 0)]
    states, prms, refs = [], [], []
    for (ny, nx), (_, prm, wts, _f) in zip(shapes, cases):
        p = dict(dt=2e-3, so=api.SO_NONE, **prm)
        s = dj_state(2, nx, ny, dx, wts, seed=nx)
        states.append(s)
        prms.append(api.params(**p))
        refs.append(oracle.step(oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=True, **p), s, 25))
    b = api.Batch.from_states(states, [dx] * len(states), prms)
    b.step_imag(25)
    b.sync()
    got = [v.cpu().numpy() for v in b.views()]
    obs = b.observables()
    b.close()
    for gi, ri, oi in zip(got, refs, obs):
        check(gi, ri)
        assert abs(oi["N"] - 1.0) < 1e-13
