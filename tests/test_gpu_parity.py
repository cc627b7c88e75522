"""GPU (HIP, gfx950) against the CPU oracle, element by element, through the
C ABI.  Tolerance (FP64): relative L2 over all components and points
<= 1e-10, and the largest pointwise difference relative to the largest
|psi| <= 1e-10; observables relative <= 1e-10 (absolute 1e-12 below 1e-2)."""
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


def close(a, b, tol=1e-10):
    """relative L2 and relative max-abs difference both within tol"""
    return rel(a, b) < tol and maxrel(a, b) < tol


def ocfg(dim, nx, ny, dx, dy, imag, **p):
    return oracle.Cfg(dim=dim, nx=nx, ny=ny, dx=dx, dy=dy, imag=imag, **p)


def gpu_run(psi0, dx, dy, imag, nsteps, dtype=torch.complex128, **p):
    t = torch.from_numpy(np.ascontiguousarray(psi0)).to(DEV).to(dtype)
    g = api.Grid(t, dx, dy)
    g.set_params(**p)
    (g.step_imag if imag else g.step_real)(nsteps)
    torch.cuda.synchronize()
    out = t.cpu().to(torch.complex128).numpy()
    obs = g.observables()
    g.close()
    return out, obs


def start_state(dim, nx, ny, dx, dy, seed=0):
    base = W.gaussian(dim, nx, ny, dx, dy, phases=(0.3, 1.1, 2.0), width=1.5)
    noise = W.random_state(base.shape, seed, 0.05)
    return base * (1 + noise)


SHAPES_2D = [(96, 80), (37, 29), (130, 67), (64, 64), (1, 7), (5, 1), (200, 3), (513, 33),
             (40, 512), (33, 700), (17, 1023),  # rows 512-1023: the XCD row grouping, full blocks and tails
             (256, 20), (512, 9), (1024, 5), (2048, 3), (1500, 4), (3, 2048), (5, 1500),
             (1, 1), (2, 2)]


@pytest.mark.parametrize("nx,ny", SHAPES_2D)
@pytest.mark.parametrize("imag", [False, True])
@pytest.mark.parametrize("so", [api.SO_NONE, api.SO_PX_SX, api.SO_ERD])
def test_2d_steps_match_oracle(nx, ny, imag, so):
    """The 2D x-derivative SO terms: gamma p_x S_x (the two coefficient
    values of the x-pass equal) and the equal mixture's -gamma p_x S_y
    (opposite values)."""
    dx, dy = 0.25, 0.3
    p = dict(c0=3.0, c2=-0.7, gamma=0.6 if so else 0.0, omega=0.25, dt=2e-3, so=so)
    psi0 = start_state(2, nx, ny, dx, dy)
    got, _ = gpu_run(psi0, dx, dy, imag, 12, **p)
    ref = oracle.step(ocfg(2, nx, ny, dx, dy, imag, **p), psi0, 12)
    assert close(got, ref), (rel(got, ref), maxrel(got, ref))


@pytest.mark.parametrize("nx", [512, 33, 1000, 2048, 1, 64, 65])
@pytest.mark.parametrize("imag", [False, True])
@pytest.mark.parametrize("so", [api.SO_NONE, api.SO_PX_SX, api.SO_PX_SY, api.SO_PX_SZ])
def test_1d_steps_match_oracle(nx, imag, so):
    dx = 0.05 if nx >= 512 else 0.3
    p = dict(c0=5.0, c2=0.8, gamma=0.5 if so else 0.0, omega=0.0 if so == api.SO_PX_SZ else 0.15,
             dt=1e-3, so=so)
    psi0 = start_state(1, nx, 1, dx, dx)
    got, _ = gpu_run(psi0, dx, dx, imag, 25, **p)
    ref = oracle.step(ocfg(1, nx, 1, dx, dx, imag, **p), psi0, 25)
    assert close(got, ref), (rel(got, ref), maxrel(got, ref))


@pytest.mark.parametrize("so", [api.SO_RASHBA, api.SO_DRESSELHAUS, api.SO_ERD])
@pytest.mark.parametrize("imag", [False, True])
def test_2d_y_derivative_so_forms(so, imag):
    nx, ny, dx = 72, 61, 0.3
    p = dict(c0=4.0, c2=0.5, gamma=0.5, omega=0.0, dt=2e-3, so=so)
    psi0 = start_state(2, nx, ny, dx, dx, seed=3)
    got, _ = gpu_run(psi0, dx, dx, imag, 10, **p)
    ref = oracle.step(ocfg(2, nx, ny, dx, dx, imag, **p), psi0, 10)
    assert close(got, ref), (rel(got, ref), maxrel(got, ref))


@pytest.mark.parametrize("nx,ny", [(64, 16), (128, 48), (65, 17), (63, 15), (127, 33), (1, 40), (40, 1),
                                   (200, 7)])
@pytest.mark.parametrize("imag", [False, True])
def test_y_derivative_so_tile_edges(nx, ny, imag):
    """Rashba on grids that fill the pointwise + SO pass's 64 x 16 tiles
    exactly, leave ragged tails in x, in y or in both, or hold a single row or
    column (halo columns and rows at the grid's ghosts)."""
    dx = 0.25
    p = dict(c0=3.0, c2=-0.4, gamma=0.7, omega=0.2, dt=2e-3, so=api.SO_RASHBA)
    psi0 = start_state(2, nx, ny, dx, dx, seed=nx + 7 * ny) + W.random_state((3, ny, nx), nx * ny, 1e-3)
    got, _ = gpu_run(psi0, dx, dx, imag, 4, **p)
    ref = oracle.step(ocfg(2, nx, ny, dx, dx, imag, **p), psi0, 4)
    assert close(got, ref), (rel(got, ref), maxrel(got, ref))


@pytest.mark.parametrize("dim", [1, 2])
def test_fixed_magnetisation_renorm(dim):
    nx, ny, dx = (200, 1, 0.1) if dim == 1 else (64, 48, 0.3)
    p = dict(c0=10.0, c2=0.5, dt=2e-3, so=api.SO_NONE, renorm=api.RENORM_FIXED_M, mag0=0.3)
    psi0 = start_state(dim, nx, ny, dx, dx, seed=4)
    got, obs = gpu_run(psi0, dx, dx, True, 40, **p)
    ref = oracle.step(ocfg(dim, nx, ny, dx, dx, True, **p), psi0, 40)
    assert close(got, ref), (rel(got, ref), maxrel(got, ref))
    assert abs(obs["N"] - 1) < 1e-13 and abs(obs["M"] - 0.3) < 1e-13


OBS_KEYS = ("N+1", "N0", "N-1", "N", "M", "E", "E_kin", "E_trap", "E_c0", "E_c2", "E_rabi", "E_so",
            "rms+1", "rms0", "rms-1", "rms")


@pytest.mark.parametrize("dim,so", [(1, api.SO_PX_SX), (1, api.SO_PX_SY), (1, api.SO_PX_SZ),
                                    (2, api.SO_PX_SX), (2, api.SO_RASHBA), (2, api.SO_ERD)])
def test_observables_match_oracle(dim, so):
    nx, ny, dx = (300, 1, 0.1) if dim == 1 else (90, 70, 0.25)
    p = dict(c0=3.0, c2=-0.4, gamma=0.7, omega=0.3, dt=1e-3, so=so)
    psi0 = start_state(dim, nx, ny, dx, dx, seed=5)
    _, obs = gpu_run(psi0, dx, dx, False, 0, **p)
    ref = oracle.observables(ocfg(dim, nx, ny, dx, dx, False, **p), psi0)
    for k in OBS_KEYS:
        if abs(ref[k]) < 1e-2:
            assert abs(obs[k] - ref[k]) < 1e-12, k
        else:
            assert abs(obs[k] - ref[k]) < TOL * abs(ref[k]), k


@pytest.mark.parametrize("dim,nx,ny", [(1, 2048, 1), (1, 257, 1), (2, 256, 5), (2, 257, 3), (2, 1, 40),
                                       (2, 600, 500), (2, 1024, 300)])
def test_observables_row_segments(dim, nx, ny):
    """The observables pass walks 256-point row segments, a workgroup per
    segment in turn: widths that fill segments exactly or leave a ragged
    one, one-point rows, and more segments than workgroups (600 x 500: 1500;
    1024 x 300: 1200)."""
    dx = 0.05 if nx >= 1024 else 0.1
    so = api.SO_PX_SX
    p = dict(c0=3.0, c2=-0.4, gamma=0.7, omega=0.3, dt=1e-3, so=so)
    psi0 = start_state(dim, nx, ny, dx, dx, seed=6) + W.random_state((3, ny, nx) if dim == 2 else (3, nx), nx * ny, 1e-3)
    _, obs = gpu_run(psi0, dx, dx, False, 0, **p)
    ref = oracle.observables(ocfg(dim, nx, ny, dx, dx, False, **p), psi0)
    for k in OBS_KEYS:
        if abs(ref[k]) < 1e-2:
            assert abs(obs[k] - ref[k]) < 1e-12, k
        else:
            assert abs(obs[k] - ref[k]) < TOL * abs(ref[k]), k


# ------------------------------------------------ the measured workloads
def test_1d_workload_full_length():
    """1D, nx = 512, dt = 5e-4, 20000 imaginary-time steps (the whole run)."""
    w = W.W1D
    p = dict(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so, renorm=w.renorm)
    psi0 = W.initial_1d(w)
    got, obs = gpu_run(psi0, w.dx, w.dx, True, w.steps, **p)
    cfg = ocfg(1, w.nx, 1, w.dx, w.dx, True, **p)
    ref = oracle.step(cfg, psi0, w.steps)
    assert close(got, ref), (rel(got, ref), maxrel(got, ref))
    oref = oracle.observables(cfg, ref)
    assert abs(obs["E"] - oref["E"]) < TOL * abs(oref["E"])


def test_2d_imag_workload_grid():
    """256^2 workload (SO + Rabi, dt = 5e-3), first 300 steps."""
    w = W.W2D_IMAG
    p = dict(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so)
    psi0 = W.initial_2d_imag(w)
    got, obs = gpu_run(psi0, w.dx, w.dy, True, 300, **p)
    cfg = ocfg(2, w.nx, w.ny, w.dx, w.dy, True, **p)
    ref = oracle.step(cfg, psi0, 300)
    assert close(got, ref), (rel(got, ref), maxrel(got, ref))
    oref = oracle.observables(cfg, ref)
    for k in ("E", "N", "rms"):
        assert abs(obs[k] - oref[k]) < TOL * abs(oref[k]), k


def test_2d_real_workload_grid():
    """1024^2 real-time quench from the interpolated ground state, 3 steps on
    the full grid (the launch configuration the benchmark times)."""
    w = W.W2D_REAL
    p = dict(c0=w.c0, c2=w.c2, gamma=w.gamma, omega=w.omega, dt=w.dt, so=w.so)
    psi0 = W.initial_2d_real(w)
    got, obs = gpu_run(psi0, w.dx, w.dy, False, 3, **p)
    cfg = ocfg(2, w.nx, w.ny, w.dx, w.dy, False, **p)
    ref = oracle.step(cfg, psi0, 3)
    assert close(got, ref), (rel(got, ref), maxrel(got, ref))
    oref = oracle.observables(cfg, ref)
    for k in ("E", "N", "M", "rms"):
        if abs(oref[k]) < 1e-2:
            assert abs(obs[k] - oref[k]) < 1e-12, k
        else:
            assert abs(obs[k] - oref[k]) < TOL * abs(oref[k]), k


@pytest.mark.parametrize("nx,ny", [(128, 128), (1024, 8), (2048, 4), (700, 9), (6, 1024)])
def test_complex64_error_against_fp64_oracle(nx, ny):
    """complex64 storage and arithmetic (coefficients from FP64, FP64 norms):
    the stated error after 200 steps is below 1e-5 relative L2."""
    dx = 0.1
    p = dict(c0=2.0, c2=-0.1, gamma=0.5, omega=0.1, dt=2.5e-3, so=api.SO_PX_SX)
    psi0 = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0))
    for imag in (True, False):
        got, obs = gpu_run(psi0, dx, dx, imag, 200, dtype=torch.complex64, **p)
        ref = oracle.step(ocfg(2, nx, ny, dx, dx, imag, **p), psi0, 200)
        err = rel(got, ref)
        assert err < 1e-5, err
        oref = oracle.observables(ocfg(2, nx, ny, dx, dx, imag, **p), ref)
        assert abs(obs["E"] - oref["E"]) < 1e-5 * abs(oref["E"])


# ------------------------------------------------------------ interfaces
def test_step_real_seq_matches_in_place_steps():
    nx, ny, dx = 80, 70, 0.25
    p = dict(c0=2.0, c2=0.3, gamma=0.4, omega=0.2, dt=2e-3, so=api.SO_PX_SX)
    psi0 = start_state(2, nx, ny, dx, dx, seed=6)
    src = torch.from_numpy(psi0).to(DEV)
    dst = torch.empty((5, 3, ny, nx), dtype=torch.complex128, device=DEV)
    g = api.Grid(src.clone(), dx, dx)
    g.set_params(**p)
    g.step_real_seq(src, dst, 5)
    torch.cuda.synchronize()
    assert g.step_index == 5
    for k in range(5):
        ref = oracle.step(ocfg(2, nx, ny, dx, dx, False, **p), psi0, k + 1)
        assert close(dst[k].cpu().numpy(), ref)
    np.testing.assert_array_equal(src.cpu().numpy(), psi0)


def test_omega_schedule_follows_step_index():
    nx, ny, dx = 48, 40, 0.3
    p = dict(c0=2.0, c2=-0.2, gamma=0.3, omega=0.0, dt=2e-3, so=api.SO_PX_SX)
    sched = [0.05, 0.3, 0.12]
    psi0 = start_state(2, nx, ny, dx, dx, seed=7)
    t = torch.from_numpy(psi0).to(DEV)
    g = api.Grid(t, dx, dx)
    g.set_params(**p)
    g.set_omega_schedule(sched, 4)
    g.step_real(14)
    torch.cuda.synchronize()
    ref = psi0
    for n in range(14):
        ref = oracle.step(ocfg(2, nx, ny, dx, dx, False, **{**p, "omega": sched[min(n // 4, 2)]}), ref, 1)
    assert close(t.cpu().numpy(), ref)


def test_runs_are_bitwise_reproducible():
    nx, ny, dx = 100, 90, 0.2
    p = dict(c0=2.0, c2=-0.2, gamma=0.3, omega=0.1, dt=2e-3, so=api.SO_PX_SX)
    psi0 = start_state(2, nx, ny, dx, dx, seed=8)
    a, oa = gpu_run(psi0, dx, dx, True, 20, **p)
    b, ob = gpu_run(psi0, dx, dx, True, 20, **p)
    np.testing.assert_array_equal(a, b)
    assert oa == ob


def test_error_paths():
    t = torch.zeros((3, 8, 8), dtype=torch.complex128, device=DEV)
    g = api.Grid(t, 0.1, 0.1)
    with pytest.raises(api.SSGPError) as e:
        g.step_real(1)
    assert e.value.code == -4
    for bad in (dict(dt=0.0), dict(dt=-1.0), dict(dt=1e-3, so=9), dict(dt=1e-3, renorm=5),
                dict(dt=1e-3, mag0=1.5), dict(dt=float("nan")), dict(dt=1e-3, so=api.SO_PX_SZ)):
        with pytest.raises(api.SSGPError) as e:
            g.set_params(**bad)
        assert e.value.code == -1
    g.set_params(dt=1e-3)
    t[1, 3, 4] = float("nan")
    with pytest.raises(api.SSGPError) as e:
        g.observables()
    assert e.value.code == -5
    g.close()
    t1 = torch.zeros((3, 16), dtype=torch.complex128, device=DEV)
    g1 = api.Grid(t1, 0.1)
    with pytest.raises(api.SSGPError):
        g1.set_params(dt=1e-3, so=api.SO_RASHBA)
    g1.close()
