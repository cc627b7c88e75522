"""The opt-in Strang scheme on the GPU against the oracle's definition of it
(P2(dt/2), the joined LUX + SO solve, LUY, P2(dt/2), RENORM in imaginary
time): relative L2 and relative max-abs <= 1e-10 in FP64 (<= 1e-5 in FP32)
over every x-pass shape (1, 2, 4 and 8 points per thread, full and ragged
rows) in real and imaginary time, runs split over calls and Omega segments
(where the closing stage of a run is its own pass), real-time RENORM, the
LDS-resident 1D kernel; exact real-time norm; graph replays bitwise equal to
one-by-one launches; second order measured on a 256^2 grid; the refusals."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2009_13507_amd import api  # noqa: E402
from paper_2009_13507_amd import workloads as W  # noqa: E402
from paper_2009_13507_amd._lib import SSGPError  # noqa: E402

DEV = "cuda:0"
PRM = dict(c0=6.0, c2=-2.5, gamma=0.7, omega=0.35, so=api.SO_PX_SX)
SHAPES = [(72, 40), (256, 20), (300, 9), (512, 9), (700, 6), (1024, 5), (1500, 3), (2048, 3), (1, 1), (3, 2)]


def start(dim, nx, ny, dx, seed):
    base = W.gaussian(dim, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0),
                      width=0.18 * min(nx, 4 * ny if dim == 2 else nx) * dx)
    return base * (1 + W.random_state(base.shape, seed, 0.05))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def check(got, want, tol=1e-10):
    assert rel(got, want) < tol and maxrel(got, want) < tol, (rel(got, want), maxrel(got, want))


def grid(psi0, dx, dtype=torch.complex128, **prm):
    t = torch.from_numpy(psi0.copy()).to(DEV, dtype)
    g = api.Grid(t, dx, dx if psi0.ndim == 3 else None)
    g.set_params(**prm)
    g.set_scheme(api.SCHEME_STRANG)
    return g, t


def run(psi0, dx, imag, calls, dtype=torch.complex128, **prm):
    g, t = grid(psi0, dx, dtype, **prm)
    for n in calls:
        (g.step_imag if imag else g.step_real)(n)
    torch.cuda.synchronize()
    out = t.cpu().numpy().astype(np.complex128)
    g.close()
    return out


@pytest.mark.parametrize("imag", [False, True], ids=["real", "imag"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_strang_matches_oracle(nx, ny, imag):
    dx, dt = 0.1, 2e-3
    psi0 = start(2, nx, ny, dx, nx + ny)
    print(f"strang nx={nx} ny={ny} imag={imag}", flush=True)
    got = run(psi0, dx, imag, (3, 1, 4), dt=dt, **PRM)
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=imag, dt=dt, **PRM)
    check(got, oracle.step_strang(cfg, psi0, 8))


@pytest.mark.parametrize("imag", [False, True], ids=["real", "imag"])
@pytest.mark.parametrize("nx", [512, 640, 33, 2048])
@pytest.mark.parametrize("so", [api.SO_PX_SX, api.SO_PX_SY, api.SO_PX_SZ, api.SO_NONE])
def test_strang_1d_matches_oracle(nx, imag, so):
    dx, dt = 0.05, 1e-3
    prm = dict(PRM, so=so, gamma=0.5 if so else 0.0, omega=0.0 if so == api.SO_PX_SZ else 0.2)
    psi0 = start(1, nx, 1, dx, nx)
    got = run(psi0, dx, imag, (5, 2), dt=dt, **prm)
    cfg = oracle.Cfg(dim=1, nx=nx, dx=dx, imag=imag, dt=dt, **prm)
    check(got, oracle.step_strang(cfg, psi0, 7))


def test_strang_equal_mixture_2d():
    nx, ny, dx, dt = 130, 70, 0.1, 2e-3
    prm = dict(PRM, so=api.SO_ERD)
    psi0 = start(2, nx, ny, dx, 3)
    got = run(psi0, dx, False, (6,), dt=dt, **prm)
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, dt=dt, **prm)
    check(got, oracle.step_strang(cfg, psi0, 6))


def test_strang_across_omega_segments():
    """Each Omega segment's run closes with its own P2 pass at that Omega."""
    nx, ny, dx, dt = 96, 48, 0.1, 2e-3
    prm = dict(PRM, omega=0.0)
    sched = [0.05, 0.4, 0.1, 0.25]
    psi0 = start(2, nx, ny, dx, 5)
    g, t = grid(psi0, dx, dt=dt, **prm)
    g.set_omega_schedule(sched, 5)
    g.step_real(13)
    g.step_real(6)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    g.close()
    ref = psi0
    for n in range(19):
        cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, dt=dt,
                         **dict(prm, omega=sched[min(n // 5, len(sched) - 1)]))
        ref = oracle.step_strang(cfg, ref, 1)
    check(got, ref)


@pytest.mark.parametrize("nx,ny", [(96, 48), (1024, 6)])
def test_strang_with_real_time_renorm(nx, ny):
    dx, dt = 0.1, 2e-3
    psi0 = start(2, nx, ny, dx, 9)
    g, t = grid(psi0, dx, dt=dt, **PRM)
    g.set_renorm_real(True)
    g.step_real(9)
    g.step_real(4)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    o = g.observables()
    g.close()
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, dt=dt, **PRM)
    ref = psi0
    for _ in range(13):
        ref = oracle.step_strang(cfg, ref, 1)
        ref, _ = oracle.renorm(cfg, ref)
    check(got, ref)
    assert abs(o["N"] - 1.0) < 1e-13


@pytest.mark.parametrize("nx,ny", [(128, 96), (1024, 5)])
def test_strang_complex64(nx, ny):
    dx, dt = 0.1, 2e-3
    psi0 = start(2, nx, ny, dx, 7)
    got = run(psi0, dx, False, (6,), dtype=torch.complex64, dt=dt, **PRM)
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, dt=dt, **PRM)
    assert rel(got, oracle.step_strang(cfg, psi0, 6)) < 1e-5


def test_strang_keeps_the_real_time_norm():
    n, dx = 256, 0.1
    psi0 = W.gaussian(2, n, n, dx, dx, phases=(0.3, 1.1, 2.0), width=2.0)
    g, _ = grid(psi0, dx, c0=2.0, c2=0.1, gamma=0.8, omega=0.2, dt=5e-3, so=api.SO_PX_SX)
    n0 = g.observables()["N"]
    g.step_real(400)
    n1 = g.observables()["N"]
    g.close()
    assert abs(n1 - n0) < 1e-12


@pytest.mark.parametrize("imag", [False, True], ids=["real", "imag"])
def test_strang_graph_replays_equal_one_by_one_launches(imag):
    nx, ny, dx, dt = 200, 90, 0.1, 2e-3
    psi0 = start(2, nx, ny, dx, 11)
    outs = []
    for every in (0, 1):
        g, t = grid(psi0, dx, dt=dt, **PRM)
        if every:
            g.profile(1, capacity=64)  # timed steps are launched one by one
        (g.step_imag if imag else g.step_real)(21)
        torch.cuda.synchronize()
        outs.append(t.cpu().numpy())
        g.close()
    np.testing.assert_array_equal(outs[0], outs[1])


def test_strang_second_order_on_256():
    """Real time to t = 0.02 at c2 = 40 on 256^2: the error against 2048
    steps falls 4-fold per halving of dt (GPU alone, beyond oracle sizes)."""
    n, dx, T = 256, 0.1, 0.02
    psi0 = W.gaussian(2, n, n, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5)
    prm = dict(c0=20.0, c2=40.0, gamma=0.6, omega=0.4, so=api.SO_PX_SX)

    def at(steps):
        return run(psi0, dx, False, (steps,), dt=T / steps, **prm)
    ref = at(2048)
    errs = [rel(at(k), ref) for k in (16, 32, 64)]
    for a, b in zip(errs, errs[1:]):
        assert 3.7 < a / b < 4.3, errs


def test_strang_refusals():
    t = torch.zeros((3, 16, 16), dtype=torch.complex128, device=DEV)
    g = api.Grid(t, 0.1, 0.1)
    g.set_params(dt=1e-3, gamma=0.5, so=api.SO_RASHBA)
    with pytest.raises(SSGPError) as e:
        g.set_scheme(api.SCHEME_STRANG)
    assert e.value.code == -1
    g.set_params(dt=1e-3, gamma=0.5, so=api.SO_PX_SX)
    g.set_scheme(api.SCHEME_STRANG)
    with pytest.raises(SSGPError) as e:
        g.set_params(dt=1e-3, gamma=0.5, so=api.SO_DRESSELHAUS)
    assert e.value.code == -1
    lam = torch.zeros_like(t)
    with pytest.raises(SSGPError) as e:
        g.step_real_adjoint(t.unsqueeze(0), lam, 1)
    assert e.value.code == -4
    g.close()
