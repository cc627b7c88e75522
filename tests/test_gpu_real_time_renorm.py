"""RENORM after every real-time step (opt-in, ssgp_set_renorm_real) on the
GPU against the oracle's definition (oracle.step_real_renorm: each step, then
the rule of Eqs. (DJ)/(DJ2)): relative L2 <= 1e-10 in FP64 for the paper's
scheme (graph-replayed runs, the y-derivative SO path included) and the unitary-SO scheme, in 2D and 1D, across Omega-schedule
segments; graph replays bitwise equal to one-by-one launches; switching it
off; and the refusals."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2009_13507_amd import api  # noqa: E402
from paper_2009_13507_amd import workloads as W  # noqa: E402
from paper_2009_13507_amd._lib import SSGPError  # noqa: E402

DEV = "cuda:0"


def start2d(nx, ny, dx, seed):
    base = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=0.18 * min(nx, 4 * ny) * dx)
    return base * (1 + W.random_state(base.shape, seed, 0.05))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def grid(psi0, dx, dim, **prm):
    t = torch.from_numpy(psi0.copy()).to(DEV)
    g = api.Grid(t, dx, dx) if dim == 2 else api.Grid(t, dx)
    g.set_params(**prm)
    g.set_renorm_real(True)
    return g, t


@pytest.mark.parametrize("so", [api.SO_PX_SX, api.SO_RASHBA], ids=["px_sx", "rashba"])
@pytest.mark.parametrize("nx,ny", [(72, 40), (256, 20), (1024, 5)])
def test_2d_matches_oracle(nx, ny, so):
    dx = 0.1
    prm = dict(c0=2.0, c2=-0.3, gamma=0.7, omega=0.15, dt=2e-3, so=so)
    psi0 = start2d(nx, ny, dx, nx + so)
    print(f"real-time RENORM 2D nx={nx} ny={ny} so={so}", flush=True)
    g, t = grid(psi0, dx, 2, **prm)
    for n in (13, 1, 20):
        g.step_real(n)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    o = g.observables()
    g.close()
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, **prm)
    want = oracle.step_real_renorm(cfg, psi0, 34)
    assert rel(got, want) < 1e-10
    assert abs(o["N"] - 1.0) < 1e-13


def test_2d_across_omega_segments():
    nx, ny, dx = 96, 48, 0.1
    prm = dict(c0=2.0, c2=0.2, gamma=0.5, omega=0.0, dt=2e-3, so=api.SO_PX_SX)
    psi0 = start2d(nx, ny, dx, 4)
    sched = [0.05, 0.3, 0.1, 0.2, 0.0]
    g, t = grid(psi0, dx, 2, **prm)
    g.set_omega_schedule(sched, 7)
    g.step_real(25)
    g.step_real(9)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    g.close()
    ref = psi0
    for s in range(34):
        cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False,
                         **dict(prm, omega=sched[min(s // 7, len(sched) - 1)]))
        ref = oracle.step_real_renorm(cfg, ref, 1)
    assert rel(got, ref) < 1e-10


@pytest.mark.parametrize("rule", ["norm", "fixed_m"])
def test_1d_matches_oracle(rule):
    nx, dx = 640, 0.05
    if rule == "norm":
        prm = dict(c0=30.0, c2=-2.0, gamma=0.6, omega=0.1, dt=5e-4, so=api.SO_PX_SX)
        wts = (0.25, 0.5, 0.25)
    else:
        prm = dict(c0=30.0, c2=2.0, dt=5e-4, renorm=api.RENORM_FIXED_M, mag0=0.2)
        wts = (0.55, 0.1, 0.35)
    psi0 = W.gaussian(1, nx, 1, dx, dx, weights=wts, phases=(0.3, 1.1, 2.0), width=3.0)
    g, t = grid(psi0, dx, 1, **prm)
    g.step_real(17)
    g.step_real(5)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    o = g.observables()
    g.close()
    cfg = oracle.Cfg(dim=1, nx=nx, ny=1, dx=dx, dy=dx, imag=False, **prm)
    want = oracle.step_real_renorm(cfg, psi0, 22)
    assert rel(got, want) < 1e-10
    assert abs(o["N"] - 1.0) < 1e-13
    if rule == "fixed_m":
        assert abs(o["M"] - 0.2) < 1e-13


@pytest.mark.parametrize("dim", [1, 2])
def test_unitary_so_scheme_with_renorm(dim):
    dx = 0.1
    prm = dict(c0=2.0, c2=-0.3, gamma=0.7, omega=0.15, dt=2e-3, so=api.SO_PX_SX)
    if dim == 2:
        nx, ny = 128, 40
        psi0 = start2d(nx, ny, dx, 8)
    else:
        nx, ny = 512, 1
        psi0 = W.gaussian(1, nx, 1, dx, dx, phases=(0.3, 1.1, 2.0), width=4.0)
    g, t = grid(psi0, dx, dim, **prm)
    g.set_scheme(api.SCHEME_UNITARY_SO)
    g.step_real(10)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    g.close()
    cfg = oracle.Cfg(dim=dim, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, **prm)
    want = oracle.step_real_renorm(cfg, psi0, 10, unitary_so=True)
    assert rel(got, want) < 1e-10


def test_graph_replays_match_one_by_one_launches():
    nx, ny, dx = 96, 64, 0.1
    prm = dict(c0=2.0, c2=-0.3, gamma=0.7, omega=0.15, dt=2e-3, so=api.SO_PX_SX)
    psi0 = start2d(nx, ny, dx, 3)
    outs = []
    for eager in (True, False):
        g, t = grid(psi0, dx, 2, **prm)
        if eager:
            g.profile(1, 100000)
        for n in (13, 64, 7):
            g.step_real(n)
            _ = (t.abs() ** 2).sum().item()
        torch.cuda.synchronize()
        outs.append(t.cpu().numpy())
        g.close()
    assert np.array_equal(outs[0], outs[1])


def test_switching_off_restores_plain_real_time_steps():
    nx, ny, dx = 80, 24, 0.1
    prm = dict(c0=2.0, c2=-0.3, gamma=0.7, omega=0.15, dt=2e-3, so=api.SO_PX_SX)
    psi0 = start2d(nx, ny, dx, 5)
    g, t = grid(psi0, dx, 2, **prm)
    g.step_real(3)
    g.set_renorm_real(False)
    g.step_real(4)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    g.close()
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, **prm)
    want = oracle.step(cfg, oracle.step_real_renorm(cfg, psi0, 3), 4)
    assert rel(got, want) < 1e-10


def test_refusals():
    nx, ny, dx = 64, 48, 0.1
    g, t = grid(start2d(nx, ny, dx, 9), dx, 2, c0=1.0, gamma=0.5, dt=1e-3, so=api.SO_PX_SX)
    assert g._lib.ssgp_set_renorm_real(g._h, 2) < 0   # only 0 or 1
    with pytest.raises(SSGPError):
        g.step_real_seq(t, torch.empty((1,) + tuple(t.shape), dtype=t.dtype, device=DEV), 1)
    g.close()


def test_2d_complex64():
    nx, ny, dx = 128, 96, 0.1
    prm = dict(c0=2.0, c2=-0.3, gamma=0.7, omega=0.15, dt=2e-3, so=api.SO_PX_SX)
    psi0 = start2d(nx, ny, dx, 6)
    t = torch.from_numpy(psi0.copy()).to(DEV, torch.complex64)
    g = api.Grid(t, dx, dx)
    g.set_params(**prm)
    g.set_renorm_real(True)
    g.step_real(20)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.complex128)
    o = g.observables()
    g.close()
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, **prm)
    assert rel(got, oracle.step_real_renorm(cfg, psi0, 20)) < 1e-5
    assert abs(o["N"] - 1.0) < 1e-6
