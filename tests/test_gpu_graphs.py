"""Runs of 2D steps replayed as HIP graphs against the same steps launched one
by one (kernel timing on every step forces the one-by-one path): bitwise
equal after every call, with other device work and synchronisations between
the replays, in imaginary and real time and across Omega-schedule segments;
and graph-replayed runs against the CPU oracle (relative L2 <= 1e-10)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2009_13507_amd import api  # noqa: E402
from paper_2009_13507_amd import workloads as W  # noqa: E402

DEV = "cuda:0"


def pair(nx, ny, dx, **prm):
    base = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5)
    psi0 = base * (1 + W.random_state(base.shape, 4, 0.05))
    grids = []
    for eager in (True, False):
        t = torch.from_numpy(psi0.copy()).to(DEV)
        g = api.Grid(t, dx, dx)
        g.set_params(**prm)
        if eager:
            g.profile(1, 100000)
        grids.append((g, t))
    return grids


def same(a, b):
    torch.cuda.synchronize()
    return np.array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("nx,ny", [(64, 48), (256, 40), (100, 37)])
def test_imaginary_time_graphs_match_eager(nx, ny):
    (ge, te), (gg, tg) = pair(nx, ny, 0.25, c0=2.0, c2=-0.3, gamma=0.5, omega=0.1, dt=2e-3, so=api.SO_PX_SX)
    for n in (13, 64, 7, 100):
        ge.step_imag(n)
        gg.step_imag(n)
        # other work on the device between the replays
        _ = (tg.abs() ** 2).sum().item()
        assert same(te, tg), n
        assert ge.observables()["E"] == gg.observables()["E"]
    ge.close()
    gg.close()


def test_real_time_graphs_match_eager_across_segments():
    (ge, te), (gg, tg) = pair(128, 64, 0.2, c0=2.0, c2=0.1, gamma=0.8, omega=0.2, dt=1e-3, so=api.SO_PX_SX)
    sched = [0.05, 0.3, 0.1, 0.0]
    for g in (ge, gg):
        g.set_omega_schedule(sched, 17)
    for n in (37, 5, 26):
        ge.step_real(n)
        gg.step_real(n)
        torch.cuda.synchronize()
        assert same(te, tg), n
    assert ge.step_index == gg.step_index == 68
    ge.close()
    gg.close()


def test_set_params_invalidates_graphs():
    (ge, te), (gg, tg) = pair(64, 64, 0.25, c0=1.0, c2=0.2, gamma=0.3, omega=0.1, dt=2e-3, so=api.SO_PX_SX)
    for g in (ge, gg):
        g.step_imag(16)
        g.set_params(c0=3.0, c2=-0.2, gamma=0.6, omega=0.05, dt=2e-3, so=api.SO_PX_SX)
        g.step_imag(16)
    assert same(te, tg)
    ge.close()
    gg.close()


@pytest.mark.parametrize("imag,calls", [(True, (13, 64, 3)), (False, (13, 64, 3))])
def test_graph_runs_match_oracle(imag, calls):
    nx, ny, dx = 72, 40, 0.25
    prm = dict(c0=2.0, c2=-0.3, gamma=0.5, omega=0.1, dt=2e-3, so=api.SO_PX_SX)
    base = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5)
    psi0 = base * (1 + W.random_state(base.shape, 5, 0.05))
    t = torch.from_numpy(psi0.copy()).to(DEV)
    g = api.Grid(t, dx, dx)
    g.set_params(**prm)
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=imag, **prm)
    ref = psi0
    for n in calls:
        (g.step_imag if imag else g.step_real)(n)
        ref = oracle.step(cfg, ref, n)
        torch.cuda.synchronize()
        got = t.cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10, n
    g.close()


@pytest.mark.parametrize("every,capacity", [(5, 1000), (7, 3)])
def test_sampled_timing_mixes_graphs_and_single_steps(every, capacity):
    """Kernel timing on every few steps (and a capacity that runs out) splits
    the runs around the timed steps; the result stays bitwise equal."""
    (ge, te), (gg, tg) = pair(96, 64, 0.25, c0=2.0, c2=0.1, gamma=0.8, omega=0.2, dt=1e-3, so=api.SO_PX_SX)
    gg.profile(every, capacity)
    for n in (37, 20):
        ge.step_real(n)
        gg.step_real(n)
        assert same(te, tg), n
    p = gg.profile_read()
    # steps 0 .. 56 of the counter; every every-th one is timed, up to capacity
    assert p["steps"] == min(capacity, len(range(0, 57, every)))
    ge.close()
    gg.close()



@pytest.mark.parametrize("imag", [False, True], ids=["real", "imag"])
def test_y_derivative_so_runs_as_graphs(imag):
    """The Rashba form (its pointwise pass writes a scratch copy that the
    x-pass reads) replayed as graphs: bitwise equal to one-by-one launches,
    and against the oracle."""
    nx, ny, dx = 80, 56, 0.25
    prm = dict(c0=2.0, c2=-0.3, gamma=0.5, omega=0.1, dt=2e-3, so=api.SO_RASHBA)
    (ge, te), (gg, tg) = pair(nx, ny, dx, **prm)
    base = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5)
    psi0 = base * (1 + W.random_state(base.shape, 4, 0.05))
    for n in (13, 64, 7):
        (ge.step_imag if imag else ge.step_real)(n)
        (gg.step_imag if imag else gg.step_real)(n)
        _ = (tg.abs() ** 2).sum().item()
        assert same(te, tg), n
    got = tg.cpu().numpy()
    ge.close()
    gg.close()
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=imag, **prm)
    want = oracle.step(cfg, psi0, 84)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-10
