"""The device-side observables log (ssgp_obs_reserve / ssgp_obs_record /
ssgp_obs_log_read) against ssgp_observables of the same states, and the Omega
rule of the Rabi energy (the Omega of the last step taken), through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2009_13507_amd import api  # noqa: E402
from paper_2009_13507_amd import workloads as W  # noqa: E402
from paper_2009_13507_amd._lib import SSGPError  # noqa: E402

DEV = "cuda:0"
KEYS = ("N+1", "N0", "N-1", "N", "M", "E", "E_kin", "E_trap", "E_c0", "E_c2", "E_rabi", "E_so",
        "rms+1", "rms0", "rms-1", "rms")


def agree(a, b, tol=1e-10):
    for k in KEYS:
        if abs(b[k]) < 1e-2:
            assert abs(a[k] - b[k]) < 1e-12, (k, a[k], b[k])
        else:
            assert abs(a[k] - b[k]) < tol * abs(b[k]), (k, a[k], b[k])


def test_log_samples_equal_synchronous_observables():
    nx, ny, dx = 96, 80, 0.2
    p = dict(c0=3.0, c2=-0.4, gamma=0.6, omega=0.3, dt=2e-3, so=api.SO_PX_SX)
    psi0 = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5)
    # reference: observables after 0, 7, 14, 21 steps, taken synchronously
    t = torch.from_numpy(psi0.copy()).to(DEV)
    g = api.Grid(t, dx, dx)
    g.set_params(**p)
    ref = [g.observables()]
    for _ in range(3):
        g.step_real(7)
        ref.append(g.observables())
    g.close()
    # the same states sampled into the device log inside the stepping loop
    t = torch.from_numpy(psi0.copy()).to(DEV)
    g = api.Grid(t, dx, dx)
    g.set_params(**p)
    g.obs_log_reserve(4)
    g.obs_record()
    for _ in range(3):
        g.step_real(7)
        g.obs_record()
    with pytest.raises(SSGPError) as e:
        g.obs_record()  # the log is full
    assert e.value.code == -4
    got = g.obs_log_read()
    g.close()
    assert len(got) == 4
    for a, b in zip(got, ref):
        agree(a, b)
    # and against the oracle's observables of the oracle's states
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, **p)
    agree(got[-1], oracle.observables(cfg, oracle.step(cfg, psi0, 21)))


def test_log_reserve_empties_the_log():
    t = torch.from_numpy(W.gaussian(2, 32, 24, 0.3, 0.3)).to(DEV)
    g = api.Grid(t, 0.3, 0.3)
    g.set_params(dt=1e-3)
    g.obs_log_reserve(2)
    g.obs_record()
    assert len(g.obs_log_read()) == 1
    g.obs_log_reserve(2)
    assert g.obs_log_read() == []
    g.close()


def test_rabi_energy_uses_the_omega_of_the_last_step():
    """With a real-time Omega schedule set, an imaginary-time state's Rabi
    energy is taken with params.omega (the Omega it was relaxed with); after
    real-time steps, with the Omega of the last one."""
    nx, ny, dx = 64, 48, 0.25
    p = dict(c0=2.0, c2=-0.3, gamma=0.0, omega=0.4, dt=2e-3, so=api.SO_NONE)
    psi0 = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5)
    t = torch.from_numpy(psi0.copy()).to(DEV)
    g = api.Grid(t, dx, dx)
    g.set_params(**p)
    sched = [0.05, 0.25]
    g.set_omega_schedule(sched, 5)
    g.step_imag(10)
    o = g.observables()
    state = t.cpu().numpy()
    cfg = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=True, **p)
    agree(o, oracle.observables(cfg, state))
    g.step_index = 0
    g.step_real(7)  # steps 0..6: the last one (6) in segment 1
    o = g.observables()
    state = t.cpu().numpy()
    cfg1 = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, **dict(p, omega=sched[1]))
    agree(o, oracle.observables(cfg1, state))
    g.set_params(**dict(p, omega=0.1))  # new parameters: params.omega again
    o = g.observables()
    cfg2 = oracle.Cfg(dim=2, nx=nx, ny=ny, dx=dx, dy=dx, imag=False, **dict(p, omega=0.1))
    agree(o, oracle.observables(cfg2, state))
    g.close()
