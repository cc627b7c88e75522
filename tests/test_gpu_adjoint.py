"""Real-time adjoint on the GPU against the CPU oracle's adjoint (dual-number
Jacobians of the pointwise map, definitional adjoints of the linear
sub-steps) and against central differences."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2009_13507_amd import api, autograd  # noqa: E402
from paper_2009_13507_amd import workloads as W  # noqa: E402

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def oracle_chain(psi0, sched, sps, steps, base):
    """Forward states and the adjoint of L = dA sum |psi_{+1}(T)|^2."""
    states = []
    psi = psi0
    for n in range(steps):
        cfg = oracle.Cfg(**{**base, "omega": sched[min(n // sps, len(sched) - 1)]})
        states.append(psi)
        psi = oracle.step(cfg, psi, 1)
    dA = base["dx"] * (base["dy"] if base["dim"] == 2 else 1.0)
    lam = np.zeros_like(psi)
    lam[0] = 2 * dA * psi[0]
    dom = np.zeros(len(sched))
    for n in reversed(range(steps)):
        cfg = oracle.Cfg(**{**base, "omega": sched[min(n // sps, len(sched) - 1)]})
        lam, d = oracle.step_adjoint(cfg, states[n], lam)
        dom[min(n // sps, len(sched) - 1)] += d
    return psi, states, lam, dom


def base_cfg(dim, nx, ny, dx, dt=2e-3, so=api.SO_PX_SX):
    return dict(dim=dim, nx=nx, ny=ny if dim == 2 else 1, dx=dx, dy=dx, c0=2.0, c2=-0.4, gamma=0.5,
                dt=dt, imag=False, so=so)


def start(dim, nx, ny, dx, seed):
    base = W.gaussian(dim, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.4)
    return base * (1 + W.random_state(base.shape, seed, 0.05))


@pytest.mark.parametrize("dim,nx,ny,so", [(2, 40, 33, api.SO_PX_SX), (2, 130, 70, api.SO_PX_SX),
                                          (2, 300, 17, api.SO_PX_SX), (1, 200, 1, api.SO_PX_SX),
                                          (1, 600, 1, api.SO_PX_SX), (2, 64, 40, api.SO_ERD),
                                          (1, 200, 1, api.SO_PX_SY), (1, 200, 1, api.SO_PX_SZ),
                                          (2, 40, 33, api.SO_NONE)])
def test_adjoint_steps_match_oracle(dim, nx, ny, so):
    """Every SO coefficient pattern of the adjoint x-pass: neighbouring
    components with equal (S_x) or opposite (S_y, the equal mixture)
    coefficients, the diagonal (S_z), none."""
    dx = 0.3 if dim == 2 else 0.1
    base = base_cfg(dim, nx, ny, dx, so=so)
    sched = [0.05, 0.25, 0.12]
    sps, steps = 3, 9
    psi0 = start(dim, nx, ny, dx, 1)
    _, states, lam_ref, dom_ref = oracle_chain(psi0, sched, sps, steps, base)
    t_states = torch.from_numpy(np.stack(states)).to(DEV)
    work = torch.from_numpy(psi0.copy()).to(DEV)
    g = api.Grid(work, dx, dx)
    g.set_params(c0=base["c0"], c2=base["c2"], gamma=base["gamma"], dt=base["dt"], so=base["so"])
    g.set_omega_schedule(sched, sps)
    g.omega_grad(reset=True)
    psiT = oracle.step(oracle.Cfg(**{**base, "omega": sched[-1]}), states[-1], 1)
    dA = dx * (dx if dim == 2 else 1.0)
    lam = np.zeros_like(psiT)
    lam[0] = 2 * dA * psiT[0]
    t_lam = torch.from_numpy(lam).to(DEV)
    g.step_index = steps
    g.step_real_adjoint(t_states, t_lam, steps)
    assert g.step_index == 0
    dom = np.array(g.omega_grad(reset=True))
    assert rel(t_lam.cpu().numpy(), lam_ref) < 1e-10
    assert rel(dom, dom_ref) < 1e-10
    g.close()


@pytest.mark.parametrize("every", [4, 1, 7, 19])
def test_autograd_with_checkpoints_matches_oracle(every):
    """Checkpoints every 4 steps (5 segments, the last partial: the two
    segment buffers of the backward pass reused in turn), every step (no
    recomputation), every 7 (3 segments) and one segment (one buffer)."""
    nx, ny, dx = 48, 40, 0.3
    base = base_cfg(2, nx, ny, dx)
    sched = [0.1, 0.2, 0.05, 0.3]
    sps, steps = 5, 19     # 4 Omega segments, the last partial
    psi0 = start(2, nx, ny, dx, 2)
    psiT_ref, _, lam_ref, dom_ref = oracle_chain(psi0, sched, sps, steps, base)
    prob = autograd.RealTimeProblem(dx=dx, dy=dx, dt=base["dt"], steps=steps, steps_per_seg=sps,
                                    c0=base["c0"], c2=base["c2"], gamma=base["gamma"], so=base["so"],
                                    checkpoint=every)
    p0 = torch.from_numpy(psi0.copy()).to(DEV).requires_grad_(True)
    om = torch.tensor(sched, dtype=torch.float64, device=DEV, requires_grad=True)
    psiT = autograd.propagate(p0, om, prob)
    loss = dx * dx * (psiT[0].abs() ** 2).sum()
    loss.backward()
    assert rel(psiT.detach().cpu().numpy(), psiT_ref) < 1e-10
    assert rel(p0.grad.cpu().numpy(), lam_ref) < 1e-10
    assert rel(om.grad.cpu().numpy(), dom_ref) < 1e-10


def test_autograd_central_differences():
    """Gradients within 1e-6 of central differences with h = 1e-6."""
    nx, ny, dx = 36, 30, 0.35
    base = base_cfg(2, nx, ny, dx, dt=4e-3)
    sched = [0.15, 0.05]
    sps, steps = 6, 12
    psi0 = start(2, nx, ny, dx, 3)
    prob = autograd.RealTimeProblem(dx=dx, dy=dx, dt=base["dt"], steps=steps, steps_per_seg=sps,
                                    c0=base["c0"], c2=base["c2"], gamma=base["gamma"], so=base["so"])

    def loss_of(p, o):
        with torch.no_grad():
            out = autograd.propagate(p, o, prob)
            return float(dx * dx * (out[0].abs() ** 2).sum())

    p0 = torch.from_numpy(psi0.copy()).to(DEV).requires_grad_(True)
    om = torch.tensor(sched, dtype=torch.float64, device=DEV, requires_grad=True)
    out = autograd.propagate(p0, om, prob)
    (dx * dx * (out[0].abs() ** 2).sum()).backward()
    gp = p0.grad.cpu().numpy().reshape(-1)
    go = om.grad.cpu().numpy()
    h = 1e-6
    base_p = torch.from_numpy(psi0.copy()).to(DEV)
    rng = np.random.default_rng(0)
    for q in rng.choice(gp.size, 8, replace=False):
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            e = torch.zeros(gp.size, dtype=torch.complex128, device=DEV)
            e[q] = h * unit
            e = e.reshape(base_p.shape)
            fd = (loss_of(base_p + e, om.detach()) - loss_of(base_p - e, om.detach())) / (2 * h)
            assert abs(fd - part(gp[q])) < 1e-6 * max(1.0, abs(fd)), (q, fd, gp[q])
    for s in range(len(sched)):
        e = torch.zeros(len(sched), dtype=torch.float64, device=DEV)
        e[s] = h
        fd = (loss_of(base_p, om.detach() + e) - loss_of(base_p, om.detach() - e)) / (2 * h)
        assert abs(fd - go[s]) < 1e-6 * max(1.0, abs(fd)), (s, fd, go[s])


def test_central_differences_on_the_512_workload():
    """The differentiable workload at full size (512^2, 2000 real-time steps,
    100 Omega segments, checkpoints every 45 steps): gradients within 1e-6 of
    central differences with h = 1e-6 for Omega segments and for the real and
    imaginary parts of psi_0 where its gradient is largest; and, with h =
    1e-5, within 1e-6 relative for psi_0 and 1e-3 relative for Omega (whose
    gradients, about 3e-8, sit where the rounding of the loss difference,
    about 1e-16 L / h, allows no closer check)."""
    w = W.W2D_ADJ
    psi0 = W.interpolate(W.ground_256(), W.W2D_IMAG.nx, W.W2D_IMAG.dx, w.nx, w.dx)
    omega = W.omega_schedule(100, seed=2)
    prob = autograd.RealTimeProblem(dx=w.dx, dy=w.dy, dt=w.dt, steps=w.steps, steps_per_seg=w.steps // 100,
                                    c0=w.c0, c2=w.c2, gamma=w.gamma, so=w.so)
    p0 = torch.from_numpy(psi0).to(DEV).requires_grad_(True)
    om = torch.tensor(omega, dtype=torch.float64, device=DEV, requires_grad=True)
    out = autograd.propagate(p0, om, prob)
    (w.dx * w.dy * (out[0].abs() ** 2).sum()).backward()
    gp = p0.grad.cpu().numpy().reshape(-1)
    go = om.grad.cpu().numpy()
    base = torch.from_numpy(psi0).to(DEV)

    def loss(p, o):
        with torch.no_grad():
            r = autograd.propagate(p, o, prob)
            return float(w.dx * w.dy * (r[0].abs() ** 2).sum())

    q = int(np.abs(gp).argmax())
    for h, rel_psi, rel_om in ((1e-6, None, None), (1e-5, 1e-6, 1e-3)):
        for s in (0, 50, 99):
            e = torch.zeros(100, dtype=torch.float64, device=DEV)
            e[s] = h
            fd = (loss(base, om.detach() + e) - loss(base, om.detach() - e)) / (2 * h)
            print(f"  h={h} Omega[{s}]: fd {fd:.6e}, adjoint {go[s]:.6e}", flush=True)
            assert abs(fd - go[s]) < 1e-6 * max(1.0, abs(fd))
            if rel_om:
                assert abs(fd - go[s]) < rel_om * abs(go[s])
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            e = torch.zeros(gp.size, dtype=torch.complex128, device=DEV)
            e[q] = h * unit
            e = e.reshape(base.shape)
            fd = (loss(base + e, om.detach()) - loss(base - e, om.detach())) / (2 * h)
            print(f"  h={h} psi0[{q}]: fd {fd:.9e}, adjoint {part(gp[q]):.9e}", flush=True)
            assert abs(fd - part(gp[q])) < 1e-6 * max(1.0, abs(fd))
            if rel_psi:
                assert abs(fd - part(gp[q])) < rel_psi * abs(part(gp[q]))
