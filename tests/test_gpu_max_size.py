"""The largest 2D grid the library accepts (2048 x 2048: rows of 2048 points,
the longest x line and the tallest y tile) against the oracle, element by
element on the whole state: the paper's scheme with the x-derivative SO form
and with the Rashba form (the y-derivative x-pass variant), the unitary-SO
scheme, in real and imaginary time; relative L2 <= 1e-10 in FP64 and
<= 1e-5 in complex64.  The state carries a small additive noise so that the
edge rows and columns hold non-zero values."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2009_13507_amd import api  # noqa: E402
from paper_2009_13507_amd import workloads as W  # noqa: E402

DEV = "cuda:0"
N = 2048
DX = 0.02
PRM = dict(c0=2.0, c2=-0.3, gamma=0.6, omega=0.2)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def start(seed):
    base = W.gaussian(2, N, N, DX, DX, phases=(0.3, 1.1, 2.0), width=0.25 * N * DX)
    return base * (1 + W.random_state(base.shape, seed, 0.05)) + W.random_state(base.shape, seed + 1, 1e-3)


def gpu(psi0, imag, nsteps, scheme=api.SCHEME_PAPER, dtype=torch.complex128, **prm):
    t = torch.from_numpy(psi0).to(DEV, dtype)
    g = api.Grid(t, DX, DX)
    g.set_params(**prm)
    g.set_scheme(scheme)
    (g.step_imag if imag else g.step_real)(nsteps)
    torch.cuda.synchronize()
    out = t.cpu().numpy().astype(np.complex128)
    g.close()
    return out


@pytest.mark.parametrize("imag", [False, True], ids=["real", "imag"])
@pytest.mark.parametrize("so", [api.SO_PX_SX, api.SO_RASHBA], ids=["px_sx", "rashba"])
def test_paper_scheme_at_2048_squared(so, imag):
    dt = 1e-3 if imag else 1e-4
    prm = dict(PRM, dt=dt, so=so)
    psi0 = start(11 + so)
    print(f"max size 2048^2 so={so} imag={imag}", flush=True)
    got = gpu(psi0, imag, 3, **prm)
    want = oracle.step(oracle.Cfg(dim=2, nx=N, ny=N, dx=DX, dy=DX, imag=imag, **prm), psi0, 3)
    assert rel(got, want) < 1e-10


@pytest.mark.parametrize("imag", [False, True], ids=["real", "imag"])
def test_unitary_so_scheme_at_2048_squared(imag):
    dt = 1e-3 if imag else 1e-4
    prm = dict(PRM, dt=dt, so=api.SO_PX_SX)
    psi0 = start(21)
    print(f"max size 2048^2 unitary SO imag={imag}", flush=True)
    got = gpu(psi0, imag, 2, scheme=api.SCHEME_UNITARY_SO, **prm)
    cfg = oracle.Cfg(dim=2, nx=N, ny=N, dx=DX, dy=DX, imag=imag, **prm)
    want = oracle.step_unitary_so(cfg, psi0, 2)
    assert rel(got, want) < 1e-10


def test_complex64_at_2048_squared():
    prm = dict(PRM, dt=1e-4, so=api.SO_PX_SX)
    psi0 = start(31)
    print("max size 2048^2 complex64", flush=True)
    got = gpu(psi0, False, 20, dtype=torch.complex64, **prm)
    want = oracle.step(oracle.Cfg(dim=2, nx=N, ny=N, dx=DX, dy=DX, imag=False, **prm), psi0, 20)
    assert rel(got, want) < 1e-5
