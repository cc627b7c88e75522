"""Seeded synthetic inputs for the spin-1 SS-CN workloads.

This module only builds inputs: grids, Gaussian trial states, seeded phases
and parameter draws, and the separable linear interpolation of a stored state
onto a finer grid.  It holds none of the time-stepping arithmetic, and both
the GPU path and the CPU oracle take their inputs from here.

States are numpy ``complex128`` arrays of shape ``(3, ny, nx)`` (2D) or
``(3, nx)`` (1D), component order (+1, 0, -1), x fastest.  Grid points are
``x_i = -nx*dx/2 + i*dx`` (a half-open box, so even ``nx`` is asymmetric by one
point), the same for y.

The imaginary-time runs start from a Gaussian trial state, which is the
paper's choice when the ground state has no vortex or stripe (Sec. 3); the
vortex and stripe trial states of SO-coupled 2D condensates, and the rule that
picks one of them, are here too.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, replace

import numpy as np

SO_NONE, SO_PX_SX, SO_PX_SY, SO_PX_SZ, SO_RASHBA, SO_DRESSELHAUS, SO_ERD = range(7)
RENORM_AUTO, RENORM_NORM, RENORM_FIXED_M = range(3)

_HERE = os.path.dirname(os.path.abspath(__file__))
_REPO = os.path.dirname(_HERE)
# Ground state of the 256^2 imaginary-time workload, written by
# tests/golden/make_ground_256.py from the CPU oracle.
GROUND_256 = os.path.join(_REPO, "tests", "golden", "ground_256.npy")


@dataclass(frozen=True)
class Workload:
    """One run: grid, model parameters, time step and step count."""
    name: str
    dim: int
    nx: int
    ny: int
    dx: float
    dy: float
    dt: float
    steps: int
    imag: bool
    c0: float
    c2: float
    gamma: float
    omega: float
    so: int = SO_PX_SX
    renorm: int = RENORM_AUTO
    mag0: float = 0.0
    kappa: float = 1.0

    @property
    def npts(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)

    def shape(self):
        return (3, self.ny, self.nx) if self.dim == 2 else (3, self.nx)


# The five workloads of the measurement plan (sizes, steps and parameters as
# stated there; the spin-orbit term of the 2D runs is gamma p_x Sigma_x).
W1D = Workload("1d-imag-512", 1, 512, 1, 0.05, 0.05, 5e-4, 20000, True,
               0.885, -0.0041, 0.0, 0.0, so=SO_NONE)
W2D_IMAG = Workload("2d-imag-256-so-rabi", 2, 256, 256, 0.1, 0.1, 5e-3, 10000, True,
                    2.0, -0.1, 0.5, 0.1)
# real-time quench: c2 -0.1 -> +0.1, gamma 0.5 -> 0.8, Omega 0.1 -> 0.2 at t = 0
W2D_REAL = Workload("2d-real-1024-quench", 2, 1024, 1024, 0.05, 0.05, 1e-4, 5000, False,
                    2.0, 0.1, 0.8, 0.2)
W2D_ADJ = Workload("2d-real-512-adjoint", 2, 512, 512, 0.05, 0.05, 2e-4, 2000, False,
                   2.0, -0.1, 0.5, 0.0)
BATCH_SIZES = (128, 192, 256, 384, 512)


def coords(n: int, h: float) -> np.ndarray:
    return -0.5 * n * h + h * np.arange(n)


def area(w) -> float:
    return w.dx * w.dy if w.dim == 2 else w.dx


def normalise(psi: np.ndarray, dA: float) -> np.ndarray:
    """Scale the input so that dA * sum |psi|^2 = 1 (rectangle rule)."""
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2) * dA)


def gaussian(dim: int, nx: int, ny: int, dx: float, dy: float,
             weights=(0.25, 0.5, 0.25), phases=(0.0, 0.0, 0.0), width: float = 1.0):
    """psi_j = sqrt(w_j) e^{i theta_j} exp(-r^2 / (2 width^2)), total norm 1."""
    x = coords(nx, dx)
    if dim == 1:
        g = np.exp(-x ** 2 / (2 * width ** 2))
        dA = dx
    else:
        y = coords(ny, dy)
        g = np.exp(-(y[:, None] ** 2 + x[None, :] ** 2) / (2 * width ** 2))
        dA = dx * dy
    psi = np.stack([np.sqrt(w) * np.exp(1j * th) * g for w, th in zip(weights, phases)])
    return normalise(psi.astype(np.complex128), dA)


def vortex(nx: int, ny: int, dx: float, dy: float, lz=(0, 0, 0),
           weights=(0.25, 0.5, 0.25), width: float = 1.0):
    """2D Gaussian trial state with a vortex of angular momentum L_j imprinted
    on component j (Sec. 3): psi_j is multiplied by (x + iy)^L_j, or by
    (x - iy)^|L_j| for an anti-vortex (L_j < 0).  Total norm 1."""
    x = coords(nx, dx)
    y = coords(ny, dy)
    X, Y = x[None, :], y[:, None]
    g = np.exp(-(X ** 2 + Y ** 2) / (2 * width ** 2))
    comps = []
    for w, L in zip(weights, lz):
        z = X + 1j * Y if L >= 0 else X - 1j * Y
        comps.append(np.sqrt(w) * g * z ** abs(int(L)))
    return normalise(np.stack(comps).astype(np.complex128), dx * dy)


def stripes(nx: int, ny: int, dx: float, dy: float, gamma: float, width: float = 1.0):
    """2D Gaussian trial state with a stripe modulation along x (Sec. 3): the
    Gaussian times the polar stripe spinor of Sec. S.2, i sin(gamma x)/sqrt(2)
    in the +-1 components and -cos(gamma x) in the 0 component.  Total norm 1."""
    x = coords(nx, dx)
    y = coords(ny, dy)
    g = np.exp(-(x[None, :] ** 2 + y[:, None] ** 2) / (2 * width ** 2))
    sp = 1j * np.sin(gamma * x)[None, :] / np.sqrt(2.0) * g
    c0 = -np.cos(gamma * x)[None, :] * g
    return normalise(np.stack([sp, c0, sp]).astype(np.complex128), dx * dy)


OPT_ST = 0.75


def so_trial_kind(so: int, gamma: float, c2: float, opt_st: float = OPT_ST):
    """The 2D trial-state rule of Sec. 3, as ("gaussian", None), ("vortex",
    (L_+1, L_0, L_-1)) or ("stripes", None).

    Polar (c2 > 0) below opt_st: (-1, 0, +1) under Rashba coupling, (+1, 0, -1)
    under Dresselhaus; above opt_st: stripes.  Ferro (c2 <= 0): (0, +1, +2)
    under Rashba, (0, -1, -2) under Dresselhaus.  The equal mixture takes a
    Gaussian in the ferro phase and stripes in the polar phase.  Without a 2D
    SO coupling the trial state is a Gaussian."""
    polar = c2 > 0
    if gamma == 0.0 or so not in (SO_RASHBA, SO_DRESSELHAUS, SO_ERD):
        return "gaussian", None
    if so == SO_ERD:
        return ("stripes", None) if polar else ("gaussian", None)
    sign = 1 if so == SO_RASHBA else -1
    if polar:
        if gamma > opt_st:
            return "stripes", None
        return "vortex", (-sign, 0, sign)
    return "vortex", (0, sign, 2 * sign)


def so_trial(nx: int, ny: int, dx: float, dy: float, so: int, gamma: float, c2: float,
             opt_st: float = OPT_ST, width: float = 1.0, weights=(0.25, 0.5, 0.25)):
    """The 2D trial state that so_trial_kind selects."""
    kind, lz = so_trial_kind(so, gamma, c2, opt_st)
    if kind == "vortex":
        return vortex(nx, ny, dx, dy, lz, weights, width)
    if kind == "stripes":
        return stripes(nx, ny, dx, dy, gamma, width)
    return gaussian(2, nx, ny, dx, dy, weights=weights, width=width)


def phases_seed0():
    """One global phase per component, drawn in the order (+1, 0, -1)."""
    return np.random.default_rng(0).uniform(0.0, 2 * np.pi, 3)


def initial_1d(w: Workload = W1D):
    return gaussian(1, w.nx, 1, w.dx, w.dx)


def initial_2d_imag(w: Workload = W2D_IMAG):
    return gaussian(2, w.nx, w.ny, w.dx, w.dy, phases=phases_seed0())


def random_state(shape, seed: int, scale: float = 1.0):
    """Uniform random complex values (for sub-step tests on small grids)."""
    rng = np.random.default_rng(seed)
    return (scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex128)


def interpolate(psi: np.ndarray, src_n: int, src_h: float, dst_n: int, dst_h: float) -> np.ndarray:
    """Separable linear interpolation of a 2D state between two centred grids,
    zero outside the source box, then normalised to 1 on the target grid."""
    xs = coords(src_n, src_h)
    xd = coords(dst_n, dst_h)
    # weights of the two source neighbours of every target point; a target
    # point outside [xs[0], xs[-1]] gets zero
    W = np.zeros((dst_n, src_n))
    for k, x in enumerate(xd):
        t = (x - xs[0]) / src_h
        if t < 0.0 or t > src_n - 1:
            continue
        lo = min(int(np.floor(t)), src_n - 2)
        fr = t - lo
        W[k, lo] += 1.0 - fr
        W[k, lo + 1] += fr
    out = np.stack([W @ psi[j] @ W.T for j in range(3)]).astype(np.complex128)
    return normalise(out, dst_h * dst_h)


def ground_256():
    """The stored ground state of the 256^2 imaginary-time workload."""
    if not os.path.exists(GROUND_256):
        raise FileNotFoundError(
            f"{GROUND_256} is missing; run tests/golden/make_ground_256.py to create it")
    return np.load(GROUND_256, allow_pickle=False)


def initial_2d_real(w: Workload = W2D_REAL):
    """The 256^2 ground state interpolated onto the workload's grid."""
    g = ground_256()
    return interpolate(g, W2D_IMAG.nx, W2D_IMAG.dx, w.nx, w.dx)


def batch_draw(n: int = 64, seed: int = 1):
    """Sizes and parameters of the batched imaginary-time workload, in a fixed
    draw order: sizes, c0, c2, gamma, Omega, then per-instance phases."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice(np.array(BATCH_SIZES), n)
    c0 = rng.uniform(0.5, 5.0, n)
    c2 = rng.uniform(-0.5, 0.5, n)
    gamma = rng.uniform(0.0, 1.0, n)
    omega = rng.uniform(0.0, 0.5, n)
    phases = rng.uniform(0.0, 2 * np.pi, (n, 3))
    out = []
    for i in range(n):
        N = int(sizes[i])
        w = Workload(f"batch-{i}-{N}", 2, N, N, 0.1, 0.1, 2.5e-3, 4000, True,
                     float(c0[i]), float(c2[i]), float(gamma[i]), float(omega[i]))
        out.append((w, phases[i]))
    return out


def batch_initial(w: Workload, phases):
    """Initial state of one batched instance: the Gaussian trial state of the
    2D imaginary-time workload with the instance's own component phases."""
    return gaussian(2, w.nx, w.ny, w.dx, w.dy, phases=tuple(phases))


def omega_schedule(nseg: int = 100, seed: int = 2):
    """Piecewise-constant Rabi control: one Omega per segment, U[0, 0.3]."""
    return np.random.default_rng(seed).uniform(0.0, 0.3, nseg)


def scaled(w: Workload, **kw) -> Workload:
    return replace(w, **kw)
