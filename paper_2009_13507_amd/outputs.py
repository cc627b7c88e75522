"""Output quantities of a converged or propagated state (the output files of
Sec. 3): component and total densities, the radial density of a 2D state, the
phases of the components, and the winding number of a component around the
trap centre, with text writers in the paper's column layout.

Everything here works on a state copied to the host (numpy, shape (3, ny, nx)
in 2D or (3, nx) in 1D, component order (+1, 0, -1), x fastest, grid points
x_i = -nx*dx/2 + i*dx).  It post-processes a result once; it does not advance
a state, and the stepping itself runs only in the HIP library.
"""
from __future__ import annotations

import numpy as np

from .workloads import coords


def density(psi: np.ndarray) -> np.ndarray:
    """rho_+1, rho_0, rho_-1 and rho = their sum, stacked: shape (4, ...)."""
    rho = np.abs(np.asarray(psi)) ** 2
    return np.concatenate([rho, rho.sum(axis=0, keepdims=True)])


def phase(psi: np.ndarray) -> np.ndarray:
    """Phases of the three components in (-pi, pi]."""
    return np.angle(np.asarray(psi))


def radial_density(psi: np.ndarray, dx: float, dy: float, dr: float | None = None,
                   rmax: float | None = None):
    """Azimuthal averages of the four densities of a 2D state over annuli of
    width dr (default min(dx, dy)) about the trap centre, out to rmax (default
    the largest circle inside the box).  Returns (r, rho) with r the annulus
    mid-radii and rho of shape (4, len(r)); an annulus that holds no grid
    point gets NaN.  For a circularly symmetric state this is the density as
    a function of r."""
    psi = np.asarray(psi)
    if psi.ndim != 3:
        raise ValueError("radial_density needs a 2D state of shape (3, ny, nx)")
    _, ny, nx = psi.shape
    dr = min(dx, dy) if dr is None else dr
    x, y = coords(nx, dx), coords(ny, dy)
    if rmax is None:
        rmax = min(-x[0], x[-1], -y[0], y[-1])
    nr = int(np.floor(rmax / dr))
    r = np.hypot(x[None, :], y[:, None])
    k = np.floor(r / dr).astype(np.int64).ravel()
    keep = k < nr
    rho = density(psi).reshape(4, -1)
    count = np.bincount(k[keep], minlength=nr).astype(np.float64)
    out = np.full((4, nr), np.nan)
    nz = count > 0
    for c in range(4):
        s = np.bincount(k[keep], weights=rho[c][keep], minlength=nr)
        out[c, nz] = s[nz] / count[nz]
    return (np.arange(nr) + 0.5) * dr, out


def winding(comp: np.ndarray, half: int) -> int:
    """Winding number of one 2D component around the grid point nearest the
    trap centre: the phase increments along the square loop of grid points at
    Chebyshev distance `half` from it, counter-clockwise (increasing x, then
    increasing y), summed and divided by 2 pi.  The loop must avoid zeros of
    the component."""
    comp = np.asarray(comp)
    ny, nx = comp.shape
    ic, jc = ny // 2, nx // 2
    if not (0 < half <= min(ic, jc, ny - 1 - ic, nx - 1 - jc)):
        raise ValueError("loop does not fit in the grid")
    path = []
    for j in range(jc - half, jc + half):          # bottom edge, +x
        path.append((ic - half, j))
    for i in range(ic - half, ic + half):          # right edge, +y
        path.append((i, jc + half))
    for j in range(jc + half, jc - half, -1):      # top edge, -x
        path.append((ic + half, j))
    for i in range(ic + half, ic - half, -1):      # left edge, -y
        path.append((i, jc - half))
    v = np.array([comp[i, j] for i, j in path])
    if np.any(np.abs(v) == 0):
        raise ValueError("the component vanishes on the loop")
    steps = np.angle(np.roll(v, -1) / v)
    return int(np.rint(steps.sum() / (2 * np.pi)))


def _write(path: str, cols) -> None:
    np.savetxt(path, np.column_stack(cols), fmt="%.10e")


def write_density(path: str, psi: np.ndarray, dx: float, dy: float | None = None) -> None:
    """Columns x (and y in 2D), rho_+1, rho_0, rho_-1, rho: one line per grid
    point, x fastest."""
    psi = np.asarray(psi)
    rho = density(psi)
    if psi.ndim == 2:
        _write(path, [coords(psi.shape[1], dx), *rho])
        return
    _, ny, nx = psi.shape
    X, Y = np.meshgrid(coords(nx, dx), coords(ny, dy))
    _write(path, [X.ravel(), Y.ravel(), *(c.ravel() for c in rho)])


def write_radial_density(path: str, psi: np.ndarray, dx: float, dy: float) -> None:
    """Columns r, rho_+1, rho_0, rho_-1, rho (annulus averages, 2D only)."""
    r, rho = radial_density(psi, dx, dy)
    _write(path, [r, *rho])


def write_phase(path: str, psi: np.ndarray, dx: float, dy: float) -> None:
    """Columns x, y and the phases of the three components (2D only)."""
    psi = np.asarray(psi)
    if psi.ndim != 3:
        raise ValueError("write_phase needs a 2D state of shape (3, ny, nx)")
    _, ny, nx = psi.shape
    X, Y = np.meshgrid(coords(nx, dx), coords(ny, dy))
    ph = phase(psi)
    _write(path, [X.ravel(), Y.ravel(), *(c.ravel() for c in ph)])
