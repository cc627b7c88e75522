"""ctypes front-end of the FP64 CPU oracle (``ssgp_oracle.c``).

TEST INFRASTRUCTURE.  The oracle is the plain, slow reference that the HIP
path is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product package never
does.  It shares no code with the GPU library.

Every array is numpy ``complex128`` of shape ``(3, ny, nx)`` (2D) or
``(3, nx)`` (1D), C-contiguous, component order (+1, 0, -1), x fastest.
Functions that change a state return a new array (the input is copied).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssgp_oracle.c")
_LIB = os.path.join(_HERE, "libssgp_oracle.so")

SO_NONE, SO_PX_SX, SO_PX_SY, SO_PX_SZ, SO_RASHBA, SO_DRESSELHAUS, SO_ERD = range(7)
RENORM_AUTO, RENORM_NORM, RENORM_FIXED_M = range(3)

OBS_NAMES = ("N+1", "N0", "N-1", "N", "M", "E", "E_kin", "E_trap", "E_c0", "E_c2",
             "E_rabi", "E_so", "rms+1", "rms0", "rms-1", "rms")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP over grid lines)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("c0", ctypes.c_double), ("c2", ctypes.c_double),
                ("gamma", ctypes.c_double), ("omega", ctypes.c_double),
                ("kappa", ctypes.c_double), ("dt", ctypes.c_double),
                ("imag", ctypes.c_int), ("so", ctypes.c_int), ("renorm", ctypes.c_int),
                ("mag0", ctypes.c_double)]


@dataclass
class Cfg:
    """Grid and model parameters of one run (Table 2 of the paper)."""
    dim: int
    nx: int
    ny: int = 1
    dx: float = 0.1
    dy: float = 0.1
    c0: float = 0.0
    c2: float = 0.0
    gamma: float = 0.0
    omega: float = 0.0
    dt: float = 1e-3
    imag: bool = True
    so: int = SO_NONE
    renorm: int = RENORM_AUTO
    mag0: float = 0.0
    kappa: float = 1.0

    def c(self) -> _Cfg:
        return _Cfg(self.dim, self.nx, self.ny if self.dim == 2 else 1, self.dx, self.dy,
                    self.c0, self.c2, self.gamma, self.omega, self.kappa, self.dt,
                    1 if self.imag else 0, self.so, self.renorm, self.mag0)

    def shape(self):
        return (3, self.ny, self.nx) if self.dim == 2 else (3, self.nx)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Cfg)
        vp = ctypes.c_void_p
        for name in ("ora_calcnu", "ora_herm", "ora_so", "ora_cn_x", "ora_cn_y",
                     "ora_pointwise_dual_value", "ora_cn_x_adjoint", "ora_cn_y_adjoint"):
            getattr(L, name).argtypes = [P, vp]
            getattr(L, name).restype = None
        L.ora_pointwise2.argtypes = [P, vp, ctypes.c_double]
        L.ora_pointwise2.restype = None
        L.ora_step.argtypes = [P, vp, ctypes.c_long]
        L.ora_step.restype = None
        L.ora_renorm.argtypes = [P, vp]
        L.ora_renorm.restype = ctypes.c_int
        L.ora_norms.argtypes = [P, vp, vp]
        L.ora_norms.restype = None
        L.ora_renorm_factors.argtypes = [P, vp, vp]
        L.ora_renorm_factors.restype = ctypes.c_int
        L.ora_uses_fixed_m.argtypes = [P]
        L.ora_uses_fixed_m.restype = ctypes.c_int
        L.ora_observables.argtypes = [P, vp, vp]
        L.ora_observables.restype = None
        L.ora_apply_hso.argtypes = [P, vp, vp]
        L.ora_apply_hso.restype = None
        L.ora_step_adjoint.argtypes = [P, vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.ora_step_adjoint.restype = ctypes.c_int
        L.ora_num_threads.argtypes = []
        L.ora_num_threads.restype = ctypes.c_int
        L.ora_set_num_threads.argtypes = [ctypes.c_int]
        L.ora_set_num_threads.restype = None
        _lib = L
    return _lib


def _arr(cfg: Cfg, psi) -> np.ndarray:
    a = np.array(psi, dtype=np.complex128, order="C", copy=True)
    if a.shape != cfg.shape():
        raise ValueError(f"state shape {a.shape} != {cfg.shape()}")
    return a


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _sub(name):
    def f(cfg: Cfg, psi):
        a = _arr(cfg, psi)
        cc = cfg.c()
        getattr(lib(), name)(ctypes.byref(cc), _ptr(a))
        return a
    f.__name__ = name
    return f


calcnu = _sub("ora_calcnu")
herm = _sub("ora_herm")
so = _sub("ora_so")
cn_x = _sub("ora_cn_x")
cn_y = _sub("ora_cn_y")
cn_x_adjoint = _sub("ora_cn_x_adjoint")
cn_y_adjoint = _sub("ora_cn_y_adjoint")
pointwise_dual_value = _sub("ora_pointwise_dual_value")


def step(cfg: Cfg, psi, nsteps: int = 1) -> np.ndarray:
    """``nsteps`` full SS-CN steps (CALCNU, HERM, SO, LUX, LUY, RENORM)."""
    a = _arr(cfg, psi)
    cc = cfg.c()
    lib().ora_step(ctypes.byref(cc), _ptr(a), int(nsteps))
    return a


def renorm(cfg: Cfg, psi):
    a = _arr(cfg, psi)
    cc = cfg.c()
    fb = lib().ora_renorm(ctypes.byref(cc), _ptr(a))
    return a, fb


def norms(cfg: Cfg, psi) -> np.ndarray:
    a = _arr(cfg, psi)
    out = np.zeros(3)
    cc = cfg.c()
    lib().ora_norms(ctypes.byref(cc), _ptr(a), _ptr(out))
    return out


def renorm_factors(cfg: Cfg, N):
    n = np.ascontiguousarray(N, dtype=np.float64)
    d = np.zeros(3)
    cc = cfg.c()
    fb = lib().ora_renorm_factors(ctypes.byref(cc), _ptr(n), _ptr(d))
    return d, fb


def uses_fixed_m(cfg: Cfg) -> bool:
    cc = cfg.c()
    return bool(lib().ora_uses_fixed_m(ctypes.byref(cc)))


def observables(cfg: Cfg, psi) -> dict:
    a = _arr(cfg, psi)
    out = np.zeros(16)
    cc = cfg.c()
    lib().ora_observables(ctypes.byref(cc), _ptr(a), _ptr(out))
    return dict(zip(OBS_NAMES, out.tolist()))


def apply_hso(cfg: Cfg, psi) -> np.ndarray:
    a = _arr(cfg, psi)
    out = np.zeros_like(a)
    cc = cfg.c()
    lib().ora_apply_hso(ctypes.byref(cc), _ptr(a), _ptr(out))
    return out


def step_adjoint(cfg: Cfg, psi_n, lam):
    """One real-time step backwards: returns (dL/dpsi^n, dL/dOmega of this step)."""
    a = _arr(cfg, psi_n)
    l = _arr(cfg, lam)
    dom = ctypes.c_double(0.0)
    cc = cfg.c()
    rc = lib().ora_step_adjoint(ctypes.byref(cc), _ptr(a), _ptr(l), ctypes.byref(dom))
    if rc != 0:
        raise ValueError("adjoint is defined for real time only")
    return l, dom.value


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (timing only)."""
    lib().ora_set_num_threads(int(n))


# ------------------------------------------- unitary-SO scheme (opt-in) --
# Beyond the paper: the SO term of Eqs. (p1)-(p2) is taken by Crank-Nicolson
# together with LUX (Table 1), so a real-time step stays unitary for
# gamma != 0.  Written from the definition: for every x line,
#   (I + s H) psi' = (I - s H) psi,  H = I_3 (x) T + gamma S_a (x) (-i D),
# T = -1/2 d^2/dx^2 and D = d/dx by the three-point and central stencils with
# zero ghosts, S_a the spin-1 matrix of Eq. (3) of the p_x Sigma_a form (the
# equal mixture of Rashba and Dresselhaus couplings is -gamma p_x Sigma_y), and
# s = i dt/2 in real time, dt/2 in imaginary time (Delta -> -i Delta).  The
# line vector is component-major (psi_{+1}(x_0..), psi_0(..), psi_{-1}(..)).

SCHEME_PAPER, SCHEME_UNITARY_SO = range(2)

_S2 = np.sqrt(2.0)
_SPIN = {  # Eq. (3)
    SO_PX_SX: np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=complex) / _S2,
    SO_PX_SY: 1j * np.array([[0, -1, 0], [1, 0, -1], [0, 1, 0]], dtype=complex) / _S2,
    SO_PX_SZ: np.diag([1.0, 0.0, -1.0]).astype(complex),
}


def _line_hamiltonian(cfg: Cfg):
    """H of one x line (sparse, 3 nx x 3 nx) for the x-derivative SO forms."""
    import scipy.sparse as sp
    n, h = cfg.nx, cfg.dx
    T = sp.diags([np.full(n - 1, -0.5 / h ** 2), np.full(n, 1.0 / h ** 2), np.full(n - 1, -0.5 / h ** 2)],
                 [-1, 0, 1])
    D = sp.diags([np.full(n - 1, -0.5 / h), np.full(n - 1, 0.5 / h)], [-1, 1])
    H = sp.kron(sp.identity(3), T)
    if cfg.so != SO_NONE and cfg.gamma != 0.0:
        if cfg.so == SO_ERD:      # gamma (0 p_y Sigma_x - p_x Sigma_y): x derivatives only
            M = -cfg.gamma * _SPIN[SO_PX_SY]
        elif cfg.so in _SPIN:
            M = cfg.gamma * _SPIN[cfg.so]
        else:
            raise ValueError("the unitary-SO scheme takes the forms without y derivatives")
        H = H + sp.kron(M, -1j * D)
    return sp.csc_matrix(H, dtype=complex)


def cn_x_so(cfg: Cfg, psi) -> np.ndarray:
    """LUX and the SO sub-step in one Crank-Nicolson solve of every x line."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    a = _arr(cfg, psi)
    s = 0.5 * cfg.dt if cfg.imag else 0.5j * cfg.dt
    H = _line_hamiltonian(cfg)
    I = sp.identity(3 * cfg.nx, dtype=complex, format="csc")
    lu = spl.splu(sp.csc_matrix(I + s * H))
    B = sp.csr_matrix(I - s * H)
    rows = a.reshape(3, -1, cfg.nx)                   # (3, lines, nx)
    lines = rows.transpose(1, 0, 2).reshape(-1, 3 * cfg.nx)
    out = lu.solve(np.ascontiguousarray((B @ lines.T)))
    a[...] = out.T.reshape(-1, 3, cfg.nx).transpose(1, 0, 2).reshape(a.shape)
    return a


def step_unitary_so(cfg: Cfg, psi, nsteps: int = 1) -> np.ndarray:
    """nsteps steps of the unitary-SO scheme: CALCNU, HERM, the joined
    LUX + SO solve, LUY (2D), and RENORM in imaginary time."""
    a = _arr(cfg, psi)
    for _ in range(int(nsteps)):
        a = herm(cfg, calcnu(cfg, a))
        a = cn_x_so(cfg, a)
        if cfg.dim == 2:
            a = cn_y(cfg, a)
        if cfg.imag:
            a, _ = renorm(cfg, a)
    return a



# -------------------------------------------- RENORM in real time (opt-in) --
# App. A keeps the norm (and, under Eq. (DJ), the magnetisation) by rescaling
# the components after each time step of the propagation; the sample real-time
# output of Sec. 3 holds its energy constant over 90,000 steps, as it does when
# the rule is applied after every real-time step too.  The plain step above
# renormalises in imaginary time only.

def step_real_renorm(cfg: Cfg, psi, nsteps: int = 1, unitary_so: bool = False) -> np.ndarray:
    """nsteps real-time steps (the paper's scheme, or the unitary-SO one),
    each followed by the RENORM rule of Eqs. (DJ)/(DJ2)."""
    if cfg.imag:
        raise ValueError("real time only")
    a = _arr(cfg, psi)
    for _ in range(int(nsteps)):
        a = step_unitary_so(cfg, a, 1) if unitary_so else step(cfg, a, 1)
        a, _ = renorm(cfg, a)
    return a


# ------------------------------------------- Strang scheme (opt-in) -------
# Beyond the paper: a second-order splitting.  One step of size dt is
#   P2(dt/2), then K(dt), then P2(dt/2), then RENORM in imaginary time,
# where K is the joined LUX + SO Crank-Nicolson solve of every x line (as in
# the unitary-SO scheme, the x-derivative SO forms) followed by LUY (2D): both
# are Cayley transforms, second order, and they commute (the SO term has no y
# derivative).  P2(tau) is the pointwise stage of ``ora_pointwise2``: CALCNU
# and HERM with their coefficients taken at a predicted midpoint state, the
# exponentials in the symmetric order, which makes it second order for c2 != 0
# where the paper's frozen-coefficient CALCNU + HERM are first order.

SCHEME_STRANG = 2


def pointwise2(cfg: Cfg, psi, tau: float) -> np.ndarray:
    """The second-order pointwise stage over tau (see ora_pointwise2)."""
    a = _arr(cfg, psi)
    cc = cfg.c()
    lib().ora_pointwise2(ctypes.byref(cc), _ptr(a), float(tau))
    return a


def step_strang(cfg: Cfg, psi, nsteps: int = 1) -> np.ndarray:
    """nsteps steps of the Strang scheme (RENORM after each in imaginary time)."""
    a = _arr(cfg, psi)
    for _ in range(int(nsteps)):
        a = pointwise2(cfg, a, 0.5 * cfg.dt)
        a = cn_x_so(cfg, a)
        if cfg.dim == 2:
            a = cn_y(cfg, a)
        a = pointwise2(cfg, a, 0.5 * cfg.dt)
        if cfg.imag:
            a, _ = renorm(cfg, a)
    return a
