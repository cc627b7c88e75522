"""Python front-end of the MI355X SS-CN stepper (thin layer over the C ABI).

PyTorch provides the device memory and the stream; every step runs in the
HIP kernels of libssgp.so.  States are torch tensors of shape (3, ny, nx)
(2D) or (3, nx) (1D), dtype complex128 or complex64, contiguous, on a HIP
device, component order (+1, 0, -1).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import Obs, Params, SSGPError, check

SO_NONE, SO_PX_SX, SO_PX_SY, SO_PX_SZ, SO_RASHBA, SO_DRESSELHAUS, SO_ERD = range(7)
RENORM_AUTO, RENORM_NORM, RENORM_FIXED_M = range(3)
# PAPER: the paper's splitting; UNITARY_SO (opt-in): the SO term by
# Crank-Nicolson together with the x kinetic term (the p_x Sigma forms)
SCHEME_PAPER, SCHEME_UNITARY_SO, SCHEME_STRANG = range(3)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return _lib.C128
    if t.dtype == torch.complex64:
        return _lib.C64
    raise TypeError(f"state dtype must be complex128 or complex64, got {t.dtype}")


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def params(c0=0.0, c2=0.0, gamma=0.0, omega=0.0, dt=1e-3, so=SO_NONE, renorm=RENORM_AUTO,
           mag0=0.0, kappa=1.0) -> Params:
    return Params(float(c0), float(c2), float(gamma), float(omega), float(kappa), float(dt),
                  float(mag0), int(so), int(renorm))


class Grid:
    """A grid bound to one state tensor (borrowed, must stay alive)."""

    def __init__(self, psi: torch.Tensor, dx: float, dy: float | None = None, stream=None):
        lib = _lib.load()
        if not psi.is_cuda:
            raise ValueError("the state must live on a HIP device")
        if not psi.is_contiguous():
            raise ValueError("the state must be contiguous")
        if psi.dim() == 2 and psi.shape[0] == 3:
            self.dim, self.ny, self.nx = 1, 1, psi.shape[1]
        elif psi.dim() == 3 and psi.shape[0] == 3:
            self.dim, self.ny, self.nx = 2, psi.shape[1], psi.shape[2]
        else:
            raise ValueError(f"state shape must be (3, nx) or (3, ny, nx), got {tuple(psi.shape)}")
        self.dx = float(dx)
        self.dy = float(dy if dy is not None else dx)
        self.dtype = psi.dtype
        self.psi = psi
        self._stream = stream
        h = ctypes.c_void_p()
        check(lib.ssgp_create_grid(self.dim, self.nx, self.ny, self.dx, self.dy, _dtype_code(psi),
                                   _ptr(psi), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.nseg = 1

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.ssgp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_state(self, t: torch.Tensor, count: int = 1):
        if t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError("state tensor must match the grid's dtype, be on the device and contiguous")
        if t.numel() != count * 3 * self.nx * self.ny:
            raise ValueError(f"expected {count} state(s) of {3 * self.nx * self.ny} elements, got {t.numel()}")

    def bind(self, psi: torch.Tensor):
        self._check_state(psi)
        check(self._lib.ssgp_set_state(self._h, _ptr(psi)))
        self.psi = psi

    def set_params(self, p: Params | None = None, **kw):
        p = p if p is not None else params(**kw)
        check(self._lib.ssgp_set_params(self._h, ctypes.byref(p)))
        self.p = p

    def set_scheme(self, scheme: int):
        check(self._lib.ssgp_set_scheme(self._h, int(scheme)))

    def set_renorm_real(self, on: bool):
        """RENORM after every real-time step too (off by default)."""
        check(self._lib.ssgp_set_renorm_real(self._h, 1 if on else 0))

    def set_omega_schedule(self, omega, steps_per_seg: int):
        arr = (ctypes.c_double * len(omega))(*[float(v) for v in omega])
        check(self._lib.ssgp_set_omega_schedule(self._h, arr, len(omega), int(steps_per_seg)))
        self.nseg = max(1, len(omega))

    @property
    def step_index(self) -> int:
        return int(self._lib.ssgp_get_step_index(self._h))

    @step_index.setter
    def step_index(self, n: int):
        check(self._lib.ssgp_set_step_index(self._h, int(n)))

    def step_imag(self, n: int):
        check(self._lib.ssgp_step_imag(self._h, int(n)))

    def step_real(self, n: int):
        check(self._lib.ssgp_step_real(self._h, int(n)))

    def step_real_seq(self, src: torch.Tensor, dst: torch.Tensor, n: int):
        """n real-time steps from src; the state after step k goes to dst[k-1]."""
        self._check_state(src)
        self._check_state(dst, n)
        check(self._lib.ssgp_step_real_seq(self._h, _ptr(src), _ptr(dst), int(n)))

    def step_real_adjoint(self, states: torch.Tensor, lam: torch.Tensor, n: int):
        self._check_state(states, n)
        self._check_state(lam)
        check(self._lib.ssgp_step_real_adjoint(self._h, _ptr(states), _ptr(lam), int(n)))

    def omega_grad(self, reset: bool = True):
        out = (ctypes.c_double * self.nseg)()
        check(self._lib.ssgp_omega_grad(self._h, out, self.nseg, 1 if reset else 0))
        return [out[i] for i in range(self.nseg)]

    def profile(self, every: int, capacity: int = 4096):
        """Records HIP events around the x- and y-pass of every every-th step."""
        check(self._lib.ssgp_profile(self._h, int(every), int(capacity)))

    def profile_read(self) -> dict:
        out = (ctypes.c_double * 5)()
        check(self._lib.ssgp_profile_read(self._h, out))
        return {"steps": int(out[0]), "x_ms": out[1], "y_ms": out[2], "x_ms_min": out[3], "y_ms_min": out[4]}

    def observables(self) -> dict:
        o = Obs()
        rc = self._lib.ssgp_observables(self._h, ctypes.byref(o))
        if rc not in (_lib.OK,):
            raise SSGPError(rc, self._lib.ssgp_last_error().decode())
        return o.as_dict()

    def obs_log_reserve(self, capacity: int):
        """Device-side log of up to ``capacity`` observable samples (cleared)."""
        check(self._lib.ssgp_obs_log_reserve(self._h, int(capacity)))

    def obs_record(self):
        """Appends the observables of the current state to the device log,
        asynchronously (no host synchronisation)."""
        check(self._lib.ssgp_obs_record(self._h))

    def obs_log_read(self) -> list:
        """Synchronises and returns the logged samples, oldest first."""
        count = ctypes.c_int(0)
        check(self._lib.ssgp_obs_log_read(self._h, None, 0, ctypes.byref(count)))
        out = (Obs * max(1, count.value))()
        rc = self._lib.ssgp_obs_log_read(self._h, out, count.value, ctypes.byref(count))
        if rc != _lib.OK:
            raise SSGPError(rc, self._lib.ssgp_last_error().decode())
        return [out[k].as_dict() for k in range(count.value)]


class Batch:
    """n independent 2D grids in one device pool, stepped together in
    imaginary time (one persistent kernel, or one launch per sweep, replayed
    from HIP graphs).  Instance i is the (3, ny_i, nx_i) view ``views[i]`` of
    the pool."""

    ALIGN = 32  # elements between instance starts are rounded up to this

    def __init__(self, pool: torch.Tensor, shapes, dxs, params_list, offsets=None, stream=None):
        lib = _lib.load()
        if not pool.is_cuda or not pool.is_contiguous() or pool.dim() != 1:
            raise ValueError("the pool must be a contiguous 1D device tensor")
        n = len(shapes)
        if not (len(dxs) == len(params_list) == n):
            raise ValueError("shapes, dxs and params_list must have one entry per instance")
        if offsets is None:
            offsets = self.packed_offsets(shapes)
        self.shapes = [(int(ny), int(nx)) for ny, nx in shapes]
        self.offsets = [int(o) for o in offsets]
        self.pool = pool
        self.dtype = pool.dtype
        nxs = (ctypes.c_int * n)(*[nx for _, nx in self.shapes])
        nys = (ctypes.c_int * n)(*[ny for ny, _ in self.shapes])
        dxa = (ctypes.c_double * n)(*[float(d) for d in dxs])
        pa = (Params * n)(*params_list)
        offa = (ctypes.c_longlong * n)(*self.offsets)
        h = ctypes.c_void_p()
        check(lib.ssgp_create_batch(n, nxs, nys, dxa, pa, _dtype_code(pool), _ptr(pool), offa,
                                    _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.n = n

    @classmethod
    def packed_offsets(cls, shapes):
        offs, at = [], 0
        for ny, nx in shapes:
            offs.append(at)
            at += -(-3 * ny * nx // cls.ALIGN) * cls.ALIGN
        return offs

    @classmethod
    def from_states(cls, states, dxs, params_list, dtype=torch.complex128, device="cuda:0", stream=None):
        """Packs (3, ny, nx) states into a new pool on the device."""
        shapes = [tuple(s.shape[1:]) for s in states]
        offs = cls.packed_offsets(shapes)
        total = offs[-1] + 3 * shapes[-1][0] * shapes[-1][1]
        pool = torch.zeros(total, dtype=dtype, device=device)
        b = cls(pool, shapes, dxs, params_list, offs, stream)
        for v, s in zip(b.views(), states):
            v.copy_(torch.as_tensor(s).to(device=device, dtype=dtype))
        return b

    def views(self):
        return [self.pool[o:o + 3 * ny * nx].view(3, ny, nx) for o, (ny, nx) in zip(self.offsets, self.shapes)]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.ssgp_destroy_batch(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step_imag(self, n: int):
        check(self._lib.ssgp_batch_step_imag(self._h, int(n)))

    def step_imag_serial(self, n: int):
        check(self._lib.ssgp_batch_step_imag_serial(self._h, int(n)))

    def set_shape(self, shape: int):
        """k > 0: persistent kernel, k workgroups per compute unit; -1: one
        launch per sweep; 0: autotune at the next step call.  (-2 and -4, the
        grids in groups on streams of their own, are switched off: the
        library refuses them.)"""
        check(self._lib.ssgp_batch_set_shape(self._h, int(shape)))

    def info(self) -> dict:
        out = (ctypes.c_double * 6)()
        check(self._lib.ssgp_batch_info(self._h, out))
        return {"shape": int(out[0]), "grid": int(out[1]), "max_per_cu": int(out[2]), "us_per_step": out[3],
                "x_items": int(out[4]), "y_items": int(out[5])}

    def sync(self):
        check(self._lib.ssgp_batch_sync(self._h))

    def observables(self):
        obs = (Obs * self.n)()
        rc = self._lib.ssgp_batch_observables(self._h, obs)
        if rc != _lib.OK:
            raise SSGPError(rc, self._lib.ssgp_last_error().decode())
        return [o.as_dict() for o in obs]


def version() -> str:
    return _lib.load().ssgp_version().decode()
