"""The allocation-free observables entry point (ssgp_observables_noalloc)
against ssgp_observables of a grid holding the same state, through the C ABI:
two calls in a row on one GPU, the second on a smaller grid, in 2D and 1D,
complex128 and complex64.  Relative 1e-10 (absolute 1e-12 below 1e-2)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2009_13507_amd import _lib, api  # noqa: E402
from paper_2009_13507_amd import workloads as W  # noqa: E402

KEYS = ("N+1", "N0", "N-1", "N", "M", "E", "E_kin", "E_trap", "E_c0", "E_c2", "E_rabi", "E_so",
        "rms+1", "rms0", "rms-1", "rms")


def noalloc(t, dim, nx, ny, dx, dy, prm):
    lib = _lib.load()
    o = _lib.Obs()
    code = _lib.C128 if t.dtype == torch.complex128 else _lib.C64
    rc = lib.ssgp_observables_noalloc(dim, nx, ny, dx, dy, code, ctypes.c_void_p(t.data_ptr()),
                                      ctypes.byref(prm), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                      ctypes.byref(o))
    _lib.check(rc)
    return o.as_dict()


def via_grid(t, dx, dy, **p):
    g = api.Grid(t, dx, dy)
    g.set_params(**p)
    o = g.observables()
    g.close()
    return o


def agree(a, b):
    for k in KEYS:
        if abs(b[k]) < 1e-2:
            assert abs(a[k] - b[k]) < 1e-12, (k, a[k], b[k])
        else:
            assert abs(a[k] - b[k]) < 1e-10 * abs(b[k]), (k, a[k], b[k])


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_observables_match_grid_observables(dtype):
    p = dict(c0=3.0, c2=-0.4, gamma=0.7, omega=0.3, dt=1e-3, so=api.SO_RASHBA)
    prm = api.params(**p)
    # first call: 2D 1024 x 1000 (the observables pass at its largest block count)
    for nx, ny, dx, seed in ((1024, 1000, 0.05, 1), (70, 90, 0.25, 2)):
        g0 = W.gaussian(2, nx, ny, dx, dx, phases=(0.3, 1.1, 2.0), width=1.5)
        psi = g0 * (1 + W.random_state(g0.shape, seed, 0.05))
        t = torch.from_numpy(psi).to("cuda:0").to(dtype)
        got = noalloc(t, 2, nx, ny, dx, dx, prm)
        want = via_grid(t, dx, dx, **p)
        agree(got, want)
    # then 1D, smaller again
    p1 = dict(c0=3.0, c2=-0.4, gamma=0.7, omega=0.3, dt=1e-3, so=api.SO_PX_SY)
    g1 = W.gaussian(1, 300, 1, 0.1, 0.1, phases=(0.3, 1.1, 2.0), width=1.5)
    t1 = torch.from_numpy(g1).to("cuda:0").to(dtype)
    agree(noalloc(t1, 1, 300, 1, 0.1, 0.1, api.params(**p1)), via_grid(t1, 0.1, None, **p1))


def test_noalloc_rejects_bad_arguments():
    lib = _lib.load()
    t = torch.zeros((3, 8, 8), dtype=torch.complex128, device="cuda:0")
    o = _lib.Obs()
    prm = api.params(dt=1e-3)
    ptr = ctypes.c_void_p(t.data_ptr())
    assert lib.ssgp_observables_noalloc(2, 4096, 8, 0.1, 0.1, 0, ptr, ctypes.byref(prm), None,
                                        ctypes.byref(o)) == _lib.EINVAL
    assert b"2048" in lib.ssgp_last_error()
    bad = api.params(dt=-1.0)
    assert lib.ssgp_observables_noalloc(2, 8, 8, 0.1, 0.1, 0, ptr, ctypes.byref(bad), None,
                                        ctypes.byref(o)) == _lib.EINVAL
    assert lib.ssgp_observables_noalloc(2, 8, 8, 0.1, 0.1, 0, None, ctypes.byref(prm), None,
                                        ctypes.byref(o)) == _lib.EINVAL
