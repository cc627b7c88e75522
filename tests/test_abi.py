"""Host-side checks of the C ABI library (no GPU needed): it loads, it exports
every entry point the public header declares, and argument validation that
precedes any device call reports EINVAL with a message."""
import ctypes
import os
import subprocess

import pytest

from paper_2009_13507_amd import _lib


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libssgp.so is not built; run __graft_entry__.build()")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _lib.exported_names()
    for required in ("ssgp_create_grid", "ssgp_set_params", "ssgp_step_imag", "ssgp_step_real",
                     "ssgp_observables", "ssgp_step_real_adjoint", "ssgp_create_batch",
                     "ssgp_batch_step_imag", "ssgp_destroy", "ssgp_last_error", "ssgp_set_scheme",
                     "ssgp_set_renorm_real"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in _lib.exported_names():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_version(lib):
    assert b"gfx950" in lib.ssgp_version()


@pytest.mark.parametrize("args,fragment", [
    ((3, 16, 16, 0.1, 0.1, 0), b"dim"),
    ((2, 0, 16, 0.1, 0.1, 0), b"nx"),
    ((2, 2049, 16, 0.1, 0.1, 1), b"nx"),
    ((2, 2049, 16, 0.1, 0.1, 0), b"nx"),
    ((2, 16, 2049, 0.1, 0.1, 0), b"ny"),
    ((2, 16, 16, -0.1, 0.1, 0), b"spacing"),
    ((2, 16, 16, 0.1, 0.0, 0), b"spacing"),
    ((2, 16, 16, 0.1, 0.1, 7), b"dtype"),
])
def test_create_grid_rejects_bad_arguments(lib, args, fragment):
    h = ctypes.c_void_p(123)
    rc = lib.ssgp_create_grid(*args, ctypes.c_void_p(1), None, ctypes.byref(h))
    assert rc == _lib.EINVAL
    assert h.value is None
    assert fragment in lib.ssgp_last_error()


def test_null_arguments(lib):
    assert lib.ssgp_create_grid(2, 8, 8, 0.1, 0.1, 0, None, None, None) == _lib.EINVAL
    assert lib.ssgp_set_scheme(None, 1) == _lib.EINVAL
    assert lib.ssgp_set_renorm_real(None, 1) == _lib.EINVAL
    h = ctypes.c_void_p()
    assert lib.ssgp_create_grid(2, 8, 8, 0.1, 0.1, 0, None, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.ssgp_step_imag(None, 1) == _lib.EINVAL
    assert lib.ssgp_set_params(None, None) == _lib.EINVAL
    assert lib.ssgp_destroy(None) == _lib.OK


def _batch_args(n, nx, ny, offsets, so=1):
    ci, cd, cll = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    prm = (_lib.Params * n)(*[_lib.Params(2.0, -0.1, 0.5, 0.1, 1.0, 1e-3, 0.0, so, 0) for _ in range(n)])
    return ((ci * n)(*nx), (ci * n)(*ny), (cd * n)(*([0.1] * n)), prm, (cll * n)(*offsets))


@pytest.mark.parametrize("n,nx,ny,offsets,so,fragment", [
    (2, [16, 16], [16, 16], [0, 3 * 256 - 1], 1, b"overlap"),
    (2, [16, 16], [16, 16], [3 * 256, 0], 0, b"ok"),
    (1, [513], [16], [0], 1, b"512"),
    (1, [16], [0], [0], 1, b"512"),
    (1, [16], [16], [-1], 1, b"offset"),
    (1, [16], [16], [0], 4, b"y-dependent"),
])
def test_create_batch_rejects_bad_arguments(lib, n, nx, ny, offsets, so, fragment):
    if fragment == b"ok":
        pytest.skip("valid arguments reach the device")
    nxa, nya, dxa, prm, offa = _batch_args(n, nx, ny, offsets, so)
    h = ctypes.c_void_p(123)
    rc = lib.ssgp_create_batch(n, nxa, nya, dxa, prm, 0, ctypes.c_void_p(1), offa, None, ctypes.byref(h))
    assert rc == _lib.EINVAL
    assert h.value is None
    assert fragment in lib.ssgp_last_error()


def test_batch_null_arguments(lib):
    nxa, nya, dxa, prm, offa = _batch_args(1, [8], [8], [0])
    h = ctypes.c_void_p()
    assert lib.ssgp_create_batch(0, nxa, nya, dxa, prm, 0, ctypes.c_void_p(1), offa, None,
                                 ctypes.byref(h)) == _lib.EINVAL
    assert lib.ssgp_create_batch(1, nxa, nya, dxa, prm, 0, None, offa, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.ssgp_batch_step_imag(None, 1) == _lib.EINVAL
    assert lib.ssgp_batch_sync(None) == _lib.EINVAL
    assert lib.ssgp_batch_set_shape(None, 1) == _lib.EINVAL
    assert lib.ssgp_destroy_batch(None) == _lib.OK
