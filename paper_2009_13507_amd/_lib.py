"""ctypes declarations of the C ABI in include/ssgp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssgp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ssgp.h")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENONFINITE = 0, -1, -2, -3, -4, -5
C128, C64 = 0, 1


class Params(ctypes.Structure):
    _fields_ = [("c0", ctypes.c_double), ("c2", ctypes.c_double), ("gamma", ctypes.c_double),
                ("omega", ctypes.c_double), ("kappa", ctypes.c_double), ("dt", ctypes.c_double),
                ("mag0", ctypes.c_double), ("so", ctypes.c_int), ("renorm", ctypes.c_int)]


class Obs(ctypes.Structure):
    _fields_ = [("N", ctypes.c_double * 3), ("Ntot", ctypes.c_double), ("M", ctypes.c_double),
                ("E", ctypes.c_double), ("E_parts", ctypes.c_double * 6), ("rms", ctypes.c_double * 3),
                ("rms_tot", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {"N+1": self.N[0], "N0": self.N[1], "N-1": self.N[2], "N": self.Ntot, "M": self.M,
             "E": self.E, "rms+1": self.rms[0], "rms0": self.rms[1], "rms-1": self.rms[2],
             "rms": self.rms_tot}
        for name, v in zip(("E_kin", "E_trap", "E_c0", "E_c2", "E_rabi", "E_so"), self.E_parts):
            d[name] = v
        return d


class SSGPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ssgp error {code}: {msg}")
        self.code = code


_lib = None


def exported_names():
    """Every function the public header declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_ ]+\*?\s*\*?(ssgp_[a-z0-9_]+)\s*\(", text, re.M)))


def load():
    """Loads libssgp.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the HIP path has no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, ci, cd, cll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    G = ctypes.c_void_p
    sig = {
        "ssgp_create_grid": ([ci, ci, ci, cd, cd, ci, vp, vp, ctypes.POINTER(G)], ci),
        "ssgp_set_state": ([G, vp], ci),
        "ssgp_set_params": ([G, ctypes.POINTER(Params)], ci),
        "ssgp_set_scheme": ([G, ci], ci),
        "ssgp_set_renorm_real": ([G, ci], ci),
        "ssgp_set_omega_schedule": ([G, ctypes.POINTER(cd), ci, ci], ci),
        "ssgp_set_step_index": ([G, cll], ci),
        "ssgp_get_step_index": ([G], cll),
        "ssgp_step_imag": ([G, ci], ci),
        "ssgp_step_real": ([G, ci], ci),
        "ssgp_step_real_seq": ([G, vp, vp, ci], ci),
        "ssgp_observables": ([G, ctypes.POINTER(Obs)], ci),
        "ssgp_obs_log_reserve": ([G, ci], ci),
        "ssgp_obs_record": ([G], ci),
        "ssgp_obs_log_read": ([G, ctypes.POINTER(Obs), ci, ctypes.POINTER(ci)], ci),
        "ssgp_observables_noalloc": ([ci, ci, ci, cd, cd, ci, vp, ctypes.POINTER(Params), vp,
                                      ctypes.POINTER(Obs)], ci),
        "ssgp_step_real_adjoint": ([G, vp, vp, ci], ci),
        "ssgp_omega_grad": ([G, ctypes.POINTER(cd), ci, ci], ci),
        "ssgp_destroy": ([G], ci),
        "ssgp_create_batch": ([ci, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(cd),
                               ctypes.POINTER(Params), ci, vp, ctypes.POINTER(cll), vp,
                               ctypes.POINTER(G)], ci),
        "ssgp_batch_step_imag": ([G, ci], ci),
        "ssgp_batch_step_imag_serial": ([G, ci], ci),
        "ssgp_batch_set_shape": ([G, ci], ci),
        "ssgp_batch_info": ([G, ctypes.POINTER(cd)], ci),
        "ssgp_batch_sync": ([G], ci),
        "ssgp_batch_observables": ([G, ctypes.POINTER(Obs)], ci),
        "ssgp_destroy_batch": ([G], ci),
        "ssgp_profile": ([G, ci, ci], ci),
        "ssgp_profile_read": ([G, ctypes.POINTER(cd)], ci),
        "ssgp_last_error": ([], ctypes.c_char_p),
        "ssgp_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(rc: int):
    if rc != OK:
        raise SSGPError(rc, load().ssgp_last_error().decode())
    return rc
