"""ctypes declarations of libdirac's C ABI (include/dirac.h).

Loading fails loudly when the shared library has not been built: there is
no fallback implementation anywhere in this package.
"""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdirac.so")

F64, F32, F16S, BF16S = 0, 1, 2, 3
LINK18, LINK12, LINK10 = 18, 12, 10
OK, EINVAL, EDEVICE, ENOCONV, EBREAKDOWN, EUNSUPPORTED, EWORKSPACE = 0, -1, -2, -3, -4, -5, -6

STATUS_NAMES = {
    OK: "DIRAC_OK", EINVAL: "DIRAC_EINVAL", EDEVICE: "DIRAC_EDEVICE", ENOCONV: "DIRAC_ENOCONV",
    EBREAKDOWN: "DIRAC_EBREAKDOWN", EUNSUPPORTED: "DIRAC_EUNSUPPORTED", EWORKSPACE: "DIRAC_EWORKSPACE",
}


class DiracOp(C.Structure):
    _fields_ = [("L", C.c_int32 * 4), ("prec", C.c_int32), ("link", C.c_int32),
                ("nrhs", C.c_int32), ("flags", C.c_int32), ("m_q", C.c_double)]


class DiracLaunch(C.Structure):
    _fields_ = [("block_sites", C.c_int32), ("rhs_per_thread", C.c_int32), ("xcd_remap", C.c_int32),
                ("nt_store", C.c_int32), ("lds", C.c_int32), ("tile_y", C.c_int32), ("tile_z", C.c_int32),
                ("t_chunk", C.c_int32), ("tuned", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CgParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("inner_prec", C.c_int32),
                ("inner_delta", C.c_double), ("inner_kmax", C.c_int32), ("check_every", C.c_int32),
                ("single_launch", C.c_int32), ("reserved", C.c_int32)]


class CgStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("outer", C.c_int32),
                ("dslash_hi", C.c_int32), ("dslash_lo", C.c_int32), ("fallback", C.c_int32),
                ("true_rel_res", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_OP = C.POINTER(DiracOp)

# name -> (restype, argtypes); every function of include/dirac.h
SIGNATURES = {
    "dirac_spinor_bytes": (C.c_int64, [_OP]),
    "dirac_gauge_bytes": (C.c_int64, [_OP]),
    "dirac_pack_gauge": (C.c_int, [_OP, _P, _P, _P]),
    "dirac_pack_spinor": (C.c_int, [_OP, _P, _P, _P]),
    "dirac_unpack_spinor": (C.c_int, [_OP, _P, _P, _P]),
    "dirac_convert_spinor": (C.c_int, [_OP, _P, _OP, _P, _P]),
    "dirac_apply": (C.c_int, [_OP, _P, _P, _P, _P]),
    "dirac_dagger_apply": (C.c_int, [_OP, _P, _P, _P, _P]),
    "dirac_mdagm_apply": (C.c_int, [_OP, _P, _P, _P, _P, _P]),
    "dirac_field_dot_workspace_bytes": (C.c_int64, [_OP]),
    "dirac_field_dot": (C.c_int, [_OP, _P, _P, _P, C.c_int64, C.POINTER(C.c_double), _P]),
    "dirac_field_dot_noalloc": (C.c_int, [_OP, _P, _P, C.POINTER(C.c_double), _P]),
    "dirac_field_axpy": (C.c_int, [_OP, C.c_double, C.c_double, _P, _P, _P]),
    "cg_workspace_bytes": (C.c_int64, [_OP, C.POINTER(CgParams)]),
    "cg_solve": (C.c_int, [_OP, _P, _P, _P, _P, _P, C.c_int64, C.POINTER(CgParams),
                           C.POINTER(CgStats), _P]),
    "dirac_schur_apply": (C.c_int, [_OP, _P, _P, _P, C.c_int32, _P]),
    "cg_workspace_bytes_eo": (C.c_int64, [_OP, C.POINTER(CgParams)]),
    "cg_solve_eo": (C.c_int, [_OP, _P, _P, _P, _P, _P, C.c_int64, C.POINTER(CgParams), C.c_int32,
                              C.POINTER(CgStats), _P]),
    "dirac_bandwidth_probe": (C.c_int, [C.c_int32, _P, _P, C.c_int64, _P]),
    "dirac_force": (C.c_int, [_OP, _P, _P, _P, C.c_double, C.c_int32, _P]),
    "dirac_multi_apply": (C.c_int, [C.c_int32, _OP, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P),
                                    C.c_int32, _P]),
    "dirac_multi_plan_create": (C.c_int, [C.c_int32, _OP, C.POINTER(_P), C.POINTER(_P),
                                          C.POINTER(_P), C.c_int32, _P, C.POINTER(_P)]),
    "dirac_plan_launch": (C.c_int, [_P, _P]),
    "dirac_plan_destroy": (C.c_int, [_P]),
    "dirac_autotune": (C.c_int, [_OP, _P, _P, _P, _P]),
    "dirac_launch_config": (C.c_int, [_OP, C.POINTER(DiracLaunch)]),
    "dirac_set_launch_config": (C.c_int, [_OP, C.POINTER(DiracLaunch)]),
    "dirac_last_error": (C.c_char_p, []),
    "dirac_version": (C.c_char_p, []),
}

_lib = None


def load():
    """The loaded library (ctypes.CDLL), with every signature declared."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libdirac.so not found at {LIB_PATH}: build it first "
            "(python -m paper_1904_08616_amd.build). "
            "There is no fallback implementation.")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DiracError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(rc, allow=()):
    """Raise DiracError for a negative status not in ``allow``."""
    if rc < 0 and rc not in allow:
        raise DiracError(int(rc), load().dirac_last_error().decode())
    return rc


def make_op(dims, prec=F64, link=LINK18, nrhs=1, m_q=0.0):
    op = DiracOp()
    for d in range(4):
        op.L[d] = int(dims[d])
    op.prec = int(prec)
    op.link = int(link)
    op.nrhs = int(nrhs)
    op.flags = 0
    op.m_q = float(m_q)
    return op
