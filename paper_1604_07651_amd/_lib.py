"""ctypes declarations of the C ABI in include/hrt.h (argument marshalling
only; every step of the transform runs in libhrt.so)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhrt.so")


class HrtDesc(C.Structure):
    _fields_ = [("nt", C.c_int32), ("nx", C.c_int32),
                ("dt", C.c_double), ("x0", C.c_double), ("dx", C.c_double),
                ("ntau", C.c_int32), ("nq", C.c_int32),
                ("tau0", C.c_double), ("dtau", C.c_double),
                ("q0", C.c_double), ("dq", C.c_double),
                ("oversample", C.c_double), ("flags", C.c_int32)]


class HrtInfo(C.Structure):
    _fields_ = [("T", C.c_double), ("X", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("a", C.c_double),
                ("O1", C.c_double), ("O2", C.c_double), ("a_r", C.c_double),
                ("dtheta0", C.c_double), ("drho0", C.c_double),
                ("dtheta", C.c_double), ("drho", C.c_double),
                ("beta_k", C.c_double),
                ("m_theta", C.c_int32), ("m_rho", C.c_int32),
                ("k1_kept", C.c_int32), ("k2_kept", C.c_int32),
                ("row_lo", C.c_int32), ("row_hi", C.c_int32),
                ("band_rows", C.c_int32), ("n_bands", C.c_int32),
                ("n_kept", C.c_int64), ("workspace_bytes", C.c_int64),
                ("alg_bytes_fwd", C.c_double), ("alg_bytes_adj", C.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("hrt_plan_describe", C.c_int, [C.POINTER(HrtDesc), C.POINTER(HrtInfo)]),
    ("hrt_plan_create", C.c_int, [C.POINTER(HrtDesc), C.POINTER(C.c_void_p)]),
    ("hrt_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_adjoint", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_normal", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_forward_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_direct_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_direct_adjoint", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_query", C.c_int, [C.c_void_p, C.POINTER(HrtInfo)]),
    ("hrt_plan_kernel", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hrt_profile_begin", C.c_int, [C.c_void_p, C.c_int32]),
    ("hrt_profile_end", C.c_int, [C.c_void_p, C.POINTER(C.c_double),
                                  C.POINTER(C.c_int64)]),
    ("hrt_ista_iterate", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                   C.c_float, C.c_void_p]),
    ("hrt_ista_graph_create", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                        C.c_float, C.POINTER(C.c_void_p)]),
    ("hrt_graph_launch", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hrt_graph_destroy", None, [C.c_void_p]),
    ("hrt_opnorm2", C.c_int, [C.c_void_p, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    ("hrt_demultiple", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_batch_create", C.c_int, [C.POINTER(HrtDesc), C.c_int32, C.POINTER(C.c_void_p)]),
    ("hrt_batch_offsets", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("hrt_batch_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_batch_adjoint", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_batch_plan", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    ("hrt_batch_destroy", None, [C.c_void_p]),
    ("hrt_batch_ista_iterate", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_int32,
                                         C.POINTER(C.c_float), C.POINTER(C.c_float),
                                         C.c_void_p]),
    ("hrt_batch_ista_graph_create", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_void_p, C.c_int32,
                                              C.POINTER(C.c_float), C.POINTER(C.c_float),
                                              C.POINTER(C.c_void_p)]),
    ("hrt_split_describe", C.c_int, [C.POINTER(HrtDesc), C.c_int32, C.POINTER(C.c_int32),
                                     C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                     C.POINTER(HrtDesc), C.POINTER(C.c_int32),
                                     C.POINTER(HrtInfo)]),
    ("hrt_split_create", C.c_int, [C.POINTER(HrtDesc), C.c_int32, C.POINTER(C.c_int32),
                                   C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_void_p)]),
    ("hrt_split_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_split_adjoint", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hrt_split_query", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(HrtInfo)]),
    ("hrt_split_destroy", None, [C.c_void_p]),
    ("hrt_plan_destroy", None, [C.c_void_p]),
    ("hrt_status_string", C.c_char_p, [C.c_int]),
    ("hrt_last_error", C.c_char_p, []),
]

_lib = None


class HrtError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


def load() -> C.CDLL:
    """Load libhrt.so (built by paper_1604_07651_amd.build); raises if it is
    missing - there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1604_07651_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int, where: str) -> None:
    if status != 0:
        lib = load()
        detail = lib.hrt_last_error().decode()
        raise HrtError(status, where, detail or lib.hrt_status_string(status).decode())


# kernel-variant bits of hrt_desc.flags (HRT_TUNE_* in hrt.h)
TUNE_ROW_RADIX8 = 1
TUNE_COL_RADIX8 = 2
TUNE_COL_PAIRS = 4
TUNE_BAND4 = 8
TUNE_BAND2 = 16
TUNE_SPREAD_HALF = 32
TUNE_GATHER_DOUBLE = 64


def make_desc(d, flags: int = 0) -> HrtDesc:
    """HrtDesc from any object with the grid attributes (nt, nx, dt, x0, dx,
    ntau, nq, tau0, dtau, q0, dq, oversample)."""
    return HrtDesc(nt=int(d.nt), nx=int(d.nx), dt=float(d.dt), x0=float(d.x0),
                   dx=float(d.dx), ntau=int(d.ntau), nq=int(d.nq),
                   tau0=float(d.tau0), dtau=float(d.dtau), q0=float(d.q0),
                   dq=float(d.dq), oversample=float(getattr(d, "oversample", 2.0)),
                   flags=int(flags))
