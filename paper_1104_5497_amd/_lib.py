"""ctypes binding of libnphc.so (argument marshalling only).

Every function here forwards plain pointers and sizes to the C ABI declared in
include/nphc.h.  The library must have been built (paper_1104_5497_amd.build);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnphc.so")

NPHC_MAX_N = 13
NPHC_BATCH_MAX_N = 9
NPHC_OK, NPHC_EINVAL, NPHC_EUNSUPPORTED, NPHC_EHIP, NPHC_EWORKSPACE = 0, -1, -2, -3, -4
NPHC_FP64, NPHC_FP32 = 0, 1

PATH_PENDING, PATH_REACHED, PATH_DIVERGED, PATH_FAIL_MINSTEP = 0, 1, 2, 3
PATH_FAIL_MAXSTEPS, PATH_FAIL_NONFINITE, PATH_STALLED, PATH_HANDOFF = 4, 5, 6, 7
END_NONSINGULAR, END_SINGULAR, END_DIVERGED, END_FAIL, END_DUPLICATE = 10, 11, 12, 13, 14

EXPORTS = [
    "nphc_default_track_opts", "nphc_default_cert_opts", "nphc_default_class_opts",
    "nphc_track_workspace_size", "nphc_track_paths", "nphc_refine_certify",
    "nphc_mark_duplicates", "nphc_duplicates_workspace_size", "nphc_select",
    "nphc_select_list", "nphc_select_workspace_size", "nphc_classify",
    "nphc_adjoint", "nphc_strerror", "nphc_version",
]


class NphcError(RuntimeError):
    pass


class Batch_(ctypes.Structure):
    _fields_ = [("num_systems", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("N_host", ctypes.c_void_p), ("path_off_host", ctypes.c_void_p),
                ("N", ctypes.c_void_p), ("path_off", ctypes.c_void_p),
                ("J", ctypes.c_void_p), ("J_off", ctypes.c_void_p), ("gamma", ctypes.c_void_p)]


class TrackOpts_(ctypes.Structure):
    _fields_ = [("h0", ctypes.c_double), ("hmax", ctypes.c_double), ("hmin", ctypes.c_double),
                ("corr_tol", ctypes.c_double), ("R_inf", ctypes.c_double),
                ("t_stall", ctypes.c_double), ("t_end", ctypes.c_double),
                ("max_corr", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("predictor", ctypes.c_int32), ("resume", ctypes.c_int32),
                ("handoff_norm", ctypes.c_double), ("handoff_rejects", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("t_endzone", ctypes.c_double),
                ("hmin_rel", ctypes.c_double), ("collapse_norm", ctypes.c_double),
                ("grow_ratio", ctypes.c_double), ("grow_cap", ctypes.c_double),
                ("grid_blocks", ctypes.c_int32), ("handoff_steps", ctypes.c_int32),
                ("pred_tol", ctypes.c_double), ("step_ctrl", ctypes.c_int32),
                ("lanes_per_path", ctypes.c_int32), ("drain_steps", ctypes.c_int32),
                ("pad3", ctypes.c_int32)]

    def copy(self, **kw) -> "TrackOpts_":
        o = TrackOpts_()
        ctypes.pointer(o)[0] = self
        for k, v in kw.items():
            setattr(o, k, v)
        return o


class CertOpts_(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("lanes_per_item", ctypes.c_int32),
                ("tol", ctypes.c_double), ("res_tol", ctypes.c_double),
                ("cond_max", ctypes.c_double), ("sing_res", ctypes.c_double),
                ("div_norm", ctypes.c_double), ("real_tol", ctypes.c_double)]

    def copy(self, **kw) -> "CertOpts_":
        o = CertOpts_()
        ctypes.pointer(o)[0] = self
        for k, v in kw.items():
            setattr(o, k, v)
        return o


class ClassOpts_(ctypes.Structure):
    _fields_ = [("eig_rel", ctypes.c_double), ("jacobi_sweeps", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libnphc.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NphcError(f"{LIB_PATH} is missing: build it with `python -m paper_1104_5497_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u64, sz, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64,
                                  ctypes.c_size_t, ctypes.c_double)
    pB = ctypes.POINTER(Batch_)
    L.nphc_default_track_opts.argtypes = [i32, ctypes.POINTER(TrackOpts_)]
    L.nphc_default_track_opts.restype = None
    L.nphc_default_cert_opts.argtypes = [ctypes.POINTER(CertOpts_)]
    L.nphc_default_cert_opts.restype = None
    L.nphc_default_class_opts.argtypes = [ctypes.POINTER(ClassOpts_)]
    L.nphc_default_class_opts.restype = None
    L.nphc_track_workspace_size.argtypes = [pB, i32]
    L.nphc_track_workspace_size.restype = sz
    L.nphc_track_paths.argtypes = [pB, vp, i64, vp, i32, ctypes.POINTER(TrackOpts_), vp, i64, vp,
                                   vp, vp, vp, vp, vp, vp, sz, vp]
    L.nphc_refine_certify.argtypes = [pB, vp, i64, vp, ctypes.POINTER(CertOpts_), vp, i64, vp, vp,
                                      vp, vp, vp, vp, vp, vp, vp]
    L.nphc_mark_duplicates.argtypes = [pB, vp, i64, vp, vp, vp, dbl, vp, i64, vp, vp, vp, sz, vp]
    L.nphc_duplicates_workspace_size.argtypes = [i64]
    L.nphc_duplicates_workspace_size.restype = sz
    L.nphc_select.argtypes = [vp, i64, u64, vp, vp, vp, sz, vp]
    L.nphc_select_list.argtypes = [vp, vp, i64, vp, u64, vp, vp, vp, sz, vp]
    L.nphc_select_workspace_size.argtypes = [i64]
    L.nphc_select_workspace_size.restype = sz
    L.nphc_classify.argtypes = [pB, vp, i64, vp, ctypes.POINTER(ClassOpts_), dbl, vp, i64, vp, vp,
                                vp, vp, vp, vp, vp, vp, vp]
    L.nphc_adjoint.argtypes = [pB, vp, i64, vp, vp, i64, vp, vp, vp, vp]
    L.nphc_strerror.argtypes = [i32]
    L.nphc_strerror.restype = ctypes.c_char_p
    L.nphc_version.argtypes = []
    L.nphc_version.restype = ctypes.c_char_p
    for f in ("nphc_track_paths", "nphc_refine_certify", "nphc_mark_duplicates", "nphc_select",
              "nphc_select_list", "nphc_classify", "nphc_adjoint"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int, what: str) -> None:
    if rc != NPHC_OK:
        raise NphcError(f"{what} failed: {lib().nphc_strerror(rc).decode()} ({rc})")


def default_track_opts(precision: int) -> TrackOpts_:
    o = TrackOpts_()
    lib().nphc_default_track_opts(precision, ctypes.byref(o))
    return o


def default_cert_opts() -> CertOpts_:
    o = CertOpts_()
    lib().nphc_default_cert_opts(ctypes.byref(o))
    return o


def default_class_opts() -> ClassOpts_:
    o = ClassOpts_()
    lib().nphc_default_class_opts(ctypes.byref(o))
    return o
