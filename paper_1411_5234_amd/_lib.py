"""ctypes binding of libnbody.so (include/nbody.h).  Argument marshalling only.

Every step of the path runs in the HIP library; this module turns torch tensors
into device pointers and torch streams into hipStream_t handles, and raises
NbError on a non-zero status.  If the library is not built the import of the
first entry point fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnbody.so")

FIELDS64 = ["x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "jx", "jy", "jz",
            "m", "t", "dt", "xp", "yp", "zp", "vxp", "vyp", "vzp"]
FIELDS32 = ["vxp32", "vyp32", "vzp32", "m32"]
# nb_hermite6: snap, crackle, predicted acceleration (FP64), FP32 copies
H6_FIELDS64 = ["sx", "sy", "sz", "cx", "cy", "cz", "axp", "ayp", "azp"]
H6_FIELDS32 = ["axp32", "ayp32", "azp32"]

NB_FP64 = 0
NB_MIXED = 1
NB_DS = 2
PRECISIONS = {"fp64": NB_FP64, "mixed": NB_MIXED, "ds": NB_DS}

STATUS = {0: "NB_OK", -1: "NB_EINVAL", -2: "NB_ENOMEM", -3: "NB_EDEVICE",
          -4: "NB_ERANGE", -5: "NB_ENAN", -6: "NB_EINDEX", -7: "NB_EUNBOUND",
          -8: "NB_ESCRATCH"}

# Every symbol include/nbody.h declares.
EXPORTS = ["nb_ctx_create", "nb_ctx_destroy", "nb_last_error", "nb_sync", "nb_select_active",
           "nb_predict", "nb_force_active", "nb_init_steps", "nb_correct", "nb_energy",
           "nb_force_plan", "nb_force_plan_lanes", "nb_force_active_plan", "nb_force_active_noalloc",
           "nb_init_steps_active", "nb_pairs_perturbation", "nb_pairs_split_energy",
           "nb_version", "nb_select_active_batch",
           "nb_predict_batch", "nb_force_active_batch", "nb_correct_batch", "nb_step_batch",
           "nb_predict6", "nb_force6_active", "nb_force6_active_plan", "nb_init_steps6",
           "nb_correct6", "nb_step6", "nb_step6_batch", "nb_tidal_active", "nb_tidal_active_batch",
           "nb_pairs_reduce", "nb_pairs_members", "nb_pairs_energy", "nb_kepler_drift",
           "nb_groups_advance", "nb_groups_advance_async", "nb_groups_wait", "nb_tidal_points",
           "nb_nearest_active_batch"]


class NbSystem(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, C.c_void_p) for f in FIELDS64 + FIELDS32]


class NbHermite6(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in H6_FIELDS64 + H6_FIELDS32]


class NbBatchItem(C.Structure):
    _fields_ = [("sys", NbSystem), ("i_idx", C.c_void_p), ("acc", C.c_void_p),
                ("jerk", C.c_void_p), ("status", C.c_void_p), ("eps", C.c_double),
                ("t_next", C.c_double), ("t_end", C.c_double), ("m", C.c_int32),
                ("startup", C.c_int32), ("error", C.c_int32), ("done", C.c_int32),
                ("lanes", C.c_int64)]


class NbTidalItem(C.Structure):
    _fields_ = [("sys", NbSystem), ("i_idx", C.c_void_p), ("m", C.c_int32), ("eps", C.c_double),
                ("tensor", C.c_void_p), ("t_out", C.c_void_p), ("status", C.c_void_p),
                ("row0", C.c_int64), ("nrows", C.c_int64)]


class NbNearestItem(C.Structure):
    _fields_ = [("sys", NbSystem), ("i_idx", C.c_void_p), ("m", C.c_int32),
                ("row_end", C.c_int64), ("dt_cap", C.c_double), ("nn", C.c_void_p),
                ("r2", C.c_void_p), ("status", C.c_void_p)]


class NbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code
        self.name = STATUS.get(code, "?")


_lib = None


def load() -> C.CDLL:
    """Load libnbody.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libnbody.so is not built (%s); run `python -m paper_1411_5234_amd.build`"
                           % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    ps = C.POINTER(NbSystem)
    ph = C.POINTER(NbHermite6)
    sig = {
        "nb_ctx_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, vp]),
        "nb_ctx_destroy": (C.c_int, [vp]),
        "nb_last_error": (C.c_char_p, [vp]),
        "nb_sync": (C.c_int, [vp]),
        "nb_select_active": (C.c_int, [vp, ps, C.POINTER(f64), vp, C.POINTER(i32)]),
        "nb_predict": (C.c_int, [vp, ps, f64]),
        "nb_force_active": (C.c_int, [vp, ps, vp, i32, i64, i64, f64, C.c_int, vp, vp]),
        "nb_force_active_plan": (C.c_int, [vp, ps, vp, i32, i64, i64, f64, C.c_int, i32, i32, i32,
                                           vp, vp]),
        "nb_force_active_noalloc": (C.c_int, [vp, ps, vp, i32, i64, i64, f64, C.c_int, vp, vp]),
        "nb_force_plan": (None, [i64, i32, C.c_int, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "nb_force_plan_lanes": (C.c_int, [i64, i32, C.c_int, i64, C.POINTER(i32), C.POINTER(i32),
                                          C.POINTER(i32)]),
        "nb_init_steps": (C.c_int, [vp, ps, vp, vp, f64, f64, f64]),
        "nb_init_steps_active": (C.c_int, [vp, ps, vp, i32, vp, vp, f64, f64, f64, f64]),
        "nb_pairs_perturbation": (C.c_int, [i32, vp, vp, vp, vp, vp, vp]),
        "nb_pairs_split_energy": (C.c_int, [i32, vp, vp, vp, f64, vp]),
        "nb_correct": (C.c_int, [vp, ps, vp, i32, vp, vp, f64, f64, f64, f64]),
        "nb_energy": (C.c_int, [vp, ps, f64, C.POINTER(f64), C.POINTER(f64)]),
        "nb_version": (C.c_char_p, []),
        "nb_select_active_batch": (C.c_int, [vp, C.POINTER(NbBatchItem), i32]),
        "nb_predict_batch": (C.c_int, [vp, C.POINTER(NbBatchItem), i32]),
        "nb_force_active_batch": (C.c_int, [vp, C.POINTER(NbBatchItem), i32, C.c_int]),
        "nb_correct_batch": (C.c_int, [vp, C.POINTER(NbBatchItem), i32, f64, f64, f64, f64]),
        "nb_step_batch": (C.c_int, [vp, C.POINTER(NbBatchItem), i32, C.c_int, f64, f64, f64, f64]),
        "nb_predict6": (C.c_int, [vp, ps, ph, f64]),
        "nb_force6_active": (C.c_int, [vp, ps, ph, vp, i32, i64, i64, f64, C.c_int, vp, vp, vp]),
        "nb_force6_active_plan": (C.c_int, [vp, ps, ph, vp, i32, i64, i64, f64, C.c_int, i32, i32,
                                            i32, vp, vp, vp]),
        "nb_init_steps6": (C.c_int, [vp, ps, ph, vp, vp, vp, f64, f64, f64]),
        "nb_correct6": (C.c_int, [vp, ps, ph, vp, i32, vp, vp, vp, f64, f64, f64, f64]),
        "nb_step6": (C.c_int, [vp, ps, ph, vp, vp, vp, vp, f64, C.c_int, f64, f64, f64, f64, vp, vp,
                               vp]),
        "nb_step6_batch": (C.c_int, [vp, C.POINTER(NbBatchItem), ph, C.POINTER(C.c_void_p), i32,
                                     C.c_int, f64, f64, f64, f64]),
        "nb_tidal_active": (C.c_int, [vp, ps, vp, i32, i64, i64, f64, vp]),
        "nb_tidal_active_batch": (C.c_int, [vp, C.POINTER(NbTidalItem), i32]),
        "nb_tidal_points": (C.c_int, [vp, vp, i32, vp, vp, C.c_double, vp]),
        "nb_nearest_active_batch": (C.c_int, [vp, C.POINTER(NbNearestItem), i32]),
        "nb_pairs_reduce": (C.c_int, [i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]),
        "nb_pairs_members": (C.c_int, [i64, vp, vp, vp, i32, vp, vp, vp, vp, vp]),
        "nb_pairs_energy": (C.c_int, [i32, vp, vp, vp, vp, vp, vp]),
        "nb_kepler_drift": (C.c_int, [f64, vp, vp, f64, vp, vp]),
        "nb_groups_advance": (C.c_int, [i32, vp, vp, vp, vp, vp, vp, vp, i32, i64, vp]),
        "nb_groups_advance_async": (C.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp, i32, i64, vp]),
        "nb_groups_wait": (C.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def force_plan(nj: int, m: int, precision: str = "mixed", lanes: int | None = None):
    """(i-bodies per lane, lanes per i-body, j-chunks) of the force launch; lanes:
    the plan's lane target (None: nb_force_plan; 0: the default target)."""
    L = load()
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    if lanes is None:
        L.nb_force_plan(int(nj), int(m), PRECISIONS[precision], C.byref(a), C.byref(b),
                        C.byref(c))
    else:
        rc = L.nb_force_plan_lanes(int(nj), int(m), PRECISIONS[precision], int(lanes),
                                   C.byref(a), C.byref(b), C.byref(c))
        if rc != 0:
            raise NbError(rc, "lane target %d out of range" % lanes)
    return a.value, b.value, c.value
