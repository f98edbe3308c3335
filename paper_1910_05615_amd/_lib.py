"""ctypes declarations of the librtdetmcd C ABI (include/rtdetmcd.h)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtdetmcd.so")

c_i32, c_i64, c_f64, c_vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p

RTDETMCD_OK = 0
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESINGULAR",
                -5: "ENONFINITE", -6: "EUNSUPPORTED"}

# exported symbols, in the header's order
SYMBOLS = [
    "rtdetmcd_create", "rtdetmcd_destroy", "rtdetmcd_set_stream", "rtdetmcd_last_error",
    "rtdetmcd_tuned_plans", "rtdetmcd_default_opts", "rtdetmcd_plan", "rtdetmcd_fit", "rtdetmcd_fit_batched",
    "rtdetmcd_chi2_quantile", "rtdetmcd_chi2_cdf", "rtdetmcd_consistency",
    "rtdetmcd_distances", "rtdetmcd_score", "rtdetmcd_select", "rtdetmcd_cstep",
    "rtdetmcd_cstep_noalloc", "rtdetmcd_profile", "rtdetmcd_profile_read",
    "rtdetmcd_sort_reruns", "rtdetmcd_backward",
]


class Opts(C.Structure):
    _fields_ = [("struct_size", c_i32), ("alpha", c_f64), ("standardize", c_i32),
                ("cstep_mode", c_i32), ("max_csteps", c_i32), ("kappa_max", c_f64),
                ("cutoff_q", c_f64), ("pool_mode", c_i32), ("rew_consistency", c_i32),
                ("omega", c_i32), ("launch", c_i32), ("graph", c_i32),
                ("rounds_per_sync", c_i32), ("distance", c_i32), ("tune", c_i32)]


class Out(C.Structure):
    _fields_ = [("mu", c_vp), ("sigma", c_vp), ("mu_raw", c_vp), ("sigma_raw", c_vp),
                ("logdet", c_vp), ("dist", c_vp), ("outlier", c_vp), ("hsubset", c_vp),
                ("block_status", c_vp), ("block_start", c_vp), ("block_iters", c_vp),
                ("loc", c_vp), ("scale", c_vp), ("n_w", c_vp), ("rew_mask", c_vp),
                ("ldtrace", c_vp), ("hmargin", c_vp), ("cmargin", c_vp)]


class DatasetDesc(C.Structure):
    _fields_ = [("X", c_vp), ("dtype", c_i32), ("n", c_i64), ("p", c_i32), ("ld", c_i64),
                ("h_sub", c_i64), ("n_chunks", c_i32), ("out", Out), ("perm", c_vp),
                ("warm_mu", c_vp), ("warm_sigma", c_vp)]


_lib = None


def load() -> C.CDLL:
    """Load the in-tree library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1910_05615_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    sig = {
        "rtdetmcd_create": (c_i32, [P(c_vp), c_i32, c_vp]),
        "rtdetmcd_destroy": (c_i32, [c_vp]),
        "rtdetmcd_set_stream": (c_i32, [c_vp, c_vp]),
        "rtdetmcd_last_error": (C.c_char_p, [c_vp]),
        "rtdetmcd_tuned_plans": (c_i32, [c_vp, P(c_i64), c_i32, P(c_i32)]),
        "rtdetmcd_default_opts": (None, [P(Opts)]),
        "rtdetmcd_plan": (c_i32, [c_i64, c_i32, c_i64, c_i32, P(Opts), P(c_i32), P(c_i64), P(c_i64)]),
        "rtdetmcd_fit": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i32, c_i64, c_i64, c_i32, P(Opts), P(Out)]),
        "rtdetmcd_fit_batched": (c_i32, [c_vp, c_i32, P(DatasetDesc), P(Opts), P(c_i32)]),
        "rtdetmcd_chi2_quantile": (c_f64, [c_f64, c_i32]),
        "rtdetmcd_chi2_cdf": (c_f64, [c_f64, c_i32]),
        "rtdetmcd_consistency": (c_f64, [c_f64, c_i32]),
        "rtdetmcd_distances": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i32, c_i64, c_vp, c_vp, c_vp]),
        "rtdetmcd_score": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i32, c_i64, c_vp, c_vp, c_f64,
                                   c_vp, c_vp]),
        "rtdetmcd_select": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_vp, c_vp]),
        "rtdetmcd_cstep": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i32, c_i64, c_i64, c_vp, c_vp,
                                   c_vp, P(Opts), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
        "rtdetmcd_cstep_noalloc": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i32, c_i64, c_i64, c_vp,
                                           c_vp, c_vp, P(Opts), c_vp, c_vp, c_vp, c_vp, c_vp,
                                           c_vp]),
        "rtdetmcd_profile": (c_i32, [c_vp, c_i32]),
        "rtdetmcd_profile_read": (c_i32, [c_vp, c_i32, P(c_f64), P(c_i64), P(c_f64), P(c_f64),
                                          P(c_f64)]),
        "rtdetmcd_sort_reruns": (c_i64, [c_vp]),
        "rtdetmcd_backward": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i32, c_i64, c_vp, c_vp, c_vp,
                                      c_vp, c_vp, c_f64, c_vp, c_vp, c_vp, c_vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
