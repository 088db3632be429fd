"""ctypes declarations of the C ABI in include/wamct.h (argument marshalling only).

torch is imported first on purpose: its ROCm wheel ships the HIP runtime, and loading
libwamct.so afterwards binds the library to that same runtime (one runtime per process,
so torch's streams and allocations are valid in the library)."""
import ctypes
import os

import torch  # noqa: F401  (must precede loading libwamct.so)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwamct.so")

OK, E_INVALID, E_UNSUPPORTED, E_OOM, E_HIP, E_NUMERIC, E_STATE = range(7)
PARALLEL, FAN, CONE = 0, 1, 2
RULE_VALUE, RULE_GRADIENT = 0, 1
F32, F64 = 0, 1
K_SYNTH, K_FORWARD, K_UPDATE, K_TREE, K_OTHER, NK = range(6)
KERNEL_CLASSES = ("synth", "forward", "update", "tree", "other")

# every entry point declared in include/wamct.h
SYMBOLS = (
    "wamct_validate", "wamct_create", "wamct_destroy", "wamct_last_error", "wamct_version",
    "wamct_set_stream", "wamct_set_data", "wamct_reset", "wamct_set_state", "wamct_get_state",
    "wamct_iterate", "wamct_expand", "wamct_solve", "wamct_synthesize", "wamct_project",
    "wamct_backproject", "wamct_backproject_split", "wamct_forward", "wamct_idiv", "wamct_get_b",
    "wamct_tree_stats", "wamct_timing", "wamct_get_timing", "wamct_loss", "wamct_loss_backward",
    "wamct_set_tiling", "wamct_get_tiling", "wamct_batch_create", "wamct_batch_destroy",
    "wamct_batch_last_error", "wamct_batch_reset", "wamct_batch_solve", "wamct_batch_autotune",
    "wamct_batch_stats", "wamct_set_subsets", "wamct_get_subsets", "wamct_set_tree_sharing",
    "wamct_get_tree_sharing", "wamct_set_tree_rule", "wamct_get_tree_rule", "wamct_set_penalty",
    "wamct_get_penalty", "wamct_set_tree_schedule", "wamct_get_tree_schedule", "wamct_idiv_noalloc",
    "wamct_set_walk_lanes", "wamct_get_walk_lanes",
)


class Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("pixel", ctypes.c_double),
                ("n_views", ctypes.c_int32), ("angle0", ctypes.c_double), ("angle_span", ctypes.c_double),
                ("n_bins", ctypes.c_int32), ("bin_pitch", ctypes.c_double), ("sod", ctypes.c_double),
                ("sdd", ctypes.c_double), ("nz", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("row_pitch", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("dtype", ctypes.c_int32), ("geometry", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("wavelet_dims", ctypes.c_int32),
                ("wavelet", ctypes.c_int32)]


class WamctError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"wamct status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1508_04458_amd.build, or __graft_entry__.build()). "
            "There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "wamct_validate": (P(Geometry), P(Options), ctypes.c_char_p, i32),
        "wamct_create": (P(Geometry), P(Options), vp, P(vp)),
        "wamct_destroy": (vp,),
        "wamct_set_stream": (vp, vp),
        "wamct_set_data": (vp, vp, vp, P(f64)),
        "wamct_reset": (vp,),
        "wamct_set_state": (vp, vp, vp),
        "wamct_get_state": (vp, vp, vp, P(i32)),
        "wamct_iterate": (vp, i32, vp),
        "wamct_expand": (vp, f64, P(i32)),
        "wamct_solve": (vp, i32, P(i32), i32, f64, vp),
        "wamct_synthesize": (vp, vp),
        "wamct_project": (vp, vp, vp),
        "wamct_backproject": (vp, vp, vp),
        "wamct_backproject_split": (vp, vp, vp, vp),
        "wamct_forward": (vp, vp, vp),
        "wamct_idiv": (vp, vp, vp),
        "wamct_get_b": (vp, vp),
        "wamct_tree_stats": (vp, P(f64), P(i64), P(i64), P(i64)),
        "wamct_timing": (vp, i32),
        "wamct_get_timing": (vp, P(f64), P(i64)),
        "wamct_loss": (vp, i32, vp, vp, vp, f64, vp, vp),
        "wamct_loss_backward": (vp, i32, vp, vp, vp, vp),
        "wamct_set_tiling": (vp, i32),
        "wamct_get_tiling": (vp, P(i32)),
        "wamct_set_subsets": (vp, i32),
        "wamct_set_tree_sharing": (vp, i32),
        "wamct_get_tree_sharing": (vp, P(i32)),
        "wamct_set_tree_rule": (vp, i32),
        "wamct_get_tree_rule": (vp, P(i32)),
        "wamct_set_penalty": (vp, ctypes.c_double),
        "wamct_get_penalty": (vp, P(ctypes.c_double)),
        "wamct_get_subsets": (vp, P(i32)),
        "wamct_set_tree_schedule": (vp, i32, P(i32), vp),
        "wamct_get_tree_schedule": (vp, P(i32), P(i32), i32),
        "wamct_idiv_noalloc": (i32, i64, i32, vp, vp, vp, vp),
        "wamct_set_walk_lanes": (vp, i32),
        "wamct_get_walk_lanes": (vp, P(i32)),
        "wamct_batch_create": (i32, P(vp), i32, i32, vp, P(vp)),
        "wamct_batch_destroy": (vp,),
        "wamct_batch_reset": (vp,),
        "wamct_batch_solve": (vp, i32, P(i32), i32, f64, P(vp)),
        "wamct_batch_autotune": (vp, i32, P(i32), i32, P(i32)),
        "wamct_batch_stats": (vp, P(i32), P(i64), P(i64), P(i64)),
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = list(args)
        fn.restype = ctypes.c_int
    lib.wamct_last_error.argtypes = [vp]
    lib.wamct_last_error.restype = ctypes.c_char_p
    lib.wamct_version.argtypes = []
    lib.wamct_version.restype = ctypes.c_char_p
    lib.wamct_batch_last_error.argtypes = [vp]
    lib.wamct_batch_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def check(status, ctx=None):
    if status != OK:
        msg = lib.wamct_last_error(ctx)
        raise WamctError(status, msg.decode() if msg else "")


def check_batch(status, batch=None):
    if status != OK:
        msg = lib.wamct_batch_last_error(batch)
        raise WamctError(status, msg.decode() if msg else "")
