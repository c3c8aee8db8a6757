"""ctypes binding of libbatchlayout.so (argument marshalling only).

Every step of the layout runs in the HIP library; this module converts numpy
arrays or torch device tensors into the pointers and structs of the C ABI
declared in include/batchlayout.h.  There is no CPU fallback: if the built
library is missing, loading fails with an error that says so.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbatchlayout.so")

BL_OK, BL_E_INVAL, BL_E_NOMEM, BL_E_HIP, BL_E_NOTREADY, BL_E_REJECTED, BL_E_NONFINITE, BL_E_TIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7
BL_EXACT, BL_BH = 0, 1
BL_FP32_KAHAN, BL_FP32_PLAIN, BL_FP64 = 0, 1, 2
BL_DEVICE_PTRS, BL_VALIDATE, BL_BH_SNAPSHOT_LEAVES, BL_EXACT_MULTI_WG, BL_ADAPTIVE_STEP = 1, 2, 4, 8, 16

EXPORTED = [
    "bl_params_init", "bl_last_error", "bl_version", "bl_footprint_bytes", "bl_layout", "bl_forces",
    "bl_graph_create", "bl_graph_set_coords", "bl_graph_get_coords", "bl_graph_run",
    "bl_graph_destroy", "bl_graph_profile", "bl_graph_profile_read", "bl_layout_batch",
    "bl_server_create", "bl_server_submit", "bl_server_poll", "bl_server_wait", "bl_server_fetch",
    "bl_server_release", "bl_server_destroy", "bl_greedy_init", "bl_quality_eval",
    "bl_layout_shuffled", "bl_quality_eval_noalloc", "bl_neighborhood_preservation",
    "bl_probe_issue_rate",
]


class BLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("batchlayout error %d: %s" % (code, msg))
        self.code = code


class CSR(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("colidx", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("batch_size", C.c_int32), ("iterations", C.c_int32), ("start_iter", C.c_int32),
                ("mode", C.c_int32), ("precision", C.c_int32), ("repulse_adjacent", C.c_int32),
                ("step0", C.c_double), ("step_decay", C.c_double), ("K", C.c_double),
                ("R", C.c_double), ("theta", C.c_double), ("flags", C.c_uint32),
                ("reserved0", C.c_int32), ("conv_tol", C.c_double), ("model_a", C.c_int32),
                ("model_r", C.c_int32), ("reserved", C.c_int32 * 2)]


class Stats(C.Structure):
    _fields_ = [("iters_run", C.c_int32), ("late_overflow", C.c_int32), ("energy_last", C.c_double),
                ("seconds", C.c_double), ("node_visits", C.c_int64), ("nonfinite_events", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Quality(C.Structure):
    _fields_ = [("stress", C.c_double), ("scale", C.c_double), ("pairs", C.c_int64),
                ("edge_energy", C.c_double), ("edge_uniformity", C.c_double), ("edges", C.c_int64),
                ("bfs_levels", C.c_int64), ("reserved", C.c_double * 2)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_lib = None


def load():
    """Load the built library (torch first, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (shares libamdhip64 with the library)
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbatchlayout.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_2002_08233_amd.build" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    lib.bl_params_init.argtypes = [P(Params)]
    lib.bl_last_error.restype = C.c_char_p
    lib.bl_version.restype = C.c_char_p
    lib.bl_footprint_bytes.argtypes = [i32, i64, P(Params)]
    lib.bl_footprint_bytes.restype = C.c_size_t
    lib.bl_layout.argtypes = [P(CSR), vp, vp, P(Params), vp, vp, vp, vp, P(Stats)]
    lib.bl_layout_shuffled.argtypes = [P(CSR), vp, vp, P(Params), C.c_uint64, vp, vp, vp, vp, P(Stats)]
    lib.bl_forces.argtypes = [P(CSR), vp, vp, vp, vp, i32, P(Params), vp, vp, vp]
    lib.bl_greedy_init.argtypes = [P(CSR), i32, vp, vp]
    lib.bl_quality_eval.argtypes = [P(CSR), vp, vp, i32, vp, dbl, C.c_uint32, vp, P(Quality)]
    lib.bl_neighborhood_preservation.argtypes = [P(CSR), vp, vp, i32, vp, C.c_uint32, vp, P(dbl), P(i64)]
    lib.bl_quality_eval_noalloc.argtypes = [P(CSR), vp, vp, i32, vp, dbl, C.c_uint32, vp, P(Quality)]
    lib.bl_graph_create.argtypes = [P(CSR), P(Params), vp, P(vp)]
    lib.bl_graph_set_coords.argtypes = [vp, vp, vp, C.c_uint32]
    lib.bl_graph_get_coords.argtypes = [vp, vp, vp, C.c_uint32]
    lib.bl_graph_run.argtypes = [vp, i32, i32, i32, vp, vp, vp, P(Stats)]
    lib.bl_graph_destroy.argtypes = [vp]
    lib.bl_graph_profile.argtypes = [vp, i32]
    lib.bl_graph_profile_read.argtypes = [vp, C.c_char_p, P(dbl), P(i64)]
    lib.bl_probe_issue_rate.argtypes = [i32, i32, i32, vp, P(dbl), P(dbl)]
    if hasattr(lib, "bl_layout_batch"):
        lib.bl_layout_batch.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp]
    if hasattr(lib, "bl_server_create"):
        lib.bl_server_create.argtypes = [C.c_size_t, i32, vp, P(vp)]
        lib.bl_server_submit.argtypes = [vp, P(CSR), vp, vp, P(Params), P(i64)]
        lib.bl_server_poll.argtypes = [vp, i64, P(i32)]
        lib.bl_server_wait.argtypes = [vp, i64, dbl]
        lib.bl_server_fetch.argtypes = [vp, i64, vp, vp, P(Stats)]
        lib.bl_server_release.argtypes = [vp, i64]
        lib.bl_server_destroy.argtypes = [vp]
    _lib = lib
    return lib


def check(rc: int):
    if rc != BL_OK:
        raise BLError(rc, load().bl_last_error().decode(errors="replace"))
    return rc
