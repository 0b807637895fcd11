"""ctypes binding of libdpr.so (argument marshalling only).

The library is built in-tree (``python -m paper_2407_00179_amd.build``).  There is
no fallback: if it is missing, importing this module raises.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# DPR_LIBRARY names another build of the same library (the test suite uses it for a
# build whose host code carries sanitizers)
LIB_PATH = os.environ.get("DPR_LIBRARY") or os.path.join(HERE, "libdpr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2407_00179_amd.build` "
                      "(the HIP library is required; there is no CPU fallback)")

# torch ships its own HIP runtime under the same soname as the system one the
# library is linked against; whichever loads first serves the whole process.
# Loading torch first keeps one runtime, torch's, for both (the other order
# leaves torch on a runtime it was not built with, and no device is found).
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)

OK = 0
STATUS = {0: "DPR_OK", -1: "DPR_ERR_INVALID_ARGUMENT", -2: "DPR_ERR_INVALID_STATE", -3: "DPR_ERR_OUT_OF_MEMORY",
          -4: "DPR_ERR_DEVICE", -5: "DPR_ERR_UNSUPPORTED"}
F32, F16 = 0, 1
FLAG_NO_SKIP, FLAG_PLAIN, FLAG_NO_GRAPH, FLAG_WIDE_OFFSETS, FLAG_F16_HALVES = 0x1, 0x2, 0x4, 0x8, 0x10
FLAG_QUEUE_COVERAGE = 0x20


class DprError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("center", C.c_double * 3), ("up", C.c_double * 3),
                ("fovy_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class PathParams(C.Structure):
    _fields_ = [("light_dir", C.c_float * 3), ("light_rgb", C.c_float * 3), ("env_rgb", C.c_float * 3),
                ("max_bounces", C.c_int32), ("spp", C.c_int32), ("seed", C.c_uint32)]


class PathStats(C.Structure):
    _fields_ = [("paths", C.c_int64), ("events", C.c_int64), ("shadow_steps", C.c_int64), ("forwards", C.c_int64),
                ("waves", C.c_int32)]


class RenderParams(C.Structure):
    _fields_ = [("step_voxels", C.c_float), ("ert_threshold", C.c_float), ("macrocell_cells", C.c_int32),
                ("flags", C.c_uint32)]


P = C.c_void_p
I64x3 = C.c_int64 * 3
I32x3 = C.c_int32 * 3

_SIGS = {
    "dpr_last_error": ([], C.c_char_p),
    "dpr_version": ([], C.c_char_p),
    "dpr_alloc_stats": ([C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "dpr_device_create": ([C.c_int, P, C.POINTER(P)], C.c_int),
    "dpr_device_set_stream": ([P, P], C.c_int),
    "dpr_device_sync": ([P], C.c_int),
    "dpr_device_release": ([P], None),
    "dpr_device_info": ([P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "dpr_world_create": ([P, I64x3, C.POINTER(P)], C.c_int),
    "dpr_world_release": ([P], None),
    "dpr_world_add_brick": ([P, P, C.c_int, C.c_int, I64x3, I64x3, I32x3, I32x3, C.POINTER(C.c_int32)], C.c_int),
    "dpr_world_commit": ([P], C.c_int),
    "dpr_world_release_linear": ([C.c_void_p], C.c_int),
    "dpr_world_brick_blocked": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_void_p, C.c_size_t], C.c_int),
    "dpr_check_partition": ([I64x3, C.c_int32, P, P, P, P], C.c_int),
    "dpr_check_camera": ([C.POINTER(Camera)], C.c_int),
    "dpr_world_brick_count": ([P, C.POINTER(C.c_int32)], C.c_int),
    "dpr_world_brick_macrocells": ([P, C.c_int32, I32x3, P, P, C.c_size_t], C.c_int),
    "dpr_set_transfer_function": ([P, P, C.c_int32, C.c_float, C.c_float, C.c_float], C.c_int),
    "dpr_set_isosurface": ([P, C.c_int32, C.c_float, C.c_float, C.c_float], C.c_int),
    "dpr_set_camera": ([P, C.POINTER(Camera)], C.c_int),
    "dpr_set_render_params": ([P, C.POINTER(RenderParams)], C.c_int),
    "dpr_frame_create": ([P, C.c_int32, C.c_int32, C.POINTER(P)], C.c_int),
    "dpr_frame_wrap": ([P, C.c_int32, C.c_int32, P, P, C.POINTER(P)], C.c_int),
    "dpr_frame_attach_counts": ([P, P], C.c_int),
    "dpr_frame_map": ([P, C.POINTER(P), C.POINTER(P)], C.c_int),
    "dpr_frame_unmap": ([P], C.c_int),
    "dpr_frame_read": ([P, P, P], C.c_int),
    "dpr_frame_release": ([P], None),
    "dpr_render_partial": ([P, C.c_int32, P], C.c_int),
    "dpr_composite": ([P, P, P, C.c_int32, P], C.c_int),
    "dpr_measure_gather": ([P, C.c_int32, P, P], C.c_int),
    "dpr_composite_noalloc": ([P, P, P, C.c_int32, P], C.c_int),
    "dpr_render_frame": ([P, P], C.c_int),
    "dpr_render_batch": ([P, P, C.c_int32, P, C.c_uint32], C.c_int),
    "dpr_autotune_batch": ([P, P, C.c_int32, P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "dpr_set_batch_tile": ([P, C.c_int32, C.c_int32], C.c_int),
    "dpr_batch_timings": ([P, C.POINTER(C.c_float), C.POINTER(C.c_float)], C.c_int),
    "dpr_batch_coverage": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "dpr_tune_cache_lookup": ([C.c_char_p, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "dpr_tune_cache_store": ([C.c_char_p, C.c_char_p, C.c_int32, C.c_int32], C.c_int),
    "dpr_deep_frame_create": ([P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(P)], C.c_int),
    "dpr_deep_frame_wrap": ([P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, C.POINTER(P)], C.c_int),
    "dpr_deep_frame_release": ([P], None),
    "dpr_render_deep": ([P, C.c_int32, P], C.c_int),
    "dpr_composite_deep": ([P, P, C.c_int32, P], C.c_int),
    "dpr_render_path": ([P, C.POINTER(PathParams), P, C.POINTER(PathStats)], C.c_int),
    "dpr_train_workspace_size": ([I64x3, P, C.c_int32, C.c_float, C.POINTER(C.c_size_t)], C.c_int),
    "dpr_render_train_forward": ([P, P, I64x3, P, C.c_int32, C.c_float, C.c_float, C.c_float,
                                  C.POINTER(RenderParams), P, C.c_int32, P, P, P, C.c_size_t], C.c_int),
    "dpr_render_backward": ([P, P, I64x3, P, C.c_int32, C.c_float, C.c_float, C.c_float,
                             C.POINTER(RenderParams), P, C.c_int32, P, P, C.c_size_t, P, P], C.c_int),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


def check(status):
    if status != OK:
        raise DprError(status, lib.dpr_last_error().decode(errors="replace"))
    return status
