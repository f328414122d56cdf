"""ctypes binding of liblocalgs.so (the C ABI declared in include/localgs.h).

Argument marshalling only: every computation happens in the HIP library.
Importing this module does not touch the GPU; loading the library fails
loudly if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblocalgs.so")

LGS_OK = 0
LGS_ERR_INVALID_ARG = 1
LGS_ERR_CAPACITY = 2
LGS_ERR_HIP = 3
LGS_ERR_UNSUPPORTED = 4

RENDER_PLAIN = 0
RENDER_HOIST = 1
RENDER_HOIST_CULL = 2
RENDER_LOCAL = 3
RENDER_FP32 = 0x10
RENDER_Q8 = 0x20
RENDER_VOTE4 = 0x40
RENDER_GLOBAL = 0x80
BWD_ACCUMULATE = 0x100
PROJ_BWD_CLEAR = 0x1

MAX_VIEWS = 16
QUEUE_WORDS = 256

SORT_NOALLOC_SCRATCH_BYTES = 64 << 20
SPLAT_FLOATS = 16   # floats per projected splat record (64 bytes)
GRAD_FLOATS = 9     # floats per packed gradient record

EXPORTS = ["lgs_last_error", "lgs_version", "lgs_project", "lgs_sort_workspace_size", "lgs_sort", "lgs_sort_noalloc",
           "lgs_tile_ranges", "lgs_render", "lgs_render_backward", "lgs_project_backward", "lgs_l1_workspace_size",
           "lgs_l1_loss",
           "lgs_project_batch", "lgs_sort_batch", "lgs_render_batch", "lgs_render_backward_batch",
           "lgs_project_backward_batch", "lgs_graph_begin", "lgs_graph_end", "lgs_graph_launch",
           "lgs_graph_destroy", "lgs_tile_order_workspace_size", "lgs_tile_order", "lgs_render_debug",
           "lgs_used_mask_words"]


class LgsCamera(C.Structure):
    _fields_ = [("viewmat", C.c_float * 12), ("campos", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("tan_fovx", C.c_float), ("tan_fovy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("znear", C.c_float), ("bg", C.c_float * 3)]


class LocalGSError(RuntimeError):
    pass


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_SIG = {
    "lgs_last_error": (C.c_char_p, []),
    "lgs_version": (C.c_char_p, []),
    "lgs_project": (C.c_int, [C.POINTER(LgsCamera), _I64, _I32] + [_P] * 9),
    "lgs_sort_workspace_size": (C.c_size_t, [_I64, _I64, _I32]),
    "lgs_sort": (C.c_int, [_I64, _I32, _I32, _P, _P, _P, _P, _P, _I64, _P, _P, _P, C.c_size_t, _P]),
    "lgs_sort_noalloc": (C.c_int, [_I64, _I32, _I32, _P, _P, _P, _P, _P, _I64, _P, _P, _P]),
    "lgs_tile_ranges": (C.c_int, [_P, _P, _P, _I64, _I32, _P, _P]),
    "lgs_render": (C.c_int, [_I32, C.POINTER(LgsCamera)] + [_P] * 8),
    "lgs_render_backward": (C.c_int, [_I32, C.POINTER(LgsCamera), _I64] + [_P] * 9),
    "lgs_project_backward": (C.c_int, [C.POINTER(LgsCamera), _I64, _I32] + [_P] * 12 + [_I32, _P]),
    "lgs_l1_workspace_size": (C.c_size_t, []),
    "lgs_l1_loss": (C.c_int, [_P, _P, _I64, _P, _P, _P, C.c_size_t, _P]),
    "lgs_project_batch": (C.c_int, [C.POINTER(LgsCamera), _I32, _I64, _I32] + [_P] * 9),
    "lgs_sort_batch": (C.c_int, [_I32, C.POINTER(_I32), C.POINTER(_I32), _I64, _P, _P, _P, _P, _P, _I64, _P, _P,
                                 _P, C.c_size_t, _P]),
    "lgs_render_batch": (C.c_int, [_I32, C.POINTER(LgsCamera), _I32] + [_P] * 7 + [_P, _P, _I32, _P, _I64, _P]),
    "lgs_used_mask_words": (_I64, [_I64, _I32]),
    "lgs_render_debug": (C.c_int, [_I32, C.POINTER(LgsCamera), _I32] + [_P] * 9),
    "lgs_tile_order_workspace_size": (C.c_size_t, [_I32]),
    "lgs_tile_order": (C.c_int, [_P, _I32, _P, _P, C.c_size_t, _P]),
    "lgs_render_backward_batch": (C.c_int, [_I32, C.POINTER(LgsCamera), _I32, _I64] + [_P] * 10
                                  + [_I32, _P, _P, _I64, _P]),
    "lgs_project_backward_batch": (C.c_int, [C.POINTER(LgsCamera), _I32, _I64, _I32] + [_P] * 12 + [_I32, _P]),
    "lgs_graph_begin": (C.c_int, [_P]),
    "lgs_graph_end": (C.c_int, [_P, C.POINTER(_P)]),
    "lgs_graph_launch": (C.c_int, [_P, _P]),
    "lgs_graph_destroy": (C.c_int, [_P]),
}

_lib = None


def lib():
    """Load liblocalgs.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LocalGSError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                               f"python -m paper_2606_16566_amd.build_lib")
        lb = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(lb, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lb
    return _lib


def check(status: int, what: str) -> None:
    if status != LGS_OK:
        msg = lib().lgs_last_error().decode(errors="replace")
        raise LocalGSError(f"{what} failed with status {status}: {msg}")


def camera_array(cams):
    """Sequence of scenes.Camera -> contiguous LgsCamera array."""
    arr = (LgsCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera_struct(c)
    return arr


def camera_struct(cam) -> LgsCamera:
    """scenes.Camera -> LgsCamera."""
    c = LgsCamera()
    vm = [float(v) for v in cam.viewmat.reshape(12)]
    for i in range(12):
        c.viewmat[i] = vm[i]
    for i in range(3):
        c.campos[i] = float(cam.campos[i])
        c.bg[i] = float(cam.bg[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.tan_fovx, c.tan_fovy = float(cam.tan_fovx), float(cam.tan_fovy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.znear = float(cam.znear)
    return c
