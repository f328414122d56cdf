"""The C-ABI library loads and exports every entry point the header declares;
host-side argument checks reject bad calls before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "localgs.h")


def _lib():
    from paper_2606_16566_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return L


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lgs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_pipeline():
    names = declared()
    for must in ["lgs_project", "lgs_sort", "lgs_tile_ranges", "lgs_render", "lgs_render_backward",
                 "lgs_project_backward", "lgs_l1_loss", "lgs_sort_workspace_size", "lgs_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lb = C.CDLL(L.LIB_PATH)
    for name in declared():
        assert hasattr(lb, name), name
    assert set(L.EXPORTS) >= set(declared())


def test_version_and_workspace_query():
    L = _lib()
    assert L.lib().lgs_version().startswith(b"localgs")
    a = L.lib().lgs_sort_workspace_size(1000, 5000, 100)
    b = L.lib().lgs_sort_workspace_size(100000, 5000000, 100)
    assert 0 < a < b and a % 256 == 0
    assert L.lib().lgs_sort_workspace_size(-1, 10, 10) == 0


def test_invalid_arguments_rejected_on_host():
    L = _lib()
    cam = L.LgsCamera()
    cam.width, cam.height, cam.fx, cam.fy = 0, 10, 100.0, 100.0          # width 0: invalid
    st = L.lib().lgs_project(C.byref(cam), 10, 0, *([None] * 9))
    assert st == L.LGS_ERR_INVALID_ARG
    assert b"camera" in L.lib().lgs_last_error()
    cam.width = 16
    st = L.lib().lgs_project(C.byref(cam), 10, 5, *([None] * 9))     # sh degree 5
    assert st == L.LGS_ERR_INVALID_ARG
    st = L.lib().lgs_project(C.byref(cam), 10, 0, *([None] * 9))     # null pointers
    assert st == L.LGS_ERR_INVALID_ARG and b"null" in L.lib().lgs_last_error()
    st = L.lib().lgs_render(7, C.byref(cam), *([None] * 8))            # unknown variant
    assert st == L.LGS_ERR_INVALID_ARG
    st = L.lib().lgs_sort(10, 4, 4, None, None, None, None, None, 100, None, None, None, 0, None)
    assert st == L.LGS_ERR_INVALID_ARG
    st = L.lib().lgs_l1_loss(None, None, 0, None, None, None, 0, None)
    assert st == L.LGS_ERR_INVALID_ARG
    # a workspace below lgs_l1_workspace_size() is rejected before any launch
    one = C.c_void_p(256)
    st = L.lib().lgs_l1_loss(one, one, 10, one, one, one, L.lib().lgs_l1_workspace_size() - 8, None)
    assert st == L.LGS_ERR_INVALID_ARG and b"workspace" in L.lib().lgs_last_error()
    assert L.lib().lgs_l1_workspace_size() >= 8


def test_sort_noalloc_rejects_sizes_beyond_its_scratch():
    """Checked on the host before any HIP call: runs without a GPU."""
    L = _lib()
    lb = L.lib()
    n = 4_000_000
    assert lb.lgs_sort_workspace_size(n, n, 64) > L.SORT_NOALLOC_SCRATCH_BYTES
    assert lb.lgs_sort_workspace_size(10_000, 50_000, 256) <= L.SORT_NOALLOC_SCRATCH_BYTES
    st = lb.lgs_sort_noalloc(n, 8, 8, None, None, None, None, None, n, None, None, None)
    assert st == L.LGS_ERR_INVALID_ARG
    msg = lb.lgs_last_error()
    assert b"scratch" in msg and str(L.SORT_NOALLOC_SCRATCH_BYTES).encode() in msg
    assert lb.lgs_sort_noalloc(-1, 8, 8, None, None, None, None, None, 0, None, None, None) == \
        L.LGS_ERR_INVALID_ARG


def test_variant_codes():
    from paper_2606_16566_amd import rasterizer as R
    L = _lib()
    assert R.variant_code("plain") == L.RENDER_PLAIN
    assert R.variant_code("local") == L.RENDER_LOCAL
    assert R.variant_code("hoist_cull_fp32") == L.RENDER_HOIST_CULL | L.RENDER_FP32


def test_batch_and_graph_arguments_rejected_on_host():
    L = _lib()
    lb = L.lib()
    cams = (L.LgsCamera * 17)()
    for c in cams:
        c.width, c.height, c.fx, c.fy = 16, 16, 100.0, 100.0
    for nv in (0, 17):
        assert lb.lgs_project_batch(cams, nv, 10, 0, *([None] * 9)) == L.LGS_ERR_INVALID_ARG
        assert lb.lgs_render_batch(3, cams, nv, *([None] * 7), None, None, 0, None, 0, None) == L.LGS_ERR_INVALID_ARG
        assert lb.lgs_render_backward_batch(3, cams, nv, 10, *([None] * 10), 0, None, None, 0, None) == \
            L.LGS_ERR_INVALID_ARG
        assert lb.lgs_project_backward_batch(cams, nv, 10, 0, *([None] * 12), 0, None) == L.LGS_ERR_INVALID_ARG
    tx = (C.c_int32 * 2)(4, 0)
    assert lb.lgs_sort_batch(2, tx, tx, 10, None, None, None, None, None, 10, None, None, None, 0, None) == \
        L.LGS_ERR_INVALID_ARG
    assert lb.lgs_graph_begin(None) == L.LGS_ERR_INVALID_ARG
    assert lb.lgs_graph_launch(None, None) == L.LGS_ERR_INVALID_ARG
    assert lb.lgs_graph_destroy(None) == L.LGS_OK
    assert lb.lgs_tile_order(None, 10, None, None, 0, None) == L.LGS_ERR_INVALID_ARG
    assert lb.lgs_tile_order_workspace_size(0) == 0
    assert lb.lgs_tile_order_workspace_size(1000) % 256 == 0
    assert lb.lgs_used_mask_words(6400, 10) == 4 * (100 + 10 + 1) and lb.lgs_used_mask_words(-1, 10) == 0


def header_arity():
    """Number of parameters of every function the header declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(lgs_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", src):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_signatures_match_header():
    L = _lib()
    ar = header_arity()
    assert set(ar) == set(declared())
    for name, n in ar.items():
        assert name in L._SIG, name
        assert len(L._SIG[name][1]) == n, (name, len(L._SIG[name][1]), n)
