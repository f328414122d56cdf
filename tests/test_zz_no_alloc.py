"""lgs_sort_noalloc, the sort on the library's own scratch (for callers that
cannot allocate), against lgs_sort with a caller workspace, through the C
ABI: bitwise-equal pairs, pair count and overflow flag on two calls in a row,
the second with a smaller input (the scratch keeps the first call's
contents), the overflow case, and the oracle's tile lists."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_16566_amd import _lib as L

pytestmark = pytest.mark.gpu


def _bins(seed, n, tiles_x, tiles_y):
    rng = np.random.default_rng(seed)
    vis = rng.uniform(size=n) < 0.85
    depth = rng.choice(np.float32([1.5, 2.0, 2.25, 3.0]), n)          # many ties
    x0 = rng.integers(0, tiles_x, n)
    y0 = rng.integers(0, tiles_y, n)
    w = rng.integers(1, 6, n)
    h = rng.integers(1, 5, n)
    rect = np.stack([x0, y0, np.minimum(x0 + w, tiles_x), np.minimum(y0 + h, tiles_y)], 1).astype(np.int32)
    rect[~vis] = 0
    depth = np.where(vis, depth, np.float32(np.inf)).astype(np.float32)
    return vis.astype(np.int32), depth, rect


def _p(t):
    return C.c_void_p(t.data_ptr())


def _sort(entry, n, tx, ty, depth, rect, cap):
    lb = L.lib()
    dev = torch.device("cuda")
    keys = torch.full((max(cap, 1),), -1, dtype=torch.int32, device=dev)
    vals = torch.full((max(cap, 1),), -1, dtype=torch.int32, device=dev)
    npairs = torch.full((1,), -1, dtype=torch.int64, device=dev)
    ovf = torch.full((1,), -1, dtype=torch.int32, device=dev)
    d = torch.from_numpy(depth).to(dev)
    r = torch.from_numpy(rect).to(dev)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if entry == "lgs_sort":
        need = lb.lgs_sort_workspace_size(n, cap, tx * ty)
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        base = ws.data_ptr()
        aligned = (base + 255) & ~255
        st = lb.lgs_sort(n, tx, ty, _p(d), _p(r), None, _p(keys), _p(vals), cap, _p(npairs), _p(ovf),
                         C.c_void_p(aligned), ws.numel() - (aligned - base), stream)
    else:
        st = lb.lgs_sort_noalloc(n, tx, ty, _p(d), _p(r), None, _p(keys), _p(vals), cap, _p(npairs), _p(ovf),
                                 stream)
    assert st == L.LGS_OK, lb.lgs_last_error()
    torch.cuda.synchronize()
    return keys.cpu().numpy(), vals.cpu().numpy(), int(npairs.item()), int(ovf.item())


def test_sort_noalloc_matches_workspace_sort():
    # the second call is smaller: its result must not depend on what the
    # first one left in the scratch
    for seed, n, tx, ty in [(21, 150000, 120, 68), (22, 7000, 37, 23)]:
        print(f"noalloc sort seed={seed} n={n} tiles={tx}x{ty}", flush=True)
        vis, depth, rect = _bins(seed, n, tx, ty)
        off, ids = O.tile_lists(vis, depth, rect, 16 * tx, 16 * ty)
        p = len(ids)
        cap = p + 100
        assert L.lib().lgs_sort_workspace_size(n, cap, tx * ty) <= L.SORT_NOALLOC_SCRATCH_BYTES
        a = _sort("lgs_sort_noalloc", n, tx, ty, depth, rect, cap)
        b = _sort("lgs_sort", n, tx, ty, depth, rect, cap)
        assert a[2] == b[2] == p and a[3] == b[3] == 0
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])      # tails untouched alike
        assert np.array_equal(a[1][:p], ids)
        assert np.array_equal(a[0][:p].astype(np.int64), np.repeat(np.arange(tx * ty), np.diff(off)))


def test_sort_noalloc_overflow_and_limit():
    vis, depth, rect = _bins(23, 20000, 50, 40)
    off, ids = O.tile_lists(vis, depth, rect, 800, 640)
    p = len(ids)
    a = _sort("lgs_sort_noalloc", 20000, 50, 40, depth, rect, p // 2)
    b = _sort("lgs_sort", 20000, 50, 40, depth, rect, p // 2)
    assert a[2] == b[2] == p and a[3] == b[3] == 1
    # a size beyond the scratch is refused on the host with the sizes named
    lb = L.lib()
    big = 4_000_000
    assert lb.lgs_sort_workspace_size(big, big, 64) > L.SORT_NOALLOC_SCRATCH_BYTES
    st = lb.lgs_sort_noalloc(big, 8, 8, None, None, None, None, None, big, None, None, None)
    assert st == L.LGS_ERR_INVALID_ARG and b"scratch" in lb.lgs_last_error()
