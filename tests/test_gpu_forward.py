"""GPU parity of the forward path against the FP64 oracle, element by element.

Tolerances (written here, derived in the design notes):
  * colour and final T vs the oracle: max-abs 2e-4 on pixels whose skip/stop
    decisions are not within the guard of their thresholds;
  * last contributor: identical id on those pixels;
  * warp-coherent (LOCAL) vs plain per-pixel renderer: max-abs 1e-6;
  * HOIST vs HOIST_CULL: bitwise (culling removes only exact zeros);
  * projection: float32 outputs within 2 ulp of the rounded FP64 values,
    depth keys and tile rectangles identical;
  * binning (sort, ranges): bitwise.
"""
import zlib

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_16566_amd import rasterizer as R
from paper_2606_16566_amd import scenes
from tests.gpu_helpers import VARIANTS, last_ids, projected_from, render_only_case, scene_tensors, to_dev

pytestmark = pytest.mark.gpu

TOL_ORACLE = 2e-4
TOL_LADDER = 1e-6
# Decision guards (log space).  Render-only inputs and the oracle's blend of
# its own projection stored as float32 (what the render stage receives) differ
# from the GPU's inputs by at most 2 ulp of the conic, opacity and colour:
# ~1e-6 in ln alpha at the 1/255 floor (q <= 2 ln 255), plus the float32
# rounding of the log2-domain exponent and v_exp/v_log (a few ulp): 1e-5.
GUARD_RENDER = 1e-5
# Against the unrounded FP64 projection the float32 rounding of the projected
# mean (half an ulp, 6.1e-5 px at 1024..2048 px) moves q by 2 |K d| |delta|:
# 1e-4 in ln alpha for the splats that reach the floor within the image's
# pixel density (the survey's guard for the FP64 chain).
GUARD_E2E = 1e-4
MAX_FLAGGED = 1e-3        # fraction of pixels a parity gate may leave out


def check_vs_oracle(img, T, lid, ref, guard, label, lists=None, max_flagged=MAX_FLAGGED, tol=TOL_ORACLE, pix=None,
                    at=None):
    """Colour and T within `tol` and identical last contributor on pixels
    whose decisions are outside `guard`.  Flagged pixels (a decision within
    the guard): with `lists` = (W, H, offsets, ids, splats, bg) of the oracle's
    blend, each must match one of the oracle's alternative blends (every
    decision within the guard taken either way, reading of the several-
    correct-results remark), so no pixel is left out; without, they are left
    out.  At most `max_flagged` of the pixels may be flagged.  `pix` selects
    sampled pixels ([m,2] x, y) of full-image GPU outputs; `at` gives the
    pixels of outputs that are already sampled."""
    if pix is not None:
        img = img[:, pix[:, 1], pix[:, 0]]
        T = T[pix[:, 1], pix[:, 0]]
        lid = lid[pix[:, 1], pix[:, 0]]
        at = pix
    flag = O.flagged(ref["margin"], guard)
    ok = ~flag
    e_img = float(np.abs(img - ref["image"])[:, ok].max()) if ok.any() else 0.0
    e_T = float(np.abs(T - ref["T"])[ok].max()) if ok.any() else 0.0
    resolved = 0
    if lists is not None and flag.any():
        W, H, off, ids, sp, bg = lists
        for i in zip(*np.nonzero(flag)):
            if at is not None:
                x, y = int(at[i[0], 0]), int(at[i[0], 1])
                colour, t, l = img[:, i[0]], T[i[0]], lid[i[0]] if lid is not None else None
            else:
                y, x = int(i[0]), int(i[1])
                colour, t, l = img[:, y, x], T[y, x], lid[y, x] if lid is not None else None
            assert O.matches_an_alternative(W, H, off, ids, sp, bg, x, y, guard, colour, t, l, tol), \
                (label, "flagged pixel matches no alternative", x, y)
            resolved += 1
    print(f"  {label}: flagged {int(flag.sum())}/{flag.size} ({flag.mean():.2e}) at guard {guard:g}, "
          f"{resolved} matched an alternative blend; max-abs colour {e_img:.2e}, T {e_T:.2e}", flush=True)
    assert flag.mean() <= max_flagged, (label, flag.mean())
    assert e_img <= tol and e_T <= tol, (label, e_img, e_T)
    if lid is not None:
        assert np.array_equal(lid[ok], ref["last_id"][ok]), label
    return flag


def _sync_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ---------------------------------------------------------------------------
# projection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cfg,n,view,deg", [(1, 10000, 0, None), (2, 20000, 0, None), (5, 20000, 2, None),
                                            (5, 20000, 7, None), (2, 10003, 0, None), (5, 5, 1, None),
                                            (2, 8000, 0, 1), (5, 8000, 4, 2)])
def test_project_parity(cfg, n, view, deg):
    sc = scenes.make_config(cfg, n=n)
    if deg is not None:                  # a lower SH degree: the leading coefficients
        sc.sh = np.ascontiguousarray(sc.sh[:, :(deg + 1) ** 2, :])
        assert sc.sh_degree == deg
    cam = sc.cameras[view]
    print(f"project cfg={cfg} n={n} view={view} sh degree {sc.sh_degree}", flush=True)
    pr = R.project(cam, *scene_tensors(sc))
    ref = O.project_scene(sc, view)
    vis = ref["visible"] == 1
    rect = _sync_np(pr.rect)
    g_vis = (rect[:, 2] > rect[:, 0]) & (rect[:, 3] > rect[:, 1])
    assert vis.sum() > n // 10
    assert np.array_equal(g_vis, vis)
    assert np.array_equal(rect[vis], ref["rect"][vis])
    assert np.array_equal(_sync_np(pr.depth)[vis], ref["depth"][vis])
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    ulp = lambda a: np.spacing(np.abs(a).astype(np.float32)).astype(np.float64)
    m2 = _sync_np(pr.means2d).astype(np.float64)[vis]
    assert np.all(np.abs(m2 - f32(ref["means2d"][vis])) <= 2 * ulp(ref["means2d"][vis]))
    co = _sync_np(pr.conic_opacity).astype(np.float64)[vis]
    rc = np.concatenate([ref["conic"], ref["opacity"][:, None]], 1)[vis]
    assert np.all(np.abs(co - f32(rc)) <= 2 * ulp(rc) + 1e-30)
    # the colour is evaluated in single precision: within 96 u sum_k |sh_k| + 8 u
    # (u = 2^-24) of the exact value, the bound the kernel's sign test uses
    rgb = _sync_np(pr.rgb).astype(np.float64)[vis]
    sh_abs = np.abs(sc.sh.reshape(n, -1, 3).astype(np.float64)).sum(1)[vis]
    tol = 2 * ulp(ref["rgb"][vis]) + (96 * sh_abs + 8) * 2.0 ** -24
    assert np.all(np.abs(rgb - f32(ref["rgb"][vis])) <= tol)
    print(f"  colour error: worst {np.max(np.abs(rgb - ref['rgb'][vis]) / tol):.3f} of the bound", flush=True)


@pytest.mark.parametrize("n", [1, 5, 8, 13, 64, 70, 1003])
def test_project_writes_nothing_past_n(n):
    """The records are stored by groups of eight lanes: with n not a multiple
    of eight (or of the 64-lane wavefront) the last group is partial, and
    nothing past the n-th record, depth or rectangle may be written.  Two
    views through the batch entry point: view 0's tail borders view 1's
    head."""
    import ctypes as C
    from paper_2606_16566_amd import _lib as L
    sc = scenes.make_config(2, n=n)
    cams = [sc.cameras[0], scenes.look_at_camera((0.5, 0, 0), (0, 0, 1), 320, 200)]
    params = scene_tensors(sc)
    pad = 9
    dev = torch.device("cuda")
    splats = torch.full((2 * n + pad, L.SPLAT_FLOATS), 7.25, device=dev)
    depth = torch.full((2 * n + pad,), 7.25, device=dev)
    rect = torch.full((2 * n + pad, 4), 7, dtype=torch.int32, device=dev)
    p = lambda t: C.c_void_p(t.data_ptr())
    L.check(L.lib().lgs_project_batch(L.camera_array(cams), 2, n, sc.sh_degree, *(p(t) for t in params), p(splats),
                                      p(depth), p(rect), C.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "lgs_project_batch")
    got_s, got_d, got_r = _sync_np(splats), _sync_np(depth), _sync_np(rect)
    assert np.all(got_s[2 * n:] == 7.25) and np.all(got_d[2 * n:] == 7.25) and np.all(got_r[2 * n:] == 7)
    # every record of both views written (culled ones as zeros), each view
    # equal to its single-view projection
    assert not np.any(got_s[:2 * n] == 7.25) and not np.any(got_d[:2 * n] == 7.25)
    for v in range(2):
        one = R.project(cams[v], *params)
        assert np.array_equal(got_s[v * n:(v + 1) * n], _sync_np(one.splats))
        assert np.array_equal(got_d[v * n:(v + 1) * n], _sync_np(one.depth))
        assert np.array_equal(got_r[v * n:(v + 1) * n], _sync_np(one.rect))


# ---------------------------------------------------------------------------
# binning
# ---------------------------------------------------------------------------
def _synthetic_bins(seed, n, tiles_x, tiles_y, ties=True, wide=False):
    rng = np.random.default_rng(seed)
    vis = rng.uniform(size=n) < 0.85
    depth = (rng.choice(np.float32([1.5, 2.0, 2.25, 3.0]), n) if ties
             else rng.uniform(0.5, 20, n).astype(np.float32))
    x0 = rng.integers(0, tiles_x, n); y0 = rng.integers(0, tiles_y, n)
    if wide:                      # splats spanning up to the whole grid width
        w = rng.integers(1, tiles_x + 1, n); h = rng.integers(1, 12, n)
        x0 = np.where(rng.uniform(size=n) < 0.3, 0, x0)
    else:
        w = rng.integers(1, 6, n); h = rng.integers(1, 5, n)
    rect = np.stack([x0, y0, np.minimum(x0 + w, tiles_x), np.minimum(y0 + h, tiles_y)], 1).astype(np.int32)
    rect[~vis] = 0
    depth = np.where(vis, depth, np.float32(np.inf)).astype(np.float32)
    return vis.astype(np.int32), depth, rect


@pytest.mark.parametrize("seed,n,tx,ty,ties,wide", [
    (0, 5000, 13, 9, True, False), (1, 40000, 120, 68, False, False), (2, 3, 1, 1, True, False),
    # grids wider than 256 tiles take the duplicate-then-sort path
    (3, 70000, 300, 260, True, False), (9, 3000, 257, 20, True, True),
    # the widest grid of the column-first path, splats over many columns
    (8, 3000, 256, 30, False, True), (10, 20000, 37, 200, True, True),
    # more than 256 tile rows: 32-bit keys between the column and row passes
    (11, 20000, 40, 300, False, True),
    # above 2^22 and 2^25 pairs: the larger radix tier
    (4, 1000000, 120, 68, False, False), (5, 800000, 300, 260, True, False),
    # above 2^22 Gaussians in the column path (the larger radix tier for the
    # depth sort), with heavily tied depths
    (13, 4300000, 120, 68, True, False),
    pytest.param(6, 6000000, 300, 260, False, False, marks=pytest.mark.slow)])
def test_sort_and_ranges_parity(seed, n, tx, ty, ties, wide):
    vis, depth, rect = _synthetic_bins(seed, n, tx, ty, ties, wide)
    print(f"sort seed={seed} n={n} tiles={tx}x{ty} wide={wide}", flush=True)
    W, H = 16 * tx, 16 * ty
    cam = scenes.look_at_camera((0, 0, 0), (0, 0, 1), W, H)
    off, ids = O.tile_lists(vis, depth, rect, W, H)
    p = len(ids)
    proj = R.Projected(None, to_dev(depth), to_dev(rect))
    b = R.Binner(capacity=p + 17).run(cam, proj)
    keys = _sync_np(b.tile_keys)[:p].astype(np.int64)
    vals = _sync_np(b.values)[:p]
    assert int(b.num_pairs.item()) == p and int(b.overflow.item()) == 0
    want_keys = np.repeat(np.arange(tx * ty), np.diff(off))
    assert np.array_equal(keys, want_keys)
    assert np.array_equal(vals, ids)
    rg = _sync_np(b.ranges).astype(np.int64)
    nonempty = np.diff(off) > 0
    assert np.array_equal(rg[nonempty, 0], off[:-1][nonempty])
    assert np.array_equal(rg[nonempty, 1], off[1:][nonempty])
    assert np.all(rg[~nonempty] == 0)


def _plan_depths(case, n, rng):
    """Visible depths whose key span (largest minus smallest bit pattern)
    sets the depth passes' digit plan: 0, 1, 24, 25 and 31 bits."""
    f = lambda bits: np.array(bits, np.uint32).view(np.float32)
    if case == "equal":                          # span 0: no digit bits at all
        return np.full(n, 2.0, np.float32)
    if case == "one_bit":                        # span 1: one pass of one bit
        return f(0x40000000 + rng.integers(0, 2, n))
    if case in ("span_24", "span_25"):           # span 2^24 - 1: 6, 6, 6, 6; 2^24: 7, 6, 6, 6
        d = f(0x3F800000 + rng.integers(0, 1 << 24, n))
        d[::97] = f(0x3F800000)
        d[1::97] = f(0x3F800000 + (1 << 24) - (case == "span_24"))
        return d
    # span 31 bits: +0 and the smallest subnormal up to the largest finite
    d = np.exp(rng.uniform(np.log(1e-37), np.log(3e38), n)).astype(np.float32)
    d[::101] = 0.0
    d[1::101] = f(1)
    d[2::101] = np.finfo(np.float32).max
    return d


@pytest.mark.parametrize("case,n", [("equal", 1100000), ("one_bit", 1100000), ("span_24", 1100000),
                                    ("span_25", 1100000), ("span_31", 1100000), ("span_31", 4300000),
                                    ("single_visible", 1100000), ("all_culled", 1100000), ("span_25", 20000)])
def test_sort_depth_plans(case, n):
    """From 2^20 Gaussians the depth passes sort only the bits in which the
    visible depth keys differ: pair lists bitwise equal to the oracle's for
    key spans from 0 to 31 bits, in both radix tiers, with culled Gaussians
    mixed in (and once below 2^20, with 8-bit passes)."""
    rng = np.random.default_rng(zlib.crc32(case.encode()) + n)
    tx, ty = 40, 23
    vis, _, rect = _synthetic_bins(int(rng.integers(1 << 30)), n, tx, ty, ties=True)
    if case == "single_visible":
        vis[:] = 0
        vis[n // 2] = 1
        depth = np.full(n, 5.0, np.float32)
        rect[:] = 0
        rect[n // 2] = (3, 4, 9, 7)
    elif case == "all_culled":
        vis[:] = 0
        depth = np.full(n, 5.0, np.float32)
        rect[:] = 0
    else:
        depth = _plan_depths(case, n, rng)
    depth = np.where(vis > 0, depth, np.float32(np.inf)).astype(np.float32)
    print(f"sort depth plan {case} n={n}", flush=True)
    W, H = 16 * tx, 16 * ty
    cam = scenes.look_at_camera((0, 0, 0), (0, 0, 1), W, H)
    off, ids = O.tile_lists(vis, depth, rect, W, H)
    p = len(ids)
    b = R.Binner(capacity=p + 9).run(cam, R.Projected(None, to_dev(depth), to_dev(rect)))
    assert int(b.num_pairs.item()) == p and int(b.overflow.item()) == 0
    if p == 0:
        assert np.all(_sync_np(b.ranges) == 0)
        return
    assert np.array_equal(_sync_np(b.tile_keys)[:p].astype(np.int64), np.repeat(np.arange(tx * ty), np.diff(off)))
    assert np.array_equal(_sync_np(b.values)[:p], ids)


@pytest.mark.parametrize("tx,ty", [(256, 256), (256, 257)])
def test_sort_extreme_rectangles(tx, ty):
    # rectangles at the limits of the 32-bit packed form (256 x 256 tiles):
    # the whole grid, the last column and row, full-height and full-width
    # strips; with 257 rows the rectangles stay 16-byte records
    rng = np.random.default_rng(12)
    fixed = [(0, 0, tx, ty), (tx - 1, ty - 1, tx, ty), (tx - 1, 0, tx, ty), (0, ty - 1, tx, ty),
             (0, 0, 1, 1), (3, 0, 4, ty), (0, 7, tx, 8), (5, 5, 5, 9), (2, 2, 9, 2)]
    n = 400
    x0 = rng.integers(0, tx, n); y0 = rng.integers(0, ty, n)
    x1 = np.minimum(x0 + rng.integers(1, 40, n), tx); y1 = np.minimum(y0 + rng.integers(1, 40, n), ty)
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    rect[:len(fixed)] = np.array(fixed, np.int32)
    vis = ((rect[:, 2] > rect[:, 0]) & (rect[:, 3] > rect[:, 1])).astype(np.int32)
    depth = np.where(vis > 0, rng.uniform(0.5, 20, n), np.inf).astype(np.float32)
    print(f"sort extreme rectangles tiles={tx}x{ty}", flush=True)
    W, H = 16 * tx, 16 * ty
    cam = scenes.look_at_camera((0, 0, 0), (0, 0, 1), W, H)
    off, ids = O.tile_lists(vis, depth, rect, W, H)
    p = len(ids)
    b = R.Binner(capacity=p + 5).run(cam, R.Projected(None, to_dev(depth), to_dev(rect)))
    assert int(b.num_pairs.item()) == p and int(b.overflow.item()) == 0
    assert np.array_equal(_sync_np(b.tile_keys)[:p].astype(np.int64), np.repeat(np.arange(tx * ty), np.diff(off)))
    assert np.array_equal(_sync_np(b.values)[:p], ids)


@pytest.mark.parametrize("case", ["gaps", "one", "none", "overflow", "first_last"])
def test_tile_ranges_write_every_tile(case):
    """lgs_tile_ranges over a buffer holding garbage: runs get [start, end),
    every other tile (0, 0), with or without pairs, and on overflow."""
    import ctypes as C
    from paper_2606_16566_amd import _lib as L
    rng = np.random.default_rng(3)
    tiles = 700
    if case == "gaps":
        keys = np.sort(rng.choice(np.arange(3, 650), 5000))
    elif case == "one":
        keys = np.array([417])
    elif case == "first_last":
        keys = np.sort(np.concatenate([np.zeros(7, int), np.full(5, tiles - 1), rng.choice(tiles, 300)]))
    else:
        keys = np.sort(rng.choice(tiles, 900))
    n = 0 if case == "none" else len(keys)
    cap = max(len(keys), 1) - (1 if case == "overflow" else 0)
    k_dev = to_dev(np.resize(keys.astype(np.uint32), max(cap, 1)).view(np.int32))
    npairs = to_dev(np.array([n if case != "overflow" else len(keys)], np.int64))
    ovf = to_dev(np.array([1 if case == "overflow" else 0], np.int32))
    ranges = torch.full((tiles, 2), -1, dtype=torch.int32, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())
    L.check(L.lib().lgs_tile_ranges(p(k_dev), p(npairs), p(ovf), cap, tiles, p(ranges),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream)), "lgs_tile_ranges")
    got = _sync_np(ranges).astype(np.int64)
    want = np.zeros((tiles, 2), np.int64)
    if case not in ("none", "overflow"):
        for t in np.unique(keys):
            idx = np.nonzero(keys == t)[0]
            want[t] = (idx[0], idx[-1] + 1)
    assert np.array_equal(got, want)


def test_sort_overflow_flag_and_empty():
    vis, depth, rect = _synthetic_bins(7, 2000, 20, 10)
    cam = scenes.look_at_camera((0, 0, 0), (0, 0, 1), 320, 160)
    off, ids = O.tile_lists(vis, depth, rect, 320, 160)
    proj = R.Projected(None, to_dev(depth), to_dev(rect))
    binner = R.Binner(capacity=len(ids) // 3)
    b = binner.run(cam, proj, check_overflow=False)
    assert int(b.overflow.item()) == 1 and int(b.num_pairs.item()) == len(ids)
    assert np.all(_sync_np(b.ranges) == 0)
    b = binner.run(cam, proj, check_overflow=True)          # grows and retries
    assert int(b.overflow.item()) == 0 and binner.capacity >= len(ids)
    assert np.array_equal(_sync_np(b.values)[:len(ids)], ids)
    # no Gaussian at all
    e = R.Projected(None, to_dev(np.zeros(0, np.float32)), to_dev(np.zeros((0, 4), np.int32)))
    b = R.Binner(capacity=16).run(cam, e)
    assert int(b.num_pairs.item()) == 0 and np.all(_sync_np(b.ranges) == 0)
    # every Gaussian culled (depth +inf, empty rectangle)
    c = R.Projected(None, to_dev(np.full(3000, np.inf, np.float32)), to_dev(np.zeros((3000, 4), np.int32)))
    b = R.Binner(capacity=16).run(cam, c)
    assert int(b.num_pairs.item()) == 0 and int(b.overflow.item()) == 0 and np.all(_sync_np(b.ranges) == 0)


# ---------------------------------------------------------------------------
# blending, render-only (identical float32 inputs on both sides)
# ---------------------------------------------------------------------------
def _render_only(seed, W, H, n, sigma=(0.3, 12.0), margin=20.0):
    cam, cen, con, op, col, dep = render_only_case(seed, W, H, n, sigma, margin)
    vis, rect = O.footprint(W, H, cen, con, op)
    dep = np.where(vis == 1, dep, np.float32(np.inf)).astype(np.float32)
    off, ids = O.tile_lists(vis, dep, rect, W, H)
    ref = O.render_tiled(W, H, off, ids, cen, con, op, col, cam.bg)
    proj = projected_from(cen, con, op, col, dep, rect)
    b = R.Binner(capacity=len(ids) + 64).run(cam, proj)
    return cam, proj, b, ref


@pytest.mark.parametrize("seed,W,H,n", [(0, 100, 70, 3000), (1, 256, 256, 20000), (2, 33, 17, 400),
                                        (3, 200, 120, 60000)])
def test_render_only_ladder(seed, W, H, n):
    cam, proj, b, ref = _render_only(seed, W, H, n)
    print(f"render-only seed={seed} {W}x{H} n={n}", flush=True)
    flag = O.flagged(ref["margin"], GUARD_RENDER)
    print(f"  flagged {int(flag.sum())}/{flag.size} at guard {GUARD_RENDER:g}", flush=True)
    assert flag.mean() <= MAX_FLAGGED
    ok = ~flag
    outs = {}
    for v in VARIANTS + [v + "_fp32" for v in VARIANTS]:
        img, T, nc = R.render(v, cam, b, proj)
        outs[v] = (_sync_np(img), _sync_np(T), _sync_np(nc))
        e_img = np.abs(outs[v][0] - ref["image"])[:, ok].max()
        e_T = np.abs(outs[v][1] - ref["T"])[ok].max()
        assert e_img <= TOL_ORACLE and e_T <= TOL_ORACLE, (v, e_img, e_T)
        if not v.endswith("_fp32"):
            assert np.array_equal(outs[v][2][ok], ref["last_pos"][ok]), v
    # ablation ladder: culling never changes a result (either sub-tile shape)
    for v in ("hoist_cull", "hoist_cull_q8"):
        for k in range(3):
            assert np.array_equal(outs["hoist"][k], outs[v][k]), v
    for k in range(3):
        for v in ("local_q8", "local_v4", "local_q8_v4"):
            assert np.array_equal(outs["local"][k], outs[v][k]), v
            assert np.array_equal(outs["local_fp32"][k], outs[v + "_fp32"][k]), v
    for v in ("hoist", "hoist_cull", "local", "hoist_cull_q8", "local_q8"):
        d = np.abs(outs[v][0] - outs["plain"][0])[:, ok].max()
        assert d <= TOL_LADDER, (v, d)
        assert np.abs(outs[v][1] - outs["plain"][1])[ok].max() <= TOL_LADDER
        assert np.array_equal(outs[v][2][ok], outs["plain"][2][ok])


def test_render_termination_stack_and_clamp():
    """20 coincident splats with alpha 0.5 at the centre pixel: 13 blended."""
    W = H = 32
    n = 20
    cen = np.full((n, 2), 12.0, np.float32)
    con = np.tile(np.float32([[0.3, 0.0, 0.3]]), (n, 1))
    op = np.full(n, 0.5, np.float32)
    col = np.tile(np.float32([[0.25, 0.5, 1.0]]), (n, 1))
    dep = np.arange(1, n + 1, dtype=np.float32)
    cam = scenes.look_at_camera((0, 0, 0), (0, 0, 1), W, H)
    vis, rect = O.footprint(W, H, cen, con, op)
    proj = projected_from(cen, con, op, col, dep, rect)
    b = R.Binner(capacity=4096).run(cam, proj)
    for v in VARIANTS + ["local_fp32", "plain_fp32"]:
        img, T, nc = (_sync_np(x) for x in R.render(v, cam, b, proj))
        assert nc[12, 12] == 13, v
        # v_log_f32 / v_exp_f32 are accurate to a few ulp, so alpha = 0.5 is
        # reproduced to ~5e-7 relative and T = 0.5^13 to ~13x that
        assert T[12, 12] == pytest.approx(2.0 ** -13, rel=2e-5)
        np.testing.assert_allclose(img[:, 12, 12], np.float32([0.25, 0.5, 1.0]) * (1 - 2.0 ** -13), rtol=2e-6)


def test_render_edge_cases():
    # no Gaussians: background, T = 1, n_contrib = 0; ragged 1x1 and 17x33 images
    for (W, H) in [(1, 1), (17, 33)]:
        cam = scenes.look_at_camera((0, 0, 0), (0, 0, 1), W, H, bg=(0.5, 0.25, 1.0))
        proj = projected_from(np.zeros((0, 2)), np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)), np.zeros(0),
                              np.zeros((0, 4)))
        b = R.Binner(capacity=16).run(cam, proj)
        for v in VARIANTS:
            img, T, nc = (_sync_np(x) for x in R.render(v, cam, b, proj))
            assert np.all(T == 1.0) and np.all(nc == 0)
            assert np.all(img == np.float32([0.5, 0.25, 1.0])[:, None, None])
    # one huge splat covering everything and opaque tiny ones
    cam, proj, b, ref = _render_only(11, 150, 90, 300, sigma=(0.05, 400.0), margin=300.0)
    flag = O.flagged(ref["margin"], GUARD_RENDER)
    assert flag.mean() <= MAX_FLAGGED
    ok = ~flag
    for v in VARIANTS:
        img, T, nc = (_sync_np(x) for x in R.render(v, cam, b, proj))
        assert np.abs(img - ref["image"])[:, ok].max() <= TOL_ORACLE
        assert np.array_equal(nc[ok], ref["last_pos"][ok])


def test_render_stats_culled_fraction():
    cam, proj, b, ref = _render_only(5, 256, 256, 20000)
    st = {}
    for v in VARIANTS:
        s = torch.zeros(8, dtype=torch.int64, device="cuda")
        R.render(v, cam, b, proj, stats=s)
        st[v] = _sync_np(s)
    # the culling variants evaluate strictly fewer wavefront steps than they meet
    for v in ("hoist_cull", "local", "hoist_cull_q8", "local_q8", "local_v4", "local_q8_v4"):
        assert 0 < st[v][1] < st[v][0]
    assert st["plain"][1] == st["plain"][0] and st["hoist"][1] == st["hoist"][0]
    # every variant stages the same batches up to its own termination point
    assert st["local"][2] > 0


# ---------------------------------------------------------------------------
# whole pipeline from raw parameters
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cfg,n,view", [(1, None, 0), (2, 30000, 0), (3, 60000, 0), (5, 40000, 1)])
def test_end_to_end_parity(cfg, n, view):
    sc = scenes.make_config(cfg, n=n)
    cam = sc.cameras[view]
    print(f"end-to-end cfg={cfg} n={n} view={view}", flush=True)
    pr = O.project_scene(sc, view)
    ref = O.render_scene(sc, view, proj=pr, stored=True)      # the float32-stored projection
    ref64 = O.render_scene(sc, view, proj=pr)                  # the unrounded FP64 projection
    lists = (cam.width, cam.height, ref["offsets"], ref["ids"], ref["proj"], cam.bg)
    lists64 = (cam.width, cam.height, ref64["offsets"], ref64["ids"], ref64["proj"], cam.bg)
    imgs = {}
    for v in ("plain", "local", "local_q8", "local_q8_v4"):
        img, T, nc, (proj, b) = R.rasterize(cam, *scene_tensors(sc), variant=v)
        imgs[v] = _sync_np(img)
        lid = last_ids(b, nc, cam)
        check_vs_oracle(imgs[v], _sync_np(T), lid, ref, GUARD_RENDER, f"{v} vs stored projection", lists)
        # the float32 storage of the projected mean alone can flip a decision
        # of the unrounded projection
        check_vs_oracle(imgs[v], _sync_np(T), lid, ref64, GUARD_E2E, f"{v} vs FP64 projection", lists64,
                        max_flagged=1e-2)
    assert np.abs(imgs["local"] - imgs["plain"]).max() <= TOL_LADDER
    assert np.array_equal(imgs["local"], imgs["local_q8"])
    assert np.array_equal(imgs["local"], imgs["local_q8_v4"])


@pytest.mark.slow
def test_full_size_sampled_parity():
    """Configuration-2 workload at full size (1M Gaussians, SH degree 3,
    1920x1080) through the benchmark's pipeline (ViewBatch) in every render
    setting the autotuner may pick (all bitwise equal), checked on sampled
    pixels that the oracle renders one by one."""
    from paper_2606_16566_amd import autotune
    from paper_2606_16566_amd.batch import ViewBatch
    sc = scenes.make_config(2)
    cam = sc.cameras[0]
    print("full-size sampled c2", flush=True)
    params = scene_tensors(sc)
    vb = ViewBatch([cam], sc.n, sc.sh_degree)
    vb.fit(params)
    outs = []
    for cfg in autotune.space("local"):
        if cfg["precision"] != "fp64" or (cfg["persistent"] and cfg["blocks_per_cu"] != 4):
            continue
        autotune.apply(vb, cfg)
        vb.forward(params)
        outs.append((vb.image(0).clone(), vb.final_T(0).clone(), vb.n_contrib(0).clone()))
    for o in outs[1:]:
        for k in range(3):
            assert torch.equal(o[k], outs[0][k])
    img, T, nc = _sync_np(outs[0][0]), _sync_np(outs[0][1]), outs[0][2]
    b = R.Binned(vb.keys, vb.vals, vb.num_pairs, vb.overflow, vb.ranges, vb.capacity)
    pr = O.project_scene(sc)
    off, ids = O.tile_lists(pr["visible"], pr["depth"], pr["rect"], cam.width, cam.height)
    assert int(b.num_pairs.item()) == len(ids)
    rng = np.random.default_rng(0)
    pix = np.stack([rng.integers(0, cam.width, 3000), rng.integers(0, cam.height, 3000)], 1)
    edges = np.array([[0, 0], [cam.width - 1, cam.height - 1], [15, 16], [16, 15], [cam.width - 1, 0]])
    pix = np.concatenate([pix, edges]).astype(np.int32)
    lid = last_ids(b, nc, cam)
    st = O.stored_projection(pr)
    ref = O.render_tiled(cam.width, cam.height, off, ids, st["means2d"], st["conic"], st["opacity"], st["rgb"],
                         cam.bg, pixels=pix)
    check_vs_oracle(img, T, lid, ref, GUARD_RENDER, "c2 full size vs stored projection",
                    (cam.width, cam.height, off, ids, st, cam.bg), max_flagged=1e-2, pix=pix)
    ref64 = O.render_tiled(cam.width, cam.height, off, ids, pr["means2d"], pr["conic"], pr["opacity"], pr["rgb"],
                           cam.bg, pixels=pix)
    check_vs_oracle(img, T, lid, ref64, GUARD_E2E, "c2 full size vs FP64 projection",
                    (cam.width, cam.height, off, ids, pr, cam.bg), max_flagged=1e-2, pix=pix)


# ---------------------------------------------------------------------------
# exact tile assignment
# ---------------------------------------------------------------------------
def _gpu_lists(b, num_tiles):
    rg = _sync_np(b.ranges).astype(np.int64) & 0xFFFFFFFF
    vals = _sync_np(b.values).astype(np.int64) & 0xFFFFFFFF
    return [vals[rg[t, 0]:rg[t, 1]] for t in range(num_tiles)]


@pytest.mark.parametrize("seed,W,H,n,sigma", [(40, 160, 96, 6000, (0.3, 20.0)), (41, 333, 97, 3000, (0.05, 150.0)),
                                              (42, 64, 64, 400, (2.0, 60.0))])
def test_exact_tile_assignment_lists(seed, W, H, n, sigma):
    """Exact mode: every tile's list is an ordered subsequence of its
    rectangle list, holds every splat whose alpha >= 1/255 ellipse meets the
    tile's pixel centres (the oracle's exact rule without slack), and only
    splats whose barely larger ellipse meets the tile's square (the oracle's
    loose rule)."""
    cam, cen, con, op, col, dep = render_only_case(seed, W, H, n, sigma=sigma, margin=40.0)
    vis, rect = O.footprint(W, H, cen, con, op)
    dep = np.where(vis == 1, dep, np.float32(np.inf)).astype(np.float32)
    off_r, ids_r = O.tile_lists(vis, dep, rect, W, H)
    off_p, ids_p = O.tile_lists_exact(vis, dep, rect, cen, con, op, W, H, tau_rel=0.0, tau_abs=0.0, pad=0.0, clip=True)
    off_l, ids_l = O.tile_lists_exact(vis, dep, rect, cen, con, op, W, H, **O.EXACT_LOOSE)
    proj = projected_from(cen, con, op, col, dep, rect)
    b = R.Binner(capacity=len(ids_r) + 64, exact=True).run(cam, proj)
    P = int(b.num_pairs.item())
    print(f"exact lists seed={seed}: rectangle pairs {len(ids_r)}, exact {P}, pure {len(ids_p)}, loose {len(ids_l)}",
          flush=True)
    assert len(ids_p) <= P <= len(ids_l) and P < len(ids_r)
    got = _gpu_lists(b, cam.num_tiles)
    for t in range(cam.num_tiles):
        r = ids_r[off_r[t]:off_r[t + 1]]
        g = got[t]
        keep = np.isin(r, g)
        assert np.array_equal(r[keep], g), t                      # ordered subsequence
        assert set(ids_p[off_p[t]:off_p[t + 1]]) <= set(g.tolist()) <= set(ids_l[off_l[t]:off_l[t + 1]]), t


@pytest.mark.parametrize("cfg,n,view", [(2, 30000, 0), (3, 60000, 0), (4, 50000, 0)])
def test_exact_tiles_render_identically(cfg, n, view):
    """Exact mode removes only list entries that no pixel of the tile blends:
    images and T are bitwise those of the rectangle mode, every pixel has the
    same last contributor, and the image matches the oracle."""
    sc = scenes.make_config(cfg, n=n)
    cam = sc.cameras[view]
    ps = scene_tensors(sc)
    res = {}
    for exact in (False, True):
        for v in ("plain", "local_q8_v4"):
            img, T, nc, (proj, b) = R.rasterize(cam, *ps, variant=v, binner=R.Binner(exact=exact))
            res[exact, v] = (_sync_np(img), _sync_np(T), last_ids(b, nc, cam), int(b.num_pairs.item()))
    print(f"exact cfg={cfg}: pairs {res[False, 'plain'][3]} -> {res[True, 'plain'][3]}", flush=True)
    assert res[True, "plain"][3] < res[False, "plain"][3]
    for v in ("plain", "local_q8_v4"):
        for k in range(3):
            assert np.array_equal(res[False, v][k], res[True, v][k]), (v, k)
    ref = O.render_scene(sc, view, stored=True)
    img, T, lid, _ = res[True, "local_q8_v4"]
    check_vs_oracle(img, T, lid, ref, GUARD_RENDER, f"exact cfg={cfg} vs stored projection",
                    (cam.width, cam.height, ref["offsets"], ref["ids"], ref["proj"], cam.bg))
