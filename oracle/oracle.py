"""ctypes front-end of the FP64 reference rasterizer (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg.  The product package never imports it.

All functions take plain numpy arrays (the float32 inputs the GPU receives,
upcast exactly to float64 inside the C code) and return numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

TILE = 16
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4


def build() -> str:
    """Compile oracle.c with gcc (no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _lib.oracle_count_pairs.restype = C.c_int64
        _lib.oracle_tile_lists.restype = C.c_int64
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def cam_block(cam) -> np.ndarray:
    """Pack a scenes.Camera into the 27-double block oracle.c reads.  Every
    value is the float32 the GPU receives, upcast exactly."""
    f = lambda x: float(np.float32(x))
    blk = np.zeros(27, dtype=np.float64)
    blk[0:12] = np.asarray(cam.viewmat, dtype=np.float32).reshape(12)
    blk[12:15] = np.asarray(cam.campos, dtype=np.float32)
    blk[15], blk[16], blk[17], blk[18] = f(cam.fx), f(cam.fy), f(cam.cx), f(cam.cy)
    blk[19], blk[20] = f(cam.tan_fovx), f(cam.tan_fovy)
    blk[21], blk[22], blk[23] = cam.width, cam.height, f(cam.znear)
    blk[24:27] = [f(b) for b in cam.bg]
    return blk


# ---------------------------------------------------------------------------
# projection
# ---------------------------------------------------------------------------
def project(cam, means3d, log_scales, quats, logits, sh) -> dict:
    n = int(means3d.shape[0])
    k = int(sh.shape[1]) if n else int(np.asarray(sh).reshape(0, -1, 3).shape[1])
    deg = int(round(np.sqrt(k))) - 1
    out = dict(visible=np.zeros(n, np.int32), means2d=np.zeros((n, 2)), conic=np.zeros((n, 3)),
               opacity=np.zeros(n), rgb=np.zeros((n, 3)), depth=np.zeros(n, np.float32),
               rect=np.zeros((n, 4), np.int32), rgb_clamped=np.zeros((n, 3), np.int32))
    a = [_f64(means3d), _f64(log_scales), _f64(quats), _f64(logits), _f64(sh)]
    lib().oracle_project(_p(cam_block(cam)), C.c_int64(n), C.c_int(deg), *map(_p, a),
                         _p(out["visible"]), _p(out["means2d"]), _p(out["conic"]), _p(out["opacity"]),
                         _p(out["rgb"]), _p(out["depth"]), _p(out["rect"]), _p(out["rgb_clamped"]))
    return out


def project_chunked(cam, means3d, log_scales, quats, logits, sh, threads=8) -> dict:
    """project() of large inputs split into chunks of Gaussians on host
    threads (the C code is reentrant and ctypes releases the GIL), results
    concatenated in order: identical to one call."""
    from concurrent.futures import ThreadPoolExecutor
    n = int(means3d.shape[0])
    chunk = max(1, -(-n // (4 * threads)))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda a: project(cam, means3d[a:a + chunk], log_scales[a:a + chunk],
                                              quats[a:a + chunk], logits[a:a + chunk], sh[a:a + chunk]),
                            range(0, max(n, 1), chunk)))
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def project_scene(scene, view=0) -> dict:
    return project(scene.cameras[view], scene.means3d, scene.log_scales, scene.quats,
                   scene.opacity_logits, scene.sh)


def project_backward(cam, means3d, log_scales, quats, logits, sh, g_means2d, g_conic, g_opacity,
                     g_rgb) -> dict:
    n = int(means3d.shape[0])
    k = int(sh.shape[1])
    deg = int(round(np.sqrt(k))) - 1
    out = dict(means3d=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), sh=np.zeros((n, k, 3)))
    a = [_f64(means3d), _f64(log_scales), _f64(quats), _f64(logits), _f64(sh)]
    g = [_f64(g_means2d), _f64(g_conic), _f64(g_opacity), _f64(g_rgb)]
    lib().oracle_project_backward(_p(cam_block(cam)), C.c_int64(n), C.c_int(deg), *map(_p, a), *map(_p, g),
                                  _p(out["means3d"]), _p(out["log_scales"]), _p(out["quats"]),
                                  _p(out["opacity_logits"]), _p(out["sh"]))
    return out


def sh_basis(deg: int, d) -> np.ndarray:
    out = np.zeros((deg + 1) ** 2)
    lib().oracle_sh_basis(C.c_int(deg), C.c_double(d[0]), C.c_double(d[1]), C.c_double(d[2]), _p(out))
    return out


# ---------------------------------------------------------------------------
# binning
# ---------------------------------------------------------------------------
def tile_lists(visible, depth, rect, width, height):
    """Per-tile Gaussian ids in ascending (depth, id) order: (offsets, ids)."""
    tx, ty = (width + TILE - 1) // TILE, (height + TILE - 1) // TILE
    visible = np.ascontiguousarray(visible, np.int32)
    rect = np.ascontiguousarray(rect, np.int32)
    depth = _f32(depth)
    n = visible.shape[0]
    p = lib().oracle_count_pairs(C.c_int64(n), _p(visible), _p(rect))
    offsets = np.zeros(tx * ty + 1, np.int64)
    ids = np.zeros(max(p, 1), np.int32)
    lib().oracle_tile_lists(C.c_int64(n), _p(visible), _p(depth), _p(rect), C.c_int(tx), C.c_int(ty),
                            _p(offsets), _p(ids))
    return offsets, ids[:p]


# exact tile assignment: the footprint's slack (as in the rectangle rule), and
# a looser ellipse that bounds any conservative float implementation of it
EXACT_TIGHT = dict(tau_rel=1e-5, tau_abs=1e-5, pad=1e-2, clip=True)
EXACT_LOOSE = dict(tau_rel=2e-3, tau_abs=2e-2, pad=2e-2, clip=False)


def rect_min_q(a, b, c, x0, x1, y0, y1) -> float:
    lib().oracle_rect_min_q.restype = C.c_double
    return lib().oracle_rect_min_q(*(C.c_double(float(v)) for v in (a, b, c, x0, x1, y0, y1)))


def tile_lists_exact(visible, depth, rect, means2d, conic, opacity, width, height, tau_rel=1e-5, tau_abs=1e-5,
                     pad=1e-2, clip=True):
    """Per-tile (depth, id)-ordered lists keeping a Gaussian only in the tiles
    of its rectangle that its alpha >= 1/255 ellipse (with the given slack)
    meets: (offsets, ids)."""
    tx, ty = (width + TILE - 1) // TILE, (height + TILE - 1) // TILE
    visible = np.ascontiguousarray(visible, np.int32)
    rect = np.ascontiguousarray(rect, np.int32)
    depth = _f32(depth)
    n = visible.shape[0]
    lb = lib()
    lb.oracle_tile_lists_exact.restype = C.c_int64
    args = [C.c_int64(n), _p(visible), _p(depth), _p(rect), _p(_f64(means2d)), _p(_f64(conic)), _p(_f64(opacity)),
            C.c_int(width), C.c_int(height), C.c_double(tau_rel), C.c_double(tau_abs), C.c_double(pad),
            C.c_int(int(clip))]
    offsets = np.zeros(tx * ty + 1, np.int64)
    p = lb.oracle_tile_lists_exact(*args, _p(offsets), None)
    ids = np.zeros(max(p, 1), np.int32)
    lb.oracle_tile_lists_exact(*args, _p(offsets), _p(ids))
    return offsets, ids[:p]


# ---------------------------------------------------------------------------
# blending
# ---------------------------------------------------------------------------
def _bg(bg):
    return _f64(np.asarray([float(np.float32(b)) for b in bg]))


def render_untiled(width, height, visible, depth, means2d, conic, opacity, rgb, bg=(0, 0, 0)) -> dict:
    n = int(np.asarray(visible).shape[0])
    hw = width * height
    out = dict(image=np.zeros((3, height, width)), T=np.zeros((height, width)),
               last_id=np.zeros((height, width), np.int32), count=np.zeros((height, width), np.int32),
               margin=np.zeros((height, width)), clamp_margin=np.zeros((height, width)))
    lib().oracle_render_untiled(C.c_int(width), C.c_int(height), C.c_int64(n),
                                _p(np.ascontiguousarray(visible, np.int32)), _p(_f32(depth)),
                                _p(_f64(means2d)), _p(_f64(conic)), _p(_f64(opacity)), _p(_f64(rgb)),
                                _p(_bg(bg)), _p(out["image"]), _p(out["T"]), _p(out["last_id"]),
                                _p(out["count"]), _p(out["margin"]), _p(out["clamp_margin"]))
    assert hw == out["T"].size
    return out


def render_tiled(width, height, offsets, ids, means2d, conic, opacity, rgb, bg=(0, 0, 0),
                 pixels=None) -> dict:
    """Blend every pixel (or only `pixels`, an [m,2] int array of (x, y)) over
    its tile's list.  Full-image outputs are [3,H,W] / [H,W]; sampled outputs
    are [3,m] / [m]."""
    if pixels is None:
        shape2, m, pix = (height, width), width * height, None
    else:
        pix = np.ascontiguousarray(pixels, np.int32)
        m = pix.shape[0]
        shape2 = (m,)
    out = dict(image=np.zeros((3,) + shape2), T=np.zeros(shape2), last_pos=np.zeros(shape2, np.int32),
               last_id=np.zeros(shape2, np.int32), count=np.zeros(shape2, np.int32),
               margin=np.zeros(shape2), clamp_margin=np.zeros(shape2))
    ids = np.ascontiguousarray(ids, np.int32) if len(ids) else np.zeros(1, np.int32)
    lib().oracle_render_tiled(C.c_int(width), C.c_int(height), _p(np.ascontiguousarray(offsets, np.int64)),
                              _p(ids), _p(_f64(means2d)), _p(_f64(conic)), _p(_f64(opacity)),
                              _p(_f64(rgb)), _p(_bg(bg)), None if pix is None else _p(pix), C.c_int64(m),
                              _p(out["image"]), _p(out["T"]), _p(out["last_pos"]), _p(out["last_id"]),
                              _p(out["count"]), _p(out["margin"]), _p(out["clamp_margin"]))
    return out


def render_backward(width, height, offsets, ids, means2d, conic, opacity, rgb, gC, gT=None,
                    bg=(0, 0, 0)) -> dict:
    n = int(np.asarray(opacity).shape[0])
    out = dict(means2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n), rgb=np.zeros((n, 3)))
    ids = np.ascontiguousarray(ids, np.int32) if len(ids) else np.zeros(1, np.int32)
    lib().oracle_render_backward(C.c_int(width), C.c_int(height), _p(np.ascontiguousarray(offsets, np.int64)),
                                 _p(ids), C.c_int64(n), _p(_f64(means2d)), _p(_f64(conic)),
                                 _p(_f64(opacity)), _p(_f64(rgb)), _p(_bg(bg)), _p(_f64(gC)),
                                 None if gT is None else _p(_f64(gT)), _p(out["means2d"]), _p(out["conic"]),
                                 _p(out["opacity"]), _p(out["rgb"]))
    return out


# ---------------------------------------------------------------------------
# whole pipeline helpers
# ---------------------------------------------------------------------------
def stored_projection(pr) -> dict:
    """The projection as the rasterizer's interface stores it: the FP64
    projected attributes (mean, conic, opacity, colour) rounded to float32 and
    upcast exactly; visibility, depth keys and tile rectangles unchanged.  The
    blend of these is the plain definition applied to float32 projected
    splats, which is what the render stage receives."""
    out = dict(pr)
    for k in ("means2d", "conic", "opacity", "rgb"):
        out[k] = np.asarray(pr[k], np.float64).astype(np.float32).astype(np.float64)
    return out


def render_scene(scene, view=0, proj=None, tiled=True, stored=False) -> dict:
    """Project and blend a whole scene in FP64 from its raw parameters
    (stored=True: blend the float32-stored projection, see stored_projection)."""
    cam = scene.cameras[view]
    pr = proj if proj is not None else project_scene(scene, view)
    if stored:
        pr = stored_projection(pr)
    if tiled:
        off, ids = tile_lists(pr["visible"], pr["depth"], pr["rect"], cam.width, cam.height)
        out = render_tiled(cam.width, cam.height, off, ids, pr["means2d"], pr["conic"], pr["opacity"],
                           pr["rgb"], cam.bg)
        out["offsets"], out["ids"] = off, ids
    else:
        out = render_untiled(cam.width, cam.height, pr["visible"], pr["depth"], pr["means2d"], pr["conic"],
                             pr["opacity"], pr["rgb"], cam.bg)
    out["proj"] = pr
    return out


def scene_gradients(scene, gC, gT=None, view=0, stored=False) -> dict:
    """dL/d(raw parameters) for L = sum(gC * image) + sum(gT * T_final)
    (stored=True: the blend's gradient is taken at the float32-stored
    projection, see stored_projection; the chain through the projection is
    FP64 either way)."""
    cam = scene.cameras[view]
    pr = project_scene(scene, view)
    off, ids = tile_lists(pr["visible"], pr["depth"], pr["rect"], cam.width, cam.height)
    bl = stored_projection(pr) if stored else pr
    g2 = render_backward(cam.width, cam.height, off, ids, bl["means2d"], bl["conic"], bl["opacity"],
                         bl["rgb"], gC, gT, cam.bg)
    g3 = project_backward(cam, scene.means3d, scene.log_scales, scene.quats, scene.opacity_logits,
                          scene.sh, g2["means2d"], g2["conic"], g2["opacity"], g2["rgb"])
    g3["projected"] = g2
    return g3


def footprint(width, height, means2d, conic, opacity):
    """(visible [n] int32, rect [n,4] int32) of screen-space splats."""
    n = int(np.asarray(opacity).shape[0])
    vis = np.zeros(n, np.int32)
    rect = np.zeros((n, 4), np.int32)
    lib().oracle_footprint(C.c_int(width), C.c_int(height), C.c_int64(n), _p(_f64(means2d)), _p(_f64(conic)),
                           _p(_f64(opacity)), _p(vis), _p(rect))
    return vis, rect


def blend_alternatives(width, height, offsets, ids, means2d, conic, opacity, rgb, bg, x, y, guard, max_alts=64):
    """All outcomes of pixel (x, y)'s blend when each decision within `guard`
    of its threshold may go either way: (image [m,3], T [m], last id [m]);
    raises if there are more than max_alts."""
    img = np.zeros((max_alts, 3))
    T = np.zeros(max_alts)
    lid = np.zeros(max_alts, np.int32)
    ids = np.ascontiguousarray(ids, np.int32) if len(ids) else np.zeros(1, np.int32)
    lib().oracle_blend_alternatives.restype = C.c_int
    m = lib().oracle_blend_alternatives(C.c_int(width), C.c_int(height), _p(np.ascontiguousarray(offsets, np.int64)),
                                        _p(ids), _p(_f64(means2d)), _p(_f64(conic)), _p(_f64(opacity)), _p(_f64(rgb)),
                                        _p(_bg(bg)), C.c_int(int(x)), C.c_int(int(y)), C.c_double(guard),
                                        C.c_int(max_alts), _p(img), _p(T), _p(lid))
    if m < 0:
        raise ValueError(f"more than {max_alts} alternative blends at pixel ({x}, {y})")
    return img[:m], T[:m], lid[:m]


def matches_an_alternative(width, height, offsets, ids, splats, bg, x, y, guard, colour, T, last_id, tol):
    """Does a blend result (colour [3], T, last contributor id) match one of
    the alternatives of pixel (x, y) within tol (and the id exactly)?"""
    img, Ts, lids = blend_alternatives(width, height, offsets, ids, splats["means2d"], splats["conic"],
                                       splats["opacity"], splats["rgb"], bg, x, y, guard)
    ok = (np.abs(img - np.asarray(colour)[None, :]).max(1) <= tol) & (np.abs(Ts - T) <= tol)
    if last_id is not None:
        ok &= lids == last_id
    return bool(ok.any())


def flagged(margin, guard):
    """Pixels whose blend took a skip / stop decision within `guard` (log
    space) of its threshold: either outcome is a correct result there."""
    return np.asarray(margin) < guard


def grad_flagged(out, guard):
    """Pixels to leave out of gradient comparisons: a skip / stop decision or
    the 0.99 clamp of a blended Gaussian (where the derivative switches)
    within `guard` (log space) of its threshold."""
    return (np.asarray(out["margin"]) < guard) | (np.asarray(out["clamp_margin"]) < guard)
