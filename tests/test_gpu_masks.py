"""The wavefront culling decisions themselves (Sec. III-C: tight vertical span
of the alpha >= 1/255 ellipse over a sub-tile's columns, cases A/B/C, and the
warp mask).  lgs_render_debug records, per list entry and wavefront sub-tile,
whether the render kernel tested the entry and whether it kept it.

Pinned here, in FP64 on the same float32 splats: every entry a wavefront
culled has alpha < 1/255 at every pixel of that sub-tile ("culled is a subset
of skipped"), for 16x4 strips and 8x8 quadrants, HOIST_CULL and LOCAL.  The
splats are drawn so that each case of the span (peak left of the columns,
right of them, inside them, and an ellipse that misses the columns though its
bounding box covers the tile) occurs, plus adversarial ones: tops and sides
within 1e-3 px of a pixel-centre row or column, nearly degenerate conics
(b^2 close to ac, axis ratios up to 2000) and the largest tau (opacity ~1).
The per-case counts and the tightness (kept entries whose sub-tile has no
pixel at alpha >= 1/255) are printed.
"""
import ctypes as C
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_16566_amd import _lib as L
from paper_2606_16566_amd import rasterizer as R
from paper_2606_16566_amd import scenes
from tests.gpu_helpers import projected_from

pytestmark = pytest.mark.gpu

W, H = 160, 100


def _conic(s1, s2, th):
    c, s = np.cos(th), np.sin(th)
    sxx = c * c * s1 ** 2 + s * s * s2 ** 2
    syy = s * s * s1 ** 2 + c * c * s2 ** 2
    sxy = c * s * (s1 ** 2 - s2 ** 2)
    det = sxx * syy - sxy * sxy
    return np.stack([syy / det, -sxy / det, sxx / det], -1)


def _splats(seed):
    rng = np.random.default_rng(seed)
    parts = []
    # general population: rotated ellipses from 0.05 to 150 px, axis ratio up to 30
    n = 2500
    s1 = np.exp(rng.uniform(np.log(0.05), np.log(150.0), n))
    s2 = s1 / np.exp(rng.uniform(0, np.log(30.0), n))
    parts.append((np.stack([rng.uniform(-30, W + 30, n), rng.uniform(-30, H + 30, n)], 1),
                  _conic(s1, s2, rng.uniform(0, np.pi, n)), np.exp(rng.uniform(np.log(0.01), 0, n))))
    # nearly degenerate conics: thin needles at all angles (b^2 close to ac)
    n = 500
    s1 = np.exp(rng.uniform(np.log(3.0), np.log(80.0), n))
    s2 = s1 / np.exp(rng.uniform(np.log(200.0), np.log(2000.0), n))
    parts.append((np.stack([rng.uniform(0, W, n), rng.uniform(0, H, n)], 1),
                  _conic(s1, s2, rng.uniform(0, np.pi, n)), rng.uniform(0.3, 0.999, n)))
    # near-tangent: axis-aligned and rotated ellipses whose top (or left side)
    # lies within 1e-3 px of a pixel-centre row (column), largest tau
    n = 800
    s1 = np.exp(rng.uniform(np.log(0.6), np.log(20.0), n))
    s2 = s1 / np.exp(rng.uniform(0, np.log(4.0), n))
    th = np.where(rng.uniform(size=n) < 0.5, 0.0, rng.uniform(0, np.pi, n))
    con = _conic(s1, s2, th)
    op = np.where(rng.uniform(size=n) < 0.5, 0.9999, rng.uniform(0.05, 0.99, n))
    tau = 2 * np.log(255 * op)
    a, b, c = con[:, 0], con[:, 1], con[:, 2]
    det = a * c - b * b
    ymax = np.sqrt(a * tau / det)                   # half height of the ellipse
    xmax = np.sqrt(c * tau / det)                   # half width
    row = rng.integers(0, H, n)
    col = rng.integers(0, W, n)
    eps = rng.uniform(-1e-3, 1e-3, n)
    vertical = rng.uniform(size=n) < 0.5
    cy = np.where(vertical, row - ymax + eps, rng.uniform(0, H, n))   # top touches row `row`
    cx = np.where(vertical, rng.uniform(0, W, n), col - xmax + eps)   # right side touches column `col`
    parts.append((np.stack([cx, cy], 1), con, op))
    cen = np.concatenate([p[0] for p in parts]).astype(np.float32)
    conic = np.concatenate([p[1] for p in parts]).astype(np.float32)
    opac = np.concatenate([p[2] for p in parts]).astype(np.float32)
    m = len(opac)
    col = rng.uniform(0, 1, (m, 3)).astype(np.float32)
    dep = rng.uniform(1, 10, m).astype(np.float32)
    return cen, conic, opac, col, dep


def _subtile(tx, ty, w, q8):
    if q8:
        x0, y0 = tx * 16 + 8 * (w & 1), ty * 16 + 8 * (w >> 1)
        x1, y1 = x0 + 7, y0 + 7
    else:
        x0, y0 = tx * 16, ty * 16 + 4 * w
        x1, y1 = x0 + 15, y0 + 3
    return x0, min(x1, W - 1), y0, min(y1, H - 1)


def _span_case(a, b, c, tau, X0, X1):
    """Which case of the tight span applies at the top of the ellipse over the
    columns [X0, X1] (relative to its centre): 'A' peak left, 'B' peak
    right, 'C' inside, 'empty' the ellipse misses the columns."""
    det = a * c - b * b
    half_w = math.sqrt(c * tau / det)
    if X1 < -half_w or X0 > half_w:
        return "empty"
    xpeak = -b * math.sqrt(a * tau / det) / a
    return "A" if xpeak < X0 else ("B" if xpeak > X1 else "C")


@pytest.mark.parametrize("variant", ["hoist_cull", "hoist_cull_q8", "local", "local_q8"])
def test_culled_entries_are_skipped_entries(variant):
    cen, conic, opac, col, dep = _splats(3)
    cam = scenes.look_at_camera((0, 0, 0), (0, 0, 1), W, H)
    vis, rect = O.footprint(W, H, cen, conic, opac)
    dep = np.where(vis == 1, dep, np.float32(np.inf)).astype(np.float32)
    off, ids = O.tile_lists(vis, dep, rect, W, H)
    P = len(ids)
    proj = projected_from(cen, conic, opac, col, dep, rect)
    b = R.Binner(capacity=P + 64).run(cam, proj)
    dev = torch.device("cuda")
    masks = torch.zeros(P + 64, dtype=torch.int32, device=dev)
    stats = torch.zeros(8, dtype=torch.int64, device=dev)
    img = torch.empty((3, H, W), device=dev)
    T = torch.empty((H, W), device=dev)
    nc = torch.empty((H, W), dtype=torch.int32, device=dev)
    p = lambda t: C.c_void_p(t.data_ptr())
    st = L.lib().lgs_render_debug(R.variant_code(variant), C.byref(L.camera_struct(cam)), 1, p(b.ranges), p(b.values),
                                  p(proj.splats), p(img), p(T), p(nc), p(stats),
                                  p(masks), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.LGS_OK, L.lib().lgs_last_error()
    torch.cuda.synchronize()
    mk = masks.cpu().numpy()[:P].astype(np.int64)
    keys = b.tile_keys.cpu().numpy()[:P].astype(np.int64)
    vals = b.values.cpu().numpy()[:P].astype(np.int64)
    assert np.array_equal(vals, ids)
    q8 = "_q8" in variant
    tiles_x = cam.tiles_x
    cen64, con64, op64 = cen.astype(np.float64), conic.astype(np.float64), opac.astype(np.float64)
    cases = {"A": 0, "B": 0, "C": 0, "empty": 0}
    culled = kept = loose = 0
    for j in range(P):
        m = int(mk[j])
        if m == 0:
            continue
        g = int(vals[j])
        tx, ty = int(keys[j]) % tiles_x, int(keys[j]) // tiles_x
        a, bb, c = con64[g]
        tau = 2.0 * math.log(255.0 * op64[g])
        for w in range(4):
            if not (m >> w) & 1:
                continue
            x0, x1, y0, y1 = _subtile(tx, ty, w, q8)
            cases[_span_case(a, bb, c, tau, x0 - cen64[g, 0], x1 - cen64[g, 0])] += 1
            xs, ys = np.meshgrid(np.arange(x0, x1 + 1, dtype=np.float64), np.arange(y0, y1 + 1, dtype=np.float64))
            dx, dy = xs - cen64[g, 0], ys - cen64[g, 1]
            al = op64[g] * np.exp(-0.5 * (a * dx * dx + 2 * bb * dx * dy + c * dy * dy))
            reach = bool((al >= 1.0 / 255.0).any())
            if (m >> (4 + w)) & 1:
                kept += 1
                loose += not reach
            else:
                culled += 1
                assert not reach, (variant, j, g, w, float(al.max()))
    print(f"{variant}: tested {culled + kept} (entry, sub-tile) pairs, culled {culled}; cases {cases}; "
          f"kept without a pixel at alpha >= 1/255: {loose} of {kept} ({loose / max(kept, 1):.3f})", flush=True)
    assert culled > 1000 and all(v >= 20 for v in cases.values()), cases
    s = stats.cpu().numpy()
    assert 0 < s[1] <= s[0]
