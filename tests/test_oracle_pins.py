"""Pins of the FP64 reference against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an invariant, a special case, brute force, or finite differences of its
own forward pass (for the analytic gradients).  None of these needs a GPU.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2606_16566_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cam(w=64, h=64, fov=60.0, pos=(0, 0, 0), target=(0, 0, 1), bg=(0, 0, 0)):
    return scenes.look_at_camera(pos, target, w, h, fov, bg=bg)


def _one(mean, log_scale, quat=(1, 0, 0, 0), logit=2.0, sh=None):
    sh = np.zeros((1, 1, 3), np.float32) if sh is None else np.asarray(sh, np.float32)[None]
    return (np.asarray([mean], np.float64), np.asarray([log_scale], np.float64),
            np.asarray([quat], np.float64), np.asarray([logit], np.float64), sh)


# ---------------------------------------------------------------------------
# constants the paper prints
# ---------------------------------------------------------------------------
def test_paper_constants(oracle):
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert oracle.ALPHA_MIN == pytest.approx(g["alpha_floor"]["value"], rel=1e-15)
    assert oracle.T_MIN == g["t_min"]["value"]
    assert oracle.TILE == g["tile_size"]["value"]
    # Sec. III-B-4 error bounds: 4 * 4000^2 * 2^-24 and 4 * 32^2 * 2^-24
    assert round(4 * 4000 ** 2 * 2.0 ** -24, 2) == g["error_bound_global"]["value"]
    assert 4 * 32 ** 2 * 2.0 ** -24 == pytest.approx(g["error_bound_local"]["value"], rel=2e-3)


def test_hoist_matrix_identity():
    """Eq. hoist_transform: V = H(dx, dy) [a, b, c, ln o] gives
    V . [x'^2, x'y', y'^2, x', y', 1] = ln o - q/2 exactly (polynomial identity)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["hoist_matrix"]["value"]
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(2000):
        a, c = np.exp(rng.uniform(-5, 1, 2))
        b = rng.uniform(-0.99, 0.99) * math.sqrt(a * c)
        lo = math.log(rng.uniform(0.01, 1))
        dx, dy = rng.uniform(-20, 36, 2)
        env = {"dx": dx, "dy": dy, "-0.5*dx^2": -0.5 * dx * dx, "-dx*dy": -dx * dy, "-0.5*dy^2": -0.5 * dy * dy}
        H = np.array([[env[v] if isinstance(v, str) else v for v in row] for row in g], float)
        V = H @ np.array([a, b, c, lo])
        for xp, yp in rng.uniform(0, 15, (8, 2)):
            B = np.array([xp * xp, xp * yp, yp * yp, xp, yp, 1.0])
            ex, ey = xp - dx, yp - dy
            direct = lo - 0.5 * (a * ex * ex + 2 * b * ex * ey + c * ey * ey)
            worst = max(worst, abs(V @ B - direct) / max(1.0, abs(a * dx * dx) + abs(c * dy * dy) + 1))
    assert worst < 1e-13


# ---------------------------------------------------------------------------
# projection closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("z,ls", [(4.0, -3.0), (2.5, -2.0), (7.0, -4.5)])
def test_projection_isotropic_on_axis(oracle, z, ls):
    cam = _cam(96, 64)
    pr = oracle.project(cam, *_one((0, 0, z), (ls, ls, ls), quat=(0.3, -0.2, 0.5, 0.7)))
    assert pr["visible"][0] == 1
    f = float(np.float32(cam.fx))
    var = (f * math.exp(ls) / z) ** 2 + 0.3
    np.testing.assert_allclose(pr["means2d"][0], [cam.cx, cam.cy], atol=1e-12)
    np.testing.assert_allclose(pr["conic"][0], [1 / var, 0, 1 / var], rtol=1e-12, atol=1e-15)
    assert pr["opacity"][0] == pytest.approx(1 / (1 + math.exp(-2.0)), rel=1e-15)
    assert pr["depth"][0] == np.float32(z)


def test_projection_isotropic_off_axis(oracle):
    """Textbook EWA for an isotropic Gaussian inside the guard band:
    Sigma2 = s^2 J J^T + 0.3 I, J = [[f/z, 0, -f x/z^2], [0, f/z, -f y/z^2]]."""
    cam = _cam(128, 128)
    f = float(np.float32(cam.fx))
    for (x, y, z, s) in [(0.5, -0.3, 4.0, 0.05), (-0.9, 0.8, 3.0, 0.02), (0.1, 0.6, 6.0, 0.1)]:
        pr = oracle.project(cam, *_one((x, y, z), (math.log(s),) * 3))
        J = np.array([[f / z, 0, -f * x / z ** 2], [0, f / z, -f * y / z ** 2]])
        S2 = s * s * J @ J.T + 0.3 * np.eye(2)
        K = np.linalg.inv(S2)
        np.testing.assert_allclose(pr["conic"][0], [K[0, 0], K[0, 1], K[1, 1]], rtol=1e-9)
        np.testing.assert_allclose(pr["means2d"][0], [f * x / z + cam.cx, f * y / z + cam.cy], rtol=1e-13)


def test_projection_rotation_swaps_axes(oracle):
    """Identity rotation: Sigma3 diagonal; a 90-degree turn about z swaps x and y."""
    cam = _cam(64, 64)
    ls = (math.log(0.08), math.log(0.02), math.log(0.05))
    p0 = oracle.project(cam, *_one((0, 0, 4), ls, quat=(1, 0, 0, 0)))
    h = math.sqrt(0.5)
    p1 = oracle.project(cam, *_one((0, 0, 4), ls, quat=(h, 0, 0, h)))
    a0, b0, c0 = p0["conic"][0]
    a1, b1, c1 = p1["conic"][0]
    assert abs(b0) < 1e-15 and abs(b1) < 1e-12
    assert a1 == pytest.approx(c0, rel=1e-12) and c1 == pytest.approx(a0, rel=1e-12)
    f = float(np.float32(cam.fx))
    assert a0 == pytest.approx(1 / ((f * 0.08 / 4) ** 2 + 0.3), rel=1e-12)
    # q and -q give the same rotation; the quaternion is normalised inside
    p2 = oracle.project(cam, *_one((0, 0, 4), ls, quat=(-3 * h, 0, 0, -3 * h)))
    np.testing.assert_allclose(p2["conic"][0], p1["conic"][0], rtol=1e-12, atol=1e-15)


def test_projection_culling(oracle):
    cam = _cam(64, 64)
    cases = [
        _one((0, 0, 0.1), (-3, -3, -3)),                  # in front of the near plane only by 0.1
        _one((0, 0, -2), (-3, -3, -3)),                   # behind the camera
        _one((0, 0, 4), (-3, -3, -3), logit=-6.0),        # opacity 0.0025 < 1/255
        _one((50, 0, 4), (-3, -3, -3)),                   # far outside the image
        _one((0, 0, 4), (-3, -3, -3), quat=(0, 0, 0, 0)),  # degenerate rotation
        _one((np.nan, 0, 4), (-3, -3, -3)),               # NaN parameters are culled
    ]
    for c in cases:
        pr = oracle.project(cam, *c)
        assert pr["visible"][0] == 0 and np.all(pr["rect"][0] == 0)
    pr = oracle.project(cam, *_one((0, 0, 4), (-3, -3, -3), logit=-5.0))   # 0.0067 > 1/255
    assert pr["visible"][0] == 1


def test_depth_key_is_float_of_camera_z(oracle):
    sc = scenes.make_config(5, n=3000)
    for v in (0, 3, 5):
        cam = sc.cameras[v]
        pr = oracle.project_scene(sc, v)
        Vm = cam.viewmat.astype(np.float64)
        z = sc.means3d.astype(np.float64) @ Vm[2, :3] + Vm[2, 3]
        vis = pr["visible"] == 1
        assert vis.sum() > 100
        d = pr["depth"][vis].astype(np.float64)
        assert np.all(np.abs(d - z[vis]) <= 1.2 * np.spacing(np.float32(z[vis]).astype(np.float32)))


# ---------------------------------------------------------------------------
# spherical harmonics
# ---------------------------------------------------------------------------
def test_sh_orthonormal_by_quadrature(oracle):
    nt, nphi = 200, 400
    th = (np.arange(nt) + 0.5) * math.pi / nt
    ph = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    G = np.zeros((16, 16))
    for t in th:
        w = math.sin(t) * (math.pi / nt) * (2 * math.pi / nphi)
        for p in ph:
            Y = oracle.sh_basis(3, (math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)))
            G += w * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=2e-4)


def test_sh_low_orders_closed_form(oracle):
    rng = np.random.default_rng(3)
    c0 = 1 / (2 * math.sqrt(math.pi))
    c1 = math.sqrt(3 / (4 * math.pi))
    for d in rng.standard_normal((20, 3)):
        d = d / np.linalg.norm(d)
        Y = oracle.sh_basis(1, d)
        # Condon-Shortley phase: Y_1^{-1} = -c1 y, Y_1^0 = c1 z, Y_1^1 = -c1 x
        np.testing.assert_allclose(Y, [c0, -c1 * d[1], c1 * d[2], -c1 * d[0]], rtol=1e-14, atol=1e-15)
        Y2 = oracle.sh_basis(2, d)
        c20 = math.sqrt(5 / (16 * math.pi))
        assert Y2[6] == pytest.approx(c20 * (3 * d[2] ** 2 - 1), rel=1e-12, abs=1e-14)


def test_sh_degree0_colour(oracle):
    cam = _cam()
    sh = np.array([[1.2, -0.4, 0.0]], np.float32)
    pr = oracle.project(cam, *_one((0.1, 0, 4), (-3, -3, -3), sh=sh))
    c0 = 1 / (2 * math.sqrt(math.pi))
    np.testing.assert_allclose(pr["rgb"][0], c0 * sh[0].astype(np.float64) + 0.5, rtol=1e-14)
    sh = np.array([[-5.0, 0.0, 0.0]], np.float32)                  # clamped at 0
    pr = oracle.project(cam, *_one((0.1, 0, 4), (-3, -3, -3), sh=sh))
    assert pr["rgb"][0, 0] == 0.0 and pr["rgb_clamped"][0, 0] == 1


# ---------------------------------------------------------------------------
# footprint, binning
# ---------------------------------------------------------------------------
def _alpha_field(pr, g, W, H):
    xs, ys = np.meshgrid(np.arange(W), np.arange(H))
    dx, dy = xs - pr["means2d"][g, 0], ys - pr["means2d"][g, 1]
    a, b, c = pr["conic"][g]
    q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
    return pr["opacity"][g] * np.exp(-0.5 * q)


@pytest.mark.parametrize("seed", [0, 1])
def test_footprint_conservative_brute_force(oracle, seed):
    sc = scenes.make_config(1, seed=100 + seed, n=600)
    sc.cameras = [_cam(80, 48)]
    sc.means3d[:, 2] -= 1.5                       # bring Gaussians closer: larger splats
    pr = oracle.project_scene(sc)
    W, H = 80, 48
    hits = 0
    for g in range(sc.n):
        if not pr["visible"][g]:
            continue
        al = _alpha_field(pr, g, W, H)
        ys, xs = np.nonzero(al >= 1 / 255)
        hits += len(xs)
        x0, y0, x1, y1 = pr["rect"][g]
        assert np.all((xs // 16 >= x0) & (xs // 16 < x1) & (ys // 16 >= y0) & (ys // 16 < y1))
    assert hits > 1000


def _rotated_splats(rng, n, W, H, sig_lo=0.05, sig_hi=400.0, ratio_hi=20.0, pad=60.0):
    """Screen-space splats drawn by covariance: rotated ellipses with major
    standard deviation log-uniform in [sig_lo, sig_hi] px, axis ratio up to
    ratio_hi, centres straddling the image edges; opacity log-uniform from
    just below 1/255 to 1."""
    cen = np.stack([rng.uniform(-pad, W - 1 + pad, n), rng.uniform(-pad, H - 1 + pad, n)], 1)
    s1 = np.exp(rng.uniform(np.log(sig_lo), np.log(sig_hi), n))
    s2 = s1 / np.exp(rng.uniform(0.0, np.log(ratio_hi), n))
    th = rng.uniform(0.0, np.pi, n)
    c, s = np.cos(th), np.sin(th)
    sxx = c * c * s1 ** 2 + s * s * s2 ** 2
    syy = s * s * s1 ** 2 + c * c * s2 ** 2
    sxy = c * s * (s1 ** 2 - s2 ** 2)
    det = sxx * syy - sxy * sxy
    conic = np.stack([syy / det, -sxy / det, sxx / det], 1)
    opac = np.exp(rng.uniform(np.log(0.9 / 255), 0.0, n))
    return cen, conic, opac


def _tile_box(xs, ys):
    return (xs.min() // 16, ys.min() // 16, xs.max() // 16 + 1, ys.max() // 16 + 1)


def _sampled_box(cen, conic, tau, W, H, k=4096, pad=0.0):
    """Pixel-centre box [x0, x1] x [y0, y1] (clipped to the image) inside the
    bounding box of the ellipse q <= tau widened by `pad` pixels, the box
    found by sampling the ellipse boundary d = sqrt(tau) L (cos t, sin t),
    Sigma = L L^T; None if it holds no pixel centre."""
    a, b, c = conic
    L = np.linalg.cholesky(np.linalg.inv(np.array([[a, b], [b, c]])))
    t = np.linspace(0.0, 2 * np.pi, k, endpoint=False)
    pts = math.sqrt(tau) * (L @ np.stack([np.cos(t), np.sin(t)]))
    x0 = max(math.ceil(cen[0] + pts[0].min() - pad), 0)
    x1 = min(math.floor(cen[0] + pts[0].max() + pad), W - 1)
    y0 = max(math.ceil(cen[1] + pts[1].min() - pad), 0)
    y1 = min(math.floor(cen[1] + pts[1].max() + pad), H - 1)
    return None if x0 > x1 or y0 > y1 else (x0, y0, x1, y1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_screen_footprint_brute_force(oracle, seed):
    """The footprint of splats given in screen space (the rule the render-only
    tests bin with).  Conservative: every pixel centre with alpha >= 1/255
    (FP64, brute force over the image) lies in the returned tile rectangle.
    Tight: the rectangle lies within the tiles of the pixel centres inside
    the bounding box of a barely larger ellipse, that box found by sampling
    the ellipse's boundary.  Culled exactly when that box holds no pixel
    centre.  An under- or over-covering rule (swapped axes, a missing factor
    of 2 in tau, the 3-sigma square) fails one of these."""
    rng = np.random.default_rng(700 + seed)
    W, H = 97, 61
    cen, conic, opac = _rotated_splats(rng, 1500, W, H)
    vis, rect = oracle.footprint(W, H, cen, conic, opac)
    xs, ys = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    n_hit = 0
    for g in range(len(opac)):
        a, b, c = conic[g]
        tau = 2.0 * math.log(255.0 * opac[g])
        if tau <= 0:
            assert vis[g] == 0, g                        # opacity below 1/255: never visible
            continue
        # the footprint's outward slack: 1e-5 relative and absolute in tau,
        # 0.01 px in the half-widths; the loose box allows a little more
        loose = _sampled_box(cen[g], conic[g], tau * 1.001 + 0.05, W, H, pad=0.02)
        if loose is None:
            assert vis[g] == 0, g
            continue
        dx, dy = xs - cen[g, 0], ys - cen[g, 1]
        q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        iy, ix = np.nonzero(q <= tau)                    # alpha >= 1/255 exactly
        x0, y0, x1, y1 = rect[g]
        if len(ix):
            n_hit += 1
            assert vis[g] == 1, g
            assert np.all((ix // 16 >= x0) & (ix // 16 < x1) & (iy // 16 >= y0) & (iy // 16 < y1)), (g, rect[g])
        if vis[g]:
            lx0, ly0, lx1, ly1 = loose
            assert x0 >= lx0 // 16 and y0 >= ly0 // 16 and x1 <= lx1 // 16 + 1 and y1 <= ly1 // 16 + 1, \
                (g, rect[g], loose)
    assert n_hit > 300
    # the draw reaches both ends: splats far larger than a tile and splats below a pixel
    assert (rect[:, 2] - rect[:, 0]).max() == (W + 15) // 16 and ((rect[:, 2] - rect[:, 0]) == 1).sum() > 50


def test_screen_footprint_equals_projection_rule(oracle):
    """The screen-space footprint of the oracle's own projected splats equals
    the rectangle the projection computed from the 2D covariance (the conic
    is its inverse, so both describe the same ellipse)."""
    sc = scenes.make_config(5, n=4000)
    for v in (0, 1, 2):
        cam = sc.cameras[v]
        pr = oracle.project_scene(sc, v)
        vis, rect = oracle.footprint(cam.width, cam.height, pr["means2d"], pr["conic"], pr["opacity"])
        assert pr["visible"].sum() > 500
        assert np.array_equal(vis, pr["visible"])
        assert np.array_equal(rect, pr["rect"])


@pytest.mark.parametrize("u,v,clamped", [(1.2, 0.0, "x"), (-1.5, 0.2, "x"), (0.3, 0.9, "y"), (1.1, -1.0, "xy"),
                                         (0.6, 0.3, "")])
def test_projection_guard_band_clamp(oracle, u, v, clamped):
    """EWA guard band: the projection Jacobian is evaluated at the camera-space
    point whose tangent coordinates are clamped to 1.3 tan(half fov), while
    the mean uses the true point.  Closed form for an isotropic Gaussian
    (Sigma3 = s^2 I, identity camera rotation):
    Sigma2 = s^2 J J^T + 0.3 I with J = [[f/z, 0, -f uc/z], [0, f/z, -f vc/z]]."""
    cam = _cam(64, 48)
    f = float(np.float32(cam.fx))
    tx, ty = float(np.float32(cam.tan_fovx)), float(np.float32(cam.tan_fovy))
    z, s = 5.0, 0.04
    x, y = u * z, v * z
    pr = oracle.project(cam, *_one((x, y, z), (math.log(s),) * 3))

    def conic_at(uc, vc):
        J = np.array([[f / z, 0, -f * uc / z], [0, f / z, -f * vc / z]])
        K = np.linalg.inv(s * s * J @ J.T + 0.3 * np.eye(2))
        return np.array([K[0, 0], K[0, 1], K[1, 1]])

    uc = float(np.clip(u, -1.3 * tx, 1.3 * tx))
    vc = float(np.clip(v, -1.3 * ty, 1.3 * ty))
    assert ("x" in clamped) == (uc != u) and ("y" in clamped) == (vc != v)
    np.testing.assert_allclose(pr["means2d"][0], [f * u + cam.cx, f * v + cam.cy], rtol=1e-13)
    # (the conic is reported also when the footprint then misses the image)
    np.testing.assert_allclose(pr["conic"][0], conic_at(uc, vc), rtol=1e-9, atol=1e-15)
    if not clamped:
        assert pr["visible"][0] == 1
    if clamped:
        # the unclamped Jacobian gives a visibly different conic
        assert np.abs(conic_at(u, v) - conic_at(uc, vc)).max() > 1e-3 * np.abs(conic_at(uc, vc)).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiled_equals_untiled(oracle, seed):
    sc = scenes.make_config(1, seed=200 + seed, n=1500)
    sc.cameras = [_cam(72, 56, bg=(0.2, 0.1, 0.7))]
    sc.means3d[:, 2] -= 1.0
    t = oracle.render_scene(sc, tiled=True)
    u = oracle.render_scene(sc, tiled=False)
    assert np.array_equal(t["image"], u["image"])
    assert np.array_equal(t["T"], u["T"])
    assert np.array_equal(t["last_id"], u["last_id"])
    assert (t["count"] > 0).mean() > 0.5


def test_tile_lists_order(oracle):
    rng = np.random.default_rng(5)
    n = 400
    vis = (rng.uniform(size=n) < 0.8).astype(np.int32)
    depth = rng.choice(np.float32([1.0, 1.5, 2.0, 2.5]), n)     # many ties
    x0 = rng.integers(0, 5, n); y0 = rng.integers(0, 4, n)
    rect = np.stack([x0, y0, x0 + rng.integers(1, 3, n), y0 + rng.integers(1, 3, n)], 1).astype(np.int32)
    rect = np.minimum(rect, [5, 4, 5, 4]).astype(np.int32)
    rect[:, 2] = np.maximum(rect[:, 2], rect[:, 0] + 1); rect[:, 3] = np.maximum(rect[:, 3], rect[:, 1] + 1)
    rect = np.minimum(rect, [4, 3, 5, 4]).astype(np.int32)
    off, ids = oracle.tile_lists(vis, depth, rect, 80, 64)
    for t in range(20):
        tx, ty = t % 5, t // 5
        want = [g for g in range(n) if vis[g] and rect[g, 0] <= tx < rect[g, 2] and rect[g, 1] <= ty < rect[g, 3]]
        want.sort(key=lambda g: (depth[g], g))
        assert list(ids[off[t]:off[t + 1]]) == want


# ---------------------------------------------------------------------------
# blending closed forms and invariants (Alg. 1, baseline column)
# ---------------------------------------------------------------------------
def _splats(means, conics, opac, rgb, depth=None):
    n = len(opac)
    depth = np.arange(1, n + 1, dtype=np.float32) if depth is None else np.asarray(depth, np.float32)
    return (np.ones(n, np.int32), depth, np.asarray(means, float), np.asarray(conics, float),
            np.asarray(opac, float), np.asarray(rgb, float))


def test_one_gaussian_closed_form(oracle):
    W = H = 32
    args = _splats([[10.3, 12.7]], [[0.05, 0.01, 0.08]], [0.8], [[0.2, 0.5, 0.9]])
    out = oracle.render_untiled(W, H, *args, bg=(0.125, 0.0, 0.375))
    for (x, y) in [(10, 12), (14, 9), (3, 25), (31, 0)]:
        dx, dy = x - 10.3, y - 12.7
        al = min(0.99, 0.8 * math.exp(-0.5 * (0.05 * dx * dx + 0.02 * dx * dy + 0.08 * dy * dy)))
        bg = np.array([0.125, 0.0, 0.375])
        if al >= 1 / 255:
            want = np.array([0.2, 0.5, 0.9]) * al + (1 - al) * bg
            assert out["T"][y, x] == pytest.approx(1 - al, rel=1e-14)
            assert out["last_id"][y, x] == 0 and out["count"][y, x] == 1
        else:
            want = bg
            assert out["T"][y, x] == 1.0 and out["last_id"][y, x] == -1
        np.testing.assert_allclose(out["image"][:, y, x], want, rtol=1e-13, atol=1e-15)
    # opacity 1 at the centre is clamped to 0.99
    out = oracle.render_untiled(W, H, *_splats([[5.0, 5.0]], [[1, 0, 1]], [1.0], [[1, 1, 1]]))
    assert out["T"][5, 5] == pytest.approx(0.01, rel=1e-14)


def test_two_gaussians_closed_form(oracle):
    args = _splats([[8.0, 8.0], [9.0, 7.5]], [[0.1, 0, 0.1], [0.05, 0.02, 0.2]], [0.6, 0.9],
                   [[1, 0, 0], [0, 1, 0]], depth=[2.0, 1.0])        # second one is in front
    out = oracle.render_untiled(16, 16, *args)
    x, y = 8, 8
    a0 = 0.6 * math.exp(-0.5 * 0.0)
    dx, dy = x - 9.0, y - 7.5
    a1 = 0.9 * math.exp(-0.5 * (0.05 * dx * dx + 0.04 * dx * dy + 0.2 * dy * dy))
    want = np.array([0, 1, 0]) * a1 + np.array([1, 0, 0]) * a0 * (1 - a1)
    np.testing.assert_allclose(out["image"][:, y, x], want, rtol=1e-14)
    assert out["T"][y, x] == pytest.approx((1 - a1) * (1 - a0), rel=1e-14)
    assert out["last_id"][y, x] == 0


def test_termination_stack(oracle):
    """20 coincident Gaussians with alpha = 0.5 at the pixel: 0.5^13 >= 1e-4 > 0.5^14,
    so exactly 13 are blended (Alg. 1 stops before the 14th)."""
    n = 20
    args = _splats([[4.0, 4.0]] * n, [[0.3, 0, 0.3]] * n, [0.5] * n, [[0.25, 0.5, 1.0]] * n)
    out = oracle.render_untiled(8, 8, *args)
    assert out["count"][4, 4] == 13 and out["last_id"][4, 4] == 12
    assert out["T"][4, 4] == pytest.approx(2.0 ** -13, rel=1e-14)
    np.testing.assert_allclose(out["image"][:, 4, 4], np.array([0.25, 0.5, 1.0]) * (1 - 2.0 ** -13), rtol=1e-14)


@pytest.mark.parametrize("seed", [0, 1])
def test_blend_invariants(oracle, seed):
    rng = np.random.default_rng(seed)
    W, H, n = 48, 40, 300
    cen, con, op, col, dep = scenes.random_projected(rng, n, W, H, sigma_px=(0.5, 8.0))
    ones = np.ones_like(col)
    vis = np.ones(n, np.int32)
    out = oracle.render_untiled(W, H, vis, dep, cen, con, op, ones)
    T = out["T"]
    assert T.min() >= 1e-4 and T.max() <= 1.0
    np.testing.assert_allclose(out["image"], np.broadcast_to(1 - T, (3, H, W)), atol=1e-13)
    out = oracle.render_untiled(W, H, vis, dep, cen, con, op, col)
    # the colour lies within [0, 1 - T] for colours in [0, 1]
    assert np.all(out["image"] >= -1e-15) and np.all(out["image"] <= (1 - T) + 1e-13)
    # permuting the storage order (distinct depths) changes nothing
    perm = rng.permutation(n)
    out2 = oracle.render_untiled(W, H, vis, dep[perm], cen[perm], con[perm], op[perm], col[perm])
    assert np.array_equal(out["image"], out2["image"]) and np.array_equal(out["T"], out2["T"])
    has = out["last_id"] >= 0
    assert np.array_equal(perm[out2["last_id"][has]], out["last_id"][has])


def test_transmittance_monotone_in_depth(oracle):
    """Adding a Gaussian behind everything can only lower T."""
    rng = np.random.default_rng(9)
    W, H, n = 32, 32, 80
    cen, con, op, col, dep = scenes.random_projected(rng, n, W, H)
    vis = np.ones(n, np.int32)
    a = oracle.render_untiled(W, H, vis[:-1], dep[:-1], cen[:-1], con[:-1], op[:-1], col[:-1])
    dep2 = dep.copy(); dep2[-1] = 100.0
    b = oracle.render_untiled(W, H, vis, dep2, cen, con, op, col)
    assert np.all(b["T"] <= a["T"])


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------
def _tiled(oracle, W, H, cen, con, op, col, dep):
    n = len(op)
    vis = np.ones(n, np.int32)
    rect = np.zeros((n, 4), np.int32)
    rect[:, 2] = (W + 15) // 16; rect[:, 3] = (H + 15) // 16         # every tile
    return oracle.tile_lists(vis, dep, rect, W, H)


def test_single_gaussian_gradient_closed_form(oracle):
    W = H = 16
    cen = np.array([[7.3, 8.6]]); con = np.array([[0.09, -0.02, 0.06]]); op = np.array([0.7])
    col = np.array([[0.3, 0.6, 0.1]]); dep = np.ones(1, np.float32)
    off, ids = _tiled(oracle, W, H, cen, con, op, col, dep)
    x, y = 9, 7
    gC = np.zeros((3, H, W)); gC[:, y, x] = [1.0, 0.0, 0.0]
    g = oracle.render_backward(W, H, off, ids, cen, con, op, col, gC)
    dx, dy = x - 7.3, y - 8.6
    a, b, c = con[0]
    G = math.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
    al = 0.7 * G
    assert g["rgb"][0, 0] == pytest.approx(al, rel=1e-14)
    assert g["opacity"][0] == pytest.approx(0.3 * G, rel=1e-13)
    np.testing.assert_allclose(g["means2d"][0], 0.3 * al * np.array([a * dx + b * dy, b * dx + c * dy]), rtol=1e-13)
    np.testing.assert_allclose(g["conic"][0], -0.5 * 0.3 * al * np.array([dx * dx, 2 * dx * dy, dy * dy]), rtol=1e-13)


def test_constant_colour_gradient_identity(oracle):
    """All colours k and bg 0: C = k (1 - T_final), so dC/dtheta = -k dT_final/dtheta."""
    rng = np.random.default_rng(11)
    W, H, n = 32, 32, 60
    cen, con, op, col, dep = scenes.random_projected(rng, n, W, H, sigma_px=(0.8, 6))
    k = 0.37
    col = np.full((n, 3), k)
    off, ids = _tiled(oracle, W, H, cen, con, op, col, dep)
    w = rng.standard_normal((H, W))
    g1 = oracle.render_backward(W, H, off, ids, cen, con, op, col, np.stack([w, 0 * w, 0 * w]))
    g2 = oracle.render_backward(W, H, off, ids, cen, con, op, col, np.zeros((3, H, W)), gT=-k * w)
    for key in ("means2d", "conic", "opacity"):
        np.testing.assert_allclose(g1[key], g2[key], rtol=1e-10, atol=1e-13)


def _sig(out):
    return np.concatenate([out["last_id"].ravel(), out["count"].ravel()])


def test_render_gradient_vs_finite_differences(oracle):
    rng = np.random.default_rng(21)
    W, H, n = 32, 32, 40
    cen, con, op, col, dep = scenes.random_projected(rng, n, W, H, sigma_px=(0.8, 5), margin=4)
    cen, con, op, col = (a.astype(np.float64) for a in (cen, con, op, col))
    off, ids = _tiled(oracle, W, H, cen, con, op, col, dep)
    gC = rng.standard_normal((3, H, W)); gT = rng.standard_normal((H, W))
    an = oracle.render_backward(W, H, off, ids, cen, con, op, col, gC, gT)
    fields = dict(means2d=cen, conic=con, opacity=op, rgb=col)

    def loss(f):
        o = oracle.render_tiled(W, H, off, ids, f["means2d"], f["conic"], f["opacity"], f["rgb"])
        return float((gC * o["image"]).sum() + (gT * o["T"]).sum()), _sig(o)

    checked = 0
    for key, arr in fields.items():
        for idx in np.ndindex(arr.shape):
            h = 1e-6 * max(1.0, abs(arr[idx]))
            fp = {k: v.copy() for k, v in fields.items()}; fm = {k: v.copy() for k, v in fields.items()}
            fp[key][idx] += h; fm[key][idx] -= h
            lp, sp = loss(fp); lm, sm = loss(fm)
            if not np.array_equal(sp, sm):
                continue
            fd = (lp - lm) / (2 * h)
            assert an[key][idx] == pytest.approx(fd, rel=1e-5, abs=1e-7), (key, idx)
            checked += 1
    assert checked > 0.9 * sum(a.size for a in fields.values())


@pytest.mark.parametrize("deg", [0, 3])
def test_scene_gradient_vs_finite_differences(oracle, deg):
    """Full chain raw parameters -> image, FP64 central differences."""
    sc = scenes.make_fd_scene(degree=deg, n=30, size=32, seed=404 + deg)
    sc.means3d[:, 2] -= 1.0
    cam = sc.cameras[0]
    rng = np.random.default_rng(7 + deg)
    gC = rng.standard_normal((3, cam.height, cam.width)); gT = rng.standard_normal((cam.height, cam.width))
    an = oracle.scene_gradients(sc, gC, gT)
    raw = dict(means3d=sc.means3d.astype(np.float64), log_scales=sc.log_scales.astype(np.float64),
               quats=sc.quats.astype(np.float64), opacity_logits=sc.opacity_logits.astype(np.float64),
               sh=sc.sh.astype(np.float64))

    def loss(r):
        pr = oracle.project(cam, r["means3d"], r["log_scales"], r["quats"], r["opacity_logits"], r["sh"])
        o = oracle.render_untiled(cam.width, cam.height, pr["visible"], pr["depth"], pr["means2d"],
                                  pr["conic"], pr["opacity"], pr["rgb"], cam.bg)
        return float((gC * o["image"]).sum() + (gT * o["T"]).sum()), np.concatenate(
            [_sig(o), pr["visible"], pr["rgb_clamped"].ravel()])

    vis = oracle.project_scene(sc)["visible"]
    assert vis.sum() >= 20
    checked = skipped = 0
    for key, arr in raw.items():
        for idx in np.ndindex(arr.shape):
            if not vis[idx[0]]:
                assert an[key][idx] == 0.0
                continue
            h = 1e-6 * max(1.0, abs(arr[idx]))
            rp = {k: v.copy() for k, v in raw.items()}; rm = {k: v.copy() for k, v in raw.items()}
            rp[key][idx] += h; rm[key][idx] -= h
            lp, sp = loss(rp); lm, sm = loss(rm)
            if not np.array_equal(sp, sm):
                skipped += 1
                continue
            fd = (lp - lm) / (2 * h)
            scale = max(abs(fd), 1e-3 * np.abs(an[key]).max())
            assert abs(an[key][idx] - fd) <= 1e-5 * scale + 1e-9, (key, idx, an[key][idx], fd)
            checked += 1
    assert checked > 10 * skipped


def test_clamp_margin_is_not_a_forward_decision(oracle):
    """min(0.99, .) is continuous: a Gaussian whose unclamped alpha sits next to
    0.99 at a pixel gives a small clamp margin there (the derivative switches),
    while the forward decision margin stays large."""
    W = H = 16
    args = _splats([[7.0, 7.0]], [[0.5, 0.0, 0.5]], [0.99 * math.exp(2e-6)], [[0.3, 0.6, 0.9]])
    out = oracle.render_untiled(W, H, *args)
    assert out["clamp_margin"][7, 7] == pytest.approx(2e-6, rel=1e-6)
    assert out["margin"][7, 7] > 1.0
    assert out["image"][0, 7, 7] == pytest.approx(0.3 * 0.99, rel=1e-15)


def test_stored_projection_rounds_the_splats_only(oracle):
    """The float32-stored projection rounds mean, conic, opacity and colour
    and keeps visibility, depth keys and rectangles."""
    sc = scenes.make_config(1, n=500)
    pr = oracle.project_scene(sc)
    st = oracle.stored_projection(pr)
    for k in ("means2d", "conic", "opacity", "rgb"):
        assert np.array_equal(st[k], pr[k].astype(np.float32).astype(np.float64))
        assert np.abs(st[k] - pr[k]).max() <= np.abs(pr[k]).max() * 2.0 ** -24
    for k in ("visible", "depth", "rect"):
        assert np.array_equal(st[k], pr[k])


def test_chunked_projection_equals_one_call(oracle):
    sc = scenes.make_config(5, n=3001)
    cam = sc.cameras[2]
    a = oracle.project_scene(sc, 2)
    b = oracle.project_chunked(cam, sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, threads=3)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


# ---------------------------------------------------------------------------
# exact tile-ellipse intersection (the tile assignment made exact)
# ---------------------------------------------------------------------------
def test_rect_min_quadratic_brute_force(oracle):
    """The closed-form minimum of a positive-definite quadratic over a
    rectangle equals a dense sampling of the rectangle (the sampled minimum is
    never below it and approaches it)."""
    rng = np.random.default_rng(31)
    for _ in range(300):
        s1, s2 = np.exp(rng.uniform(-2, 4, 2))
        th = rng.uniform(0, np.pi)
        c_, s_ = math.cos(th), math.sin(th)
        S = np.array([[c_ * c_ * s1 * s1 + s_ * s_ * s2 * s2, c_ * s_ * (s1 * s1 - s2 * s2)],
                      [c_ * s_ * (s1 * s1 - s2 * s2), s_ * s_ * s1 * s1 + c_ * c_ * s2 * s2]])
        K = np.linalg.inv(S)
        a, b, c = K[0, 0], K[0, 1], K[1, 1]
        x0, y0 = rng.uniform(-60, 40, 2)
        x1, y1 = x0 + rng.uniform(0.5, 30), y0 + rng.uniform(0.5, 30)
        got = oracle.rect_min_q(a, b, c, x0, x1, y0, y1)
        xs, ys = np.meshgrid(np.linspace(x0, x1, 401), np.linspace(y0, y1, 401))
        q = a * xs * xs + 2 * b * xs * ys + c * ys * ys
        assert got <= q.min() * (1 + 1e-12) + 1e-300
        # the grid's spacing bounds how far above the true minimum it can be
        h = max(x1 - x0, y1 - y0) / 400
        grad = 2 * np.sqrt(max(a, c) * max(q.min(), 1e-300)) + 2 * max(a, c) * h
        assert q.min() - got <= grad * h * 2 + 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_tile_lists_conservative_and_within_rectangles(oracle, seed):
    """Exact lists: a subset of the rectangle lists in the same order, a
    superset of the tiles holding a pixel centre with alpha >= 1/255 (brute
    force), and contained in the lists of the looser ellipse."""
    rng = np.random.default_rng(800 + seed)
    W, H = 109, 77
    cen, conic, opac = _rotated_splats(rng, 800, W, H, sig_hi=60.0)
    vis, rect = oracle.footprint(W, H, cen, conic, opac)
    depth = rng.uniform(1, 5, len(opac)).astype(np.float32)
    off_r, ids_r = oracle.tile_lists(vis, depth, rect, W, H)
    off_e, ids_e = oracle.tile_lists_exact(vis, depth, rect, cen, conic, opac, W, H, **oracle.EXACT_TIGHT)
    off_l, ids_l = oracle.tile_lists_exact(vis, depth, rect, cen, conic, opac, W, H, **oracle.EXACT_LOOSE)
    ntx = (W + 15) // 16
    xs, ys = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    need = [set() for _ in range(len(off_r) - 1)]
    for g in np.nonzero(vis)[0]:
        a, b, c = conic[g]
        dx, dy = xs - cen[g, 0], ys - cen[g, 1]
        hit = a * dx * dx + 2 * b * dx * dy + c * dy * dy <= 2 * math.log(255 * opac[g])
        for t in np.unique((ys[hit] // 16) * ntx + xs[hit] // 16).astype(int):
            need[t].add(int(g))
    dropped = 0
    for t in range(len(off_r) - 1):
        r = list(ids_r[off_r[t]:off_r[t + 1]])
        e = list(ids_e[off_e[t]:off_e[t + 1]])
        lo = set(ids_l[off_l[t]:off_l[t + 1]])
        assert e == [g for g in r if g in set(e)], t          # same order, a subsequence
        assert need[t] <= set(e) <= lo, t
        dropped += len(r) - len(e)
    assert dropped > 0.1 * len(ids_r)


@pytest.mark.parametrize("seed", [0, 1])
def test_exact_tiled_equals_untiled(oracle, seed):
    """Blending over the exact lists gives the untiled definition bitwise."""
    sc = scenes.make_config(1, seed=300 + seed, n=1500)
    sc.cameras = [_cam(88, 56, bg=(0.3, 0.2, 0.1))]
    sc.means3d[:, 2] -= 1.0
    cam = sc.cameras[0]
    pr = oracle.project_scene(sc)
    off, ids = oracle.tile_lists_exact(pr["visible"], pr["depth"], pr["rect"], pr["means2d"], pr["conic"],
                                       pr["opacity"], cam.width, cam.height, **oracle.EXACT_TIGHT)
    t = oracle.render_tiled(cam.width, cam.height, off, ids, pr["means2d"], pr["conic"], pr["opacity"], pr["rgb"],
                            cam.bg)
    u = oracle.render_scene(sc, tiled=False)
    assert np.array_equal(t["image"], u["image"]) and np.array_equal(t["T"], u["T"])
    assert np.array_equal(t["last_id"], u["last_id"])
    off_r, ids_r = oracle.tile_lists(pr["visible"], pr["depth"], pr["rect"], cam.width, cam.height)
    assert len(ids) < len(ids_r)


# ---------------------------------------------------------------------------
# alternatives of near-threshold decisions
# ---------------------------------------------------------------------------
def _alts(oracle, means, conics, opac, rgb, W, H, x, y, guard, bg=(0, 0, 0)):
    vis, dep, m, k, o, c = _splats(means, conics, opac, rgb)
    rect = np.tile(np.int32([[0, 0, (W + 15) // 16, (H + 15) // 16]]), (len(o), 1))
    off, ids = oracle.tile_lists(vis, dep, rect, W, H)
    return oracle.blend_alternatives(W, H, off, ids, m, k, o, c, bg, x, y, guard), (off, ids, m, k, o, c)


def test_alternatives_single_outcome_off_threshold(oracle):
    """Far from every threshold a pixel has exactly one outcome, the blend."""
    rng = np.random.default_rng(5)
    n = 30
    means = rng.uniform(0, 31, (n, 2))
    conics = np.tile([[0.05, 0.01, 0.06]], (n, 1))
    opac = rng.uniform(0.2, 0.9, n)
    rgb = rng.uniform(0, 1, (n, 3))
    (img, T, lid), lists = _alts(oracle, means, conics, opac, rgb, 32, 32, 11, 17, 1e-9, bg=(0.2, 0.3, 0.4))
    ref = oracle.render_untiled(32, 32, *_splats(means, conics, opac, rgb), bg=(0.2, 0.3, 0.4))
    assert len(T) == 1 and ref["margin"][17, 11] > 1e-9
    np.testing.assert_allclose(img[0], ref["image"][:, 17, 11], rtol=0, atol=1e-15)
    assert T[0] == pytest.approx(ref["T"][17, 11], abs=1e-15) and lid[0] == ref["last_id"][17, 11]


def test_alternatives_floor_and_stop_knife_edges(oracle):
    """A Gaussian at alpha = 1/255 (1 + 1e-9) gives both outcomes of the
    floor; a stop test at T (1 - alpha) = 1e-4 (1 + 1e-9) both outcomes of
    the stop.  With the floor Gaussian in front of the stop test: three, as
    blending it lowers T by 1/255, which moves the later stop test off its
    threshold (it stops), while skipping it leaves the knife edge (two)."""
    W = H = 16
    # floor: o exp(-q/2) = 1/255 (1 + 1e-9) at pixel (5, 5) with the centre at (5, 5 + d)
    o = 0.5
    d = math.sqrt(2 * math.log(o * 255 / (1 + 1e-9)) / 0.2)
    (img, T, lid), _ = _alts(oracle, [[5.0, 5.0 + d]], [[0.2, 0.0, 0.2]], [o], [[0.9, 0.5, 0.1]], W, H, 5, 5, 1e-6)
    assert len(T) == 2
    al = 1 / 255 * (1 + 1e-9)
    got = sorted(zip(T, lid))
    assert got[0][0] == pytest.approx(1 - al, rel=1e-12) and got[0][1] == 0
    assert got[1] == (1.0, -1)
    # stop: alpha_1 = 0.99, then T (1 - alpha_2) = 1e-4 (1 + 1e-9)
    a2 = 1 - 0.01 * (1 + 1e-9)
    o2 = a2                                               # centred: alpha = o
    means = [[8.0, 8.0], [8.0, 8.0]]
    (img, T, lid), _ = _alts(oracle, means, [[0.3, 0, 0.3]] * 2, [0.995, o2], [[1, 0, 0], [0, 1, 0]], W, H, 8, 8, 1e-6)
    assert len(T) == 2
    got = {int(l): (t, tuple(c)) for l, t, c in zip(lid, T, img)}
    assert got[0][0] == pytest.approx(0.01, rel=1e-12) and got[0][1][1] == 0.0       # stopped before the second
    assert got[1][0] == pytest.approx(1e-4 * (1 + 1e-9), rel=1e-9)                  # blended the second
    # both knife edges on one pixel
    means = [[8.0, 8.0 + d], [8.0, 8.0], [8.0, 8.0]]
    (img, T, lid), _ = _alts(oracle, means, [[0.2, 0, 0.2], [0.3, 0, 0.3], [0.3, 0, 0.3]], [o, 0.995, o2],
                             [[0, 0, 1], [1, 0, 0], [0, 1, 0]], W, H, 8, 8, 1e-6)
    assert len(T) == 3
    want = sorted([(1 - al) * 0.01, 0.01, 1e-4 * (1 + 1e-9)])
    np.testing.assert_allclose(sorted(T), want, rtol=1e-9)
