"""GPU parity of the gradient path against the FP64 oracle.

Tolerance: for each parameter tensor, ||g - g*|| / ||g*|| <= 1e-3 and, for
every element, |g - g*| <= 1e-3 * max(|g*|, 1e-3 * max|g*|).  Pixels whose
skip / stop decisions or 0.99 clamp lie within the guard of their thresholds
get a zero incoming gradient on both sides (either decision is correct there,
and such a pixel then contributes nothing to any gradient).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_16566_amd import rasterizer as R
from paper_2606_16566_amd import scenes
from tests.gpu_helpers import projected_from, render_only_case, scene_tensors, to_dev

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def assert_grad_close(got, want, name, tol=GRAD_TOL):
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    scale = np.abs(want).max()
    if scale == 0:
        assert np.abs(got).max() == 0, name
        return
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel <= tol, (name, rel)
    err = np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * scale)
    print(f"  {name}: relative norm error {rel:.2e}, worst element {err.max():.2e}", flush=True)
    assert err.max() <= tol, (name, int((err > tol).sum()), err.size, float(err.max()))


@pytest.mark.parametrize("seed,W,H,n", [(0, 96, 64, 2000), (1, 160, 128, 12000), (2, 33, 47, 300)])
@pytest.mark.parametrize("variant", ["plain", "local", "local_q8", "plain_fp32", "local_fp32", "local_q8_fp32"])
def test_render_backward_parity(seed, W, H, n, variant):
    """The backward after each forward variant, replayed with that forward's
    own exponent precision.  Single-precision forwards decide the 1/255 floor
    and the 0.99 clamp from a float exponent, which is up to ~4e-5 off in
    ln alpha for the hoisted form (tile-centre coordinates, small splats) and
    ~1e-5 for the direct one, so their guard is 1e-4."""
    cam, cen, con, op, col, dep = render_only_case(100 + seed, W, H, n, sigma=(0.4, 10.0))
    vis, rect = O.footprint(W, H, cen, con, op)
    dep = np.where(vis == 1, dep, np.float32(np.inf)).astype(np.float32)
    off, ids = O.tile_lists(vis, dep, rect, W, H)
    ref = O.render_tiled(W, H, off, ids, cen, con, op, col, cam.bg)
    rng = np.random.default_rng(seed)
    gC = rng.standard_normal((3, H, W)).astype(np.float32)
    gT = rng.standard_normal((H, W)).astype(np.float32)
    fp32 = variant.endswith("_fp32")
    flag = O.grad_flagged(ref, 1e-4 if fp32 else 1e-5)
    print(f"render backward {variant} seed={seed}: flagged {int(flag.sum())}/{flag.size}", flush=True)
    assert flag.mean() <= (1e-2 if fp32 else 1e-3)
    gC[:, flag] = 0.0
    gT[flag] = 0.0
    want = O.render_backward(W, H, off, ids, cen, con, op, col, gC, gT, cam.bg)
    proj = projected_from(cen, con, op, col, dep, rect)
    b = R.Binner(capacity=len(ids) + 64).run(cam, proj)
    img, T, nc = R.render(variant, cam, b, proj)
    got = R.render_backward(variant, cam, b, proj, T, nc, to_dev(gC), to_dev(gT))
    for k in ("means2d", "conic", "opacity", "rgb"):
        assert_grad_close(_np(got[k]), want[k], k)


@pytest.mark.parametrize("cfg,n,view", [(1, 5000, 0), (2, 5000, 0), (5, 8000, 3)])
def test_project_backward_parity(cfg, n, view):
    sc = scenes.make_config(cfg, n=n)
    cam = sc.cameras[view]
    rng = np.random.default_rng(cfg)
    g = dict(means2d=rng.standard_normal((n, 2)), conic=rng.standard_normal((n, 3)) * 100,
             opacity=rng.standard_normal(n), rgb=rng.standard_normal((n, 3)))
    g32 = {k: v.astype(np.float32) for k, v in g.items()}
    want = O.project_backward(cam, sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh,
                              g32["means2d"], g32["conic"], g32["opacity"], g32["rgb"])
    ps = scene_tensors(sc)
    proj = R.project(cam, *ps)
    gd = {k: to_dev(v) for k, v in g32.items()}
    got = R.project_backward(cam, *ps, proj.rect, R.pack_grads(gd["means2d"], gd["conic"], gd["opacity"], gd["rgb"]))
    for k in ("means3d", "log_scales", "quats", "opacity_logits", "sh"):
        assert_grad_close(_np(got[k]), want[k], k, tol=1e-5)


@pytest.mark.parametrize("V,n,seed,cfg,deg,clear", [(16, 3001, 11, 5, 3, True), (9, 500, 15, 4, 0, True),
                                                    (8, 300, 16, 5, 3, True), (5, 130, 12, 5, 3, True),
                                                    (1, 777, 13, 4, 0, True), (16, 64, 14, 2, 3, True),
                                                    (10, 700, 17, 5, 1, True), (12, 400, 18, 5, 2, True),
                                                    (11, 900, 19, 5, 3, False), (4, 900, 20, 5, 3, False)])
def test_project_backward_batch_sparse_views(V, n, seed, cfg, deg, clear):
    """The batch backward of the projection: up to 8 views one lane per
    Gaussian loops over them; beyond, it lists, per 64 Gaussians, the
    (Gaussian, view) pairs whose gradient record is nonzero over a nonempty
    rectangle and takes them 64 at a time, several views of one Gaussian in
    one round (two lists of 5 and 4 views with 9).  Against the oracle's
    single-view backward summed over the views, at SH degrees 0 to 3: sparse
    records (a Gaussian in no view, in some, or in nearly all), nonzero
    records over empty rectangles (no contribution; cleared like the others),
    n not a multiple of 64, and the records all zero afterwards (untouched
    without the clear flag).  Tolerance
    1e-5 (1e-4 for the SH gradient summed in single precision by the loop)."""
    import ctypes as C
    from paper_2606_16566_amd import _lib as L
    from tests.test_gpu_batch import ring_cameras
    sc = scenes.make_config(cfg, n=n)
    sc.sh = np.ascontiguousarray(sc.sh[:, :(deg + 1) ** 2, :])        # lower degrees: the leading coefficients
    assert sc.sh_degree == deg
    cams = ring_cameras([(64 + 16 * (v % 5), 48 + 8 * (v % 3)) for v in range(V)])
    rng = np.random.default_rng(seed)
    # per Gaussian, the share of views with a gradient: none, some, most
    share = rng.choice([0.0, 0.2, 0.6, 0.95], size=n, p=[0.3, 0.4, 0.2, 0.1])
    rect = np.zeros((V, n, 4), np.int32)
    rec = np.zeros((V, n, L.GRAD_FLOATS), np.float32)
    want = {k: 0.0 for k in ("means3d", "log_scales", "quats", "opacity_logits", "sh")}
    listed = 0
    for v, cam in enumerate(cams):
        pr = O.project(cam, sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh)
        rect[v] = pr["rect"]
        vis = pr["visible"] == 1
        has = rng.uniform(size=n) < np.where(vis, share, 0.5)      # some over empty rectangles too
        g = rng.standard_normal((n, L.GRAD_FLOATS)).astype(np.float32)
        g[:, 0:3] *= 100.0                                          # conic gradients
        g[~has] = 0.0
        rec[v] = g
        listed += int((has & vis).sum())
        d = O.project_backward(cam, sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh,
                               g[:, 4:6], g[:, 0:3], g[:, 3], g[:, 6:9])
        for k in want:
            want[k] = want[k] + d[k]
    print(f"V={V} n={n}: {listed} listed pairs of {V * n}", flush=True)
    ps = scene_tensors(sc)
    dev = torch.device("cuda")
    r_dev = to_dev(rect.reshape(V * n, 4))
    g_dev = to_dev(rec.reshape(V * n, L.GRAD_FLOATS))
    out = dict(means3d=torch.empty((n, 3), device=dev), log_scales=torch.empty((n, 3), device=dev),
               quats=torch.empty((n, 4), device=dev), opacity_logits=torch.empty(n, device=dev),
               sh=torch.empty(tuple(sc.sh.shape), device=dev))
    p = lambda t: C.c_void_p(t.data_ptr())
    L.check(L.lib().lgs_project_backward_batch(L.camera_array(cams), V, n, sc.sh_degree, *(p(t) for t in ps),
                                               p(r_dev), p(g_dev), p(out["means3d"]), p(out["log_scales"]),
                                               p(out["quats"]), p(out["opacity_logits"]), p(out["sh"]),
                                               L.PROJ_BWD_CLEAR if clear else 0,
                                               C.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "lgs_project_backward_batch")
    for k in want:
        # up to 8 views the SH gradient is summed over the views in single
        # precision (its stored precision): each view adds a rounded product
        # to a rounded sum, 1e-4; everything else (and every sum of the
        # listed pairs) in double, 1e-5
        assert_grad_close(_np(out[k]), want[k], k, tol=1e-4 if (k == "sh" and V <= 8) else 1e-5)
    if clear:
        assert not bool(g_dev.any()), "gradient records left nonzero"
    else:
        assert np.array_equal(_np(g_dev), rec.reshape(V * n, L.GRAD_FLOATS).astype(np.float64)), "records changed"


def test_l1_loss_kernel():
    rng = np.random.default_rng(3)
    x = rng.uniform(size=(3, 77, 131)).astype(np.float32)
    y = rng.uniform(size=(3, 77, 131)).astype(np.float32)
    y[0, 0, :5] = x[0, 0, :5]
    loss, grad = R.l1_loss(to_dev(x), to_dev(y))
    assert float(loss.item()) == pytest.approx(np.abs(x.astype(np.float64) - y).mean(), rel=1e-6)
    want = np.sign(x - y) / x.size
    assert np.array_equal(_np(grad), want.astype(np.float32).astype(np.float64))
    # deterministic: the partial sums are added in a fixed order
    loss2, _ = R.l1_loss(to_dev(x), to_dev(y))
    assert float(loss2.item()) == float(loss.item())


def test_l1_loss_concurrent_streams():
    """Two losses in flight on two streams at once, each with its own
    workspace, each get their own value (no shared accumulator)."""
    rng = np.random.default_rng(4)
    n = 3 * 1080 * 1920
    xs = [to_dev(rng.uniform(size=n).astype(np.float32)) for _ in range(2)]
    ys = [to_dev(rng.uniform(size=n).astype(np.float32) * (k + 1)) for k in range(2)]
    want = [float(np.abs(_np(x) - _np(y)).mean()) for x, y in zip(xs, ys)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for rep in range(20):
        outs = []
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                outs.append(R.l1_loss(xs[k], ys[k]))
        torch.cuda.synchronize()
        for k in range(2):
            assert float(outs[k][0].item()) == pytest.approx(want[k], rel=1e-6), (rep, k)


def _scene_grad_check(sc, guard=1e-5, variant="local", fd_params=0, seed=0):
    cam = sc.cameras[0]
    ref = O.render_scene(sc, stored=True)
    target = scenes.make_target(cam.height, cam.width, 100 + seed)
    ps = [p.requires_grad_() for p in scene_tensors(sc)]
    img, T, nc = R.LocalGSFunction.apply(*ps, cam, variant, None)
    loss, gimg = R.l1_loss(img.detach().contiguous(), to_dev(target))
    # incoming gradient: the L1 gradient, zeroed where a decision is ambiguous
    # and where the L1 sign itself is within rounding
    flag = O.grad_flagged(ref, guard)
    print(f"scene gradients {variant} n={sc.n}: flagged {int(flag.sum())}/{flag.size}", flush=True)
    assert flag.mean() <= 1e-3
    g = _np(gimg).astype(np.float32)
    g[:, flag] = 0.0
    g[np.abs(ref["image"] - target) < 1e-4] = 0.0
    img.backward(to_dev(g))
    want = O.scene_gradients(sc, g.astype(np.float64), stored=True)
    names = ("means3d", "log_scales", "quats", "opacity_logits", "sh")
    for p, k in zip(ps, names):
        assert_grad_close(_np(p.grad), want[k], k)
    if fd_params:
        rng = np.random.default_rng(seed)
        raw = dict(zip(names, [a.astype(np.float64) for a in (sc.means3d, sc.log_scales, sc.quats,
                                                               sc.opacity_logits, sc.sh)]))
        vis = np.nonzero(ref["proj"]["visible"])[0]

        def lin(r):
            pr = O.project(cam, r["means3d"], r["log_scales"], r["quats"], r["opacity_logits"], r["sh"])
            off, ids = O.tile_lists(pr["visible"], pr["depth"], pr["rect"], cam.width, cam.height)
            o = O.render_tiled(cam.width, cam.height, off, ids, pr["means2d"], pr["conic"], pr["opacity"],
                               pr["rgb"], cam.bg)
            return float((g * o["image"]).sum()), np.concatenate([o["last_id"].ravel(), o["count"].ravel()])

        checked = 0
        for _ in range(fd_params):
            k = names[rng.integers(0, 5)]
            gi = vis[rng.integers(0, len(vis))]
            idx = (gi,) + tuple(rng.integers(0, s) for s in raw[k].shape[1:])
            h = 1e-6 * max(1.0, abs(raw[k][idx]))
            rp = {a: v.copy() for a, v in raw.items()}; rm = {a: v.copy() for a, v in raw.items()}
            rp[k][idx] += h; rm[k][idx] -= h
            lp, sp = lin(rp); lm, sm = lin(rm)
            if not np.array_equal(sp, sm):
                continue
            fd = (lp - lm) / (2 * h)
            gk = dict(zip(names, ps))[k].grad[idx].item()
            scale = np.abs(want[k]).max()
            assert abs(gk - fd) <= GRAD_TOL * max(abs(fd), 1e-3 * scale), (k, idx, gk, fd)
            checked += 1
        assert checked >= fd_params // 2


@pytest.mark.parametrize("degree", [0, 3])
def test_autograd_vs_oracle_and_fd_small(degree):
    """2k-Gaussian 64x64 subset of the configuration-4 recipe (and degree 3)."""
    sc = scenes.make_fd_scene(degree=degree, n=2000, size=64, seed=404)
    _scene_grad_check(sc, fd_params=60, seed=degree)


@pytest.mark.parametrize("variant", ["plain", "local", "local_q8"])
def test_autograd_vs_oracle_medium(variant):
    sc = scenes.make_config(4, n=100000)
    sc.cameras = [scenes.look_at_camera((0, 0, 0), (0, 0, 1), 480, 270)]
    _scene_grad_check(sc, variant=variant)


@pytest.mark.slow
def test_full_size_config4_gradients():
    """Configuration 4 at full size: 3M Gaussians, 1920x1080, L1 loss."""
    sc = scenes.make_config(4)
    _scene_grad_check(sc)
