"""Multi-view batches, persistent render, longest-first order and step graphs.

Forward: every view of a batch equals the single-view pipeline bitwise
(image, final T, last contributor), in grid and persistent mode and with
either tile order; one view is also checked against the FP64 oracle at the
forward tolerance (2e-4).  Backward: the batch's raw-parameter gradients equal
the sum of the per-view gradients up to float summation order (relative 2e-5
of each tensor's scale); the per-view projected gradients agree likewise.
Graphs: a captured forward + L1 + backward step, replayed several times with
eager work and synchronisations between the replays, matches the eager step
after every replay.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_16566_amd import _lib as L
from paper_2606_16566_amd import batch as B
from paper_2606_16566_amd import rasterizer as R
from paper_2606_16566_amd import scenes
from tests.gpu_helpers import scene_tensors, to_dev

pytestmark = pytest.mark.gpu

SUM_TOL = 2e-5


def ring_cameras(sizes, radius=12.0):
    cams = []
    for v, (w, h) in enumerate(sizes):
        th = 2.0 * math.pi * v / len(sizes)
        cams.append(scenes.look_at_camera((radius * math.sin(th), 0.0, -radius * math.cos(th)), (0, 0, 0), w, h,
                                          bg=(0.125, 0.25, 0.0)))
    return cams


def single_view(cam, params, variant):
    img, T, nc, _ = R.rasterize(cam, *params, variant=variant, binner=R.Binner(capacity=0), check_overflow=True)
    torch.cuda.synchronize()
    return img.cpu().numpy(), T.cpu().numpy(), nc.cpu().numpy()


def _close_scaled(got, want, name, tol=SUM_TOL):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = max(np.abs(want).max(), 1e-30)
    err = np.abs(got - want).max() / scale
    assert err <= tol, (name, err)


@pytest.mark.parametrize("variant", ["local", "plain", "hoist_cull", "local_fp32", "local_q8_v4"])
def test_batch_forward_bitwise_small(variant):
    sc = scenes.make_config(5, n=20000)
    cams = ring_cameras([(160, 120), (203, 150), (96, 64), (33, 47)])
    params = scene_tensors(sc)
    modes = [dict(persistent=False), dict(persistent=False, lpt=True), dict(persistent=True, lpt=False),
             dict(persistent=True, lpt=True, blocks_per_cu=2)]
    refs = [single_view(c, params, variant) for c in cams]
    for mode in modes:
        vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant=variant, **mode)
        vb.fit(params)
        vb.forward(params)
        torch.cuda.synchronize()
        assert not vb.overflowed()
        for v, (img, T, nc) in enumerate(refs):
            assert np.array_equal(vb.image(v).cpu().numpy(), img), (mode, v)
            assert np.array_equal(vb.final_T(v).cpu().numpy(), T), (mode, v)
            assert np.array_equal(vb.n_contrib(v).cpu().numpy(), nc), (mode, v)


def test_batch_forward_bitwise_wide_view():
    """A view wider than 256 tiles sends the whole batch down the stored
    duplication path; the narrow view must still match its single-view
    (column-first) result bitwise, and the wide one its own."""
    sc = scenes.make_config(5, n=20000)
    cams = ring_cameras([(4200, 64), (160, 120)])
    params = scene_tensors(sc)
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant="local")
    vb.fit(params)
    vb.forward(params)
    torch.cuda.synchronize()
    assert not vb.overflowed()
    for v, c in enumerate(cams):
        img, T, nc = single_view(c, params, "local")
        assert np.array_equal(vb.image(v).cpu().numpy(), img), v
        assert np.array_equal(vb.final_T(v).cpu().numpy(), T), v
        assert np.array_equal(vb.n_contrib(v).cpu().numpy(), nc), v


def test_batch_forward_bitwise_mixed_sizes():
    """Four views of the 16-view clustered recipe at its own resolutions."""
    sc = scenes.make_config(5, n=100000)
    cams = sc.cameras[:4]
    params = scene_tensors(sc)
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant="local", persistent=True, lpt=True)
    vb.fit(params)
    vb.forward(params)
    torch.cuda.synchronize()
    for v, c in enumerate(cams):
        img, T, nc = single_view(c, params, "local")
        assert np.array_equal(vb.image(v).cpu().numpy(), img), v
        assert np.array_equal(vb.final_T(v).cpu().numpy(), T), v
        assert np.array_equal(vb.n_contrib(v).cpu().numpy(), nc), v


def test_batch_view_matches_oracle():
    sc = scenes.make_config(5, n=4000)
    cams = ring_cameras([(120, 90), (96, 80), (64, 64)])
    sc.cameras = cams
    params = scene_tensors(sc)
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant="local", persistent=True, lpt=True)
    vb.fit(params)
    vb.forward(params)
    torch.cuda.synchronize()
    for v in range(len(cams)):
        ref = O.render_scene(sc, view=v, stored=True)
        flag = O.flagged(ref["margin"], 1e-5)
        assert flag.mean() <= 1e-3
        got = vb.image(v).cpu().numpy().astype(np.float64)
        err = np.abs(got - ref["image"])[:, ~flag]
        assert err.size > 0 and err.max() <= 2e-4, (v, err.max())


def test_tile_order_is_longest_first_permutation():
    sc = scenes.make_config(5, n=50000)
    cams = ring_cameras([(320, 240), (256, 256)])
    params = scene_tensors(sc)
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, persistent=True, lpt=True)
    vb.fit(params)
    vb.forward(params)
    torch.cuda.synchronize()
    order = vb.order.cpu().numpy().astype(np.int64)
    rng_ = vb.ranges.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(vb.num_tiles))
    length = (rng_[:, 1] - rng_[:, 0])[order]
    # classes split each octave into 8 equal steps: a later tile is never
    # 9/8 times as long as an earlier one, and the longest class comes first
    run_max = np.maximum.accumulate(length[::-1])[::-1]
    assert np.all(run_max[1:] < np.maximum(length[:-1], 1) * 1.125)
    # within a class the tiles keep index order
    same = length[1:] == length[:-1]
    assert np.all(order[1:][same] > order[:-1][same])
    # empty tiles last
    nz = np.nonzero(length)[0]
    if nz.size < length.size:
        assert np.all(length[nz.max() + 1:] == 0)


@pytest.mark.parametrize("variant,bwd_lpt,bwd_persistent,bpc", [
    ("local", True, False, 0), ("local", False, False, 0), ("local", True, True, 4), ("local", False, True, 2),
    ("local_q8", True, True, 4), ("local_q8_v4", True, True, 8), ("plain", True, True, 4), ("plain", False, False, 0),
    ("local_q8_fp32", True, True, 4)])
def test_batch_backward_equals_sum_of_views(variant, bwd_lpt, bwd_persistent, bpc):
    """The batch backward (one launch over the tiles of all views, grid or
    persistent queue, index or longest-first order) equals the sum of the
    single-view backwards; mixed view sizes with ragged edge tiles."""
    sc = scenes.make_config(5, n=6000)
    cams = ring_cameras([(128, 96), (100, 100), (64, 48), (37, 53)])
    params = scene_tensors(sc)
    rng = np.random.default_rng(7)
    gCs = [rng.standard_normal((3, c.height, c.width)).astype(np.float32) for c in cams]
    print(f"batch backward {variant} lpt={bwd_lpt} persistent={bwd_persistent} bpc={bpc}", flush=True)
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant=variant, bwd_lpt=bwd_lpt, bwd_persistent=bwd_persistent,
                     bwd_blocks_per_cu=bpc)
    vb.fit(params)
    vb.forward(params)
    # the blend's backward and the projection's backward separately, to check
    # the gradient records in between; the projection's backward clears them
    vb.backward_render(grad_rgb=vb.pack([to_dev(g) for g in gCs]), accumulate=vb.g_clear)
    torch.cuda.synchronize()
    g_records = vb.g_splats.clone()
    vb.backward_project(params, clear=True)
    torch.cuda.synchronize()
    assert not bool(vb.g_splats.any()), "the projection's backward left nonzero gradient records"
    vb.g_splats.copy_(g_records)
    want = {k: 0.0 for k in ("means3d", "log_scales", "quats", "opacity_logits", "sh")}
    for v, c in enumerate(cams):
        img, T, nc, (proj, binned) = R.rasterize(c, *params, variant=variant, binner=R.Binner(capacity=0))
        g = R.render_backward(R.backward_variant(variant), c, binned, proj, T, nc, to_dev(gCs[v]))
        d = R.project_backward(c, *params, proj.rect, g)
        torch.cuda.synchronize()
        sl = slice(v * sc.n, (v + 1) * sc.n)
        _close_scaled(vb.g_means2d[sl].cpu().numpy(), g["means2d"].cpu().numpy(), f"means2d[{v}]")
        _close_scaled(vb.g_conic[sl].cpu().numpy(), g["conic"].cpu().numpy(), f"conic[{v}]")
        _close_scaled(vb.g_opacity[sl].cpu().numpy(), g["opacity"].cpu().numpy(), f"opacity[{v}]")
        _close_scaled(vb.g_rgb[sl].cpu().numpy(), g["rgb"].cpu().numpy(), f"rgb[{v}]")
        for k in want:
            want[k] = want[k] + d[k].cpu().numpy().astype(np.float64)
    got = vb.grads()
    for k in want:
        _close_scaled(got[k].cpu().numpy(), want[k], k)


def test_consecutive_steps_do_not_carry_gradients():
    """The batch's step clears the gradient records in the projection's
    backward and the next step adds into them without a clear: two steps on
    the same parameters give the same raw gradients (up to the order of the
    float atomics), also when the visible set changes between steps."""
    sc = scenes.make_config(5, n=8000)
    cams = ring_cameras([(128, 96), (100, 100), (64, 48)])
    params = scene_tensors(sc)
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant="local_q8_v4", bwd_persistent=True, bwd_blocks_per_cu=4)
    vb.fit(params)
    rng = np.random.default_rng(3)
    target = torch.from_numpy(rng.uniform(0, 1, size=vb.out_rgb.numel()).astype(np.float32)).cuda()
    moved = [p.clone() for p in params]
    moved[0].add_(0.05)                          # shifts the means: another visible set
    runs = []
    for ps in (params, params, moved, params):
        vb.fit(ps)
        vb.train_step(ps, target)
        torch.cuda.synchronize()
        runs.append({k: v.cpu().numpy().copy() for k, v in vb.grads().items()})
        assert vb.g_clear and not bool(vb.g_splats.any())
    for k in runs[0]:
        _close_scaled(runs[1][k], runs[0][k], f"{k} second step", tol=1e-5)
        _close_scaled(runs[3][k], runs[0][k], f"{k} after a different visible set", tol=1e-5)


def test_step_graph_replays_match_eager():
    sc = scenes.make_config(5, n=8000)
    cams = ring_cameras([(128, 96), (96, 96)])
    params = scene_tensors(sc)
    rng = np.random.default_rng(11)
    target = to_dev(rng.uniform(0, 1, size=3 * sum(c.num_pixels for c in cams)).astype(np.float32))
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant="local", persistent=True, lpt=True)
    vb.fit(params)
    graph = B.StepGraph(lambda: vb.train_step(params, target))
    try:
        for rep in range(3):
            # eager work between replays: perturb the parameters in place
            with torch.no_grad():
                params[0].add_(torch.randn_like(params[0]) * 1e-3)
                params[4].mul_(1.0 + 1e-3 * rep)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            g_img = vb.out_rgb.clone()
            g_loss = vb.loss.clone()
            g_d = {k: t.clone() for k, t in vb.grads().items()}
            assert not vb.overflowed()
            vb.train_step(params, target)
            torch.cuda.synchronize()
            assert torch.equal(g_img, vb.out_rgb), rep
            assert abs(float(g_loss) - float(vb.loss)) <= 1e-6 * abs(float(vb.loss)), rep
            for k, t in vb.grads().items():
                _close_scaled(g_d[k].cpu().numpy(), t.cpu().numpy(), f"{k}@{rep}")
    finally:
        graph.close()


def test_backward_stats_count_replayed_steps():
    """The backward's counters: replayed steps <= candidate steps, taken
    pairs <= 64 x replayed steps, identical in grid and persistent mode."""
    sc = scenes.make_config(5, n=8000)
    cams = ring_cameras([(160, 120), (96, 64)])
    params = scene_tensors(sc)
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant="local_q8")
    vb.fit(params)
    vb.forward(params)
    rng = np.random.default_rng(3)
    vb.grad_rgb.copy_(to_dev(rng.standard_normal(vb.grad_rgb.numel()).astype(np.float32)))
    res = []
    for pers in (False, True):
        vb.configure(bwd_persistent=pers, bwd_blocks_per_cu=2)
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        vb.backward_render(stats=st)
        res.append(st.cpu().numpy())
    for st in res:
        assert 0 < st[1] <= st[0] and 0 < st[2] <= 64 * st[1] and st[3] == 64 * st[1]
    assert np.array_equal(res[0][:4], res[1][:4])


@pytest.mark.parametrize("variant,persistent", [("local_q8", True), ("local", False), ("local_q8_v4", True)])
def test_backward_replays_exactly_the_used_entries(variant, persistent):
    """With the forward's used-entry masks the backward visits exactly the
    entries some pixel of each sub-tile blended: every candidate step is
    replayed (candidates == replayed steps), the steps replayed and pairs
    taken equal those without the masks, and the gradients agree with the
    culling-driven replay up to the order of float atomics."""
    sc = scenes.make_config(5, n=12000)
    cams = ring_cameras([(160, 120), (96, 64), (203, 150)])
    params = scene_tensors(sc)
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant=variant, persistent=persistent, blocks_per_cu=2,
                     bwd_persistent=True, bwd_blocks_per_cu=2)
    vb.fit(params)
    vb.forward(params)
    assert vb.used_valid
    rng = np.random.default_rng(11)
    vb.grad_rgb.copy_(to_dev(rng.standard_normal(vb.grad_rgb.numel()).astype(np.float32)))
    runs = []
    for with_masks in (True, False):
        vb.used_valid = with_masks
        st = torch.zeros(8, dtype=torch.int64, device="cuda")
        vb.backward_render(stats=st)
        torch.cuda.synchronize()
        runs.append((st.cpu().numpy(), vb.g_splats.cpu().numpy().astype(np.float64)))
    (sm, gm), (sc_, gc) = runs
    print(f"{variant}: candidates with masks {sm[0]} (replayed {sm[1]}), with culling {sc_[0]} (replayed {sc_[1]})",
          flush=True)
    assert sm[0] == sm[1] == sc_[1] and sm[2] == sc_[2] and sc_[0] >= sc_[1]
    _close_scaled(gm, gc, "gradient records", tol=1e-5)
    # a forward that records no masks (the kernel without the per-step
    # compare) renders the same images, and the backward then culls itself
    img = vb.out_rgb.clone(), vb.out_T.clone(), vb.out_nc.clone()
    vb.configure(record_used=False)
    vb.forward(params)
    assert not vb.used_valid
    assert torch.equal(img[0], vb.out_rgb) and torch.equal(img[1], vb.out_T) and torch.equal(img[2], vb.out_nc)
    vb.backward_render()
    torch.cuda.synchronize()
    _close_scaled(vb.g_splats.cpu().numpy().astype(np.float64), gm, "gradient records without masks", tol=1e-5)


def test_captured_step_grows_and_recaptures():
    """A captured step whose pair count outgrows its capacity (the splats
    grow between replays) overflows, and check() regrows the buffers,
    captures again and redoes the step: then it equals the eager step."""
    sc = scenes.make_config(5, n=8000)
    cams = ring_cameras([(128, 96), (96, 96)])
    params = scene_tensors(sc)
    rng = np.random.default_rng(12)
    target = to_dev(rng.uniform(0, 1, size=3 * sum(c.num_pixels for c in cams)).astype(np.float32))
    vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant="local_q8", persistent=True, lpt=True,
                     bwd_persistent=True)
    vb.fit(params, headroom=1.05)
    cap0 = vb.capacity
    step = B.CapturedStep(vb, lambda: vb.train_step(params, target), headroom=1.1)
    try:
        step.replay()
        assert step.check() is False and step.recaptures == 0
        with torch.no_grad():
            params[1].add_(3.0)                           # 20x larger splats: 2.4x the pairs
        step.replay()
        assert step.check() is True and step.recaptures >= 1 and vb.capacity > cap0
        assert not vb.overflowed()
        g_img = vb.out_rgb.clone()
        g_d = {k: t.clone() for k, t in vb.grads().items()}
        step.replay()
        assert step.check() is False
        assert torch.equal(g_img, vb.out_rgb)
        vb.train_step(params, target)
        torch.cuda.synchronize()
        assert torch.equal(g_img, vb.out_rgb)
        for k, t in vb.grads().items():
            _close_scaled(g_d[k].cpu().numpy(), t.cpu().numpy(), k)
    finally:
        step.close()


def test_single_view_batch_equals_plain_entry_points():
    """num_views = 1 through the batch entry points == the single-view calls."""
    sc = scenes.make_config(1, n=5000)
    cam = sc.cameras[0]
    params = scene_tensors(sc)
    vb = B.ViewBatch([cam], sc.n, sc.sh_degree, variant="local", persistent=False)
    vb.fit(params)
    vb.forward(params)
    proj = R.project(cam, *params)
    torch.cuda.synchronize()
    for a, b in ((vb.means2d, proj.means2d), (vb.conic_opacity, proj.conic_opacity), (vb.rgb, proj.rgb),
                 (vb.depth, proj.depth), (vb.rect, proj.rect)):
        assert torch.equal(a, b)


def test_batch_exact_tiles_equal_rectangles():
    """The batch in exact-tile mode: the same images bitwise and gradients up
    to float summation order as with whole rectangles, with fewer pairs."""
    sc = scenes.make_config(5, n=20000)
    cams = ring_cameras([(160, 120), (203, 150), (96, 64), (33, 47)])
    params = scene_tensors(sc)
    rng = np.random.default_rng(9)
    target = to_dev(rng.uniform(0, 1, size=3 * sum(c.num_pixels for c in cams)).astype(np.float32))
    out = {}
    for exact in (False, True):
        vb = B.ViewBatch(cams, sc.n, sc.sh_degree, variant="local_q8_v4", persistent=True, lpt=True,
                         bwd_persistent=True, exact_tiles=exact)
        vb.fit(params)
        vb.train_step(params, target)
        torch.cuda.synchronize()
        out[exact] = (vb.out_rgb.clone(), vb.out_T.clone(), int(vb.num_pairs.item()),
                      {k: t.cpu().numpy() for k, t in vb.grads().items()})
    assert out[True][2] < out[False][2]
    assert torch.equal(out[True][0], out[False][0]) and torch.equal(out[True][1], out[False][1])
    for k in out[True][3]:
        _close_scaled(out[True][3][k], out[False][3][k], k)
