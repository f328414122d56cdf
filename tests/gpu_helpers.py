"""Shared helpers of the GPU parity tests (inputs via torch, calls via the C ABI)."""
import numpy as np
import torch

from paper_2606_16566_amd import rasterizer as R
from paper_2606_16566_amd import scenes

VARIANTS = ["plain", "hoist", "hoist_cull", "local", "hoist_cull_q8", "local_q8", "local_v4", "local_q8_v4"]


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def scene_tensors(sc):
    return [to_dev(sc.means3d), to_dev(sc.log_scales), to_dev(sc.quats), to_dev(sc.opacity_logits), to_dev(sc.sh)]


def projected_from(means2d, conic, opacity, rgb, depth, rect):
    """R.Projected from float32 screen-space attributes (render-only inputs)."""
    co = np.concatenate([np.asarray(conic, np.float32), np.asarray(opacity, np.float32)[:, None]], 1)
    splats = R.pack_splats(to_dev(np.asarray(means2d, np.float32)), to_dev(co), to_dev(np.asarray(rgb, np.float32)))
    return R.Projected(splats, to_dev(np.asarray(depth, np.float32)), to_dev(np.asarray(rect, np.int32)))


def last_ids(binned, nc, cam):
    """Gaussian id of each pixel's last contributor (-1 if none)."""
    ranges = binned.ranges.cpu().numpy().astype(np.int64)
    vals = binned.values.cpu().numpy()
    nc = nc.cpu().numpy().astype(np.int64)
    H, W = nc.shape
    ty, tx = np.meshgrid(np.arange(H) // 16, np.arange(W) // 16, indexing="ij")
    tile = ty * cam.tiles_x + tx
    pos = ranges[tile, 0] + nc - 1
    out = np.where(nc > 0, vals[np.clip(pos, 0, len(vals) - 1)], -1)
    return out


def render_only_case(seed, W, H, n, sigma=(0.3, 12.0), margin=20.0):
    rng = np.random.default_rng(seed)
    cen, con, op, col, dep = scenes.random_projected(rng, n, W, H, sigma_px=sigma, margin=margin)
    cam = scenes.look_at_camera((0, 0, 0), (0, 0, 1), W, H, bg=(0.25, 0.5, 0.125))
    return cam, cen, con, op, col, dep
