"""Torch-facing wrappers of the rasterizer's C ABI.

PyTorch provides device memory and the current HIP stream; every step of the
pipeline (projection, binning, sort, ranges, blending and their gradients)
runs in liblocalgs.so.  All tensors are float32/int32 CUDA (HIP) tensors.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

VARIANTS = {"plain": L.RENDER_PLAIN, "hoist": L.RENDER_HOIST, "hoist_cull": L.RENDER_HOIST_CULL,
            "local": L.RENDER_LOCAL}


def variant_code(variant) -> int:
    """'local' / 'plain' / ... with optional '_q8', '_v4', '_global' and
    '_fp32' suffixes (in that order, e.g. 'local_q8_v4_fp32'), or an int."""
    if isinstance(variant, int):
        return variant
    v = variant.lower()
    code = 0
    if v.endswith("_fp32"):
        v, code = v[:-5], code | L.RENDER_FP32
    if v.endswith("_global"):
        v, code = v[:-7], code | L.RENDER_GLOBAL
    if v.endswith("_v4"):
        v, code = v[:-3], code | L.RENDER_VOTE4
    if v.endswith("_q8"):
        v, code = v[:-3], code | L.RENDER_Q8
    return VARIANTS[v] | code


def backward_variant(variant) -> int:
    """The backward replay matching a forward variant: PLAIN after the plain
    renderer, LOCAL after any hoisted one, with the forward's sub-tile shape
    and precision."""
    code = variant_code(variant)
    base = L.RENDER_PLAIN if code & 0xF == L.RENDER_PLAIN else L.RENDER_LOCAL
    return base | (code & (L.RENDER_Q8 | L.RENDER_FP32 | L.RENDER_GLOBAL))


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _req(t, dtype, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    return t


@dataclass
class Projected:
    splats: torch.Tensor         # [n, SPLAT_FLOATS] records: a b c o | x y | r g b | unused
    depth: torch.Tensor          # [n]
    rect: torch.Tensor           # [n,4] int32

    @property
    def conic_opacity(self):     # [n,4] view
        return None if self.splats is None else self.splats[:, 0:4]

    @property
    def means2d(self):           # [n,2] view
        return None if self.splats is None else self.splats[:, 4:6]

    @property
    def rgb(self):               # [n,3] view
        return None if self.splats is None else self.splats[:, 6:9]


def pack_splats(means2d, conic_opacity, rgb) -> torch.Tensor:
    """Splat records [n, SPLAT_FLOATS] from separate attribute tensors [n,2],
    [n,4], [n,3] (on their device; unused floats zero)."""
    n = means2d.shape[0]
    s = torch.zeros((n, L.SPLAT_FLOATS), dtype=torch.float32, device=means2d.device)
    s[:, 0:4] = conic_opacity
    s[:, 4:6] = means2d
    s[:, 6:9] = rgb
    return s


def pack_grads(means2d, conic, opacity, rgb) -> dict:
    """Gradient records (as grad_views) from separate tensors [n,2], [n,3],
    [n], [n,3] on their device."""
    n = means2d.shape[0]
    g = torch.zeros((n, L.GRAD_FLOATS), dtype=torch.float32, device=means2d.device)
    g[:, 0:3] = conic
    g[:, 3] = opacity
    g[:, 4:6] = means2d
    g[:, 6:9] = rgb
    return grad_views(g)


def grad_views(g_splats: torch.Tensor) -> dict:
    """Named views of gradient records [n, GRAD_FLOATS] (the splat record's
    first nine fields, packed); 'splats' is the record tensor itself."""
    return dict(splats=g_splats, conic=g_splats[:, 0:3], opacity=g_splats[:, 3], means2d=g_splats[:, 4:6],
                rgb=g_splats[:, 6:9])


@dataclass
class Binned:
    tile_keys: torch.Tensor      # [capacity] int32 (uint32 bits)
    values: torch.Tensor         # [capacity] int32 (uint32 bits)
    num_pairs: torch.Tensor      # [1] int64 (device)
    overflow: torch.Tensor       # [1] int32 (device)
    ranges: torch.Tensor         # [tiles,2] int32 (uint32 bits)
    capacity: int


def project(cam, means3d, log_scales, quats, opacity_logits, sh) -> Projected:
    n = means3d.shape[0]
    dev = means3d.device
    for t, nm in ((means3d, "means3d"), (log_scales, "log_scales"), (quats, "quats"),
                  (opacity_logits, "opacity_logits"), (sh, "sh")):
        _req(t, torch.float32, nm)
    deg = int(round(sh.shape[1] ** 0.5)) - 1
    out = Projected(torch.empty((n, L.SPLAT_FLOATS), device=dev), torch.empty(n, device=dev),
                    torch.empty((n, 4), device=dev, dtype=torch.int32))
    L.check(L.lib().lgs_project(C.byref(L.camera_struct(cam)), n, deg, _p(means3d), _p(log_scales), _p(quats),
                                _p(opacity_logits), _p(sh), _p(out.splats), _p(out.depth), _p(out.rect),
                                _stream()), "lgs_project")
    return out


class Binner:
    """Keeps the pair buffers and the sort workspace between calls and grows
    them when the pair count exceeds the capacity.  exact=True: the exact
    tile assignment (only tiles the splat's alpha >= 1/255 ellipse meets),
    given the projected splats; else every tile of its rectangle."""

    def __init__(self, capacity: int = 0, exact: bool = False):
        self.capacity = int(capacity)
        self.exact = bool(exact)
        self.ws = None
        self.keys = self.vals = None
        self.num_pairs = self.overflow = None
        self.ranges = None

    def _ensure(self, n, num_tiles, dev):
        cap = max(self.capacity, 1)
        need = L.lib().lgs_sort_workspace_size(n, cap, num_tiles)
        if self.ws is None or self.ws.numel() < need or self.ws.device != dev:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        if self.keys is None or self.keys.numel() < cap or self.keys.device != dev:
            self.keys = torch.empty(cap, dtype=torch.int32, device=dev)
            self.vals = torch.empty(cap, dtype=torch.int32, device=dev)
        if self.num_pairs is None or self.num_pairs.device != dev:
            self.num_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
            self.overflow = torch.zeros(1, dtype=torch.int32, device=dev)
        if self.ranges is None or self.ranges.shape[0] != num_tiles or self.ranges.device != dev:
            self.ranges = torch.empty((num_tiles, 2), dtype=torch.int32, device=dev)

    def run(self, cam, proj: Projected, check_overflow: bool = True) -> Binned:
        n = proj.depth.shape[0]
        dev = proj.depth.device
        tx, ty = cam.tiles_x, cam.tiles_y
        for _ in range(3):
            self._ensure(n, tx * ty, dev)
            cap = max(self.capacity, 1)
            ws_base = self.ws.data_ptr()
            ws_aligned = (ws_base + 255) & ~255
            geo = self.exact and proj.splats is not None
            L.check(L.lib().lgs_sort(n, tx, ty, _p(proj.depth), _p(proj.rect), _p(proj.splats) if geo else None,
                                     _p(self.keys), _p(self.vals), cap,
                                     _p(self.num_pairs), _p(self.overflow), C.c_void_p(ws_aligned),
                                     self.ws.numel() - (ws_aligned - ws_base), _stream()), "lgs_sort")
            if check_overflow:
                p = int(self.num_pairs.item())
                if p > cap:
                    self.capacity = int(p * 1.25) + 1024
                    continue
            break
        L.check(L.lib().lgs_tile_ranges(_p(self.keys), _p(self.num_pairs), _p(self.overflow), max(self.capacity, 1),
                                        tx * ty, _p(self.ranges), _stream()), "lgs_tile_ranges")
        return Binned(self.keys, self.vals, self.num_pairs, self.overflow, self.ranges, max(self.capacity, 1))


def render(variant, cam, binned: Binned, proj: Projected, stats: torch.Tensor | None = None):
    """Blend: returns (image [3,H,W], T [H,W], n_contrib [H,W] int32)."""
    dev = proj.depth.device
    H, W = cam.height, cam.width
    img = torch.empty((3, H, W), device=dev)
    T = torch.empty((H, W), device=dev)
    nc = torch.empty((H, W), device=dev, dtype=torch.int32)
    L.check(L.lib().lgs_render(variant_code(variant), C.byref(L.camera_struct(cam)), _p(binned.ranges),
                               _p(binned.values), _p(proj.splats), _p(img), _p(T), _p(nc), _p(stats), _stream()),
            "lgs_render")
    return img, T, nc


def render_backward(variant, cam, binned: Binned, proj: Projected, T, nc, grad_rgb, grad_T=None):
    n = proj.depth.shape[0]
    dev = proj.depth.device
    g = grad_views(torch.empty((n, L.GRAD_FLOATS), device=dev))
    _req(grad_rgb, torch.float32, "grad_rgb")
    L.check(L.lib().lgs_render_backward(variant_code(variant), C.byref(L.camera_struct(cam)), n, _p(binned.ranges),
                                        _p(binned.values), _p(proj.splats), _p(T), _p(nc), _p(grad_rgb),
                                        _p(grad_T), _p(g["splats"]), _stream()), "lgs_render_backward")
    return g


def project_backward(cam, means3d, log_scales, quats, opacity_logits, sh, rect, g, clear: bool = False):
    """Raw-parameter gradients from the gradient records g["splats"]; with
    clear=True the records are zero afterwards."""
    n = means3d.shape[0]
    deg = int(round(sh.shape[1] ** 0.5)) - 1
    d = dict(means3d=torch.empty_like(means3d), log_scales=torch.empty_like(log_scales),
             quats=torch.empty_like(quats), opacity_logits=torch.empty_like(opacity_logits),
             sh=torch.empty_like(sh))
    L.check(L.lib().lgs_project_backward(C.byref(L.camera_struct(cam)), n, deg, _p(means3d), _p(log_scales),
                                         _p(quats), _p(opacity_logits), _p(sh), _p(rect), _p(g["splats"]),
                                         _p(d["means3d"]),
                                         _p(d["log_scales"]), _p(d["quats"]), _p(d["opacity_logits"]),
                                         _p(d["sh"]), L.PROJ_BWD_CLEAR if clear else 0, _stream()),
            "lgs_project_backward")
    return d


def l1_workspace(device) -> torch.Tensor:
    """Scratch for lgs_l1_loss's partial sums (one per concurrent call)."""
    return torch.empty(L.lib().lgs_l1_workspace_size() // 8, dtype=torch.float64, device=device)


def l1_loss(image, target, workspace: torch.Tensor | None = None):
    """(loss [1], grad) of mean |image - target|."""
    loss = torch.empty(1, device=image.device)
    grad = torch.empty_like(image)
    ws = l1_workspace(image.device) if workspace is None else workspace
    L.check(L.lib().lgs_l1_loss(_p(image), _p(target), image.numel(), _p(loss), _p(grad), _p(ws),
                                ws.numel() * ws.element_size(), _stream()), "lgs_l1_loss")
    return loss, grad


def rasterize(cam, means3d, log_scales, quats, opacity_logits, sh, variant="local", binner: Binner | None = None,
              stats=None, check_overflow=True):
    """Full forward pipeline for one camera.  Returns (image, T, n_contrib,
    context) where the context holds what the backward needs."""
    proj = project(cam, means3d, log_scales, quats, opacity_logits, sh)
    binner = binner or Binner(capacity=max(1024, 8 * means3d.shape[0]))
    binned = binner.run(cam, proj, check_overflow=check_overflow)
    img, T, nc = render(variant, cam, binned, proj, stats)
    return img, T, nc, (proj, binned)


class LocalGSFunction(torch.autograd.Function):
    """Differentiable rasterization of one camera with respect to the raw
    Gaussian parameters.  Outputs (image [3,H,W], T_final [H,W]); the
    last-contributor map is available through ctx only."""

    @staticmethod
    def forward(ctx, means3d, log_scales, quats, opacity_logits, sh, cam, variant, binner):
        img, T, nc, (proj, binned) = rasterize(cam, means3d, log_scales, quats, opacity_logits, sh, variant, binner)
        ctx.cam, ctx.variant = cam, variant
        ctx.proj, ctx.binned = proj, binned
        ctx.save_for_backward(means3d, log_scales, quats, opacity_logits, sh, T, nc)
        ctx.mark_non_differentiable(nc)
        return img, T, nc

    @staticmethod
    def backward(ctx, grad_img, grad_T, grad_nc):
        means3d, log_scales, quats, opacity_logits, sh, T, nc = ctx.saved_tensors
        grad_img = grad_img.contiguous() if grad_img is not None else torch.zeros((3,) + T.shape, device=T.device)
        grad_T = grad_T.contiguous() if grad_T is not None else None
        g = render_backward(backward_variant(ctx.variant), ctx.cam, ctx.binned, ctx.proj, T, nc, grad_img, grad_T)
        d = project_backward(ctx.cam, means3d, log_scales, quats, opacity_logits, sh, ctx.proj.rect, g)
        return d["means3d"], d["log_scales"], d["quats"], d["opacity_logits"], d["sh"], None, None, None
