"""Multi-view batches and step graphs.

`ViewBatch` renders up to 16 cameras of one Gaussian set with one launch per
pipeline stage: view-batched projection (raw parameters read once), one sort
over the global tile space of all views, one persistent render whose
wavefronts pull 16x4 strips from a device queue (optionally longest tile
first), and the matching backward that sums the gradients over the views.
Every buffer is allocated up front, so a whole step enqueues library calls
only and can be captured once with `StepGraph` and replayed.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .rasterizer import _p, _req, _stream, backward_variant, variant_code


def _aligned(buf: torch.Tensor):
    base = buf.data_ptr()
    a = (base + 255) & ~255
    return C.c_void_p(a), buf.numel() - (a - base)


class ViewBatch:
    """Device buffers and launch settings for rendering `cams` from n
    Gaussians of SH degree `sh_degree`.

    variant        render variant name or code (see rasterizer.variant_code)
    persistent     queue-driven render for the culling variants
    blocks_per_cu  workgroups per compute unit of the persistent render (0: 8)
    lpt            render tiles longest first (queue order, or workgroup order)
    capacity       initial pair capacity; `fit()` grows it from a measured count
    bwd_lpt        the backward takes its tiles longest first
    bwd_persistent the backward is one persistent launch of bwd_blocks_per_cu
                   workgroups per compute unit taking tiles from a queue
    exact_tiles    exact tile assignment in the sort (only the tiles a splat's
                   alpha >= 1/255 ellipse meets), else whole rectangles
    record_used    the LOCAL forward records which list entries each
                   sub-tile blended, for the backward to replay exactly those
                   (off for forward-only use: saves a compare per step)
    """

    def __init__(self, cams, n: int, sh_degree: int, variant="local_q8", persistent: bool = False,
                 blocks_per_cu: int = 0, lpt: bool = False, capacity: int = 0, device="cuda", bwd_lpt: bool = True,
                 bwd_persistent: bool = False, bwd_blocks_per_cu: int = 0, exact_tiles: bool = False,
                 record_used: bool = True):
        cams = list(cams)
        if not 1 <= len(cams) <= L.MAX_VIEWS:
            raise ValueError(f"a batch holds 1..{L.MAX_VIEWS} cameras, got {len(cams)}")
        self.cams = cams
        self.V = V = len(cams)
        self.n = int(n)
        self.deg = int(sh_degree)
        self.K = (self.deg + 1) ** 2
        self.variant = variant_code(variant)
        self.persistent = bool(persistent)
        self.blocks_per_cu = int(blocks_per_cu)
        self.lpt = bool(lpt)
        self.record_used = bool(record_used)
        self.dev = torch.device(device)
        self.cam_arr = L.camera_array(cams)
        self.tiles_x = (C.c_int32 * V)(*[c.tiles_x for c in cams])
        self.tiles_y = (C.c_int32 * V)(*[c.tiles_y for c in cams])
        self.tile_off = np.concatenate([[0], np.cumsum([c.num_tiles for c in cams])]).astype(np.int64)
        self.pix_off = np.concatenate([[0], np.cumsum([c.num_pixels for c in cams])]).astype(np.int64)
        self.num_tiles = int(self.tile_off[-1])
        self.num_pixels = int(self.pix_off[-1])
        E = V * self.n
        f32, i32, dev = torch.float32, torch.int32, self.dev
        z = lambda *shape, dtype=f32: torch.zeros(shape, dtype=dtype, device=dev)
        # projected splat records [V*n, SPLAT_FLOATS] and gradient records
        # [V*n, GRAD_FLOATS], view-major, with named views of their fields
        self.splats, self.g_splats = z(E, L.SPLAT_FLOATS), z(E, L.GRAD_FLOATS)
        self.g_clear = True         # the gradient records are known to be zero
        self.conic_opacity, self.means2d, self.rgb = self.splats[:, 0:4], self.splats[:, 4:6], self.splats[:, 6:9]
        self.g_conic, self.g_opacity = self.g_splats[:, 0:3], self.g_splats[:, 3]
        self.g_means2d, self.g_rgb = self.g_splats[:, 4:6], self.g_splats[:, 6:9]
        self.depth, self.rect = z(E), z(E, 4, dtype=i32)
        # raw-parameter gradients [n, ...], summed over views
        self.d_means3d, self.d_log_scales, self.d_quats = z(self.n, 3), z(self.n, 3), z(self.n, 4)
        self.d_logits, self.d_sh = z(self.n), z(self.n, self.K, 3)
        # packed images
        self.out_rgb, self.out_T = z(3 * self.num_pixels), z(self.num_pixels)
        self.out_nc = z(self.num_pixels, dtype=i32)
        self.grad_rgb = z(3 * self.num_pixels)
        self.loss = z(1)
        self.l1_ws = torch.empty(L.lib().lgs_l1_workspace_size() // 8, dtype=torch.float64, device=dev)
        # binning
        self.num_pairs = z(1, dtype=torch.int64)
        self.overflow = z(1, dtype=i32)
        self.ranges = z(self.num_tiles, 2, dtype=i32)
        self.queue = z(L.QUEUE_WORDS, dtype=i32)
        self.bwd_queue = z(L.QUEUE_WORDS, dtype=i32)
        self.order = z(self.num_tiles, dtype=i32)
        self.bwd_lpt = bool(bwd_lpt)
        self.bwd_persistent = bool(bwd_persistent)
        self.bwd_blocks_per_cu = int(bwd_blocks_per_cu)
        self.exact_tiles = bool(exact_tiles)
        self.order_ws = torch.empty(L.lib().lgs_tile_order_workspace_size(self.num_tiles) + 256, dtype=torch.uint8,
                                    device=dev)
        self.capacity = 0
        self._alloc_pairs(max(int(capacity), 1024))

    # -- buffers ---------------------------------------------------------
    def _alloc_pairs(self, cap: int):
        self.capacity = int(cap)
        self.keys = torch.empty(cap, dtype=torch.int32, device=self.dev)
        self.vals = torch.empty(cap, dtype=torch.int32, device=self.dev)
        need = L.lib().lgs_sort_workspace_size(self.V * self.n, cap, self.num_tiles)
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.dev)
        # used-entry masks of the LOCAL forward, read by the backward
        self.used = torch.empty(L.lib().lgs_used_mask_words(cap, self.num_tiles), dtype=torch.int64, device=self.dev)
        self.used_valid = False

    def fit(self, params, headroom: float = 1.15) -> int:
        """Run the forward once and grow the pair buffers until the pair
        count fits (host synchronisation; call before capturing)."""
        for _ in range(4):
            self.forward(params)
            p = int(self.num_pairs.item())
            if p <= self.capacity:
                return p
            self._alloc_pairs(int(p * headroom) + 1024)
        raise RuntimeError("pair count did not settle")

    def overflowed(self) -> bool:
        return bool(int(self.overflow.item()))

    # -- views of the packed outputs ---------------------------------------
    def image(self, v: int) -> torch.Tensor:
        c = self.cams[v]
        a, b = self.pix_off[v], self.pix_off[v + 1]
        return self.out_rgb[3 * a:3 * b].view(3, c.height, c.width)

    def final_T(self, v: int) -> torch.Tensor:
        c = self.cams[v]
        return self.out_T[self.pix_off[v]:self.pix_off[v + 1]].view(c.height, c.width)

    def n_contrib(self, v: int) -> torch.Tensor:
        c = self.cams[v]
        return self.out_nc[self.pix_off[v]:self.pix_off[v + 1]].view(c.height, c.width)

    def pack(self, images) -> torch.Tensor:
        """Per-view [3,H,W] tensors -> one packed buffer in the output layout."""
        return torch.cat([im.reshape(-1) for im in images]).contiguous()

    # -- the step ------------------------------------------------------------
    def _check(self, params):
        means3d, log_scales, quats, logits, sh = params
        for t, nm in ((means3d, "means3d"), (log_scales, "log_scales"), (quats, "quats"), (logits, "logits"),
                      (sh, "sh")):
            _req(t, torch.float32, nm)
        if means3d.shape[0] != self.n or sh.shape[1] != self.K:
            raise ValueError("parameters do not match the batch's n / SH degree")

    def forward(self, params, stats: torch.Tensor | None = None):
        """Enqueue project -> sort -> ranges -> [order] -> render for all views."""
        self.bin(params)
        self.render(stats)

    def configure(self, variant=None, persistent=None, blocks_per_cu=None, lpt=None, bwd_lpt=None,
                  bwd_persistent=None, bwd_blocks_per_cu=None, exact_tiles=None, record_used=None):
        """Change launch settings (e.g. from the autotuner); buffers are kept
        (a change of exact_tiles changes the pair count: re-fit)."""
        if exact_tiles is not None:
            self.exact_tiles = bool(exact_tiles)
        if record_used is not None:
            self.record_used = bool(record_used)
        if variant is not None:
            self.variant = variant_code(variant)
            self.used_valid = False            # recorded for another sub-tile shape
        if persistent is not None:
            self.persistent = bool(persistent)
        if blocks_per_cu is not None:
            self.blocks_per_cu = int(blocks_per_cu)
        if lpt is not None:
            self.lpt = bool(lpt)
        if bwd_lpt is not None:
            self.bwd_lpt = bool(bwd_lpt)
        if bwd_persistent is not None:
            self.bwd_persistent = bool(bwd_persistent)
        if bwd_blocks_per_cu is not None:
            self.bwd_blocks_per_cu = int(bwd_blocks_per_cu)

    def bin(self, params):
        """Enqueue project -> sort -> ranges for all views."""
        self.project(params)
        self.sort()

    def project(self, params):
        """Enqueue the view-batched projection."""
        self._check(params)
        lb, s = L.lib(), _stream()
        means3d, log_scales, quats, logits, sh = params
        L.check(lb.lgs_project_batch(self.cam_arr, self.V, self.n, self.deg, _p(means3d), _p(log_scales), _p(quats),
                                     _p(logits), _p(sh), _p(self.splats), _p(self.depth), _p(self.rect), s),
                "lgs_project_batch")

    def sort(self):
        """Enqueue the pair sort and the tile ranges of all views."""
        self.used_valid = False                # new lists
        lb, s = L.lib(), _stream()
        ws, wsb = _aligned(self.ws)
        ex = self.exact_tiles
        L.check(lb.lgs_sort_batch(self.V, self.tiles_x, self.tiles_y, self.n, _p(self.depth), _p(self.rect),
                                  _p(self.splats) if ex else None, _p(self.keys), _p(self.vals), self.capacity, _p(self.num_pairs), _p(self.overflow),
                                  ws, wsb, s), "lgs_sort_batch")
        L.check(lb.lgs_tile_ranges(_p(self.keys), _p(self.num_pairs), _p(self.overflow), self.capacity,
                                   self.num_tiles, _p(self.ranges), s), "lgs_tile_ranges")

    def render(self, stats: torch.Tensor | None = None):
        """Enqueue [order] -> render over the binned pairs."""
        self.tile_order()
        self.blend(stats)

    def _fwd_lpt(self):
        return self.lpt

    def tile_order(self, force: bool = False):
        """Enqueue the longest-first tile order (when the settings use it)."""
        if force or self._fwd_lpt():
            ows, owsb = _aligned(self.order_ws)
            L.check(L.lib().lgs_tile_order(_p(self.ranges), self.num_tiles, _p(self.order), ows, owsb, _stream()),
                    "lgs_tile_order")

    def blend(self, stats: torch.Tensor | None = None):
        """Enqueue the render launch itself."""
        lb, s = L.lib(), _stream()
        order = _p(self.order) if self.lpt else None
        rec = (self.variant & 0xF) == L.RENDER_LOCAL and self.record_used
        L.check(lb.lgs_render_batch(self.variant, self.cam_arr, self.V, _p(self.ranges), _p(self.vals),
                                    _p(self.splats), _p(self.out_rgb), _p(self.out_T), _p(self.out_nc), _p(stats),
                                    _p(self.queue) if self.persistent else None, order, self.blocks_per_cu,
                                    _p(self.used) if rec else None, self.used.numel(), s),
                "lgs_render_batch")
        self.used_valid = rec

    def l1(self, target_packed: torch.Tensor):
        """Enqueue L = mean |images - target| (loss -> self.loss) and its
        gradient (-> self.grad_rgb)."""
        _req(target_packed, torch.float32, "target")
        if target_packed.numel() != self.out_rgb.numel():
            raise ValueError("target does not match the packed image size")
        L.check(L.lib().lgs_l1_loss(_p(self.out_rgb), _p(target_packed), self.out_rgb.numel(), _p(self.loss),
                                    _p(self.grad_rgb), _p(self.l1_ws), self.l1_ws.numel() * 8, _stream()),
                "lgs_l1_loss")

    def backward(self, params, grad_rgb: torch.Tensor | None = None, grad_T: torch.Tensor | None = None):
        """Enqueue the gradient of the step into d_* (raw parameters, summed
        over views).  grad_rgb defaults to self.grad_rgb (set by l1).  The
        projection's backward clears the gradient records it reads, so the
        next step's blend backward adds into zero records without a clear."""
        self._check(params)
        self.backward_render(grad_rgb, grad_T, accumulate=self.g_clear)
        self.backward_project(params, clear=True)

    def backward_render(self, grad_rgb: torch.Tensor | None = None, grad_T: torch.Tensor | None = None,
                        stats: torch.Tensor | None = None, accumulate: bool = False):
        """Enqueue the blend's backward into the projected gradients g_*
        (overwritten, or added to with accumulate=True)."""
        self.g_clear = False
        lb, s = L.lib(), _stream()
        g = self.grad_rgb if grad_rgb is None else _req(grad_rgb, torch.float32, "grad_rgb")
        bv = backward_variant(self.variant) | (L.BWD_ACCUMULATE if accumulate else 0)
        if self.bwd_lpt and not self._fwd_lpt():
            self.tile_order(force=True)                  # the forward did not compute it
        L.check(lb.lgs_render_backward_batch(bv, self.cam_arr, self.V, self.V * self.n, _p(self.ranges),
                                             _p(self.vals), _p(self.splats), _p(self.out_T), _p(self.out_nc), _p(g),
                                             _p(grad_T), _p(self.g_splats), _p(self.order) if self.bwd_lpt else None,
                                             _p(self.bwd_queue) if self.bwd_persistent else None,
                                             self.bwd_blocks_per_cu, _p(stats),
                                             _p(self.used) if self.used_valid else None, self.used.numel(), s),
                "lgs_render_backward_batch")

    def backward_project(self, params, clear: bool = False):
        """Enqueue the projection's backward into the raw-parameter gradients;
        clear=True sets the gradient records back to zero as they are read."""
        self._check(params)
        lb, s = L.lib(), _stream()
        means3d, log_scales, quats, logits, sh = params
        L.check(lb.lgs_project_backward_batch(self.cam_arr, self.V, self.n, self.deg, _p(means3d), _p(log_scales),
                                              _p(quats), _p(logits), _p(sh), _p(self.rect), _p(self.g_splats),
                                              _p(self.d_means3d), _p(self.d_log_scales), _p(self.d_quats),
                                              _p(self.d_logits), _p(self.d_sh), L.PROJ_BWD_CLEAR if clear else 0, s),
                "lgs_project_backward_batch")
        if clear:
            self.g_clear = True

    def train_step(self, params, target_packed):
        """forward + L1 + backward, all enqueued."""
        self.forward(params)
        self.l1(target_packed)
        self.backward(params)

    def grads(self):
        return dict(means3d=self.d_means3d, log_scales=self.d_log_scales, quats=self.d_quats,
                    opacity_logits=self.d_logits, sh=self.d_sh)


class StepGraph:
    """A sequence of library calls captured once as a HIP graph and replayed.

    `fn` must only enqueue library work on the current stream (no host reads,
    no tensor allocation); it runs `warmup` times eagerly, then once under
    capture on a private stream.  `replay()` launches the whole sequence on
    the caller's current stream.
    """

    def __init__(self, fn, warmup: int = 1):
        self.stream = torch.cuda.Stream()
        self.handle = None
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            for _ in range(warmup):
                fn()
        self.stream.synchronize()
        h = C.c_void_p()
        sp = C.c_void_p(self.stream.cuda_stream)
        with torch.cuda.stream(self.stream):
            L.check(L.lib().lgs_graph_begin(sp), "lgs_graph_begin")
            try:
                fn()
            finally:
                st = L.lib().lgs_graph_end(sp, C.byref(h))
            L.check(st, "lgs_graph_end")
        self.handle = h

    def replay(self):
        """Launch the graph on the caller's current stream (ordered with the
        caller's other work on that stream like any kernel launch)."""
        if self.handle is None:
            raise RuntimeError("graph destroyed")
        L.check(L.lib().lgs_graph_launch(self.handle, _stream()), "lgs_graph_launch")

    def close(self):
        if self.handle is not None:
            L.check(L.lib().lgs_graph_destroy(self.handle), "lgs_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CapturedStep:
    """A ViewBatch step (`fn`, which enqueues library calls on `vb`'s
    buffers) captured once as a graph and replayed, grown and re-captured
    when the pair count outgrows the capacity it was captured with.

    A replay never synchronises the host.  `check()` does (it reads the
    overflow flag the sort left on the device): if the last replay
    overflowed, its outputs are invalid (every tile list came out empty); the
    pair buffers are then regrown to the pair count the sort reported, with
    `headroom`, the step is captured again on the new buffers and replayed.
    """

    def __init__(self, vb: ViewBatch, fn, headroom: float = 1.15, warmup: int = 1):
        self.vb, self.fn, self.headroom, self.warmup = vb, fn, float(headroom), int(warmup)
        self.recaptures = 0
        self.graph = StepGraph(fn, warmup=self.warmup)

    def replay(self):
        self.graph.replay()

    def check(self, max_grow: int = 4) -> bool:
        """True if the last replay had overflowed (and has now been redone on
        grown buffers)."""
        grown = False
        for _ in range(max_grow):
            torch.cuda.current_stream().synchronize()
            if not self.vb.overflowed():
                return grown
            p = int(self.vb.num_pairs.item())
            self.graph.close()
            self.vb._alloc_pairs(int(p * self.headroom) + 1024)
            self.graph = StepGraph(self.fn, warmup=self.warmup)
            self.recaptures += 1
            self.graph.replay()
            grown = True
        raise RuntimeError("pair count did not settle")

    def close(self):
        self.graph.close()
