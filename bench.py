"""Benchmark: rendering throughput (Mpix/s) of the Local-GS pipeline on one
MI355X, against the plain per-pixel renderer on the same GPU.

Headline workload: 1M Gaussians, SH degree 3, one 1920x1080 view (uniform
cloud 4 units in front of the camera; see paper_2606_16566_amd/scenes.py).
A step is one whole forward pass: projection, binning (depth sort, pair
duplication, tile sort), tile ranges, [tile order] and blending, with inputs
resident in HBM.  The render launch settings come from the autotuner
(median render time among settings whose image matches the reference
setting); the plain renderer runs the same pipeline with its own kernel.

Also reported: forward + L1 + backward (3M Gaussians, 1920x1080, SH degree 0)
as a captured step graph, and the 16-view batch (10M clustered Gaussians,
mixed resolutions) forward + backward as one captured graph.

Prints one JSON line.  `roofline` covers the dominant kernel (the blend),
whose average launch duration is measured with HIP events on the stream it
is launched on; `cpu_baseline` times the FP64 oracle on this host for one
full frame of the headline workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# full-rate VALU lane operations: 256 CUs x 4 SIMD16 x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic lane operations per evaluated (pixel, Gaussian) pair of the
# uniform blend: 5 FMA dot product, exp, clamp, select, w = alpha*T, 3 FMA
# colour, T update, termination compare
OPS_PER_PAIR = 14

# HBM bytes per launch of the blend kernel, from the rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs summarised in profiles/forward_uniform-1M-1920x1080-sh3_
# hbm_counters.md (24.7 MiB read, 41.3 MiB written, after the copy-kernel
# calibration), valid for the variant, workload and kernel sources they were
# taken with; anything else reports null.
RENDER_TRAFFIC = {"variant": 0x63, "sources_sha": "1c0df08ca7f369ae", "bytes": (24.7 + 41.3) * 2 ** 20,
                  "workload": 2}
RENDER_SOURCES = ("paper_2606_16566_amd/csrc/render.hip", "paper_2606_16566_amd/csrc/render_common.hpp",
                  "paper_2606_16566_amd/csrc/common.hpp")


def render_traffic(variant: int, config: int):
    import hashlib
    h = hashlib.sha256()
    for f in RENDER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    ok = (h.hexdigest()[:16] == RENDER_TRAFFIC["sources_sha"] and variant == RENDER_TRAFFIC["variant"]
          and config == RENDER_TRAFFIC["workload"])
    return RENDER_TRAFFIC["bytes"] if ok else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--extra", action="store_true", help="also time every render variant")
    ap.add_argument("--no-fwdbwd", action="store_true", help="skip the forward+backward workload")
    ap.add_argument("--no-multiview", action="store_true", help="skip the 16-view batch workload")
    ap.add_argument("--only", choices=["forward", "fwdbwd", "multiview"], default=None,
                    help="run one workload alone (profiling); prints its JSON section")
    ap.add_argument("--render", default=None,
                    help="render variant for the Local pipeline instead of the autotuner's choice (e.g. local_q8_v4)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first copy this many MiB device-to-device (calibrates HBM byte counters)")
    ap.add_argument("--no-tune", action="store_true", help="default render settings instead of the autotuner")
    ap.add_argument("--tune-cache", default=None, help="autotuner JSON cache (default ~/.cache/localgs)")
    ap.add_argument("--retune", action="store_true", help="ignore cached autotuner results")
    return ap.parse_args()


def tensors(sc, torch, grad=False):
    dev = torch.device("cuda:0")
    out = [torch.from_numpy(a).to(dev) for a in (sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh)]
    if grad:
        for t in out:
            t.requires_grad_()
    return out


def timed_forward(vb, params, steps, warmup, torch, np):
    """Per-step stage times (HIP events on the launching stream) and wall
    time per step of vb.forward."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        vb.forward(params)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    t0 = time.perf_counter()
    for e in ev:
        e[0].record(stream)
        vb.project(params)
        e[1].record(stream)
        vb.sort()
        e[2].record(stream)
        vb.tile_order()
        e[3].record(stream)
        vb.blend()
        e[4].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    if vb.overflowed():
        raise RuntimeError("pair capacity overflow inside the timed region")
    st = lambda i: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in ev]))
    return dict(wall_ms=wall, project_ms=st(0), sort_ms=st(1), order_ms=st(2), render_ms=st(3),
                num_pairs=int(vb.num_pairs.item()))


def timed_graph(step, steps, warmup, torch):
    """Wall time per replay of a captured step."""
    from paper_2606_16566_amd.batch import StepGraph
    g = StepGraph(step, warmup=1)
    try:
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps
    finally:
        g.close()


def fwdbwd_single(args, torch, np):
    """Forward + L1 + backward, one 1920x1080 view of 3M Gaussians (SH 0):
    captured step graph (Local and Plain) and the eager autograd Function."""
    from paper_2606_16566_amd import autotune, scenes
    from paper_2606_16566_amd import rasterizer as R
    from paper_2606_16566_amd.batch import ViewBatch
    sc = scenes.make_config(4)
    cam = sc.cameras[0]
    params = tensors(sc, torch)
    target = torch.from_numpy(scenes.make_target(cam.height, cam.width, 104)).cuda().reshape(-1)
    vb = ViewBatch([cam], sc.n, sc.sh_degree)
    tuned = autotune.tune(vb, params, cache_path=args.tune_cache, use_cache=not args.retune) if not args.no_tune \
        else None
    steps = max(5, args.steps // 2)
    res = {}
    vb.fit(params)
    ms_local = timed_graph(lambda: vb.train_step(params, target), steps, 2, torch)
    vb.configure(variant="plain", persistent=False, lpt=False)
    ms_plain = timed_graph(lambda: vb.train_step(params, target), steps, 2, torch)
    if vb.overflowed():
        raise RuntimeError("pair capacity overflow in the forward+backward workload")
    px = cam.width * cam.height
    res["local"] = {"ms_per_step": ms_local, "mpix_s": px / (ms_local * 1e-3) / 1e6}
    res["plain"] = {"ms_per_step": ms_plain, "mpix_s": px / (ms_plain * 1e-3) / 1e6}
    res["local_over_plain"] = ms_plain / ms_local
    res["tuned"] = tuned["best"] if tuned else None
    res["workload"] = f"{scenes.CONFIG_NAMES[4]}: forward + L1 loss + backward to raw parameters, step graph"
    del vb
    # eager autograd path (torch.autograd.Function + L1 kernel)
    gp = [p.detach().clone().requires_grad_() for p in params]
    binner = R.Binner(capacity=0)
    R.rasterize(cam, *[p.detach() for p in gp], variant="local", binner=binner, check_overflow=True)
    img_target = target.view(3, cam.height, cam.width)

    def step():
        for p in gp:
            p.grad = None
        img, T, nc = R.LocalGSFunction.apply(*gp, cam, "local", binner)
        loss, g = R.l1_loss(img.detach(), img_target)
        img.backward(g)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    res["autograd_local"] = {"ms_per_step": ms, "mpix_s": px / (ms * 1e-3) / 1e6}
    return res


def multiview(args, torch, np):
    """16 views (mixed resolutions) of 10M clustered Gaussians, SH degree 3:
    one captured graph of forward + L1 + backward over the whole batch."""
    from paper_2606_16566_amd import autotune, scenes
    from paper_2606_16566_amd.batch import ViewBatch
    sc = scenes.make_config(5)
    params = tensors(sc, torch)
    vb = ViewBatch(sc.cameras, sc.n, sc.sh_degree)
    tuned = autotune.tune(vb, params, cache_path=args.tune_cache, use_cache=not args.retune, reps=3) \
        if not args.no_tune else None
    vb.fit(params)
    rng = np.random.default_rng(105)
    target = torch.from_numpy(rng.uniform(0, 1, size=3 * vb.num_pixels).astype(np.float32)).cuda()
    steps = max(3, args.steps // 4)
    ms_fwd = timed_graph(lambda: vb.forward(params), steps, 1, torch)
    ms = timed_graph(lambda: vb.train_step(params, target), steps, 1, torch)
    if vb.overflowed():
        raise RuntimeError("pair capacity overflow in the multi-view batch")
    px = vb.num_pixels
    return {"workload": f"{scenes.CONFIG_NAMES[5]}: 16 views in one batch, step graph",
            "pixels": px, "pairs": int(vb.num_pairs.item()), "tiles": vb.num_tiles,
            "fwd": {"ms_per_step": ms_fwd, "mpix_s": px / (ms_fwd * 1e-3) / 1e6},
            "fwd_bwd": {"ms_per_step": ms, "mpix_s": px / (ms * 1e-3) / 1e6},
            "tuned": tuned["best"] if tuned else None}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2606_16566_amd import autotune, scenes
    from paper_2606_16566_amd.batch import ViewBatch

    if args.calib_copy_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counter
        # readings give the scale from counter units to bytes
        nel = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nel, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only == "fwdbwd":
        print(json.dumps({"fwd_bwd": fwdbwd_single(args, torch, np)}), flush=True)
        return
    if args.only == "multiview":
        print(json.dumps({"multiview": multiview(args, torch, np)}), flush=True)
        return
    if args.only == "forward":
        args.no_fwdbwd = args.no_multiview = args.no_cpu = True

    sc = scenes.make_config(args.config)
    cam = sc.cameras[0]
    params = tensors(sc, torch)
    vb = ViewBatch([cam], sc.n, sc.sh_degree, variant=args.render or "local", persistent=False)
    tuned = None
    if not args.no_tune and not args.render:
        tuned = autotune.tune(vb, params, cache_path=args.tune_cache, use_cache=not args.retune)
    vb.fit(params)
    torch.cuda.synchronize()
    local_settings = (vb.variant, vb.persistent, vb.blocks_per_cu, vb.lpt)
    res = timed_forward(vb, params, args.steps, args.warmup, torch, np)
    res["graph_ms"] = timed_graph(lambda: vb.forward(params), args.steps, args.warmup, torch)
    vb.configure(variant="plain", persistent=False, lpt=False)
    base = timed_forward(vb, params, args.steps, args.warmup, torch, np)
    base["graph_ms"] = timed_graph(lambda: vb.forward(params), args.steps, args.warmup, torch)
    vb.configure(variant=local_settings[0], persistent=local_settings[1], blocks_per_cu=local_settings[2],
                 lpt=local_settings[3])
    if vb.overflowed():
        raise RuntimeError("pair capacity overflow inside the timed region")
    px = cam.width * cam.height
    # a step is one forward pass replayed from its captured graph (the same
    # kernels as the eager launches, without per-launch host work)
    ms_step, ms_base = res["graph_ms"], base["graph_ms"]
    mpix = px / (ms_step * 1e-3) / 1e6
    mpix_base = px / (ms_base * 1e-3) / 1e6

    # parity of the timed settings against the plain renderer (same GPU)
    vb.forward(params)
    img_local = vb.out_rgb.clone()
    vb.configure(variant="plain", persistent=False, lpt=False)
    vb.forward(params)
    diff = (vb.out_rgb - img_local).abs().view(3, -1).amax(0)
    parity = {"max_abs_diff_vs_plain": float(diff.max()), "pixels_over_2e-4": int((diff > 2e-4).sum())}
    vb.configure(variant=local_settings[0], persistent=local_settings[1], blocks_per_cu=local_settings[2],
                 lpt=local_settings[3])

    # counters of the dominant kernel (separate, untimed instantiation)
    vb.bin(params)
    vb.tile_order()
    st = torch.zeros(8, dtype=torch.int64, device="cuda:0")
    vb.blend(stats=st)
    st = st.cpu().numpy()
    lane_evals = int(st[3])
    achieved = lane_evals * OPS_PER_PAIR / (res["render_ms"] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": f"render_wave_kernel (variant code {vb.variant})", "achieved": achieved,
                "peak": PEAK_VALU_TOPS, "unit": "Tops/s (full-rate VALU lane ops)",
                "frac": achieved / PEAK_VALU_TOPS, "traffic": render_traffic(vb.variant, args.config),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE, calibrated "
                                "on a 512 MiB copy)", "ops_per_pair": OPS_PER_PAIR,
                "lane_evaluations": lane_evals, "launch_ms": res["render_ms"],
                "culled_wave_fraction": float(1.0 - st[1] / max(st[0], 1))}

    extra = {}
    if args.extra:
        for v in ["plain", "hoist", "hoist_cull", "local", "hoist_cull_q8", "local_q8", "plain_fp32",
                  "hoist_fp32", "hoist_cull_fp32", "local_fp32"]:
            vb.configure(variant=v, persistent=False, lpt=False)
            extra[v] = timed_forward(vb, params, max(5, args.steps // 2), 2, torch, np)["render_ms"]
        vb.configure(variant=local_settings[0], persistent=local_settings[1], blocks_per_cu=local_settings[2],
                     lpt=local_settings[3])

    fwdbwd = None if args.no_fwdbwd else fwdbwd_single(args, torch, np)
    mv = None if args.no_multiview else multiview(args, torch, np)

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        t0 = time.perf_counter()
        ref = O.render_scene(sc)
        dt = time.perf_counter() - t0
        cpu = {"value": px / dt / 1e6, "unit": "Mpix/s", "cores": 1, "kind": "oracle",
               "sample": f"one full {cam.width}x{cam.height} frame of the same workload (project + bin + blend), "
                         f"single-threaded FP64, {dt:.1f} s"}
        del ref

    out = {
        "metric": "Mpix/s fwd and fwd+bwd vs plain per-pixel raster on same MI355X at 2e-4 tol",
        "value": mpix, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if (local_settings[0] & 0x10) else "f32 (exponent of alpha in f64)", "data": "synthetic",
        "config": {"workload": f"{scenes.CONFIG_NAMES[args.config]} forward", "gaussians": sc.n,
                   "sh_degree": sc.sh_degree, "width": cam.width, "height": cam.height,
                   "render": tuned["best"] if tuned else f"{args.render or 'local'}, one workgroup per tile",
                   "pairs": res["num_pairs"]},
        "plain_value": mpix_base, "local_over_plain": mpix / mpix_base,
        "eager_ms_per_step": {"local": res["wall_ms"], "plain": base["wall_ms"]},
        "stages_ms": {k: res[k] for k in ("project_ms", "sort_ms", "order_ms", "render_ms")},
        "plain_stages_ms": {k: base[k] for k in ("project_ms", "sort_ms", "order_ms", "render_ms")},
        "render_only_speedup": base["render_ms"] / res["render_ms"],
        "parity": parity, "roofline": roofline, "cpu_baseline": cpu,
    }
    if extra:
        out["render_ms_by_variant"] = extra
    if fwdbwd:
        out["fwd_bwd"] = fwdbwd
    if mv:
        out["multiview"] = mv
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
