"""Benchmark: forward rendering throughput (Mpix/s) of the Local-GS pipeline on
one MI355X, against the plain per-pixel renderer on the same GPU.

Workload (default): 1M Gaussians, SH degree 3, one 1920x1080 view
(uniform cloud 4 units in front of the camera; see paper_2606_16566_amd/scenes.py).
A step is one whole forward pass: projection, binning (depth sort, duplication,
tile sort), tile ranges and blending, with inputs resident in HBM.

Prints one JSON line.  `roofline` covers the dominant kernel (blending), whose
average launch duration is measured with HIP events on its own stream;
`cpu_baseline` times the FP64 oracle on this host for one full frame.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# full-rate VALU lane operations: 256 CUs x 4 SIMD16 x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic lane operations per evaluated (pixel, Gaussian) pair of the
# uniform blend: 5 FMA dot product, exp, clamp, select, w = alpha*T, 3 FMA
# colour, T update, termination compare
OPS_PER_PAIR = 14


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--variant", default="local")
    ap.add_argument("--baseline", default="plain")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--extra", action="store_true", help="also time every render variant")
    ap.add_argument("--no-fwdbwd", action="store_true", help="skip the forward+backward workload")
    return ap.parse_args()


def time_fwdbwd(args, R, scenes, torch, np):
    """Forward + L1 loss + backward through the autograd Function on the
    3M-Gaussian 1920x1080 workload (SH degree 0), Local vs Plain."""
    dev = torch.device("cuda:0")
    sc = scenes.make_config(4)
    cam = sc.cameras[0]
    params = [torch.from_numpy(a).to(dev).requires_grad_() for a in
              (sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh)]
    target = torch.from_numpy(scenes.make_target(cam.height, cam.width, 104)).to(dev)
    binner = R.Binner(capacity=0)
    R.rasterize(cam, *[p.detach() for p in params], variant="local", binner=binner, check_overflow=True)
    torch.cuda.synchronize()
    res = {}
    for variant in ("local", "plain"):
        def step():
            for p in params:
                p.grad = None
            img, T, nc = R.LocalGSFunction.apply(*params, cam, variant, binner)
            loss, g = R.l1_loss(img.detach(), target)
            img.backward(g)
            return loss
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        steps = max(3, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[variant] = {"ms_per_step": ms, "mpix_s": cam.width * cam.height / (ms * 1e-3) / 1e6}
    res["local_over_plain"] = res["local"]["mpix_s"] / res["plain"]["mpix_s"]
    res["workload"] = f"{scenes.CONFIG_NAMES[4]}: forward + L1 loss + backward to raw parameters"
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2606_16566_amd import rasterizer as R
    from paper_2606_16566_amd import scenes

    dev = torch.device("cuda:0")
    sc = scenes.make_config(args.config)
    cam = sc.cameras[0]
    params = [torch.from_numpy(a).to(dev) for a in (sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh)]
    binner = R.Binner(capacity=0)
    # size the pair buffers once (host readback happens only here)
    R.rasterize(cam, *params, variant=args.variant, binner=binner, check_overflow=True)
    torch.cuda.synchronize()

    def timed(variant, steps, warmup):
        stream = torch.cuda.current_stream()
        ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(steps)] for k in "abcde"}
        for _ in range(warmup):
            R.rasterize(cam, *params, variant=variant, binner=binner, check_overflow=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ev["a"][i].record(stream)
            proj = R.project(cam, *params)
            ev["b"][i].record(stream)
            b = binner.run(cam, proj, check_overflow=False)
            ev["c"][i].record(stream)
            R.render(variant, cam, b, proj)
            ev["d"][i].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if int(b.overflow.item()):
            raise RuntimeError("pair capacity overflow inside the timed region")
        ms = lambda x, y: float(np.mean([ev[x][i].elapsed_time(ev[y][i]) for i in range(steps)]))
        return dict(wall_ms=wall * 1e3 / steps, project_ms=ms("a", "b"), bin_ms=ms("b", "c"), render_ms=ms("c", "d"),
                    num_pairs=int(b.num_pairs.item()))

    res = timed(args.variant, args.steps, args.warmup)
    base = timed(args.baseline, args.steps, args.warmup)
    px = cam.width * cam.height
    mpix = px / (res["wall_ms"] * 1e-3) / 1e6
    mpix_base = px / (base["wall_ms"] * 1e-3) / 1e6

    # counters of the dominant kernel (separate, untimed instantiation)
    proj = R.project(cam, *params)
    b = binner.run(cam, proj, check_overflow=False)
    st = torch.zeros(8, dtype=torch.int64, device=dev)
    R.render(args.variant, cam, b, proj, stats=st)
    st = st.cpu().numpy()
    lane_evals = int(st[3])
    achieved = lane_evals * OPS_PER_PAIR / (res["render_ms"] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "render_kernel<LOCAL,double>", "achieved": achieved,
                "peak": PEAK_VALU_TOPS, "unit": "Tops/s (full-rate VALU lane ops)", "frac": achieved / PEAK_VALU_TOPS,
                "traffic": None, "ops_per_pair": OPS_PER_PAIR, "lane_evaluations": lane_evals,
                "culled_wave_fraction": float(1.0 - st[1] / max(st[0], 1))}

    extra = {}
    if args.extra:
        for v in ["plain", "hoist", "hoist_cull", "local", "plain_fp32", "hoist_fp32", "hoist_cull_fp32",
                  "local_fp32"]:
            extra[v] = timed(v, max(5, args.steps // 2), 2)["render_ms"]

    fwdbwd = None
    if not args.no_fwdbwd:
        fwdbwd = time_fwdbwd(args, R, scenes, torch, np)

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
        "ms_per_step": res["wall_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 storage, f64 exponent and transmittance", "data": "synthetic",
        "config": {"workload": f"{scenes.CONFIG_NAMES[args.config]} forward", "gaussians": sc.n,
                   "sh_degree": sc.sh_degree, "width": cam.width, "height": cam.height, "variant": args.variant,
                   "pairs": res["num_pairs"]},
        "plain_value": mpix_base, "local_over_plain": mpix / mpix_base,
        "stages_ms": {k: res[k] for k in ("project_ms", "bin_ms", "render_ms")},
        "plain_stages_ms": {k: base[k] for k in ("project_ms", "bin_ms", "render_ms")},
        "render_only_speedup": base["render_ms"] / res["render_ms"],
        "roofline": roofline, "cpu_baseline": cpu,
    }
    if extra:
        out["render_ms_by_variant"] = extra
    if fwdbwd:
        out["fwd_bwd"] = fwdbwd
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
