"""Autotuner of the render launch settings.

Search space of the culling families ('local', 'hoist_cull'; every point
computes the same blend; only the schedule, the wavefront sub-tile and the
exponent precision change):

  shape          16x4 row strips or 8x8 quadrants per wavefront
  vote           termination vote after every Gaussian, or once per four
  precision      exponent in double, or single precision throughout
  schedule       one workgroup per tile (XCD-banded index order or longest
                 first), or a persistent queue of blocks_per_cu workgroups per
                 compute unit (2, 4, 8) handing out sub-tiles in index or
                 longest-first tile order

The plain per-pixel renderer (family 'plain', the comparison baseline) is
tuned over what it has: exponent precision (double, or the 3DGS float
expression) and tile order (XCD-banded or longest first); its workgroups
share LDS batches, so it has no sub-tile shape, vote or queue.

`tune_backward` chooses the backward's schedule the same way: one workgroup
per tile or persistent (2, 4, 8 workgroups per CU), index or longest-first
order (the gradients agree up to float summation order).

Objective: median duration of the render launch over `reps` timed runs
(HIP events on the launching stream).  A point is admissible only if its
image agrees with the reference point (one workgroup per tile, 16x4, double
exponent) within `tol` at all but `max_bad_frac` of the pixels.  The default
bound is the one the Local-GS renderer must keep against the plain per-pixel
renderer (1e-6 everywhere), which the reference point meets; every
double-exponent point reproduces it bitwise, while single precision moves
colours by up to ~1e-4 and is admitted only under a looser bound (2e-4, the
oracle tolerance).  Results are cached in a JSON file keyed by device,
workload and bound.
"""
from __future__ import annotations

import itertools
import json
import os
import time

import numpy as np
import torch

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "localgs", "autotune.json")

REFERENCE = dict(shape="16x4", vote=1, precision="fp64", persistent=False, blocks_per_cu=0, lpt=False)
KEYS = ("family", "shape", "vote", "precision", "persistent", "blocks_per_cu", "lpt")


def space(family: str = "local"):
    """All candidate settings of one variant family ('local', 'hoist_cull'
    or 'plain')."""
    if family == "plain":
        return [dict(family="plain", shape="16x4", vote=1, precision=prec, persistent=False, blocks_per_cu=0, lpt=lpt)
                for prec in ("fp64", "fp32") for lpt in (False, True)]
    votes = (1, 4) if family == "local" else (1,)
    pts = []
    for shape, vote, prec in itertools.product(("16x4", "8x8"), votes, ("fp64", "fp32")):
        base = dict(family=family, shape=shape, vote=vote, precision=prec)
        pts.append(dict(base, persistent=False, blocks_per_cu=0, lpt=False))
        pts.append(dict(base, persistent=False, blocks_per_cu=0, lpt=True))
        for bpc, lpt in itertools.product((2, 4, 8), (False, True)):
            pts.append(dict(base, persistent=True, blocks_per_cu=bpc, lpt=lpt))
    return pts


def variant_name(cfg) -> str:
    name = cfg.get("family", "local")
    if cfg.get("shape") == "8x8":
        name += "_q8"
    if cfg.get("vote", 1) == 4:
        name += "_v4"
    if cfg.get("precision") == "fp32":
        name += "_fp32"
    return name


def apply(vb, cfg):
    """Set a ViewBatch's launch settings from a tuned point."""
    vb.configure(variant=variant_name(cfg), persistent=cfg["persistent"], blocks_per_cu=cfg["blocks_per_cu"],
                 lpt=cfg["lpt"])


def workload_key(vb, num_pairs: int, family: str) -> str:
    # the ISA and compute-unit count identify the device (the marketing name
    # can come back empty where the driver's name table is not installed)
    props = torch.cuda.get_device_properties(vb.dev)
    dev = f"{props.gcnArchName.split(':')[0]}/{props.multi_processor_count}cu"
    sizes = ",".join(f"{c.width}x{c.height}" for c in vb.cams)
    pairs = float(f"{num_pairs:.2g}")
    return f"{dev}|{family}|n={vb.n}|deg={vb.deg}|views={sizes}|pairs~{pairs:.0f}"


def load_cache(path: str | None = None) -> dict:
    path = path or DEFAULT_CACHE
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str | None = None):
    path = path or DEFAULT_CACHE
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_render(vb, reps: int, warmup: int):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        vb.render()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        vb.render()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def tune(vb, params, family: str = "local", reps: int = 9, warmup: int = 2, tol: float = 1e-6,
         max_bad_frac: float = 0.0, cache_path: str | None = None, use_cache: bool = True, points=None) -> dict:
    """Tune the render settings of `vb` for `params` (binned once, then only
    the render is re-launched).  Leaves `vb` configured with the best point
    and returns {"key", "best", "results", "cached"}."""
    vb.fit(params)
    vb.bin(params)
    torch.cuda.synchronize()
    num_pairs = int(vb.num_pairs.item())
    key = workload_key(vb, num_pairs, family) + f"|tol={tol:g}/{max_bad_frac:g}"
    cache = load_cache(cache_path) if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["best"]
        apply(vb, best)
        return {"key": key, "best": best, "results": cache[key].get("results", []), "cached": True}

    apply(vb, dict(REFERENCE, family=family))
    vb.render()
    torch.cuda.synchronize()
    ref = vb.out_rgb.clone()
    results = []
    t0 = time.perf_counter()
    for cfg in (points or space(family)):
        apply(vb, cfg)
        times = _time_render(vb, reps, warmup)
        diff = (vb.out_rgb - ref).abs().view(3, -1).amax(0)
        bad = float((diff > tol).float().mean())
        ok = bad <= max_bad_frac
        results.append(dict(cfg, median_ms=float(np.median(times)), min_ms=float(np.min(times)),
                            max_diff=float(diff.max()), bad_frac=bad, admissible=ok))
    adm = [r for r in results if r["admissible"]]
    best = min(adm, key=lambda r: r["median_ms"])
    best_cfg = {k: best[k] for k in KEYS}
    apply(vb, best_cfg)
    if use_cache:
        cache = load_cache(cache_path)
        cache[key] = {"best": best_cfg, "median_ms": best["median_ms"], "results": results,
                      "tuned_s": time.perf_counter() - t0}
        save_cache(cache, cache_path)
    return {"key": key, "best": best_cfg, "results": results, "cached": False}


BWD_KEYS = ("bwd_persistent", "bwd_blocks_per_cu", "bwd_lpt")


def backward_space():
    pts = [dict(bwd_persistent=False, bwd_blocks_per_cu=0, bwd_lpt=lpt) for lpt in (False, True)]
    pts += [dict(bwd_persistent=True, bwd_blocks_per_cu=b, bwd_lpt=lpt) for b in (2, 4, 8) for lpt in (False, True)]
    return pts


def tune_backward(vb, params, grad_rgb=None, reps: int = 5, warmup: int = 1, cache_path: str | None = None,
                  use_cache: bool = True) -> dict:
    """Tune the backward render's schedule on `vb` (forward settings as
    configured; the forward is run once, then only the backward render is
    re-launched with `grad_rgb`, default the batch's own buffer).  Leaves `vb`
    configured with the fastest point."""
    vb.forward(params)
    torch.cuda.synchronize()
    num_pairs = int(vb.num_pairs.item())
    key = workload_key(vb, num_pairs, "backward") + f"|variant={vb.variant}"
    cache = load_cache(cache_path) if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["best"]
        vb.configure(**best)
        return {"key": key, "best": best, "results": cache[key].get("results", []), "cached": True}
    stream = torch.cuda.current_stream()
    results = []
    for cfg in backward_space():
        vb.configure(**cfg)
        for _ in range(warmup):
            vb.backward_render(grad_rgb)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            vb.backward_render(grad_rgb)
            b.record(stream)
        torch.cuda.synchronize()
        t = [a.elapsed_time(b) for a, b in ev]
        results.append(dict(cfg, median_ms=float(np.median(t)), min_ms=float(np.min(t))))
    best = min(results, key=lambda r: r["median_ms"])
    best_cfg = {k: best[k] for k in BWD_KEYS}
    vb.configure(**best_cfg)
    if use_cache:
        cache = load_cache(cache_path)
        cache[key] = {"best": best_cfg, "median_ms": best["median_ms"], "results": results}
        save_cache(cache, cache_path)
    return {"key": key, "best": best_cfg, "results": results, "cached": False}
