"""Benchmark: rendering throughput (Mpix/s) of the Local-GS pipeline on one
MI355X, against the plain per-pixel renderer on the same GPU, forward and
forward + backward, at the 2e-4 oracle tolerance.

Headline (`value`): the largest single-GPU workload, 10M clustered Gaussians
(SH degree 3) seen by 16 cameras of mixed resolution (640x480 to 1920x1080),
one training step = projection, binning, tile ranges, tile order, blend, L1
loss, backward blend and backward projection for all 16 views, replayed from
one captured HIP graph with the inputs resident in HBM.  Render and backward
schedules come from the autotuner.  `plain_value` is the same step with the
plain per-pixel renderer (tuned over its own settings).

Every other workload is reported beside it (`configs`): 10k Gaussians at
256x256, 1M SH-3 at 1920x1080 and 6M clustered SH-3 at 1264x832 (forward),
3M SH-0 at 1920x1080 (forward + backward) and the 16-view batch forward; the
render ablation ladder (PLAIN -> HOIST -> HOIST_CULL -> LOCAL, double and
single precision, with the oracle error of each step), the precision
experiment at 3840x2160 (tile-local against global coordinates), and the
1x / 2x resolution sweep.  Parity records compare GPU outputs with the FP64
oracle on sampled pixels (the oracle runs on host threads while the GPU
works); `cpu_baseline` times the oracle on a stated sample of the headline
workload.

Prints one JSON line.  `roofline` covers the dominant kernel of the headline
step (its average launch duration measured with HIP events on the stream it
is launched on); `rooflines` gives every stage against its bound.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# full-rate VALU lane operations: 256 CUs x 4 SIMD16 x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
# algorithmic lane operations per evaluated (pixel, Gaussian) pair of the
# uniform blend: 5 FMA dot product, exp, clamp, select, w = alpha*T, 3 FMA
# colour, T update, termination compare
OPS_PER_PAIR = 14
# per replayed (pixel, Gaussian) step of the backward blend: 5 FMA exponent,
# exp, floor select and clamp (2), 1/(1 - alpha) (2), T recovery and
# w = alpha T (2), dL/dalpha = T (gC . c) - G / (1 - alpha) (5), the update
# of the scalar G = gC . R + gT T_f (1), 17 for the nine partials (dx, dy,
# alpha dL/dalpha and its products with dx and dy, the chain to the mean, the
# conic and the opacity, the colour gradient) and 9 additions of the
# partials into the per-Gaussian sums
OPS_PER_BWD_STEP = 44

SAMPLE_PIXELS = 3000
GUARD_STORED = 1e-5      # decision guard against the float32-stored projection
GUARD_FP64 = 1e-4        # against the unrounded FP64 projection
TOL = 2e-4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--only", default=None,
                    help="comma-separated subset of c1,c2,c3,c4,c5,sweep (profiling); skips the CPU work")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (CPU baseline and parity samples)")
    ap.add_argument("--no-tune", action="store_true", help="default settings instead of the autotuner")
    ap.add_argument("--tune-cache", default=None, help="autotuner JSON cache (default ~/.cache/localgs)")
    ap.add_argument("--retune", action="store_true", help="ignore cached autotuner results")
    ap.add_argument("--local-only", action="store_true",
                    help="time only the Local-GS renderer (profiling runs; no Plain comparison)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first copy this many MiB device-to-device (calibrates HBM byte counters)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# small helpers
# ---------------------------------------------------------------------------
T0 = time.perf_counter()


def log(msg):
    """Progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.perf_counter() - T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def pct(xs):
    import numpy as np
    xs = np.asarray(xs, float)
    return {"median_ms": float(np.median(xs)), "p10_ms": float(np.percentile(xs, 10)),
            "p90_ms": float(np.percentile(xs, 90)), "n": int(len(xs))}


def mpix(px, ms):
    return px / (ms * 1e-3) / 1e6


def tensors(sc, torch):
    dev = torch.device("cuda:0")
    return [torch.from_numpy(a).to(dev) for a in (sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh)]


def gpu_clock_mhz(torch):
    """Current shader clock (MHz) from the amdgpu driver's sysfs table of
    shader clock levels (the active level is starred), or None.  Read from a
    file so that no child process is started after the GPU is initialised."""
    paths = []
    try:
        p = torch.cuda.get_device_properties(0)
        paths.append(f"/sys/bus/pci/devices/{p.pci_domain_id:04x}:{p.pci_bus_id:02x}:{p.pci_device_id:02x}.0"
                     "/pp_dpm_sclk")
    except (AttributeError, RuntimeError):
        pass
    for path in paths:
        try:
            with open(path) as f:
                for line in f:
                    if line.rstrip().endswith("*"):
                        return float(line.split(":", 1)[1].lower().split("mhz")[0])
        except (OSError, ValueError, IndexError):
            pass
    return None


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def timed_graph(step, steps, warmup, torch):
    """Replays of a captured step: wall ms per replay over exactly `steps`
    replays (synchronised on both sides) and per-replay HIP-event times."""
    from paper_2606_16566_amd.batch import StepGraph
    g = StepGraph(step, warmup=1)
    try:
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            g.replay()
            b.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        out = pct([a.elapsed_time(b) for a, b in ev])
        out["wall_ms"] = wall
        return out
    finally:
        g.close()


def stage_times(vb, params, target, steps, warmup, torch, bwd):
    """Per-stage HIP-event times of eager steps on the launching stream
    (lists of ms): project, sort (binning + ranges), order, render[, l1,
    bwd_render (adding into the gradient records that the previous
    bwd_project cleared), bwd_project (clearing them)]."""
    names = ["project", "sort", "order", "render"] + (["l1", "bwd_render", "bwd_project"] if bwd else [])
    calls = [lambda: vb.project(params), vb.sort, vb.tile_order, vb.blend]
    if bwd:
        calls += [lambda: vb.l1(target), lambda: vb.backward_render(accumulate=vb.g_clear),
                  lambda: vb.backward_project(params, clear=True)]
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        for c in calls:
            c()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)] for _ in range(steps)]
    for e in ev:
        e[0].record(stream)
        for i, c in enumerate(calls):
            c()
            e[i + 1].record(stream)
    torch.cuda.synchronize()
    if vb.overflowed():
        raise RuntimeError("pair capacity overflow inside the timed region")
    import numpy as np
    return {n: float(np.median([e[i].elapsed_time(e[i + 1]) for e in ev])) for i, n in enumerate(names)}


def kernel_times(fn, reps, torch):
    """HIP-event times of `fn` (one library call) on the current stream."""
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return pct([a.elapsed_time(b) for a, b in ev])


def hbm_roof(name, bytes_, ms, what):
    gbs = bytes_ / (ms * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "algorithmic_bytes": float(bytes_), "ms": ms, "per_unit": what}


def valu_roof(name, lane_units, ops, ms, what):
    t = lane_units * ops / (ms * 1e-3) / 1e12
    return {"kernel": name, "bound": "alu", "achieved": t, "peak": PEAK_VALU_TOPS,
            "unit": "T lane-ops/s (full-rate VALU)", "frac": t / PEAK_VALU_TOPS, "lane_units": int(lane_units),
            "ops_per_unit": ops, "ms": ms, "per_unit": what}


# HBM bytes per launch of the headline step's dominant kernel, from two
# rocprofv3 --pmc runs of `bench.py --only c5 --local-only` (FETCH_SIZE, then
# WRITE_SIZE, each scaled by what it reads for a 512 MiB device-to-device copy:
# x2.0 and x1.0); valid only while the kernel's sources hash to the values the
# counters were taken on, else the roofline's traffic is null
MEASURED_TRAFFIC = {
    "render_bwd_kernel": {
        "sources": ["include/localgs.h", "paper_2606_16566_amd/csrc/common.hpp",
                    "paper_2606_16566_amd/csrc/render_common.hpp", "paper_2606_16566_amd/csrc/render_bwd.hip"],
        "sha256": "b683aeb8579518f09669b54f483e9d2bde7975ec89ea180dc780ebcf30a7942a",
        "read_bytes": 15249092930,
        "write_bytes": 3732327653,
        "profile": "profiles/train_clustered-10M-16views_hbm_counters.md",
    },
}


def sources_sha256(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """Counter-measured HBM bytes per launch of `kernel`, or None when no
    counters were taken on its current sources."""
    e = MEASURED_TRAFFIC.get(kernel)
    if e is None or e["sha256"] is None or sources_sha256(e["sources"]) != e["sha256"]:
        return None
    return float(e["read_bytes"] + e["write_bytes"])


def proj_bytes(n, K, V):
    """Algorithmic HBM bytes of the view-batched projection: raw parameters
    read once (44 B + 12 K B), 56 B of projected attributes written per
    (view, Gaussian)."""
    return n * (44 + 12 * K) + n * V * 56


def proj_bwd_bytes(n, K, V):
    """Backward projection: raw parameters read and their gradients written
    once (2 (44 + 12 K) B), rectangle and projected gradients read per view
    (16 + 36 B)."""
    return 2 * n * (44 + 12 * K) + n * V * 52


def binning_bytes(E, P, tiles):
    """Ideal one-pass binning: read each element's depth key and rectangle
    (20 B), write every pair (tile key + id, 8 B), read the tile keys once
    for the ranges (4 B per pair) and write the ranges (8 B per tile).  The
    two-stage radix sort moves several times this; the fraction against it
    says how far the binning is from any sort's floor."""
    return E * 20 + P * 12 + tiles * 8


# ---------------------------------------------------------------------------
# oracle work on host threads (ctypes releases the GIL in the C calls)
# ---------------------------------------------------------------------------
class OracleSamples:
    """FP64 oracle results on sampled pixels of the benchmark's workloads,
    computed on a host thread pool while the GPU runs.  Projections are split
    into chunks of Gaussians; each workload then builds its tile lists and
    blends the sampled pixels of the float32-stored projection and of the
    unrounded one."""

    def __init__(self, workers):
        self.pool = ThreadPoolExecutor(max_workers=workers)
        self.workers = workers
        self.jobs = {}

    def _project(self, sc, cam):
        import numpy as np
        from oracle import oracle as O
        n = sc.n
        chunk = max(1, -(-n // (2 * self.workers)))
        futs = [self.pool.submit(O.project, cam, sc.means3d[a:a + chunk], sc.log_scales[a:a + chunk],
                                 sc.quats[a:a + chunk], sc.opacity_logits[a:a + chunk], sc.sh[a:a + chunk])
                for a in range(0, n, chunk)]
        parts = [f.result() for f in futs]
        return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}

    def submit(self, key, sc, cam, full=False, seed=0):
        def job():
            import numpy as np
            from oracle import oracle as O
            pr = self._project(sc, cam)
            off, ids = O.tile_lists(pr["visible"], pr["depth"], pr["rect"], cam.width, cam.height)
            if full:
                pix = None
            else:
                rng = np.random.default_rng(seed)
                pix = np.stack([rng.integers(0, cam.width, SAMPLE_PIXELS), rng.integers(0, cam.height, SAMPLE_PIXELS)],
                               1)
                edges = np.array([[0, 0], [cam.width - 1, cam.height - 1], [15, 16], [16, 15], [cam.width - 1, 0]])
                pix = np.concatenate([pix, edges]).astype(np.int32)
            st = O.stored_projection(pr)
            ref = O.render_tiled(cam.width, cam.height, off, ids, st["means2d"], st["conic"], st["opacity"],
                                 st["rgb"], cam.bg, pixels=pix)
            ref64 = O.render_tiled(cam.width, cam.height, off, ids, pr["means2d"], pr["conic"], pr["opacity"],
                                   pr["rgb"], cam.bg, pixels=pix)
            return {"pix": pix, "stored": ref, "fp64": ref64, "pairs": int(len(ids)),
                    "lists": (cam.width, cam.height, off, ids), "splats": {"stored": st, "fp64": pr}, "bg": cam.bg}
        # the job itself waits on chunk futures: run it on its own thread
        ex = ThreadPoolExecutor(max_workers=1)
        self.jobs[key] = ex.submit(job)
        ex.shutdown(wait=False)

    def get(self, key):
        f = self.jobs.get(key)
        return None if f is None else f.result()


def gpu_outputs(vb, v=0):
    """(image [3,H,W], T, last contributor id) of view v, as numpy."""
    import numpy as np
    import torch
    cam = vb.cams[v]
    img = vb.image(v).cpu().numpy()
    T = vb.final_T(v).cpu().numpy()
    nc = vb.n_contrib(v).to(torch.int64)
    H, W = cam.height, cam.width
    ty = torch.arange(H, device=nc.device)[:, None] // 16
    tx = torch.arange(W, device=nc.device)[None, :] // 16
    tile = vb.tile_off[v] + ty * cam.tiles_x + tx
    start = vb.ranges.view(-1, 2)[tile, 0].to(torch.int64) & 0xFFFFFFFF
    pos = torch.clamp(start + nc - 1, min=0)
    vals = vb.vals.to(torch.int64) & 0xFFFFFFFF
    lid = torch.where(nc > 0, vals[pos] - v * vb.n, torch.full_like(nc, -1)).cpu().numpy()
    return img, T, lid


def parity_vs(sample, outs):
    """Max-abs colour / T error and last-contributor agreement on the sampled
    pixels outside the decision guard, for the stored and FP64 projections."""
    import numpy as np
    img, T, lid = outs
    pix = sample["pix"]
    if pix is not None:
        img, T, lid = img[:, pix[:, 1], pix[:, 0]], T[pix[:, 1], pix[:, 0]], lid[pix[:, 1], pix[:, 0]]
    from oracle import oracle as O
    res = {}
    W, H, off, ids = sample["lists"]
    for name, guard in (("stored", GUARD_STORED), ("fp64", GUARD_FP64)):
        ref = sample[name]
        flag = np.asarray(ref["margin"]) < guard
        ok = ~flag
        e_img = float(np.abs(img - ref["image"])[:, ok].max()) if ok.any() else 0.0
        e_T = float(np.abs(T - ref["T"])[ok].max()) if ok.any() else 0.0
        # a flagged pixel (a decision within the guard) must match one of the
        # oracle's alternative blends, each such decision taken either way
        matched = 0
        for i in zip(*np.nonzero(flag)):
            if pix is not None:
                x, y, col, t, l = int(pix[i[0], 0]), int(pix[i[0], 1]), img[:, i[0]], T[i[0]], lid[i[0]]
            else:
                y, x = int(i[0]), int(i[1])
                col, t, l = img[:, y, x], T[y, x], lid[y, x]
            matched += O.matches_an_alternative(W, H, off, ids, sample["splats"][name], sample["bg"], x, y, guard,
                                                col, t, l, TOL)
        res[name] = {"max_abs": max(e_img, e_T), "max_abs_colour": e_img, "max_abs_T": e_T,
                     "flagged": int(flag.sum()), "flagged_matching_an_alternative": int(matched),
                     "pixels": int(flag.size), "guard": guard,
                     "last_id_mismatch": int((lid[ok] != ref["last_id"][ok]).sum()),
                     "pass": bool(max(e_img, e_T) <= TOL and (lid[ok] == ref["last_id"][ok]).all()
                                  and matched == int(flag.sum()))}
    return res


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def tune_all(vb, params, args, family="local", **kw):
    from paper_2606_16566_amd import autotune
    if args.no_tune:
        cfg = dict(autotune.REFERENCE, family=family)
        autotune.apply(vb, cfg)
        return cfg
    return autotune.tune(vb, params, family=family, cache_path=args.tune_cache, use_cache=not args.retune,
                         **kw)["best"]


def exact_tiles_ab(vb, params, local, torch, steps, args, bwd, target=None, bwd_cfg=None):
    """The Local pipeline with the exact tile assignment (row f2) against
    whole rectangles: pair count, binning and blend time, whole step."""
    from paper_2606_16566_amd import autotune
    res = {}
    for exact in (False, True):
        autotune.apply(vb, local)
        if bwd_cfg:
            vb.configure(**bwd_cfg)
        vb.configure(exact_tiles=exact)
        vb.fit(params)
        if bwd:
            vb.l1(target)
            g = timed_graph(lambda: vb.train_step(params, target), steps, args.warmup, torch)
        else:
            g = timed_graph(lambda: vb.forward(params), steps, args.warmup, torch)
        st = stage_times(vb, params, target, max(5, steps // 2), 1, torch, bwd=bwd)
        res["exact" if exact else "rectangles"] = {"pairs": int(vb.num_pairs.item()), "graph": g, "stages_ms": st}
    vb.configure(exact_tiles=False)
    vb.fit(params)
    r, e = res["rectangles"], res["exact"]
    res["pair_ratio"] = e["pairs"] / max(r["pairs"], 1)
    res["step_speedup"] = r["graph"]["median_ms"] / e["graph"]["median_ms"]
    return res


def forward_workload(label, sc, cam, args, torch, oracle=None, ladder=False, steps=None, exact_ab=False):
    """Forward pipeline of one view, tuned Local against tuned Plain (best
    Plain within 2e-4 of the double-precision plain renderer, and the best
    plain point within 1e-6 of it), graph replays, stage times, the blend's
    VALU roofline and, if given, oracle parity on sampled pixels."""
    import numpy as np
    from paper_2606_16566_amd import autotune
    from paper_2606_16566_amd.batch import ViewBatch
    steps = steps or max(10, args.steps)
    log(f"{label}: forward workload")
    params = tensors(sc, torch)
    vb = ViewBatch([cam], sc.n, sc.sh_degree, record_used=False)     # forward only: no backward follows
    px = cam.width * cam.height
    local = tune_all(vb, params, args, "local")
    plain2 = tune_all(vb, params, args, "plain", tol=2e-4)
    plain6 = tune_all(vb, params, args, "plain", tol=1e-6)
    vb.fit(params)
    out = {"workload": f"{label}: {sc.n} Gaussians, SH {sc.sh_degree}, {cam.width}x{cam.height}, forward",
           "pixels": px, "tuned": {"local": local, "plain": plain2, "plain_1e-6": plain6}}
    outs = {}
    for name, cfg in (("local", local), ("plain", plain2), ("plain_1e-6", plain6)):
        log(f"{label}: {name} {cfg}")
        autotune.apply(vb, cfg)
        g = timed_graph(lambda: vb.forward(params), steps, args.warmup, torch)
        st = stage_times(vb, params, None, steps, 2, torch, bwd=False)
        vb.forward(params)
        torch.cuda.synchronize()
        outs[name] = gpu_outputs(vb)
        out[name] = {"graph": g, "mpix_s": mpix(px, g["median_ms"]), "stages_ms": st}
        if name == "local":
            s = torch.zeros(8, dtype=torch.int64, device="cuda:0")
            vb.tile_order()
            vb.blend(stats=s)
            s = s.cpu().numpy()
            kt = kernel_times(vb.blend, steps, torch)
            out["pairs"] = int(vb.num_pairs.item())
            out["render_roofline"] = valu_roof("render_wave_kernel", s[3], OPS_PER_PAIR, kt["median_ms"],
                                               "evaluated (lane, Gaussian) step of the blend")
            out["render_roofline"]["culled_wave_fraction"] = float(1.0 - s[1] / max(s[0], 1))
    if exact_ab:
        out["exact_tiles"] = exact_tiles_ab(vb, params, local, torch, steps, args, bwd=False)
    out["local_over_plain"] = out["plain"]["graph"]["median_ms"] / out["local"]["graph"]["median_ms"]
    out["local_over_plain_1e-6"] = out["plain_1e-6"]["graph"]["median_ms"] / out["local"]["graph"]["median_ms"]
    out["render_only_speedup"] = out["plain"]["stages_ms"]["render"] / out["local"]["stages_ms"]["render"]
    d = np.abs(outs["local"][0] - outs["plain_1e-6"][0]).max()
    out["local_vs_plain_max_abs"] = float(d)
    # the oracle's samples (computed on host threads meanwhile) are waited for
    # only now, after the timed work
    sample = oracle() if oracle is not None else None
    if sample is not None:
        out["parity"] = {k: parity_vs(sample, v) for k, v in outs.items()}
    if ladder:
        out["ablation"] = ablation(vb, params, local, torch, sample, steps)
    del vb, params
    torch.cuda.empty_cache()
    return out


def ablation(vb, params, local, torch, oracle, steps):
    """Render-kernel time of each step of the paper's cumulative ladder
    (PLAIN -> HOIST -> HOIST_CULL -> LOCAL) in double-exponent and single
    precision (and the global-coordinate single-precision hoist), with each
    step's oracle error on the sampled pixels."""
    from paper_2606_16566_amd import autotune
    shape = "_q8" if local.get("shape") == "8x8" else ""
    ladder = ["plain", "hoist", "hoist_cull" + shape, "local" + shape]
    names = ladder + [v + "_fp32" for v in ladder] + ["local" + shape + "_global_fp32"]
    res = {}
    for v in names:
        vb.configure(variant=v, persistent=False, lpt=False)
        vb.forward(params)
        kt = kernel_times(vb.blend, max(5, steps // 2), torch)
        ent = {"render_ms": kt["median_ms"], "p10_ms": kt["p10_ms"], "p90_ms": kt["p90_ms"]}
        if oracle is not None:
            p = parity_vs(oracle, gpu_outputs(vb))
            ent["max_abs_vs_oracle"] = p["stored"]["max_abs"]
            ent["max_abs_vs_oracle_fp64"] = p["fp64"]["max_abs"]
        res[v] = ent
    autotune.apply(vb, local)
    return res


def train_workload(label, sc, cams, args, torch, target_seed, steps=None, fwd_too=False, exact_ab=False):
    """Forward + L1 + backward over the views `cams` (one ViewBatch), Local
    and Plain each tuned, replayed as one captured graph per step; stage
    times, backward and forward blend rooflines, HBM fractions per stage."""
    import numpy as np
    from paper_2606_16566_amd import autotune
    from paper_2606_16566_amd.batch import ViewBatch
    steps = steps or args.steps
    log(f"{label}: training-step workload")
    params = tensors(sc, torch)
    vb = ViewBatch(cams, sc.n, sc.sh_degree)
    px = vb.num_pixels
    rng = np.random.default_rng(target_seed)
    target = torch.from_numpy(rng.uniform(0, 1, size=3 * px).astype(np.float32)).cuda()
    local = tune_all(vb, params, args, "local", reps=3 if len(cams) > 1 else 9)
    plain2 = plain6 = None
    if not args.local_only:
        plain2 = tune_all(vb, params, args, "plain", tol=2e-4, reps=3 if len(cams) > 1 else 9)
        plain6 = tune_all(vb, params, args, "plain", tol=1e-6, reps=3 if len(cams) > 1 else 9)
    vb.fit(params)
    res = {"workload": f"{label}: {sc.n} Gaussians, SH {sc.sh_degree}, {len(cams)} view(s), "
                       f"{px} pixels, forward + L1 + backward", "pixels": px, "views": len(cams),
           "tuned": {"local": local, "plain": plain2, "plain_1e-6": plain6}}
    runs = (("local", local),) if args.local_only else (("local", local), ("plain", plain2), ("plain_1e-6", plain6))
    for name, cfg in runs:
        log(f"{label}: {name} {cfg}")
        autotune.apply(vb, cfg)
        vb.l1(target)
        if not args.no_tune:
            bt = autotune.tune_backward(vb, params, reps=3, cache_path=args.tune_cache, use_cache=not args.retune)
            res["tuned"][name + "_backward"] = bt["best"]
        ent = {}
        if fwd_too:
            vb.configure(record_used=False)                       # forward only: no backward follows
            g = timed_graph(lambda: vb.forward(params), steps, args.warmup, torch)
            vb.configure(record_used=True)
            ent["fwd"] = {"graph": g, "mpix_s": mpix(px, g["median_ms"])}
        g = timed_graph(lambda: vb.train_step(params, target), steps, args.warmup, torch)
        ent["fwd_bwd"] = {"graph": g, "mpix_s": mpix(px, g["median_ms"])}
        ent["stages_ms"] = stage_times(vb, params, target, max(5, steps // 2), 1, torch, bwd=True)
        if name == "local":
            res["pairs"] = int(vb.num_pairs.item())
            res["tiles"] = vb.num_tiles
            # blend and backward blend: counters from the statistics
            # instantiations, kernel-only times with HIP events
            vb.forward(params)
            vb.l1(target)
            s = torch.zeros(8, dtype=torch.int64, device="cuda:0")
            vb.blend(stats=s)
            sb = torch.zeros(8, dtype=torch.int64, device="cuda:0")
            vb.backward_render(stats=sb)
            s, sb = s.cpu().numpy(), sb.cpu().numpy()
            t_fwd = kernel_times(vb.blend, max(5, steps // 2), torch)["median_ms"]
            vb.g_splats.zero_()
            t_bwd = kernel_times(lambda: vb.backward_render(accumulate=True), max(5, steps // 2), torch)["median_ms"]
            E, K, V, n = vb.V * vb.n, vb.K, vb.V, vb.n
            st = ent["stages_ms"]
            roofs = {
                "render": valu_roof("render_wave_kernel", s[3], OPS_PER_PAIR, t_fwd,
                                    "evaluated (lane, Gaussian) step of the blend"),
                "bwd_render": valu_roof("render_bwd_kernel", sb[3], OPS_PER_BWD_STEP, t_bwd,
                                        "replayed (lane, Gaussian) step of the backward blend"),
                "project": hbm_roof("project_fwd_kernel", proj_bytes(n, K, V), st["project"],
                                    "raw parameters once, projected attributes per view"),
                "sort": hbm_roof("binning (depth sort, pair generation, tile sort, ranges)",
                                 binning_bytes(E, res["pairs"], vb.num_tiles), st["sort"],
                                 "ideal one-pass binning bytes"),
                "bwd_project": hbm_roof("project_bwd_kernel", proj_bwd_bytes(n, K, V), st["bwd_project"],
                                        "raw parameters and their gradients once, projected gradients per view"),
            }
            roofs["render"]["culled_wave_fraction"] = float(1.0 - s[1] / max(s[0], 1))
            roofs["bwd_render"]["taken_pairs"] = int(sb[2])
            roofs["bwd_render"]["culled_or_skipped_step_fraction"] = float(1.0 - sb[1] / max(sb[0], 1))
            res["rooflines"] = roofs
        res[name] = ent
    if args.local_only:
        del vb, params, target
        torch.cuda.empty_cache()
        return res
    if exact_ab:
        res["exact_tiles"] = exact_tiles_ab(vb, params, local, torch, max(5, steps // 2), args, bwd=True,
                                            target=target, bwd_cfg=res["tuned"].get("local_backward"))
    res["local_over_plain"] = res["plain"]["fwd_bwd"]["graph"]["median_ms"] / res["local"]["fwd_bwd"]["graph"][
        "median_ms"]
    res["local_over_plain_1e-6"] = res["plain_1e-6"]["fwd_bwd"]["graph"]["median_ms"] / \
        res["local"]["fwd_bwd"]["graph"]["median_ms"]
    if fwd_too:
        res["fwd_local_over_plain"] = res["plain"]["fwd"]["graph"]["median_ms"] / res["local"]["fwd"]["graph"][
            "median_ms"]
    if vb.overflowed():
        raise RuntimeError(f"pair capacity overflow in {label}")
    del vb, params, target
    torch.cuda.empty_cache()
    return res


def cpu_baseline_job(sc5):
    """The FP64 oracle, single-threaded, on a bounded sample of the headline
    workload: view 0 (640x480) of the 16 cameras with every 10th Gaussian of
    the 10M scene (1M Gaussians): projection, tile lists, blend, L1 loss,
    backward blend and backward projection."""
    import numpy as np
    from oracle import oracle as O
    from paper_2606_16566_amd import scenes
    sub = sc5.subset(np.arange(0, sc5.n, 10))
    sub.cameras = [sc5.cameras[0]]
    cam = sub.cameras[0]
    target = scenes.make_target(cam.height, cam.width, 105)
    t0 = time.perf_counter()
    ref = O.render_scene(sub)
    g = np.sign(ref["image"] - target) / target.size
    O.scene_gradients(sub, g)
    dt = time.perf_counter() - t0
    px = cam.width * cam.height
    return {"value": px / dt / 1e6, "unit": "Mpix/s", "cores": 1, "kind": "oracle",
            "sample": f"view 0 ({cam.width}x{cam.height}) of the 16-view workload with every 10th Gaussian "
                      f"({sub.n} of {sc5.n}): FP64 projection, binning, blend, L1 and backward "
                      f"(the forward is recomputed inside the gradient call), single-threaded, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2606_16566_amd import scenes

    only = set(args.only.split(",")) if args.only else {"c1", "c2", "c3", "c4", "c5", "sweep"}
    use_cpu = not args.no_cpu and args.only is None
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

    model, avail = host_cpu()
    workers = max(1, min(12, avail - 2))
    orc = OracleSamples(workers) if use_cpu else None
    clock0 = gpu_clock_mhz(torch)

    # scenes (host) and oracle jobs, submitted first so the oracle works while the GPU does
    log("generating scenes")
    sc = {}
    for k in (1, 2, 3, 4, 5):
        if f"c{k}" in only or (k in (2, 3) and "sweep" in only):
            sc[k] = scenes.make_config(k)
    big = {}
    if "sweep" in only:
        for k in (2, 3):
            c = sc[k].cameras[0]
            big[k] = scenes.look_at_camera(tuple(c.campos), (0, 0, 0) if k == 3 else (0, 0, 1),
                                           2 * c.width, 2 * c.height)
    cpu_fut = None
    if orc is not None:
        if 1 in sc:
            orc.submit("c1", sc[1], sc[1].cameras[0], full=True)
        for k in (2, 3):
            if k in sc:
                orc.submit(f"c{k}", sc[k], sc[k].cameras[0])
        for k in (2, 3):
            if k in big:
                orc.submit(f"c{k}x2", sc[k], big[k])
        if 5 in sc:
            ex = ThreadPoolExecutor(max_workers=1)
            cpu_fut = ex.submit(cpu_baseline_job, sc[5])
            ex.shutdown(wait=False)
    # lazy handles: a workload waits for its oracle sample only after its timed work
    get = (lambda key: (lambda: orc.get(key))) if orc is not None else (lambda key: None)

    configs = {}
    if 1 in sc and "c1" in only:
        configs["c1"] = forward_workload(scenes.CONFIG_NAMES[1], sc[1], sc[1].cameras[0], args, torch, get("c1"))
    if 2 in sc and "c2" in only:
        configs["c2"] = forward_workload(scenes.CONFIG_NAMES[2], sc[2], sc[2].cameras[0], args, torch, get("c2"),
                                         ladder=True, exact_ab=True)
    if 3 in sc and "c3" in only:
        configs["c3"] = forward_workload(scenes.CONFIG_NAMES[3], sc[3], sc[3].cameras[0], args, torch, get("c3"),
                                         ladder=True, exact_ab=True)
    sweep = {}
    if "sweep" in only:
        for k in (2, 3):
            r = forward_workload(f"{scenes.CONFIG_NAMES[k]} at 2x", sc[k], big[k], args, torch, get(f"c{k}x2"),
                                 ladder=(k == 2))
            sweep[f"c{k}"] = {"1x": configs.get(f"c{k}", {}).get("local", {}).get("mpix_s"),
                              "1x_plain": configs.get(f"c{k}", {}).get("plain", {}).get("mpix_s"),
                              "2x": r["local"]["mpix_s"], "2x_plain": r["plain"]["mpix_s"],
                              "2x_local_over_plain": r["local_over_plain"],
                              "1x_local_over_plain": configs.get(f"c{k}", {}).get("local_over_plain"),
                              "2x_size": f"{big[k].width}x{big[k].height}", "2x_detail": r}
    if 4 in sc and "c4" in only:
        configs["c4"] = train_workload(scenes.CONFIG_NAMES[4], sc[4], sc[4].cameras, args, torch, 104,
                                       steps=max(10, args.steps), exact_ab=True)
        del sc[4]
    head = None
    if 5 in sc and "c5" in only:
        head = train_workload(scenes.CONFIG_NAMES[5], sc[5], sc[5].cameras, args, torch, 105, steps=args.steps,
                              fwd_too=True)
        configs["c5"] = head
    clock1 = gpu_clock_mhz(torch)
    log("GPU work done; waiting for the oracle")
    cpu = None
    if cpu_fut is not None:
        cpu = cpu_fut.result()
        cpu["cores"] = 1
        cpu["host_cpu"] = model
        cpu["host_threads_available"] = avail

    # the headline line
    if head is not None:
        hl = head["local"]["fwd_bwd"]
        value = mpix(head["pixels"], hl["graph"]["wall_ms"])
        plain_value = mpix(head["pixels"], head["plain"]["fwd_bwd"]["graph"]["wall_ms"]) if "plain" in head else None
        ms_step = hl["graph"]["wall_ms"]
        roofs = head["rooflines"]
        dom = max(roofs, key=lambda k: roofs[k]["ms"])
        roof = dict(roofs[dom])
        roof["traffic"] = measured_traffic(roof["kernel"])
        workload = "clustered-10M-16views-mixed forward+backward (16 views, one captured graph per step)"
        cfg = {"workload": workload, "gaussians": int(sc[5].n), "sh_degree": int(sc[5].sh_degree),
               "views": head["views"], "pixels": head["pixels"], "pairs": head["pairs"], "tuned": head["tuned"]}
    else:
        # a subset run (profiling): the first workload that ran stands in
        name, r = next(iter(configs.items())) if configs else (None, None)
        value = plain_value = ms_step = None
        roof, cfg = None, {"workload": f"subset run: {args.only}"}
        if r is not None:
            key = "fwd_bwd" if "fwd_bwd" in r.get("local", {}) else None
            g = r["local"][key]["graph"] if key else r["local"]["graph"]
            value, ms_step = mpix(r["pixels"], g["wall_ms"]), g["wall_ms"]
            roof = r.get("rooflines", {}).get("bwd_render") or r.get("render_roofline")
            cfg["workload"] = r["workload"]
    out = {
        "metric": "Mpix/s fwd and fwd+bwd vs plain per-pixel raster on same MI355X at 2e-4 tol",
        "value": value, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (alpha exponent in f64)", "data": "synthetic", "config": cfg,
        "plain_value": plain_value,
        "local_over_plain": (value / plain_value) if (value and plain_value) else None,
        "timing": head["local"]["fwd_bwd"]["graph"] if head else None,
        "gpu_clock_mhz": {"before": clock0, "after": clock1},
        "roofline": roof, "cpu_baseline": cpu,
        "stages_ms": head["local"]["stages_ms"] if head else None,
        "rooflines": head["rooflines"] if head else None,
        "configs": configs,
    }
    if sweep:
        out["resolution_sweep"] = sweep
    abl = {k: configs[k]["ablation"] for k in ("c2", "c3") if k in configs and "ablation" in configs[k]}
    if "c2" in sweep and "ablation" in sweep["c2"]["2x_detail"]:
        out["precision_3840x2160"] = sweep["c2"]["2x_detail"]["ablation"]
    if abl:
        out["ablation"] = abl
    par = {}
    for k, r in list(configs.items()) + [(f"{k}@2x", v["2x_detail"]) for k, v in sweep.items()]:
        if "parity" in r:
            par[k] = {v: {"stored": p["stored"], "fp64": p["fp64"]} for v, p in r["parity"].items()}
    out["parity"] = par
    print(json.dumps(out, default=float), flush=True)


if __name__ == "__main__":
    main()
