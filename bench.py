#!/usr/bin/env python3
"""Throughput of the hierarchical-3DGS forward render on one MI355X:
batched learned-LOD rendering against the plain threshold cut.

Workload (plan2m-lod): the 2M-leaf floor-plan scene (20 x 15 m, SH degree 3,
8-level hierarchy) seen from 500 held-out robot poses at 1280x720 (fx = 900,
1.2 m height, uniform yaw).  One step renders a batch of views (default 50)
through the whole path -- learned LOD cut, projection, depth sort, pair
emission, tile sort, compositing -- in one call; the batches cycle through
the held-out poses, inputs resident in HBM.  The learned cut's network is
the committed checkpoint trained on the scene's 2,000 training poses with
the library's kernels (trained here if absent).

Prints one JSON line: Mpixels/s of the batched learned path (value) and, on
the same poses, the batched threshold cut at tau = 1, the batched threshold
cut at the tau whose PSNR loss matches the learned cut's, the plain
single-view tau = 1 path, the PSNR loss against ground-truth images of the
synthetic surfaces, the roofline of the dominant kernel (stage times from HIP
events recorded on the render stream) and the FP64 CPU oracle's rate on a
bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixels/s at 720p: batched learned-LOD vs plain cut at ≤0.1 dB PSNR loss"
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# Algorithmic FP32 vector operations of one evaluated (pixel, Gaussian) pair
# in the compositor: dx, dy, q, the exponent scale -q/2 log2(e), exp2, alpha,
# the 0.99 cap, two compares, T', the weight, three colour FMAs and one depth
# FMA -- 21 lane operations.  Counting flops instead (an FMA as two, the
# tile-relative offsets and conic factors written out) gives 24.
OPS_PER_PAIR = 21
FLOPS_PER_PAIR_ALT = 24
TRAFFIC_FILE = "composite_traffic_plan2m_lod_50x720p.txt"
# Launch plans the autotuner chose on MI355X for the workloads below (scene,
# views, LOD and lanes key each line); its top plans lie within a fraction
# of a percent of each other, so a stored plan keeps the timed kernels, and
# the profiles taken of them, the same from run to run.
PLAN_CACHE = os.path.join(ROOT, "paper_2603_15186_amd", "plans", "mi355x.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--views", type=int, default=50, help="views per step")
    ap.add_argument("--poses", type=int, default=500, help="held-out poses cycled through")
    ap.add_argument("--single", type=int, default=100, help="poses timed on the single-view path")
    ap.add_argument("--model", default=None, help="learned-cut checkpoint (.npz)")
    ap.add_argument("--cpu-frames", type=int, default=8, help="held-out frames the CPU oracle renders")
    ap.add_argument("--oracle-pixels", type=int, default=4000,
                    help="building30m: pixels per quality view the oracle's full-leaf render computes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch kernels instead of replaying a graph")
    ap.add_argument("--workload", default="plan2m-lod",
                    choices=["plan2m-lod", "box20k", "plan2m", "plan8m", "building30m", "slice", "nav", "backward"],
                    help="plan2m-lod (the metric's workload), box20k (the flat 20k-Gaussian box, one 256x256 "
                         "view), plan2m (the 2M-leaf plan's 200-pose trajectory, tau=1), plan8m (256 "
                         "mixed-resolution views of the "
                         "8M-leaf plan, threshold cuts), building30m (64 1080p views of the 30M-leaf "
                         "two-floor building, learned cut), slice (GS-slice collision map of the 30M-leaf "
                         "building), nav (expert trajectories on the building's navigable maps) or backward "
                         "(the backward pass of the headline batch); the last five are reported for "
                         "reference")
    ap.add_argument("--plan-cache", default=PLAN_CACHE,
                    help="launch-plan cache of the library's autotuner: a plan stored for the same scene, views "
                         "and LOD is applied without timing; a missing one is tuned and appended")
    ap.add_argument("--retune", action="store_true", help="tune every launch plan afresh (cache not used)")
    ap.add_argument("--quick", action="store_true",
                    help="only the timed batched learned path (for profilers): no quality evaluation, no "
                         "threshold or single-view comparison")
    ap.add_argument("--with-backward", action="store_true",
                    help="with --quick: also time the backward pass of the learned batch")
    return ap.parse_args()


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_frames(scene, cams, model=None, tau=1.0):
    """The FP64 oracle renders whole frames of `cams`: the threshold cut at
    tau, or the learned cut of `model` (FP64 features and network), then
    projection and per-pixel compositing of every pixel.  Returns (seconds,
    pixels, Gaussians per frame)."""
    from oracle import mlp as M
    from oracle import oracle as O
    t0 = time.perf_counter()
    px, sizes = 0, []
    for cam in cams:
        if model is None:
            ids = O.cut(scene, cam, O.MODE_THRESHOLD, tau)
        else:
            ids, _ = O.cut_learned(scene, cam, M.bf16_value(model.bf16), model.mean, model.std, model.p_star,
                                   model.s_hi, tau=tau)
        O.render(scene, cam, ids=ids)
        px += cam.width * cam.height
        sizes.append(int(ids.size))
    return time.perf_counter() - t0, px, sizes


def hbm_probe(r, torch, gib=1, reps=10):
    """Attainable HBM bandwidth (GB/s, read + write) of the library's
    streaming copy over a `gib` GiB buffer, HIP events on the stream."""
    n = (gib << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        r.stream_copy(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        r.stream_copy(a, b)
    e1.record(stream)
    torch.cuda.synchronize()
    ok = bool(torch.equal(a, b))
    gbs = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs, ok


# Algorithmic bytes of the HBM-bound stages (the minimum each must move):
# cut: a visited (node, view) reads its 16-byte bounding sphere and 8-byte
# child range, an emitted id is 4 bytes; projection: a cut Gaussian reads
# its 236 bytes (mean, scale, quaternion, opacity, degree-3 SH) and 4-byte
# id and writes a 48-byte record; binning: the tile-count scan reads 8 bytes
# per Gaussian, pair emission writes 12 bytes per pair, the sort reads and
# writes each pair once (24 bytes), the tile ranges read 8.
def stage_bytes(visited, cut, pairs, sh_bytes=192):
    return {"cut": 24 * visited + 4 * cut,
            "project": (44 + sh_bytes + 4 + 48) * cut,
            "sort": 8 * cut + (12 + 24 + 8) * pairs}


def composite_kernel(plan):
    """Name of the compositing kernel a launch plan runs (as rocprofv3 shows
    it): the batch depth is capped at the tile's thread count."""
    tw, th, px = plan["tile_w"], plan["tile_h"], plan["pixels_per_thread"]
    if plan["persistent"] and (tw, th) == (16, 16):
        return f"k_composite_persistent<{plan['batch_depth']}, false, false>"
    if (tw, th) == (16, 16):
        px = 1 if plan["persistent"] else px
    return f"k_composite<{tw}, {th}, {px}, {min(plan['batch_depth'], tw * th // px)}, false, false>"


def traffic_entry(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size),
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    e = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            e[k.strip()] = v.strip()
    if e.get("kernel") != kernel:
        return None
    h = hashlib.sha1()
    for name in e["source"].split():
        with open(os.path.join(ROOT, "paper_2603_15186_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != e.get("source_sha1"):
        return None
    return int(e["bytes_per_launch"])


def timed_loop(r, hgs, torch, batches, outs, steps, warmup, stage_timing):
    """Render `steps` batches (cycling) after `warmup` untimed ones; returns
    (ms per step, stats with stage sums)."""
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        r.set_cameras(batches[i % len(batches)])
        r.render(outs)
    r.set_option(hgs.HGS_OPT_SYNC_CHECK, 0)
    if stage_timing:
        r.set_option(hgs.HGS_OPT_STAGE_TIMING, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        r.set_cameras(batches[i % len(batches)])
        r.render(outs, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if r.check() != hgs.HGS_OK:
        raise RuntimeError("work buffers overflowed inside the timed region")
    st = r.stats()
    if stage_timing:
        r.set_option(hgs.HGS_OPT_STAGE_TIMING, 0)
    r.set_option(hgs.HGS_OPT_SYNC_CHECK, 1)
    return (t1 - t0) * 1e3 / steps, st


def apply_plan(r, hgs, plan):
    """Set the launch options of an autotuned plan."""
    r.set_tile_shape(plan["tile_w"], plan["tile_h"], plan["pixels_per_thread"])
    r.set_option(hgs.HGS_OPT_BATCH_DEPTH, plan["batch_depth"])
    r.set_option(hgs.HGS_OPT_PERSISTENT, plan["persistent"])
    r.set_option(hgs.HGS_OPT_SORT_DIGIT_BITS, plan["sort_digit_bits"])


def time_backward(r, hgs, torch, batches, outs, steps, lanes=1, keep=True):
    """ms per backward pass of a batch: each step renders a batch (untimed
    part of the stream; with keep, keeping its pixel states for the backward
    pass) and runs the backward pass with fixed random image gradients; only
    the backward is inside the HIP events."""
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
    r.set_option(hgs.HGS_OPT_LANES, 1)          # the backward pass needs a one-pass render
    r.set_tile_shape(16, 16, 1)                 # and 16x16 tiles
    r.set_option(hgs.HGS_OPT_KEEP_STATE, 1 if keep else 0)
    gen = torch.Generator(device="cuda").manual_seed(0)
    grads = [tuple(torch.randn(t.shape, generator=gen, device="cuda") for t in o) for o in outs]
    stream = torch.cuda.current_stream()
    total = 0.0
    acc = None
    for i in range(steps + 1):
        r.set_cameras(batches[i % len(batches)])
        r.render(outs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        acc = r.backward(grads, out=acc)
        e1.record(stream)
        torch.cuda.synchronize()
        if i:                                   # the first one warms up
            total += e0.elapsed_time(e1)
    r.set_option(hgs.HGS_OPT_KEEP_STATE, 0)
    r.set_option(hgs.HGS_OPT_LANES, lanes)
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 1)
    return total / steps


# FP32 operations per evaluated (pixel, Gaussian) pair of the backward
# compositing kernel, counted from its formulas (FMA = 2): the reverse step
# (64: q and alpha 13, transmittance recovery 2, dL/dalpha 14, colour and
# depth gradients 4, what-lies-behind updates 8, the conic and mean gradients
# 19, opacity 2, rounded up to whole FMAs).  The timed renders keep their
# pixel states, so the kernel does not replay the forward walk (24 more
# per pair when it does).
FLOPS_PER_PAIR_BWD = 64


def run_backward(args):
    """Backward pass of the headline batch: 50 held-out 1280x720 views of
    plan2m-lod with the learned cut, random image gradients; each step
    renders the batch and runs the backward pass, only the backward is timed
    (HIP events on the stream).  The oracle's FP64 autograd gradients are
    timed on a 128x128 window of one view for the CPU baseline."""
    import numpy as np
    import torch
    from paper_2603_15186_amd import hgs, lod
    from paper_2603_15186_amd.synth import workloads as W
    scene, _, eval_cams = W.plan2m_lod()
    B = args.views
    batches = [eval_cams[i:i + B] for i in range(0, min(len(eval_cams), args.poses) - B + 1, B)]
    px_per_step = B * eval_cams[0].width * eval_cams[0].height
    r = hgs.Renderer(0)
    r.load_scene(scene)
    model = lod.LodModel.load(args.model or lod.default_model_path())
    model.install(r)
    r.set_lod(hgs.HGS_LOD_LEARNED, 1.0)
    r.set_cameras(batches[0])
    outs = r.alloc_outputs()
    gen = torch.Generator(device="cuda").manual_seed(0)
    grads = [tuple(torch.randn(t.shape, generator=gen, device="cuda") for t in o) for o in outs]
    # evaluated pairs per batch (forward count; the backward walks the same pairs)
    r.set_option(hgs.HGS_OPT_COUNT_NALG, 1)
    n_alg = []
    for bt in batches:
        r.set_cameras(bt)
        r.render(outs)
        n_alg.append(r.stats()["n_alg"])
    r.set_option(hgs.HGS_OPT_COUNT_NALG, 0)
    # the renders keep their pixel states for the backward pass
    r.set_option(hgs.HGS_OPT_KEEP_STATE, 1)
    acc = None
    for i in range(args.warmup):
        r.set_cameras(batches[i % len(batches)])
        r.render(outs)
        acc = r.backward(grads, out=acc)
    torch.cuda.synchronize()
    r.set_option(hgs.HGS_OPT_STAGE_TIMING, 1)
    stream = torch.cuda.current_stream()
    total = 0.0
    alg = 0
    for i in range(args.steps):
        r.set_cameras(batches[i % len(batches)])
        r.render(outs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        acc = r.backward(grads, out=acc)
        e1.record(stream)
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
        alg += n_alg[i % len(batches)]
    st = r.stats()
    r.set_option(hgs.HGS_OPT_STAGE_TIMING, 0)
    ms = total / args.steps
    # for reference: the backward pass replaying the forward walk itself
    r.set_option(hgs.HGS_OPT_KEEP_STATE, 0)
    ms_replay = time_backward(r, hgs, torch, batches, outs, args.steps, keep=False)
    ms_comp = st["ms_bwd_composite"] / max(st["timed_backwards"], 1)
    achieved = FLOPS_PER_PAIR_BWD * (alg / args.steps) / (ms_comp * 1e-3) / 1e12
    log(f"backward {ms:.3f} ms per batch (compositing {ms_comp:.3f} ms), {px_per_step / ms / 1e3:.1f} Mpix/s")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import grad as G
        from oracle import oracle as O
        cam = batches[0][0]
        x0, y0, w = 576, 296, 128
        ids = O.cut(scene, cam, O.MODE_THRESHOLD, 1.0)
        pr = O.project(scene, ids, cam)
        ok = pr[:, O.PF["valid"]] > 0
        ex = np.sqrt(9.0 * pr[:, O.PF["S00"]]) + 1
        ey = np.sqrt(9.0 * pr[:, O.PF["S11"]]) + 1
        near = ok & (pr[:, O.PF["u"]] + ex >= x0) & (pr[:, O.PF["u"]] - ex <= x0 + w) & \
            (pr[:, O.PF["v"]] + ey >= y0) & (pr[:, O.PF["v"]] - ey <= y0 + w)
        sub = ids[near]
        yy, xx = np.mgrid[y0:y0 + w, x0:x0 + w]
        rng = np.random.default_rng(0)
        P = w * w
        up = (rng.normal(size=(P, 3)), rng.normal(size=P), rng.normal(size=P))
        t0 = time.perf_counter()
        p = G.leaf_params(scene, sub)
        G.render(p, scene.sh_degree, cam, xx.ravel(), yy.ravel(), upstream=up)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": P / t_cpu / 1e6, "unit": "Mpixels/s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": f"FP64 autograd gradients of a {w}x{w} window of one view ({sub.size} Gaussians "
                         f"reaching it, threshold cut tau=1), {t_cpu:.2f} s"}
    out = {"metric": "Mpixels/s, backward pass (image gradients to Gaussian parameters) of the 720p "
                     "learned-LOD batch",
           "value": px_per_step / ms / 1e3, "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "plan2m-lod 50 x 1280x720 held-out views, learned LOD cut, random image "
                                  "gradients", "kept_pixel_states": True, "parallelism": "single GPU"},
           "roofline": {"kernel": "k_composite_bwd", "bound": "alu", "achieved": achieved,
                        "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                        "traffic": None, "ms_per_launch": ms_comp, "n_alg_per_launch": alg / args.steps,
                        "flops_per_pair": FLOPS_PER_PAIR_BWD},
           "cpu_baseline": cpu,
           "extra": {"ms_backward_composite": ms_comp,
                     "ms_backward_params": st["ms_bwd_total"] / max(st["timed_backwards"], 1) - ms_comp,
                     "ms_per_step_replaying_forward": ms_replay}}
    print(json.dumps(out), flush=True)
    r.close()


def composite_roofline(r, hgs, torch, batches, outs, steps):
    """Compositor roofline of the batches as rendered now: evaluated pairs
    per step (counted in an untimed pass) and the compositing kernel's mean
    time (HIP events on the render stream, eager launches)."""
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
    r.set_option(hgs.HGS_OPT_COUNT_NALG, 1)
    n_alg = n_eval = 0
    for bt in batches:
        r.set_cameras(bt)
        r.render(outs)
        st = r.stats()
        n_alg += st["n_alg"]
        n_eval += st["n_eval"]
    r.set_option(hgs.HGS_OPT_COUNT_NALG, 0)
    _, st = timed_loop(r, hgs, torch, batches, outs, steps, 1, True)
    n = st["timed_renders"]
    stage = {k: st["ms_" + k] / n for k in ("cut", "project", "sort", "composite")}
    per_step = n_alg / len(batches)
    achieved = OPS_PER_PAIR * per_step / (stage["composite"] * 1e-3) / 1e12
    roof = {"kernel": "k_composite", "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
            "ms_per_launch": stage["composite"], "n_alg_per_launch": per_step, "ops_per_pair": OPS_PER_PAIR}
    return roof, stage, {"lane_efficiency": n_alg / max(n_eval, 1), "cut_entries": st["cut_size"],
                         "pairs": st["pairs"]}


def run_box20k(args):
    """The flat scene: 20,000 Gaussians in a 4 x 4 x 3 m box, one 256 x 256
    camera (f = 256) 1 m outside the box looking in; every render is the
    whole path for that one view (no hierarchy), replayed from a graph."""
    import torch
    from paper_2603_15186_amd import hgs
    from paper_2603_15186_amd.synth import workloads as W
    scene, cams = W.box20k()
    r = hgs.Renderer(0)
    r.load_scene(scene)
    r.set_cameras(cams)
    outs = r.alloc_outputs()
    px = cams[0].width * cams[0].height
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0 if args.no_graph else 1)
    ms, _ = timed_loop(r, hgs, torch, [cams], outs, args.steps, args.warmup, False)
    roof, stage, info = composite_roofline(r, hgs, torch, [cams], outs, args.steps)
    log(f"box20k: {ms * 1e3:.1f} us per frame, {px / (ms * 1e-3) / 1e6:.0f} Mpix/s")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        t_cpu, npx, _ = oracle_frames(scene, cams)
        cpu = {"value": npx / t_cpu / 1e6, "unit": "Mpixels/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"the whole 256x256 frame ({t_cpu:.2f} s); host CPU {cpu_model()}"}
    out = {"metric": "Mpixels/s, flat 20k-Gaussian scene, one 256x256 view per render",
           "value": px / (ms * 1e-3) / 1e6, "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "box20k: 20,000 Gaussians, 4x4x3 m box, one 256x256 view, f=256",
                      "parallelism": "single GPU"},
           "roofline": roof, "cpu_baseline": cpu,
           "extra": {"stage_ms_eager": stage, **info}}
    print(json.dumps(out), flush=True)
    r.close()


def run_plan2m(args):
    """The 2M-leaf plan along its 200-pose robot trajectory at 1280x720 with
    the tau = 1 threshold cut: batches of 50 consecutive poses in one call,
    and the plain path of one view per call."""
    import numpy as np
    import torch
    from paper_2603_15186_amd import hgs
    from paper_2603_15186_amd.synth import workloads as W
    scene, cams = W.plan2m()
    r = hgs.Renderer(0)
    r.load_scene(scene)
    r.set_lod(hgs.HGS_LOD_THRESHOLD, 1.0)
    B = args.views
    batches = [cams[i:i + B] for i in range(0, len(cams) - B + 1, B)]
    px = B * cams[0].width * cams[0].height
    r.set_cameras(batches[0])
    outs = r.alloc_outputs()
    r.autotune(None if args.retune else args.plan_cache, reps=2)
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0 if args.no_graph else 1)
    ms, _ = timed_loop(r, hgs, torch, batches, outs, args.steps, args.warmup, False)
    roof, stage, info = composite_roofline(r, hgs, torch, batches, outs, args.steps)
    # plain single-view path over the whole trajectory
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
    r.set_cameras([cams[0]])
    o1 = r.alloc_outputs()
    ms1, _ = timed_loop(r, hgs, torch, [[c] for c in cams], o1, len(cams), 3, False)
    px1 = cams[0].width * cams[0].height
    log(f"plan2m: batched {ms:.3f} ms per {B} views ({px / (ms * 1e-3) / 1e6:.0f} Mpix/s), single view "
        f"{ms1:.3f} ms ({px1 / (ms1 * 1e-3) / 1e6:.0f} Mpix/s)")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        sample = cams[::len(cams) // args.cpu_frames][:args.cpu_frames]
        t_cpu, npx, sizes = oracle_frames(scene, sample)
        cpu = {"value": npx / t_cpu / 1e6, "unit": "Mpixels/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"{len(sample)} of the 200 trajectory poses, whole frames (threshold cut tau=1, "
                         f"{int(np.mean(sizes))} Gaussians per frame), {t_cpu:.1f} s; host CPU {cpu_model()}"}
    out = {"metric": "Mpixels/s, 2M-leaf plan, 200-pose trajectory at 1280x720, threshold cut tau=1",
           "value": px / (ms * 1e-3) / 1e6, "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"plan2m trajectory, {B} views per call, 1280x720 fx=900, tau=1",
                      "nodes": scene.n, "parallelism": "single GPU"},
           "roofline": roof, "cpu_baseline": cpu,
           "extra": {"stage_ms_eager": stage, "single_view_ms": ms1, "single_view_mpix_s": px1 / (ms1 * 1e-3) / 1e6,
                     "speedup_batched_vs_single": (px / ms) / (px1 / ms1), **info}}
    print(json.dumps(out), flush=True)
    r.close()


def run_plan8m(args):
    """256 views (128 @ 320x240, 96 @ 640x480, 32 @ 1280x720) of the
    8M-leaf 40 x 30 m plan in one call, threshold cuts at tau 1, 2, 4."""
    import torch
    from paper_2603_15186_amd import hgs
    from paper_2603_15186_amd.synth import workloads as W
    t = time.perf_counter()
    scene, views = W.plan8m()
    log(f"plan8m: {scene.n} nodes, {len(views)} views ({time.perf_counter() - t:.1f} s)")
    r = hgs.Renderer(0)
    r.load_scene(scene)
    r.set_cameras(views)
    outs = r.alloc_outputs()
    px = sum(c.width * c.height for c in views)
    res = {}
    for tau in (1.0, 2.0, 4.0):
        r.set_lod(hgs.HGS_LOD_THRESHOLD, tau)
        plan = r.autotune(None if args.retune else args.plan_cache, reps=2)
        r.set_option(hgs.HGS_OPT_USE_GRAPH, 0 if args.no_graph else 1)
        ms, _ = timed_loop(r, hgs, torch, [views], outs, args.steps, args.warmup, False)
        r.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
        _, st = timed_loop(r, hgs, torch, [views], outs, 3, 1, True)
        n = st["timed_renders"]
        res[f"tau{tau:g}"] = {"ms_per_batch": ms, "mpix_s": px / (ms * 1e-3) / 1e6, "cut": st["cut_size"],
                               "pairs": st["pairs"], "passes": st["passes"],
                               "plan": {k: plan[k] for k in ("lanes", "batch_depth", "persistent", "sort_digit_bits")},
                               "stage_ms": {k: st["ms_" + k] / n for k in ("cut", "project", "sort", "composite")}}
        log(f"tau={tau}: {ms:.2f} ms per batch, {res[f'tau{tau:g}']['mpix_s']:.0f} Mpix/s")
    out = {"metric": "Mpixels/s, 256 mixed-resolution views of the 8M-leaf plan in one call",
           "value": res["tau1"]["mpix_s"], "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["tau1"]["ms_per_batch"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "plan8m 256 views (128@320x240, 96@640x480, 32@1280x720), threshold tau=1",
                      "nodes": scene.n, "pixels_per_batch": px, "parallelism": "single GPU"},
           "extra": res}
    print(json.dumps(out), flush=True)
    r.close()


def run_building(args):
    """64 views at 1920x1080 (f = 1300) along trajectories on both floors of
    the 30M-leaf building, rendered in one call with the learned cut (the
    2M-leaf plan's network; threshold fallback) and with the tau = 1 cut.
    Frames/s, Mpixels/s, peak device memory in use, and PSNR of 8 sampled
    views against the full-leaf render and the surfaces' ground truth."""
    import numpy as np
    import torch
    from paper_2603_15186_amd import hgs, lod
    from paper_2603_15186_amd.synth import workloads as W
    t = time.perf_counter()
    scene, views, plan = W.building30m(with_plan=True)
    log(f"building30m: {scene.n} nodes, {len(views)} views ({time.perf_counter() - t:.1f} s)")
    r = hgs.Renderer(0)
    r.load_scene(scene)
    r.set_surfaces(plan.surfaces)
    own = lod.default_model_path("building30m_lod_mlp.npz")
    calib = W.building30m_calibration(plan)
    table, closs = [], float("nan")
    if args.model is None and os.path.exists(own):
        # the building's own network (trained and calibrated on its poses)
        model = lod.LodModel.load(own)
        origin = os.path.relpath(own, ROOT)
        p_star = model.p_star
    else:
        # the 2M-leaf plan's network: p* is calibrated again on 16 poses of
        # this building (other trajectories); the threshold cut is the
        # fallback when no p* keeps the loss within budget
        model = lod.LodModel.load(args.model or lod.default_model_path())
        origin = os.path.relpath(args.model or lod.default_model_path(), ROOT)
        crefs = lod.reference_images(r, calib)
        cbase, _, _ = lod.evaluate(r, calib, crefs, None, tau=1.0)
        p_star, closs, table = lod.calibrate(r, model, calib, crefs, cbase)
        model.p_star = p_star
        del crefs
    log(f"learned cut: {origin}, p* = {p_star}")
    model.install(r)
    free0, total = torch.cuda.mem_get_info()
    peak = total - free0
    r.set_cameras(views)
    outs = r.alloc_outputs()
    px = sum(c.width * c.height for c in views)
    res = {}
    for name, mode in (("learned", hgs.HGS_LOD_LEARNED), ("tau1", hgs.HGS_LOD_THRESHOLD)):
        r.set_lod(mode, 1.0)
        plan_ = r.autotune(None if args.retune else args.plan_cache, reps=2)
        r.set_option(hgs.HGS_OPT_USE_GRAPH, 0 if args.no_graph else 1)
        ms, _ = timed_loop(r, hgs, torch, [views], outs, args.steps, args.warmup, False)
        free, _ = torch.cuda.mem_get_info()
        peak = max(peak, total - free)
        r.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
        _, st = timed_loop(r, hgs, torch, [views], outs, 2, 1, True)
        n = st["timed_renders"]
        res[name] = {"ms_per_batch": ms, "frames_s": len(views) / (ms * 1e-3), "mpix_s": px / (ms * 1e-3) / 1e6,
                     "cut": st["cut_size"], "pairs": st["pairs"], "passes": st["passes"],
                     "plan": {k: plan_[k] for k in ("batch_depth", "persistent", "sort_digit_bits")},
                     "stage_ms": {k: st["ms_" + k] / n for k in ("cut", "project", "sort", "composite")}}
        log(f"{name}: {ms:.2f} ms per batch, {res[name]['mpix_s']:.0f} Mpix/s, cut {st['cut_size']}")
    del outs
    torch.cuda.empty_cache()
    # quality on 8 sampled views (untimed)
    sample = views[::8]
    full = lod.render_rgb(r, sample, hgs.HGS_LOD_ALL_LEAVES, 1.0)
    gt = lod.reference_images(r, sample)
    q, imgs = {}, {}
    for name, mode in (("learned", hgs.HGS_LOD_LEARNED), ("tau1", hgs.HGS_LOD_THRESHOLD)):
        img = lod.render_rgb(r, sample, mode, 1.0)
        imgs[name] = [t.cpu().numpy() for t in img]
        q[name] = {"psnr_vs_gpu_full_leaf_render_db": float(np.mean(lod.psnr(r, img, full))),
                   "psnr_vs_surfaces_db": float(np.mean(lod.psnr(r, img, gt)))}
        free, _ = torch.cuda.mem_get_info()
        peak = max(peak, total - free)
    imgs["gpu_full_leaf"] = [t.cpu().numpy() for t in full]
    del full, gt
    torch.cuda.empty_cache()
    # the FP64 oracle's full-leaf render (every leaf projected, no cut) of
    # sampled pixels of the same 8 views: the PSNR reference, and the
    # oracle's time per 1080p frame extrapolated from the sample
    from oracle import oracle as O
    rng = np.random.default_rng(8)
    n_px = args.oracle_pixels
    se = {k: 0.0 for k in imgs}
    t_proj = t_pix = 0.0
    leaves = O.cut(scene, sample[0], O.MODE_ALL_LEAVES)
    for v, cam in enumerate(sample):
        t0 = time.perf_counter()
        pr = O.project(scene, leaves, cam)
        t1 = time.perf_counter()
        sx = rng.integers(0, cam.width, n_px)
        sy = rng.integers(0, cam.height, n_px)
        pres = O.render_pixels(pr, cam, sx, sy)
        t_pix += time.perf_counter() - t1
        t_proj += t1 - t0
        ref = pres.primary[:, :3]
        for k, im in imgs.items():
            se[k] += float(((im[v][:, sy, sx].T.astype(np.float64) - ref) ** 2).sum())
        del pr
    npx_frame = sample[0].width * sample[0].height
    for k in imgs:
        mse = max(se[k] / (3 * n_px * len(sample)), 1e-10)
        q.setdefault(k, {})["psnr_vs_oracle_full_leaf_db"] = float(10.0 * np.log10(1.0 / mse))
    oracle_s_frame = (t_proj + t_pix * npx_frame / n_px) / len(sample)
    q["oracle_reference"] = (f"FP64 oracle full-leaf render ({leaves.size} leaves projected per view) of {n_px} "
                             f"random pixels in each of the 8 views; PSNR over those pixels")
    log(f"quality: {q}")
    out = {"metric": "Mpixels/s, 64 views at 1920x1080 of the 30M-leaf building in one call (learned cut)",
           "value": res["learned"]["mpix_s"], "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["learned"]["ms_per_batch"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "building30m 64 views 1920x1080 fx=1300, learned cut (threshold tau=1 fallback)",
                      "nodes": scene.n,
                      "pixels_per_batch": px,
                      "parallelism": "single GPU"},
           "cpu_baseline": {"value": npx_frame / oracle_s_frame / 1e6, "unit": "Mpixels/s", "cores": O.num_threads(),
                            "kind": "oracle",
                            "sample": f"full-leaf 1920x1080 frames of the 8 quality views: every leaf projected "
                                      f"({t_proj / len(sample):.2f} s per view), {n_px} random pixels composited "
                                      f"per view ({t_pix / len(sample):.2f} s), frame time extrapolated to "
                                      f"{oracle_s_frame:.1f} s; host CPU {cpu_model()}"},
           "extra": {"render": res, "quality_8_views": q, "peak_device_gb": peak / 1e9,
                     "p_star": p_star, "model": origin,
                     "calibration": {"poses": len(calib), "loss_db": closs, "table": [list(t) for t in table]},
                     "frames_s_learned": res["learned"]["frames_s"],
                     "speedup_learned_vs_tau1": res["tau1"]["ms_per_batch"] / res["learned"]["ms_per_batch"]}}
    print(json.dumps(out), flush=True)
    r.close()


def run_slice(args):
    """GS-slice collision maps of the 30M-leaf building's two floors: 15
    planes 0.1 .. 1.5 m above each floor over its 20 x 15 m extent at 5 cm
    (404 x 304 cells), every leaf Gaussian sliced; timed with HIP events on
    the stream; the FP64 oracle timed on the host for the same maps."""
    import numpy as np
    import torch
    from paper_2603_15186_amd import hgs
    from paper_2603_15186_amd.synth import workloads as W
    t = time.perf_counter()
    scene, _, plan = W.building30m(with_plan=True)
    log(f"building30m: {scene.n} nodes ({time.perf_counter() - t:.1f} s)")
    r = hgs.Renderer(0)
    r.load_scene(scene)
    n_leaves = int(np.count_nonzero(scene.child_count == 0))
    floors = [np.arange(0.1, 1.55, 0.1) + f * plan.ceiling for f in range(2)]
    nx, ny, cell = 404, 304, 0.05
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        for h in floors:
            r.slice_occupancy(-0.1, -0.1, cell, nx, ny, h)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        for h in floors:
            occ, m = r.slice_occupancy(-0.1, -0.1, cell, nx, ny, h)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    frac = [float(r.slice_occupancy(-0.1, -0.1, cell, nx, ny, h)[1].float().mean()) for h in floors]
    # collision checks of 1M disc robots (radius 0.25 m) against floor 0's map
    _, m0 = r.slice_occupancy(-0.1, -0.1, cell, nx, ny, floors[0], occ=False)
    rng = np.random.default_rng(0)
    q = torch.from_numpy(rng.uniform([-0.1, -0.1], [20.1, 15.1], size=(1 << 20, 2))).cuda()
    r.disc_collision(m0, -0.1, -0.1, cell, q, 0.25)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        hits = r.disc_collision(m0, -0.1, -0.1, cell, q, 0.25)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_q = e0.elapsed_time(e1) / args.steps
    log(f"maps {ms:.3f} ms per step; 1M collision queries {ms_q:.3f} ms ({float(hits.float().mean()):.3f} colliding)")
    planes = sum(len(h) for h in floors)
    cells = planes * nx * ny
    # algorithmic bytes per step: each leaf's 48-byte record and id per map,
    # every plane and union byte written once
    alg = len(floors) * (n_leaves * 52 + (len(floors[0]) + 1) * nx * ny)
    gbs = alg / (ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        ids = np.nonzero(scene.child_count == 0)[0]
        t0 = time.perf_counter()
        for h in floors:
            O.slice_occupancy(scene.means[ids], scene.scales[ids], scene.quats[ids], scene.opacity[ids], -0.1, -0.1,
                              cell, nx, ny, h.astype(np.float32))
        t_cpu = time.perf_counter() - t0
        cpu = {"value": cells / t_cpu / 1e6, "unit": "Mcells/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"both floors' maps once ({t_cpu:.2f} s)"}
    out = {"metric": "Mcells/s, GS-slice collision maps of the 30M-leaf building (2 floors x 15 planes, 5 cm)",
           "value": cells / (ms * 1e-3) / 1e6, "unit": "Mcells/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "building30m leaves, 2 floors x 15 planes 0.1-1.5 m, 404x304 cells of 5 cm",
                      "leaves": n_leaves, "parallelism": "single GPU"},
           "roofline": {"kernel": "k_slice", "bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                        "frac": gbs / 8000.0, "traffic": None},
           "cpu_baseline": cpu,
           "extra": {"occupied_fraction_per_floor": frac, "algorithmic_bytes_per_step": alg,
                     "collision_queries_per_s": (1 << 20) / (ms_q * 1e-3), "collision_radius_m": 0.25}}
    print(json.dumps(out), flush=True)
    r.close()


def run_nav(args):
    """Expert trajectories on the 30M-leaf building: per floor the GS-slice
    collision map (15 planes, 404 x 304 cells of 5 cm, built once,
    untimed), then per step the navigable map of a 0.25 m disc robot,
    distance fields to 9 goals and 200 shortest-path trajectories per goal
    (3,600 per step over both floors, the two floors in flight together);
    the FP64 oracle timed on the host for the same step."""
    import numpy as np
    import torch
    from paper_2603_15186_amd import hgs
    from paper_2603_15186_amd.synth import workloads as W
    t = time.perf_counter()
    scene, _, plan = W.building30m(with_plan=True)
    log(f"building30m: {scene.n} nodes ({time.perf_counter() - t:.1f} s)")
    r = hgs.Renderer(0)
    r.load_scene(scene)
    nx, ny, cell, radius, cap = 404, 304, 0.05, 0.25, 2048
    floors = []
    for f in range(2):
        _, m = r.slice_occupancy(-0.1, -0.1, cell, nx, ny, np.arange(0.1, 1.55, 0.1) + f * plan.ceiling, occ=False)
        nav0 = r.navigable_map(m, -0.1, -0.1, cell, radius).cpu().numpy()
        goals, starts, slots = W.nav_queries(nav0, n_goals=9, per_goal=200, seed=f)
        floors.append((m, goals, torch.from_numpy(starts).cuda(), torch.from_numpy(slots).cuda()))

    # The floors are independent problems: each runs on a context and a HIP
    # stream of its own (the second context holds no scene; planning reads
    # only its maps), floor 1 from a worker thread, since a distance-field
    # call waits on the host between batches of rounds (the library's calls
    # release the GIL).  Together the two floors give the GPU twice the
    # waves of one, which the latency-bound relaxation rounds need.
    from concurrent.futures import ThreadPoolExecutor
    ctxs = [r, hgs.Renderer(0)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    pool = ThreadPoolExecutor(max_workers=1)
    torch.cuda.synchronize()

    def floor_step(i):
        m, goals, st, sl = floors[i]
        R, s = ctxs[i], streams[i]
        with torch.cuda.stream(s):
            nav = R.navigable_map(m, -0.1, -0.1, cell, radius, stream=s)
            dist, rounds = R.distance_fields(nav, goals, stream=s)
            paths, lens = R.trace_paths(nav, dist, st, sl, cap, stream=s)
        return nav, dist, rounds, paths, lens

    def step():
        fut = pool.submit(floor_step, 1)
        out0 = floor_step(0)
        return [out0, fut.result()]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    n_traj = sum(int(st.numel()) for _, _, st, _ in floors)
    lens = np.concatenate([x[4].cpu().numpy() for x in res])
    rounds = [x[2] for x in res]
    # stage times with HIP events, one floor at a time on one stream
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    st_ms = np.zeros(3)
    for m, goals, stt, sl in floors:
        ev[0].record(stream)
        nav = r.navigable_map(m, -0.1, -0.1, cell, radius)
        ev[1].record(stream)
        dist, _ = r.distance_fields(nav, goals)
        ev[2].record(stream)
        r.trace_paths(nav, dist, stt, sl, cap)
        ev[3].record(stream)
        torch.cuda.synchronize()
        st_ms += [ev[k].elapsed_time(ev[k + 1]) for k in range(3)]
    log(f"nav step {ms:.3f} ms (floors concurrent); one floor after the other: navigable / fields / traces "
        f"{st_ms.round(3).tolist()} ms; rounds {rounds}; "
        f"path cells mean {lens.mean():.1f} max {lens.max()}")
    cells = nx * ny
    # algorithmic bytes of the fields: every cell's 8-byte pair written once
    # and its navigable byte read once, per goal
    alg = sum(len(g) for _, g, _, _ in floors) * cells * 9
    gbs = alg / (st_ms[1] * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        maps = [(x[0].cpu().numpy(), x[1], x[2].cpu().numpy(), x[3].cpu().numpy()) for x in floors]
        t0 = time.perf_counter()
        reps = 0
        while True:
            for m, goals, stt, sl in maps:
                nav = O.navigable(m, -0.1, -0.1, cell, radius)
                d = O.distance_fields((nav == 1).astype(np.uint8), goals)
                O.trace_paths((nav == 1).astype(np.uint8), d, stt, sl, cap)
            reps += 1
            if time.perf_counter() - t0 > 3.0:
                break
        t_cpu = (time.perf_counter() - t0) / reps
        cpu = {"value": n_traj / t_cpu, "unit": "trajectories/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"the whole step ({reps} repetitions, {t_cpu * 1e3:.1f} ms each)"}
    out = {"metric": "expert trajectories/s (navigable map, distance fields, shortest paths) on the 30M-leaf "
                     "building's collision maps",
           "value": n_traj / (ms * 1e-3), "unit": "trajectories/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "building30m, 2 floors x 404x304 cells of 5 cm, 0.25 m robot, 9 goals x 200 "
                                  "starts per floor", "parallelism": "single GPU, the two floors on two streams"},
           "roofline": {"kernel": "k_dist_round", "bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                        "frac": gbs / 8000.0, "traffic": None},
           "cpu_baseline": cpu,
           "extra": {"stage_ms_one_floor_after_the_other": {"navigable": st_ms[0], "fields": st_ms[1],
                                                            "traces": st_ms[2]},
                     "relaxation_rounds": rounds, "path_cells_mean": float(lens.mean()),
                     "path_cells_max": int(lens.max()), "unreachable": int((lens <= 0).sum())}}
    print(json.dumps(out), flush=True)
    pool.shutdown()
    ctxs[1].close()
    r.close()


def main():
    args = parse()
    if args.workload == "box20k":
        return run_box20k(args)
    if args.workload == "plan2m":
        return run_plan2m(args)
    if args.workload == "plan8m":
        return run_plan8m(args)
    if args.workload == "building30m":
        return run_building(args)
    if args.workload == "slice":
        return run_slice(args)
    if args.workload == "nav":
        return run_nav(args)
    if args.workload == "backward":
        return run_backward(args)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE {world}) is not supported: the "
              "renderer shards by view across GPUs with no exchange, and only the single-GPU share is built "
              "and measured.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2603_15186_amd import hgs, lod
    from paper_2603_15186_amd.synth import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    t = time.perf_counter()
    scene, train_cams, eval_cams, plan = W.plan2m_lod(with_plan=True)
    eval_cams = eval_cams[:args.poses]
    log(f"scene: {scene.n} nodes, {scene.n_levels} levels ({time.perf_counter() - t:.1f} s)")
    B = args.views
    batches = [eval_cams[i:i + B] for i in range(0, len(eval_cams) - B + 1, B)]
    px_per_step = B * eval_cams[0].width * eval_cams[0].height

    r = hgs.Renderer(0)
    r.load_scene(scene)
    r.set_surfaces(plan.surfaces)
    path = args.model or lod.default_model_path()
    if os.path.exists(path):
        model = lod.LodModel.load(path)
        origin = os.path.relpath(path, ROOT)
    else:
        log("no checkpoint: training the learned cut ...")
        model = lod.train_pipeline(r, train_cams, calib_n=64, per_view=256, epochs=40, seed=0, log=log)
        origin = "trained in this run"
    log(f"learned cut: p*={model.p_star}, s_hi={model.s_hi} ({origin})")

    base_psnr = learn_psnr = loss = loss_m = float("nan")
    full_q = None
    base_cut = learn_cut = 1
    tau_m = 1.0
    if not args.quick:
        # quality on all held-out poses (untimed): PSNR against ground truth
        refs = lod.reference_images(r, eval_cams)
        base_psnr, base_cut, _ = lod.evaluate(r, eval_cams, refs, None, tau=1.0)
        learn_psnr, learn_cut, _ = lod.evaluate(r, eval_cams, refs, model)
        loss = base_psnr - learn_psnr
        tau_m, loss_m, cut_m = lod.tau_matched(r, eval_cams, refs, base_psnr, max(loss, 0.0))
        log(f"PSNR tau=1 {base_psnr:.3f} dB, learned {learn_psnr:.3f} dB (loss {loss:.3f} dB), "
            f"cut {learn_cut / base_cut:.3f} of tau=1; matched tau {tau_m:.2f} (loss {loss_m:.3f}, cut "
            f"{(cut_m or base_cut) / base_cut:.3f})")
        del refs
        # the same views against the full-leaf render (every leaf, no cut)
        fulls = []
        for i in range(0, len(eval_cams), B):
            fulls += [t.clone() for t in lod.render_rgb(r, eval_cams[i:i + B], hgs.HGS_LOD_ALL_LEAVES, 1.0)]
        fb, _, fb_all = lod.evaluate(r, eval_cams, fulls, None, tau=1.0)
        fl, _, fl_all = lod.evaluate(r, eval_cams, fulls, model)
        fm, _, _ = lod.evaluate(r, eval_cams, fulls, None, tau=tau_m)
        full_q = {"tau1_db": fb, "learned_db": fl, "matched_tau_db": fm, "learned_loss_db": fb - fl,
                  "note": "mean over views of per-view PSNR (MSE floored at 1e-10, i.e. at most 100 dB) against "
                          "the GPU's all-leaves render of the same view"}
        log(f"PSNR vs full-leaf render: tau=1 {fb:.2f} dB, learned {fl:.2f} dB, matched tau {fm:.2f} dB")
        del fulls
        torch.cuda.empty_cache()

    r.set_cameras(batches[0])
    outs = r.alloc_outputs()
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0 if args.no_graph else 1)
    # algorithmic counts of one learned step (untimed)
    model.install(r)
    r.set_lod(hgs.HGS_LOD_LEARNED, 1.0)
    r.set_option(hgs.HGS_OPT_COUNT_NALG, 1)
    n_alg = n_eval = 0
    per = {"visited": 0, "cut_size": 0, "pairs": 0}
    for bt in batches:
        r.set_cameras(bt)
        r.render(outs)
        st0 = r.stats()
        n_alg += st0["n_alg"]
        n_eval += st0["n_eval"]
        for k in per:
            per[k] += st0[k]
    n_alg_step = n_alg / len(batches)
    n_eval_step = n_eval / len(batches)
    per = {k: v / len(batches) for k, v in per.items()}
    r.set_option(hgs.HGS_OPT_COUNT_NALG, 0)
    # launch plan (batch depth, persistent compositing, radix digit width)
    # picked by the library's autotuner on the first batch; images do not
    # depend on it
    r.set_cameras(batches[0])
    plan = r.autotune(None if args.retune else args.plan_cache, reps=3)
    log(f"autotuned plan: {plan}")
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0 if args.no_graph else 1)

    # batched learned cut: the headline value (stage timing needs eager launches)
    ms_learn, _ = timed_loop(r, hgs, torch, batches, outs, args.steps, args.warmup, False)
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
    ms_learn_eager, st = timed_loop(r, hgs, torch, batches, outs, args.steps, 1, True)
    r.set_option(hgs.HGS_OPT_USE_GRAPH, 0 if args.no_graph else 1)
    value = px_per_step / (ms_learn * 1e-3) / 1e6
    log(f"batched learned: {ms_learn:.3f} ms/step ({ms_learn_eager:.3f} eager), {value:.1f} Mpix/s")
    n = st["timed_renders"]
    stage = {k: st["ms_" + k] / n for k in ("cut", "project", "sort", "composite")}

    if args.quick and args.with_backward:
        ms_bwd_q = time_backward(r, hgs, torch, batches, outs, args.steps, plan["lanes"])
        apply_plan(r, hgs, plan)
        log(f"backward: {ms_bwd_q:.3f} ms per batch")
    single = eval_cams[:args.single]
    px1 = single[0].width * single[0].height
    ms_t1 = ms_tm = ms_single = ms_blend = ms_bwd = ms_lanes2 = float("nan")
    if args.quick and args.with_backward:
        ms_bwd = ms_bwd_q
    plan2 = None
    if not args.quick:
        # batched threshold cuts
        r.set_lod(hgs.HGS_LOD_THRESHOLD, 1.0)
        ms_t1, _ = timed_loop(r, hgs, torch, batches, outs, args.steps, args.warmup, False)
        r.set_lod(hgs.HGS_LOD_THRESHOLD, tau_m)
        ms_tm, _ = timed_loop(r, hgs, torch, batches, outs, args.steps, args.warmup, False)
        # the learned cut with level-of-detail transition blending
        r.set_lod(hgs.HGS_LOD_LEARNED, 1.0)
        r.set_option(hgs.HGS_OPT_LOD_BLEND, 1)
        ms_blend, _ = timed_loop(r, hgs, torch, batches, outs, args.steps, args.warmup, False)
        r.set_option(hgs.HGS_OPT_LOD_BLEND, 0)
        # backward pass of the learned batch (random image gradients),
        # eager launches, timed with HIP events on the stream
        ms_bwd = time_backward(r, hgs, torch, batches, outs, args.steps, plan["lanes"])
        apply_plan(r, hgs, plan)
        # the learned batch on two pipeline lanes (passes overlapping on two
        # streams; same images), with its own launch plan
        r.set_option(hgs.HGS_OPT_LANES, 2)
        plan2 = r.autotune(None if args.retune else args.plan_cache, reps=3)
        r.set_option(hgs.HGS_OPT_USE_GRAPH, 0 if args.no_graph else 1)
        ms_lanes2, _ = timed_loop(r, hgs, torch, batches, outs, args.steps, args.warmup, False)
        r.set_option(hgs.HGS_OPT_LANES, 1)
        apply_plan(r, hgs, plan)

        # plain single-view path, tau = 1
        r.set_option(hgs.HGS_OPT_USE_GRAPH, 0)
        r.set_lod(hgs.HGS_LOD_THRESHOLD, 1.0)
        r.set_cameras([single[0]])
        o1 = r.alloc_outputs()
        stream = torch.cuda.current_stream()
        r.render(o1)
        r.set_option(hgs.HGS_OPT_SYNC_CHECK, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in single:
            r.set_cameras([c])
            r.render(o1, stream)
        torch.cuda.synchronize()
        ms_single = (time.perf_counter() - t0) * 1e3 / len(single)
        if r.check() != hgs.HGS_OK:
            raise RuntimeError("overflow in single-view timing")
        r.set_option(hgs.HGS_OPT_SYNC_CHECK, 1)
    mpix = lambda ms, px: px / (ms * 1e-3) / 1e6  # noqa: E731

    comp_ms = stage["composite"]
    # the probe's copies (1 GiB read + 1 GiB written each) also scale the
    # profiler's HBM byte counters
    probe_gbs, probe_ok = hbm_probe(r, torch)
    log(f"HBM probe: {probe_gbs:.0f} GB/s (copy {'correct' if probe_ok else 'WRONG'})")
    sb = stage_bytes(per["visited"], per["cut_size"], per["pairs"])
    stage_roof = {}
    t_min = 0.0
    for k, b in sb.items():
        gbs = b / (stage[k] * 1e-3) / 1e9
        stage_roof[k] = {"bound": "hbm", "alg_bytes": b, "ms": stage[k], "achieved_gbs": gbs,
                         "frac": gbs / HBM_PEAK_GBS, "frac_of_probe": gbs / probe_gbs}
        t_min += b / (HBM_PEAK_GBS * 1e9)
    t_min += OPS_PER_PAIR * n_alg_step / (FP32_PEAK_TFLOPS * 1e12)
    achieved = OPS_PER_PAIR * n_alg_step / (comp_ms * 1e-3) / 1e12
    stage_roof["composite"] = {"bound": "alu", "alg_ops": OPS_PER_PAIR * n_alg_step, "ms": comp_ms,
                               "achieved_tflops": achieved, "frac": achieved / FP32_PEAK_TFLOPS}
    alt = FLOPS_PER_PAIR_ALT * n_alg_step / (comp_ms * 1e-3) / 1e12
    kname = composite_kernel(plan)
    roof = {"kernel": kname, "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic_entry(kname),
            "ms_per_launch": comp_ms, "n_alg_per_launch": n_alg_step, "ops_per_pair": OPS_PER_PAIR}
    extra = {
        "composite_tflops_at_24_flops_per_pair": alt, "composite_frac_at_24_flops_per_pair": alt / FP32_PEAK_TFLOPS,
        # the build disables packed FP32 (v_pk_*): the attainable FP32 vector
        # peak is half the published one
        "composite_frac_of_unpacked_fp32_peak": achieved / (FP32_PEAK_TFLOPS / 2),
        "batched_threshold_tau1_mpix_s": mpix(ms_t1, px_per_step),
        "batched_threshold_matched_mpix_s": mpix(ms_tm, px_per_step),
        "batched_learned_blended_mpix_s": mpix(ms_blend, px_per_step),
        "backward_ms_per_step": ms_bwd, "backward_mpix_s": mpix(ms_bwd, px_per_step),
        "batched_learned_two_lanes_mpix_s": mpix(ms_lanes2, px_per_step),
        "two_lanes_plan": None if plan2 is None else {k: plan2[k] for k in ("tile_w", "tile_h", "pixels_per_thread",
                                                                               "batch_depth", "persistent",
                                                                               "sort_digit_bits")},
        "matched_tau": tau_m, "matched_tau_loss_db": loss_m,
        "plain_single_view_tau1_mpix_s": mpix(ms_single, px1),
        "speedup_vs_plain_single_view": value / mpix(ms_single, px1),
        "speedup_vs_batched_threshold_tau1": value / mpix(ms_t1, px_per_step),
        "psnr_tau1_db": base_psnr, "psnr_learned_db": learn_psnr, "psnr_loss_db": loss,
        "psnr_reference": "ray-cast ground truth of the synthetic surfaces, 3x3 supersampled",
        "psnr_vs_full_leaf_render": full_q,
        "cut_learned_over_tau1": learn_cut / base_cut,
        "learned_p_star": model.p_star, "learned_s_hi": model.s_hi, "learned_model": origin,
        "stage_ms_per_step_eager": stage, "ms_per_step_eager": ms_learn_eager, "graph": not args.no_graph,
        "stage_roofline": stage_roof, "hbm_probe_gbs": probe_gbs, "hbm_probe_correct": probe_ok,
        "frame_roofline_frac": t_min * 1e3 / ms_learn,
        "frame_roofline_frac_eager": t_min * 1e3 / sum(stage.values()),
        "cut_visited_per_step": per["visited"],
        "n_alg_per_step": n_alg_step, "held_out_poses": len(eval_cams),
        "composite_slots_per_step": n_eval_step, "composite_lane_efficiency": n_alg_step / max(n_eval_step, 1),
        "cut_entries_per_step": st["cut_size"], "visible_per_step": st["visible"], "pairs_per_step": st["pairs"],
    }
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        from oracle import oracle as O
        sample = batches[0][:args.cpu_frames]
        t_l, px_l, sz_l = oracle_frames(scene, sample, model)
        t_t, px_t, sz_t = oracle_frames(scene, sample, None, 1.0)
        cpu = {"value": px_l / t_l / 1e6, "unit": "Mpixels/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"{len(sample)} held-out 1280x720 poses (the first of the timed batch) with the learned "
                         f"cut ({int(np.mean(sz_l))} Gaussians per frame), whole frames: the oracle's cut, "
                         f"projection and every pixel composited, {t_l:.1f} s; host CPU {cpu_model()}"}
        extra["cpu_oracle"] = {"cpu_model": cpu_model(), "threads": O.num_threads(), "frames": len(sample),
                               "learned_s_per_frame": t_l / len(sample), "learned_mpix_s": px_l / t_l / 1e6,
                               "tau1_s_per_frame": t_t / len(sample), "tau1_mpix_s": px_t / t_t / 1e6,
                               "tau1_gaussians_per_frame": float(np.mean(sz_t)),
                               "learned_gaussians_per_frame": float(np.mean(sz_l))}
        log(f"oracle: learned {t_l / len(sample):.2f} s/frame, tau=1 {t_t / len(sample):.2f} s/frame")
    out = {
        "metric": METRIC, "value": value, "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_learn, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plan2m-lod 1280x720 held-out poses, batched learned LOD cut",
                   "leaves": int(np.count_nonzero(scene.child_count == 0)), "nodes": scene.n,
                   "views_per_step": B, "resolution": "1280x720", "fx": 900,
                   "lod": f"learned (p*={model.p_star}, s_hi={model.s_hi}px, threshold tau=1 fallback)",
                   "plan": {k: plan[k] for k in ("lanes", "tile_w", "tile_h", "pixels_per_thread", "batch_depth",
                                                 "persistent", "sort_digit_bits")},
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    r.close()


if __name__ == "__main__":
    main()
