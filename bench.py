"""Benchmark: one full training step of the 6D Gaussian renderer on one MI355X.

Workload: 300k view-conditioned 6D Gaussians on a noisy unit sphere with strong
view dependence (spatial-direction Cholesky entries N(0, 0.3), direction means
along the inward normals), one 800x800 camera.  A step is forward render, L1
loss against a target render of a perturbed copy, backward to the 76 raw
parameters and an Adam update -- every stage in lib6dgs.so on one stream.

Prints one JSON line (see the README of the benchmark contract in the design
notes): value = whole-step throughput in Mpixels/s, plus the roofline of the
dominant kernel and the FP64 oracle timed on the host as a CPU baseline.
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

METRIC = "fwd+bwd Mpixels/sec & train steps/sec at 300k 6D Gaussians 800x800; HBM GB/s"
HBM_PEAK_GBS = 8000.0
# MI355X's published fp32 vector peak (it counts packed fp32 issue)
FP32_PEAK_TFLOPS = 157.3
# the same without packed issue, which this code does not use: 256 CUs x 4 SIMDs
# x 16 lanes x 2 flop (FMA) x 2.4 GHz
ALU_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

# Algorithmic flops of the compositing kernels per contributing (pixel,
# Gaussian) pair -- the pairs whose alpha reaches 1/255 before the pixel
# saturates, the work any implementation must do: evaluating the Gaussian
# (offset, quadratic form, exp2, opacity, clamp: 12) plus blending it (10) in
# the forward, or plus the reverse step and its nine screen-space gradients
# (40) in the backward.
FWD_FLOPS_PER_CONTRIB = 12 + 10
BWD_FLOPS_PER_CONTRIB = 12 + 40


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the batched-views leg of the default run")
    ap.add_argument("--cpu-pixels", type=int, default=32768)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB once (a kernel of known traffic that "
                         "scales the HBM byte counters of a profiler run)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "render"],
                    help="c2: the training-step benchmark (default); c3: 16 uneven views batched in one "
                         "captured forward+backward vs 16 per-view launches; c4: 8-view training steps "
                         "from a 64-camera 1920x1080 pool, one captured graph per camera group; render: "
                         "forward-only frames per second on two 1408x1408 scenes")
    return ap.parse_args()


def source_digest(names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2410_04974_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this renderer has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "render":
        return bench_render(args)

    import numpy as np
    import torch

    import synth
    from paper_2410_04974_amd import Renderer, Trainer, _lib

    dev = torch.device("cuda:0")
    w = synth.workload("c2")
    cam = w.cameras[0]
    params_np = synth.make_scene(w.scene)
    n = params_np.shape[1]
    px = cam.width * cam.height

    tgt_r = Renderer()
    target = tgt_r.forward(torch.from_numpy(synth.perturbed(params_np)).to(dev), [cam])
    torch.cuda.synchronize()
    del tgt_r

    params = torch.from_numpy(params_np).to(dev)
    r = Renderer()
    tr = Trainer(params, r)
    # first step in grow-on-demand mode, then a fixed pair capacity: no host waits per step
    tr.step([cam], target)
    torch.cuda.synchronize()
    pairs = r.ctx.sizes()["pairs"]
    r.configure(pair_capacity=int(pairs * 1.5) + 4096)
    for _ in range(max(args.warmup - 1, 0)):
        tr.step([cam], target)
    torch.cuda.synchronize()

    # which kernel dominates a step
    r.ctx.set_timing(0x1F)
    for _ in range(3):
        tr.step([cam], target)
    kt = {k: r.ctx.kernel_time(k)[0] / 3 for k in _lib.KERNEL_NAMES}
    dom = max(kt, key=kt.get)

    # timed region: only the dominant kernel is bracketed by events
    r.ctx.set_timing(1 << dom)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        tr.step([cam], target)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r.ctx.check()  # raises if the fixed pair capacity overflowed
    ms_step = e0.elapsed_time(e1) / args.steps
    dom_ms, dom_launches = r.ctx.kernel_time(dom)
    dom_avg_ms = dom_ms / max(dom_launches, 1)

    # the same step captured as one graph and replayed (context: the timed
    # region above launches every kernel from the host)
    r.ctx.set_timing(0)
    tr.capture([cam], target, warmup=1)
    ms_graph = _timed(tr.replay, args.steps)
    r.ctx.check()

    # sizes of this workload for the algorithmic byte / flop counts
    sz = r.ctx.sizes()
    nb, P = sz["binned"], sz["pairs"]
    tiles = sz["tiles"]
    roof = roofline(r, dom, dom_avg_ms, n, nb, P, px, tiles, params, cam, target)

    out = {
        "metric": METRIC,
        "value": round(px / (ms_step * 1e-3) / 1e6, 3),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator, random-init 6D Gaussians)",
        "config": {"workload": "c2: 300k 6D Gaussians, noisy unit sphere, strong view dependence, "
                               "800x800, L1 + Adam training step",
                   "gaussians": n, "width": cam.width, "height": cam.height, "views_per_step": 1,
                   "binned": nb, "pairs": P, "tiles": tiles, "tile": [r.ctx.settings.tile_w, r.ctx.settings.tile_h],
                   "batch": sz["batch"], "chunk": sz["chunk"]},
        "train_steps_per_s": round(1e3 / ms_step, 2),
        "graph_replay": {"ms_per_step": round(ms_graph, 4), "mpixels_per_s": round(px / (ms_graph * 1e-3) / 1e6, 3)},
        "wall_s_timed": round(wall, 3),
        "kernel_ms": {_lib.KERNEL_NAMES[k]: round(v, 4) for k, v in kt.items()},
        "roofline": roof,
        "hbm": hbm_report({_lib.KERNEL_NAMES[k]: v for k, v in kt.items()}, ms_step, n, nb, P, px, tiles),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(params_np, cam, args.cpu_pixels)
    if not args.no_c3:
        del tr, r, target
        torch.cuda.empty_cache()
        out["c3_batched_views"] = c3_leg(args.steps, args.warmup)
    if args.copy_probe_mib > 0:
        a = torch.empty(args.copy_probe_mib << 18, device=dev, dtype=torch.float32).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = a.numel() * 4
    print(json.dumps(out), flush=True)


def roofline(r, dom, avg_ms, n, nb, P, px, tiles, params, cam, target):
    import numpy as np
    import torch
    from paper_2410_04974_amd import _lib

    name = _lib.KERNEL_NAMES[dom]
    sz = r.ctx.sizes()
    settings = {"tile": [r.ctx.settings.tile_w, r.ctx.settings.tile_h], "batch": sz["batch"], "chunk": sz["chunk"]}
    if dom in (_lib.K_BLEND_FWD, _lib.K_BLEND_BWD):
        # count the contributing (pixel, Gaussian) pairs in one extra forward
        cnt_r = Renderer_with_counts(r)
        cnt_r.forward(params, [cam])
        counts = float(cnt_r.ctx.export(_lib.EXPORT_COUNTS).astype(np.float64).sum())
        per = FWD_FLOPS_PER_CONTRIB if dom == _lib.K_BLEND_FWD else BWD_FLOPS_PER_CONTRIB
        achieved = per * counts / (avg_ms * 1e-3) / 1e12
        out = {"kernel": name, "bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
               "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": traffic(name, settings),
               "peak_nonpacked": round(ALU_NONPACKED_TFLOPS, 2),
               "frac_nonpacked": round(achieved / ALU_NONPACKED_TFLOPS, 4),
               "avg_ms": round(avg_ms, 4), "contributions_per_launch": counts, "flops_per_contribution": per}
        if dom == _lib.K_BLEND_BWD:
            visited = visited_block_pairs(cnt_r.ctx, cam)
            out["visited_block_pairs"] = visited
            out["lane_utilisation"] = round(counts / (64.0 * visited), 4) if visited else None
        return out
    if dom == _lib.K_PREPROCESS:
        bytes_ = 304 * n + 4 * n + 52 * nb
    elif dom == _lib.K_PREPROCESS_BWD:
        bytes_ = alg_bytes(n, nb, P, px, tiles)["preprocess_bwd"]
    else:  # integer stage: depth keys and pair lists (sort passes read and write 8 B per item)
        bytes_ = 4 * n + 8 * nb * 2 * 4 + 8 * P * 2 * 2 + 8 * tiles
    achieved = bytes_ / (avg_ms * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic(name, settings), "avg_ms": round(avg_ms, 4)}


def alg_bytes(n, nb, P, px, tiles):
    """Algorithmic HBM bytes per launch of each stage of a one-view training
    step: what the method has to read and write (n Gaussians, nb of them binned
    in the view, P (tile, Gaussian) pairs, px pixels)."""
    return {
        "preprocess": 304 * n + 4 * n + 52 * nb,            # params; tile count; record + depth
        "binning": 64 * nb + 24 * P + 4 * P + 8 * tiles,    # depth sort; pair build + tile sort; ranges
        "blend_fwd": 40 * P + 20 * px,                      # record per pair; colour, T, last per pixel
        "l1": 12 * 3 * px,                                  # image, target, gradient
        "blend_bwd": 40 * P + 32 * px + 36 * nb,            # as the forward + dL/dI; screen-space gradients
        # the chain rule fused with Adam: params, m, v in and out; tile counts; screen-space gradients
        "preprocess_bwd": 6 * 304 * n + 4 * n + 36 * nb,
    }


def hbm_report(kernel_ms, ms_step, n, nb, P, px, tiles):
    """Achieved algorithmic GB/s and the fraction of the 8 TB/s HBM peak per
    stage and for the whole step (the blend kernels are ALU-bound; their GB/s
    is reported for completeness, their roofline is the fp32 rate).  The
    step's Adam runs inside the preprocess backward."""
    b = alg_bytes(n, nb, P, px, tiles)
    ms = dict(kernel_ms)
    kernels = {}
    for k, t in ms.items():
        if k in b and t > 0:
            gbs = b[k] / (t * 1e-3) / 1e9
            kernels[k] = {"ms": round(t, 4), "bytes": int(b[k]), "GBs": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4),
                          "bound": "alu" if k in ("blend_fwd", "blend_bwd") else "hbm"}
    total = sum(b.values())
    step_gbs = total / (ms_step * 1e-3) / 1e9
    return {"step_bytes": int(total), "step_GBs": round(step_gbs, 1), "step_frac": round(step_gbs / HBM_PEAK_GBS, 4),
            "peak_GBs": HBM_PEAK_GBS, "kernels": kernels}


def c3_leg(steps, warmup):
    """The batched-views comparison at the library's automatic settings (no
    autotuning, so it fits the default run): 16 uneven cameras, 500k
    Gaussians, one captured forward + backward over all views against 16
    per-view eager forward + backward calls, images compared bitwise."""
    import torch

    import synth
    from paper_2410_04974_amd import Renderer

    w = synth.workload("c3")
    cams = w.cameras
    params = torch.from_numpy(synth.make_scene(w.scene)).to("cuda:0")
    px = sum(c.width * c.height for c in cams)
    gen = torch.Generator(device="cuda:0").manual_seed(2)
    dls = [torch.randn((3, c.height, c.width), device="cuda:0", generator=gen) for c in cams]
    rb = Renderer()
    imgs = rb.forward(params, cams)
    torch.cuda.synchronize()
    sz = rb.ctx.sizes()
    rb.configure(pair_capacity=int(sz["pairs"] * 1.3) + 4096)
    grad = torch.empty_like(params)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            rb.forward(params, cams, out=imgs)
            rb.backward(params, dls, grad=grad)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rb.forward(params, cams, out=imgs)
        rb.backward(params, dls, grad=grad)
    for _ in range(warmup):
        g.replay()
    ms_b = _timed(g.replay, steps)
    rb.ctx.check()
    per = [Renderer() for _ in cams]
    gsum = torch.empty_like(params)

    def per_view():
        for r1, c, d in zip(per, cams, dls):
            r1.forward(params, [c])
            r1.backward(params, [d], grad=gsum)

    per_view()
    torch.cuda.synchronize()
    for r1 in per:
        r1.configure(pair_capacity=int(r1.ctx.sizes()["pairs"] * 1.3) + 4096)
    equal = all(torch.equal(per[k].forward(params, [c])[0], imgs[k]) for k, c in enumerate(cams))
    for _ in range(max(1, warmup // 2)):
        per_view()
    ms_v = _timed(per_view, max(2, steps // 4))
    return {"workload": "c3: 500k 6D Gaussians, 16 Fibonacci cameras cycling 400x400, 800x800, 1280x720, "
                        "1600x900, forward + backward", "pixels": px, "pairs": sz["pairs"],
            "batched_graph": {"ms_per_step": round(ms_b, 4), "mpixels_per_s": round(px / (ms_b * 1e-3) / 1e6, 3),
                              "batch": sz["batch"], "chunk": sz["chunk"]},
            "per_view_launches": {"ms_per_step": round(ms_v, 4), "mpixels_per_s": round(px / (ms_v * 1e-3) / 1e6, 3)},
            "speedup": round(ms_v / ms_b, 3), "images_bitwise_equal": bool(equal)}


def _timed(fn, steps):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_c3(args):
    """16 uneven cameras: one captured forward+backward over all views (tile
    shape, LDS batch depth and backward chunk autotuned) against 16 per-view
    eager calls (each with its own automatic batch depth and chunk and a fixed
    pair capacity, so neither side waits on the host)."""
    import torch

    import synth
    from paper_2410_04974_amd import Renderer
    from paper_2410_04974_amd.autotune import autotune

    w = synth.workload("c3")
    cams = w.cameras
    params = torch.from_numpy(synth.make_scene(w.scene)).to("cuda:0")
    px = sum(c.width * c.height for c in cams)
    tune = autotune(params, cams, use_cache=False)
    gen = torch.Generator(device="cuda:0").manual_seed(2)
    dls = [torch.randn((3, c.height, c.width), device="cuda:0", generator=gen) for c in cams]

    rb = Renderer(tile=tune["tile"], batch=tune["batch"], chunk=tune["chunk"])
    imgs = rb.forward(params, cams)
    torch.cuda.synchronize()
    pairs = rb.ctx.sizes()["pairs"]
    rb.configure(pair_capacity=int(pairs * 1.3) + 4096)
    grad = torch.empty_like(params)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            rb.forward(params, cams, out=imgs)
            rb.backward(params, dls, grad=grad)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rb.forward(params, cams, out=imgs)
        rb.backward(params, dls, grad=grad)
    for _ in range(args.warmup):
        g.replay()
    ms_batched = _timed(g.replay, args.steps)
    rb.ctx.check()

    # each per-view context picks its batch depth and chunk for its own (single view's) tile count
    per = [Renderer(tile=tune["tile"]) for _ in cams]
    gsum = torch.empty_like(params)

    def per_view():
        for r1, c, d in zip(per, cams, dls):
            r1.forward(params, [c])
            r1.backward(params, [d], grad=gsum)

    per_view()
    torch.cuda.synchronize()
    for r1 in per:  # fixed capacities, as in the batched graph: no host waits inside the timed calls
        r1.configure(pair_capacity=int(r1.ctx.sizes()["pairs"] * 1.3) + 4096)
    equal = all(torch.equal(per[k].forward(params, [c])[0], imgs[k]) for k, c in enumerate(cams))
    for _ in range(max(1, args.warmup // 2)):
        per_view()
    ms_per_view = _timed(per_view, max(1, args.steps // 4))
    out = {"metric": "fwd+bwd Mpixels/sec, 16 uneven views batched in one captured graph", "workload": "c3",
           "value": round(px / (ms_batched * 1e-3) / 1e6, 3), "unit": "Mpixels/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_batched, 4), "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "c3: 500k 6D Gaussians on a noisy sphere, 16 Fibonacci cameras cycling "
                                  "400x400, 800x800, 1280x720, 1600x900", "pixels": px, "pairs": pairs,
                      "tile": list(tune["tile"]), "batch": tune["batch"], "chunk": tune["chunk"]},
           "per_view_launches": {"ms_per_step": round(ms_per_view, 4),
                                 "value": round(px / (ms_per_view * 1e-3) / 1e6, 3)},
           "speedup_vs_per_view": round(ms_per_view / ms_batched, 3),
           "images_bitwise_equal": bool(equal), "autotune_ms": {k: round(v, 3) for k, v in tune["timings"].items()}}
    print(json.dumps(out), flush=True)


def bench_c4(args):
    """8-view training steps over a 64-camera 1920x1080 pool with Adam and
    densification statistics; one captured graph per camera group."""
    import torch

    import synth
    from paper_2410_04974_amd import Renderer, Trainer

    w = synth.workload("c4")
    pool = w.cameras
    pn = synth.make_scene(w.scene)
    tr_r = Renderer()
    pert = torch.from_numpy(synth.perturbed(pn)).to("cuda:0")
    targets = []
    for c in pool:
        targets.append(tr_r.forward(pert, [c])[0])
    del tr_r
    params = torch.from_numpy(pn).to("cuda:0")
    r = Renderer()
    tr = Trainer(params, r)
    dens = torch.zeros((2, pn.shape[1]), device="cuda:0")
    groups = len(pool) // 8
    # size the fixed pair capacity from one eager pass over every group
    pmax = 0
    for gi in range(groups):
        vs = synth.c4_step_views(gi)
        tr.step([pool[i] for i in vs], [targets[i] for i in vs], densify=dens)
        torch.cuda.synchronize()
        pmax = max(pmax, r.ctx.sizes()["pairs"])
    r.configure(pair_capacity=int(pmax * 1.3) + 4096)
    for gi in range(groups):
        vs = synth.c4_step_views(gi)
        tr.capture([pool[i] for i in vs], [targets[i] for i in vs], densify=dens, warmup=1, key=gi)
    torch.cuda.synchronize()
    steps = args.steps
    step = [0]

    def one():
        tr.replay(step[0] % groups)
        step[0] += 1

    ms = _timed(one, steps)
    r.ctx.check()
    px = sum(pool[i].width * pool[i].height for i in synth.c4_step_views(0))
    out = {"metric": "train steps/sec, 8 views per step at 1M 6D Gaussians 1920x1080", "workload": "c4",
           "value": round(1e3 / ms, 3), "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": groups,
           "ms_per_step": round(ms, 4), "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "mpixels_per_s": round(px / (ms * 1e-3) / 1e6, 3),
           "config": {"workload": "c4: 1M 6D Gaussians (70% sphere, 30% cube), 64-camera 1920x1080 pool, "
                                  "8 views per step, L1 + Adam + densification statistics",
                      "pairs_max": pmax},
           "final_loss": float(tr.loss), "densify_visible_max": float(dens[1].max())}
    print(json.dumps(out), flush=True)


def bench_render(args):
    """Forward-only renders (slice, projection, binning and sort, blending) of
    two 1408x1408 scenes, frames per second; the pair capacity is fixed from a
    first render, so a frame has no host waits."""
    import torch

    import synth
    from paper_2410_04974_amd import Renderer, build_cache

    res = {}
    for name in ("r1", "r2"):
        w = synth.workload(name)
        cam = w.cameras[0]
        params = torch.from_numpy(synth.make_scene(w.scene)).to("cuda:0")
        r = Renderer()
        img = [torch.empty((3, cam.height, cam.width), device="cuda:0")]
        r.forward(params, [cam], out=img)
        torch.cuda.synchronize()
        sizes = r.ctx.sizes()
        r.configure(pair_capacity=int(sizes["pairs"] * 1.5) + 4096)
        for _ in range(args.warmup):
            r.forward(params, [cam], out=img)
        ms = _timed(lambda: r.forward(params, [cam], out=img), args.steps)
        r.ctx.check()
        # the render-only path: the slice's direction-independent part read from
        # an inference cache built once, no state kept for a backward
        cache = build_cache(params)
        for _ in range(args.warmup):
            r.forward_cached(params, cache, [cam], out=img)
        ms_c = _timed(lambda: r.forward_cached(params, cache, [cam], out=img), args.steps)
        r.ctx.check()
        res[name] = {"fps": round(1e3 / ms, 2), "ms_per_frame": round(ms, 4),
                     "mpixels_per_s": round(cam.width * cam.height / (ms * 1e-3) / 1e6, 3),
                     "fps_cached": round(1e3 / ms_c, 2), "ms_per_frame_cached": round(ms_c, 4),
                     "gaussians": int(w.scene.n), "pairs": int(sizes["pairs"]), "description": w.description}
    out = {"metric": "forward render frames/sec at 1408x1408 (render only)", "workload": "render",
           "value": res["r2"]["fps"], "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["r2"]["ms_per_frame"], "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "vs_baseline": None, "config": {"workload": "r2: " + res["r2"]["description"]}, "scenes": res}
    print(json.dumps(out), flush=True)


def visited_block_pairs(ctx, cam):
    """(8x8 block, Gaussian) pairs the backward evaluates on one view: a
    Gaussian of the tile's list whose alpha >= 1/255 ellipse meets the block
    (the kernels' conservative test), at a list position before the block's
    last contributor.  64 lanes evaluate each such pair, so contributions over
    64 of these is the share of lanes doing work that counts."""
    import numpy as np
    from paper_2410_04974_amd import _lib

    s = ctx.settings
    tw, th = int(s.tile_w), int(s.tile_h)
    W, H = int(cam.width), int(cam.height)
    rec = ctx.export(_lib.EXPORT_RECORDS).astype(np.float64)
    vals = ctx.export(_lib.EXPORT_VALUES).astype(np.int64)
    rng = ctx.export(_lib.EXPORT_RANGES).astype(np.int64)
    last = ctx.export(_lib.EXPORT_LAST)[: W * H].reshape(H, W).astype(np.int64)
    ntx, nty = -(-W // tw), -(-H // th)
    T = ntx * nty
    n_t = rng[:T, 1] - rng[:T, 0]
    idx = np.concatenate([np.arange(a, b) for a, b in rng[:T]] + [np.zeros(0, np.int64)])
    t_of = np.repeat(np.arange(T), n_t)
    j_of = idx - np.repeat(rng[:T, 0], n_t)  # list position within the tile
    r = rec[vals[idx]]
    u, v, qa, qb, qc, al, ex, ey = (r[:, k] for k in range(8))
    lim = 2.0 * np.log(np.maximum(255.0 * al, 1e-30)) * 1.001 + 1e-3
    pad = np.zeros((nty * th, ntx * tw), np.int64)
    pad[:H, :W] = last
    total = 0
    for by in range(0, th, 8):
        for bx in range(0, tw, 8):
            blk = pad.reshape(nty, th, ntx, tw)[:, by:by + 8, :, bx:bx + 8].max(axis=(1, 3)).reshape(-1)
            x0 = (t_of % ntx) * tw + bx + 0.5
            y0 = (t_of // ntx) * th + by + 0.5
            box = (u + ex >= x0 - 1) & (u - ex <= x0 + 8) & (v + ey >= y0 - 1) & (v - ey <= y0 + 8)
            xl, yl = x0 - u, y0 - v
            xh, yh = xl + 7, yl + 7
            inx, iny = (xl <= 0) & (xh >= 0), (yl <= 0) & (yh >= 0)
            best = np.full(u.shape, np.inf)
            with np.errstate(divide="ignore", invalid="ignore"):
                dx = np.where(xl > 0, xl, xh)
                dy = np.clip(-qb * dx / qc, yl, yh)
                best = np.where(~inx, np.minimum(best, qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy), best)
                dy = np.where(yl > 0, yl, yh)
                dx = np.clip(-qb * dy / qa, xl, xh)
                best = np.where(~iny, np.minimum(best, qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy), best)
            hit = box & ((inx & iny) | (best <= lim))
            total += int(np.count_nonzero(hit & (j_of < blk[t_of])))
    return total


def Renderer_with_counts(r):
    from paper_2410_04974_amd import Renderer
    s = r.ctx.settings
    return Renderer(lambda_opa=s.lambda_opa, z_near=s.z_near, bg=tuple(s.bg), tile=(s.tile_w, s.tile_h),
                    batch=s.batch, flags=1)


def traffic(kernel, settings=None):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources with the same tile shape, batch depth
    and backward chunk; else null."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
        e = t.get(kernel)
        if not e or e.get("source_digest") != source_digest(e.get("sources", [])):
            return None
        if settings is not None and e.get("settings") != settings:
            return None
        return e.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(params_np, cam, npix):
    """The FP64 oracle (forward + analytic backward) on a seeded pixel sample."""
    import numpy as np

    import oracle
    import synth

    pix = synth.pixel_subset(cam.width, cam.height, npix, seed=5)
    dl = np.random.default_rng(6).normal(size=(len(pix), 3))
    t0 = time.perf_counter()
    oracle.render_plain(params_np, cam, pixels=pix)
    oracle.backward(params_np, cam, dl, pixels=pix)
    dt = time.perf_counter() - t0
    return {"value": round(len(pix) / dt / 1e6, 6), "unit": "Mpixels/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"{len(pix)} seeded pixels of the same 800x800 view, forward + backward, "
                      "brute force over all 300k Gaussians per pixel"}


if __name__ == "__main__":
    main()
