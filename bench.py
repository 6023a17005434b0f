"""Benchmark of the forest-of-octrees raycasting hot path on one MI355X.

Step = one full render of the adaptive workload: visibility/compaction,
segment generation (RK4 x 4 on trilinear fields) and sort-free compositing,
with all inputs resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-bwd] [--no-batch] [--no-shell]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray-segments/s + images/s at 1 GPU, % HBM roofline; fwd+bwd vs fwd time"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 instructions (and the FP64 vector
# peak): 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# MI355X's published FP32 vector peak, which counts packed FP32 (two lanes'
# worth per instruction); this build compiles without packed FP32 instructions
FP32_PUBLISHED_TFLOPS = 157.3

# Algorithmic cost per unit (the work the method must do, not what a kernel
# happens to issue):
#   trilinear segment: cubic restriction ~120, field values at the RK4 stage
#   points 16 x 2 fields x Horner 6 = 192, four RK4 steps ~160, combines 9
#   -> ~480 FP32 flop per segment; ray and slab predicate ~20 FP64 per candidate;
#   shell segment: Newton inversion at 16 stage points x 2-3 iterations x ~80
#   -> ~3500 FP64 flop per segment on top.
SEG_FLOPS_FP32 = 480
CAND_FLOPS_FP64 = 20
SHELL_SEG_FLOPS_FP64 = 3500
#   surface candidate: pixel ray ~12, two directions normal to the ray ~18,
#   eight projections ~40, the quadratic ~20 and per root the other parameter,
#   the point and its depth ~35 -> ~160 FP64 flop per candidate (plus ~30 FP32
#   and two transcendentals per hit for the surface model)
SURF_CAND_FLOPS_FP64 = 160
#   compositing: every leaf record read once (8 B; shell 2 x 16 B + 1 B) and
#   A, B, I written (12 B per pixel);  visibility: 13 B read per leaf and
#   about 20 B written per visible pair.
REC_BYTES = 8
SHELL_REC_BYTES = 33
PIX_BYTES = 12
#   constant-coefficient segment: per visible leaf its level and anchor (13 B),
#   kappa and eps (8 B), rectangle and candidate offset (16 B), read once.
ANALYTIC_LEAF_BYTES = 37

# HBM traffic of the kernels priced here, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (calibrated on a 256 MiB device copy: bytes = 2 FETCH_SIZE +
# WRITE_SIZE), summed over one step's launches of the kernel on the named
# workload, valid for the kernel sources whose SHA-256 is given.
_SEG_SRC = ("rc_segments.hip", "rc_internal.h")
_SEG_SHA = "95c8edce3a98347301bbfdb80034476fdd7e32ae8ac86566e27863749e32628e"
_COMP_SRC = ("rc_composite.hip", "rc_composite.h", "rc_internal.h")
_COMP_SHA = "4945f60540f3f8c2cf8e282264d362436b88e76e74ffbcd8ba014cd880d36acb"
MEASURED_TRAFFIC = {
    # keyed by (kernel, candidates of the workload): the 64 views, then the single 1024^2 view; valid for the
    # launch shapes and skipped levels of the measured run (the workload's entry in the tuning cache)
    ("k_segments_rk4<2, 4, 1>", 1331258581): {"bytes": 18745298354, "sources": _SEG_SRC, "sha256": _SEG_SHA,
                                              "tuning": {"seg_blocks": 32768}},
    ("composite", 1331258581): {"bytes": 25802320571, "sources": _COMP_SRC, "sha256": _COMP_SHA,
                                "tuning": {"fold_blocks": 16384, "root_blocks": 8192, "fold_skip": 12}},
    ("k_segments_rk4<2, 4, 1>", 14164540): {"bytes": 240264920, "sources": _SEG_SRC, "sha256": _SEG_SHA,
                                            "tuning": {"seg_blocks": 8192}},
    ("composite", 14164540): {"bytes": 381697767, "sources": _COMP_SRC, "sha256": _COMP_SHA,
                              "tuning": {"fold_blocks": 8192, "root_blocks": 8192, "fold_skip": 2}},
}
COPY_CALIB_BYTES = 256 << 20


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_region(torch, fn, steps):
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms


TUNING_CACHE = os.path.join(ROOT, "paper_1809_01334_amd", "tuning.json")


def torch_mod():
    import torch

    return torch


def tune(r, args, adjoint=False):
    """Launch shapes and skipped levels for the renderer (and with `adjoint`
    the leaf adjoint's workgroups): the autotuner's choice, kept per workload
    in the tuning cache (searched again with --retune); the images do not
    depend on them, the gradients by rounding only."""
    from paper_1809_01334_amd.tune import autotune

    if args.retune:
        # repetitions so that each timing covers about 5 ms
        r.forward()
        reps = int(min(50, max(3, math.ceil(5.0 / max(time_region(torch_mod(), r.forward, 3), 1e-3)))))
        res = autotune(r, reps=reps)
        if adjoint:
            from paper_1809_01334_amd.tune import autotune_adjoint

            g = torch_mod().ones(r.cams.npix, device=r.device)
            adj = autotune_adjoint(r, g, reps=reps)
            res["tuning"]["adj_blocks"] = adj["adj_blocks"]
            res["ms"]["adj_blocks"] = adj["ms"]
        cache = args.retune_out or TUNING_CACHE
        known = json.load(open(cache)) if os.path.exists(cache) else {}
        known[res["signature"]] = res
        if os.path.dirname(cache):
            os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1)
    else:
        res = autotune(r, reps=3, cache=TUNING_CACHE)
    log(f"[bench] tuning {res['tuning']}")
    return dict(res["tuning"])


def measured_traffic(kernel, r=None):
    """Calibrated HBM bytes of one step's launches of `kernel` on the renderer's
    workload, or None when none were taken for it or the kernel's sources changed
    since."""
    import hashlib

    key = (kernel, r.counts["ncand"] if r is not None else None)
    m = MEASURED_TRAFFIC.get(key)
    if m and any(int(getattr(r.tuning, k)) != v for k, v in m["tuning"].items()):
        return None  # taken with other launch shapes or skipped levels
    if not m or m["bytes"] is None:
        return None
    h = hashlib.sha256()
    for f in m["sources"]:
        with open(os.path.join(ROOT, "paper_1809_01334_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return m["bytes"] if h.hexdigest() == m["sha256"] else None


def copy_calibration(torch):
    """Three plain device copies of 256 MiB (read and written): the reference
    against which FETCH_SIZE and WRITE_SIZE are scaled to bytes."""
    src = torch.ones(COPY_CALIB_BYTES // 4, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 3 copies of {COPY_CALIB_BYTES} bytes")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(forest, fields, cams, method, substeps, every=4, frac=1 / 16, frac_one=1 / 512):
    """The FP64 oracle, as it stands, on a seeded pixel sample of the workload's
    views: every `every`-th view, `frac` of its pixels with all OpenMP threads,
    then `frac_one` of them on one thread.  Rate = oracle segments / wall time."""
    from oracle import oracle as O

    views = cams[::every]

    def run(fr, seed):
        rng = np.random.default_rng([1809, 1334, 4, seed])
        segs, npx = 0, 0
        t0 = time.perf_counter()
        for cam in views:
            n = max(1, int(cam.npix * fr))
            pix = np.sort(rng.choice(cam.npix, n, replace=False))
            segs += O.render(forest, fields, cam, method, substeps, pixels=pix)["segments"]
            npx += n
        return segs, npx, time.perf_counter() - t0

    nthreads = O.threads()
    segs, npx, dt = run(frac, 1)
    O.threads(1)
    segs1, npx1, dt1 = run(frac_one, 2)
    O.threads(nthreads)
    return {"value": segs / dt, "unit": "ray-segments/s", "cores": nthreads, "kind": "oracle",
            "sample": f"every {every}th of the {len(cams)} views ({len(views)} views), a seeded 1/{round(1 / frac)} "
                      f"of each view's pixels: {npx} pixels, {segs} segments, {dt:.1f} s on {nthreads} OpenMP "
                      f"threads (FP64)",
            "cpu_model": cpu_model(),
            "one_thread": {"value": segs1 / dt1, "unit": "ray-segments/s", "cores": 1,
                           "sample": f"the same views, 1/{round(1 / frac_one)} of each view's pixels: {npx1} "
                                     f"pixels, {segs1} segments, {dt1:.1f} s"}}


def render_launches(r):
    """Launches of k_render_level per rc_render call: one per non-empty level below the root, one root pass."""
    lb = r.index.level_begin()
    return 1 + sum(1 for l in range(1, r.index.maxlevel) if lb[l + 1] > lb[l])


def seg_roofline(r, S, C, t_seg, kernel="k_segments_rk4<2, 4, 1>"):
    """The segment kernel (one launch per rc_segments call) against the FP32 vector peak."""
    flops = SEG_FLOPS_FP32 * S + CAND_FLOPS_FP64 * C
    achieved = flops / (t_seg * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP32_PUBLISHED_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PUBLISHED_TFLOPS, "traffic": measured_traffic(kernel, r),
            "kernel": kernel, "launches_per_step": 1, "flop_per_launch": flops, "avg_launch_ms": t_seg,
            "per_unit": f"{SEG_FLOPS_FP32} FP32/segment + {CAND_FLOPS_FP64} FP64/candidate",
            "peak_unpacked": FP32_PEAK_TFLOPS, "frac_unpacked": achieved / FP32_PEAK_TFLOPS}


def composite_roofline(r, C, t_comp):
    """rc_composite against HBM: every leaf record read once and A, B, I written (the node records of the
    coarsening are traffic, not algorithmic bytes)."""
    nbytes = C * REC_BYTES + r.cams.npix * PIX_BYTES
    traffic = measured_traffic("composite", r)
    return {"bound": "hbm", "algorithmic_bytes": nbytes, "achieved_GBs": nbytes / (t_comp * 1e-3) / 1e9,
            "frac": nbytes / (t_comp * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_GBs": traffic / (t_comp * 1e-3) / 1e9 if traffic else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--only", choices=("headline", "single", "config1", "shell"), default=None,
                    help="time only this workload (for profiling runs)")
    ap.add_argument("--no-plain", action="store_true", help="skip the 64 plain per-view forwards")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-shell", action="store_true")
    ap.add_argument("--no-integrators", action="store_true")
    ap.add_argument("--no-shares", action="store_true")
    ap.add_argument("--no-surface", action="store_true")
    ap.add_argument("--no-surface-ho", action="store_true")
    ap.add_argument("--no-volume", action="store_true")
    ap.add_argument("--no-channels", action="store_true")
    ap.add_argument("--no-analytic", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="end with plain 256 MiB device copies, the reference for HBM byte counters")
    ap.add_argument("--retune", action="store_true",
                    help="search the launch shapes and skipped levels of the headline and single-view workloads again "
                         "and store them in the tuning cache (default: take them from the cache)")
    ap.add_argument("--retune-out", default=None, metavar="PATH",
                    help="with --retune, write the choices to this JSON file instead of the package's tuning cache")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the forest share of one "
              f"process is rendered on one GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1809_01334_amd as P
    import synth

    log("[bench] generating the adaptive forest (levels 4-9)")
    scene = synth.config_scene(2)
    r1 = None
    out = None
    if args.only in (None, "headline"):
        out = bench_headline(torch, P, synth, scene, args)
        r1 = out.pop("_renderer")
    if args.only in (None, "single"):
        single = bench_single(torch, P, synth, scene, args, index=r1.index if r1 else None)
        r1 = single.pop("_renderer")
        if out is None:
            out = single
        else:
            out["single_view_workload"] = single
    if args.only in (None, "config1"):
        c1 = bench_config1(torch, P, synth, args.steps)
        if out is None:
            out = c1
        else:
            out["config1_workload"] = c1
    if args.only == "shell":
        out = bench_shell(torch, P, synth, max(args.steps // 5, 3))
    if args.only is not None:
        if args.copy_calib:
            copy_calibration(torch)
        print(json.dumps(out), flush=True)
        return

    sv = out["single_view_workload"]
    if not args.no_bwd:
        r = r1
        g = torch.ones(r.cams.npix, device="cuda:0")
        r.capture(backward=True, dLdI=g)
        for _ in range(2):
            r.replay()
        ms_fb = time_region(torch, r.replay, max(args.steps // 2, 5))
        sv["fwd_bwd_ms"] = ms_fb
        sv["fwd_bwd_over_fwd"] = ms_fb / sv["ms_per_step"]
        log(f"[bench] single view forward+backward {ms_fb:.3f} ms (graph)")
        r.capture()
        out["adjoint_workload"] = bench_adjoint(torch, P, synth, max(args.steps // 2, 5))
    if not args.no_integrators:
        out["integrators"] = bench_integrators(torch, P, r1, max(args.steps // 5, 3))
    if not args.no_channels:
        out["channels"] = bench_channels(torch, P, synth, scene, r1, max(args.steps // 5, 3))
    if not args.no_analytic:
        out["analytic_workload"] = bench_analytic(torch, P, synth, scene, r1, max(args.steps // 5, 3))
    if not args.no_batch:
        out["small_views"] = bench_small_views(torch, P, synth, r1, max(args.steps // 5, 3))
    if not args.no_shell:
        out["shell_workload"] = bench_shell(torch, P, synth, max(args.steps // 5, 3))
    if not args.no_surface:
        out["surface_workload"] = bench_surface(torch, P, synth, max(args.steps // 5, 3))
    if not args.no_surface_ho:
        out["surface_ho_workload"] = bench_surface_ho(torch, P, synth, max(args.steps // 5, 3))
    if not args.no_volume:
        out["volume_workload"] = bench_volume(torch, P, synth, max(args.steps // 5, 3))
    if not args.no_shares:
        out["shares"] = bench_shares(torch, P, synth, scene, r1, max(args.steps // 5, 3))

    if args.copy_calib:
        copy_calibration(torch)
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a sample of the headline workload")
        out["cpu_baseline"] = cpu_baseline(scene.forest, scene.fields, synth.config4_cameras(), "rk4", 4)
        log(f"[bench] CPU oracle: {out['cpu_baseline']['value']:.3e} ray-segments/s on "
            f"{out['cpu_baseline']['cores']} threads")
    print(json.dumps(out), flush=True)


def bench_headline(torch, P, synth, scene, args):
    """The forest of the adaptive workload seen by 64 cameras of uneven resolution
    ({256, 512, 1024, 2048}^2), its forward (prune, segments, composite) captured in
    one HIP graph: the largest single-GPU workload by segments per step."""
    cams = synth.config4_cameras()
    npix = int(sum(c.npix for c in cams))
    log(f"[bench] headline: {scene.forest.nleaves} leaves, {len(cams)} cameras, {npix} pixels")
    r = P.Renderer(scene.forest, scene.fields, cams, "rk4", 4, device="cuda:0")
    counts = r.counts
    S = r.count_segments()
    C = counts["ncand"]
    log(f"[bench] visible pairs {counts['nvis']}, candidates {C}, segments {S}, node records {counts['nrec']}")
    tuning = tune(r, args)
    for _ in range(args.warmup):
        r.forward()
    ms_eager = time_region(torch, r.forward, args.steps)
    r.capture()
    for _ in range(args.warmup):
        r.replay()
    ms = time_region(torch, r.replay, args.steps)
    t_prune = time_region(torch, r.prune, args.steps)
    t_seg = time_region(torch, r.segments, args.steps)
    t_comp = time_region(torch, r.composite, args.steps)
    t_render = time_region(torch, r.render_step, args.steps)
    log(f"[bench] headline: one graph {ms:.3f} ms (eager {ms_eager:.3f}); prune {t_prune:.3f}, segments "
        f"{t_seg:.3f}, composite {t_comp:.3f} ms; rc_render (fused) {t_render:.3f} ms")
    res = {}
    for c in cams:
        res[str(c.w)] = res.get(str(c.w), 0) + 1
    out = {
        "metric": METRIC,
        "value": S / (ms * 1e-3),
        "unit": "ray-segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"adaptive octree levels 4-9 refined at 0.2 crossings of 8 Gaussians "
                        f"({scene.forest.nleaves} leaves), trilinear kappa/eps, RK4 x 4 substeps, seen by "
                        f"{len(cams)} perspective cameras of uneven resolution in one HIP graph",
            "views": len(cams), "resolutions": res, "leaves": scene.forest.nleaves, "visible": counts["nvis"],
            "candidates": C, "segments": S, "node_records": counts["nrec"], "pixels": npix,
            "tuning": tuning,
        },
        "images_per_s": len(cams) / (ms * 1e-3),
        "forward_eager_ms": ms_eager,
        "phase_ms": {"prune": t_prune, "segments": t_seg, "composite": t_comp},
        "fused_render_ms": t_render,
        "roofline": seg_roofline(r, S, C, t_seg),
    }
    pb = scene.forest.nleaves * len(cams) * 13 + counts["nvis"] * 20
    out["phase_roofline"] = {"composite": composite_roofline(r, C, t_comp),
                             "prune": {"bound": "hbm", "algorithmic_bytes": pb,
                                       "achieved_GBs": pb / (t_prune * 1e-3) / 1e9,
                                       "frac": pb / (t_prune * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    if not args.no_plain:
        singles = [P.Renderer(r.forest, r.fields, [c], "rk4", 4, device="cuda:0", index=r.index) for c in cams]

        def plain():
            for x in singles:
                x.forward()

        plain()
        t_plain = time_region(torch, plain, max(args.steps // 5, 3))
        log(f"[bench] 64 plain per-view forwards {t_plain:.2f} ms")
        out["plain_sum_ms"] = t_plain
        out["plain_over_batched"] = t_plain / ms
        del singles
        torch.cuda.empty_cache()
    out["_renderer"] = None
    del r
    torch.cuda.empty_cache()
    return out


def bench_single(torch, P, synth, scene, args, index=None):
    """One 1024^2 perspective view of the adaptive forest (the single-view workload)."""
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, "rk4", 4, device="cuda:0", index=index)
    counts = r.counts
    S = r.count_segments()
    C = counts["ncand"]
    log(f"[bench] single view: visible {counts['nvis']}, candidates {C}, segments {S}, node records {counts['nrec']}")
    tuning = tune(r, args, adjoint=True)
    for _ in range(args.warmup):
        r.forward()
    ms_eager = time_region(torch, r.forward, args.steps)
    r.capture()
    for _ in range(args.warmup):
        r.replay()
    ms = time_region(torch, r.replay, args.steps)
    t_prune = time_region(torch, r.prune, args.steps)
    t_seg = time_region(torch, r.segments, args.steps)
    t_comp = time_region(torch, r.composite, args.steps)
    t_render = time_region(torch, r.render_step, args.steps)
    log(f"[bench] single view: one graph {ms:.3f} ms; prune {t_prune:.3f}, segments {t_seg:.3f}, composite "
        f"{t_comp:.3f} ms; rc_render (fused) {t_render:.3f} ms")
    out = {"workload": f"the adaptive forest ({scene.forest.nleaves} leaves), one 1024x1024 perspective view, "
                       f"trilinear kappa/eps, RK4 x 4",
           "leaves": scene.forest.nleaves, "visible": counts["nvis"], "candidates": C, "segments": S,
           "node_records": counts["nrec"], "tuning": tuning, "pixels": r.cams.npix, "ms_per_step": ms,
           "forward_eager_ms": ms_eager,
           "ray_segments_per_s": S / (ms * 1e-3), "images_per_s": 1e3 / ms,
           "phase_ms": {"prune": t_prune, "segments": t_seg, "composite": t_comp},
           "fused_render_ms": t_render,
           "roofline": seg_roofline(r, S, C, t_seg)}
    pb = scene.forest.nleaves * 13 + counts["nvis"] * 20
    out["phase_roofline"] = {"composite": composite_roofline(r, C, t_comp),
                             "prune": {"bound": "hbm", "algorithmic_bytes": pb,
                                       "achieved_GBs": pb / (t_prune * 1e-3) / 1e9,
                                       "frac": pb / (t_prune * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    out["_renderer"] = r
    return out


def bench_config1(torch, P, synth, steps):
    """Uniform level-3 cube (512 leaves), constant coefficients, 64x64 orthographic view, closed form: a
    latency-scale case (a few microseconds of work per launch)."""
    sc = synth.config_scene(1)
    r = P.Renderer(sc.forest, sc.fields, sc.cameras, "analytic", 1, device="cuda:0")
    S = r.count_segments()
    r.forward()
    r.capture()
    r.replay()
    ms = time_region(torch, r.replay, max(steps, 20))
    log(f"[bench] config 1: {S} segments, one graph {ms:.4f} ms")
    return {"workload": "uniform level-3 unit cube (512 leaves), per-leaf constants, 64x64 orthographic view, "
                        "closed form", "segments": S, "ms_per_step": ms, "ray_segments_per_s": S / (ms * 1e-3),
            "images_per_s": 1e3 / ms}


def bench_adjoint(torch, P, synth, steps):
    """512^2 view, background 0.5: forward vs forward + adjoint of L = sum (I - I*)^2."""
    log("[bench] adjoint workload: generating")
    sc = synth.config_scene(5)
    r = P.Renderer(sc.forest, sc.fields, sc.cameras, "rk4", 4, device="cuda:0")
    tgt = P.Renderer(r.forest, P.DeviceFields.from_synth(sc.extra["target_fields"], r.device), sc.cameras, "rk4", 4,
                     device="cuda:0", index=r.index)
    _, _, It = tgt.forward()
    It = It.clone()
    g = torch.empty_like(It)

    def fwd():
        r.forward()

    def fwd_bwd():
        _, _, I = r.forward()
        torch.mul(torch.sub(I, It), 2.0, out=g)
        r.backward(g, r.g_dk, r.g_de)

    r.g_dk = torch.empty_like(r.fields.kappa)
    r.g_de = torch.empty_like(r.fields.eps)
    for _ in range(3):
        fwd_bwd()
    t_f = time_region(torch, fwd, steps)
    t_fb = time_region(torch, fwd_bwd, steps)
    S = r.count_segments()
    log(f"[bench] adjoint workload: {sc.forest.nleaves} leaves, {S} segments, fwd {t_f:.3f} ms, fwd+bwd {t_fb:.3f} ms")
    return {"workload": f"{sc.forest.nleaves}-leaf adaptive forest, 512x512, background 0.5, "
                        f"loss sum (I - I_target)^2 with perturbed target fields",
            "segments": S, "fwd_ms": t_f, "fwd_bwd_ms": t_fb, "fwd_bwd_over_fwd": t_fb / t_f}


def bench_small_views(torch, P, synth, r, steps):
    """64 views of 128^2 of the same forest, where per-view launches weigh most:
    one graph for all views versus 64 plain per-view forwards."""
    rng = np.random.default_rng([1809, 1334, 128])
    small = [synth.random_perspective_camera(rng, 128, 128) for _ in range(64)]
    rs = P.Renderer(r.forest, r.fields, small, "rk4", 4, device="cuda:0", index=r.index)
    rs.capture()
    rs.replay()
    t_small = time_region(torch, rs.replay, steps)
    singles = [P.Renderer(r.forest, r.fields, [c], "rk4", 4, device="cuda:0", index=r.index) for c in small]

    def plain_small():
        for x in singles:
            x.forward()

    plain_small()
    t_small_plain = time_region(torch, plain_small, steps)
    log(f"[bench] 64 views of 128^2: one graph {t_small:.3f} ms, 64 plain forwards {t_small_plain:.3f} ms")
    del singles, rs
    torch.cuda.empty_cache()
    return {"views": 64, "resolution": 128, "batched_ms": t_small, "plain_sum_ms": t_small_plain,
            "plain_over_batched": t_small_plain / t_small}


def bench_integrators(torch, P, r, steps):
    """Segment phase and adjoint of the adaptive workload with each integrator
    (Sec. 2.7): RK4, implicit Gauss and Simpson over 4 pieces, and RK4 and Gauss
    with the recursion."""
    out = {}
    for name, method, sub, c_rk in (("rk4_x4", "rk4", 4, 0.0), ("gauss2_x4", "gauss2", 4, 0.0),
                                    ("simpson_x4", "simpson", 4, 0.0), ("rk4_adaptive_c0.5", "rk4", 1, 0.5),
                                    ("gauss2_adaptive_c0.5", "gauss2", 1, 0.5)):
        ri = P.Renderer(r.forest, r.fields, r.cams.raw, method, sub, device="cuda:0", index=r.index, c_rk=c_rk)
        ri.segments()
        t = time_region(torch, ri.segments, steps)
        # the adjoint of the same integrator (its pieces recomputed), after a forward
        ri.forward()
        g = torch.ones(ri.cams.npix, device="cuda:0")
        ri.backward(g)
        t_bwd = time_region(torch, lambda: ri.backward(g), steps)
        out[name] = {"segments_ms": t, "backward_ms": t_bwd}
        log(f"[bench] integrator {name}: segments phase {t:.3f} ms, adjoint {t_bwd:.3f} ms")
        del ri
    return out


def bench_shell(torch, P, synth, steps):
    """Six-tree cubed-sphere shell, levels 3-7, trilinear fields, 2048x2048 view:
    curved pairing (planes and spheres, up to two intervals), RK4 x 4 with FP64
    Newton field points, depth-merging fold."""
    log("[bench] shell workload: generating")
    sc = synth.config_scene(3)
    r = P.Renderer(sc.forest, sc.fields, sc.cameras, "rk4", 4, device="cuda:0")
    c = r.counts
    S = r.count_segments()
    log(f"[bench] shell: {sc.forest.nleaves} leaves, visible {c['nvis']}, candidates {c['ncand']}, segments {S}, "
        f"node records {c['nrec']}")
    for _ in range(2):
        r.forward()
    ms_eager = time_region(torch, r.forward, steps)
    r.capture()
    r.replay()
    ms = time_region(torch, r.replay, steps)
    t_prune = time_region(torch, r.prune, steps)
    t_seg = time_region(torch, r.segments, steps)
    t_comp = time_region(torch, r.composite, steps)
    log(f"[bench] shell: forward {ms:.2f} ms (graph), {ms_eager:.2f} ms (eager); prune {t_prune:.2f}, "
        f"segments {t_seg:.2f}, composite {t_comp:.2f} ms")
    out = {"workload": f"6-tree cubed-sphere shell r in [0.55, 1], levels 3-7 ({sc.forest.nleaves} leaves), "
                       f"trilinear kappa/eps, 2048x2048 perspective view, RK4 x 4, FP64 Newton field points",
           "leaves": sc.forest.nleaves, "visible": c["nvis"], "candidates": c["ncand"], "segments": S,
           "node_records": c["nrec"], "ms_per_step": ms, "forward_eager_ms": ms_eager,
           "ray_segments_per_s": S / (ms * 1e-3), "images_per_s": 1e3 / ms,
           "phase_ms": {"prune": t_prune, "segments": t_seg, "composite": t_comp}}
    flops = (SEG_FLOPS_FP32 + SHELL_SEG_FLOPS_FP64) * S + CAND_FLOPS_FP64 * c["ncand"]
    ach = flops / (t_seg * 1e-3) / 1e12
    out["roofline"] = {"bound": "alu", "kernel": "k_segments_shell<4>", "achieved": ach, "peak": FP32_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS, "flop_per_launch": flops,
                       "per_unit": f"{SEG_FLOPS_FP32} FP32 + {SHELL_SEG_FLOPS_FP64} FP64 per segment, "
                                   f"{CAND_FLOPS_FP64} FP64 per candidate"}
    cb = c["ncand"] * SHELL_REC_BYTES + r.cams.npix * PIX_BYTES
    out["composite"] = {"bound": "hbm", "algorithmic_bytes": cb, "achieved_GBs": cb / (t_comp * 1e-3) / 1e9,
                        "frac": cb / (t_comp * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del r
    torch.cuda.empty_cache()
    return out


def bench_channels(torch, P, synth, scene, r, steps):
    """The headline view with three channels (RGB-like: the fields scaled per
    channel): one pairing feeds all three integrations."""
    f = scene.fields
    rgb = synth.stack_channels([synth.Fields(f.kind, (f.kappa * s).astype(np.float32), (f.eps * t).astype(np.float32))
                                for s, t in ((1.0, 1.0), (0.7, 1.3), (1.4, 0.6))])
    r3 = P.Renderer(scene.forest, rgb, r.cams.raw, "rk4", 4, device="cuda:0", index=r.index)
    r3.forward()
    r3.capture()
    r3.replay()
    ms = time_region(torch, r3.replay, steps)
    t_seg = time_region(torch, r3.segments, steps)
    t_seg1 = time_region(torch, r.segments, steps)
    log(f"[bench] 3 channels: forward {ms:.3f} ms, segments {t_seg:.3f} ms (one channel {t_seg1:.3f} ms)")
    del r3
    torch.cuda.empty_cache()
    return {"channels": 3, "ms_per_step": ms, "segments_ms": t_seg, "segments_one_channel_ms": t_seg1,
            "segments_ratio_to_one_channel": t_seg / t_seg1}


def bench_analytic(torch, P, synth, scene, r, steps):
    """The headline forest and view with one (kappa, eps) per leaf, each leaf's
    corner mean, in closed form (eq. ABconstant): the same visibility and
    pairing, and segment generation priced against HBM."""
    sc = synth.constant_variant(scene)
    ra = P.Renderer(sc.forest, sc.fields, r.cams.raw, "analytic", 1, device="cuda:0", index=r.index)
    c = ra.counts
    S = ra.count_segments()
    ra.forward()
    ra.capture()
    ra.replay()
    ms = time_region(torch, ra.replay, steps)
    t_render = time_region(torch, ra.render_step, steps)
    t_seg = time_region(torch, ra.segments, steps)
    nbytes = c["nvis"] * ANALYTIC_LEAF_BYTES + c["ncand"] * REC_BYTES
    gbs = nbytes / (t_seg * 1e-3) / 1e9
    log(f"[bench] constant coefficients: forward {ms:.3f} ms, segments {t_seg:.3f} ms ({gbs:.0f} GB/s "
        f"algorithmic); rc_render (fused) {t_render:.3f} ms")
    kernel = "k_segments_analytic<1>"
    traffic = measured_traffic(kernel, ra)
    del ra
    torch.cuda.empty_cache()
    return {"workload": "the single-view forest and view, one (kappa, eps) per leaf (corner means), closed form",
            "segments": S, "ms_per_step": ms, "ray_segments_per_s": S / (ms * 1e-3), "segments_ms": t_seg,
            "fused_render_ms": t_render,
            "roofline": {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_launch": nbytes,
                         "per_unit": f"{ANALYTIC_LEAF_BYTES} B per visible leaf + {REC_BYTES} B per candidate"}}


def bench_surface(torch, P, synth, steps):
    """Mandelbrot surface (Sec. 4.1): two quadtrees on the hexagon, levels 4-11
    refined where corner iteration counts differ; the two image instances
    (opaque grey-to-white, transparent near-maximum highlight) at 1024^2, each
    its own camera and transfer function."""
    log("[bench] surface workload: generating")
    f, val = synth.mandelbrot_forest(4, 11)
    cams = synth.hexagon_cameras(1024, 1024)
    out = {"workload": f"Mandelbrot surface on the hexagon, two quadtrees, levels 4-11 ({f.nleaves} leaves), "
                       f"two 1024x1024 instances (opaque / transparent transfer)", "leaves": f.nleaves,
           "instances": []}
    index = None
    for inst in (0, 1):
        r = P.Renderer(f, synth.mandelbrot_fields(val, inst), [cams[inst]], "analytic", 1, device="cuda:0",
                       index=index)
        index = r.index
        c = r.counts
        hit, _ = r.debug_segments(intervals=False)
        H = int(hit[:c["ncand"]].to(torch.int64).sum().item())
        r.forward()
        r.capture()
        r.replay()
        ms = time_region(torch, r.replay, steps)
        t_prune = time_region(torch, r.prune, steps)
        t_seg = time_region(torch, r.segments, steps)
        t_comp = time_region(torch, r.composite, steps)
        flops = SURF_CAND_FLOPS_FP64 * c["ncand"]
        ach = flops / (t_seg * 1e-3) / 1e12
        log(f"[bench] surface instance {inst}: visible {c['nvis']}, candidates {c['ncand']}, hits {H}; forward "
            f"{ms:.3f} ms; prune {t_prune:.3f}, segments {t_seg:.3f}, composite {t_comp:.3f} ms")
        out["instances"].append({
            "visible": c["nvis"], "candidates": c["ncand"], "hits": H, "ms_per_step": ms,
            "hits_per_s": H / (ms * 1e-3), "images_per_s": 1e3 / ms,
            "phase_ms": {"prune": t_prune, "segments": t_seg, "composite": t_comp},
            "roofline": {"bound": "alu", "kernel": "k_segments_surface", "achieved": ach,
                         "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                         "per_unit": f"{SURF_CAND_FLOPS_FP64} FP64 per candidate"}})
        del r
    torch.cuda.empty_cache()
    return out


def bench_surface_ho(torch, P, synth, steps):
    """Degree-2 surface: the hexagon lifted to z = 0.35 sin(2x) cos(1.5y) and
    interpolated on the Gauss-Lobatto grid of each tree, carrying the
    Mandelbrot refinement (levels 4-11) and the transparent transfer, 1024^2."""
    log("[bench] degree-2 surface workload: generating")
    base, val = synth.mandelbrot_forest(4, 11)
    trees = synth.ho_hexagon_trees(2, lambda x, y: 0.35 * np.sin(2 * x) * np.cos(1.5 * y))
    f = synth.ho_surface_forest(trees, 2, base.level, base.x, base.y, base.tree_of_leaf())
    cam = synth.hexagon_cameras(1024, 1024)[0]
    r = P.Renderer(f, synth.mandelbrot_fields(val, 1), [cam], "analytic", 1, device="cuda:0")
    c = r.counts
    hit, _ = r.debug_segments(intervals=False)
    H = int(hit[:c["ncand"]].to(torch.int64).sum().item())
    r.forward()
    r.capture()
    r.replay()
    ms = time_region(torch, r.replay, steps)
    t_prune = time_region(torch, r.prune, steps)
    t_seg = time_region(torch, r.segments, steps)
    t_comp = time_region(torch, r.composite, steps)
    log(f"[bench] degree-2 surface: visible {c['nvis']}, candidates {c['ncand']}, hits {H}; forward {ms:.3f} ms; "
        f"prune {t_prune:.3f}, segments {t_seg:.3f}, composite {t_comp:.3f} ms")
    del r
    torch.cuda.empty_cache()
    return {"workload": f"degree-2 lifted hexagon, Mandelbrot refinement levels 4-11 ({f.nleaves} leaves), "
                        f"1024x1024, transparent transfer", "leaves": f.nleaves, "visible": c["nvis"],
            "candidates": c["ncand"], "hits": H, "ms_per_step": ms, "hits_per_s": H / (ms * 1e-3),
            "phase_ms": {"prune": t_prune, "segments": t_seg, "composite": t_comp}}


def bench_volume(torch, P, synth, steps):
    """Degree-2 volume trees (curved elements): an adaptive forest of levels
    2-6 refined around Gaussians on one curved tree, trilinear fields, RK4 x 4,
    one 512x512 perspective view."""
    log("[bench] degree-2 volume workload: generating")
    sc = synth.volume_scene(7, R=2, lmin=2, lmax=6, w=512, h=512, amp=0.08)
    r = P.Renderer(sc.forest, sc.fields, sc.cameras, "rk4", 4, device="cuda:0")
    c = r.counts
    r.forward()
    hit, _ = r.debug_segments()
    S = int(hit[:c["ncand"]].to(torch.int64).sum().item())
    r.forward()
    r.capture()
    r.replay()
    ms = time_region(torch, r.replay, steps)
    t_prune = time_region(torch, r.prune, steps)
    t_seg = time_region(torch, r.segments, steps)
    t_comp = time_region(torch, r.composite, steps)
    log(f"[bench] degree-2 volume: {sc.forest.nleaves} leaves, visible {c['nvis']}, candidates {c['ncand']}, "
        f"intervals {S}; forward {ms:.3f} ms; prune {t_prune:.3f}, segments {t_seg:.3f}, composite {t_comp:.3f} ms")
    del r
    torch.cuda.empty_cache()
    return {"workload": f"degree-2 volume tree (curved elements), adaptive levels 2-6 ({sc.forest.nleaves} leaves), "
                        f"trilinear kappa/eps, RK4 x 4, 512x512", "leaves": sc.forest.nleaves, "visible": c["nvis"],
            "candidates": c["ncand"], "intervals": S, "ms_per_step": ms, "ray_segments_per_s": S / (ms * 1e-3),
            "phase_ms": {"prune": t_prune, "segments": t_seg, "composite": t_comp}}


def bench_shares(torch, P, synth, scene, r, steps, nshares=8):
    """The headline workload cut into equal curve-order leaf ranges, one per
    process share (Sec. 3.3): each share's per-pixel lists of its maximal
    complete subtrees, then the merge of all lists into the image (Sec. 3.5)."""
    N = scene.forest.nleaves
    cuts = [N * k // nshares for k in range(1, nshares)]
    shares = []
    for f, fl in synth.split_shares(scene.forest, scene.fields, cuts):
        rs = P.Renderer(f, fl, r.cams.raw, "rk4", 4, device="cuda:0")
        rs.forward_lists()
        shares.append(rs)
    lists = [(rs.list_offset, rs.entries) for rs in shares]
    npix = r.cams.npix
    A, B, I = (torch.empty(npix, device="cuda:0") for _ in range(3))
    ov = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    P.rc_merge_lists(r.cams, lists, A, B, I, ov)
    torch.cuda.synchronize()
    n_ent = [int(rs.n_entries.item()) for rs in shares]
    diff = float((I - r.I).abs().max().item())
    t_lists = [time_region(torch, rs.lists_step, steps) for rs in shares]
    t_fwd = [time_region(torch, rs.forward_lists_enqueue, steps) for rs in shares]
    t_merge = time_region(torch, lambda: P.rc_merge_lists(r.cams, lists, A, B, I, None), steps)

    def step():
        for rs in shares:
            rs.forward_lists_enqueue()
        P.rc_merge_lists(r.cams, lists, A, B, I, None)

    # the whole share pipeline (every share's prune, segments and lists, then the merge) as one HIP graph
    cur = torch.cuda.current_stream()
    s = torch.cuda.Stream()
    s.wait_stream(cur)
    with torch.cuda.stream(s):
        for _ in range(2):
            step()
    cur.wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    g.replay()
    t_graph = time_region(torch, g.replay, steps)
    diff_graph = float((I - r.I).abs().max().item())
    E = sum(n_ent)
    # lists: every leaf record read (8 B), every entry written (16 B), one offset per pixel
    lb = sum(rs.counts["ncand"] for rs in shares) * REC_BYTES + E * 16 + nshares * (npix + 1) * 8
    # merge: every entry read, every list's offsets read, A, B, I written
    mb = E * 16 + nshares * (npix + 1) * 8 + npix * PIX_BYTES
    log(f"[bench] {nshares} shares: {E} entries, overlaps {int(ov.item())}, max |I - I_full| {diff:.2e}; "
        f"lists {sum(t_lists):.3f} ms, share forwards {sum(t_fwd):.3f} ms, merge {t_merge:.3f} ms; "
        f"all shares + merge in one graph {t_graph:.3f} ms (max |I - I_full| {diff_graph:.2e})")
    return {"workload": f"headline workload cut into {nshares} equal curve-order leaf ranges",
            "shares": nshares, "entries": E, "entries_per_share": n_ent, "overlaps": int(ov.item()),
            "max_abs_diff_vs_full_render": diff,
            "lists_ms": t_lists, "share_forward_ms": t_fwd, "merge_ms": t_merge, "pipeline_graph_ms": t_graph,
            "pipeline_graph_max_abs_diff": diff_graph,
            "lists": {"bound": "hbm", "algorithmic_bytes": lb, "achieved_GBs": lb / (sum(t_lists) * 1e-3) / 1e9,
                      "frac": lb / (sum(t_lists) * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "merge": {"bound": "hbm", "algorithmic_bytes": mb, "achieved_GBs": mb / (t_merge * 1e-3) / 1e9,
                      "frac": mb / (t_merge * 1e-3) / 1e9 / HBM_PEAK_GBS}}


if __name__ == "__main__":
    main()
