"""Benchmark of the forest-of-octrees raycasting hot path on one MI355X.

Step = one full render of the adaptive workload: visibility/compaction,
segment generation (RK4 x 4 on trilinear fields) and sort-free compositing,
with all inputs resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-bwd] [--no-batch] [--no-shell]
"""

from __future__ import annotations

import argparse
import json
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

# HBM traffic per launch of the kernels priced here (per call for the
# composite), from rocprofv3 FETCH_SIZE and WRITE_SIZE (calibrated on a
# 256 MiB device copy: x2.0 and x1.0), valid for the kernel sources whose
# SHA-256 is given.
MEASURED_TRAFFIC = {
    "k_segments_rk4<2, 4, 1>": {"bytes": 240462056, "sources": ("rc_segments.hip", "rc_internal.h"),
                             "sha256": "40869d34fe93ba4e3ee438249da176c63ce982bd3eaab3cf59d5429d6ec8ef3c"},
    "k_segments_analytic<1>": {"bytes": 181928926, "sources": ("rc_segments.hip", "rc_internal.h"),
                               "sha256": "40869d34fe93ba4e3ee438249da176c63ce982bd3eaab3cf59d5429d6ec8ef3c"},
    # per forward of the headline view: every fold launch of one rc_composite call
    "composite": {"bytes": 404472661, "sources": ("rc_composite.hip", "rc_composite.h", "rc_internal.h"),
                  "sha256": "2def90bce3a0d1cd4a8773ad5a878d086aae9cfd8215ea884d4bba65427180b2"},
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


def measured_traffic(kernel):
    """Calibrated HBM bytes per launch, or None when the kernel's sources
    changed since the counters were taken."""
    import hashlib

    m = MEASURED_TRAFFIC.get(kernel)
    if not m or m["bytes"] is None:
        return None
    h = hashlib.sha256()
    for f in m["sources"]:
        with open(os.path.join(ROOT, "paper_1809_01334_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return m["bytes"] if h.hexdigest() == m["sha256"] else None


def cpu_baseline(scene, reps=4):
    """The FP64 oracle rendering the workload's full view `reps` times on the host cores."""
    from oracle import oracle as O

    cam = scene.cameras[0]
    t0 = time.perf_counter()
    for _ in range(reps):
        r = O.render(scene.forest, scene.fields, cam, scene.method, scene.substeps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": reps * r["segments"] / dt, "unit": "ray-segments/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} renders of the full {cam.w}x{cam.h} view of the workload ({r['segments']} segments "
                      f"each, FP64, {dt:.1f} s in total)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--res", type=int, default=1024)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-shell", action="store_true")
    ap.add_argument("--no-integrators", action="store_true")
    ap.add_argument("--no-shares", action="store_true")
    ap.add_argument("--no-surface", action="store_true")
    ap.add_argument("--no-surface-ho", action="store_true")
    ap.add_argument("--no-channels", action="store_true")
    ap.add_argument("--no-analytic", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="end with plain 256 MiB device copies, the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the forest share of one "
              f"process is rendered on one GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1809_01334_amd as P
    import synth

    log("[bench] generating workload")
    scene = synth.config_scene(2, w=args.res)
    log(f"[bench] {scene.forest.nleaves} leaves; building renderer")
    r = P.Renderer(scene.forest, scene.fields, scene.cameras, "rk4", 4, device="cuda:0")
    counts = r.counts
    S = r.count_segments()
    C = counts["ncand"]
    log(f"[bench] visible {counts['nvis']}, candidates {C}, segments {S}, node records {counts['nrec']}")

    for _ in range(args.warmup):
        r.forward()
    torch.cuda.synchronize()
    ms_eager = time_region(torch, r.forward, args.steps)
    log(f"[bench] forward (eager launches) {ms_eager:.3f} ms")
    r.capture()
    for _ in range(args.warmup):
        r.replay()
    ms = time_region(torch, r.replay, args.steps)
    log(f"[bench] forward (one HIP graph) {ms:.3f} ms")

    # per-phase times (same stream, HIP events)
    t_prune = time_region(torch, r.prune, args.steps)
    t_seg = time_region(torch, r.segments, args.steps)
    t_comp = time_region(torch, r.composite, args.steps)
    log(f"[bench] prune {t_prune:.3f} ms, segments {t_seg:.3f} ms, composite {t_comp:.3f} ms")

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
                        f"({scene.forest.nleaves} leaves), trilinear kappa/eps, {args.res}x{args.res} perspective "
                        f"view, RK4 x 4 substeps",
            "leaves": scene.forest.nleaves,
            "visible": counts["nvis"],
            "candidates": C,
            "segments": S,
            "pixels": r.cams.npix,
        },
        "images_per_s": 1e3 / ms,
        "forward_eager_ms": ms_eager,
        "phase_ms": {"prune": t_prune, "segments": t_seg, "composite": t_comp},
    }
    # dominant kernel: segment generation, one launch of k_segments_rk4<2, 4, 1> per call
    flops = SEG_FLOPS_FP32 * S + CAND_FLOPS_FP64 * C
    achieved = flops / (t_seg * 1e-3) / 1e12
    out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": achieved / FP32_PEAK_TFLOPS, "traffic": measured_traffic("k_segments_rk4<2, 4, 1>"),
                       "kernel": "k_segments_rk4<2, 4, 1>", "flop_per_launch": flops,
                       "per_unit": f"{SEG_FLOPS_FP32} FP32/segment + {CAND_FLOPS_FP64} FP64/candidate"}
    # the other steps against their own bounds
    comp_bytes = C * REC_BYTES + r.cams.npix * PIX_BYTES
    prune_bytes = scene.forest.nleaves * 13 + counts["nvis"] * 20
    comp_traffic = measured_traffic("composite")
    out["phase_roofline"] = {
        "composite": {"bound": "hbm", "algorithmic_bytes": comp_bytes,
                      "achieved_GBs": comp_bytes / (t_comp * 1e-3) / 1e9,
                      "frac": comp_bytes / (t_comp * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      # measured HBM bytes, the node records of the coarsening included
                      "traffic": comp_traffic,
                      "traffic_GBs": comp_traffic / (t_comp * 1e-3) / 1e9 if comp_traffic else None},
        "prune": {"bound": "hbm", "algorithmic_bytes": prune_bytes,
                  "achieved_GBs": prune_bytes / (t_prune * 1e-3) / 1e9,
                  "frac": prune_bytes / (t_prune * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }

    if not args.no_bwd:
        g = torch.ones(r.cams.npix, device="cuda:0")
        for _ in range(2):
            r.forward()
            r.backward(g)

        def fb():
            r.forward()
            r.backward(g)

        ms_fb_eager = time_region(torch, fb, max(args.steps // 2, 5))
        r.capture(backward=True, dLdI=g)
        for _ in range(2):
            r.replay()
        ms_fb = time_region(torch, r.replay, max(args.steps // 2, 5))
        out["fwd_bwd_ms"] = ms_fb
        out["fwd_bwd_eager_ms"] = ms_fb_eager
        out["fwd_bwd_over_fwd"] = ms_fb / ms
        log(f"[bench] forward+backward {ms_fb:.3f} ms (graph), {ms_fb_eager:.3f} ms (eager)")

    if not args.no_bwd:
        out["adjoint_workload"] = bench_adjoint(torch, P, synth, max(args.steps // 2, 5))
    if not args.no_integrators:
        out["integrators"] = bench_integrators(torch, P, r, max(args.steps // 5, 3))
    if not args.no_channels:
        out["channels"] = bench_channels(torch, P, synth, scene, r, max(args.steps // 5, 3))
    if not args.no_analytic:
        out["analytic_workload"] = bench_analytic(torch, P, synth, scene, r, max(args.steps // 5, 3))
    if not args.no_batch:
        out["batched_workload"] = bench_batched(torch, P, synth, r, max(args.steps // 10, 3))
    if not args.no_shell:
        out["shell_workload"] = bench_shell(torch, P, synth, max(args.steps // 10, 3))
    if not args.no_surface:
        out["surface_workload"] = bench_surface(torch, P, synth, max(args.steps // 5, 3))
    if not args.no_surface_ho:
        out["surface_ho_workload"] = bench_surface_ho(torch, P, synth, max(args.steps // 5, 3))
    if not args.no_shares:
        out["shares"] = bench_shares(torch, P, synth, scene, r, max(args.steps // 5, 3))

    if args.copy_calib:
        # a plain copy of known size: 256 MiB read + 256 MiB written per launch
        src = torch.ones(COPY_CALIB_BYTES // 4, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {COPY_CALIB_BYTES} bytes")
        del src, dst
    if not args.no_cpu:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(scene)
    print(json.dumps(out), flush=True)


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


def bench_batched(torch, P, synth, r, steps):
    """The forest of the main workload seen by 64 cameras of uneven resolution: one
    graph launch for all views (autotuned) versus 64 plain per-view forwards."""
    cams = synth.config4_cameras()
    log(f"[bench] batched workload: {len(cams)} cameras, {sum(c.npix for c in cams)} pixels")
    rb = P.Renderer(r.forest, r.fields, cams, "rk4", 4, device="cuda:0", index=r.index)
    from paper_1809_01334_amd.tune import autotune

    tune = autotune(rb, reps=2)
    log(f"[bench] autotuned launch shapes {tune['tuning']}")
    rb.capture()
    rb.replay()
    t_batch = time_region(torch, rb.replay, steps)
    S = rb.count_segments()
    rb_counts = rb.counts
    singles = [P.Renderer(r.forest, r.fields, [c], "rk4", 4, device="cuda:0", index=r.index) for c in cams]

    def plain():
        for x in singles:
            x.forward()

    plain()
    t_plain = time_region(torch, plain, steps)
    log(f"[bench] batched: one graph {t_batch:.2f} ms, 64 plain forwards {t_plain:.2f} ms, segments {S}")
    del singles
    del rb
    # small views, where per-view launches dominate: 64 cameras of 128^2
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
    return {"workload": "64 cameras, resolutions from {256,512,1024,2048}^2, same forest",
            "views": len(cams), "pixels": int(sum(c.npix for c in cams)), "candidates": rb_counts["ncand"],
            "segments": S, "batched_ms": t_batch, "plain_sum_ms": t_plain, "plain_over_batched": t_plain / t_batch,
            "ray_segments_per_s": S / (t_batch * 1e-3), "images_per_s": len(cams) / (t_batch * 1e-3),
            "tuning": tune["tuning"],
            "small_views": {"views": 64, "resolution": 128, "batched_ms": t_small, "plain_sum_ms": t_small_plain,
                            "plain_over_batched": t_small_plain / t_small}}


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
    t_seg = time_region(torch, ra.segments, steps)
    nbytes = c["nvis"] * ANALYTIC_LEAF_BYTES + c["ncand"] * REC_BYTES
    gbs = nbytes / (t_seg * 1e-3) / 1e9
    log(f"[bench] constant coefficients: forward {ms:.3f} ms, segments {t_seg:.3f} ms ({gbs:.0f} GB/s algorithmic)")
    del ra
    torch.cuda.empty_cache()
    return {"workload": "the headline forest and view, one (kappa, eps) per leaf (corner means), analytic segments",
            "segments": S, "ms_per_step": ms, "ray_segments_per_s": S / (ms * 1e-3), "segments_ms": t_seg,
            "roofline": {"bound": "hbm", "kernel": "k_segments_analytic<1>", "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "traffic": measured_traffic("k_segments_analytic<1>"), "bytes_per_launch": nbytes,
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
