"""Autotuner for the launch shapes of a Renderer (rc_tuning).

For a fixed forest and camera set it times the forward with candidate
workgroup counts for the segment kernel, the level folds and the root fold,
and the levels of the coarsening whose node records compositing leaves out
(coordinate descent, HIP events on the renderer's stream), and keeps the
fastest.  Forward results are identical for every shape, so tuning changes
time only.  Chosen shapes can be cached in a JSON file keyed by the
workload's signature.
"""

from __future__ import annotations

import json
import os
from typing import Dict, Optional

import torch

from . import _lib as L

SEG_BLOCKS = (2048, 4096, 8192, 16384, 32768)
FOLD_BLOCKS = (1024, 2048, 4096, 8192, 16384)
ROOT_BLOCKS = (1024, 2048, 4096, 8192)
# levels whose node records the forward leaves out, folded by the pass above
FOLD_SKIP = (0, 0b10, 0b100, 0b1000, 0b1010, 0b1100)
# workgroups of the leaf adjoint (rc_segments_backward)
ADJ_BLOCKS = (1024, 2048, 4096, 8192, 16384)


def _time(renderer, fn, reps: int) -> float:
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize(renderer.device)
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    torch.cuda.synchronize(renderer.device)
    return start.elapsed_time(end) / reps


def signature(renderer) -> str:
    c = renderer.counts
    wh = ",".join(f"{w}x{h}" for w, h in renderer.cams.wh)
    return f"N{renderer.forest.nleaves}-vis{c['nvis']}-cand{c['ncand']}-rec{c['nrec']}-m{renderer.method}-s{renderer.substeps}-{wh}"


def autotune(renderer, reps: int = 5, cache: Optional[str] = None, keys: Optional[tuple] = None) -> Dict:
    """Pick rc_tuning for `renderer` in place; returns the choice and the timings.
    keys: tune only these fields (the others keep the renderer's values)."""
    sig = signature(renderer)
    if cache and os.path.exists(cache):
        try:
            known = json.load(open(cache))
        except (OSError, ValueError):
            known = {}
        if sig in known:
            renderer.tuning = L.RcTuning(**known[sig]["tuning"])
            return known[sig]
    renderer.prune()
    renderer.segments()
    t0 = renderer.tuning
    best = {k: int(getattr(t0, k)) for k in ("seg_blocks", "fold_blocks", "root_blocks", "adj_blocks", "fold_skip")}
    if keys is None:
        best = {k: 0 for k in best}
    log = {}
    for key, opts, fn in (("seg_blocks", SEG_BLOCKS, renderer.segments),
                          ("fold_blocks", FOLD_BLOCKS, renderer.composite),
                          ("root_blocks", ROOT_BLOCKS, renderer.composite),
                          ("fold_skip", FOLD_SKIP, renderer.composite)):
        if keys is not None and key not in keys:
            continue
        times = {}
        for v in opts:
            renderer.tuning = L.RcTuning(**{**best, key: v})
            times[v] = _time(renderer, fn, reps)
        best[key] = min(times, key=times.get)
        log[key] = {str(k): round(t, 4) for k, t in times.items()}
    renderer.tuning = L.RcTuning(**best)
    result = {"tuning": best, "ms": log, "signature": sig}
    if cache:
        known = {}
        if os.path.exists(cache):
            try:
                known = json.load(open(cache))
            except (OSError, ValueError):
                known = {}
        known[sig] = result
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1)
    return result


def autotune_adjoint(renderer, dLdI: torch.Tensor, reps: int = 5) -> Dict:
    """Workgroups of the leaf adjoint (rc_tuning.adj_blocks): the backward
    after a forward meant for the adjoint, timed with each candidate.  For a
    given grid the gradients are reproducible bit for bit; between grids they
    differ by rounding only (a (chunk, pair) partial sums its hits in batches
    whose split depends on the grid).  Sets the renderer's adj_blocks to the
    fastest; returns it with the timings."""
    renderer.forward(for_adjoint=True)
    dk = torch.empty_like(renderer.fields.kappa)
    de = torch.empty_like(renderer.fields.eps)
    times = {}
    for v in ADJ_BLOCKS:
        renderer.tuning.adj_blocks = v
        times[v] = _time(renderer, lambda: renderer.backward(dLdI, dk, de), reps)
    best = min(times, key=times.get)
    renderer.tuning.adj_blocks = best
    return {"adj_blocks": best, "ms": {str(k): round(t, 4) for k, t in times.items()}}
