"""Schedule autotuner of the heterogeneous persistent launch.

For a given handle and batch, times every candidate schedule of
bysdf_eval_batched (chunk of tiles per queue visit, persistent grid size,
LDS staging of fiber tables, workgroup size = queries per tile, and the
register budget: one or two wavefronts per SIMD) with HIP events on the
current stream, keeps the fastest, and caches it per (device, workload
signature) in a JSON file.  Schedules change only which workgroup
evaluates which tile and how many registers its kernel may hold, never the
arithmetic of a query, so every candidate returns identical outputs.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import bysdf

DEFAULT_CANDIDATES = [dict(chunk=c, grid=g, use_lds=l, block=b, min_waves=w)
                      for c in (1, 4, 16) for g in (512, 1024, 2048, 4096) for l in (1, 0)
                      for b in (128, 256) for w in (1, 2)]


def signature(types: bysdf.Types, offsets_host) -> str:
    counts = np.diff(np.asarray(offsets_host, dtype=np.int64))
    h = hashlib.sha256()
    h.update(np.asarray([types.n_types, counts.sum(), counts.min(initial=0),
                         counts.max(initial=0)], dtype=np.int64).tobytes())
    h.update(np.histogram(np.log2(np.maximum(counts, 1)), bins=16, range=(0, 24))[0].tobytes())
    h.update(np.bincount([d["n_plies"] for d in types.dicts], minlength=9).tobytes())
    return h.hexdigest()[:16]


def _device_name():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def autotune_batched(types, offsets, q, offsets_host, out=None, candidates=None, reps=3,
                     cache_path=None):
    """Returns dict(schedule=..., ms=..., timings=[(schedule, ms), ...])."""
    import torch
    key = "%s/%s" % (_device_name(), signature(types, offsets_host))
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}  # a corrupt cache is ignored and rewritten
        if key in cache:
            return dict(cache[key], cached=True)
    cands = candidates or DEFAULT_CANDIDATES
    n = int(q["h"].numel())
    out = out if out is not None else bysdf.alloc_eval_out(n)
    ws = bysdf.alloc_workspace(bysdf.bysdf_batched_workspace_size(types.n_types))
    stream = torch.cuda.current_stream()
    timings = []
    for sc in cands:
        bysdf.bysdf_eval_batched(types, offsets, q, out, sc, ws)  # warm-up
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            bysdf.bysdf_eval_batched(types, offsets, q, out, sc, ws)
            b.record(stream)
            b.synchronize()
            ms.append(a.elapsed_time(b))
        timings.append((sc, float(np.median(ms))))
    best = min(timings, key=lambda t: t[1])
    res = dict(schedule=best[0], ms=best[1], timings=timings)
    if cache_path:
        cache[key] = dict(schedule=best[0], ms=best[1])
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f)
        os.replace(tmp, cache_path)
    return res
