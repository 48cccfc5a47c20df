"""Tile autotuner for batches (rsvd_batch_tuning).

For a batch signature (shapes, ranks, p, v, dtype) it plans the batch with
every candidate tuning, captures one rsvd_subspace_batched call into a HIP
graph per candidate, times replays of the graph with events, and keeps the
fastest.  Results are cached in a JSON file keyed by the signature, so a
batch of the same shapes is planned with the stored choice.

The candidates span the two choices that set the grouped launches' tiles:
how many compute units the contraction-split planning assumes (0 = no
splits: with hundreds of matrices the batch alone fills the GPU) and how
many 16-row blocks each wave of a view owns.
"""

import hashlib
import json
import os

from . import BatchPlan

CANDIDATES = [(0, 1), (0, 2), (32, 1), (32, 2), (256, 1), (256, 2)]


def signature(mats, ks, p, v):
    h = hashlib.sha256()
    for A, k in zip(mats, ks):
        h.update(f"{tuple(A.shape)}:{A.stride(0)}:{A.dtype}:{int(k)};".encode())
    h.update(f"p={p};v={v}".encode())
    return h.hexdigest()[:24]


def time_plan(plan, reps=5):
    """Median milliseconds of a graph replay of one batched call."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run()                      # warm up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run()
    g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2], g


def tune(mats, ks, p, v, seed=0, cache_path=None, candidates=CANDIDATES, reps=5, log=None):
    """Returns (best tuning, {tuning: ms}); uses and updates the cache."""
    key = signature(mats, ks, p, v)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        entry = cache[key]
        return tuple(entry["best"]), {tuple(map(int, t.split(","))): ms for t, ms in entry["times"].items()}
    results = {}
    for cand in candidates:
        plan = BatchPlan(mats, ks, p, v, seed=seed, tuning=cand)
        ms, _ = time_plan(plan, reps)
        results[cand] = ms
        if log:
            log(f"autotune {cand}: {ms:.3f} ms ({plan.launches} launches)")
        del plan
    best = min(results, key=results.get)
    if cache_path:
        cache[key] = {"best": list(best), "times": {f"{a},{b}": ms for (a, b), ms in results.items()}}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, results
