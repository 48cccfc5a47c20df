#!/usr/bin/env python
"""Throughput of the randomized-SVD views on one MI355X.

Workload (the FP32 plain-method configuration): A is 65536 x 16384 FP32
(4 GiB), A = U diag(sigma) V^T + N with Haar U, V of rank 2048,
sigma_j = j^-1.5 and iid Gaussian noise N of spectral norm about 1e-4 sigma_1;
target rank k = 100, oversampling p = 20 (s = 120).

One step is one pass of the hot path over A: the generalized subspace
iteration (Alg. 2) with v views plus the one-view method (Alg. 7, Psi with
2s+1 = 241 rows).  Inputs are resident in HBM before timing starts.

value = (views per step) x (bytes of A) / (step time), in GB/s.
The roofline entry is the range-view kernel (Y = A X), timed with HIP events
recorded by the library on its own stream around every view of the timed
steps.  cpu_baseline times the CPU oracle on a row sample of the same A.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--views", type=int, default=3, help="views of the subspace iteration per step")
    ap.add_argument("--m", type=int, default=65536)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--rank", type=int, default=2048)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--p", type=int, default=20)
    ap.add_argument("--cpu-rows", type=int, default=16384, help="row sample for the CPU oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-single-pass", action="store_true")
    return ap.parse_args()


def make_matrix(args, torch):
    import numpy as np
    import synth

    sigma = np.arange(1, args.rank + 1, dtype=np.float64) ** -1.5
    return synth.spectral_matrix_torch(args.m, args.n, sigma, synth.GEN_SEED + 2, noise=1e-4,
                                       dtype=torch.float32, device="cuda")


def cpu_baseline(args, A, torch):
    """The oracle as it stands on a row sample of A: Alg. 2 (v views) + Alg. 7."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import synth
    from oracle import rsvd as orsvd

    rows = min(args.cpu_rows, args.m)
    sample = A[:rows].cpu().numpy()
    threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    t0 = time.perf_counter()
    orsvd.alg2_gensubit(sample, args.k, args.p, args.views, synth.METHOD_SEED)
    views = args.views
    if not args.no_single_pass:
        orsvd.alg7_one_view(sample, args.k, args.p, synth.METHOD_SEED)
        views += 1
    dt = time.perf_counter() - t0
    gbs = views * sample.nbytes / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"rows 0..{rows - 1} of A ({rows}x{args.n} FP32, {sample.nbytes / 2**30:.2f} GiB), "
                      f"same step (Alg. 2 with {args.views} views + Alg. 7), {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by rows of A across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1804_07531_amd as rs
    import synth

    torch.cuda.init()
    A = make_matrix(args, torch)
    torch.cuda.synchronize()
    m, n, k, p = args.m, args.n, args.k, args.p
    s = k + p
    seed = synth.METHOD_SEED
    ws_sub = torch.empty(rs.workspace_bytes(A, k, p, args.views, rs._lib.ALGO_SUBSPACE), dtype=torch.uint8,
                         device="cuda")
    ws_one = torch.empty(max(rs.workspace_bytes(A, k, p, 1, rs._lib.ALGO_SINGLE_PASS), 256), dtype=torch.uint8,
                         device="cuda")
    timers = []

    def step(trace_list=None):
        t1 = rs.ViewTimer(16) if trace_list is not None else None
        rs.subspace(A, k, p, args.views, seed=seed, workspace=ws_sub, trace=t1.trace if t1 else None)
        t2 = None
        if not args.no_single_pass:
            t2 = rs.ViewTimer(16) if trace_list is not None else None
            rs.single_pass(A, k, p, seed=seed, workspace=ws_one, trace=t2.trace if t2 else None)
        if trace_list is not None:
            trace_list.append((t1, t2))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(timers)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3

    range_ms, corange_ms, one_ms = [], [], []
    for t1, t2 in timers:
        for kind, ms in t1.results():
            (range_ms if kind == 0 else corange_ms).append(ms)
        if t2 is not None:
            one_ms.append(sum(ms for _, ms in t2.results()))
    views_per_step = args.views + (0 if args.no_single_pass else 1)
    bytes_a = m * n * 4
    value = views_per_step * bytes_a / (ms_step * 1e-3) / 1e9

    r_ms = sum(range_ms) / len(range_ms)
    flops = 2.0 * m * n * s
    achieved_tf = flops / (r_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved_tf, 2), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tf / PEAK_FP32_TFLOPS, 4), "traffic": None,
                "kernel": "range view Y = A X (FP32 matrix cores)",
                "kernel_ms": round(r_ms, 4),
                "hbm_gbs": round(bytes_a / (r_ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(bytes_a / (r_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    extra = {"corange_view_ms": round(sum(corange_ms) / max(1, len(corange_ms)), 4)}
    if one_ms:
        extra["one_view_pass_ms"] = round(sum(one_ms) / len(one_ms), 4)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, A, torch)

    line = {
        "metric": "HBM GB/s per view (views of A per step x bytes of A / step time)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"FP32 {m}x{n} A, sigma_j=j^-1.5 (rank {args.rank}) + 1e-4 noise; k={k}, p={p}; "
                               f"step = Alg. 2 with v={args.views} + Alg. 7 (s_w={2 * s + 1})",
                   "views_per_step": views_per_step, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
