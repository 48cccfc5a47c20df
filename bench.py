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
The roofline entry is the kernel with the largest share of the step: the
co-range product W += Psi_b A_b that the one-view sweep takes on each
4096-row panel (s_w = 241 thin rows), timed with HIP events the library
records on its own stream around each panel product of the timed steps
(trace hook with inner = 1); the range view Y = A X of the subspace
iteration is reported beside it.  cpu_baseline times the CPU oracle on the
same A with all host threads, and on a row sample single-threaded.
"""

import argparse
import json
import math
import os
import sys
import tempfile
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
    ap.add_argument("--cpu-rows", type=int, default=65536,
                    help="row sample for the CPU oracle baseline (default: all rows of the 65536-row A)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-single-pass", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision, batch and gradient measurements reported under detail")
    ap.add_argument("--tuning-cache", default=None, help="JSON cache of the batch autotuner")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the range view three times and a 1 GiB copy three times (for HBM counters)")
    ap.add_argument("--precision-profile", choices=["bf16", "fp8"], nargs="?", const="bf16", default=None,
                    help="only run four BF16 (or FP8) + refinement solves of the precision workload "
                         "(for kernel traces)")
    ap.add_argument("--no-precision-oracle", action="store_true",
                    help="skip the FP64 oracle runs that state the precision workload's errors")
    ap.add_argument("--cpu-single-rows", type=int, default=8192,
                    help="row sample of the single-threaded CPU oracle timing")
    ap.add_argument("--gradient-profile", action="store_true",
                    help="only run three forward + backward passes of the differentiation workload (for kernel traces)")
    ap.add_argument("--lp-view-probe", action="store_true",
                    help="only run the cheap BF16 and FP8 views of the precision workload three times each "
                         "(for counters)")
    ap.add_argument("--batch-profile", action="store_true",
                    help="only run five graph replays of the 512-matrix batch (for kernel traces)")
    return ap.parse_args()


# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (each
# scaled by the same counter on a 1 GiB copy), valid for the view sources with
# this digest; reported as null once those sources change.  "range": the
# range view Y = A X at s = 120; "corange_panel": the one-view co-range
# product on a 4096-row panel at s_w = 241.
TRAFFIC = {"sources_sha256": "cb93d776afcf095e5c4bbe329dd27321fbda1858400b2fddc8a7387444a95b1e",
           "range": 4423458521, "corange_panel": 363714552}
TRAFFIC_SOURCES = ["paper_1804_07531_amd/csrc/views.hip", "paper_1804_07531_amd/csrc/views.h",
                   "paper_1804_07531_amd/csrc/launch.h", "paper_1804_07531_amd/csrc/common.h"]


def view_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_probe(args):
    import torch

    import paper_1804_07531_amd as rs
    torch.cuda.init()
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    # the traffic of a view does not depend on the values of A: a Gaussian A of the same shape
    A = torch.randn(args.m, args.n, device="cuda", dtype=torch.float32, generator=g)
    s = args.k + args.p
    XT = torch.randn(s, args.n, device="cuda", dtype=torch.float32, generator=g)
    for _ in range(3):
        rs.view_range(A, XT)
    # the one-view sweep's panel products: 16 panels of 4096 rows, s = 120 and s_w = 241
    PsiT = torch.randn(2 * s + 1, 4096, device="cuda", dtype=torch.float32, generator=g)
    for r0 in range(0, args.m, 4096):
        Ab = A[r0:r0 + 4096]
        rs.view_range(Ab, XT)
        rs.view_corange(Ab, PsiT)
    a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda").fill_(1.0)   # 1 GiB
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"traffic probe done; view sources {view_sources_sha256()}", flush=True)


# ---------------------------------------------------------------------------
# extra workloads (reported under "detail"; the headline value is the FP32 step)
# ---------------------------------------------------------------------------

def _time_ms(fn, torch, reps=3):
    fn()
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        t.append((time.perf_counter() - t0) * 1e3)
    t.sort()
    return t[len(t) // 2]


def _rel_frob_error(A, U, S, V, torch, chunk=8192):
    """||A - U diag(S) V^T||_F / ||A||_F in FP64 (U, V orthonormal), one pass over A."""
    a2, cross = 0.0, 0.0
    Vd = V.double()
    Sd = S.double()
    for r0 in range(0, A.shape[0], chunk):
        Ab = A[r0:r0 + chunk].double()
        a2 += float((Ab * Ab).sum())
        cross += float(((Ab @ Vd) * U[r0:r0 + chunk].double() * Sd[None, :]).sum())
        del Ab
    e2 = max(0.0, a2 - 2.0 * cross + float((Sd * Sd).sum()))
    return math.sqrt(e2 / a2)


class _StoredRows:
    """A BF16 or FP8 matrix as the oracle reads it: exact FP64 values of the
    stored bytes (times the row scales for FP8), one block of rows at a time."""

    def __init__(self, fmt, bits, scale):
        self.fmt, self.bits, self.scale = fmt, bits, scale
        self.shape = bits.shape

    def rows_f64(self, r0, r1):
        from oracle import formats as oformats
        if self.fmt == "bf16":
            return oformats.bf16_bits_to_f64(self.bits[r0:r1])
        return oformats.fp8_rows_to_f64(self.bits[r0:r1], self.scale[r0:r1])


def _precision_oracle(fmt, bits, scale, k, p, v, seed):
    """The FP64 oracle (Alg. 2) on the exact values of the stored bytes."""
    from oracle import rsvd as orsvd
    t0 = time.perf_counter()
    ref = orsvd.alg2_gensubit(_StoredRows(fmt, bits, scale), k, p, v, seed)
    print(f"bench: FP64 oracle on the stored {fmt} values, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    return ref


def _against_oracle(fmt, res, ref, A_val, torch):
    """sigma and reconstruction error of a GPU solve against the FP64 oracle's."""
    import numpy as np
    U, S, V = res
    rel = float(np.max(np.abs(S.cpu().numpy() - ref.S) / ref.S))
    Ur, Sr, Vr = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (ref.U, ref.S, ref.V))
    e_ref = _rel_frob_error(A_val, Ur, Sr, Vr, torch)
    return {f"{fmt}_sigma_rel_err_vs_oracle": rel, f"oracle_{fmt}_rel_err": e_ref}


def extra_precision(torch, rs, synth, with_oracle=True):
    """131072 x 32768, sigma_j = 10^(-j/25) (rank 256) + noise 1e-6: k = 200, p = 20, v = 3.
    Stored BF16 (and FP8 E4M3 with row scales) with one FP32 refinement view, against
    plain FP32 on the same stored values; time to solution and relative Frobenius error."""
    import numpy as np
    m, n, k, p, v = 131072, 32768, 200, 20, 3
    sigma = 10.0 ** (-np.arange(1, 257, dtype=np.float64) / 25.0)
    A32 = synth.spectral_matrix_torch(m, n, sigma, synth.GEN_SEED + 3, noise=1e-6, dtype=torch.float32)
    Ab = A32.to(torch.bfloat16)
    del A32
    torch.cuda.empty_cache()
    seed = synth.METHOD_SEED
    out = {"workload": f"{m}x{n}, sigma_j=10^(-j/25) (rank 256) + 1e-6 noise, k={k}, p={p}, v={v}"}
    # BF16 storage, last view FP32-accurate; the views are traced on a warm call
    out["bf16_refine_ms"] = round(_time_ms(lambda: rs.subspace(Ab, k, p, v, seed=seed, refine=1), torch), 3)
    t = rs.ViewTimer(8)
    res = rs.subspace(Ab, k, p, v, seed=seed, refine=1, trace=t.trace)
    views = t.results()
    out["bf16_view_ms"] = [round(ms, 3) for _, ms in views]   # cheap range, cheap co-range, refinement range
    out["bf16_view_gbs"] = [round(m * n * 2 / (ms * 1e-3) / 1e9, 1) for _, ms in views]
    out["bf16_cheap_view_gbs"] = round(m * n * 2 / (views[0][1] * 1e-3) / 1e9, 1)
    A_cmp = Ab.float()                       # the same stored values, FP32
    out["bf16_refine_rel_err"] = _rel_frob_error(A_cmp, *res, torch)
    if with_oracle:
        ref = _precision_oracle("bf16", Ab.view(torch.int16).cpu().numpy().view(np.uint16), None, k, p, v, seed)
        out.update(_against_oracle("bf16", res, ref, A_cmp, torch))
    del res
    # plain FP32 on the same stored values (FP32 matrix cores; the split mode takes at most 192
    # thin columns and would fall back to them at s = 220)
    res = rs.subspace(A_cmp, k, p, v, seed=seed, f32_mode=rs.F32_MFMA)
    out["fp32_ms"] = round(_time_ms(lambda: rs.subspace(A_cmp, k, p, v, seed=seed, f32_mode=rs.F32_MFMA), torch), 3)
    out["fp32_rel_err"] = _rel_frob_error(A_cmp, *res, torch)
    if with_oracle:
        out["fp32_sigma_rel_err_vs_oracle"] = float(np.max(np.abs(res[1].cpu().numpy() - ref.S) / ref.S))
        del ref
    del res
    out["bf16_speedup_vs_fp32"] = round(out["fp32_ms"] / out["bf16_refine_ms"], 2)
    out["bf16_error_ratio_vs_fp32"] = round(out["bf16_refine_rel_err"] / out["fp32_rel_err"], 5)
    # FP8 E4M3 with row scales (stored values = scale * e4m3)
    scale = (A_cmp.abs().amax(dim=1) / 448.0).clamp_min(1e-30)
    A8 = (A_cmp / scale[:, None]).to(torch.float8_e4m3fn)
    del A_cmp, Ab
    torch.cuda.empty_cache()
    res = rs.subspace(A8, k, p, v, seed=seed, refine=1, row_scale=scale)
    out["fp8_refine_ms"] = round(_time_ms(lambda: rs.subspace(A8, k, p, v, seed=seed, refine=1, row_scale=scale),
                                          torch), 3)
    t8 = rs.ViewTimer(8)
    rs.subspace(A8, k, p, v, seed=seed, refine=1, row_scale=scale, trace=t8.trace)
    views8 = t8.results()
    out["fp8_view_ms"] = [round(ms, 3) for _, ms in views8]   # cheap range, cheap co-range, refinement range
    out["fp8_view_gbs"] = [round(m * n * 1 / (ms * 1e-3) / 1e9, 1) for _, ms in views8]
    A8f = A8.float() * scale[:, None]
    out["fp8_refine_rel_err"] = _rel_frob_error(A8f, *res, torch)
    if with_oracle:
        ref = _precision_oracle("fp8", A8.view(torch.uint8).cpu().numpy(), scale.cpu().numpy(), k, p, v, seed)
        out.update(_against_oracle("fp8", res, ref, A8f, torch))
        del ref
    del A8, A8f, res
    torch.cuda.empty_cache()
    return out


def _batch_mats(torch, synth):
    """The 512 matrices of the batch workload (rows padded to 16 bytes), their k, and the bytes of A."""
    import numpy as np
    m, n, k = synth.batch_shapes(512, synth.GEN_SEED)
    mats = []
    nbytes = 0
    for b in range(512):
        r = int(min(m[b], n[b], 256))
        sigma = np.arange(1, r + 1, dtype=np.float64) ** -2.0
        ld = (int(n[b]) + 3) // 4 * 4        # rows padded to 16 bytes
        buf = torch.empty(int(m[b]), ld, dtype=torch.float32, device="cuda")
        buf[:, :int(n[b])] = synth.spectral_matrix_torch(int(m[b]), int(n[b]), sigma, synth.GEN_SEED + 4 + b,
                                                         dtype=torch.float32)
        mats.append(buf[:, :int(n[b])])
        nbytes += int(m[b]) * int(n[b]) * 4
    return mats, [int(x) for x in k], nbytes


def extra_batched(torch, rs, synth, cache_path):
    """512 FP32 matrices, m log-uniform in [500, 8000], n in [200, 4000], k in {8..64}, p = 8,
    v = 3, sigma_j = j^-2 (rank min(m, n, 256)); one graph replay of the batched call, tiles
    chosen by the autotuner."""
    from paper_1804_07531_amd import autotune
    mats, ks, nbytes = _batch_mats(torch, synth)
    p, v = 8, 3
    best, times = autotune.tune(mats, ks, p, v, seed=synth.METHOD_SEED, cache_path=cache_path, reps=3)
    plan = rs.BatchPlan(mats, ks, p, v, seed=synth.METHOD_SEED, tuning=best)
    ms, _ = autotune.time_plan(plan, reps=5)
    seq_ms = _time_ms(lambda: [rs.subspace(A, kk, p, v, seed=synth.METHOD_SEED) for A, kk in zip(mats, ks)], torch,
                      reps=1)
    return {"workload": "512 FP32 matrices (m in [500, 8000], n in [200, 4000], k in [8, 64], p=8, v=3)",
            "bytes_of_A": nbytes, "batched_graph_ms": round(ms, 3), "launches": plan.launches,
            "gbs_per_view": round(v * nbytes / (ms * 1e-3) / 1e9, 1), "tuning": list(best),
            "autotune_ms": {f"{a},{b}": round(t, 3) for (a, b), t in times.items()},
            "sequential_calls_ms": round(seq_ms, 3)}


def extra_gradient(torch, rs, synth):
    """32768 x 8192 FP32, sigma_j = j^-1 (full Haar factors), row sweep k = 64, p = 16, v = 4,
    1024-row blocks; loss sum_i w_i sigma_i + ||A - Q_c Q_c^T A||_F^2."""
    import numpy as np
    from oracle import grad as ograd
    from paper_1804_07531_amd.autograd import row_sweep_svd
    m, n, k, p, v = 32768, 8192, 64, 16, 4
    sigma = np.arange(1, n + 1, dtype=np.float64) ** -1.0
    A = synth.spectral_matrix_torch(m, n, sigma, synth.GEN_SEED + 5, dtype=torch.float32)
    w = torch.from_numpy(ograd.loss_weights(k)).cuda()
    seed = synth.METHOD_SEED

    def fwd():
        S, E, _, _ = row_sweep_svd(A, k, p, v, seed, 1024)
        return (w * S).sum() + E

    def fwd_bwd():
        Ar = A.detach().requires_grad_(True)
        S, E, _, _ = row_sweep_svd(Ar, k, p, v, seed, 1024)
        return torch.autograd.grad((w * S).sum() + E, Ar)[0]

    f_ms = _time_ms(fwd, torch)
    fb_ms = _time_ms(fwd_bwd, torch)
    del A
    torch.cuda.empty_cache()
    return {"workload": f"{m}x{n} FP32, sigma_j=j^-1, row sweep k={k} p={p} v={v}, 1024-row blocks",
            "forward_ms": round(f_ms, 3), "forward_backward_ms": round(fb_ms, 3)}


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

    from threadpoolctl import threadpool_limits

    def run(sample):
        t0 = time.perf_counter()
        orsvd.alg2_gensubit(sample, args.k, args.p, args.views, synth.METHOD_SEED)
        views = args.views
        if not args.no_single_pass:
            orsvd.alg7_one_view(sample, args.k, args.p, synth.METHOD_SEED)
            views += 1
        dt = time.perf_counter() - t0
        return views * sample.nbytes / dt / 1e9, dt

    rows = min(args.cpu_rows, args.m)
    sample = A[:rows].cpu().numpy()
    threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    gbs, dt = run(sample)
    out = {"value": round(gbs, 3), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
           "sample": f"rows 0..{rows - 1} of A ({rows}x{args.n} FP32, {sample.nbytes / 2**30:.2f} GiB), "
                     f"same step (Alg. 2 with {args.views} views + Alg. 7), {dt:.1f} s", "cpu_model": _cpu_model(),
           "logical_cpus": os.cpu_count()}
    rows1 = min(args.cpu_single_rows, args.m)
    if rows1 >= args.k + args.p and rows1 >= 2 * (args.k + args.p) + 1:
        with threadpool_limits(limits=1, user_api="blas"):
            gbs1, dt1 = run(sample[:rows1])
        out["single_thread"] = {"value": round(gbs1, 3), "unit": "GB/s", "cores": 1,
                                "sample": f"rows 0..{rows1 - 1} of A, the same step, {dt1:.1f} s"}
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def precision_profile(fmt):
    """Four BF16 (or FP8) + refinement solves of the 131072 x 32768 precision workload, nothing else."""
    import numpy as np
    import torch

    import paper_1804_07531_amd as rs
    import synth
    m, n, k, p, v = 131072, 32768, 200, 20, 3
    sigma = 10.0 ** (-np.arange(1, 257, dtype=np.float64) / 25.0)
    A32 = synth.spectral_matrix_torch(m, n, sigma, synth.GEN_SEED + 3, noise=1e-6, dtype=torch.float32)
    Ab = A32.to(torch.bfloat16)
    del A32
    torch.cuda.empty_cache()
    extra = {}
    if fmt == "fp8":
        Af = Ab.float()
        scale = (Af.abs().amax(dim=1) / 448.0).clamp_min(1e-30)
        Ab = (Af / scale[:, None]).to(torch.float8_e4m3fn)
        extra = {"row_scale": scale}
        del Af
        torch.cuda.empty_cache()
    for _ in range(4):
        rs.subspace(Ab, k, p, v, seed=synth.METHOD_SEED, refine=1, **extra)
    torch.cuda.synchronize()
    print(f"precision profile ({fmt}) done", flush=True)


def lp_view_probe():
    """The cheap views of the precision workload (131072 x 32768, s = 220): BF16 range and co-range,
    FP8 range and co-range, three of each, on a Gaussian A of the stored shape (a view's traffic and
    time do not depend on A's values)."""
    import torch

    import paper_1804_07531_amd as rs
    m, n, s = 131072, 32768, 220
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    Ab = torch.empty(m, n, dtype=torch.bfloat16, device="cuda")
    for r0 in range(0, m, 8192):
        Ab[r0:r0 + 8192] = torch.randn(8192, n, device="cuda", generator=g).to(torch.bfloat16)
    XT = torch.randn(s, n, device="cuda", generator=g)
    YT = torch.randn(s, m, device="cuda", generator=g)
    for _ in range(3):
        rs.view_range(Ab, XT, refine=0)
    for _ in range(3):
        rs.view_corange(Ab, YT, refine=0)
    Af = Ab.float()
    scale = (Af.abs().amax(dim=1) / 448.0).clamp_min(1e-30)
    A8 = torch.empty(m, n, dtype=torch.float8_e4m3fn, device="cuda")
    for r0 in range(0, m, 8192):
        A8[r0:r0 + 8192] = (Af[r0:r0 + 8192] / scale[r0:r0 + 8192, None]).to(torch.float8_e4m3fn)
    del Af
    torch.cuda.empty_cache()
    for _ in range(3):
        rs.view_range(A8, XT, refine=0, row_scale=scale)
    for _ in range(3):
        rs.view_corange(A8, YT, refine=0, row_scale=scale)
    torch.cuda.synchronize()
    print("lp view probe done", flush=True)


def batch_profile():
    """Five graph replays of the 512-matrix batch with tuning (0, 1), the autotuner's pick on
    MI355X, after one eager warm-up call; nothing else."""
    import torch

    import paper_1804_07531_amd as rs
    import synth
    from paper_1804_07531_amd import autotune
    mats, ks, _ = _batch_mats(torch, synth)
    plan = rs.BatchPlan(mats, ks, 8, 3, seed=synth.METHOD_SEED, tuning=(0, 1))
    ms, _ = autotune.time_plan(plan, reps=5)
    torch.cuda.synchronize()
    print(f"batch profile done: {plan.launches} launches, {ms:.3f} ms per replay", flush=True)


def gradient_profile():
    """Three forward + backward passes of the 32768 x 8192 differentiation workload, nothing else."""
    import numpy as np
    import torch

    import synth
    from oracle import grad as ograd
    from paper_1804_07531_amd.autograd import row_sweep_svd
    m, n, k, p, v = 32768, 8192, 64, 16, 4
    sigma = np.arange(1, n + 1, dtype=np.float64) ** -1.0
    A = synth.spectral_matrix_torch(m, n, sigma, synth.GEN_SEED + 5, dtype=torch.float32)
    w = torch.from_numpy(ograd.loss_weights(k)).cuda()
    for _ in range(3):
        Ar = A.detach().requires_grad_(True)
        S, E, _, _ = row_sweep_svd(Ar, k, p, v, synth.METHOD_SEED, 1024)
        torch.autograd.grad((w * S).sum() + E, Ar)
    torch.cuda.synchronize()
    print("gradient profile done", flush=True)


def main():
    args = parse()
    if args.traffic_probe:
        traffic_probe(args)
        return
    if args.precision_profile:
        precision_profile(args.precision_profile)
        return
    if args.gradient_profile:
        gradient_profile()
        return
    if args.batch_profile:
        batch_profile()
        return
    if args.lp_view_probe:
        lp_view_probe()
        return
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
            # the panel products inside the one-view sweep, each between its own events
            t2 = rs.ViewTimer(4 * (m // 256 + 2), inner=True) if trace_list is not None else None
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

    range_ms, corange_ms, one_ms, panel_r, panel_c = [], [], [], [], []
    for t1, t2 in timers:
        for kind, ms in t1.results():
            (range_ms if kind == 0 else corange_ms).append(ms)
        if t2 is not None:
            res2 = t2.results()
            one_ms.append(sum(ms for _, ms in res2))
            panel_r += [ms for kind, ms in res2 if kind == 0]
            panel_c += [ms for kind, ms in res2 if kind == 1]
    views_per_step = args.views + (0 if args.no_single_pass else 1)
    bytes_a = m * n * 4
    value = views_per_step * bytes_a / (ms_step * 1e-3) / 1e9
    same_sources = TRAFFIC["sources_sha256"] == view_sources_sha256()

    def mfma_roofline(kernel, flops, nbytes, ms, traffic_key):
        tf = flops / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / PEAK_FP32_TFLOPS, 4),
                "traffic": TRAFFIC[traffic_key] if same_sources else None, "kernel": kernel,
                "kernel_ms": round(ms, 4), "algorithmic_bytes": nbytes,
                "hbm_gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}

    r_ms = sum(range_ms) / len(range_ms)
    range_roof = mfma_roofline("range view Y = A X, s = 120 (FP32 matrix cores)", 2.0 * m * n * s, bytes_a, r_ms,
                               "range")
    extra = {"corange_view_ms": round(sum(corange_ms) / max(1, len(corange_ms)), 4)}
    if panel_c:
        rows = min(m, 4096)
        sw = 2 * s + 1
        c_ms = sum(panel_c) / len(panel_c)
        roofline = mfma_roofline(f"one-view co-range panel product W += Psi_b A_b ({rows} rows, s_w = {sw}; "
                                 "FP32 matrix cores)", 2.0 * rows * n * sw, rows * n * 4, c_ms, "corange_panel")
        roofline["launches_per_step"] = len(panel_c) // len(timers)
        extra["roofline_range_view"] = range_roof
        extra["one_view_panel_range_ms"] = round(sum(panel_r) / len(panel_r), 4)
        extra["one_view_pass_ms"] = round(sum(one_ms) / len(one_ms), 4)
    else:
        roofline = range_roof
    # the exact BF16 split of the FP32 views (six BF16 products, Sect. on precision in the design notes)
    if not args.no_extras:
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        XT = torch.randn(s, n, device="cuda", dtype=torch.float32, generator=g)
        YT = torch.randn(s, m, device="cuda", dtype=torch.float32, generator=g)
        split = {}
        for name, mode in (("mfma", rs.F32_MFMA), ("bf16x6", rs.F32_BF16X6)):
            split[f"{name}_range_view_ms"] = round(_time_ms(lambda: rs.view_range(A, XT, f32_mode=mode), torch), 3)
            split[f"{name}_corange_view_ms"] = round(
                _time_ms(lambda: rs.view_corange(A, YT, f32_mode=mode), torch), 3)
            split[f"{name}_subspace_ms"] = round(_time_ms(
                lambda: rs.subspace(A, k, p, args.views, seed=seed, workspace=ws_sub, f32_mode=mode), torch), 3)
        extra["fp32_split_mode_s120"] = split
        del XT, YT
    if not args.no_extras:
        # the extended one-view sketch (Sect. 6.7) on the same A, core of 2s + 1 rows: a whole call
        sc = 2 * s + 1
        ws_ext = torch.empty(max(rs.workspace_bytes(A, k, p, 1, rs._lib.ALGO_SINGLE_PASS, core_rows=sc), 256),
                             dtype=torch.uint8, device="cuda")
        extra["extended_one_view_ms"] = round(_time_ms(
            lambda: rs.single_pass(A, k, p, seed=seed, workspace=ws_ext, core_rows=sc), torch), 3)
        extra["single_pass_call_ms"] = round(_time_ms(
            lambda: rs.single_pass(A, k, p, seed=seed, workspace=ws_one), torch), 3)
        del ws_ext

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, A, torch)

    if not args.no_extras:
        del A, ws_sub, ws_one
        torch.cuda.empty_cache()
        cache = args.tuning_cache or os.path.join(tempfile.gettempdir(), "rsvd_batch_tuning.json")
        for name, fn in (("precision", lambda: extra_precision(torch, rs, synth, not args.no_precision_oracle)),
                         ("batched", lambda: extra_batched(torch, rs, synth, cache)),
                         ("gradient", lambda: extra_gradient(torch, rs, synth))):
            print(f"bench: {name} workload", file=sys.stderr, flush=True)
            extra[name] = fn()
            torch.cuda.empty_cache()

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
