"""Benchmark: st-HOSVD-ALS on one MI355X.

Workload: 200x200x200x200 FP32 tensor, core 20^4 with entries
N(0,1) exp(-(i+j+k+l)/10) times orthonormal 200x20 factors plus 1e-4 relative
Gaussian noise (seeded, generated on the GPU); st-HOSVD-ALS to ranks
(20,20,20,20) with eta = 1e-4.

A step is one full st-HOSVD-ALS call (norm, initial sketches, every ALS sweep,
QRs, the TTM truncations) on the resident input.  `value` is the step's
algorithmic HBM bytes (one read of the current tensor per pass plus the TTM
writes) divided by the step time.  The `roofline` object times the fused ALS
sweep kernel alone on mode 1 (6.4 GB per launch) with HIP events on the stream
it is launched on.  Its arithmetic intensity (per fibre of I = 200 FP32
values: 2IR flops for v_j, 2IR for the L_acc update, 2R^2 for G_V, i.e. 21
flop/B at R = 20) lies above the FP32 matrix-core ridge (157.3 TFLOP/s over
8 TB/s = 19.7 flop/B), so the roof that binds is the FP32 matrix core; the
HBM figures are reported beside it.  `cpu_baseline` times the FP64 CPU oracle's literal ALS
sweeps on a sample of the mode-1 unfolding.

Beside the headline line, the same JSON carries BF16 storage on the same
workload (time to tolerance against plain FP32), the 512-tensor batched
workload, and the 1024^3 t-HOSVD-ALS workload in FP32 and BF16 storage
(`large_*` keys; `--no-large` skips it, `--only-large` runs it alone).
`--paper-tucker` times, alone, the paper's largest 4-way Tucker test case
(Section 6.1.2: 5000 x 100^3 FP32, 20 GB), whose first mode (I = 5000,
R = 50) is beyond the fused kernels and runs on the generic two-pass path.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3     # MI355X dense FP32 matrix-core peak
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_fused_sweep_mode1_200x4_f32_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2004_02583_amd", "csrc", "k_fused.hip")
DIMS = (200, 200, 200, 200)
RANK = 20
TOL = 1e-4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def step_bytes(dims, ranks, iters, elem=4):
    """Algorithmic HBM bytes of one st-HOSVD-ALS call in natural order: per
    mode n on the current tensor B (s bytes): the initial sketch pass (which
    also yields ||B||), iters+1 sweeps, and the truncation (read s, write
    s*R_n/I_n)."""
    cur = list(dims)
    total = 0.0
    size = float(elem)
    for d in cur:
        size *= d
    for n in range(len(dims)):
        total += size                  # sketch pass (+ norm)
        total += (iters[n] + 1) * size  # sweeps
        nxt = size * ranks[n] / cur[n]
        total += size + nxt            # TTM read + write
        cur[n] = ranks[n]
        size = nxt
    return total


def relerr_gpu(tk, A, G, Us):
    import torch
    Ah = tk.tucker_reconstruct(G, Us)
    e = torch.linalg.vector_norm((A.double() - Ah.double()).float()).item()
    return e / torch.linalg.vector_norm(A.float()).item()


def time_sweep_kernel(tk, A, Lq, launches=10, mode=0):
    """Average duration of the fused sweep kernel on a mode (default the
    first), HIP events on the stream the kernel is launched on (torch's
    current stream, which is the stream handed to the library)."""
    import torch
    ws = tk.step_workspace(A, mode, Lq.shape[1])
    stream = torch.cuda.current_stream()
    for _ in range(2):
        tk.als_sweep_kernel(A, mode, Lq, reduce=False, workspace=ws)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(launches):
        tk.als_sweep_kernel(A, mode, Lq, reduce=False, workspace=ws)
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / launches


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the fused sweep (mode 1) from the committed
    FETCH_SIZE / WRITE_SIZE summary, scaled by the copy-kernel calibration;
    None when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size, for scaling the FETCH_SIZE /
    WRITE_SIZE counters (read nbytes, write nbytes)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {nbytes} bytes")


def bench_large(tk, steps, n=1024, core=64, rank=48, tol=1e-4):
    """The 1024^3 workload: core 64^3 with entries N(0,1) 0.9^(i+j+k) times
    orthonormal 1024x64 factors plus 1e-3 relative noise (seeded, generated
    on the GPU); t-HOSVD-ALS to (48,48,48) with eta = 1e-4 in FP32 and in BF16
    storage: time to tolerance, error against A, and the sweep kernel of each
    mode with the returned factor (bytes = one read of the tensor)."""
    import torch
    from workloads import synth
    A, _, _ = synth.tucker_lowrank_torch(2, (n,) * 3, (core,) * 3, 1e-3,
                                         decay=synth.decay_geom((core,) * 3, 0.9),
                                         device="cuda", out_dtype=torch.float32)
    ranks = (rank,) * 3
    out = {}
    for name, X in (("f32", A), ("bf16", None)):
        if X is None:
            X = A.to(torch.bfloat16)
        ws = torch.empty(tk.workspace_bytes("t", X.shape, X.dtype, ranks), dtype=torch.uint8,
                         device="cuda")
        G, Us, info = tk.als_thosvd(X, ranks, tol=tol, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            G, Us, info = tk.als_thosvd(X, ranks, tol=tol, workspace=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        e = relerr_gpu(tk, A, G, Us)
        kms = [time_sweep_kernel(tk, X, Us[m].contiguous(), launches=5, mode=m) for m in range(3)]
        nb = X.numel() * X.element_size()
        log(f"1024^3 {name}: t-HOSVD-ALS {dt*1e3:.2f} ms iters={info['iters']} relerr={e:.4e} "
            f"sweep kernels {['%.3f' % k for k in kms]} ms")
        out[f"large_{name}_ms_per_thosvd"] = round(dt * 1e3, 3)
        out[f"large_{name}_relerr"] = e
        out[f"large_{name}_iters"] = info["iters"]
        out[f"large_{name}_sweep_kernel_ms"] = [round(k, 4) for k in kms]
        out[f"large_{name}_sweep_gbs"] = [round(nb / (k * 1e-3) / 1e9, 1) for k in kms]
        del ws, G, Us
        if name == "bf16":
            del X
    out["large_bf16_speedup_vs_f32"] = round(out["large_f32_ms_per_thosvd"] /
                                             out["large_bf16_ms_per_thosvd"], 3)
    out["large_workload"] = ("t-HOSVD-ALS, 1024^3, core 64^3 N(0,1)0.9^(i+j+k) x orthonormal "
                             "1024x64 factors + 1e-3 relative noise, ranks (48,48,48), eta 1e-4")
    return out


def bench_batched(tk, steps, sample=64):
    """The 512-tensor batched workload (I_n in [16,128], R_n in [4,16], 1e-3 noise): one
    batched call (a replayed HIP graph of the persistent kernel) against the
    single-tensor driver on the first ``sample`` tensors, scaled to the batch."""
    import torch
    from workloads import synth
    items = synth.workload_batched(count=512)
    As = [torch.from_numpy(it["A"]).float().cuda() for it in items]
    ranks = [it["ranks"] for it in items]
    plan = tk.BatchedPlan(As, ranks)
    plan.run(tol=TOL)                       # autotune and capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(tol=TOL)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    res = plan.results()
    nbytes = sum(step_bytes(tuple(A.shape), r, it) for A, r, (_, _, it) in zip(As, ranks, res))
    for A, r in zip(As[:sample], ranks[:sample]):
        tk.als_sthosvd(A, r, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for A, r in zip(As[:sample], ranks[:sample]):
        tk.als_sthosvd(A, r, tol=TOL)
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) / sample * len(As)
    log(f"batched {dt*1e3:.3f} ms, single-tensor loop {seq*1e3:.1f} ms (scaled from {sample})")
    return dict(batched_ms=round(dt * 1e3, 3), batched_gbs=round(nbytes / dt / 1e9, 1),
                batched_input_mb=round(plan.algorithmic_bytes_per_pass / 1e6, 1),
                batched_single_loop_ms=round(seq * 1e3, 2),
                batched_speedup_vs_single=round(seq / dt, 2))


def cpu_baseline(A, ncols=8_000_000, sweeps=3):
    """Literal Algorithm 3.3 sweeps of the FP64 oracle on the first ``ncols``
    columns of the mode-1 unfolding (a 200 x ncols sample)."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import tucker_oracle as o
    An = A.reshape(A.shape[0], -1)[:, :ncols].double().cpu().numpy()
    L0 = o.als_initial_guess(An, o.init_sketch(0, 0, An.shape[1], RANK))
    t0 = time.perf_counter()
    o.als(An, RANK, L0, tol=0.0, max_iters=sweeps - 1, norm_ref=o.frob(An))
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    gbs = sweeps * An.shape[0] * An.shape[1] * 4 / dt / 1e9
    return dict(value=round(gbs, 4), unit="GB/s", cores=int(threads), kind="oracle",
                sample=f"{sweeps} literal ALS sweeps (Alg. 3.3, explicit residual) of the "
                       f"FP64 oracle on a 200 x {An.shape[1]} slice of the mode-1 unfolding; "
                       f"{dt:.1f} s; bytes counted as FP32 (4 B/element) per sweep")


def bench_paper_tucker(tk, steps, I=5000, eta=1e-4):
    """Section 6.1.2's largest case: I x 100^3 FP32, core (I/100, 10, 10, 10) with
    entries U[5, 10] times orthonormal factors plus 1e-4 absolute Gaussian noise
    (seeded, generated on the GPU); t- and st-HOSVD-ALS to the core dims."""
    import torch
    from workloads import synth
    log(f"generating the {I} x 100^3 Tucker test case on the GPU")
    Ah, A, _, _ = synth.tucker_paper_torch(6, I, out_dtype=torch.float32)
    del A
    torch.cuda.empty_cache()
    ranks = (max(1, round(0.01 * I)), 10, 10, 10)
    out = {"paper_tucker_workload": f"{I} x 100^3 FP32 ({Ah.numel() * 4 / 1e9:.1f} GB), core "
                                    f"{ranks} U[5,10] x orthonormal factors + 1e-4 absolute "
                                    f"noise, eta {eta}"}
    for which, run in (("st", tk.als_sthosvd), ("t", tk.als_thosvd)):
        G, Us, info = run(Ah, ranks, tol=eta)          # warm-up
        del G, Us
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            G, Us, info = run(Ah, ranks, tol=eta)
            del G, Us
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        log(f"{I} x 100^3 {which}-HOSVD-ALS: {dt * 1e3:.1f} ms, iters {info['iters']}")
        out[f"paper_tucker_{which}_ms"] = round(dt * 1e3, 2)
        out[f"paper_tucker_{which}_iters"] = info["iters"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^3 t-HOSVD leg")
    ap.add_argument("--only-large", action="store_true",
                    help="run the 1024^3 t-HOSVD leg alone (for profiling its kernels)")
    ap.add_argument("--paper-tucker", action="store_true",
                    help="time the paper's largest Tucker test case (5000 x 100^3) alone")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on exactly one GPU; runs on more than one GPU are not "
              "supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2004_02583_amd as tk
    from workloads import synth

    tk.load_library()
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration()
    if args.only_large:
        print(json.dumps(bench_large(tk, max(1, min(args.steps, 3)))), flush=True)
        return
    if args.paper_tucker:
        print(json.dumps(bench_paper_tucker(tk, max(1, min(args.steps, 3)))), flush=True)
        return
    log("generating 200^4 FP32 workload on the GPU")
    w = synth.workload_4way_torch(DIMS, RANK, 1e-4, device=dev)
    A = w["A"]
    ranks = w["ranks"]
    torch.cuda.synchronize()
    ws = torch.empty(tk.workspace_bytes("st", A.shape, A.dtype, ranks), dtype=torch.uint8,
                     device=dev)

    log("warmup")
    info = None
    for _ in range(args.warmup):
        G, Us, info = tk.als_sthosvd(A, ranks, tol=TOL, workspace=ws)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    iters_seen = []
    for _ in range(args.steps):
        G, Us, info = tk.als_sthosvd(A, ranks, tol=TOL, workspace=ws)
        iters_seen.append(tuple(info["iters"]))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    iters = list(iters_seen[-1])
    nbytes = step_bytes(DIMS, ranks, iters)
    value = nbytes / dt / 1e9
    e32 = relerr_gpu(tk, A, G, Us)
    log(f"fp32 step {dt*1e3:.2f} ms iters={iters} relerr={e32:.4e}")

    log("fused sweep kernel timing")
    Lq = Us[0].contiguous()
    k_ms = time_sweep_kernel(tk, A, Lq)
    sweep_bytes = A.numel() * A.element_size()
    achieved = sweep_bytes / (k_ms * 1e-3) / 1e9
    n_i, n_j, n_r = A.shape[0], A.numel() // A.shape[0], Lq.shape[1]
    sweep_flops = float(n_j) * (4.0 * n_i * n_r + 2.0 * n_r * n_r)
    tflops = sweep_flops / (k_ms * 1e-3) / 1e12

    extra = {}
    if not args.no_bf16:
        log("bf16 storage time-to-tolerance")
        Ab = A.to(torch.bfloat16)
        wsb = torch.empty(tk.workspace_bytes("st", Ab.shape, Ab.dtype, ranks),
                          dtype=torch.uint8, device=dev)
        for _ in range(args.warmup):
            Gb, Ub, infob = tk.als_sthosvd(Ab, ranks, tol=TOL, workspace=wsb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Gb, Ub, infob = tk.als_sthosvd(Ab, ranks, tol=TOL, workspace=wsb)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / args.steps
        eb = relerr_gpu(tk, A, Gb, Ub)
        kb_ms = time_sweep_kernel(tk, Ab, Ub[0].contiguous())
        extra = dict(bf16_ms_per_step=round(dtb * 1e3, 3), bf16_relerr=eb,
                     bf16_iters=infob["iters"], bf16_sweep_kernel_ms=round(kb_ms, 4),
                     bf16_speedup_vs_fp32=round(dt / dtb, 3))
        del Ab, wsb
        log(f"bf16 step {dtb*1e3:.2f} ms relerr={eb:.4e}")

    if not args.no_batched:
        log("batched st-HOSVD-ALS (512 tensors)")
        extra.update(bench_batched(tk, args.steps))

    if not args.no_large:
        log("1024^3 t-HOSVD-ALS, FP32 and BF16 storage")
        del G, Us
        if not args.no_bf16:
            del Gb, Ub
        torch.cuda.empty_cache()
        extra.update(bench_large(tk, max(1, min(args.steps, 3))))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(A)

    out = {
        "metric": "ALS sweep GB/s (% HBM peak); st-HOSVD time-to-tol vs plain FP32 at set error",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "st-HOSVD-ALS, 200^4 FP32, core 20^4 N(0,1)exp(-(i+j+k+l)/10) "
                               "x orthonormal 200x20 factors + 1e-4 relative noise",
                   "dims": list(DIMS), "ranks": list(ranks), "tol": TOL,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(tflops, 2),
                     "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP32_MFMA_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(), "kernel": "k_fused (ALS sweep, mode 1, FP32)",
                     "kernel_ms": round(k_ms, 4), "flops_per_launch": sweep_flops,
                     "bytes_per_launch": sweep_bytes, "hbm_gbs": round(achieved, 1),
                     "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu,
        "iters": iters,
        "relerr": e32,
        "step_bytes": nbytes,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
