"""Benchmark of the RandomizedNNLS hot path on one MI355X.

One step = one pass of the whole path over one instance resident in HBM:
random streams, sketch transform, reduce, FP64 moments, Lawson-Hanson and its
KKT certificate (rnnls_rand_nnls).  Default workload: the single instance at
scale, tf-idf-like A of 2^20 x 64 (1% mean density, Zipf(1.1) column
densities, lognormal values, L2-normalised columns, stored dense FP32),
b = A x* + 5% noise, r = 4096.

Prints one JSON line (metric, value = solves/s, roofline of the sketch kernel
from HIP events recorded on its launch stream, and the CPU oracle timed on a
bounded sample as a reported baseline).

    python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--no-cpu-baseline]
                    [--workload single_2p20x64|single_4096x16|single_2p22x128]
    python bench.py --copy-mib 1024   # plain copies only, to scale byte counters
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NNLS solves/s at ≤1e-2 rel. residual gap vs plain; SRHT GB/s vs HBM peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "srht_tiled_2p20x64_r4096_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_0812_4547_amd", "csrc", "srht.hip")

WORKLOADS = {
    # name: (n, d, r, data seed, sketch seed)
    "single_2p20x64": (1 << 20, 64, 4096, 2, 2),
    "single_4096x16": (4096, 16, 512, 1, 1),
    "single_2p22x128": (1 << 22, 128, 8192, 3, 3),
}
# batching forms: 256 uneven tf-idf-like instances (n log-uniform in
# [2^14, 2^18], d uniform in [8, 96], r = max(32 d, 1024)), and one A of
# 2^20 x 64 with 512 right-hand sides (r = 2048)
BATCH_WORKLOADS = ("batch_256", "multi_2p20x64_k512", "learned_4096", "fig1_2p20x64",
                   "boost_2p20x64_k4", "nmf_2p16x2048_q32", "density_sweep_1e4x128",
                   "box_2p20x64")

# oracle instances per cpu_baseline sample (about 10-30 s on one host core)
CPU_SAMPLES = {"single_2p20x64": 6, "single_4096x16": 1500, "single_2p22x128": 1}

CPU_SAMPLE = r"""
import json, sys, time
sys.path.insert(0, {root!r})
from paper_0812_4547_amd import workloads
from oracle import rand_nnls
n, d, r, ds = {n}, {d}, {r}, {ds}
p = workloads.uniform_planted(n=n, d=d, seed=ds) if {planted} else workloads.tfidf_like(n, d, seed=ds)
seeds = {seeds}
t0 = time.perf_counter()
for s in seeds:
    rand_nnls.rand_nnls(p.A, p.b, r, s)
dt = time.perf_counter() - t0
print(json.dumps({{"seconds": dt, "instances": len(seeds)}}))
"""


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch of the sketch kernel from the committed rocprofv3
    counter summary, or None when absent or taken on different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(n, d, r, ds, planted, nsamples):
    seeds = [1000 + i for i in range(nsamples)]
    code = CPU_SAMPLE.format(root=ROOT, n=n, d=d, r=r, ds=ds, planted=planted, seeds=seeds)
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=600)
    if out.returncode != 0:
        raise RuntimeError("cpu baseline failed: " + out.stderr[-2000:])
    res = json.loads(out.stdout.strip().splitlines()[-1])
    return {
        "value": res["instances"] / res["seconds"],
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{res['instances']} full instances of the same workload (sketch seeds "
                  f"{seeds[0]}..{seeds[-1]}), FP64 numpy oracle, one thread, "
                  f"{res['seconds']:.1f} s",
    }


CPU_BATCH_SAMPLE = r"""
import json, sys, time
sys.path.insert(0, {root!r})
from paper_0812_4547_amd import workloads
from oracle import rand_nnls
shapes = workloads.batch_shapes()[:{count}]
probs = [workloads.batch_instance(i, n, d) for i, (n, d, r) in enumerate(shapes)]
t0 = time.perf_counter()
for i, ((n, d, r), p) in enumerate(zip(shapes, probs)):
    rand_nnls.rand_nnls(p.A, p.b, r, 1000 + i)
dt = time.perf_counter() - t0
print(json.dumps({{"seconds": dt, "instances": len(shapes)}}))
"""

CPU_MULTI_SAMPLE = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, {root!r})
from paper_0812_4547_amd import workloads
from oracle import hadamard, nnls
A, B, _ = workloads.tfidf_multi_rhs(1 << 20, 64, 512, seed=4)
k = {count}
t0 = time.perf_counter()
Y, _, _, _ = hadamard.srht_sketch(np.column_stack([A, B[:, :k]]).astype(np.float64), None, 2048, 4)
for j in range(k):
    nnls.lawson_hanson(Y[:, :64], Y[:, 64 + j])
dt = time.perf_counter() - t0
print(json.dumps({{"seconds": dt, "instances": k}}))
"""


def _run_cpu_sample(code, what):
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=600)
    if out.returncode != 0:
        raise RuntimeError("cpu baseline failed: " + out.stderr[-2000:])
    res = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": res["instances"] / res["seconds"], "unit": "solves/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{what}: {res['instances']} solves, FP64 numpy oracle, one thread, "
                      f"{res['seconds']:.1f} s"}


def _timed(fn, steps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def read_stream_peak(mib=1024, reps=20):
    """GB/s of the library's streaming-read reference kernel over a buffer of
    `mib` MiB (larger than the 256 MB last-level cache): the practical read
    ceiling the sketch's HBM fraction is also stated against."""
    import torch

    from paper_0812_4547_amd import rnnls
    x = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    parts = rnnls.stream_read(x)
    for _ in range(3):
        rnnls.stream_read(x, parts)
    torch.cuda.synchronize()
    rnnls.timing_enable(True)
    rnnls.timing_read(rnnls.TIMER_STREAM_READ)
    for _ in range(reps):
        rnnls.stream_read(x, parts)
    torch.cuda.synchronize()
    ms, k = rnnls.timing_read(rnnls.TIMER_STREAM_READ)
    rnnls.timing_enable(False)
    if abs(float(parts.double().sum().item()) - x.numel()) > 1e-3 * x.numel():
        raise RuntimeError("streaming-read reference returned a wrong sum")
    del x
    return (mib << 20) / (ms / max(k, 1) * 1e-3) / 1e9


def _with_read_peak(roof):
    """Add the measured streaming-read ceiling to a roofline record."""
    peak = read_stream_peak()
    roof["read_stream_peak"] = peak
    roof["frac_of_read_stream"] = roof["achieved"] / peak
    return roof


def _base_record(args, value, ms, config, dtype="f32"):
    return {"metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def bench_batch(args):
    """One step = one pass of the batch plan (graph replay) over 256 uneven
    instances resident in HBM."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls, workloads
    shapes = workloads.batch_shapes()
    probs, dev = [], []
    alg = 0
    for i, (n, d, r) in enumerate(shapes):
        p = workloads.batch_instance(i, n, d)
        A = rnnls.colmajor(p.A)
        b = torch.from_numpy(p.b).cuda()
        dev.append((A, b, r, 1000 + i))
        probs.append(p)
        alg += 4 * n * (d + 1) + 4 * r * (d + 1)
    del probs
    batch = rnnls.Batch(dev)
    stream = torch.cuda.current_stream()
    batch.run()
    torch.cuda.synchronize()
    eager_ms_default = _timed(batch.run, max(3, args.steps // 5), stream)
    choice = batch.autotune()
    batch.capture()
    for _ in range(args.warmup):
        batch.launch()
    ms = _timed(batch.launch, args.steps, stream)
    eager_ms = _timed(batch.run, max(3, args.steps // 5), stream)
    # sketch stage alone, eager, with the library's event timers
    rnnls.timing_enable(True)
    for t in (rnnls.TIMER_SKETCH, rnnls.TIMER_MOMENTS, rnnls.TIMER_SOLVE):
        rnnls.timing_read(t)
    reps = 5
    for _ in range(reps):
        batch.run()
    torch.cuda.synchronize()
    sk_ms, sk_n = rnnls.timing_read(rnnls.TIMER_SKETCH)
    mo_ms, _ = rnnls.timing_read(rnnls.TIMER_MOMENTS)
    lh_ms, _ = rnnls.timing_read(rnnls.TIMER_SOLVE)
    rnnls.timing_enable(False)
    st = batch.status.cpu().numpy()
    sketch_ms = sk_ms / reps
    achieved = alg / (sketch_ms * 1e-3) / 1e9
    rec = _base_record(args, len(shapes) * 1000.0 / ms, ms, {
        "workload": f"batch of {len(shapes)} tf-idf-like instances, n log-uniform in "
                    f"[2^14, 2^18], d uniform in [8, 96], r = max(32 d, 1024)",
        "instances": len(shapes), "batch_seed": 4, "sketch_seeds": "1000 + i",
        "algorithmic_bytes": alg, "autotuned_tile": list(choice),
        "launch": "hipGraph replay of the batch plan"})
    rec["roofline"] = _with_read_peak({
        "kernel": "srht_tiled_kernel (all sketch launches of the pass)",
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
        "algorithmic_bytes_per_pass": alg, "sketch_ms_per_pass": sketch_ms,
        "sketch_launches_per_pass": sk_n / reps})
    rec["breakdown_ms_per_pass_eager"] = {"sketch": sketch_ms, "moments": mo_ms / reps,
                                          "lawson_hanson": lh_ms / reps}
    rec["eager_ms_per_pass"] = eager_ms
    rec["eager_ms_per_pass_default_tile"] = eager_ms_default
    rec["status_ok"] = int((st == 0).sum())
    batch.close()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = _run_cpu_sample(
            CPU_BATCH_SAMPLE.format(root=ROOT, count=args.cpu_samples or 12),
            "the first instances of the same batch")
    print(json.dumps(rec), flush=True)


def bench_multi(args):
    """One step = Algorithm 1 for 512 right-hand sides sharing one A of
    2^20 x 64 (one sketch, one G, 512 Lawson-Hanson solves)."""
    import torch

    from paper_0812_4547_amd import rnnls, workloads
    n, d, k, r = 1 << 20, 64, 512, 2048
    A_h, B_h, _ = workloads.tfidf_multi_rhs(n, d, k, seed=4)
    A = rnnls.colmajor(A_h)
    B = rnnls.colmajor(B_h)
    del A_h, B_h
    ws = rnnls.multi_workspace(n, d, k, r)
    out = rnnls.rand_nnls_multi(A, B, r, 4, ws=ws)
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        rnnls.rand_nnls_multi(A, B, r, 4 + i, ws=ws, out=out)
    it = iter(range(10**9))
    ms = _timed(lambda: rnnls.rand_nnls_multi(A, B, r, 4 + next(it), ws=ws, out=out),
                args.steps, stream)
    # per-kernel durations from a second run of the same steps with events
    rnnls.timing_enable(True)
    for t in (rnnls.TIMER_SKETCH, rnnls.TIMER_MOMENTS, rnnls.TIMER_SOLVE):
        rnnls.timing_read(t)
    it = iter(range(10**9))
    _timed(lambda: rnnls.rand_nnls_multi(A, B, r, 4 + next(it), ws=ws, out=out), args.steps, stream)
    sk_ms, sk_n = rnnls.timing_read(rnnls.TIMER_SKETCH)
    mo_ms, _ = rnnls.timing_read(rnnls.TIMER_MOMENTS)
    lh_ms, _ = rnnls.timing_read(rnnls.TIMER_SOLVE)
    rnnls.timing_enable(False)
    alg = 4 * n * (d + k) + 4 * r * (d + k)
    sk = sk_ms / max(sk_n, 1)
    achieved = alg / (sk * 1e-3) / 1e9
    st = out.status.cpu().numpy()
    rec = _base_record(args, k * 1000.0 / ms, ms, {
        "workload": "tf-idf-like A 2^20 x 64 FP32 with 512 right-hand sides B = A X* + 5% "
                    "noise (nonnegative-factorisation-style update), r = 2048",
        "n": n, "d": d, "k": k, "r": r, "data_seed": 4})
    rec["roofline"] = _with_read_peak({
        "kernel": "srht_tiled_kernel", "bound": "hbm", "achieved": achieved,
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": None, "algorithmic_bytes_per_launch": alg, "avg_launch_ms": sk})
    rec["breakdown_ms_per_step"] = {"sketch_kernel": sk_ms / args.steps,
                                    "moments": mo_ms / args.steps,
                                    "lawson_hanson": lh_ms / args.steps}
    rec["status_ok"] = int((st == 0).sum())
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = _run_cpu_sample(
            CPU_MULTI_SAMPLE.format(root=ROOT, count=args.cpu_samples or 8),
            "one FP64 sketch of [A | 8 right-hand sides] and their 8 solves")
    print(json.dumps(rec), flush=True)


def bench_learned(args):
    """Learned warm start: collect features and passive labels from problems of
    the batch generator solved cold on the device, train the perceptron with
    the device kernels, then solve held-out problems cold and warm-started
    (KKT-judged).  One step = one pass of a 1024-problem batch plan."""
    import torch

    from paper_0812_4547_amd import learned, rnnls
    train_count = args.train_instances
    t0 = time.perf_counter()
    Xs, ys, ok = [], [], True
    chunk = 1024
    for c0 in range(0, train_count, chunk):
        X, y, o = learned.collect(min(chunk, train_count - c0), seed=100 + c0 // chunk)
        Xs.append(X)
        ys.append(y)
        ok = ok and o
        print(f"collected {c0 + chunk} / {train_count} training problems "
              f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    X = torch.cat(Xs)
    y = torch.cat(ys)
    collect_s = time.perf_counter() - t0
    mlp = rnnls.Mlp(learned.init_params(1))
    t1 = time.perf_counter()
    hist = learned.train(mlp, X, y, epochs=args.epochs, batch_rows=8192, lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    prob, _ = mlp.forward(X)
    acc = float(((prob > 0.5).to(torch.uint8) == y).double().mean().item())
    print(f"trained: loss {hist[0]:.4f} -> {hist[-1]:.4f}, accuracy {acc:.4f}",
          file=sys.stderr, flush=True)
    ev = learned.evaluate(mlp, args.heldout, seed=2_000_000, chunk=1024, reps=max(1, args.steps))
    rec = _base_record(args, args.heldout * 1000.0 / ev.warm_ms, ev.warm_ms / (args.heldout / 1024),
                       {"workload": f"learned warm start: {train_count} training and "
                                    f"{args.heldout} held-out problems of the batch generator "
                                    "(n log-uniform in [2^14, 2^18], d uniform in [8, 96], "
                                    "r = max(32 d, 1024)), device-generated tf-idf-like data",
                        "network": "8-128-128-1 perceptron, BF16 weights, FP32 accumulation",
                        "step": "one eager pass of a 1024-problem batch plan"})
    rec["vs_cold"] = {"warm_solves_per_s": args.heldout * 1000.0 / ev.warm_ms,
                      "cold_solves_per_s": args.heldout * 1000.0 / ev.cold_ms,
                      "speedup": ev.cold_ms / ev.warm_ms,
                      "lawson_hanson_ms_cold": ev.cold_lh_ms, "lawson_hanson_ms_warm": ev.warm_lh_ms,
                      "outer_iterations_cold": ev.cold_iters, "outer_iterations_warm": ev.warm_iters,
                      "warm_start_kept": ev.warm_kept,
                      "max_rel_residual_gap_vs_cold": ev.max_gap, "all_status_ok": ev.all_ok}
    rec["training"] = {"rows": int(X.shape[0]), "epochs": args.epochs, "loss_first": hist[0],
                       "loss_last": hist[-1], "train_accuracy": acc, "collect_s": collect_s,
                       "train_s": train_s, "labels_all_ok": ok}
    print(json.dumps(rec), flush=True)


def bench_fig1(args):
    """Figure 1's comparison on the tf-idf-like 2^20 x 64 workload: for
    r = d + 50 i (i = 1..8), the randomized solve's time split into
    preprocessing (signs and rows, sketch, moments) and small problem
    (Lawson-Hanson), beside the exact NNLS of the whole problem (moments over
    all n rows, then Lawson-Hanson), and the relative error of x~ (residual
    ratio minus one, Figure 1's measure).  One step = one randomized solve at
    the largest r; every point is a mean over `steps` solves."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls, workloads
    n, d, ds = 1 << 20, 64, 2
    p = workloads.tfidf_like(n, d, seed=ds)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    stream = torch.cuda.current_stream()
    timers = (rnnls.TIMER_SKETCH, rnnls.TIMER_MOMENTS, rnnls.TIMER_SOLVE)

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ms = _timed(fn, reps, stream)  # without per-kernel events
        rnnls.timing_enable(True)
        for t in timers:
            rnnls.timing_read(t)
        _timed(fn, reps, stream)       # the same calls again, for the solve's share
        lh_ms, _ = rnnls.timing_read(rnnls.TIMER_SOLVE)
        for t in timers[:2]:
            rnnls.timing_read(t)
        rnnls.timing_enable(False)
        return ms, lh_ms / reps

    ws_plain = rnnls.workspace(rnnls.OP_SOLVE, n, d, 0)
    plain = rnnls.nnls_solve(A, b, ws=ws_plain)
    plain_ms, plain_lh = timed(lambda: rnnls.nnls_solve(A, b, ws=ws_plain), max(3, args.steps // 5))
    xp = plain.x.cpu().numpy()
    res_plain = float(np.linalg.norm(A64 @ xp - b64))
    rows = []
    for i in range(1, 9):
        r = d + 50 * i
        ws = rnnls.workspace(rnnls.OP_RAND_NNLS, n, d, r)
        out = rnnls.rand_nnls(A, b, r, 1000, ws=ws)
        it = iter(range(10**9))
        ms, lh = timed(lambda: rnnls.rand_nnls(A, b, r, 1000 + next(it), ws=ws, out=out), args.steps)
        errs = []
        for s in range(5):
            x = rnnls.rand_nnls(A, b, r, 2000 + s, ws=ws).x.cpu().numpy()
            errs.append(float(np.linalg.norm(A64 @ x - b64)) / res_plain - 1.0)
        rows.append({"r": r, "overall_ms": ms, "preprocessing_ms": ms - lh, "small_problem_ms": lh,
                     "relative_error_mean": float(np.mean(errs)),
                     "relative_error_max": float(np.max(errs)), "error_seeds": 5,
                     "status": int(out.status.item())})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    last = rows[-1]
    rec = _base_record(args, 1000.0 / last["overall_ms"], last["overall_ms"], {
        "workload": f"Figure 1-shaped comparison on tf-idf-like A {n}x{d} FP32: "
                    "r = d + 50 i, i = 1..8, against the exact NNLS of the whole problem",
        "n": n, "d": d, "data_seed": ds, "r_values": [row["r"] for row in rows],
        "step": "one randomized solve at the largest r"})
    rec["plain_full"] = {"overall_ms": plain_ms, "moments_ms": plain_ms - plain_lh,
                         "small_problem_ms": plain_lh, "status": int(plain.status.item()),
                         "residual": res_plain}
    rec["fig1"] = rows
    print(json.dumps(rec), flush=True)


def bench_boost(args):
    """Repetition on the single-instance workload: one step = Algorithm 1 with
    four seeds on tf-idf-like A 2^20 x 64 (r = 4096) plus the one pass over A
    that forms the four full residuals and keeps the least."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls, workloads
    n, d, r, k, ds = 1 << 20, 64, 4096, 4, 2
    p = workloads.tfidf_like(n, d, seed=ds)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    ws = rnnls.boost_workspace(n, d, r, k)
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        rnnls.rand_nnls_boost(A, b, r, k, 100 * i, ws=ws)
    torch.cuda.synchronize()
    it = iter(range(10**9))
    ms = _timed(lambda: rnnls.rand_nnls_boost(A, b, r, k, 1000 + k * next(it), ws=ws),
                args.steps, stream)
    # the residual kernel's duration from a second run of the same steps with events
    rnnls.timing_enable(True)
    rnnls.timing_read(rnnls.TIMER_RESIDUAL)
    it = iter(range(10**9))
    _timed(lambda: rnnls.rand_nnls_boost(A, b, r, k, 1000 + k * next(it), ws=ws), args.steps, stream)
    res_ms, res_n = rnnls.timing_read(rnnls.TIMER_RESIDUAL)
    rnnls.timing_enable(False)
    res_avg = res_ms / max(res_n, 1)
    alg = 4 * n * (d + 1)
    achieved = alg / (res_avg * 1e-3) / 1e9
    out = rnnls.rand_nnls_boost(A, b, r, k, 7, ws=ws)
    torch.cuda.synchronize()
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    plain = rnnls.nnls_solve(A, b)
    res_plain = float(np.linalg.norm(A64 @ plain.x.cpu().numpy() - b64))
    resid = out.resid.cpu().numpy()[:k]
    rec = _base_record(args, 1000.0 / ms, ms, {
        "workload": f"repetition of Algorithm 1: {k} seeds on tf-idf-like A {n}x{d} FP32, "
                    f"r = {r}, keeping the least full residual",
        "n": n, "d": d, "r": r, "k": k, "data_seed": ds})
    rec["roofline"] = _with_read_peak({
        "kernel": "boost_residual_kernel", "bound": "hbm", "achieved": achieved,
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
        "algorithmic_bytes_per_launch": alg, "avg_launch_ms": res_avg, "launches": res_n})
    rec["quality"] = {"residual_loss_kept_vs_plain_full_nnls": float(resid.min()) / res_plain - 1.0,
                      "residual_loss_per_seed": [float(v) / res_plain - 1.0 for v in resid],
                      "kept": int(out.best.item()), "status": int(out.status.item())}
    print(json.dumps(rec), flush=True)


def bench_box(args):
    """Box constraints on the same sketch: one step = Algorithm 1 on tf-idf-like
    A 2^20 x 64 (r = 4096) with 0 <= x <= 0.5 in step 5 (rnnls_rand_box)."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls, workloads
    n, d, r, ds, ub = 1 << 20, 64, 4096, 2, 0.5
    p = workloads.tfidf_like(n, d, seed=ds)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    lo = torch.zeros(d, dtype=torch.float64, device="cuda")
    hi = torch.full((d,), ub, dtype=torch.float64, device="cuda")
    ws = rnnls.workspace(rnnls.OP_RAND_NNLS, n, d, r)
    out = rnnls.Solution(torch.empty(d, dtype=torch.float64, device="cuda"), None,
                         torch.empty(1, dtype=torch.float64, device="cuda"),
                         torch.empty(1, dtype=torch.int32, device="cuda"),
                         torch.empty(1, dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        rnnls.rand_box(A, b, r, 100 + i, lo, hi, ws=ws, out=out)
    torch.cuda.synchronize()
    it = iter(range(10**9))
    ms = _timed(lambda: rnnls.rand_box(A, b, r, 1000 + next(it), lo, hi, ws=ws, out=out),
                args.steps, stream)
    rnnls.timing_enable(True)
    for t in (rnnls.TIMER_SKETCH, rnnls.TIMER_MOMENTS, rnnls.TIMER_SOLVE):
        rnnls.timing_read(t)
    it = iter(range(10**9))
    _timed(lambda: rnnls.rand_box(A, b, r, 1000 + next(it), lo, hi, ws=ws, out=out),
           args.steps, stream)
    sk_ms, sk_n = rnnls.timing_read(rnnls.TIMER_SKETCH)
    mo_ms, mo_n = rnnls.timing_read(rnnls.TIMER_MOMENTS)
    so_ms, so_n = rnnls.timing_read(rnnls.TIMER_SOLVE)
    rnnls.timing_enable(False)
    sk_avg = sk_ms / max(sk_n, 1)
    alg = 4 * n * (d + 1) + 4 * r * (d + 1)
    achieved = alg / (sk_avg * 1e-3) / 1e9
    rnnls.rand_box(A, b, r, 7, lo, hi, ws=ws, out=out)
    torch.cuda.synchronize()
    x = out.x.cpu().numpy()
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    plain = rnnls.rand_nnls(A, b, r, 7)
    torch.cuda.synchronize()
    rec = _base_record(args, 1000.0 / ms, ms, {
        "workload": f"Algorithm 1 with box bounds 0 <= x <= {ub} in step 5 on tf-idf-like A "
                    f"{n}x{d} FP32, r = {r}", "n": n, "d": d, "r": r, "data_seed": ds})
    rec["unit"] = "box solves/s"
    rec["roofline"] = _with_read_peak({
        "kernel": "srht_tiled_kernel", "bound": "hbm", "achieved": achieved,
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
        "algorithmic_bytes_per_launch": alg, "avg_launch_ms": sk_avg, "launches": sk_n})
    rec["breakdown_ms"] = {"sketch": sk_avg, "moments": mo_ms / max(mo_n, 1),
                           "box_solve": so_ms / max(so_n, 1)}
    rec["quality"] = {
        "status": int(out.status.item()), "outer_steps": int(out.iters.item()),
        "at_lower": int(np.sum(x == 0.0)), "at_upper": int(np.sum(x == ub)),
        "free": int(np.sum((x > 0.0) & (x < ub))),
        "full_residual_over_norm_b": float(np.linalg.norm(A64 @ x - b64) / np.linalg.norm(b64)),
        "unbounded_algorithm1_residual_over_norm_b":
            float(np.linalg.norm(A64 @ plain.x.cpu().numpy() - b64) / np.linalg.norm(b64))}
    print(json.dumps(rec), flush=True)


def bench_nmf(args):
    """Nonnegative factorisation by alternating NNLS, each half-step Algorithm 1
    for many right-hand sides: tf-idf-like A 2^16 x 2048, rank 32.  One step =
    one iteration (an H half-step of 2048 problems on 2^16 rows and a W
    half-step of 2^16 problems on 2048 rows, in chunks of 4096)."""
    import torch

    from paper_0812_4547_amd import nmf, rnnls, workloads
    m, n, q, r_h, r_w = 1 << 16, 2048, 32, 1024, 512
    p = workloads.tfidf_like(m, n, seed=6)
    A = rnnls.colmajor(p.A)
    del p
    stream = torch.cuda.current_stream()
    res = nmf.nmf_als(A, q, max(1, args.warmup), r_h, r_w, seed=1)
    W0 = res.W
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = nmf.nmf_als(A, q, args.steps, r_h, r_w, seed=1, W0=W0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    rec = _base_record(args, (m + n) * 1000.0 / ms, ms, {
        "workload": f"nonnegative factorisation by alternating NNLS of tf-idf-like A {m}x{n}, "
                    f"rank {q}, sketch rows {r_h} (H half-step) and {r_w} (W half-step)",
        "m": m, "n": n, "q": q, "r_h": r_h, "r_w": r_w, "data_seed": 6,
        "step": "one iteration (m + n NNLS solves)"})
    rec["sketched_objective_per_half_step"] = res.sketched_objective
    rec["frobenius_norm_of_A"] = float(torch.linalg.vector_norm(A).item())
    print(json.dumps(rec), flush=True)


def bench_density(args):
    """The sparse-versus-dense experiment (Section 4.2) with d = 128 (this
    solver's limit; the paper uses 300): n = 10,000, densities 2..64%, for each
    density 10 random n x (d+1) matrices (nonzeros uniform in [0, 1]) and 10
    choices of the column that becomes b (100 problems); r = d, d+50, d+100,
    d+150 in both sampling modes, against the exact solve on all n rows.
    Relative error = residual ratio minus one; times are GPU means per solve."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls, workloads
    n, d = 10_000, 128
    densities = (0.02, 0.04, 0.08, 0.16, 0.32, 0.64)
    rs = (d, d + 50, d + 100, d + 150)
    stream = torch.cuda.current_stream()
    rows = []
    for di, dens in enumerate(densities):
        probs = []
        for mi in range(10):
            M = workloads.density_matrix(n, d + 1, dens, seed=1000 * di + mi)
            g = np.random.default_rng(5000 + 10 * di + mi)
            for col in g.choice(d + 1, size=10, replace=False):
                p = workloads.density_problem(M, int(col))
                probs.append((rnnls.colmajor(p.A), torch.from_numpy(p.b).cuda(),
                              p.A.astype(np.float64), p.b.astype(np.float64)))
        ws_plain = rnnls.workspace(rnnls.OP_SOLVE, n, d, 0)
        plain = [rnnls.nnls_solve(A, b, ws=ws_plain) for A, b, _, _ in probs]
        torch.cuda.synchronize()
        exact_ms = _timed(lambda: [rnnls.nnls_solve(A, b, ws=ws_plain) for A, b, _, _ in probs],
                          1, stream) / len(probs)
        res_plain = [float(np.linalg.norm(A64 @ s.x.cpu().numpy() - b64))
                     for (_, _, A64, b64), s in zip(probs, plain)]
        for mode in ("bernoulli", "exact"):
            opts = rnnls.make_opts(mode)
            for r in rs:
                ws = rnnls.workspace(rnnls.OP_RAND_NNLS, n, d, r, opts)
                sols = [rnnls.rand_nnls(A, b, r, 7 + i, opts=opts, ws=None)
                        for i, (A, b, _, _) in enumerate(probs)]
                torch.cuda.synchronize()
                ms = _timed(lambda: [rnnls.rand_nnls(A, b, r, 7 + i, opts=opts, ws=ws)
                                     for i, (A, b, _, _) in enumerate(probs)], 1, stream) / len(probs)
                err = [float(np.linalg.norm(A64 @ s.x.cpu().numpy() - b64)) / rp - 1.0
                       for (_, _, A64, b64), s, rp in zip(probs, sols, res_plain)]
                ok = sum(int(s.status.item()) == 0 for s in sols)
                rows.append({"density": dens, "mode": mode, "r": r, "problems": len(probs),
                             "relative_error_mean": float(np.mean(err)),
                             "relative_error_max": float(np.max(err)), "status_ok": ok,
                             "rand_ms": ms, "exact_full_ms": exact_ms,
                             "speedup_vs_exact_full": exact_ms / ms})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    last = rows[-1]
    rec = _base_record(args, 1000.0 / last["rand_ms"], last["rand_ms"], {
        "workload": "sparse-versus-dense experiment: n = 10,000, d = 128, densities 2..64%, "
                    "100 problems per density, r = d + 50 i (i = 0..3), both sampling modes",
        "n": n, "d": d, "densities": list(densities), "r_values": list(rs),
        "step": "one randomized solve (density 64%, exact mode, r = d + 150)"})
    rec["sweep"] = rows
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="single_2p20x64",
                    choices=sorted(WORKLOADS) + list(BATCH_WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=0,
                    help="instances the oracle times (default: about 10-30 s of CPU work)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "split_bf16"],
                    help="sketch transform: FP32 vector units, or BF16 matrix cores with "
                         "split hi + lo operands and FP32 accumulation")
    ap.add_argument("--train-instances", type=int, default=100_000)
    ap.add_argument("--heldout", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run 5 plain device copies of this many MiB (the "
                         "reference kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU: --gpus must be 1 (sharding "
                                   "across GPUs is not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls, workloads

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written":
                          dst.numel() * 4, "launches": 5}), flush=True)
        return

    if args.workload == "batch_256":
        return bench_batch(args)
    if args.workload == "multi_2p20x64_k512":
        return bench_multi(args)
    if args.workload == "learned_4096":
        return bench_learned(args)
    if args.workload == "fig1_2p20x64":
        return bench_fig1(args)
    if args.workload == "boost_2p20x64_k4":
        return bench_boost(args)
    if args.workload == "nmf_2p16x2048_q32":
        return bench_nmf(args)
    if args.workload == "box_2p20x64":
        return bench_box(args)
    if args.workload == "density_sweep_1e4x128":
        return bench_density(args)

    n, d, r, ds, ss = WORKLOADS[args.workload]
    planted = args.workload == "single_4096x16"
    p = workloads.uniform_planted(n=n, d=d, seed=ds) if planted else workloads.tfidf_like(n, d, seed=ds)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    opts = rnnls.make_opts(precision=args.precision)
    ws = rnnls.workspace(rnnls.OP_RAND_NNLS, n, d, r, opts)
    out = rnnls.Solution(torch.empty(d, dtype=torch.float64, device="cuda"), None,
                         torch.empty(1, dtype=torch.float64, device="cuda"),
                         torch.empty(1, dtype=torch.int32, device="cuda"),
                         torch.empty(1, dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        rnnls.rand_nnls(A, b, r, ss + i, opts=opts, ws=ws, out=out)
    torch.cuda.synchronize()

    # the timed steps run without the library's per-kernel events (two event
    # records around each timed launch lengthen a step by several percent)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        rnnls.rand_nnls(A, b, r, ss + i, opts=opts, ws=ws, out=out)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = start.elapsed_time(stop)
    # the same steps again with every launch of the sketch, moments and solve
    # bracketed by HIP events on its stream: per-kernel durations
    rnnls.timing_enable(True)
    for t in (rnnls.TIMER_SKETCH, rnnls.TIMER_MOMENTS, rnnls.TIMER_SOLVE):
        rnnls.timing_read(t)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for i in range(args.steps):
        rnnls.rand_nnls(A, b, r, ss + i, opts=opts, ws=ws, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_timed_total = t0.elapsed_time(t1)
    sk_ms, sk_n = rnnls.timing_read(rnnls.TIMER_SKETCH)
    mo_ms, mo_n = rnnls.timing_read(rnnls.TIMER_MOMENTS)
    lh_ms, lh_n = rnnls.timing_read(rnnls.TIMER_SOLVE)
    rnnls.timing_enable(False)
    status = int(out.status.item())

    ms_per_step = ms_total / args.steps
    sk_avg = sk_ms / max(sk_n, 1)
    alg_bytes = 4 * n * (d + 1) + 4 * r * (d + 1)
    achieved = alg_bytes / (sk_avg * 1e-3) / 1e9
    traffic = load_traffic() if (args.precision == "fp32" and args.workload == "single_2p20x64") else None

    # quality of x~ (untimed): the paper's residual loss against the exact NNLS
    # of the whole problem, both solved on the GPU (nnls_solve on all n rows is
    # the plain path), residuals in FP64 on the host
    sol = rnnls.rand_nnls(A, b, r, ss, opts=opts)
    plain = rnnls.nnls_solve(A, b, opts=opts)
    torch.cuda.synchronize()
    A64 = p.A.astype(np.float64)
    b64 = p.b.astype(np.float64)
    res_sk = float(np.linalg.norm(A64 @ sol.x.cpu().numpy() - b64))
    res_pl = float(np.linalg.norm(A64 @ plain.x.cpu().numpy() - b64))
    loss = res_sk / res_pl - 1.0

    rec = {
        "metric": METRIC,
        "value": 1000.0 / ms_per_step,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x2-f32acc",
        "data": "synthetic",
        "config": {
            "workload": (f"single RandomizedNNLS instance, tf-idf-like A {n}x{d} FP32 dense, "
                         f"r={r}") if not planted else f"single instance, U[0,1] A {n}x{d}, r={r}",
            "n": n, "d": d, "r": r, "data_seed": ds, "sketch_seed_first": ss,
            "sample_mode": "exact",
            "precision": ("sketch f32" if args.precision == "fp32" else
                          "sketch: two Hadamard factors on BF16 matrix cores (x = hi + lo, FP32 "
                          "accumulate), third factor and combine f32") +
                         ", moments and Lawson-Hanson f64",
        },
        "roofline": {
            "kernel": "srht_tiled_kernel" if args.precision == "fp32" else "srht_mfma_kernel",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "avg_launch_ms": sk_avg,
            "launches": sk_n,
        },
        "breakdown_ms_per_step": {
            "sketch_kernel": sk_ms / args.steps,
            "moments": mo_ms / args.steps,
            "lawson_hanson": lh_ms / args.steps,
            "other": ms_timed_total / args.steps - (sk_ms + mo_ms + lh_ms) / args.steps,
            "note": "from a second run of the same steps with per-kernel events "
                    f"({ms_timed_total / args.steps:.4f} ms per step there)",
        },
        "wall_s": wall,
        "last_status": status,
        "quality": {
            "residual_loss_vs_plain_full_nnls": loss,
            "rand_status": int(sol.status.item()),
            "plain_status": int(plain.status.item()),
        },
    }
    _with_read_peak(rec["roofline"])
    if not args.no_cpu_baseline:
        ns = args.cpu_samples or CPU_SAMPLES[args.workload]
        rec["cpu_baseline"] = cpu_baseline(n, d, r, ds, planted, ns)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
