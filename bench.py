"""Benchmark of the RandomizedNNLS hot path on one MI355X.

Default workload (the metric's configuration): batched, warm-started solves.
A passive-set perceptron is trained on the device from 100k problems of the
batch generator solved cold by the method itself; 4096 held-out problems of
the same generator (n log-uniform in [2^14, 2^18], d uniform in [8, 96],
r = max(32 d, 1024), tf-idf-like entries), all resident in HBM, run as one
batch plan of 4096 problems replayed as a HIP graph (--plan-size 256 runs 16
plans of 256).  One step = one pass over all 4096 problems.  `value` = warm-started solves/s; beside it the plain
cold-start rate of the same plans, the relative residual gap of every
warm-started solution against the cold one on the same sketch (max, mean),
the fallback rate and the outer iterations.  The `roofline` is the sketch
kernel's over the pass, stated for the transform kernel alone and for the
whole sketch (random streams + transform + reduce); `single_2p20x64` adds the
single instance at scale (tf-idf-like 2^20 x 64, r = 4096) with warm- and
cold-cache medians of the sketch over 50 repetitions.  `cpu_baseline` is the
FP64 oracle on a bounded sample of the held-out problems, on all host cores.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
                    [--workload warm_batch_4096|single_2p20x64|...]
    python bench.py --copy-mib 1024   # plain copies only, to scale byte counters
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import shutil
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NNLS solves/s at ≤1e-2 rel. residual gap vs plain; SRHT GB/s vs HBM peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "srht_tiled_2p20x64_r4096_traffic.json")
TRAFFIC_FILE_BATCH = os.path.join(ROOT, "profiles", "srht_tiled_warm_batch_4096_traffic.json")
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
                   "boost_2p20x64_k4", "nmf_2p16x2048_q32", "density_sweep_1e4x300",
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


def load_traffic(path=TRAFFIC_FILE, log_tile=None):
    """HBM bytes per launch of the sketch kernel from the committed rocprofv3
    counter summary, or None when absent or taken on different kernel source.
    With log_tile, the figure of the tile-size variant of that size (a batch
    summary holds one per variant the autotuner timed)."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    if log_tile is not None:
        return (t.get("variants") or {}).get(str(log_tile), {}).get("hbm_bytes_per_launch")
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


CPU_ORACLE_WORKER = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, {root!r})
from oracle import rand_nnls
secs = 0.0
files = {files!r}
for f in files:
    z = np.load(f)
    A, b, r, seed = z["A"], z["b"], int(z["r"]), int(z["seed"])
    t0 = time.perf_counter()
    rand_nnls.rand_nnls(A, b, r, seed)
    secs += time.perf_counter() - t0
print(json.dumps({{"seconds": secs, "instances": len(files)}}))
"""


def host_cpus() -> int:
    """Host cores this process may use, at most 16 (a one-GPU machine's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_all_cores(problems, what):
    """The FP64 oracle (Algorithm 1 as written, oracle.rand_nnls) over
    `problems` = [(A (n, d) float32, b, r, sketch seed)], one single-threaded
    worker process per host core (longest problems first).  Rate = problems
    over the slowest worker's compute time; the one-core rate = problems over
    the summed compute time."""
    import numpy as np
    workers = min(host_cpus(), len(problems))
    tmp = tempfile.mkdtemp(prefix="rnnls_oracle_")
    try:
        files = []
        for i, (A, b, r, seed) in enumerate(problems):
            f = os.path.join(tmp, f"p{i}.npz")
            np.savez(f, A=A, b=b, r=np.int64(r), seed=np.int64(seed))
            files.append(f)
        order = sorted(range(len(problems)), key=lambda i: -problems[i][0].size)
        buckets, loads = [[] for _ in range(workers)], [0] * workers
        for i in order:
            w = loads.index(min(loads))
            buckets[w].append(files[i])
            loads[w] += problems[i][0].size
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = "1"
        procs = [subprocess.Popen([sys.executable, "-c",
                                   CPU_ORACLE_WORKER.format(root=ROOT, files=bk)],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                                  env=env) for bk in buckets]
        res = []
        for pr in procs:
            out, err = pr.communicate(timeout=900)
            if pr.returncode != 0:
                raise RuntimeError("cpu baseline worker failed: " + err[-2000:])
            res.append(json.loads(out.strip().splitlines()[-1]))
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    makespan = max(r["seconds"] for r in res)
    total = sum(r["seconds"] for r in res)
    return {"value": len(problems) / makespan, "unit": "solves/s", "cores": workers,
            "kind": "oracle", "cpu_model": cpu_model(),
            "single_core_value": len(problems) / total,
            "sample": f"{what}: {len(problems)} solves (FP64 numpy oracle of Algorithm 1, "
                      f"exact-r rows), {workers} single-threaded worker processes, "
                      f"{total:.1f} s of CPU work, slowest worker {makespan:.1f} s"}


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


ALL_TIMERS = (0, 1, 2, 5, 6)  # sketch, moments, solve, streams, reduce


def _whole(alg, ms):
    """Roofline of steps 1-4 as a whole: random streams + transform + reduce
    (their summed kernel durations `ms` per unit of `alg` bytes)."""
    ach = alg / (ms * 1e-3) / 1e9
    return {"kernels": "streams + srht transform + srht reduce", "ms": ms, "achieved": ach,
            "frac": ach / HBM_PEAK_GBS}


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
    """The sparse-versus-dense experiment (Section 4.2) at the paper's size:
    n = 10,000, d = 300, densities 2..64%; for each density 10 random
    n x (d+1) matrices (nonzeros uniform in [0, 1]) and 10 choices of the
    column that becomes b (100 problems); r = d, d+50, d+100, d+150 in both
    sampling modes, against the exact solve on all n rows.  Relative error =
    residual ratio minus one; times are GPU means per solve."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls, workloads
    n, d = 10_000, 300
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
        plain_ok = sum(int(s.status.item()) == 0 for s in plain)
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
                             "rand_ms": ms, "exact_full_ms": exact_ms, "exact_status_ok": plain_ok,
                             "speedup_vs_exact_full": exact_ms / ms})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    last = rows[-1]
    rec = _base_record(args, 1000.0 / last["rand_ms"], last["rand_ms"], {
        "workload": "sparse-versus-dense experiment at the paper's size: n = 10,000, d = 300, "
                    "densities 2..64%, 100 problems per density, r = d + 50 i (i = 0..3), both "
                    "sampling modes",
        "n": n, "d": d, "densities": list(densities), "r_values": list(rs),
        "step": "one randomized solve (density 64%, exact mode, r = d + 150)"})
    rec["sweep"] = rows
    print(json.dumps(rec), flush=True)


def bench_warm_batch(args):
    """The metric's configuration: batched, warm-started solves/s against the
    plain cold-start path on the same plans (see the module docstring)."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import learned, rnnls
    stream = torch.cuda.current_stream()
    # 1. training set: problems of the batch generator solved cold on the device
    t0 = time.perf_counter()
    Xs, ys, labels_ok = [], [], True
    chunk = 1024
    for c0 in range(0, args.train_instances, chunk):
        X, y, o = learned.collect(min(chunk, args.train_instances - c0), seed=100 + c0 // chunk)
        Xs.append(X)
        ys.append(y)
        labels_ok = labels_ok and o
        if (c0 // chunk) % 20 == 0:
            print(f"collected {min(c0 + chunk, args.train_instances)} / {args.train_instances} "
                  f"training problems ({time.perf_counter() - t0:.0f} s)", file=sys.stderr,
                  flush=True)
    X = torch.cat(Xs)
    y = torch.cat(ys)
    del Xs, ys
    collect_s = time.perf_counter() - t0
    mlp = rnnls.Mlp(learned.init_params(1))
    t1 = time.perf_counter()
    hist = learned.train(mlp, X, y, epochs=args.epochs, batch_rows=8192, lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    prob, _ = mlp.forward(X)
    acc = float(((prob > 0.5).to(torch.uint8) == y).double().mean().item())
    train_rows = int(X.shape[0])
    del X, y, prob
    print(f"trained: loss {hist[0]:.4f} -> {hist[-1]:.4f}, accuracy {acc:.4f} "
          f"({train_s:.1f} s)", file=sys.stderr, flush=True)

    # 2. held-out problems, all resident in HBM, as plans of `plan_size`
    count, per, hseed = args.heldout, args.plan_size, 2_000_000
    shp = learned.shapes(count, seed=hseed)
    alg = sum(4 * n * (d + 1) + 4 * r * (d + 1) for n, d, r in shp)
    plans, sample = [], []
    for c0 in range(0, count, per):
        probs = learned.device_problems(shp[c0:c0 + per], hseed * 1_000_003 + c0)
        if c0 == 0 and not args.no_cpu_baseline:
            for A, b, r, sd in probs[:args.cpu_samples or 64]:
                sample.append((A.t().contiguous().cpu().numpy().T, b.cpu().numpy(), r, sd))
        plans.append(rnnls.Batch(probs))
        del probs
    torch.cuda.synchronize()
    tiles = [P.autotune() for P in plans]
    print(f"{len(plans)} plans of {per} held-out problems resident "
          f"({alg / 1e9:.1f} GB of [A | b]), autotuned", file=sys.stderr, flush=True)

    # several plans: their graph replays are spread over a few streams (all of
    # default priority), forked from and joined back into the timed stream,
    # so one plan's latency-bound solves overlap the next plans' sketches
    side = [torch.cuda.Stream() for _ in range(min(4, len(plans)))] if len(plans) > 1 else []

    def one_pass():
        if not side:
            for P in plans:
                P.launch()
            return
        fork = torch.cuda.Event()
        fork.record(stream)
        for st in side:
            st.wait_event(fork)
        for i, P in enumerate(plans):
            P.launch(side[i % len(side)])
        for st in side:
            done = torch.cuda.Event()
            done.record(st)
            stream.wait_event(done)

    def phase(model):
        for P in plans:
            P.set_model(model)
            P.run()
        torch.cuda.synchronize()
        for P in plans:
            P.capture()
        for _ in range(args.warmup):
            one_pass()
        ms = _timed(one_pass, args.steps, stream)
        res = {"ms": ms,
               "rnorm": torch.cat([P.rnorm for P in plans]).clone(),
               "iters": torch.cat([P.iters for P in plans]).clone(),
               "status": torch.cat([P.status for P in plans]).clone(),
               "warm_used": (torch.cat([P.warm_used() for P in plans])
                             if model is not None else None)}
        # per-kernel durations from eager passes with the library's events on
        rnnls.timing_enable(True)
        for t in ALL_TIMERS:
            rnnls.timing_read(t)
        reps = 3
        for _ in range(reps):
            for P in plans:
                P.run()
        torch.cuda.synchronize()
        names = ("sketch", "moments", "lawson_hanson", "streams", "reduce")
        res["kernels_ms"] = {nm: rnnls.timing_read(t)[0] / reps
                             for nm, t in zip(names, ALL_TIMERS)}
        rnnls.timing_enable(False)
        return res

    cold = [phase(None)]
    warm = [phase(mlp)]
    cold.append(phase(None))
    warm.append(phase(mlp))
    cold_ms = float(np.mean([c["ms"] for c in cold]))
    warm_ms = float(np.mean([w["ms"] for w in warm]))
    rn_c, rn_w = cold[-1]["rnorm"], warm[-1]["rnorm"]
    gap = (rn_w / rn_c.clamp_min(1e-300) - 1.0).cpu().numpy()
    st_c = cold[-1]["status"].cpu().numpy()
    st_w = warm[-1]["status"].cpu().numpy()
    used = warm[-1]["warm_used"].double().cpu().numpy()
    kc, kw = cold[-1]["kernels_ms"], warm[-1]["kernels_ms"]
    sk_ms = kw["sketch"]
    achieved = alg / (sk_ms * 1e-3) / 1e9
    rec = _base_record(args, count * 1000.0 / warm_ms, warm_ms, {
        "workload": f"batched warm-started RandomizedNNLS: {count} held-out problems of the "
                    "batch generator (n log-uniform in [2^14, 2^18], d uniform in [8, 96], "
                    "r = max(32 d, 1024); tf-idf-like entries generated on the device) in "
                    f"{len(plans)} batch plans of {per}, HIP graph replay"
                    f"{f' on {len(side)} streams' if side else ''}, autotuned tiles; "
                    "Lawson-Hanson warm-started from the learned passive-set proposal, "
                    "KKT-judged with cold fallback",
        "problems": count, "plan_size": per, "heldout_seed": hseed,
        "algorithmic_bytes_per_pass": alg, "autotuned_tiles": sorted(set(tiles)),
        "network": "8-128-128-1 perceptron, BF16 weights, FP32 accumulation",
        "step": f"one pass over all {count} problems"})
    rec["vs_cold"] = {
        "warm_solves_per_s": count * 1000.0 / warm_ms,
        "cold_solves_per_s": count * 1000.0 / cold_ms,
        "speedup": cold_ms / warm_ms,
        "ms_per_pass_cold": [c["ms"] for c in cold], "ms_per_pass_warm": [w["ms"] for w in warm],
        "max_rel_residual_gap_vs_cold": float(gap.max()),
        "max_abs_rel_residual_gap_vs_cold": float(np.abs(gap).max()),
        "mean_rel_residual_gap_vs_cold": float(gap.mean()),
        "gap_bar": 1e-2, "within_bar": bool(np.abs(gap).max() <= 1e-2),
        "fallback_rate": float(1.0 - used.mean()),
        "status_ok_cold": int((st_c == 0).sum()), "status_ok_warm": int((st_w == 0).sum()),
        "outer_iterations_cold_mean": float(cold[-1]["iters"].double().mean().item()),
        "outer_iterations_warm_mean": float(warm[-1]["iters"].double().mean().item()),
        "kernels_ms_per_pass_cold": kc, "kernels_ms_per_pass_warm": kw,
        "gap_definition": "||S(Ax_warm - b)|| / ||S(Ax_cold - b)|| - 1 on the same sketch"}
    rec["roofline"] = _with_read_peak({
        "kernel": "srht_tiled_kernel (every sketch launch of the pass)", "bound": "hbm",
        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        # counters were taken per tile-size variant on one plan of 4096
        "traffic": (load_traffic(TRAFFIC_FILE_BATCH, log_tile=tiles[0][0])
                    if (per == count == 4096 and len(set(tiles)) == 1) else None),
        "algorithmic_bytes_per_pass": alg, "sketch_ms_per_pass": sk_ms,
        "whole_sketch": _whole(alg, kw["streams"] + sk_ms + kw["reduce"])})
    rec["training"] = {"problems": args.train_instances, "rows": train_rows,
                       "epochs": args.epochs, "loss_first": hist[0], "loss_last": hist[-1],
                       "train_accuracy": acc, "collect_s": collect_s, "train_s": train_s,
                       "labels_all_ok": labels_ok}
    for P in plans:
        P.close()
    del plans
    torch.cuda.empty_cache()
    single = run_single(args, "single_2p20x64", with_extras=False)
    rec["single_2p20x64"] = {k: single[k] for k in ("value", "ms_per_step", "config", "roofline",
                                                    "breakdown_ms_per_step", "quality",
                                                    "srht_medians")}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = oracle_all_cores(sample, "the first held-out problems")
    print(json.dumps(rec), flush=True)


def srht_medians(A, b, r, seed, n, d, reps=50, warmups=5):
    """Steps 1-4 of Algorithm 1 (rnnls_srht_sketch: random streams, transform,
    reduce) timed one call at a time, `reps` times after `warmups`, with the
    last-level cache warm (calls back to back) and cold (a 1 GiB read between
    calls; also a 1 GiB write, which leaves dirty lines).  Medians of the
    transform kernel alone and of the three kernels
    together (their event-timed durations), and of the call bracketed by two
    events (launch gaps included); HBM fractions of the algorithmic bytes
    4 n (d+1) + 4 r (d+1)."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls
    stream = torch.cuda.current_stream()
    ws = rnnls.workspace(rnnls.OP_SKETCH, n, d, r)
    flush = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    parts = rnnls.stream_read(flush)
    alg = 4 * n * (d + 1) + 4 * r * (d + 1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    timers = (rnnls.TIMER_STREAMS, rnnls.TIMER_SKETCH, rnnls.TIMER_REDUCE)
    out = {}
    for mode in ("warm", "cold", "cold_dirty"):
        for i in range(warmups):
            rnnls.srht_sketch(A, b, r, seed + i, ws=ws)
        torch.cuda.synchronize()
        rnnls.timing_enable(True)
        for t in timers:
            rnnls.timing_read(t)
        tiled, whole, call = [], [], []
        for i in range(reps):
            if mode == "cold":        # evict [A | b] with clean lines
                rnnls.stream_read(flush, parts)
            elif mode == "cold_dirty":  # evict it with dirty lines
                flush.fill_(float(i))
            e0.record(stream)
            rnnls.srht_sketch(A, b, r, seed + i, ws=ws)
            e1.record(stream)
            torch.cuda.synchronize()
            st, sk, rd = (rnnls.timing_read(t)[0] for t in timers)
            tiled.append(sk)
            whole.append(st + sk + rd)
            call.append(e0.elapsed_time(e1))
        rnnls.timing_enable(False)
        t_ms, w_ms, c_ms = (float(np.median(v)) for v in (tiled, whole, call))
        out[mode] = {"transform_kernel_us": t_ms * 1e3,
                     "transform_frac": alg / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "streams_transform_reduce_us": w_ms * 1e3,
                     "streams_transform_reduce_frac": alg / (w_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "call_us": c_ms * 1e3,
                     "call_frac": alg / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del flush
    out["reps"] = reps
    out["algorithmic_bytes"] = alg
    out["cold"]["flush"] = ("1 GiB device read between calls (the last-level cache holds 256 MB), "
                            "so no line of [A | b] stays cached")
    out["cold_dirty"]["flush"] = ("1 GiB device write between calls: the cache then holds dirty "
                                  "lines whose write-back lands inside the timed call")
    return out


def run_single(args, name, with_extras=True):
    """One step = rnnls_rand_nnls on one instance resident in HBM."""
    import numpy as np
    import torch

    from paper_0812_4547_amd import rnnls, workloads
    n, d, r, ds, ss = WORKLOADS[name]
    planted = name == "single_4096x16"
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
    for t in ALL_TIMERS:
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
    st_ms, _ = rnnls.timing_read(rnnls.TIMER_STREAMS)
    rd_ms, _ = rnnls.timing_read(rnnls.TIMER_REDUCE)
    rnnls.timing_enable(False)
    status = int(out.status.item())

    ms_per_step = ms_total / args.steps
    sk_avg = sk_ms / max(sk_n, 1)
    alg_bytes = 4 * n * (d + 1) + 4 * r * (d + 1)
    achieved = alg_bytes / (sk_avg * 1e-3) / 1e9
    traffic = load_traffic() if (args.precision == "fp32" and name == "single_2p20x64") else None

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
            "whole_sketch": _whole(alg_bytes, (st_ms + sk_ms + rd_ms) / args.steps),
        },
        "breakdown_ms_per_step": {
            "streams": st_ms / args.steps,
            "sketch_kernel": sk_ms / args.steps,
            "reduce": rd_ms / args.steps,
            "moments": mo_ms / args.steps,
            "lawson_hanson": lh_ms / args.steps,
            "other": ms_timed_total / args.steps
                     - (st_ms + sk_ms + rd_ms + mo_ms + lh_ms) / args.steps,
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
    if args.precision == "fp32":
        rec["srht_medians"] = srht_medians(A, b, r, ss, n, d)
    if with_extras:
        _with_read_peak(rec["roofline"])
        if not args.no_cpu_baseline:
            ns = args.cpu_samples or CPU_SAMPLES[name]
            rec["cpu_baseline"] = cpu_baseline(n, d, r, ds, planted, ns)
    return rec




def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="warm_batch_4096",
                    choices=["warm_batch_4096"] + sorted(WORKLOADS) + list(BATCH_WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=0,
                    help="instances the oracle times (default: about 10-30 s of CPU work)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "split_bf16"],
                    help="sketch transform: FP32 vector units, or BF16 matrix cores with "
                         "split hi + lo operands and FP32 accumulation")
    ap.add_argument("--train-instances", type=int, default=100_000)
    ap.add_argument("--heldout", type=int, default=4096)
    ap.add_argument("--plan-size", type=int, default=4096,
                    help="problems per batch plan of the default workload (4096: the "
                         "held-out set in one plan, so that the solves of many problems "
                         "share the device; 256: the batch size of the batching form)")
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
    if args.workload == "density_sweep_1e4x300":
        return bench_density(args)

    if args.workload == "warm_batch_4096":
        return bench_warm_batch(args)
    print(json.dumps(run_single(args, args.workload)), flush=True)


if __name__ == "__main__":
    main()
