"""Learned warm start: data collection, training and evaluation driver.

Every numerical step runs in the library's kernels (batch plans for the
sketch, moments and Lawson-Hanson; the feature, perceptron, gradient and Adam
kernels for the network).  This module only generates seeded device inputs,
orders the calls, shuffles row indices and keeps the bookkeeping.

Protocol: problems from the batch generator (n log-uniform, d uniform,
r = max(32 d, 1024)) are solved cold; the passive set x_j > 0 of each
solution labels the features of its columns; the network learns
p(passive | features); held-out problems are then solved cold and warm-started
from the network's proposal (KKT-judged, cold fallback) and compared.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import rnnls, workloads


def init_params(seed: int, device="cuda") -> torch.Tensor:
    """He-uniform weights, zero biases, as one flat FP32 vector in the
    library's parameter order (W1, b1, W2, b2, w3, b3)."""
    g = np.random.default_rng(seed)
    F, H = rnnls.MLP_FEATURES, rnnls.MLP_WIDTH
    parts = [g.uniform(-1, 1, (H, F)) * np.sqrt(6.0 / F), np.zeros(H),
             g.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H), np.zeros(H),
             g.uniform(-1, 1, H) * np.sqrt(6.0 / H), np.zeros(1)]
    theta = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    return torch.from_numpy(theta).to(device)


def save_checkpoint(mlp: rnnls.Mlp, path: str) -> None:
    """The perceptron's FP32 parameters, Adam moments and step count to an
    .npz file (plain arrays: loadable without unpickling).  The BF16 weights
    are not stored: they are the rounding of the parameters."""
    np.savez(path, theta=mlp.theta.cpu().numpy(), m=mlp.m.cpu().numpy(),
             v=mlp.v.cpu().numpy(), step=np.int64(mlp.step))


def load_checkpoint(path: str, device="cuda") -> rnnls.Mlp:
    """An Mlp restored from save_checkpoint: the same parameters, BF16 weights
    (rounded again on the device), Adam moments and step, so training
    continues exactly where it stopped."""
    with np.load(path, allow_pickle=False) as z:
        mlp = rnnls.Mlp(torch.from_numpy(z["theta"].astype(np.float32)).to(device))
        mlp.m.copy_(torch.from_numpy(z["m"].astype(np.float32)))
        mlp.v.copy_(torch.from_numpy(z["v"].astype(np.float32)))
        mlp.step = int(z["step"])
    return mlp


def shapes(count: int, seed: int, log2_n=(14.0, 18.0)):
    return workloads.batch_shapes(count=count, seed=seed, log2_n=log2_n)


def device_problems(shp, seed0: int, device="cuda"):
    """(A, b, r, sketch seed) per shape, generated on the device."""
    out = []
    for i, (n, d, r) in enumerate(shp):
        A, b, _ = workloads.tfidf_like_device(n, d, seed0 + i, device=device)
        out.append((A, b, r, seed0 + i))
    return out


def collect(count: int, seed: int, chunk: int = 512, log2_n=(14.0, 18.0), device="cuda"):
    """Features and passive labels of `count` problems solved cold.  Returns
    (X (rows, 8) float32, y (rows,) uint8, all statuses OK)."""
    shp = shapes(count, seed, log2_n)
    Xs, ys, ok = [], [], True
    for c0 in range(0, count, chunk):
        probs = device_problems(shp[c0:c0 + chunk], seed * 1_000_003 + c0, device)
        batch = rnnls.Batch(probs)
        batch.run()
        X, y = batch.features()
        ok = ok and bool((batch.status == rnnls.SOLVE_OK).all().item())
        Xs.append(X)
        ys.append(y)
        batch.close()
        del probs, batch
    return torch.cat(Xs), torch.cat(ys), ok


def train(mlp: rnnls.Mlp, X: torch.Tensor, y: torch.Tensor, epochs: int, batch_rows: int = 8192,
          lr: float = 1e-3, seed: int = 0):
    """Mini-batch Adam on the device kernels; returns the mean loss per epoch."""
    rows = X.shape[0]
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    history = []
    for _ in range(epochs):
        perm = torch.randperm(rows, generator=gen, device=X.device)
        total = torch.zeros((), dtype=torch.float64, device=X.device)
        steps = 0
        for s0 in range(0, rows, batch_rows):
            idx = perm[s0:s0 + batch_rows]
            Xb = X.index_select(0, idx).contiguous()
            yb = y.index_select(0, idx).contiguous()
            mlp.train_step(Xb, yb, lr, loss=loss)
            total += loss.double()[0] * idx.numel()
            steps += 1
        history.append(float(total.item()) / rows)
    return history


@dataclass
class Evaluation:
    problems: int
    cold_ms: float            # one eager pass of the batch plan, cold
    warm_ms: float            # the same pass with the learned proposal
    cold_lh_ms: float
    warm_lh_ms: float
    cold_iters: float         # mean outer iterations
    warm_iters: float
    warm_kept: float          # fraction of problems whose warm start passed KKT
    max_gap: float            # max over problems of rnorm_warm / rnorm_cold - 1
    all_ok: bool


def _timed_pass(batch, reps: int):
    """(ms per pass timed without per-kernel events, Lawson-Hanson ms per pass
    from a second run of the same passes with the solve's events on)."""
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        batch.run()
    e1.record(stream)
    torch.cuda.synchronize()
    rnnls.timing_enable(True)
    rnnls.timing_read(rnnls.TIMER_SOLVE)
    for _ in range(reps):
        batch.run()
    torch.cuda.synchronize()
    lh_ms, _ = rnnls.timing_read(rnnls.TIMER_SOLVE)
    rnnls.timing_enable(False)
    return e0.elapsed_time(e1) / reps, lh_ms / reps


def evaluate(mlp: rnnls.Mlp, count: int, seed: int, chunk: int = 1024, threshold: float = 0.5,
             reps: int = 3, log2_n=(14.0, 18.0), device="cuda") -> Evaluation:
    shp = shapes(count, seed, log2_n)
    tot = dict(cold_ms=0.0, warm_ms=0.0, cold_lh=0.0, warm_lh=0.0, ci=0.0, wi=0.0, kept=0.0)
    max_gap, all_ok = 0.0, True
    for c0 in range(0, count, chunk):
        probs = device_problems(shp[c0:c0 + chunk], seed * 1_000_003 + c0, device)
        batch = rnnls.Batch(probs)
        batch.set_model(None)
        batch.run()
        torch.cuda.synchronize()
        ms, lh = _timed_pass(batch, reps)
        tot["cold_ms"] += ms
        tot["cold_lh"] += lh
        rn_cold = batch.rnorm.clone()
        it_cold = batch.iters.clone()
        all_ok = all_ok and bool((batch.status == rnnls.SOLVE_OK).all().item())
        batch.set_model(mlp, threshold)
        batch.run()
        torch.cuda.synchronize()
        ms, lh = _timed_pass(batch, reps)
        tot["warm_ms"] += ms
        tot["warm_lh"] += lh
        all_ok = all_ok and bool((batch.status == rnnls.SOLVE_OK).all().item())
        gap = (batch.rnorm / rn_cold.clamp_min(1e-300) - 1.0).max().item()
        max_gap = max(max_gap, gap)
        tot["ci"] += float(it_cold.double().sum().item())
        tot["wi"] += float(batch.iters.double().sum().item())
        tot["kept"] += float(batch.warm_used().double().sum().item())
        batch.close()
        del probs, batch
    return Evaluation(count, tot["cold_ms"], tot["warm_ms"], tot["cold_lh"], tot["warm_lh"],
                      tot["ci"] / count, tot["wi"] / count, tot["kept"] / count, max_gap, all_ok)
