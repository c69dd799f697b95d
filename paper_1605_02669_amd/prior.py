"""Learned edge prior: label generation, training and equal-time evaluation.

Orchestration only: the colonies, the features, the network's forward and
backward passes and the optimizer step all run in libacs kernels; this
module moves tensors between those calls.

* Labels: each training instance is solved by plain ACS (a batch of
  independent colonies, asynchronous mode) from several seeds; the label of
  candidate edge (i, r) is the fraction of those runs whose best tour
  contains the edge {i, r-th nearest neighbour of i}.
* Training: mean binary cross-entropy between sigmoid(z) and the label,
  Adam on fp32 master weights, bf16 matrix-core products.
* Evaluation: plain ACS (eta^beta) against ACS whose candidate weights are
  the network's scores, each given the same wall-clock budget (the network's
  inference counts in it), best tour length per seed.

Usage: python -m paper_1605_02669_amd.prior train --out params.npy
       python -m paper_1605_02669_amd.prior eval --params params.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "prior_params.npy")
CL = 16


def _torch():
    import torch
    return torch


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases, packed as the library expects."""
    from . import acs
    g = np.random.default_rng(seed)

    def he(fan_in, shape):
        lim = math.sqrt(6.0 / fan_in)
        return g.uniform(-lim, lim, size=shape).astype(np.float32)

    return acs.pack_prior({"W1": he(4, (4, 64)), "b1": np.zeros(64, np.float32),
                           "W2": he(64, (64, 64)), "b2": np.zeros(64, np.float32),
                           "W3": he(64, (64, 1)), "b3": np.zeros(1, np.float32)})


def training_instances(count: int, seed: int, nmin: int = 500, nmax: int = 2000):
    from . import inputs
    return inputs.batch(count, seed=seed, nmin=nmin, nmax=nmax)


def make_training_set(insts, runs: int = 2, ants: int = 128, iters: int = 100, seed: int = 1,
                      log=print):
    """Features (rows, 4) and labels (rows,) as GPU tensors, rows = sum n_i * 16."""
    torch = _torch()
    from . import acs
    best_tours = [[] for _ in insts]
    cand = None
    for r in range(runs):
        t0 = time.perf_counter()
        b = acs.Batch(insts, m=ants, cl=CL, seed=seed + r, instance=1 << 20)
        b.iterate(iters)
        for i in range(len(insts)):
            best_tours[i].append(b.best(i)[0])
        if cand is None:
            cand = [acs.acs_candidates(b.handle(i), len(x), CL) for i, x in enumerate(insts)]
            feats = []
            for i, x in enumerate(insts):
                X = torch.empty((len(x) * 16, 4), dtype=torch.float32, device="cuda")
                acs._check(acs.load().acs_prior_features(b.handle(i),
                                                         acs.C.c_void_p(X.data_ptr())))
                feats.append(X)
        info = b.info()
        b.close()
        log(f"labels: run {r}: {iters} iterations of {len(insts)} instances, "
            f"{info['steps_per_iteration'] * iters / (time.perf_counter() - t0) / 1e9:.2f} G steps/s")
    labels = []
    for i, x in enumerate(insts):
        n = len(x)
        hit = np.zeros((n, CL), dtype=np.float32)
        for tour in best_tours[i]:
            nxt = np.empty(n, dtype=np.int64)
            prv = np.empty(n, dtype=np.int64)
            nxt[tour] = np.roll(tour, -1)
            prv[tour] = np.roll(tour, 1)
            c = cand[i]
            hit += ((c == nxt[:, None]) | (c == prv[:, None])).astype(np.float32)
        labels.append(torch.tensor((hit / len(best_tours[i])).reshape(-1), device="cuda"))
    return torch.cat(feats), torch.cat(labels)


def train(X, Y, epochs: int = 20, batch: int = 65536, lr: float = 3e-3, seed: int = 0,
          log=print):
    """Trains the network on (X, Y) with the library's kernels; returns the
    parameter tensor (cuda, float32) and the per-epoch mean loss."""
    torch = _torch()
    from . import acs
    P = torch.tensor(init_params(seed), device="cuda")
    G = torch.zeros_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    L = torch.zeros(1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    rows = X.shape[0]
    history = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(rows, device="cuda", generator=gen)
        L.zero_()
        for s0 in range(0, rows, batch):
            idx = perm[s0:s0 + batch]
            xb = X.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            acs.prior_grad(P, xb, yb, G, L)
            step += 1
            acs.prior_adam(P, G, M, V, step, lr=lr)
        torch.cuda.synchronize()
        history.append(L.item() / rows)
        log(f"epoch {ep}: mean loss {history[-1]:.5f}")
    return P, history


def run_equal_time(xy, budget_s: float, seed: int, params=None, cl: int = CL):
    """Best tour length after `budget_s` seconds of asynchronous ACS: with the
    network's scores (params, cl = 16), or plain with candidate lists of cl."""
    torch = _torch()
    from . import acs
    col = acs.Colony(xy, cl=CL if params is not None else cl, mode=acs.ACS_ASYNC_ATOMIC,
                     seed=seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if params is not None:
        col.apply_prior(params)
    iters = 0
    while time.perf_counter() - t0 < budget_s:
        col.iterate(1)
        iters += 1
    best = col.best()[1]
    col.close()
    return best, iters


def evaluate(params, sizes=(2392,), kinds=("uniform", "clustered"), seeds=10,
             budget_s: float = 1.0, log=print):
    """Equal wall-clock comparison per instance: plain ACS with the
    configured candidate lists (cl = 32), plain ACS with the network's list
    length (cl = 16), and ACS with the network's scores (cl = 16).  The gap
    and the one-sided rank-sum p (learned shorter) are against plain cl = 32,
    and against plain cl = 16 under the `_cl16` keys."""
    from scipy.stats import mannwhitneyu

    from . import inputs
    out = {}
    for n in sizes:
        for kind in kinds:
            xy = inputs.uniform(n) if kind == "uniform" else inputs.clustered(n)
            plain = [run_equal_time(xy, budget_s, s, cl=32) for s in range(seeds)]
            plain16 = [run_equal_time(xy, budget_s, s, cl=CL) for s in range(seeds)]
            learned = [run_equal_time(xy, budget_s, s, params) for s in range(seeds)]
            a = np.array([b for b, _ in plain], dtype=np.float64)
            a16 = np.array([b for b, _ in plain16], dtype=np.float64)
            b = np.array([b for b, _ in learned], dtype=np.float64)
            res = {"plain_mean": a.mean(), "plain_cl16_mean": a16.mean(),
                   "learned_mean": b.mean(),
                   "gap_percent": 100.0 * (b.mean() - a.mean()) / a.mean(),
                   "gap_percent_cl16": 100.0 * (b.mean() - a16.mean()) / a16.mean(),
                   "plain_iterations": float(np.mean([i for _, i in plain])),
                   "plain_cl16_iterations": float(np.mean([i for _, i in plain16])),
                   "learned_iterations": float(np.mean([i for _, i in learned])),
                   "rank_sum_p": float(mannwhitneyu(b, a, alternative="less").pvalue),
                   "rank_sum_p_cl16": float(mannwhitneyu(b, a16, alternative="less").pvalue),
                   "seeds": seeds, "budget_s": budget_s}
            out[f"{kind}_{n}"] = res
            log(f"{kind} n={n}: plain cl=32 {a.mean():.0f}, plain cl=16 {a16.mean():.0f}, "
                f"learned {b.mean():.0f} ({res['gap_percent']:+.2f}% vs cl=32, "
                f"p={res['rank_sum_p']:.3g}; {res['gap_percent_cl16']:+.2f}% vs cl=16)")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--instances", type=int, default=256)
    t.add_argument("--runs", type=int, default=2)
    t.add_argument("--ants", type=int, default=128)
    t.add_argument("--iters", type=int, default=100)
    t.add_argument("--epochs", type=int, default=20)
    t.add_argument("--out", default=DEFAULT_PARAMS)
    e = sub.add_parser("eval")
    e.add_argument("--params", default=DEFAULT_PARAMS)
    e.add_argument("--seeds", type=int, default=10)
    e.add_argument("--budget", type=float, default=1.0)
    args = ap.parse_args(argv)
    torch = _torch()
    log = lambda s: print(s, flush=True)  # noqa: E731
    if args.cmd == "train":
        t0 = time.perf_counter()
        insts = training_instances(args.instances, seed=10 ** 6)
        X, Y = make_training_set(insts, runs=args.runs, ants=args.ants, iters=args.iters, log=log)
        log(f"training set: {X.shape[0]} rows, mean label {Y.mean().item():.4f}")
        P, hist = train(X, Y, epochs=args.epochs, log=log)
        np.save(args.out, P.cpu().numpy())
        log(json.dumps({"rows": int(X.shape[0]), "loss": hist, "seconds": time.perf_counter() - t0}))
    else:
        P = torch.tensor(np.load(args.params), device="cuda")
        log(json.dumps(evaluate(P, seeds=args.seeds, budget_s=args.budget, log=log)))


if __name__ == "__main__":
    sys.exit(main())
