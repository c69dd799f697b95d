"""Writes the stored expected digests of long synchronous runs.

Calls only the CPU oracle (and the seeded input generators): every stored
value below comes from ``oracle/``, never from the HIP library.  For each
workload it runs the synchronous schedule (Alg. 1 with every ant reading the
pheromone as it was at the start of the step) and records, after every
iteration, 128-bit xxh3 digests of

* the tours (m x n int32, row-major, little-endian),
* the tour lengths (m int64),
* the best-so-far tour (n int32) followed by its length (int64),
* the pheromone: dense memory the logical n x n float32 matrix; selective
  memory the records as nodes (n x s int32), values (n x s float32) and the
  index of the most recently added slot (n int32), in that order,

plus the best-so-far length itself.  The GPU tests rebuild the same digests
from the library's read-back calls and compare them iteration by iteration.

Usage: python -m tests.golden.make_golden [name ...] [--threads T]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import xxhash

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1605_02669_amd import inputs  # noqa: E402

# name -> (instance kind, n, instance seed, oracle keyword arguments, iterations)
WORKLOADS = {
    "n2392_uniform_sync_1000": ("uniform", 2392, 2392, dict(m=0, cl=32, seed=0), 1000),
    "n1000_clustered_sync_1000": ("clustered", 1000, 1000, dict(m=0, cl=32, seed=0), 1000),
    "n20000_spm_sync_10": ("uniform", 20000, 20000,
                           dict(m=1024, cl=16, memory=oracle.SPM, spm_s=8, seed=0), 10),
}
COMMON = dict(beta=2.0, q0=0.9, phi=0.1, rho=0.1)


def digest(*arrays) -> str:
    h = xxhash.xxh3_128()
    for a in arrays:
        h.update(memoryview(np.ascontiguousarray(a)))
    return h.hexdigest()


def coords(kind: str, n: int, seed: int) -> np.ndarray:
    return inputs.uniform(n, seed) if kind == "uniform" else inputs.clustered(n, seed)


def run(name: str) -> dict:
    kind, n, iseed, kw, iters = WORKLOADS[name]
    xy = coords(kind, n, iseed)
    o = oracle.Oracle(xy, **COMMON, **kw)
    rec = {"workload": name, "kind": kind, "n": n, "instance_seed": iseed,
           "params": {**COMMON, **{k: int(v) for k, v in kw.items()}},
           "iterations": iters, "hash": "xxh3_128",
           "tours": [], "lengths": [], "best": [], "pheromone": [], "best_length": []}
    t0 = time.time()
    for it in range(iters):
        o.iterate(1)
        t, L = o.best()
        rec["tours"].append(digest(o.tours()))
        rec["lengths"].append(digest(o.lengths()))
        rec["best"].append(digest(t, np.array([L], dtype=np.int64)))
        if kw.get("memory", oracle.DENSE) == oracle.DENSE:
            rec["pheromone"].append(digest(o.tau()))
        else:
            nodes, vals, tail = o.spm()
            rec["pheromone"].append(digest(nodes, vals, tail))
        rec["best_length"].append(int(L))
        if it % 50 == 0 or it == iters - 1:
            print(f"{name}: iteration {it + 1}/{iters}, L_gb {L}, "
                  f"{time.time() - t0:.0f} s", flush=True)
    rec["counts"] = o.counts()
    o.close()
    return rec


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(WORKLOADS))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    oracle.set_threads(a.threads)
    for name in a.names:
        rec = run(name)
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(rec, f, separators=(",", ":"))
            f.write("\n")


if __name__ == "__main__":
    main()
