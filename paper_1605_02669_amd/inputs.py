"""Seeded synthetic Euclidean TSP instances.

This module only produces inputs: city coordinates drawn from a seeded
generator.  It holds none of the method's arithmetic (no distances, no
pheromone, no random numbers the ants draw), so both the CPU oracle's tests and
the HIP path may use it.

The paper evaluates on TSPLIB instances (d198 ... pr2392, pcb3038 ... brd14051,
Sec. 4); those files are not available here, so instances of the same sizes
are generated instead:

* ``uniform(n, seed)``: n points, each coordinate uniform in [0, 10000).
* ``clustered(n, seed)``: 20 centres uniform in [0, 10000)^2; every point
  picks a centre uniformly and adds N(0, 300^2) noise per axis; a point that
  falls outside the square is drawn again.
* ``batch(count, seed)``: ``count`` instances with n log-uniform in
  [100, 2000], alternating uniform / clustered.
* ``lattice(side, seed)``: the side x side integer grid with spacing 7, its
  points in a seeded random order (many equal distances, so ties everywhere).

All generators use numpy's Philox bit generator keyed by the seed, so an
instance is fully determined by (kind, n, seed).
"""
from __future__ import annotations

import math

import numpy as np

SIDE = 10000.0


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed) & (2**64 - 1), int(stream)]))


def uniform(n: int, seed: int | None = None) -> np.ndarray:
    """n points uniform in [0, SIDE)^2, float64 array of shape (n, 2)."""
    if seed is None:
        seed = n
    g = _rng(seed, 0xC0DE)
    return np.ascontiguousarray(g.random((n, 2)) * SIDE, dtype=np.float64)


def clustered(n: int, seed: int | None = None, clusters: int = 20,
              sigma: float = 300.0) -> np.ndarray:
    """n points around ``clusters`` Gaussian centres, kept inside [0, SIDE]^2."""
    if seed is None:
        seed = n
    g = _rng(seed, 0xC1A5)
    centres = g.random((clusters, 2)) * SIDE
    out = np.empty((n, 2), dtype=np.float64)
    for i in range(n):
        c = centres[g.integers(0, clusters)]
        while True:
            p = c + g.normal(0.0, sigma, size=2)
            if 0.0 <= p[0] <= SIDE and 0.0 <= p[1] <= SIDE:
                break
        out[i] = p
    return out


def batch(count: int, seed: int = 256, nmin: int = 100, nmax: int = 2000):
    """``count`` instances with log-uniform sizes; even index uniform, odd clustered."""
    g = _rng(seed, 0xBA7C)
    sizes = np.exp(g.uniform(math.log(nmin), math.log(nmax), size=count))
    sizes = np.clip(np.rint(sizes).astype(np.int64), nmin, nmax)
    insts = []
    for i, n in enumerate(sizes):
        s = seed * 100003 + i
        insts.append(uniform(int(n), s) if i % 2 == 0 else clustered(int(n), s))
    return insts


def coincident(n: int, seed: int, dup: int = 4) -> np.ndarray:
    """Uniform points where the first ``dup`` cities share one location and
    some pairs sit closer than 0.5 (degenerate zero-distance edges)."""
    xy = uniform(n, seed)
    xy[1:dup] = xy[0]
    if n > dup + 1:
        xy[dup + 1] = xy[dup] + np.array([0.2, -0.1])
    return xy


def lattice(side: int, seed: int = 0, spacing: float = 7.0) -> np.ndarray:
    """side * side grid points, shuffled by the seed, float64 array (side^2, 2)."""
    g = _rng(seed, 0x6A1D)
    ix, iy = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel()], axis=1).astype(np.float64) * spacing
    return np.ascontiguousarray(pts[g.permutation(side * side)])
