"""Independent definitions used by the pin tests.

These are brute-force restatements of the definitions (exact rational
arithmetic, exhaustive enumeration); they do not call the oracle and the
oracle does not call them.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np


def exact_dist(xi: float, yi: float, xj: float, yj: float) -> int:
    """Nearest integer (halves up) of sqrt(s), s = dx*dx + dy*dy in double.

    d is the largest integer with (2d - 1)^2 <= 4 s, i.e. (d - 1/2)^2 <= s.
    Python floats are IEEE doubles and evaluate each operation separately.
    """
    dx = xi - xj
    dy = yi - yj
    s = Fraction(dx * dx + dy * dy)
    k = math.isqrt(math.floor(4 * s))  # largest k with k^2 <= 4s
    return (k + 1) // 2


def edge_dists(xy: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """exact_dist of the pairs (u[k], v[k]), vectorised: the integer d >= 0 with
    (d - 1/2)^2 <= s < (d + 1/2)^2 (d = 0 for s < 1/4), found from a rounded square root and
    corrected by those two exact comparisons (every square of d +- 1/2 below
    2^26 is exact in double)."""
    dx = xy[u, 0] - xy[v, 0]
    dy = xy[u, 1] - xy[v, 1]
    s = dx * dx + dy * dy
    d = np.floor(np.sqrt(s) + 0.5)
    for _ in range(2):
        d = np.where((d >= 1) & ((d - 0.5) * (d - 0.5) > s), d - 1, d)
        d = np.where((d + 0.5) * (d + 0.5) <= s, d + 1, d)
    return d.astype(np.int64)


def tour_lengths(xy: np.ndarray, tours: np.ndarray) -> np.ndarray:
    """Length of every row of `tours` (closing edge included)."""
    t = np.asarray(tours, dtype=np.int64)
    return edge_dists(xy, t, np.roll(t, -1, axis=1)).sum(axis=1)


def dist_matrix(xy: np.ndarray) -> np.ndarray:
    n = len(xy)
    d = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        for j in range(i + 1, n):
            d[i, j] = d[j, i] = exact_dist(float(xy[i, 0]), float(xy[i, 1]),
                                           float(xy[j, 0]), float(xy[j, 1]))
    return d


def nn_tour(d: np.ndarray, start: int) -> list[int]:
    """Greedy nearest-neighbour tour (ties: lowest index)."""
    n = len(d)
    seen = [False] * n
    tour = [start]
    seen[start] = True
    cur = start
    for _ in range(n - 1):
        best = None
        for j in range(n):
            if not seen[j] and (best is None or d[cur, j] < d[cur, best]):
                best = j
        tour.append(best)
        seen[best] = True
        cur = best
    return tour


def tour_length(d: np.ndarray, tour) -> int:
    t = np.asarray(tour)
    return int(d[t, np.roll(t, -1)].sum())


def brute_force_optimum(d: np.ndarray) -> int:
    """Shortest tour by enumerating every permutation of cities 1..n-1."""
    n = len(d)
    perms = np.array(list(itertools.permutations(range(1, n))), dtype=np.int64)
    tours = np.concatenate([np.zeros((len(perms), 1), np.int64), perms], axis=1)
    lens = d[tours, np.roll(tours, -1, axis=1)].sum(axis=1)
    return int(lens.min())


def round_to_f32(q: Fraction) -> np.float32:
    """Correctly rounded (nearest, ties to even) float32 of an exact rational."""
    if q == 0:
        return np.float32(0.0)
    sign = -1 if q < 0 else 1
    q = abs(q)
    e = math.floor(math.log2(q.numerator) - math.log2(q.denominator))
    # fix e so that 2^e <= q < 2^(e+1)
    while Fraction(2) ** e > q:
        e -= 1
    while Fraction(2) ** (e + 1) <= q:
        e += 1
    e = max(e, -126)
    scale = Fraction(2) ** (e - 23)
    m = q / scale
    fl = math.floor(m)
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return np.float32(sign * float(fl * scale))


def fmaf32(a, x, b) -> np.float32:
    """a * x + b for float32 operands, rounded once to float32 (what fmaf
    computes)."""
    return round_to_f32(Fraction(float(a)) * Fraction(float(x)) + Fraction(float(b)))
