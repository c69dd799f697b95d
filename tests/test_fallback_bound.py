"""The fact the dense fallback's prefix bound rests on, checked in exact
arithmetic on the CPU.

Before a construction the kernel bounds every pheromone value beyond a row's
prefix by T = max(largest start value, hi), with hi = fl32(b / (1 - a) *
(1 + 2^-20)) for the local map f(x) = fmaf(a, x, b) of Eq. 3 (a = fl32(1 -
phi), b = fl32(phi * tau0)).  That is sound if f never lifts a value above
max(x, hi): then no chain of local updates during the construction can.
"""
from __future__ import annotations

import numpy as np
import pytest

from tests import defs

CASES = [
    (0.1, 1.0 / (2392 * 433509.0)),   # the headline instance's scale
    (0.1, 1.0 / (198 * 15808.0)),
    (0.01, 3.1e-7),
    (0.5, 2.0e-9),
    (0.9, 0.37),
]


def _consts(phi, tau0):
    a = np.float32(1.0 - phi)
    b = np.float32(phi * tau0)
    fix = float(b) / (1.0 - float(a))
    hi = np.float32(fix * (1.0 + 2.0 ** -20))
    return a, b, fix, hi


@pytest.mark.parametrize("phi,tau0", CASES)
def test_local_map_never_exceeds_bound(phi, tau0):
    a, b, fix, hi = _consts(phi, tau0)
    assert float(hi) > fix
    # every float32 in a window around the real fixed point ...
    centre = np.float32(fix)
    xs = [centre]
    up = down = centre
    for _ in range(600):
        up = np.nextafter(up, np.float32(np.inf))
        down = np.nextafter(down, np.float32(0))
        xs += [up, down]
    # ... and values spread far below and above it
    g = np.random.default_rng(7)
    xs += list((fix * np.exp(g.uniform(-3.0, 6.0, 400))).astype(np.float32))
    for x in xs:
        y = defs.fmaf32(a, x, b)
        assert y <= max(x, hi), (x, y, hi)


@pytest.mark.parametrize("phi,tau0", CASES)
def test_chains_from_below_stay_under_hi(phi, tau0):
    a, b, fix, hi = _consts(phi, tau0)
    for start in (np.float32(fix * 0.5), np.float32(fix * (1 - 2.0 ** -18)), np.float32(0.0)):
        x = start
        for _ in range(200):
            x = defs.fmaf32(a, x, b)
            assert x <= hi
