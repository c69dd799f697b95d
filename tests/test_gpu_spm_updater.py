"""Asynchronous selective-memory construction with the updater wave.

The ant waves of k_construct_async_spm_q hand one entry per visited city to
their block's updater wave, which applies Alg. 3 for the edge that reached
the city and then for the edge that left it.  With one ant nothing races,
so both update paths (updater wave, ant-issued) and both update kinds
(compare-and-swap, plain stores) must equal the oracle's schedule bit for
bit: tours, records (with evictions: s below the number of trails a city
gets), insert counters and hit/miss counts, over several iterations and
local-update periods.  With many ants every update must still be applied
exactly once in the compare-and-swap mode (hits plus misses count them).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1605_02669_amd import inputs
from tests import defs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def acs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_02669_amd import acs as mod
    mod.load()
    return mod


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    # (name, n, spm_s, cl, local-update period, iterations)
    ("s3_k1", 230, 3, 12, 1, 6),
    ("s6_k1", 150, 6, 16, 1, 6),
    ("s2_k3_ragged", 101, 2, 8, 3, 6),
    ("s4_k2_cl4_fallbacks", 180, 4, 4, 2, 5),
    ("s1_k1", 64, 1, 6, 1, 5),
]


@pytest.mark.parametrize("path", [2, 1], ids=["updater", "inwave"])
@pytest.mark.parametrize("mode", ["ASYNC_ATOMIC", "ASYNC_RACY"])
@pytest.mark.parametrize("name,n,s,cl,k,iters", CASES, ids=[c[0] for c in CASES])
def test_single_ant_equals_oracle(acs, name, n, s, cl, k, iters, mode, path):
    _say(f"SPM one ant {name} {mode} path {path}")
    xy = inputs.uniform(n, 900 + n)
    kw = dict(m=1, cl=cl, memory=1, spm_s=s, seed=4, local_update_period=k)
    col = acs.Colony(xy, mode=getattr(acs, "ACS_" + mode), update_path=path, **kw)
    orc = oracle.Oracle(xy, **kw)
    for it in range(iters):
        col.iterate(1)
        orc.iterate(1)
        assert np.array_equal(col.tours(), orc.tours()), f"tours differ at iteration {it}"
        assert np.array_equal(col.lengths(), orc.lengths()), it
        assert col.best()[1] == orc.best()[1], it
        for x, y, what in zip(col.spm(), orc.spm(), ("nodes", "vals", "tail")):
            assert np.array_equal(x, y), f"records: {what} differ at iteration {it}"
        st, oc = col.stats(), orc.counts()
        for c in ("greedy", "roulette", "fallback", "spm_hits", "spm_misses"):
            assert st[c] == oc[c], f"{c}: {st[c]} != {oc[c]} at iteration {it}"
    col.close()


@pytest.mark.parametrize("n,m,s,k", [(600, 600, 8, 1), (3000, 1024, 4, 1), (1000, 333, 8, 5)])
def test_many_ants_every_update_applied_once(acs, n, m, s, k):
    """Compare-and-swap mode through the updater: each update counts as one
    hit or one miss, the records stay well formed and the tours valid."""
    _say(f"SPM updater n={n} m={m} s={s} k={k}")
    xy = inputs.uniform(n, 31)
    col = acs.Colony(xy, m=m, cl=16, memory=1, spm_s=s, mode=acs.ACS_ASYNC_ATOMIC, seed=7,
                     local_update_period=k, update_path=2)
    per_ant = len(range(k, n, k)) + 1  # updated steps, plus the closing edge
    for it in range(3):
        col.iterate(1)
        tours, lens = col.tours(), col.lengths()
        assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
        assert np.array_equal(defs.tour_lengths(xy, tours), lens)
        st = col.stats()
        assert st["spm_hits"] + st["spm_misses"] == (it + 1) * (2 * m * per_ant + 2 * n)
        nodes, vals, tail = col.spm()
        assert np.all((nodes >= -1) & (nodes < n))
        assert np.all(np.isfinite(vals)) and vals.min() >= np.float32(st["tau0"]) * np.float32(0.999)
        assert np.all((tail >= 0) & (tail < s))
    col.close()
