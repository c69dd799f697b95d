"""Learned candidate scores in Eq. 1 and Eq. 2, synchronous mode, bit-exact
against the oracle given the same scores.

The scores replace eta^beta of the candidates only; the greedy fallback over
all unvisited cities keeps eta^beta.  Scores reach the library either from
the host (acs_set_candidate_scores) or from the network
(acs_prior_apply, read back with acs_candidate_weights); the oracle takes
them through orc_set_candidate_weights.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
from paper_1605_02669_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def acs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_02669_amd import acs as mod
    mod.load()
    return mod


def _compare(col, orc, it, tau=True):
    assert np.array_equal(col.tours(), orc.tours()), f"tours differ at iteration {it}"
    assert np.array_equal(col.lengths(), orc.lengths()), f"lengths differ at iteration {it}"
    gt, gl = col.best()
    ot, ol = orc.best()
    assert gl == ol and np.array_equal(gt, ot), f"best differs at iteration {it}"
    if tau:
        bad = np.argwhere(col.tau() != orc.tau())
        assert bad.size == 0, f"pheromone differs at {len(bad)} entries (iteration {it})"
    st, oc = col.stats(), orc.counts()
    for k in ("greedy", "roulette", "fallback"):
        assert st[k] == oc[k], f"{k} count {st[k]} != {oc[k]} at iteration {it}"


def _scores(n, cl, seed):
    # spread over two decades so the scores, not the pheromone, decide
    g = np.random.default_rng(seed)
    return (10.0 ** g.uniform(-2.0, 0.0, size=(n, cl))).astype(np.float32)


CASES = [
    ("n198_cl32_100it", lambda: inputs.uniform(198), dict(cl=32), 100),
    ("grid225_cl16_fallbacks", lambda: inputs.lattice(15, 3), dict(cl=16, m=120), 20),
    ("n2392_cl32_2it", lambda: inputs.uniform(2392), dict(cl=32), 2),
]


@pytest.mark.parametrize("name,mk,kw,iters", CASES, ids=[c[0] for c in CASES])
def test_host_scores_sync_parity(acs, name, mk, kw, iters):
    xy = mk()
    n = len(xy)
    col = acs.Colony(xy, mode=acs.ACS_SYNC, seed=11, **kw)
    orc = oracle.Oracle(xy, seed=11, **kw)
    sc = _scores(n, col.cl, 5)
    col.set_candidate_scores(sc)
    orc.set_candidate_weights(sc)
    assert np.array_equal(col.candidate_weights(), sc)
    _say(f"{name}: {iters} iterations")
    for it in range(iters):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it, tau=(it % 10 == 9 or it == iters - 1 or n < 1000))
    if name.startswith("grid"):
        assert orc.counts()["fallback"] > 0
    col.close()


def test_network_scores_sync_parity(acs):
    """Scores written by acs_prior_apply (the committed parameters), read back
    through acs_candidate_weights and given to the oracle: the synchronous
    run with them is bit-exact, and it differs from the plain run."""
    import torch
    from paper_1605_02669_amd import prior as pr
    P = torch.tensor(np.load(pr.DEFAULT_PARAMS), dtype=torch.float32, device="cuda")
    xy = inputs.clustered(400, 77)
    col = acs.Colony(xy, mode=acs.ACS_SYNC, cl=16, seed=2)
    plain = acs.Colony(xy, mode=acs.ACS_SYNC, cl=16, seed=2)
    col.apply_prior(P)
    w = col.candidate_weights()
    assert np.all(w > 0) and np.all(np.isfinite(w))
    orc = oracle.Oracle(xy, cl=16, seed=2)
    orc.set_candidate_weights(w)
    for it in range(20):
        col.iterate(1)
        plain.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it, tau=(it % 5 == 4))
    assert not np.array_equal(col.tours(), plain.tours())
    col.close()
    plain.close()
