"""The local search after the construction (2-opt and Or-opt descent along
the candidate lists, and with kind 2 the 3-opt move as well) on the GPU
against the oracle's descent: in the
synchronous mode, and with one ant in the asynchronous mode, tours,
lengths, best-so-far tour, pheromone and the number of moves must be equal
bit for bit after every iteration (the descent's move order and its
rewriting of the tour array are fixed, and every decision compares integer
lengths)."""
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
    # (name, coordinates, parameters, iterations)
    ("n200_cl32", lambda: inputs.uniform(200, 41), dict(), 5),
    ("n733_clustered_m96_cl16", lambda: inputs.clustered(733, 42), dict(m=96, cl=16), 3),
    ("n150_period4_q0", lambda: inputs.uniform(150, 43), dict(local_update_period=4, q0=0.0), 4),
    ("lattice_cl4_ties", lambda: inputs.lattice(12, 44), dict(cl=4, beta=0.0), 4),
    ("n7_cl6", lambda: inputs.uniform(7, 45), dict(cl=6), 6),
    ("n5_cl4", lambda: inputs.uniform(5, 46), dict(cl=4), 4),
]


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("name,make,kw,iters", CASES, ids=[c[0] for c in CASES])
def test_sync_with_local_search_equals_oracle(acs, name, make, kw, iters, kind):
    _say(f"local search {kind}, synchronous: {name}")
    xy = make()
    oracle.set_threads(8)
    col = acs.Colony(xy, mode=acs.ACS_SYNC, seed=13, local_search=kind, **kw)
    orc = oracle.Oracle(xy, seed=13, local_search=kind, **kw)
    for it in range(iters):
        col.iterate(1)
        orc.iterate(1)
        assert np.array_equal(col.tours(), orc.tours()), f"tours differ at iteration {it}"
        assert np.array_equal(col.lengths(), orc.lengths()), it
        gt, gl = col.best()
        ot, ol = orc.best()
        assert gl == ol and np.array_equal(gt, ot), it
        assert np.array_equal(col.tau(), orc.tau()), f"pheromone differs at iteration {it}"
        assert col.stats()["ls_moves"] == orc.ls_moves(), it
    assert orc.ls_moves() > 0
    oracle.set_threads(1)
    col.close()
    orc.close()


@pytest.mark.parametrize("path,kind", [(2, 1), (1, 1), (1, 2)])
def test_async_one_ant_with_local_search_equals_oracle(acs, path, kind):
    xy = inputs.uniform(260, 47)
    col = acs.Colony(xy, m=1, mode=acs.ACS_ASYNC_ATOMIC, seed=2, local_search=kind,
                     update_path=path)
    orc = oracle.Oracle(xy, m=1, seed=2, local_search=kind)
    for it in range(6):
        col.iterate(1)
        orc.iterate(1)
        assert np.array_equal(col.tours(), orc.tours()), it
        assert np.array_equal(col.tau(), orc.tau()), it
    col.close()


@pytest.mark.parametrize("kind", [1, 2])
def test_headline_size_with_local_search_valid(acs, kind):
    n = 2392
    xy = inputs.uniform(n)
    col = acs.Colony(xy, mode=acs.ACS_ASYNC_ATOMIC, seed=0, local_search=kind)
    plain = acs.Colony(xy, mode=acs.ACS_ASYNC_ATOMIC, seed=0)
    col.iterate(2)
    plain.iterate(2)
    tours, lens = col.tours(), col.lengths()
    assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
    assert np.array_equal(defs.tour_lengths(xy, tours), lens)
    st = col.stats()
    _say(f"n=2392 with local search {kind}: best {st['best_length']} ({plain.stats()['best_length']} "
         f"without), {st['ls_moves']} moves, iteration {st['iterate_ms']:.2f} ms")
    assert st["best_length"] < plain.stats()["best_length"]
    col.close()
    plain.close()
