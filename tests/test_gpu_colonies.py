"""Several colonies on one instance with a periodic best-so-far exchange
(the multi-colony model the paper's Sec. 2 describes): a batch of copies of
one instance, each colony with its own random numbers, exchanging along a
topology every few iterations.  With one ant per colony nothing races, so
every colony must equal an oracle colony that runs the same schedule and
the oracle's exchange (oracle.exchange_best) at the same iterations: tours,
pheromone, best-so-far tour and length, bit for bit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1605_02669_amd import inputs

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


@pytest.mark.parametrize("topology,period,colonies,mode", [
    (0, 2, 4, "ASYNC_ATOMIC"), (1, 3, 5, "ASYNC_ATOMIC"), (0, 1, 3, "ASYNC_RACY")])
def test_colonies_one_ant_each_equal_oracle(acs, topology, period, colonies, mode):
    _say(f"colonies={colonies} topology={topology} period={period} {mode}")
    xy = inputs.uniform(140, 71)
    b = acs.Batch([xy] * colonies, m=1, cl=16, seed=5, lanes_per_ant=64, update_path=2,
                  mode=getattr(acs, "ACS_" + mode))
    b.set_exchange(topology, period)
    orcs = [oracle.Oracle(xy, m=1, cl=16, seed=5, instance=i) for i in range(colonies)]
    adopted = 0
    for it in range(9):
        b.iterate(1)
        for o in orcs:
            o.iterate(1)
        if (it + 1) % period == 0:
            before = [o.best()[1] for o in orcs]
            oracle.exchange_best(orcs, topology)
            adopted += sum(o.best()[1] != L for o, L in zip(orcs, before))
        for i, o in enumerate(orcs):
            assert np.array_equal(b.tours(i), o.tours()), (i, it)
            gt, gl = b.best(i)
            ot, ol = o.best()
            assert gl == ol and np.array_equal(gt, ot), (i, it, gl, ol)
            assert np.array_equal(b.tau(i), o.tau()), (i, it)
    assert adopted > 0  # some colony took another's tour
    b.close()


def test_exchange_needs_one_instance(acs):
    b = acs.Batch([inputs.uniform(60, 1), inputs.uniform(61, 2)], m=4, cl=16, seed=1)
    with pytest.raises(acs.AcsError) as e:
        b.set_exchange(0, 2)
    assert e.value.code == acs.ACS_E_INVALID
    b.close()
