"""Error handling of the bounded device waits, forced from the host.

Every wait inside the kernels (the updater wave's ring, the ants' wait for
ring space, the grid barrier) gives up after a bounded number of polls,
raises the instance's error flag and lets every wave run to its end.  A
tiny wait_limit makes the idle updater wave give up almost at once; the
call must then fail with ACS_E_DEVICE instead of returning results with
local updates missing.  Without the limit the same workloads succeed.
"""
from __future__ import annotations

import pytest

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


def test_exhausted_ring_wait_fails_the_batch_call(acs):
    insts = [inputs.uniform(198, 1), inputs.clustered(150, 2), inputs.uniform(300, 3)]
    b = acs.Batch(insts, update_path=2, lanes_per_ant=64, wait_limit=1, seed=1)
    with pytest.raises(acs.AcsError) as e:
        b.iterate(1)
    assert e.value.code == acs.ACS_E_DEVICE
    assert "bounded device wait" in str(e.value)
    b.close()
    ok = acs.Batch(insts, update_path=2, lanes_per_ant=64, seed=1)
    ok.iterate(3)
    for i, x in enumerate(insts):
        t, L = ok.best(i)
        assert sorted(t.tolist()) == list(range(len(x)))
    ok.close()


def test_exhausted_ring_wait_fails_the_iterate_call(acs):
    xy = inputs.uniform(300, 4)
    col = acs.Colony(xy, mode=acs.ACS_ASYNC_ATOMIC, update_path=2, wait_limit=1, seed=2)
    with pytest.raises(acs.AcsError) as e:
        col.iterate(1)
    assert e.value.code == acs.ACS_E_DEVICE
    col.close()
    ok = acs.Colony(xy, mode=acs.ACS_ASYNC_ATOMIC, update_path=2, seed=2)
    ok.iterate(2)
    assert sorted(ok.best()[0].tolist()) == list(range(300))
    ok.close()
