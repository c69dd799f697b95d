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


def test_workspace_one_byte_short_is_rejected(acs):
    """A caller workspace below acs_workspace_bytes is refused with
    ACS_E_BUFSIZE before any device work; one of exactly that size runs, and
    gives the same synchronous run as the library's own allocation."""
    import numpy as np
    import torch
    xy = inputs.uniform(240, 5)
    p = acs.make_params(mode=acs.ACS_SYNC, seed=4)
    need = acs.acs_workspace_bytes(240, p)
    short = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    p.workspace, p.workspace_bytes = short.data_ptr(), need - 1
    with pytest.raises(acs.AcsError) as e:
        acs.acs_create(xy, p)
    assert e.value.code == acs.ACS_E_BUFSIZE and "workspace" in str(e.value)
    exact = acs.Colony(xy, mode=acs.ACS_SYNC, seed=4)  # a torch tensor of exactly `need`
    own = acs.Colony(xy, mode=acs.ACS_SYNC, seed=4, torch_memory=False)
    exact.iterate(3)
    own.iterate(3)
    assert np.array_equal(exact.tours(), own.tours())
    assert np.array_equal(exact.tau(), own.tau())
    exact.close()
    own.close()


def test_device_allocation_failure_is_reported(acs):
    """A batch whose workspace exceeds the device memory (seven n = 60000
    instances, about 47 GiB each) fails with ACS_E_NOMEM from its device
    allocation and leaves nothing behind: a normal batch works afterwards."""
    import numpy as np
    big = [inputs.uniform(60000, 50 + i) for i in range(7)]
    p = acs.make_params(mode=acs.ACS_ASYNC_ATOMIC)
    need = acs.acs_batch_workspace_bytes([60000] * 7, p)
    import torch
    assert need > torch.cuda.get_device_properties(0).total_memory
    with pytest.raises(acs.AcsError) as e:
        acs.Batch(big, seed=1, torch_memory=False)
    assert e.value.code == acs.ACS_E_NOMEM and "hipMalloc" in str(e.value)
    small = [inputs.uniform(120, 7), inputs.uniform(90, 8)]
    ok = acs.Batch(small, seed=1, torch_memory=False)
    ok.iterate(2)
    for i, x in enumerate(small):
        assert np.array_equal(np.sort(ok.best(i)[0]), np.arange(len(x)))
    ok.close()
