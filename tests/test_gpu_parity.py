"""Parity of the HIP path with the CPU oracle (synchronous mode: bit-exact).

Every test drives the library through its C-ABI (ctypes binding) on the GPU
and the oracle on the CPU with the same instance, parameters and seed, and
compares tours, lengths, the best-so-far tour and the pheromone element by
element after every iteration.
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


def _pair(acs, xy, **kw):
    memory = kw.pop("memory", 0)
    mode = kw.pop("mode", 0)
    col = acs.Colony(xy, memory=memory, mode=mode, **kw)
    orc = oracle.Oracle(xy, memory=memory, **kw)
    return col, orc


def _compare(col, orc, it, tau=True):
    assert np.array_equal(col.tours(), orc.tours()), f"tours differ at iteration {it}"
    assert np.array_equal(col.lengths(), orc.lengths()), f"lengths differ at iteration {it}"
    gt, gl = col.best()
    ot, ol = orc.best()
    assert gl == ol, f"best length {gl} != {ol} at iteration {it}"
    assert np.array_equal(gt, ot), f"best tour differs at iteration {it}"
    if tau:
        if col.memory == 0:
            a, b = col.tau(), orc.tau()
            bad = np.argwhere(a != b)
            assert bad.size == 0, f"pheromone differs at {len(bad)} entries, first {bad[:3].tolist()} (iteration {it})"
        else:
            for x, y, name in zip(col.spm(), orc.spm(), ("nodes", "vals", "tail")):
                assert np.array_equal(x, y), f"SPM {name} differ at iteration {it}"
    st, oc = col.stats(), orc.counts()
    for k in ("greedy", "roulette", "fallback"):
        assert st[k] == oc[k], f"{k} count {st[k]} != {oc[k]} at iteration {it}"


def test_instance_preparation_matches(acs):
    for n, kind in [(198, "uniform"), (1000, "clustered"), (67, "coincident")]:
        _say(f"prep n={n} {kind}")
        xy = {"uniform": inputs.uniform, "clustered": inputs.clustered,
              "coincident": lambda n: inputs.coincident(n, 3)}[kind](n)
        col, orc = _pair(acs, xy)
        assert np.array_equal(col.cand(), orc.cand())
        st, c = col.stats(), orc.constants()
        assert st["nn_length"] == c["lnn"]
        assert np.float32(st["tau0"]) == c["tau0"]
        col.close()


def test_config1_n198_sync_100_iterations(acs):
    """n=198 uniform, m=198, cl=32, beta=2, q0=0.9, phi=rho=0.1, dense, sync."""
    xy = inputs.uniform(198)
    col, orc = _pair(acs, xy, seed=0)
    for it in range(100):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


@pytest.mark.parametrize("n,kind,iters", [(1000, "clustered", 3), (2392, "uniform", 2)])
def test_full_size_sync_first_iterations(acs, n, kind, iters):
    oracle.set_threads(16)
    xy = inputs.uniform(n) if kind == "uniform" else inputs.clustered(n)
    col, orc = _pair(acs, xy, seed=7)
    for it in range(iters):
        _say(f"n={n} {kind} iteration {it}")
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()
    oracle.set_threads(1)


EDGE_CASES = [
    # (name, n, kwargs)
    ("n3", 3, {}),
    ("n4_cl1", 4, {"cl": 1}),
    ("n5_m1", 5, {"m": 1}),
    ("n33_cl16", 33, {"cl": 16}),
    ("n65_cl48", 65, {"cl": 48}),
    ("n70_cl64", 70, {"cl": 64}),
    ("n100_q0_0", 100, {"q0": 0.0}),
    ("n100_q0_1", 100, {"q0": 1.0}),
    ("n129_m37", 129, {"m": 37}),
    ("n257_m600", 257, {"m": 600, "cl": 20}),
    ("n50_beta3", 50, {"beta": 3.0, "phi": 0.01, "rho": 0.2}),
    ("coincident", 60, {}),
]


@pytest.mark.parametrize("name,n,kw", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
def test_edge_cases_sync(acs, name, n, kw):
    _say(f"edge case {name}")
    xy = inputs.coincident(n, 5) if name == "coincident" else inputs.uniform(n, 100 + n)
    col, orc = _pair(acs, xy, seed=3, **kw)
    for it in range(5):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


def test_split_iterate_calls(acs):
    xy = inputs.uniform(150, 9)
    a = acs.Colony(xy, seed=4)
    b = acs.Colony(xy, seed=4)
    a.iterate(3)
    b.iterate(1); b.iterate(2)
    assert np.array_equal(a.tau(), b.tau())
    assert np.array_equal(a.tours(), b.tours())
    a.close(); b.close()


def test_library_stream_and_memory(acs):
    """The library's own stream and allocation give the same results."""
    xy = inputs.uniform(120, 2)
    a = acs.Colony(xy, seed=5, torch_memory=False)
    orc = oracle.Oracle(xy, seed=5)
    for it in range(3):
        a.iterate(1)
        orc.iterate(1)
        _compare(a, orc, it)
    a.close()


# ---------------------------------------------------------------------------
# Asynchronous atomic mode: no bit-exact reference (reads race with the
# other ants' updates).  Checked by validity, by one ant (where it must equal
# the synchronous schedule exactly) and by its quality distribution.
# ---------------------------------------------------------------------------
def test_async_single_ant_equals_oracle(acs):
    xy = inputs.uniform(300, 4)
    col = acs.Colony(xy, m=1, mode=acs.ACS_ASYNC_ATOMIC, seed=2)
    orc = oracle.Oracle(xy, m=1, seed=2)
    for it in range(10):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


@pytest.mark.parametrize("n,kind", [(198, "uniform"), (1000, "clustered"), (2392, "uniform")])
def test_async_tours_valid(acs, n, kind):
    xy = inputs.uniform(n) if kind == "uniform" else inputs.clustered(n)
    col = acs.Colony(xy, mode=acs.ACS_ASYNC_ATOMIC, seed=1)
    orc = oracle.Oracle(xy, m=1)
    d = orc.dist().astype(np.int64)
    c = orc.constants()
    for it in range(3):
        _say(f"async n={n} iteration {it}")
        col.iterate(1)
        tours, lens = col.tours(), col.lengths()
        assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
        rec = d[tours, np.roll(tours, -1, axis=1)].sum(axis=1)
        assert np.array_equal(rec, lens)
        best, L = col.best()
        assert L == lens.min() or L < lens.min()
        assert defs.tour_length(d, best) == L
        tau = col.tau()
        assert np.all(np.isfinite(tau)) and np.all(tau > 0)
        # the local map pulls toward tau0 and the global one toward 1/L_gb
        assert tau.min() >= c["tau0"] * np.float32(0.999)
        st = col.stats()
        assert st["steps"] == (it + 1) * n * (n - 1)
    col.close()


def test_async_quality_distribution(acs):
    """20 seeds of async vs sync on n=198 after 50 iterations: both beat the
    nearest-neighbour tour and their mean best lengths are within 3%."""
    from scipy.stats import mannwhitneyu
    xy = inputs.uniform(198)
    res = {0: [], 1: []}
    for mode in (0, 1):
        for s in range(20):
            col = acs.Colony(xy, mode=mode, seed=s)
            col.iterate(50)
            res[mode].append(col.best()[1])
            lnn = col.stats()["nn_length"]
            col.close()
    sync, asy = np.array(res[0]), np.array(res[1])
    assert sync.max() < lnn and asy.max() < lnn
    assert abs(asy.mean() - sync.mean()) / sync.mean() < 0.03
    p = mannwhitneyu(sync, asy).pvalue
    _say(f"sync mean {sync.mean():.1f}, async mean {asy.mean():.1f}, rank-sum p={p:.3f}")
