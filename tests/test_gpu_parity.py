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


def test_n198_sync_100_iterations(acs):
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
    # the dense fallback's prefix (the 128 cities after the candidates) is
    # used from n - 1 > cl + 128 on
    ("n162_cl32_prefix", 162, {}),
    ("n161_cl32_no_prefix", 161, {}),
    ("n400_cl2_fallbacks", 400, {"cl": 2}),
    ("lattice_n400_cl4", 400, {"cl": 4}),
    ("lattice_n324_cl8_beta0", 324, {"cl": 8, "beta": 0.0}),
]


@pytest.mark.parametrize("name,n,kw", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
def test_edge_cases_sync(acs, name, n, kw):
    _say(f"edge case {name}")
    if name == "coincident":
        xy = inputs.coincident(n, 5)
    elif name.startswith("lattice"):
        xy = inputs.lattice(int(round(n ** 0.5)), n)
    else:
        xy = inputs.uniform(n, 100 + n)
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


@pytest.mark.parametrize("gpu", [dict(update_path=2), dict(update_path=1),
                                 dict(lanes_per_ant=32), dict(lanes_per_ant=16)],
                         ids=["queued", "inwave", "lanes32", "lanes16"])
def test_async_single_ant_fallback_heavy_equals_oracle(acs, gpu):
    """One ant on a 20 x 20 grid with cl = 4: the fallback decides many steps
    (through its prefix or the whole row) once the global updates have made
    the trails unequal, and one ant must follow the synchronous schedule."""
    xy = inputs.lattice(20, 5)
    col = acs.Colony(xy, m=1, cl=4, mode=acs.ACS_ASYNC_ATOMIC, seed=4, **gpu)
    orc = oracle.Oracle(xy, m=1, cl=4, seed=4)
    for it in range(12):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    assert col.stats()["fallback"] == orc.counts()["fallback"] > 0
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


# ---------------------------------------------------------------------------
# Selective pheromone memory (Sec. 3.2, Alg. 3): records, tails and tours
# bit-exact in synchronous mode.
# ---------------------------------------------------------------------------
SPM_CASES = [
    ("n300_m60_s8", 300, dict(m=60, cl=16, spm_s=8), 6),
    ("n201_m201_s4", 201, dict(cl=32, spm_s=4), 4),
    ("n150_m33_s1", 150, dict(m=33, cl=10, spm_s=1), 4),
    ("n97_m200_s16_q0", 97, dict(m=200, cl=20, spm_s=16, q0=0.0), 4),
    # about 130 updates of each record in every step: the record's update
    # list is longer than one wave and is gathered by scanning every
    # registration instead
    ("n6_m400_s2", 6, dict(m=400, cl=3, spm_s=2), 4),
]


@pytest.mark.parametrize("name,n,kw,iters", SPM_CASES, ids=[c[0] for c in SPM_CASES])
def test_spm_sync_parity(acs, name, n, kw, iters):
    _say(f"SPM sync {name}")
    xy = inputs.uniform(n, 500 + n)
    col, orc = _pair(acs, xy, memory=1, seed=11, **kw)
    for it in range(iters):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
        st, oc = col.stats(), orc.counts()
        assert st["spm_hits"] == oc["spm_hits"] and st["spm_misses"] == oc["spm_misses"]
    col.close()


def test_spm_without_eviction_equals_dense_on_gpu(acs):
    n = 16
    xy = inputs.uniform(n, 77)
    spm = acs.Colony(xy, cl=8, memory=1, spm_s=n - 1, seed=2)
    den = acs.Colony(xy, cl=8, memory=0, seed=2)
    for it in range(8):
        spm.iterate(1)
        den.iterate(1)
        assert np.array_equal(spm.tours(), den.tours())
        # the logical pheromone of the records equals the dense matrix
        nodes, vals, _ = spm.spm()
        tau = np.full((n, n), np.float32(spm.stats()["tau0"]))
        for i in range(n):
            for slot in range(n - 1):
                if nodes[i, slot] >= 0:
                    tau[i, nodes[i, slot]] = vals[i, slot]
        dt = den.tau()
        off = ~np.eye(n, dtype=bool)
        assert np.array_equal(tau[off], dt[off])
    spm.close(); den.close()


def test_spm_full_size_first_iteration(acs):
    """n=20000 uniform, m=1024, cl=16, s=8: the first iteration bit-exact."""
    oracle.set_threads(16)
    xy = inputs.uniform(20000)
    _say("SPM n=20000 create")
    col = acs.Colony(xy, m=1024, cl=16, memory=1, spm_s=8, seed=3)
    orc = oracle.Oracle(xy, m=1024, cl=16, memory=1, spm_s=8, seed=3)
    _say("SPM n=20000 iteration 0")
    col.iterate(1)
    orc.iterate(1)
    _compare(col, orc, 0)
    col.close()
    oracle.set_threads(1)


@pytest.mark.parametrize("n,m", [(300, 300), (20000, 1024)])
def test_spm_async_tours_valid(acs, n, m):
    xy = inputs.uniform(n)
    col = acs.Colony(xy, m=m, cl=16, memory=1, spm_s=8, mode=acs.ACS_ASYNC_ATOMIC, seed=1)
    for it in range(2):
        _say(f"SPM async n={n} iteration {it}")
        col.iterate(1)
        tours, lens = col.tours(), col.lengths()
        assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
        d = None
        if n <= 1000:
            d = defs.dist_matrix(xy)
            rec = d[tours, np.roll(tours, -1, axis=1)].sum(axis=1)
            assert np.array_equal(rec, lens)
        nodes, vals, tail = col.spm()
        assert np.all((nodes >= -1) & (nodes < n))
        assert np.all(np.isfinite(vals)) and np.all(vals > 0)
        assert np.all((tail >= 0) & (tail < 8))
        st = col.stats()
        assert st["steps"] == (it + 1) * m * (n - 1)
        assert st["spm_hits"] + st["spm_misses"] == (it + 1) * (2 * m * n + 2 * n)
    col.close()


def _grid_instance(kind, n, seed):
    if kind == "clustered":
        return inputs.clustered(n, seed)
    if kind == "line":
        xy = inputs.uniform(n, seed)
        xy[:, 1] = 5000.0  # every city on one horizontal line: a grid one cell high
        return xy
    # every location taken by four cities: distance 0 within a group, ties
    # between the group's cities everywhere else
    return np.ascontiguousarray(np.repeat(inputs.uniform(n // 4, seed), 4, axis=0))


# The selective memory's fallback past its 128-city list searches a grid of
# cells ring by ring (exact, ties to the lower index).  Short candidate lists
# on instances where the list runs out often: clustered cities, cities on a
# line (a grid one cell high) and coincident cities (distance 0).
GRID_CASES = [
    ("clustered_n600", "clustered", 600, dict(m=64, cl=4, spm_s=4), 3),
    ("line_n400", "line", 400, dict(m=50, cl=4, spm_s=8), 3),
    ("coincident_n320", "coincident", 320, dict(m=40, cl=3, spm_s=2), 3),
]


@pytest.mark.parametrize("name,kind,n,kw,iters", GRID_CASES, ids=[c[0] for c in GRID_CASES])
def test_spm_grid_search_sync_parity(acs, name, kind, n, kw, iters):
    _say(f"SPM grid search {name}")
    xy = _grid_instance(kind, n, 900 + n)
    col, orc = _pair(acs, xy, memory=1, seed=5, **kw)
    for it in range(iters):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    assert col.stats()["fallback"] > 0
    col.close()


@pytest.mark.parametrize("kind", ["clustered", "line"])
def test_spm_grid_search_single_ant_equals_oracle(acs, kind):
    _say(f"SPM grid search, one asynchronous ant, {kind}")
    xy = _grid_instance(kind, 500, 77)
    col = acs.Colony(xy, m=1, cl=4, memory=1, spm_s=4, mode=acs.ACS_ASYNC_ATOMIC, seed=4)
    orc = oracle.Oracle(xy, m=1, cl=4, memory=1, spm_s=4, seed=4)
    for it in range(4):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


def test_spm_async_single_ant_equals_oracle(acs):
    xy = inputs.uniform(250, 6)
    col = acs.Colony(xy, m=1, cl=12, memory=1, spm_s=6, mode=acs.ACS_ASYNC_ATOMIC, seed=8)
    orc = oracle.Oracle(xy, m=1, cl=12, memory=1, spm_s=6, seed=8)
    for it in range(6):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


# ---------------------------------------------------------------------------
# Batches: many instances in one graph-replayed launch per iteration.
# ---------------------------------------------------------------------------
def test_batch_single_ant_equals_oracle(acs):
    """With one ant per instance the asynchronous schedule equals the
    synchronous one, so every instance of the batch must match the oracle
    run with its own counter word (instance = i) bit for bit."""
    insts = inputs.batch(6, seed=31, nmin=40, nmax=300)
    b = acs.Batch(insts, m=1, cl=16, seed=5)
    orcs = [oracle.Oracle(x, m=1, cl=16, seed=5, instance=i) for i, x in enumerate(insts)]
    assert b.info()["count"] == 6
    for it in range(4):
        b.iterate(1)
        for i, o in enumerate(orcs):
            o.iterate(1)
            assert np.array_equal(b.tours(i), o.tours()), (i, it)
            assert np.array_equal(b.lengths(i), o.lengths()), (i, it)
            assert b.best(i)[1] == o.best()[1], (i, it)
            assert np.array_equal(b.tau(i), o.tau()), (i, it)
    b.close()


def test_batch_single_ant_fallback_heavy_equals_oracle(acs):
    """Grids with cl = 4 in a batch (fallbacks at many steps, every weight
    tied), one ant each, over the iterations in which the batch tries every
    launch shape: each instance matches the oracle bit for bit."""
    insts = [inputs.lattice(14, 1), inputs.lattice(20, 2), inputs.uniform(300, 3),
             inputs.lattice(11, 4)]
    b = acs.Batch(insts, m=1, cl=4, seed=8)
    orcs = [oracle.Oracle(x, m=1, cl=4, seed=8, instance=i) for i, x in enumerate(insts)]
    for it in range(6):
        b.iterate(1)
        for i, o in enumerate(orcs):
            o.iterate(1)
            assert np.array_equal(b.tours(i), o.tours()), (i, it)
            assert np.array_equal(b.tau(i), o.tau()), (i, it)
    b.close()


def test_batch_tours_valid(acs):
    insts = inputs.batch(24, seed=7, nmin=60, nmax=400)
    b = acs.Batch(insts, seed=2)
    info = b.info()
    _say(f"batch info {info}")
    b.iterate(3)
    total = 0
    for i, xy in enumerate(insts):
        n = len(xy)
        tours, lens = b.tours(i), b.lengths(i)
        assert tours.shape == (n, n)
        assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
        d = defs.dist_matrix(xy)
        assert np.array_equal(d[tours, np.roll(tours, -1, axis=1)].sum(axis=1), lens)
        best, L = b.best(i)
        assert defs.tour_length(d, best) == L
        st = b.stats(i)
        assert st["steps"] == 3 * n * (n - 1) and st["iteration"] == 3
        total += n * (n - 1)
    assert info["steps_per_iteration"] == total
    b.close()


# ---------------------------------------------------------------------------
# Local-update period k (Sec. 4): only the edges of steps k, 2k, ... and the
# closing edge get Eq. 3.  Synchronous mode stays bit-exact; one ant makes
# the asynchronous and batched kernels equal the oracle too.
# ---------------------------------------------------------------------------
PERIOD_CASES = [
    ("dense_k2_n198", 198, dict(local_update_period=2), 6),
    ("dense_k5_ragged", 141, dict(m=77, cl=16, local_update_period=5), 6),
    ("dense_k16_n1000_clustered", 1000, dict(m=256, local_update_period=16), 2),
    ("dense_k_n_minus_1", 97, dict(local_update_period=96), 4),
    ("dense_k_above_n", 64, dict(local_update_period=1000), 4),
    ("spm_k4", 300, dict(cl=16, memory=1, spm_s=8, local_update_period=4), 4),
    ("spm_k7_ragged", 173, dict(m=61, cl=12, memory=1, spm_s=4, local_update_period=7), 4),
]


@pytest.mark.parametrize("name,n,kw,iters", PERIOD_CASES, ids=[c[0] for c in PERIOD_CASES])
def test_local_update_period_sync_parity(acs, name, n, kw, iters):
    _say(f"period case {name}")
    xy = inputs.clustered(n, n + 3) if "clustered" in name else inputs.uniform(n, n + 3)
    col, orc = _pair(acs, xy, seed=4, **kw)
    for it in range(iters):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


@pytest.mark.parametrize("memory", [0, 1])
def test_local_update_period_async_single_ant(acs, memory):
    xy = inputs.uniform(260, 19)
    kw = dict(m=1, cl=16, memory=memory, spm_s=6, seed=3, local_update_period=3)
    col = acs.Colony(xy, mode=acs.ACS_ASYNC_ATOMIC, **kw)
    orc = oracle.Oracle(xy, **kw)
    for it in range(5):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


def test_local_update_period_batch_single_ant(acs):
    insts = inputs.batch(5, seed=41, nmin=50, nmax=250)
    b = acs.Batch(insts, m=1, cl=16, seed=6, local_update_period=4)
    orcs = [oracle.Oracle(x, m=1, cl=16, seed=6, instance=i, local_update_period=4)
            for i, x in enumerate(insts)]
    for it in range(3):
        b.iterate(1)
        for i, o in enumerate(orcs):
            o.iterate(1)
            assert np.array_equal(b.tours(i), o.tours()), (i, it)
            assert np.array_equal(b.tau(i), o.tau()), (i, it)
    b.close()


def test_local_update_period_async_valid(acs):
    n = 1000
    xy = inputs.uniform(n, 5)
    col = acs.Colony(xy, mode=acs.ACS_ASYNC_ATOMIC, seed=1, local_update_period=8)
    col.iterate(3)
    tours, lens = col.tours(), col.lengths()
    assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
    assert np.array_equal(defs.tour_lengths(xy, tours), lens)
    col.close()


# ---------------------------------------------------------------------------
# Unsynchronised mode without atomics (the paper's ACS-GPU-Alt): updates that
# race are lost, so only one ant has an exact reference; many ants are
# checked for valid tours, consistent lengths and pheromone bounds.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("memory", [0, 1])
def test_racy_single_ant_equals_oracle(acs, memory):
    xy = inputs.uniform(240, 23)
    kw = dict(m=1, cl=16, memory=memory, spm_s=5, seed=9)
    col = acs.Colony(xy, mode=acs.ACS_ASYNC_RACY, **kw)
    orc = oracle.Oracle(xy, **kw)
    for it in range(6):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


@pytest.mark.parametrize("n,m,memory", [(1000, 1000, 0), (2392, 2392, 0), (20000, 1024, 1)])
def test_racy_tours_valid(acs, n, m, memory):
    _say(f"racy n={n} m={m} memory={memory}")
    xy = inputs.uniform(n)
    cl = 16 if memory else 32
    col = acs.Colony(xy, m=m, cl=cl, memory=memory, spm_s=8, mode=acs.ACS_ASYNC_RACY, seed=3)
    col.iterate(2 if n < 20000 else 1)
    tours, lens = col.tours(), col.lengths()
    assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
    assert np.array_equal(defs.tour_lengths(xy, tours), lens)
    c = col.stats()
    if memory == 0:
        tau = col.tau()
        assert np.all(np.isfinite(tau)) and tau.min() >= np.float32(c["tau0"]) * np.float32(0.999)
    else:
        nodes, vals, _ = col.spm()
        assert np.all((nodes == -1) | ((nodes >= 0) & (nodes < n)))
        assert np.all(np.isfinite(vals)) and vals.min() >= np.float32(c["tau0"]) * np.float32(0.999)
    col.close()


def test_racy_batch_single_ant_equals_oracle(acs):
    insts = inputs.batch(4, seed=51, nmin=50, nmax=200)
    b = acs.Batch(insts, m=1, cl=16, seed=2, mode=acs.ACS_ASYNC_RACY)
    orcs = [oracle.Oracle(x, m=1, cl=16, seed=2, instance=i) for i, x in enumerate(insts)]
    for it in range(3):
        b.iterate(1)
        for i, o in enumerate(orcs):
            o.iterate(1)
            assert np.array_equal(b.tours(i), o.tours()), (i, it)
            assert np.array_equal(b.tau(i), o.tau()), (i, it)
    b.close()


# ---------------------------------------------------------------------------
# First iteration of the asynchronous kernels.  Every entry starts at tau0 and
# the local map fixes tau0 (f(tau0) = tau0 in FP32, checked on the oracle),
# so no read can see another ant's update: with any number of ants, any
# number of ants per wavefront and either update kind, the first iteration's
# tours must equal the synchronous oracle's bit for bit.
# ---------------------------------------------------------------------------
ASYNC_FIRST = [
    ("atomic_l64", dict(), 64, "ASYNC_ATOMIC"),
    ("atomic_l32", dict(), 32, "ASYNC_ATOMIC"),
    ("racy_l32", dict(), 32, "ASYNC_RACY"),
    ("atomic_l16_cl16", dict(cl=16), 16, "ASYNC_ATOMIC"),
    ("racy_l16_ragged", dict(cl=12, m=203), 16, "ASYNC_RACY"),
    ("racy_l64", dict(m=333), 64, "ASYNC_RACY"),
    ("spm_atomic", dict(cl=16, memory=1, spm_s=8), 0, "ASYNC_ATOMIC"),
    ("spm_racy", dict(cl=16, memory=1, spm_s=4, m=250), 0, "ASYNC_RACY"),
    ("queued_atomic", dict(), -2, "ASYNC_ATOMIC"),
    ("queued_racy_ragged", dict(m=333), -2, "ASYNC_RACY"),
    # a grid with cl = 4: fallbacks at many steps, ties in every weight
    ("queued_atomic_lattice_cl4", dict(cl=4), -2, "ASYNC_ATOMIC"),
    ("inwave_atomic_lattice_cl4", dict(cl=4), -1, "ASYNC_ATOMIC"),
    ("inwave_racy_lattice_cl4", dict(cl=4), -1, "ASYNC_RACY"),
    ("atomic_l32_lattice_cl4", dict(cl=4), 32, "ASYNC_ATOMIC"),
    ("atomic_l16_lattice_cl4", dict(cl=4), 16, "ASYNC_ATOMIC"),
    ("racy_l32_lattice_cl4", dict(cl=4), 32, "ASYNC_RACY"),
]


@pytest.mark.parametrize("name,kw,lanes,mode", ASYNC_FIRST, ids=[c[0] for c in ASYNC_FIRST])
def test_async_first_iteration_equals_oracle(acs, name, kw, lanes, mode):
    n = 733
    if "lattice" in name:
        xy = inputs.lattice(27, 77)
    else:
        xy = inputs.clustered(n, 77) if "ragged" in name else inputs.uniform(n, 77)
    orc = oracle.Oracle(xy, seed=12, **kw)
    c = orc.constants()
    assert orc.local_map_k(c["tau0"], 1) == c["tau0"]
    gpu = dict(lanes_per_ant=lanes) if lanes >= 0 else dict(update_path=-lanes)
    col = acs.Colony(xy, mode=getattr(acs, "ACS_" + mode), seed=12, **gpu, **kw)
    col.iterate(1)
    orc.iterate(1)
    assert np.array_equal(col.tours(), orc.tours())
    assert np.array_equal(col.lengths(), orc.lengths())
    assert col.best()[1] == orc.best()[1]
    st, oc = col.stats(), orc.counts()
    for k in ("greedy", "roulette", "fallback"):
        assert st[k] == oc[k], k
    col.close()


@pytest.mark.parametrize("lanes", [32, 16])
def test_grouped_single_ant_equals_oracle(acs, lanes):
    xy = inputs.uniform(310, 31)
    col = acs.Colony(xy, m=1, cl=16, mode=acs.ACS_ASYNC_ATOMIC, seed=5, lanes_per_ant=lanes)
    orc = oracle.Oracle(xy, m=1, cl=16, seed=5)
    for it in range(6):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


@pytest.mark.parametrize("lanes,mode", [(32, "ASYNC_ATOMIC"), (16, "ASYNC_RACY")])
def test_grouped_tours_valid(acs, lanes, mode):
    n = 1500
    xy = inputs.uniform(n, 8)
    col = acs.Colony(xy, cl=16, mode=getattr(acs, "ACS_" + mode), seed=2, lanes_per_ant=lanes)
    col.iterate(3)
    tours, lens = col.tours(), col.lengths()
    assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
    assert np.array_equal(defs.tour_lengths(xy, tours), lens)
    assert col.stats()["steps"] == 3 * n * (n - 1)
    col.close()


def test_batch_tuner_picks_a_shape_and_keeps_iterating(acs):
    insts = inputs.batch(40, seed=61, nmin=100, nmax=700)
    b = acs.Batch(insts, cl=16, seed=3)
    assert b.tuning()["chosen"] is None
    b.iterate(2)  # warm-up + first candidate
    b.iterate(3)  # the other candidates, then the chosen shape
    tu = b.tuning()
    _say(f"batch tuning {tu}")
    assert set(tu["candidates"]) == {"64", "64u", "32", "16"}
    assert all(v > 0 for v in tu["candidates"].values())
    assert tu["chosen"] == min(tu["candidates"], key=tu["candidates"].get)
    for i, xy in enumerate(insts):
        tours, lens = b.tours(i), b.lengths(i)
        assert np.all(np.sort(tours, axis=1) == np.arange(len(xy))[None, :])
        assert np.array_equal(defs.tour_lengths(xy, tours), lens)
        assert b.stats(i)["iteration"] == 5
    b.close()


@pytest.mark.parametrize("lanes", [32, 16])
def test_batch_grouped_single_ant_equals_oracle(acs, lanes):
    insts = inputs.batch(5, seed=71, nmin=40, nmax=260)
    b = acs.Batch(insts, m=1, cl=16, seed=4, lanes_per_ant=lanes)
    orcs = [oracle.Oracle(x, m=1, cl=16, seed=4, instance=i) for i, x in enumerate(insts)]
    for it in range(3):
        b.iterate(1)
        for i, o in enumerate(orcs):
            o.iterate(1)
            assert np.array_equal(b.tours(i), o.tours()), (i, it)
            assert np.array_equal(b.tau(i), o.tau()), (i, it)
    b.close()


# ---------------------------------------------------------------------------
# Local updates through the updater wave's LDS rings (update_path = 2).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["ASYNC_ATOMIC", "ASYNC_RACY"])
def test_queued_single_ant_equals_oracle(acs, mode):
    xy = inputs.uniform(280, 33)
    col = acs.Colony(xy, m=1, mode=getattr(acs, "ACS_" + mode), seed=6, update_path=2)
    orc = oracle.Oracle(xy, m=1, seed=6)
    for it in range(6):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


@pytest.mark.parametrize("n,m,period", [(2392, 2392, 1), (30, 2000, 1), (1000, 1001, 3)])
def test_queued_tours_valid(acs, n, m, period):
    """Full size, heavy contention on a tiny instance (many updates of the
    same entries at once) and a ragged ant count with a local-update period."""
    _say(f"queued n={n} m={m} period={period}")
    xy = inputs.uniform(n, 44)
    col = acs.Colony(xy, m=m, cl=min(32, n - 1), mode=acs.ACS_ASYNC_ATOMIC, seed=7,
                     update_path=2, local_update_period=period)
    c = None
    for it in range(3):
        col.iterate(1)
        tours, lens = col.tours(), col.lengths()
        assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
        assert np.array_equal(defs.tour_lengths(xy, tours), lens)
        c = col.stats()
        assert c["steps"] == (it + 1) * m * (n - 1)
    tau = col.tau()
    assert np.all(np.isfinite(tau)) and tau.min() >= np.float32(c["tau0"]) * np.float32(0.999)
    col.close()


@pytest.mark.parametrize("mode", ["ASYNC_ATOMIC", "ASYNC_RACY"])
def test_updater_path_quality_matches_inwave(acs, mode):
    """The updater wave applies a crossing's update a few steps after the
    crossing; the ant applying it itself does so one step after.  On n=198
    (where a delay is a large share of a tour) 10 seeds of 50 iterations of
    both paths must reach mean best lengths within 2.5% of each other, so
    the hand-over changes neither when updates become visible nor how many
    are lost in any way that shows in the search."""
    xy = inputs.uniform(198)
    means = {}
    for path in (1, 2):
        res = []
        for s in range(10):
            col = acs.Colony(xy, mode=getattr(acs, "ACS_" + mode), seed=s, update_path=path)
            col.iterate(50)
            res.append(col.best()[1])
            col.close()
        means[path] = float(np.mean(res))
    _say(f"{mode}: in-wave {means[1]:.0f}, updater {means[2]:.0f}")
    assert abs(means[2] - means[1]) / means[1] < 0.025, means


ACCUMULATE_PATHS = [("queued", dict(update_path=2)), ("inwave", dict(update_path=1)),
                    ("lanes32", dict(lanes_per_ant=32))]


@pytest.mark.parametrize("path,gkw", ACCUMULATE_PATHS, ids=[p[0] for p in ACCUMULATE_PATHS])
def test_async_local_updates_accumulate_exactly(acs, path, gkw):
    """Many ants, compare-and-swap mode: whatever the interleaving, every
    entry ends the iteration at f^c(tau) (Eq. 3 applied c times in fp32, c =
    the number of ants whose tour crosses the edge, closing edges included),
    followed on the best-so-far tour's edges by Eq. 4, and the matrix stays
    symmetric: no local update is lost or applied to one direction only."""
    n = 1000
    _say(f"accumulate {path} n={n} m={n}")
    xy = inputs.uniform(n, 61)
    col = acs.Colony(xy, m=n, mode=acs.ACS_ASYNC_ATOMIC, seed=5, **gkw)
    orc = oracle.Oracle(xy, m=1, seed=5)
    c = orc.constants()
    col.iterate(4)
    before = col.tau()
    assert np.array_equal(before, before.T)
    col.iterate(1)
    after = col.tau()
    assert np.array_equal(after, after.T)
    tours = col.tours().astype(np.int64)
    a, b = tours, np.roll(tours, -1, axis=1)
    key = np.minimum(a, b) * n + np.maximum(a, b)
    keys, counts = np.unique(key.ravel(), return_counts=True)
    crossed = dict(zip(keys.tolist(), counts.tolist()))
    best, L = col.best()
    bt = np.asarray(best, dtype=np.int64)
    bkeys = (np.minimum(bt, np.roll(bt, -1)) * n + np.maximum(bt, np.roll(bt, -1))).tolist()
    # Eq. 4's deposit as the library computes it: rho / L_gb in double, then float
    bg = np.float32(0.1 / L)
    expect = {}
    for kk, cnt in crossed.items():
        u, v = divmod(kk, n)
        expect[kk] = orc.local_map_k(before[u, v], cnt)
    for kk in bkeys:
        u, v = divmod(kk, n)
        x = expect.get(kk, before[u, v])
        expect[kk] = defs.fmaf32(c["a_glob"], x, bg)
    # entries away from tau0 that ants crossed: there a lost or doubled
    # local update changes the result (tau0 is the local map's fixed point)
    strong = 0
    for kk, want in expect.items():
        u, v = divmod(kk, n)
        assert after[u, v] == want, (u, v, crossed.get(kk, 0), before[u, v], after[u, v], want)
        strong += int(kk in crossed and before[u, v] != c["tau0"])
    # every other entry keeps its value
    touched = np.zeros(n * n, dtype=bool)
    touched[list(expect)] = True
    touched = touched.reshape(n, n)
    touched |= touched.T
    assert np.array_equal(after[~touched], before[~touched])
    assert len(expect) > n and strong > n // 2, (len(expect), strong)
    col.close()


# ---------------------------------------------------------------------------
# Edge cases of the asynchronous kernels (default updater path, in-wave
# updates, several ants per wavefront): one ant must equal the oracle, any
# number of ants must give valid tours.
# ---------------------------------------------------------------------------
ASYNC_EDGE = [
    ("n3", 3, dict()),
    ("n4_cl1", 4, dict(cl=1)),
    ("n5_q0_zero", 5, dict(q0=0.0)),
    ("n9_q0_one", 9, dict(q0=1.0)),
    ("n65_cl64", 65, dict(cl=64)),
    ("n130_cl16_beta3", 130, dict(cl=16, beta=3.0)),
]
ASYNC_PATHS = [("queued", dict(update_path=2)), ("inwave", dict(update_path=1)),
               ("lanes16", dict(lanes_per_ant=16))]


@pytest.mark.parametrize("path,gkw", ASYNC_PATHS, ids=[p[0] for p in ASYNC_PATHS])
@pytest.mark.parametrize("name,n,kw", ASYNC_EDGE, ids=[c[0] for c in ASYNC_EDGE])
def test_async_edge_cases(acs, name, n, kw, path, gkw):
    if path == "lanes16" and kw.get("cl", 32) > 16 and n - 1 > 16:
        pytest.skip("16 lanes per ant hold at most 16 candidates")
    xy = inputs.uniform(n, 1000 + n)
    col = acs.Colony(xy, m=1, mode=acs.ACS_ASYNC_ATOMIC, seed=7, **kw, **gkw)
    orc = oracle.Oracle(xy, m=1, seed=7, **kw)
    for it in range(4):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()
    m = 3 * n + 5
    col = acs.Colony(xy, m=m, mode=acs.ACS_ASYNC_ATOMIC, seed=7, **kw, **gkw)
    col.iterate(3)
    tours, lens = col.tours(), col.lengths()
    assert np.all(np.sort(tours, axis=1) == np.arange(n)[None, :])
    assert np.array_equal(defs.tour_lengths(xy, tours), lens)
    col.close()


def test_batch_updater_wave_single_ant_equals_oracle(acs):
    insts = inputs.batch(5, seed=81, nmin=40, nmax=300)
    b = acs.Batch(insts, m=1, cl=16, seed=8, lanes_per_ant=64, update_path=2)
    assert set(b.tuning()["candidates"]) == {"64u"}
    orcs = [oracle.Oracle(x, m=1, cl=16, seed=8, instance=i) for i, x in enumerate(insts)]
    for it in range(3):
        b.iterate(1)
        for i, o in enumerate(orcs):
            o.iterate(1)
            assert np.array_equal(b.tours(i), o.tours()), (i, it)
            assert np.array_equal(b.tau(i), o.tau()), (i, it)
    b.close()


# ---------------------------------------------------------------------------
# Sequential mode (Alg. 1 read literally, in-step Gauss-Seidel): bit-exact
# against the oracle's sequential schedule.
# ---------------------------------------------------------------------------
SEQ_CASES = [
    ("n198", 198, dict(), 4),
    ("n141_m77_cl16_ragged", 141, dict(m=77, cl=16), 4),
    ("n300_clustered_m300", 300, dict(), 3),
    ("n120_period3", 120, dict(local_update_period=3), 4),
    ("n1000_clustered_m64", 1000, dict(m=64), 2),
    ("n65_cl64", 65, dict(cl=64), 3),
    ("n3_m1", 3, dict(m=1), 3),
    ("n5_q0_zero_m9", 5, dict(m=9, q0=0.0), 3),
    ("n40_q0_one_m40", 40, dict(q0=1.0), 3),
    ("lattice_n400_cl4", 400, dict(cl=4), 3),
]


@pytest.mark.parametrize("name,n,kw,iters", SEQ_CASES, ids=[c[0] for c in SEQ_CASES])
def test_sequential_equals_oracle(acs, name, n, kw, iters):
    _say(f"sequential {name}")
    if "clustered" in name:
        xy = inputs.clustered(n, n + 9)
    elif name.startswith("lattice"):
        xy = inputs.lattice(int(round(n ** 0.5)), n)
    else:
        xy = inputs.uniform(n, n + 9)
    col = acs.Colony(xy, mode=acs.ACS_SEQUENTIAL, seed=6, **kw)
    orc = oracle.Oracle(xy, mode=oracle.SEQUENTIAL, seed=6, **kw)
    for it in range(iters):
        col.iterate(1)
        orc.iterate(1)
        _compare(col, orc, it)
    col.close()


def test_sequential_differs_from_sync_when_ants_meet(acs):
    """With many ants the in-step order matters: on n=198, m=n the sequential
    and step-snapshot schedules give different tours (and each equals its own
    oracle schedule, checked above)."""
    xy = inputs.uniform(198, 207)
    a = acs.Colony(xy, mode=acs.ACS_SEQUENTIAL, seed=6)
    b = acs.Colony(xy, mode=acs.ACS_SYNC, seed=6)
    a.iterate(2)
    b.iterate(2)
    assert not np.array_equal(a.tours(), b.tours())
    a.close()
    b.close()
