"""Pins of the CPU oracle against things other than itself.

Each test checks one part of the oracle against a value fixed by the paper's
definitions or by mathematics: an independent Philox implementation, exact
rational arithmetic, brute force on tiny instances, closed forms and
special cases (q0 = 1 gives nearest-neighbour tours, s >= n-1 makes the
selective memory a dense matrix, one ant makes every schedule the same).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1605_02669_amd import inputs
from tests import defs


# --------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's host engine (an independent implementation
# of the same published generator).
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_philox_exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND cross-check")
    src = os.path.join(os.path.dirname(__file__), "philox_xcheck", "rocrand_philox.cpp")
    d = tempfile.mkdtemp(prefix="philox_xcheck_")
    exe = os.path.join(d, "rocrand_philox")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, cwd=d,
                   stdout=subprocess.PIPE, stderr=subprocess.PIPE)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_philox_exe):
    rng = np.random.default_rng(1)
    cases = [[0] * 6, [0xFFFFFFFF] * 6]
    cases += rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64).tolist()
    # counters of the shape the method uses: (step, ant, iteration, instance)
    for step, ant, it in [(0, 0, 0), (1, 5, 0), (2391, 2391, 999), (19999, 1023, 499)]:
        cases.append([0x1234, 0, step, ant, it, 0])
    text = "\n".join(" ".join(f"{int(v):x}" for v in c) for c in cases) + "\n"
    res = subprocess.run([rocrand_philox_exe], input=text, capture_output=True,
                         text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == len(cases)
    for c, line in zip(cases, lines):
        want = [int(x, 16) for x in line.split()]
        got = oracle.philox(c[2:], c[:2]).tolist()
        assert got == want, (c, got, want)


# --------------------------------------------------------------------------
# Distances, candidate lists, eta^beta, nearest-neighbour tour, tau0.
# --------------------------------------------------------------------------
def test_exact_distance_definition():
    rng = np.random.default_rng(2)
    pts = rng.random((4000, 4)) * 10000.0
    for xi, yi, xj, yj in pts:
        assert oracle.exact_dist(xi, yi, xj, yj) == defs.exact_dist(xi, yi, xj, yj)
    # half-integer and near-half cases, zero and tiny distances
    specials = [(0, 0, 3, 4), (0, 0, 0.5, 0), (0, 0, 1.5, 0), (0, 0, 2.5, 0),
                (0, 0, 0, 0), (1, 1, 1.2, 1.1), (0, 0, 0.4999999999, 0),
                (0, 0, 0.5000000001, 0), (0, 0, 10000, 10000),
                (0, 0, np.nextafter(2.5, 0), 0), (0, 0, np.nextafter(2.5, 3), 0)]
    for xi, yi, xj, yj in specials:
        assert oracle.exact_dist(xi, yi, xj, yj) == defs.exact_dist(xi, yi, xj, yj)
    # agrees with nint(sqrt) away from exact ties
    for xi, yi, xj, yj in pts[:500]:
        s = (xi - xj) ** 2 + (yi - yj) ** 2
        assert oracle.exact_dist(xi, yi, xj, yj) == int(np.sqrt(s) + 0.5)


@pytest.mark.parametrize("kind,n", [("uniform", 60), ("clustered", 45), ("coincident", 40)])
def test_distance_matrix_and_candidates(kind, n):
    xy = {"uniform": inputs.uniform, "clustered": inputs.clustered,
          "coincident": lambda n: inputs.coincident(n, 7)}[kind](n)
    o = oracle.Oracle(xy, cl=16)
    d = defs.dist_matrix(xy)
    assert np.array_equal(o.dist(), d)
    cand = o.cand()
    for i in range(n):
        js = np.array([j for j in range(n) if j != i])
        order = np.lexsort((js, d[i, js]))  # by (d, j)
        assert np.array_equal(cand[i], js[order][:16])


def test_candidate_list_clamped_to_n_minus_1():
    xy = inputs.uniform(7, 3)
    o = oracle.Oracle(xy, cl=32)
    assert o.cl == 6
    assert o.cand().shape == (7, 6)


@pytest.mark.parametrize("beta", [2.0, 3.0, 2.5])
def test_eta_beta_table(beta):
    o = oracle.Oracle(inputs.uniform(20), beta=beta)
    eta = o.eta(15000)
    assert eta[0] == np.float32(2.0 ** beta)  # zero distance read as d = 1/2
    for d in [1, 2, 3, 7, 100, 1000, 14142]:
        exact = Fraction(1) / Fraction(d) ** 2 if beta == 2.0 else None
        if exact is not None:
            assert eta[d] == defs.round_to_f32(exact)
        else:
            assert abs(float(eta[d]) * d ** beta - 1.0) < 1.2e-7
    assert np.all(np.diff(eta[1:].astype(np.float64)) < 0)  # strictly decreasing


@pytest.mark.parametrize("n,kind", [(50, "uniform"), (37, "clustered"), (198, "uniform")])
def test_nn_tour_length_and_tau0(n, kind):
    xy = inputs.uniform(n) if kind == "uniform" else inputs.clustered(n)
    o = oracle.Oracle(xy)
    d = defs.dist_matrix(xy)
    c = o.constants()
    L = defs.tour_length(d, defs.nn_tour(d, 0))
    assert c["lnn"] == L
    assert c["tau0"] == defs.round_to_f32(Fraction(1, n * L))
    assert c["a_loc"] == np.float32(0.9)
    assert c["q0_24"] == 15099495  # ceil(0.9 * 2^24)


# --------------------------------------------------------------------------
# Eq. 1 with q0 = 1: every ant builds the nearest-neighbour tour from its
# start.  This pins the candidate filter, the argmax with its tie rule, the
# fallback and the uniform initial pheromone at once.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,cl,kind", [(60, 8, "uniform"), (45, 5, "clustered"),
                                        (40, 4, "coincident"), (120, 16, "uniform")])
def test_q0_one_gives_nearest_neighbour_tours(n, cl, kind):
    xy = {"uniform": inputs.uniform, "clustered": inputs.clustered,
          "coincident": lambda n: inputs.coincident(n, 11)}[kind](n)
    o = oracle.Oracle(xy, cl=cl, q0=1.0, seed=5)
    c = o.constants()
    # precondition of the pin: the local map keeps tau0 fixed in float
    assert o.local_map_k(c["tau0"], 1) == c["tau0"]
    o.construct()
    d = defs.dist_matrix(xy)
    tours = o.tours()
    lens = o.lengths()
    for a in range(o.m):
        nn = defs.nn_tour(d, int(tours[a, 0]))
        assert tours[a].tolist() == nn
        assert lens[a] == defs.tour_length(d, nn)
    counts = o.counts()
    assert counts["roulette"] == 0 and counts["fallback"] > 0


# --------------------------------------------------------------------------
# Local update (Eq. 3) against its closed form.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("phi", [0.1, 0.01])
def test_local_map_closed_form(phi):
    o = oracle.Oracle(inputs.uniform(198), phi=phi)
    c = o.constants()
    a = Fraction(float(c["a_loc"]))
    b = Fraction(float(c["b_loc"]))
    t0 = float(c["tau0"])
    fix = b / (1 - a)
    rng = np.random.default_rng(3)
    xs = [np.float32(t0 * s) for s in np.concatenate([[1.0, 1.0001, 2.0], rng.uniform(1, 2000, 40)])]
    for x in xs:
        # trajectory y_1..y_K by single applications; each rounding adds at
        # most half an ulp of y_j, later scaled by a^(k-j)
        traj = [x]
        for _ in range(512):
            traj.append(o.local_map_k(traj[-1], 1))
        for k in (1, 2, 3, 4, 16, 64, 512):
            y = o.local_map_k(x, k)
            assert y == traj[k]
            ulp = float(np.spacing(np.float32(y)))
            exact = fix + a ** k * (Fraction(float(x)) - fix)
            err = abs(Fraction(float(y)) - exact)
            bound = sum(Fraction(float(np.spacing(traj[j]))) / 2 * a ** (k - j)
                        for j in range(1, k + 1))
            assert err <= bound, (x, k, float(err / bound))
            if k <= 2:
                # the map read with exact phi and tau0: within 2 ulp (beyond
                # k = 2 the rounding of 1 - phi to float adds a drift of
                # about 0.2 ulp per application on top of the rounding)
                exact_phi = Fraction(t0) + Fraction(1 - phi) ** k * (Fraction(float(x)) - Fraction(t0))
                assert abs(float(Fraction(float(y)) - exact_phi)) / ulp <= 2.0
        assert o.local_map_k(x, 1) == defs.round_to_f32(a * Fraction(float(x)) + b)


# --------------------------------------------------------------------------
# Eq. 2 by roulette: the selection frequencies over every 24-bit draw equal
# the proportional probabilities up to float rounding of the prefix sums.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("cl,seed", [(32, 0), (16, 1), (7, 2), (32, 3)])
def test_roulette_matches_proportional_rule(cl, seed):
    rng = np.random.default_rng(seed)
    w = (rng.random(cl) ** 3 * 1e-9).astype(np.float32)
    unv = (rng.random(cl) < 0.6).astype(np.uint8)
    unv[rng.integers(cl)] = 1
    w = np.where(unv == 1, w, np.float32(0)).astype(np.float32)
    counts = oracle.roulette_hist(w, unv)
    assert counts.sum() == 2 ** 24
    p = w.astype(np.float64) / w.astype(np.float64).sum()
    freq = counts / 2.0 ** 24
    assert np.all(counts[unv == 0] == 0)
    assert np.max(np.abs(freq - p)) < cl * 2.0 ** -21
    # single candidate, and a spike
    one = np.zeros(cl, np.float32); one[cl // 2] = 1e-10
    assert oracle.roulette_hist(one, (one > 0).astype(np.uint8))[cl // 2] == 2 ** 24


def test_roulette_first_exceeding_prefix():
    w = np.array([1, 0, 2, 0, 1], dtype=np.float32)
    unv = np.array([1, 0, 1, 0, 1], dtype=np.uint8)
    # prefix sums 1,1,3,3,4; r = u*4
    assert oracle.roulette_pick(w, unv, 0) == 0
    assert oracle.roulette_pick(w, unv, (1 << 22) - 1) == 0   # u*4 < 1
    assert oracle.roulette_pick(w, unv, 1 << 22) == 2         # r == 1 -> P > 1 first at k=2
    assert oracle.roulette_pick(w, unv, 3 << 22) == 4         # r == 3
    assert oracle.roulette_pick(w, unv, (1 << 24) - 1) == 4


# --------------------------------------------------------------------------
# Whole iterations.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("memory,mode", [(oracle.DENSE, oracle.SYNC), (oracle.SPM, oracle.SYNC),
                                         (oracle.DENSE, oracle.SEQUENTIAL)])
def test_tours_are_permutations_with_recomputed_lengths(memory, mode):
    xy = inputs.clustered(150, 9)
    o = oracle.Oracle(xy, m=40, cl=16, memory=memory, spm_s=8, mode=mode, seed=3)
    d = defs.dist_matrix(xy)
    for _ in range(4):
        o.iterate(1)
        tours, lens = o.tours(), o.lengths()
        for a in range(o.m):
            assert sorted(tours[a].tolist()) == list(range(150))
            assert lens[a] == defs.tour_length(d, tours[a])
        ib, lib = o.iter_best()
        assert lib == lens.min() and ib == int(np.argmin(lens))
        best, L = o.best()
        assert L == defs.tour_length(d, best) and sorted(best.tolist()) == list(range(150))


def test_greedy_share_follows_q0():
    o = oracle.Oracle(inputs.uniform(300), q0=0.75, seed=1)
    o.iterate(2)
    c = o.counts()
    share = c["greedy"] / (c["greedy"] + c["roulette"])
    # binomial with ~1.2e5 trials: sd ~ 0.0013
    assert abs(share - 0.75) < 0.01
    assert c["steps"] == 2 * 300 * 299


def test_start_cities_cover_range():
    o = oracle.Oracle(inputs.uniform(64), m=4096, cl=8, seed=2)
    o.construct()
    starts = o.tours()[:, 0]
    counts = np.bincount(starts, minlength=64)
    assert counts.min() > 30 and counts.max() < 100  # 64 expected per city


@pytest.mark.parametrize("n", [5, 6, 7, 8, 9, 10])
def test_small_instances_reach_bruteforce_optimum(n):
    for s in range(20):
        xy = inputs.uniform(n, 1000 + 17 * n + s)
        d = defs.dist_matrix(xy)
        opt = defs.brute_force_optimum(d)
        o = oracle.Oracle(xy, seed=s)
        o.iterate(300)
        _, L = o.best()
        assert L == opt, (n, s, L, opt)


def test_split_iterations_equal_joined():
    xy = inputs.uniform(80, 4)
    a = oracle.Oracle(xy, seed=9)
    b = oracle.Oracle(xy, seed=9)
    a.iterate(3)
    b.iterate(1); b.iterate(1); b.iterate(1)
    assert np.array_equal(a.tau(), b.tau())
    assert np.array_equal(a.tours(), b.tours())


def test_one_ant_makes_schedules_coincide():
    xy = inputs.uniform(90, 5)
    for memory in (oracle.DENSE, oracle.SPM):
        s = oracle.Oracle(xy, m=1, mode=oracle.SYNC, memory=memory, seed=4)
        q = oracle.Oracle(xy, m=1, mode=oracle.SEQUENTIAL, memory=memory, seed=4)
        for _ in range(5):
            s.iterate(1); q.iterate(1)
            assert np.array_equal(s.tours(), q.tours())
            assert np.array_equal(s.tau(), q.tau())


def test_sync_and_sequential_differ_with_many_ants():
    xy = inputs.uniform(90, 5)
    s = oracle.Oracle(xy, mode=oracle.SYNC, seed=4)
    q = oracle.Oracle(xy, mode=oracle.SEQUENTIAL, seed=4)
    s.iterate(3); q.iterate(3)
    assert not np.array_equal(s.tau(), q.tau())


# --------------------------------------------------------------------------
# Local-update period k (Sec. 4, limiting the number of local updates): the
# map follows only the edges an ant selects at steps k, 2k, ... plus the
# closing edge.  Pinned by recounting, from the tours alone, how often each
# entry must have been mapped: f composes, so every entry must end at
# f^c(before) with c its count, whatever the order of the updates.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 2, 5, 16])
@pytest.mark.parametrize("mode", [oracle.SYNC, oracle.SEQUENTIAL])
def test_local_update_period_counts_crossings(k, mode):
    n, m = 60, 24
    xy = inputs.uniform(n, 12)
    o = oracle.Oracle(xy, m=m, cl=8, mode=mode, seed=3, local_update_period=k)
    o.iterate(6)  # moves the entries of the best tours off the fixed point tau0
    before = o.tau()
    o.construct()
    tours = o.tours()
    cnt = np.zeros((n, n), dtype=np.int64)
    for a in range(m):
        edges = [(tours[a, t - 1], tours[a, t]) for t in range(1, n) if t % k == 0]
        edges.append((tours[a, n - 1], tours[a, 0]))
        for u, v in edges:
            cnt[u, v] += 1
            cnt[v, u] += 1
    expect = before.copy()
    for i, j in zip(*np.nonzero(cnt)):
        expect[i, j] = o.local_map_k(float(before[i, j]), int(cnt[i, j]))
    assert np.array_equal(o.tau(), expect)
    tau0 = np.float32(o.constants()["tau0"])
    assert np.count_nonzero((cnt > 0) & (before != tau0)) >= 10  # the check has teeth


def test_local_update_period_changes_the_run():
    xy = inputs.uniform(120, 13)
    a = oracle.Oracle(xy, seed=2)
    b = oracle.Oracle(xy, seed=2, local_update_period=4)
    a.iterate(3); b.iterate(3)
    assert not np.array_equal(a.tours(), b.tours())
    with pytest.raises(ValueError):
        oracle.Oracle(xy, local_update_period=0)


@pytest.mark.parametrize("k", [3, 8])
def test_spm_without_eviction_equals_dense_with_period(k):
    n = 50
    xy = inputs.clustered(n, 14)
    den = oracle.Oracle(xy, m=20, cl=10, seed=5, local_update_period=k)
    spm = oracle.Oracle(xy, m=20, cl=10, seed=5, local_update_period=k,
                        memory=oracle.SPM, spm_s=n - 1)
    for _ in range(4):
        den.iterate(1); spm.iterate(1)
        assert np.array_equal(den.tours(), spm.tours())
    assert np.array_equal(den.tau(), spm.tau())


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_spm_without_eviction_equals_dense(kind):
    n = 70
    xy = inputs.uniform(n, 8) if kind == "uniform" else inputs.clustered(n, 8)
    den = oracle.Oracle(xy, m=30, cl=12, seed=6)
    spm = oracle.Oracle(xy, m=30, cl=12, memory=oracle.SPM, spm_s=n - 1, seed=6)
    for _ in range(6):
        den.iterate(1); spm.iterate(1)
        assert np.array_equal(den.tours(), spm.tours())
        assert np.array_equal(den.lengths(), spm.lengths())
        assert np.array_equal(den.tau(), spm.tau())


def test_spm_record_invariants():
    n, m, s = 120, 50, 4
    o = oracle.Oracle(inputs.uniform(n, 12), m=m, cl=10, memory=oracle.SPM, spm_s=s, seed=1)
    c = o.constants()
    for it in range(5):
        o.iterate(1)
        nodes, vals, tail = o.spm()
        for i in range(n):
            used = nodes[i][nodes[i] >= 0]
            assert len(set(used.tolist())) == len(used)  # no duplicates
            assert i not in used.tolist()
            assert 0 <= tail[i] < s
            # unused slots are the oldest: at most s entries, filled in order
            assert np.all(vals[i][nodes[i] >= 0] > 0)
        cnt = o.counts()
        # every crossing updates two records: m*n crossings per iteration,
        # plus 2n global updates
        assert cnt["spm_hits"] + cnt["spm_misses"] == (it + 1) * (2 * m * n + 2 * n)
        tau = o.tau()
        off = tau[nodes < 0] if False else None
        # entries not in a record read tau0
        mask = np.ones((n, n), bool)
        for i in range(n):
            mask[i, nodes[i][nodes[i] >= 0]] = False
        assert np.all(tau[mask] == c["tau0"])


def test_global_update_touches_exactly_best_tour():
    n = 60
    o = oracle.Oracle(inputs.uniform(n, 21), m=20, cl=10, seed=2)
    o.construct()
    o.select_best()
    before = o.tau()
    o.global_update()
    after = o.tau()
    best, L = o.best()
    c = o.constants()
    a = Fraction(float(c["a_glob"]))
    b = defs.round_to_f32(Fraction(1, 10) / L)  # rho / L_gb rounded to float
    edges = set()
    for p in range(n):
        u, v = int(best[p]), int(best[(p + 1) % n])
        edges.add((u, v)); edges.add((v, u))
    assert len(edges) == 2 * n
    changed = set(zip(*np.nonzero(after != before)))
    assert changed <= edges
    for (u, v) in edges:
        want = defs.round_to_f32(a * Fraction(float(before[u, v])) + Fraction(float(b)))
        assert after[u, v] == want


def test_invalid_arguments_rejected():
    xy = inputs.uniform(10)
    with pytest.raises(ValueError):
        oracle.Oracle(xy[:2])
    with pytest.raises(ValueError):
        oracle.Oracle(xy, q0=1.5)
    with pytest.raises(ValueError):
        oracle.Oracle(xy, phi=0.0)
    bad = xy.copy(); bad[3, 0] = np.nan
    with pytest.raises(ValueError):
        oracle.Oracle(bad)


def test_vectorised_edge_distances_match_exact_definition():
    """The vectorised helper the GPU tests use for large tours agrees with
    the rational-arithmetic definition, including near-half cases."""
    g = np.random.default_rng(17)
    xy = np.concatenate([inputs.uniform(400, 3), inputs.clustered(300, 3),
                         np.array([[0.0, 0.0], [0.5, 0.0], [1.5, 0.0], [3.0, 4.0], [0.0, 2.5]])])
    u = g.integers(0, len(xy), size=4000)
    v = g.integers(0, len(xy), size=4000)
    u = np.concatenate([u, [700, 700, 700, 700]])
    v = np.concatenate([v, [701, 702, 703, 704]])
    got = defs.edge_dists(xy, u, v)
    want = [defs.exact_dist(*xy[a], *xy[b]) for a, b in zip(u, v)]
    assert np.array_equal(got, want)


def test_fmaf32_helper_rounds_once():
    """The tests' exact fma (used to predict Eq. 4 on the GPU) against C's
    fmaf inside the oracle's local map, and against a case where rounding
    the product first gives another float."""
    o = oracle.Oracle(inputs.uniform(50, 3), m=1)
    c = o.constants()
    g = np.random.default_rng(8)
    for x in g.uniform(float(c["tau0"]) * 0.5, float(c["tau0"]) * 50, size=200).astype(np.float32):
        assert defs.fmaf32(c["a_loc"], x, c["b_loc"]) == o.local_map_k(x, 1)
    a, x, b = np.float32(1 + 2 ** -12), np.float32(1 + 2 ** -12), np.float32(-1)
    # exact: 2^-11 + 2^-24; a product rounded to float first loses the 2^-24
    assert defs.fmaf32(a, x, b) == np.float32(2 ** -11 + 2 ** -24)
    assert np.float32(a * x) + b == np.float32(2 ** -11)


# --------------------------------------------------------------------------
# Alg. 3 (Sec. 3.2) worked by hand on one record with s = 3.  A miss writes
# slot (tail + 1) mod s, the slot of the trail inserted longest ago, whatever
# its value or how recently it was hit; a hit maps the stored value in place
# and leaves tail alone; a miss stores the map applied to tau0.  The map here
# (a = 1/2, b = tau0) moves tau0 so that every application shows.
# --------------------------------------------------------------------------
def test_spm_alg3_eviction_worked_by_hand():
    o = oracle.Oracle(inputs.uniform(8, 31), m=2, cl=4, memory=oracle.SPM, spm_s=3, seed=1)
    t0 = np.float32(o.constants()["tau0"])
    a, b = np.float32(0.5), t0
    f = lambda x: defs.fmaf32(a, x, b)  # noqa: E731
    ag = np.float32(o.constants()["a_glob"])
    bg = np.float32(0.25)
    g = lambda x: defs.fmaf32(ag, x, bg)  # noqa: E731

    def rec():
        nodes, vals, tail = o.spm()
        return nodes[0].tolist(), vals[0].copy(), int(tail[0])

    nodes, vals, tail = rec()
    assert nodes == [-1, -1, -1] and tail == 2  # empty record, first insert -> slot 0
    o.spm_update(0, 1, a, b)                     # miss: slot 0
    nodes, vals, tail = rec()
    assert nodes == [1, -1, -1] and tail == 0 and vals[0] == f(t0)
    o.spm_update(0, 2, a, b)                     # miss: slot 1
    o.spm_update(0, 1, a, b)                     # hit: slot 0 mapped again, tail stays
    nodes, vals, tail = rec()
    assert nodes == [1, 2, -1] and tail == 1
    assert vals[0] == f(f(t0)) and vals[1] == f(t0)
    o.spm_update(0, 3, a, b)                     # miss: slot 2
    o.spm_update(0, 4, a, b)                     # miss: evicts slot 0 (v = 1, hit last)
    nodes, vals, tail = rec()
    assert nodes == [4, 2, 3] and tail == 0
    assert vals[0] == f(t0) and vals[1] == f(t0) and vals[2] == f(t0)
    o.spm_update(0, 2, a, b)                     # hit on slot 1
    o.spm_update(0, 5, ag, bg)                   # a global-update miss: g(tau0) in slot 1
    nodes, vals, tail = rec()
    assert nodes == [4, 5, 3] and tail == 1
    assert vals[1] == g(t0) and vals[0] == f(t0) and vals[2] == f(t0)
    # the ants read the record as Eq. 1 needs it: a stored trail, else tau0
    tau = o.tau()
    assert tau[0, 4] == f(t0) and tau[0, 5] == g(t0) and tau[0, 3] == f(t0)
    assert tau[0, 1] == t0 and tau[0, 2] == t0 and tau[0, 6] == t0
    # the other records are untouched
    nodes_all, _, tail_all = o.spm()
    assert np.all(nodes_all[1:] == -1) and np.all(tail_all[1:] == 2)
    cnt = o.counts()
    assert cnt["spm_hits"] == 2 and cnt["spm_misses"] == 5


# --------------------------------------------------------------------------
# Alg. 1 read literally (ORC_SEQUENTIAL), worked by hand on 5 cities: two
# ants start at city 0, whose neighbours 1 and 2 are both at distance 100
# (equal eta^beta), with tau(0, 1) = 10.5 tau0 and tau(0, 2) = 10 tau0; q0 = 1
# makes every choice the argmax of Eq. 1.  Ant 0 takes city 1 and its local
# update (Eq. 3) lowers tau(0, 1) to 0.9 * 10.5 tau0 + 0.1 tau0 = 9.55 tau0
# < 10 tau0 before ant 1 chooses, so ant 1 takes city 2.  In the synchronous
# schedule both read the step-start value and take city 1; with the ants in
# the opposite order ant 1 would take city 1 and ant 0 city 2.
# --------------------------------------------------------------------------
def _seed_with_shared_start(n, m):
    for seed in range(5000):
        key = [seed & 0xFFFFFFFF, seed >> 32]
        st = [int((int(oracle.philox([0, a, 0, 0], key)[2]) * n) >> 32) for a in range(m)]
        if st[0] == 0 and st[1] == 0 and all(s != 0 for s in st[2:]):
            return seed
    raise AssertionError("no seed found")


def test_sequential_step_reads_earlier_ants_updates_by_hand():
    xy = np.array([[5000, 5000], [5100, 5000], [5000, 5100], [4700, 5000], [5000, 4700]],
                  dtype=np.float64)
    n, m = 5, 3
    seed = _seed_with_shared_start(n, m)
    picks = {}
    for mode in (oracle.SEQUENTIAL, oracle.SYNC):
        o = oracle.Oracle(xy, m=m, cl=n - 1, q0=1.0, phi=0.1, mode=mode, seed=seed)
        t0 = np.float32(o.constants()["tau0"])
        tau = np.full((n, n), t0, dtype=np.float32)
        tau[0, 1] = tau[1, 0] = np.float32(10.5) * t0
        tau[0, 2] = tau[2, 0] = np.float32(10.0) * t0
        o.set_tau(tau)
        o.construct()
        tours = o.tours()
        assert tours[0, 0] == 0 and tours[1, 0] == 0 and tours[2, 0] != 0
        picks[mode] = (int(tours[0, 1]), int(tours[1, 1]))
        # the map of Eq. 3 at this value really lands below 10 tau0
        assert o.local_map_k(float(tau[0, 1]), 1) < tau[0, 2]
    assert picks[oracle.SEQUENTIAL] == (1, 2)
    assert picks[oracle.SYNC] == (1, 1)


# --------------------------------------------------------------------------
# Learned candidate scores in Eq. 1 and Eq. 2.  (1) Scores equal to eta^beta
# reproduce the plain run bit for bit.  (2) With q0 = 1 and uniform
# pheromone, the first iteration's tours are greedy walks by the largest
# score among the unvisited candidates (ties: nearest position), and, when
# every candidate is visited, by the nearest unvisited city (ties: lowest
# index): the fallback keeps eta^beta, which decreases with d.
# --------------------------------------------------------------------------
def test_scores_equal_to_eta_reproduce_plain_run():
    xy = inputs.uniform(80, 33)
    plain = oracle.Oracle(xy, m=40, cl=12, seed=3)
    sc = oracle.Oracle(xy, m=40, cl=12, seed=3)
    d = plain.dist()
    cand = plain.cand()
    eta = plain.eta(int(d.max()) + 1)
    sc.set_candidate_weights(eta[d[np.arange(80)[:, None], cand]])
    for _ in range(4):
        plain.iterate(1); sc.iterate(1)
        assert np.array_equal(plain.tours(), sc.tours())
        assert np.array_equal(plain.tau(), sc.tau())
    assert plain.counts() == sc.counts()


@pytest.mark.parametrize("n,cl,seed", [(60, 6, 1), (45, 4, 2)])
def test_scores_drive_the_greedy_choice_and_fallback_keeps_eta(n, cl, seed):
    xy = inputs.uniform(n, 40 + seed)
    d = defs.dist_matrix(xy)
    # candidate lists from a plain sort by (d, j)
    cand = np.array([sorted((j for j in range(n) if j != i), key=lambda j: (d[i, j], j))[:cl]
                     for i in range(n)])
    rng = np.random.default_rng(seed)
    scores = rng.uniform(0.1, 1.0, size=(n, cl)).astype(np.float32)
    o = oracle.Oracle(xy, m=n, cl=cl, q0=1.0, seed=seed)
    c = o.constants()
    assert o.local_map_k(c["tau0"], 1) == c["tau0"]  # pheromone stays uniform
    o.set_candidate_weights(scores)
    o.construct()
    tours = o.tours()
    fallbacks = 0
    for a in range(n):
        cur = int(tours[a, 0])
        seen = {cur}
        walk = [cur]
        for _ in range(n - 1):
            opts = [k for k in range(cl) if int(cand[cur, k]) not in seen]
            if opts:
                k = max(opts, key=lambda k: (scores[cur, k], -k))
                nxt = int(cand[cur, k])
            else:
                fallbacks += 1
                nxt = min((j for j in range(n) if j not in seen), key=lambda j: (d[cur, j], j))
            walk.append(nxt)
            seen.add(nxt)
            cur = nxt
        assert tours[a].tolist() == walk
    assert fallbacks > 0  # the fallback rule was exercised
    with pytest.raises(ValueError):
        o.set_candidate_weights(np.zeros((n, cl), np.float32))


# --------------------------------------------------------------------------
# Exchange of best-so-far solutions between colonies (the multi-colony model
# of Sec. 2): after an exchange from the shortest, every colony holds a valid
# tour of the shortest length; a ring passes the shortest to every colony
# within count - 1 exchanges and never lengthens a colony's best.
# --------------------------------------------------------------------------
def test_exchange_best_between_colonies():
    xy = inputs.uniform(40, 50)
    d = defs.dist_matrix(xy)
    C = 5
    for topology in (0, 1):
        cols = [oracle.Oracle(xy, m=4, cl=8, seed=7, instance=c) for c in range(C)]
        for o in cols:
            o.iterate(2)
        lens0 = [o.best()[1] for o in cols]
        gmin = min(lens0)
        assert len(set(lens0)) > 1  # the colonies differ before the exchange
        rounds = 1 if topology == 0 else C - 1
        prev = lens0
        for r in range(rounds):
            oracle.exchange_best(cols, topology)
            now = [o.best()[1] for o in cols]
            assert all(x <= y for x, y in zip(now, prev))
            if topology == 1 and r == 0:
                # one ring step: colony c holds min(own, colony c - 1's)
                assert now == [min(prev[c], prev[c - 1]) for c in range(C)]
            prev = now
        for o in cols:
            t, L = o.best()
            assert sorted(t.tolist()) == list(range(40))
            assert L == defs.tour_length(d, t) == gmin
        if topology == 0:
            g = lens0.index(gmin)
            ref = cols[g].best()[0]
            assert all(np.array_equal(o.best()[0], ref) for o in cols)
