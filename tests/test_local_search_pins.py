"""Pins of the oracle's local search (2-opt and Or-opt descent over the
candidate lists, first improvement, a queue of cities to examine; the
paper's Sec. 5.1 names a local search such as 3-opt as further research).

Each check rests on something other than the oracle's own code:
* two tiny tours worked by hand from the move order and the array rules
  (the expected arrays and lengths are derived in the comments);
* the definition of a tour: a permutation whose length, recomputed from the
  array with exact distances, equals the length the descent reports, never
  longer than the start, shorter by at least one per move (integer costs);
* with complete candidate lists the descent ends 2-opt optimal: no pair of
  edges, checked exhaustively, can be exchanged for a shorter pair;
* ACS with the local search on: every ant's tour is the descent of the tour
  the construction built (the iteration best and the global update then
  use the improved tours);
* the 3-opt move (kind 2): from tours where 2-opt and Or-opt find nothing,
  the first move equals the first improving reconnection of an enumeration
  that builds every candidate tour by slicing and measures it from the
  distance matrix, for each of the four reconnections.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1605_02669_amd import inputs
from tests import defs


def _orc(xy, **kw):
    return oracle.Oracle(np.asarray(xy, dtype=np.float64), m=1, seed=0, **kw)


def test_square_crossing_is_uncrossed_by_one_2opt_move():
    # square 0 (0,0), 1 (10,0), 2 (10,10), 3 (0,10); start tour 0 2 1 3
    # (edges 14 + 10 + 14 + 10 = 48).  City 0 is popped first: its successor
    # b = 2 (d = 14); its first candidate c = 1 (d = 10 < 14), e = succ(1) = 3,
    # delta = d(0,1) + d(2,3) - d(0,2) - d(1,3) = 10 + 10 - 14 - 14 = -8.
    # The forward path 2 .. 1 holds 2 of 4 cities (not more than half), so it
    # is reversed in place: 0 1 2 3, length 40; no further move shortens it.
    o = _orc([(0, 0), (10, 0), (10, 10), (0, 10)], cl=3)
    t, L, mv = o.local_search_tour([0, 2, 1, 3], 48)
    assert t.tolist() == [0, 1, 2, 3] and L == 40 and mv == 1
    o.close()


def test_hexagon_first_move_is_an_or_opt_of_two_cities():
    # 0 (0,0), 1 (10,0), 2 (20,0), 3 (20,10), 4 (10,10), 5 (0,10); start tour
    # 0 1 4 3 2 5: 10 + 10 + 10 + 10 + 22 + 10 = 72 (d(2,5) = nint(22.36)).
    # City 0 first: candidates by (d, j) are 1 (10), 5 (10), 4 (14), 2 (20),
    # 3 (22).  2-opt on the successor stops at once (d(0,1) = d(0,b = 1)), so
    # does 2-opt on the predecessor (d(0,1) = d(5,0)).  Or-opt L = 1 (S = 0,
    # p = 5, x = 1, gain 10 + 10 - 14 = 6) has no shortening placement: the
    # deltas are 8 (c = 1), 2 (c = 5), 20 and 8 (c = 4), 2 and 26 (c = 2),
    # 26 and 20 (c = 3).  Or-opt L = 2 (S = 0 1, p = 5, x = 4, gain
    # 10 + 10 - 10 = 10): c = 1 lies in S, c = 5 = p rules out side A, side B
    # puts S reversed between f = pred(5) = 2 and 5: d(2,1) + d(0,5) - d(2,5)
    # - 10 = 10 + 10 - 22 - 10 = -12.  Block C = 5 (one city) is shorter than
    # block B = 4 3 2, so 5 moves two places on and "1 0" fills the gap:
    # array 0 5 4 3 2 1, the rectangle's perimeter 60.
    o = _orc([(0, 0), (10, 0), (20, 0), (20, 10), (10, 10), (0, 10)], cl=5)
    t, L, mv = o.local_search_tour([0, 1, 4, 3, 2, 5], 72)
    assert t.tolist() == [0, 5, 4, 3, 2, 1] and L == 60 and mv == 1
    o.close()


@pytest.mark.parametrize("n,cl", [(40, 8), (120, 16), (300, 32), (64, 63)])
def test_descent_gives_a_valid_shorter_tour(n, cl):
    xy = inputs.uniform(n, 70 + n)
    d = defs.dist_matrix(xy) if n <= 120 else None
    o = oracle.Oracle(xy, m=6, cl=cl, seed=3)
    o.construct()
    rng = np.random.default_rng(n)
    starts = list(o.tours()) + [rng.permutation(n).astype(np.int32) for _ in range(4)]
    for t0 in starts:
        L0 = int(defs.tour_lengths(xy, np.asarray(t0)[None, :])[0])
        t, L, mv = o.local_search_tour(t0, L0)
        assert sorted(t.tolist()) == list(range(n))
        assert L == int(defs.tour_lengths(xy, t[None, :])[0])
        assert L <= L0 and L0 - L >= mv
    o.close()


def test_complete_lists_end_two_opt_optimal():
    rng = np.random.default_rng(5)
    for trial in range(150):
        n = int(rng.integers(6, 16))
        xy = inputs.uniform(n, 2000 + trial)
        d = defs.dist_matrix(xy)
        o = oracle.Oracle(xy, m=1, cl=n - 1, seed=trial)
        t0 = rng.permutation(n).astype(np.int32)
        t, L, _ = o.local_search_tour(t0, defs.tour_length(d, t0))
        T = t.tolist()
        for i in range(n):
            for j in range(i + 2, n):
                if i == 0 and j == n - 1:
                    continue
                a, b, c, e = T[i], T[(i + 1) % n], T[j], T[(j + 1) % n]
                assert d[a, c] + d[b, e] >= d[a, b] + d[c, e], (trial, i, j)
        o.close()


def test_acs_with_local_search_improves_every_ant():
    xy = inputs.uniform(150, 9)
    plain = oracle.Oracle(xy, m=12, cl=16, seed=4)
    ls = oracle.Oracle(xy, m=12, cl=16, seed=4, local_search=1)
    plain.construct()
    ls.construct()
    # the construction itself is the same; the descent then runs per ant
    assert np.array_equal(plain.tours(), ls.tours())
    built, blen = plain.tours(), plain.lengths()
    ls.local_search()
    for a in range(12):
        t, L, _ = plain.local_search_tour(built[a], blen[a])
        assert np.array_equal(ls.tours()[a], t) and ls.lengths()[a] == L
    assert ls.ls_moves() > 0
    plain.close()
    ls.close()


# --- the 3-opt move (kind 2) -----------------------------------------------
#
# Reconnections of a [B = b..c] [C = d..e] f (b = succ(a)), in the order the
# descent tries them, with the city whose candidates give the second new edge:
#   (i) C B (y = e from b), (ii) C B' (y = e from c), (iii) C' B (x = e,
#   y = d from b), (iv) B' C' (x = c, y = e from b).
# The enumeration below builds each candidate tour by list slicing and takes
# its length from the distance matrix, so neither the gain formulas nor the
# in-place reversals of the oracle enter it.


def _cands(d, cl):
    n = d.shape[0]
    return [sorted((j for j in range(n) if j != i), key=lambda j: (d[i, j], j))[:cl]
            for i in range(n)]


def _first_three_opt(d, cand, T):
    """First improving 3-opt move over the cities in array order: (expected
    array, its length, reconnection index 0..3), or None."""
    n = len(T)
    L0 = defs.tour_length(d, T)
    for i in range(n):
        a, b = T[i], T[(i + 1) % n]
        off = {T[(i + k) % n]: k for k in range(n)}
        at = lambda k: T[(i + k) % n]  # noqa: E731
        for typ in range(4):
            for x in cand[a]:
                if not d[a, x] < d[a, b]:
                    continue
                ox = off[x]
                if typ in (0, 1):
                    if ox < 2:
                        continue
                    frm, g = (b if typ == 0 else at(ox - 1)), d[a, b] - d[a, x] + d[at(ox - 1), x]
                elif typ == 2:
                    if ox < 3:
                        continue
                    frm, g = b, d[a, b] - d[a, x] + d[x, at(ox + 1)]
                else:
                    if ox < 2 or ox > n - 3:
                        continue
                    frm, g = b, d[a, b] - d[a, x] + d[x, at(ox + 1)]
                for y in cand[frm]:
                    if not d[frm, y] < g:
                        continue
                    oy = off[y]
                    if typ == 0:
                        od, oe, ok = ox, oy, oy >= ox
                    elif typ == 1:
                        od, oe, ok = ox, oy, oy > ox
                    elif typ == 2:
                        od, oe, ok = oy, ox, 2 <= oy < ox
                    else:
                        od, oe, ok = ox + 1, oy, oy > ox + 1
                    if not ok:
                        continue
                    B = [at(k) for k in range(1, od)]
                    C = [at(k) for k in range(od, oe + 1)]
                    block = [C + B, C + B[::-1], C[::-1] + B, B[::-1] + C[::-1]][typ]
                    E = list(T)
                    for k, city in enumerate(block):
                        E[(i + 1 + k) % n] = city
                    L = defs.tour_length(d, E)
                    if L < L0:
                        return E, L, typ
    return None


def test_three_opt_first_move_matches_enumeration():
    rng = np.random.default_rng(11)
    seen = [0, 0, 0, 0]
    for trial in range(300):
        n = int(rng.integers(16, 41))
        make = inputs.uniform if trial % 2 else inputs.clustered
        xy = make(n, 3000 + trial)
        d = defs.dist_matrix(xy)
        cl = min(int(rng.choice([6, 10, n - 1])), n - 1)
        cand = _cands(d, cl)
        o1 = oracle.Oracle(xy, m=1, cl=cl, seed=trial, local_search=1)
        T = rng.permutation(n).astype(np.int32)
        L = defs.tour_length(d, T)
        for _ in range(20):  # 2-opt and Or-opt until a fresh descent moves nothing
            T, L, mv = o1.local_search_tour(T, L)
            if mv == 0:
                break
        o1.close()
        if mv:
            continue
        o2 = oracle.Oracle(xy, m=1, cl=cl, seed=trial, local_search=2)
        o2.set_local_search_cap(1)
        t, L2, mv2, kinds = o2.local_search_tour(T, L, kinds=True)
        o2.close()
        want = _first_three_opt(d, cand, T.tolist())
        if want is None:
            assert mv2 == 0 and t.tolist() == T.tolist(), trial
            continue
        E, LE, typ = want
        assert mv2 == 1 and kinds[2 + typ] == 1, (trial, kinds, typ)
        assert t.tolist() == E and L2 == LE, trial
        seen[typ] += 1
    assert min(seen) > 0, seen


@pytest.mark.parametrize("n,cl,kind", [(40, 8, "uniform"), (120, 16, "uniform"),
                                       (300, 32, "clustered"), (64, 63, "uniform"),
                                       (6, 5, "uniform")])
def test_three_opt_descent_gives_a_valid_shorter_tour(n, cl, kind):
    xy = getattr(inputs, kind)(n, 170 + n)
    o = oracle.Oracle(xy, m=6, cl=cl, seed=3, local_search=2)
    o.construct()
    rng = np.random.default_rng(n)
    starts = list(o.tours()) + [rng.permutation(n).astype(np.int32) for _ in range(4)]
    for t0 in starts:
        L0 = int(defs.tour_lengths(xy, np.asarray(t0)[None, :])[0])
        t, L, mv, kinds = o.local_search_tour(t0, L0, kinds=True)
        assert sorted(t.tolist()) == list(range(n))
        assert L == int(defs.tour_lengths(xy, t[None, :])[0])
        assert L <= L0 and L0 - L >= mv and sum(kinds) == mv
    o.close()


def test_acs_with_three_opt_is_the_descent_of_every_ant():
    xy = inputs.clustered(160, 12)
    plain = oracle.Oracle(xy, m=10, cl=16, seed=6)
    ls = oracle.Oracle(xy, m=10, cl=16, seed=6, local_search=2)
    plain.construct()
    ls.construct()
    built, blen = plain.tours(), plain.lengths()
    ls.local_search()
    three = 0
    for a in range(10):
        t, L, _, kinds = ls.local_search_tour(built[a], blen[a], kinds=True)
        assert np.array_equal(ls.tours()[a], t) and ls.lengths()[a] == L
        three += sum(kinds[2:])
    assert three > 0
    plain.close()
    ls.close()
