"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It never touches the HIP library and the HIP library
never touches it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

DENSE, SPM = 0, 1
SYNC, SEQUENTIAL = 0, 1

_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, u32, i64, u64, dbl, f32 = C.c_int32, C.c_uint32, C.c_int64, C.c_uint64, C.c_double, C.c_float
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [P, i32, i32, i32, dbl, dbl, dbl, dbl, dbl, i32, i32, i32, u64, u32]
    lib.orc_destroy.argtypes = [P]
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_set_local_period.argtypes = [P, i32]
    lib.orc_set_local_period.restype = C.c_int
    for name in ("orc_iterate",):
        getattr(lib, name).argtypes = [P, i32]
    for name in ("orc_construct", "orc_select_best", "orc_global_update"):
        getattr(lib, name).argtypes = [P]
    for name in ("orc_n", "orc_m", "orc_cl"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = i32
    lib.orc_iteration.argtypes = [P]
    lib.orc_iteration.restype = u32
    lib.orc_constants.argtypes = [P, P, P, P, P, P, P]
    for name in ("orc_get_dist", "orc_get_cand", "orc_get_tau", "orc_get_tours",
                 "orc_get_lengths", "orc_get_counts"):
        getattr(lib, name).argtypes = [P, P]
    lib.orc_get_eta.argtypes = [P, P, i32]
    lib.orc_get_spm.argtypes = [P, P, P, P]
    lib.orc_get_best.argtypes = [P, P]
    lib.orc_get_best.restype = i64
    lib.orc_get_iter_best.argtypes = [P, P]
    lib.orc_get_iter_best.restype = i64
    lib.orc_philox.argtypes = [P, P, P]
    lib.orc_exact_dist.argtypes = [dbl, dbl, dbl, dbl]
    lib.orc_exact_dist.restype = i32
    lib.orc_roulette_pick.argtypes = [P, P, i32, u32]
    lib.orc_roulette_pick.restype = i32
    lib.orc_roulette_hist.argtypes = [P, P, i32, P]
    lib.orc_local_map_k.argtypes = [P, f32, i32]
    lib.orc_local_map_k.restype = f32
    lib.orc_set_candidate_weights.argtypes = [P, P]
    lib.orc_set_candidate_weights.restype = C.c_int
    lib.orc_set_best.argtypes = [P, P, i64]
    lib.orc_set_best.restype = C.c_int
    lib.orc_exchange_best.argtypes = [P, i32, i32]
    lib.orc_exchange_best.restype = C.c_int
    lib.orc_set_tau.argtypes = [P, P]
    lib.orc_set_tau.restype = C.c_int
    lib.orc_spm_update.argtypes = [P, i32, i32, f32, f32]
    lib.orc_spm_update.restype = C.c_int
    lib.orc_set_local_search.argtypes = [P, i32]
    lib.orc_set_local_search.restype = C.c_int
    lib.orc_local_search_tour.argtypes = [P, P, i64, P, P]
    lib.orc_local_search_tour.restype = i64
    lib.orc_set_local_search_cap.argtypes = [P, i64]
    lib.orc_set_local_search_cap.restype = C.c_int
    lib.orc_local_search.argtypes = [P]
    lib.orc_ls_moves.argtypes = [P]
    lib.orc_ls_moves.restype = i64
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key) -> np.ndarray:
    lib = load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def exact_dist(xi, yi, xj, yj) -> int:
    return int(load().orc_exact_dist(xi, yi, xj, yj))


def roulette_pick(w, unvisited, u24: int) -> int:
    w = np.ascontiguousarray(w, dtype=np.float32)
    unv = np.ascontiguousarray(unvisited, dtype=np.uint8)
    return int(load().orc_roulette_pick(_ptr(w), _ptr(unv), len(w), u24))


def roulette_hist(w, unvisited) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float32)
    unv = np.ascontiguousarray(unvisited, dtype=np.uint8)
    out = np.zeros(len(w), dtype=np.int64)
    load().orc_roulette_hist(_ptr(w), _ptr(unv), len(w), _ptr(out))
    return out


def set_threads(t: int) -> None:
    load().orc_set_threads(int(t))


def exchange_best(colonies, topology: int = 0) -> None:
    """Best-so-far exchange between oracle colonies of one instance
    (topology 0: from the colony with the shortest; 1: ring from c - 1)."""
    arr = (C.c_void_p * len(colonies))(*[c.h for c in colonies])
    if load().orc_exchange_best(arr, len(colonies), int(topology)) != 0:
        raise ValueError("oracle: invalid exchange")


class Oracle:
    """One ACS colony on one instance, computed on the CPU."""

    def __init__(self, xy, m=None, cl=32, beta=2.0, q0=0.9, phi=0.1, rho=0.1,
                 tau0=0.0, memory=DENSE, spm_s=8, mode=SYNC, seed=0, instance=0,
                 local_update_period=1, local_search=0):
        self.lib = load()
        self.xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        n = self.xy.shape[0]
        if m is None or m == 0:
            m = n
        self.h = self.lib.orc_create(_ptr(self.xy), n, m, cl, beta, q0, phi, rho,
                                     tau0, memory, spm_s, mode, seed, instance)
        if not self.h:
            raise ValueError("oracle: invalid arguments")
        if self.lib.orc_set_local_period(self.h, int(local_update_period)) != 0:
            self.close()
            raise ValueError("oracle: local_update_period must be >= 1")
        if self.lib.orc_set_local_search(self.h, int(local_search)) != 0:
            self.close()
            raise ValueError("oracle: local_search must be 0, 1 or 2")
        self.n, self.m = n, m
        self.cl = self.lib.orc_cl(self.h)
        self.memory, self.spm_s = memory, spm_s

    def close(self):
        if self.h:
            self.lib.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # iteration control
    def iterate(self, k=1):
        self.lib.orc_iterate(self.h, k)

    def construct(self):
        self.lib.orc_construct(self.h)

    def select_best(self):
        self.lib.orc_select_best(self.h)

    def local_search(self):
        """The local search on every ant's tour (when it is set)."""
        self.lib.orc_local_search(self.h)

    def local_search_tour(self, tour, length: int, kinds: bool = False):
        """The descent on one tour: (improved tour, its length, moves), and
        with ``kinds`` the moves by kind (2-opt, Or-opt, 3-opt (i) .. (iv))."""
        t = np.array(tour, dtype=np.int32)
        mv = C.c_int64()
        kd = np.zeros(6, dtype=np.int64)
        L = int(self.lib.orc_local_search_tour(self.h, _ptr(t), int(length), C.byref(mv),
                                               _ptr(kd)))
        return (t, L, mv.value, kd.tolist()) if kinds else (t, L, mv.value)

    def set_local_search_cap(self, moves: int):
        """At most ``moves`` moves per descent (0: the default 50 n)."""
        if self.lib.orc_set_local_search_cap(self.h, int(moves)) != 0:
            raise ValueError("oracle: the move cap must be >= 0")

    def ls_moves(self) -> int:
        return int(self.lib.orc_ls_moves(self.h))

    def global_update(self):
        self.lib.orc_global_update(self.h)

    @property
    def iteration(self) -> int:
        return int(self.lib.orc_iteration(self.h))

    # state
    def constants(self) -> dict:
        lnn = C.c_int64()
        tau0, al, bl, ag = C.c_float(), C.c_float(), C.c_float(), C.c_float()
        q = C.c_uint32()
        self.lib.orc_constants(self.h, C.byref(lnn), C.byref(tau0), C.byref(al),
                               C.byref(bl), C.byref(ag), C.byref(q))
        return dict(lnn=lnn.value, tau0=np.float32(tau0.value), a_loc=np.float32(al.value),
                    b_loc=np.float32(bl.value), a_glob=np.float32(ag.value), q0_24=q.value)

    def dist(self) -> np.ndarray:
        out = np.empty((self.n, self.n), dtype=np.int32)
        self.lib.orc_get_dist(self.h, _ptr(out))
        return out

    def cand(self) -> np.ndarray:
        out = np.empty((self.n, self.cl), dtype=np.int32)
        self.lib.orc_get_cand(self.h, _ptr(out))
        return out

    def eta(self, count) -> np.ndarray:
        out = np.empty(count, dtype=np.float32)
        self.lib.orc_get_eta(self.h, _ptr(out), count)
        return out

    def tau(self) -> np.ndarray:
        out = np.empty((self.n, self.n), dtype=np.float32)
        self.lib.orc_get_tau(self.h, _ptr(out))
        return out

    def spm(self):
        nodes = np.empty((self.n, self.spm_s), dtype=np.int32)
        vals = np.empty((self.n, self.spm_s), dtype=np.float32)
        tail = np.empty(self.n, dtype=np.int32)
        self.lib.orc_get_spm(self.h, _ptr(nodes), _ptr(vals), _ptr(tail))
        return nodes, vals, tail

    def tours(self) -> np.ndarray:
        out = np.empty((self.m, self.n), dtype=np.int32)
        self.lib.orc_get_tours(self.h, _ptr(out))
        return out

    def lengths(self) -> np.ndarray:
        out = np.empty(self.m, dtype=np.int64)
        self.lib.orc_get_lengths(self.h, _ptr(out))
        return out

    def best(self):
        t = np.empty(self.n, dtype=np.int32)
        L = int(self.lib.orc_get_best(self.h, _ptr(t)))
        return (t if L >= 0 else None), L

    def iter_best(self):
        a = C.c_int32()
        L = int(self.lib.orc_get_iter_best(self.h, C.byref(a)))
        return a.value, L

    def counts(self) -> dict:
        out = np.zeros(6, dtype=np.int64)
        self.lib.orc_get_counts(self.h, _ptr(out))
        keys = ("steps", "greedy", "roulette", "fallback", "spm_hits", "spm_misses")
        return {k: int(v) for k, v in zip(keys, out)}

    def set_candidate_weights(self, w) -> None:
        """Scores (n, cl) in place of eta^beta of the candidates; None restores."""
        if w is None:
            self.lib.orc_set_candidate_weights(self.h, None)
            return
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(self.n, self.cl)
        if self.lib.orc_set_candidate_weights(self.h, _ptr(w)) != 0:
            raise ValueError("oracle: candidate weights must be positive and finite")

    def set_best(self, tour, length: int) -> None:
        t = np.ascontiguousarray(tour, dtype=np.int32)
        if self.lib.orc_set_best(self.h, _ptr(t), int(length)) != 0:
            raise ValueError("oracle: not a permutation")

    def set_tau(self, tau) -> None:
        """Dense pheromone matrix (n, n) to start from."""
        t = np.ascontiguousarray(tau, dtype=np.float32).reshape(self.n, self.n)
        if self.lib.orc_set_tau(self.h, _ptr(t)) != 0:
            raise ValueError("oracle: set_tau needs a dense handle and positive values")

    def spm_update(self, u: int, v: int, a: float, b: float) -> None:
        """Alg. 3 on the record of u for neighbour v with x -> fmaf(a, x, b)."""
        if self.lib.orc_spm_update(self.h, u, v, float(np.float32(a)),
                                   float(np.float32(b))) != 0:
            raise ValueError("oracle: spm_update on a dense handle or bad city")

    def local_map_k(self, x: float, k: int) -> np.float32:
        return np.float32(self.lib.orc_local_map_k(self.h, float(np.float32(x)), k))
