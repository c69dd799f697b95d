"""Python binding of libacs (ctypes).  Argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch is used
for the plumbing the C-ABI accepts: a device workspace tensor and the current
HIP stream.  If libacs.so has not been built the import fails loudly; there
is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libacs.so")

ACS_OK = 0
ACS_E_INVALID = -1
ACS_E_NOMEM = -2
ACS_E_DEVICE = -3
ACS_E_BUFSIZE = -4
ACS_E_STATE = -5
ACS_E_UNSUPPORTED = -6

ACS_DENSE, ACS_SPM = 0, 1
ACS_SYNC, ACS_ASYNC_ATOMIC, ACS_ASYNC_RACY, ACS_SEQUENTIAL = 0, 1, 2, 3


class acs_params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("m", C.c_uint32), ("cl", C.c_uint32),
        ("memory", C.c_uint32), ("spm_s", C.c_uint32), ("mode", C.c_uint32),
        ("local_update_period", C.c_uint32), ("instance", C.c_uint32),
        ("beta", C.c_double), ("q0", C.c_double), ("phi", C.c_double),
        ("rho", C.c_double), ("tau0", C.c_double), ("seed", C.c_uint64),
        ("stream", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
        ("lanes_per_ant", C.c_uint32), ("update_path", C.c_uint32),
        ("wait_limit", C.c_uint32), ("local_search", C.c_uint32),
    ]


class acs_stats_t(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("iteration", C.c_uint32),
        ("best_length", C.c_int64), ("iter_best_length", C.c_int64),
        ("iter_best_ant", C.c_int32), ("n", C.c_int32), ("m", C.c_int32), ("cl", C.c_int32),
        ("nn_length", C.c_int64), ("tau0", C.c_float), ("pad0", C.c_float),
        ("steps", C.c_int64), ("greedy", C.c_int64), ("roulette", C.c_int64),
        ("fallback", C.c_int64), ("spm_hits", C.c_int64), ("spm_misses", C.c_int64),
        ("fallback_unvisited", C.c_int64), ("cas_retries", C.c_int64),
        ("construct_ms", C.c_double), ("construct_launches", C.c_int32), ("pad1", C.c_int32),
        ("iterate_ms", C.c_double), ("ls_moves", C.c_int64),
    ]


class AcsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libacs error {code}: {msg}")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Loads libacs.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "python -m paper_1605_02669_amd.build")
    lib = C.CDLL(LIB_PATH)
    P, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.acs_default_params.argtypes = [C.POINTER(acs_params)]
    lib.acs_workspace_bytes.argtypes = [i32, C.POINTER(acs_params), C.POINTER(sz)]
    lib.acs_create.argtypes = [P, i32, C.POINTER(acs_params), C.POINTER(P)]
    lib.acs_iterate.argtypes = [P, i32]
    lib.acs_best_tour.argtypes = [P, P, C.POINTER(i64)]
    lib.acs_pheromone_snapshot.argtypes = [P, P, sz]
    lib.acs_spm_snapshot.argtypes = [P, P, P, P]
    lib.acs_tours.argtypes = [P, P, sz]
    lib.acs_lengths.argtypes = [P, P, sz]
    lib.acs_candidates.argtypes = [P, P, sz]
    lib.acs_stats.argtypes = [P, C.POINTER(acs_stats_t)]
    lib.acs_destroy.argtypes = [P]
    lib.acs_destroy.restype = None
    lib.acs_batch_workspace_bytes.argtypes = [P, i32, C.POINTER(acs_params), C.POINTER(sz)]
    lib.acs_batch_create.argtypes = [P, P, i32, C.POINTER(acs_params), C.POINTER(P)]
    lib.acs_batch_iterate.argtypes = [P, i32]
    lib.acs_batch_info.argtypes = [P, C.POINTER(i32), C.POINTER(i64), C.POINTER(i32),
                                   C.POINTER(C.c_double)]
    lib.acs_batch_tuning.argtypes = [P, C.POINTER(i32), C.POINTER(i32), P, P, P, i32]
    lib.acs_batch_instance.argtypes = [P, i32, C.POINTER(P)]
    lib.acs_batch_set_exchange.argtypes = [P, i32, i32]
    lib.acs_batch_best_tour.argtypes = [P, i32, P, C.POINTER(i64)]
    lib.acs_batch_destroy.argtypes = [P]
    lib.acs_batch_destroy.restype = None
    lib.acs_prior_features.argtypes = [P, P]
    lib.acs_prior_forward.argtypes = [P, P, i32, P, P]
    lib.acs_prior_grad.argtypes = [P, P, P, i32, P, P, P]
    lib.acs_prior_adam.argtypes = [P, P, P, P, i32, C.c_float, C.c_float, C.c_float, C.c_float, P]
    lib.acs_prior_apply.argtypes = [P, P]
    lib.acs_set_candidate_scores.argtypes = [P, P]
    lib.acs_candidate_weights.argtypes = [P, P, sz]
    lib.acs_solve_static.argtypes = [P, i32, C.POINTER(acs_params), i32, P, C.POINTER(i64)]
    lib.acs_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != ACS_OK:
        raise AcsError(rc, load().acs_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def acs_default_params() -> acs_params:
    p = acs_params()
    _check(load().acs_default_params(C.byref(p)))
    return p


def acs_workspace_bytes(n: int, p: acs_params) -> int:
    out = C.c_size_t()
    _check(load().acs_workspace_bytes(n, C.byref(p), C.byref(out)))
    return out.value


def acs_create(xy: np.ndarray, p: acs_params) -> C.c_void_p:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    h = C.c_void_p()
    _check(load().acs_create(_ptr(xy), xy.shape[0], C.byref(p), C.byref(h)))
    return h


def acs_iterate(h, k: int) -> None:
    _check(load().acs_iterate(h, k))


def acs_best_tour(h, n: int):
    t = np.empty(n, dtype=np.int32)
    L = C.c_int64()
    _check(load().acs_best_tour(h, _ptr(t), C.byref(L)))
    return t, L.value


def acs_pheromone_snapshot(h, n: int) -> np.ndarray:
    out = np.empty((n, n), dtype=np.float32)
    _check(load().acs_pheromone_snapshot(h, _ptr(out), out.size))
    return out


def acs_spm_snapshot(h, n: int, s: int):
    nodes = np.empty((n, s), dtype=np.int32)
    vals = np.empty((n, s), dtype=np.float32)
    tail = np.empty(n, dtype=np.int32)
    _check(load().acs_spm_snapshot(h, _ptr(nodes), _ptr(vals), _ptr(tail)))
    return nodes, vals, tail


def acs_tours(h, m: int, n: int) -> np.ndarray:
    out = np.empty((m, n), dtype=np.int32)
    _check(load().acs_tours(h, _ptr(out), out.size))
    return out


def acs_lengths(h, m: int) -> np.ndarray:
    out = np.empty(m, dtype=np.int64)
    _check(load().acs_lengths(h, _ptr(out), out.size))
    return out


def acs_candidates(h, n: int, cl: int) -> np.ndarray:
    out = np.empty((n, cl), dtype=np.int32)
    _check(load().acs_candidates(h, _ptr(out), out.size))
    return out


def acs_stats(h) -> dict:
    s = acs_stats_t()
    s.struct_size = C.sizeof(acs_stats_t)
    _check(load().acs_stats(h, C.byref(s)))
    return {name: getattr(s, name) for name, _ in acs_stats_t._fields_
            if not name.startswith("pad") and name != "struct_size"}


def acs_destroy(h) -> None:
    load().acs_destroy(h)


def acs_solve_static(xy: np.ndarray, p: acs_params, iterations: int):
    """Best tour and length after `iterations` iterations, with the device
    workspace in the library's static array (no device allocation)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    t = np.empty(xy.shape[0], dtype=np.int32)
    L = C.c_int64()
    _check(load().acs_solve_static(_ptr(xy), xy.shape[0], C.byref(p), iterations, _ptr(t),
                                   C.byref(L)))
    return t, L.value


def make_params(m=0, cl=32, beta=2.0, q0=0.9, phi=0.1, rho=0.1, tau0=0.0, memory=ACS_DENSE,
                spm_s=8, mode=ACS_SYNC, seed=0, instance=0, local_update_period=1,
                lanes_per_ant=0, update_path=0, wait_limit=0, local_search=0) -> acs_params:
    p = acs_default_params()
    p.m, p.cl, p.beta, p.q0, p.phi, p.rho, p.tau0 = m, cl, beta, q0, phi, rho, tau0
    p.memory, p.spm_s, p.mode, p.seed, p.instance = memory, spm_s, mode, seed, instance
    p.local_update_period = local_update_period
    p.lanes_per_ant = lanes_per_ant
    p.update_path = update_path
    p.wait_limit = wait_limit
    p.local_search = local_search
    return p


class Colony:
    """One colony on one instance, owning its handle.

    With ``torch_memory`` the device workspace is a torch tensor and the
    library runs on torch's current stream; otherwise the library allocates
    and uses a stream of its own.
    """

    def __init__(self, xy, m=0, cl=32, beta=2.0, q0=0.9, phi=0.1, rho=0.1, tau0=0.0,
                 memory=ACS_DENSE, spm_s=8, mode=ACS_SYNC, seed=0, instance=0,
                 local_update_period=1, lanes_per_ant=0, update_path=0, wait_limit=0,
                 local_search=0, torch_memory=True):
        self.xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        n = self.xy.shape[0]
        p = make_params(m=m, cl=cl, beta=beta, q0=q0, phi=phi, rho=rho, tau0=tau0, memory=memory,
                        spm_s=spm_s, mode=mode, seed=seed, instance=instance,
                        local_update_period=local_update_period, lanes_per_ant=lanes_per_ant,
                        update_path=update_path, wait_limit=wait_limit,
                        local_search=local_search)
        self._ws = None
        if torch_memory:
            import torch
            nbytes = acs_workspace_bytes(n, p)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            p.workspace, p.workspace_bytes = self._ws.data_ptr(), nbytes
            p.stream = torch.cuda.current_stream().cuda_stream
        self.params = p
        self.h = acs_create(self.xy, p)
        st = acs_stats(self.h)
        self.n, self.m, self.cl = st["n"], st["m"], st["cl"]
        self.memory, self.spm_s = memory, spm_s

    def close(self):
        if getattr(self, "h", None):
            acs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, k=1):
        acs_iterate(self.h, k)

    def best(self):
        return acs_best_tour(self.h, self.n)

    def tau(self):
        return acs_pheromone_snapshot(self.h, self.n)

    def spm(self):
        return acs_spm_snapshot(self.h, self.n, self.spm_s)

    def tours(self):
        return acs_tours(self.h, self.m, self.n)

    def lengths(self):
        return acs_lengths(self.h, self.m)

    def cand(self):
        return acs_candidates(self.h, self.n, self.cl)

    def stats(self):
        return acs_stats(self.h)

    def candidate_weights(self):
        out = np.empty((self.n, self.cl), dtype=np.float32)
        _check(load().acs_candidate_weights(self.h, _ptr(out), out.size))
        return out

    def set_candidate_scores(self, scores):
        sc = np.ascontiguousarray(scores, dtype=np.float32).reshape(self.n, self.cl)
        _check(load().acs_set_candidate_scores(self.h, _ptr(sc)))

    def prior_features(self):
        """Edge features (n*16, 4) as a torch tensor on the GPU."""
        import torch
        X = torch.empty((self.n * 16, 4), dtype=torch.float32, device="cuda")
        _check(load().acs_prior_features(self.h, C.c_void_p(X.data_ptr())))
        return X

    def apply_prior(self, params):
        """Replace the candidate weights by the network's scores (params: cuda tensor)."""
        _check(load().acs_prior_apply(self.h, C.c_void_p(params.data_ptr())))


def acs_batch_workspace_bytes(sizes, p: acs_params) -> int:
    n = np.ascontiguousarray(sizes, dtype=np.int32)
    out = C.c_size_t()
    _check(load().acs_batch_workspace_bytes(_ptr(n), len(n), C.byref(p), C.byref(out)))
    return out.value


class Batch:
    """Many instances, one colony each, iterated together (asynchronous mode)."""

    def __init__(self, instances, m=0, cl=32, beta=2.0, q0=0.9, phi=0.1, rho=0.1, tau0=0.0,
                 seed=0, instance=0, local_update_period=1, mode=ACS_ASYNC_ATOMIC,
                 lanes_per_ant=0, update_path=0, wait_limit=0, torch_memory=True):
        self.xys = [np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2) for x in instances]
        sizes = np.array([x.shape[0] for x in self.xys], dtype=np.int32)
        p = acs_default_params()
        p.m, p.cl, p.beta, p.q0, p.phi, p.rho, p.tau0 = m, cl, beta, q0, phi, rho, tau0
        p.mode, p.memory, p.seed, p.instance = mode, ACS_DENSE, seed, instance
        p.local_update_period = local_update_period
        p.lanes_per_ant = lanes_per_ant
        p.update_path = update_path
        p.wait_limit = wait_limit
        self._ws = None
        if torch_memory:
            import torch
            nbytes = acs_batch_workspace_bytes(sizes, p)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            p.workspace, p.workspace_bytes = self._ws.data_ptr(), nbytes
            p.stream = torch.cuda.current_stream().cuda_stream
        ptrs = (C.c_void_p * len(self.xys))(*[x.ctypes.data for x in self.xys])
        h = C.c_void_p()
        _check(load().acs_batch_create(ptrs, _ptr(sizes), len(sizes), C.byref(p), C.byref(h)))
        self.h = h
        self.sizes = sizes
        self.params = p

    def close(self):
        if getattr(self, "h", None):
            load().acs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, k=1):
        _check(load().acs_batch_iterate(self.h, k))

    def info(self) -> dict:
        c, steps, g, ms = C.c_int32(), C.c_int64(), C.c_int32(), C.c_double()
        _check(load().acs_batch_info(self.h, C.byref(c), C.byref(steps), C.byref(g), C.byref(ms)))
        return dict(count=c.value, steps_per_iteration=steps.value, graph=bool(g.value),
                    last_iterate_ms=ms.value)

    def tuning(self) -> dict:
        """Launch-shape candidates, named by lanes per ant ("64u": 64 lanes
        with an updater wave), with the ms of their timed iterations, and
        the chosen one (None while tuning)."""
        ch, cnt = C.c_int32(), C.c_int32()
        lanes, upd = (C.c_int32 * 8)(), (C.c_int32 * 8)()
        ms = (C.c_double * 8)()
        _check(load().acs_batch_tuning(self.h, C.byref(ch), C.byref(cnt), lanes, upd, ms, 8))
        names = [f"{lanes[j]}{'u' if upd[j] else ''}" for j in range(cnt.value)]
        return dict(chosen=names[ch.value] if ch.value >= 0 else None,
                    candidates={names[j]: float(ms[j]) for j in range(cnt.value)})

    def set_exchange(self, topology: int, period: int) -> None:
        """Best-so-far exchange between the instances (colonies of one
        instance) after every `period`-th iteration; topology 0 from the best
        colony, 1 from colony c - 1."""
        _check(load().acs_batch_set_exchange(self.h, topology, period))

    def handle(self, i: int):
        h = C.c_void_p()
        _check(load().acs_batch_instance(self.h, i, C.byref(h)))
        return h

    def best(self, i: int):
        return acs_best_tour(self.handle(i), int(self.sizes[i]))

    def tours(self, i: int):
        n = int(self.sizes[i])
        m = self.params.m or n
        return acs_tours(self.handle(i), m, n)

    def lengths(self, i: int):
        n = int(self.sizes[i])
        return acs_lengths(self.handle(i), self.params.m or n)

    def tau(self, i: int):
        return acs_pheromone_snapshot(self.handle(i), int(self.sizes[i]))

    def stats(self, i: int):
        return acs_stats(self.handle(i))


PRIOR_PARAMS = 4545


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def prior_forward(P, X):
    """Logits of the rows of X (cuda float32 tensors)."""
    import torch
    Z = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(load().acs_prior_forward(C.c_void_p(P.data_ptr()), C.c_void_p(X.data_ptr()),
                                    X.shape[0], C.c_void_p(Z.data_ptr()), _stream_ptr()))
    return Z


def prior_grad(P, X, Y, G, L):
    """Accumulates the mean-BCE gradient into G and the summed loss into L."""
    _check(load().acs_prior_grad(C.c_void_p(P.data_ptr()), C.c_void_p(X.data_ptr()),
                                 C.c_void_p(Y.data_ptr()), X.shape[0], C.c_void_p(G.data_ptr()),
                                 C.c_void_p(L.data_ptr()), _stream_ptr()))


def prior_adam(P, G, M, V, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load().acs_prior_adam(C.c_void_p(P.data_ptr()), C.c_void_p(G.data_ptr()),
                                 C.c_void_p(M.data_ptr()), C.c_void_p(V.data_ptr()), step, lr,
                                 beta1, beta2, eps, _stream_ptr()))


def pack_prior(p: dict) -> np.ndarray:
    """Parameter dict (W1, b1, W2, b2, W3, b3) -> flat float32 vector."""
    v = np.concatenate([p["W1"].reshape(-1), p["b1"].reshape(-1), p["W2"].reshape(-1),
                        p["b2"].reshape(-1), p["W3"].reshape(-1), p["b3"].reshape(-1)])
    assert v.size == PRIOR_PARAMS
    return v.astype(np.float32)


def unpack_prior(v) -> dict:
    v = np.asarray(v, dtype=np.float32)
    return {"W1": v[0:256].reshape(4, 64), "b1": v[256:320], "W2": v[320:4416].reshape(64, 64),
            "b2": v[4416:4480], "W3": v[4480:4544].reshape(64, 1), "b3": v[4544:4545]}
