"""Python binding of libknnd.so: comparator-based K-nearest-neighbor descent
with the Kullback-Leibler comparator on an AMD MI355X (gfx950).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Host inputs are numpy arrays; device inputs are torch tensors on the
current HIP device (torch supplies memory and the stream).  The names mirror
the C ABI in include/knnd.h.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libknnd.so")

KNND_OK = 0
KNND_WARN_MAX_ROUNDS = 1
KNND_ERR_ARG = -1
KNND_ERR_DOMAIN = -2
KNND_ERR_NOMEM = -3
KNND_ERR_DEVICE = -4
KNND_ERR_UNSUPPORTED = -5

KNND_F32, KNND_F64 = 0, 1
KNND_PREC_FP64, KNND_PREC_MIXED_BF16, KNND_PREC_MIXED_FP16, KNND_PREC_AUTO = 0, 1, 2, 3
KNND_FLAG_NO_SKIP = 0x1
KNND_FLAG_PULL = 0x2
KNND_FLAG_ATOMIC_CSR = 0x4
KNND_FLAG_NO_CARRY = 0x8
KNND_FLAG_NO_GRAPH = 0x10
KNND_FLAG_NO_TUNE = 0x20
KNND_STOP_FCR, KNND_STOP_FIXED_POINT, KNND_STOP_DELTA = 0, 1, 2
KNND_CMP_KL, KNND_CMP_KL_REVERSE, KNND_CMP_HELLINGER, KNND_CMP_L2 = 0, 1, 2, 3

EXPORTED = [
    "knnd_default_params", "knnd_status_string", "knnd_abi_version", "knnd_build",
    "knnd_build_ex", "knnd_ctx_create", "knnd_ctx_init_graph", "knnd_ctx_set_graph",
    "knnd_ctx_round", "knnd_ctx_round_share", "knnd_ctx_get_graph", "knnd_ctx_get_log_table", "knnd_ctx_rounds",
    "knnd_ctx_destroy", "knnd_build_batched", "knnd_exact_knn", "knnd_release_cache",
    "knnd_build_noalloc", "knnd_ctx_get_cofriends", "knnd_memory_stats", "knnd_test_fail_alloc",
]
KNND_NOALLOC_MAX_BYTES = 256 << 20


ABI_VERSION = 7


class knnd_params(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("fcr_samples", ctypes.c_int64), ("max_rounds", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("stop_rule", ctypes.c_int32),
                ("comparator", ctypes.c_int32), ("delta", ctypes.c_double)]


class knnd_round_stats(ctypes.Structure):
    _fields_ = [("updates", ctypes.c_int64), ("fcr_hits", ctypes.c_int64),
                ("evals_alg", ctypes.c_int64), ("evals_performed", ctypes.c_int64),
                ("rescues", ctypes.c_int64), ("ms", ctypes.c_double),
                ("ms_join", ctypes.c_double), ("ms_hub", ctypes.c_double),
                ("ms_recv", ctypes.c_double), ("carried", ctypes.c_int64),
                ("evals_carried", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class knnd_instance(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("K", ctypes.c_int32), ("seed", ctypes.c_uint64), ("out_idx", ctypes.c_void_p),
                ("out_kl", ctypes.c_void_p), ("stats", ctypes.POINTER(knnd_round_stats)),
                ("out_rounds", ctypes.POINTER(ctypes.c_int32)), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class KnndError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None


def lib():
    """The loaded library.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    L.knnd_abi_version.restype = ctypes.c_int
    if L.knnd_abi_version() != ABI_VERSION:  # (before binding names an old library may lack)
        raise RuntimeError(f"{LIB_PATH} has ABI version {L.knnd_abi_version()}, this binding "
                           f"expects {ABI_VERSION}; rebuild the library")
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    P = ctypes.POINTER
    sig = {
        "knnd_default_params": (None, [P(knnd_params)]),
        "knnd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "knnd_abi_version": (ctypes.c_int, []),
        "knnd_build": (ctypes.c_int, [vp, i64, i32, i32, u64, vp, vp, i32, vp]),
        "knnd_build_ex": (ctypes.c_int, [vp, i64, i32, i32, u64, P(knnd_params), i32, vp, vp, vp,
                                         P(knnd_round_stats), vp]),
        "knnd_ctx_create": (ctypes.c_int, [vp, i64, i32, i32, u64, P(knnd_params), i32, vp,
                                           P(vp)]),
        "knnd_ctx_init_graph": (ctypes.c_int, [vp, P(knnd_round_stats)]),
        "knnd_ctx_set_graph": (ctypes.c_int, [vp, vp, vp, i32, i32]),
        "knnd_ctx_round": (ctypes.c_int, [vp, P(knnd_round_stats)]),
        "knnd_ctx_round_share": (ctypes.c_int, [vp, i64, i64, P(knnd_round_stats)]),
        "knnd_ctx_get_graph": (ctypes.c_int, [vp, vp, vp, i32]),
        "knnd_ctx_get_log_table": (ctypes.c_int, [vp, vp, i32]),
        "knnd_ctx_get_cofriends": (ctypes.c_int, [vp, vp, vp, i32]),
        "knnd_ctx_rounds": (ctypes.c_int, [vp]),
        "knnd_ctx_destroy": (ctypes.c_int, [vp]),
        "knnd_build_batched": (ctypes.c_int, [P(knnd_instance), i32, P(knnd_params), i32, vp]),
        "knnd_exact_knn": (ctypes.c_int, [vp, i64, i32, i32, i32, i32, vp, i64, vp, i32, vp, vp, vp]),
        "knnd_release_cache": (ctypes.c_int, []),
        "knnd_memory_stats": (ctypes.c_int, [vp, vp]),
        "knnd_test_fail_alloc": (i64, [i64]),
        "knnd_build_noalloc": (ctypes.c_int, [vp, i64, i32, i32, u64, P(knnd_params), vp, vp, vp,
                                              P(knnd_round_stats), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_string(status):
    return lib().knnd_status_string(status).decode()


def release_cache():
    """Return the library's cached device memory to the device."""
    return lib().knnd_release_cache()


def memory_stats():
    """(live, cached): bytes of device memory in use by live contexts and
    running calls, and held in the library's cache."""
    live, cached = ctypes.c_int64(), ctypes.c_int64()
    lib().knnd_memory_stats(ctypes.byref(live), ctypes.byref(cached))
    return live.value, cached.value


def inject_alloc_failure(k):
    """Failure injection (tests): the k-th device allocation from now on
    fails as out of memory (k <= 0 disarms).  Returns how many allocations
    were still to go before the previously armed failure (0: none armed, or
    it fired)."""
    return lib().knnd_test_fail_alloc(int(k))


def default_params(**kw):
    p = knnd_params()
    lib().knnd_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _is_device(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def _ptr(a):
    if a is None:
        return None
    return a.data_ptr() if _is_device(a) else a.ctypes.data


def _stream_of(a, stream):
    if stream is not None:
        return stream
    if _is_device(a):
        import torch
        return torch.cuda.current_stream(a.device).cuda_stream
    return None


def _dtype_code(points):
    name = str(points.dtype)
    if name.endswith("float32"):
        return KNND_F32
    if name.endswith("float64"):
        return KNND_F64
    raise TypeError("points must be float32 or float64")


def _empty(like, shape, kind):
    """Output buffer of numpy dtype `kind` on the same side as `like`."""
    if _is_device(like):
        import torch
        tdt = {np.int32: torch.int32, np.float64: torch.float64}[kind]
        return torch.empty(shape, dtype=tdt, device=like.device)
    return np.empty(shape, dtype=kind)


def _check_points(points, d):
    if points.ndim != 2 or points.shape[1] != d + 1:
        raise ValueError(f"points must have shape [n][{d + 1}]")
    if _is_device(points):
        if not points.is_contiguous():
            raise ValueError("device points must be contiguous")
        return points
    return np.ascontiguousarray(points)


def knnd_build(points, d, K, seed, max_rounds=100):
    """Basic call: host FP32 points [n][d+1] -> (idx [n][K] int32, per-round
    update counts, rounds)."""
    points = np.ascontiguousarray(points, dtype=np.float32)
    if points.ndim != 2 or points.shape[1] != d + 1:
        raise ValueError(f"points must have shape [n][{d + 1}]")
    n = points.shape[0]
    idx = np.empty((n, K), dtype=np.int32)
    upd = np.zeros(max(max_rounds, 1), dtype=np.int64)
    rounds = ctypes.c_int32(0)
    st = lib().knnd_build(points.ctypes.data, n, d, K, seed, idx.ctypes.data, upd.ctypes.data,
                          max_rounds, ctypes.byref(rounds))
    if st < 0:
        raise KnndError(st, "knnd_build")
    return idx, upd[:rounds.value].copy(), rounds.value, st


def knnd_build_ex(points, d, K, seed, params=None, stream=None, with_kl=True):
    """Extended call.  points: numpy array (host) or torch tensor on the GPU
    (device); outputs are on the same side.  Returns a dict with status, idx,
    kl, stats (one dict per round, entry 0 = start) and rounds."""
    points = _check_points(points, d)
    n = points.shape[0]
    p = params if params is not None else default_params()
    p.dtype = _dtype_code(points)
    R = (p.max_rounds if p.max_rounds > 0 else 100) + 1
    stats = (knnd_round_stats * R)()
    idx = _empty(points, (n, K), np.int32)
    kl = _empty(points, (n, K), np.float64) if with_kl else None
    rounds = ctypes.c_int32(0)
    dev = 1 if _is_device(points) else 0
    st = lib().knnd_build_ex(_ptr(points), n, d, K, seed, ctypes.byref(p), dev,
                             _stream_of(points, stream), _ptr(idx), _ptr(kl), stats,
                             ctypes.byref(rounds))
    if st < 0:
        raise KnndError(st, "knnd_build_ex")
    r = rounds.value
    return {"status": st, "idx": idx, "kl": kl, "rounds": r,
            "stats": [stats[i].as_dict() for i in range(r + 1)]}


def knnd_build_noalloc(points, d, K, seed, params=None, stream=None, idx=None, kl=None):
    """The descent with every device buffer in the library's fixed scratch
    array (knnd_build_noalloc: nothing is allocated).  points: torch tensor on
    the GPU; idx / kl: optional caller-allocated device outputs ([n][K] int32
    and FP64; kl=False for none), allocated here when not given.  Returns a
    dict like knnd_build_ex's."""
    points = _check_points(points, d)
    if not _is_device(points):
        raise ValueError("knnd_build_noalloc takes device tensors")
    n = points.shape[0]
    p = params if params is not None else default_params()
    p.dtype = _dtype_code(points)
    R = (p.max_rounds if p.max_rounds > 0 else 100) + 1
    stats = (knnd_round_stats * R)()
    if idx is None:
        idx = _empty(points, (n, K), np.int32)
    if kl is None:
        kl = _empty(points, (n, K), np.float64)
    elif kl is False:
        kl = None
    rounds = ctypes.c_int32(0)
    st = lib().knnd_build_noalloc(_ptr(points), n, d, K, seed, ctypes.byref(p),
                                  _stream_of(points, stream), _ptr(idx), _ptr(kl), stats,
                                  ctypes.byref(rounds))
    if st < 0:
        raise KnndError(st, "knnd_build_noalloc")
    r = rounds.value
    return {"status": st, "idx": idx, "kl": kl, "rounds": r,
            "stats": [stats[i].as_dict() for i in range(r + 1)]}


def knnd_build_batched(instances, params=None, stream=None, with_kl=True):
    """Batched call.  instances: list of (points, d, K, seed), every points
    array on the same side (numpy host arrays or torch device tensors) and of
    the same dtype.  Returns (status, list of dicts like knnd_build_ex's)."""
    if not instances:
        raise ValueError("no instances")
    p = params if params is not None else default_params()
    p.dtype = _dtype_code(instances[0][0])
    R = (p.max_rounds if p.max_rounds > 0 else 100) + 1
    arr = (knnd_instance * len(instances))()
    keep = []
    dev = 1 if _is_device(instances[0][0]) else 0
    for b, (points, d, K, seed) in enumerate(instances):
        points = _check_points(points, d)
        if (1 if _is_device(points) else 0) != dev or _dtype_code(points) != p.dtype:
            raise ValueError("every instance must have the same memory kind and dtype")
        n = points.shape[0]
        idx = _empty(points, (n, K), np.int32)
        kl = _empty(points, (n, K), np.float64) if with_kl else None
        stats = (knnd_round_stats * R)()
        rounds = ctypes.c_int32(0)
        keep.append((points, idx, kl, stats, rounds))
        arr[b].points, arr[b].n, arr[b].d, arr[b].K, arr[b].seed = _ptr(points), n, d, K, seed
        arr[b].out_idx, arr[b].out_kl = _ptr(idx), _ptr(kl)
        arr[b].stats = stats
        arr[b].out_rounds = ctypes.pointer(rounds)
    st = lib().knnd_build_batched(arr, len(instances), ctypes.byref(p), dev,
                                  _stream_of(instances[0][0], stream))
    if st < 0:
        raise KnndError(st, "knnd_build_batched")
    out = []
    for b, (points, idx, kl, stats, rounds) in enumerate(keep):
        r = rounds.value
        out.append({"status": arr[b].status, "idx": idx, "kl": kl, "rounds": r,
                    "stats": [stats[i].as_dict() for i in range(r + 1)]})
    return st, out


def knnd_exact_knn(points, d, K, queries, tau=None, stream=None, with_kl=True, comparator=KNND_CMP_KL):
    """Exact K nearest neighbours of the points listed in `queries` (int32
    indices), by exhaustive comparison under `comparator`.  points/queries/
    tau: numpy host arrays or torch device tensors (all on the same side);
    outputs on that side.  Returns (idx [nq][K], kl [nq][K] or None)."""
    points = _check_points(points, d)
    n = points.shape[0]
    dev = 1 if _is_device(points) else 0
    if dev:
        import torch
        queries = queries.to(device=points.device, dtype=torch.int32).contiguous()
        if tau is not None:
            tau = tau.to(device=points.device, dtype=torch.float64).contiguous()
    else:
        queries = np.ascontiguousarray(queries, dtype=np.int32)
        if tau is not None:
            tau = np.ascontiguousarray(tau, dtype=np.float64)
    nq = queries.shape[0]
    idx = _empty(points, (nq, K), np.int32)
    kl = _empty(points, (nq, K), np.float64) if with_kl else None
    st = lib().knnd_exact_knn(_ptr(points), n, d, K, _dtype_code(points), comparator, _ptr(queries), nq,
                              _ptr(tau), dev, _stream_of(points, stream), _ptr(idx), _ptr(kl))
    if st < 0:
        raise KnndError(st, "knnd_exact_knn")
    return idx, kl


class Context:
    """The step-by-step interface (knnd_ctx_*)."""

    def __init__(self, points, d, K, seed, params=None, stream=None):
        points = _check_points(points, d)
        self.points = points
        self.n, self.d, self.K = points.shape[0], d, K
        self.device = _is_device(points)
        p = params if params is not None else default_params()
        p.dtype = _dtype_code(points)
        self._stream = _stream_of(points, stream)
        h = ctypes.c_void_p()
        st = lib().knnd_ctx_create(_ptr(points), self.n, d, K, seed, ctypes.byref(p),
                                   1 if self.device else 0, self._stream, ctypes.byref(h))
        if st != KNND_OK:
            raise KnndError(st, "knnd_ctx_create")
        self.h = h

    def init_graph(self):
        s = knnd_round_stats()
        st = lib().knnd_ctx_init_graph(self.h, ctypes.byref(s))
        if st != KNND_OK:
            raise KnndError(st, "knnd_ctx_init_graph")
        return s.as_dict()

    def set_graph(self, idx, kl, rnd=0):
        if self.device:
            st = lib().knnd_ctx_set_graph(self.h, _ptr(idx), _ptr(kl), rnd, 1)
        else:
            idx = np.ascontiguousarray(idx, dtype=np.int32)
            kl = np.ascontiguousarray(kl, dtype=np.float64)
            st = lib().knnd_ctx_set_graph(self.h, idx.ctypes.data, kl.ctypes.data, rnd, 0)
        if st != KNND_OK:
            raise KnndError(st, "knnd_ctx_set_graph")

    def round(self):
        s = knnd_round_stats()
        st = lib().knnd_ctx_round(self.h, ctypes.byref(s))
        if st != KNND_OK:
            raise KnndError(st, "knnd_ctx_round")
        return s.as_dict()

    def round_share(self, first, count):
        """One round in which only the lists of points first .. first+count-1
        are recomputed; every other list is carried over, and the next round
        skips no candidate pair."""
        s = knnd_round_stats()
        st = lib().knnd_ctx_round_share(self.h, int(first), int(count), ctypes.byref(s))
        if st != KNND_OK:
            raise KnndError(st, "knnd_ctx_round_share")
        return s.as_dict()

    def get_graph(self, with_kl=True):
        idx = _empty(self.points, (self.n, self.K), np.int32)
        kl = _empty(self.points, (self.n, self.K), np.float64) if with_kl else None
        st = lib().knnd_ctx_get_graph(self.h, _ptr(idx), _ptr(kl), 1 if self.device else 0)
        if st != KNND_OK:
            raise KnndError(st, "knnd_ctx_get_graph")
        return idx, kl

    def cofriends(self):
        """(rowptr [n+1] int64, col [nK] int32): the co-friend lists of the
        current graph, each segment in increasing order (host arrays)."""
        n = self.points.shape[0]
        rowptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(n * self.K, dtype=np.int32)
        st = lib().knnd_ctx_get_cofriends(self.h, rowptr.ctypes.data, col.ctypes.data, 0)
        if st < 0:
            raise KnndError(st, "knnd_ctx_get_cofriends")
        return rowptr, col

    def log_table(self):
        L = _empty(self.points, (self.n, self.d + 1), np.float64)
        st = lib().knnd_ctx_get_log_table(self.h, _ptr(L), 1 if self.device else 0)
        if st != KNND_OK:
            raise KnndError(st, "knnd_ctx_get_log_table")
        return L

    @property
    def rounds(self):
        return lib().knnd_ctx_rounds(self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().knnd_ctx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
