"""ctypes binding of the CPU oracle (oracle/knnd_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports or links it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knnd_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, WARN_MAX_ROUNDS, ERR_ARG, ERR_DOMAIN = 0, 1, -1, -2
# comparators: D(x||y) (the paper's), D(y||x), sum (sqrt x - sqrt y)^2, sum (x - y)^2
CMP_KL, CMP_KL_REVERSE, CMP_HELLINGER, CMP_L2 = 0, 1, 2, 3


def build():
    """Compile liboracle.so with g++ (always recompiles)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
           "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lquadmath"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, i64, i32, u64, c_int = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_uint64, ctypes.c_int)
    sig = {
        "oracle_abi_version": (c_int, []),
        "oracle_mix64": (u64, [u64]),
        "oracle_hash": (u64, [u64, u64, u64, u64]),
        "oracle_bound": (u64, [u64, u64]),
        "oracle_log_table": (None, [vp, i64, vp, c_int]),
        "oracle_key": (ctypes.c_double, [vp, vp, c_int, i64, i64, c_int]),
        "oracle_initial_graph": (c_int, [vp, vp, i64, c_int, c_int, u64, vp, vp, c_int, c_int]),
        "oracle_fcr": (i64, [vp, i64, c_int, u64, i64, i64]),
        "oracle_fcr_exhaustive": (None, [vp, i64, c_int, vp, vp]),
        "oracle_candidates": (i64, [vp, i64, c_int, i64, vp, i64]),
        "oracle_round": (c_int, [vp, vp, i64, c_int, c_int, vp, vp, vp, vp, vp, vp, c_int, c_int]),
        "oracle_round_subset": (c_int, [vp, vp, i64, c_int, c_int, vp, vp, vp, i64, vp, vp,
                                        vp, vp, c_int, c_int]),
        "oracle_bruteforce": (c_int, [vp, vp, i64, c_int, c_int, vp, i64, vp, vp, c_int, c_int]),
        "oracle_should_stop": (c_int, [i64, i64, i64, c_int, c_int]),
        "oracle_build": (c_int, [vp, c_int, i64, c_int, c_int, u64, i64, c_int, c_int, vp, vp,
                                 vp, vp, vp, vp, vp, c_int, ctypes.c_double, c_int]),
        "oracle_stop_rule": (c_int, [c_int, ctypes.c_double, i64, c_int, i64, i64, i64, c_int, c_int, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data


def mix64(z):
    return int(_load().oracle_mix64(z))


def hash64(s, t, a, b):
    return int(_load().oracle_hash(s, t, a, b))


def bound(h, m):
    return int(_load().oracle_bound(h, m))


def widen(points):
    """FP64 copy of the points (exact widening from FP32)."""
    return np.ascontiguousarray(points, dtype=np.float64)


def log_table(P64, threads=0):
    P64 = np.ascontiguousarray(P64, dtype=np.float64)
    L = np.empty_like(P64)
    _load().oracle_log_table(_p(P64), P64.size, _p(L), threads)
    return L


def key(P64, L, x, y, cmp=CMP_KL):
    return float(_load().oracle_key(_p(P64), _p(L), P64.shape[1], x, y, cmp))


def initial_graph(P64, L, K, seed, threads=0, cmp=CMP_KL):
    n, D = P64.shape
    F = np.empty((n, K), dtype=np.int32)
    keys = np.empty((n, K), dtype=np.float64)
    rc = _load().oracle_initial_graph(_p(P64), _p(L), n, D, K, seed, _p(F), _p(keys), threads,
                                      cmp)
    if rc != OK:
        raise ValueError(f"oracle_initial_graph status {rc}")
    return F, keys


def fcr(F, seed, rnd, M):
    F = np.ascontiguousarray(F, dtype=np.int32)
    n, K = F.shape
    return int(_load().oracle_fcr(_p(F), n, K, seed, rnd, M))


def fcr_exhaustive(F):
    F = np.ascontiguousarray(F, dtype=np.int32)
    n, K = F.shape
    h = ctypes.c_int64()
    p = ctypes.c_int64()
    _load().oracle_fcr_exhaustive(_p(F), n, K, ctypes.byref(h), ctypes.byref(p))
    return h.value, p.value


def candidates(F, x):
    F = np.ascontiguousarray(F, dtype=np.int32)
    n, K = F.shape
    cap = n
    out = np.empty(cap, dtype=np.int32)
    m = _load().oracle_candidates(_p(F), n, K, x, _p(out), cap)
    return out[:m].copy()


def round_step(P64, L, F, keys, threads=0, cmp=CMP_KL):
    """One synchronous round; returns (F_next, keys_next, updates, evals)."""
    n, D = P64.shape
    K = F.shape[1]
    F = np.ascontiguousarray(F, dtype=np.int32)
    keys = np.ascontiguousarray(keys, dtype=np.float64)
    Fn = np.empty_like(F)
    kn = np.empty_like(keys)
    u = np.zeros(1, dtype=np.int64)
    e = np.zeros(1, dtype=np.int64)
    rc = _load().oracle_round(_p(P64), _p(L), n, D, K, _p(F), _p(keys), _p(Fn), _p(kn), _p(u),
                              _p(e), threads, cmp)
    if rc != OK:
        raise ValueError(f"oracle_round status {rc}")
    return Fn, kn, int(u[0]), int(e[0])


def round_subset(P64, L, F, keys, xs, threads=0, cmp=CMP_KL):
    """The round's update for vertices xs only: (F rows, key rows, updates, evals)."""
    n, D = P64.shape
    K = F.shape[1]
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    m = xs.size
    Fo = np.empty((m, K), dtype=np.int32)
    ko = np.empty((m, K), dtype=np.float64)
    up = np.empty(m, dtype=np.int64)
    ev = np.empty(m, dtype=np.int64)
    _load().oracle_round_subset(_p(P64), _p(L), n, D, K, _p(np.ascontiguousarray(F, np.int32)),
                                _p(np.ascontiguousarray(keys, np.float64)), _p(xs), m, _p(Fo),
                                _p(ko), _p(up), _p(ev), threads, cmp)
    return Fo, ko, up, ev


def bruteforce(P64, L, K, qs, threads=0, cmp=CMP_KL):
    n, D = P64.shape
    qs = np.ascontiguousarray(qs, dtype=np.int64)
    out = np.empty((qs.size, K), dtype=np.int32)
    keys = np.empty((qs.size, K), dtype=np.float64)
    rc = _load().oracle_bruteforce(_p(P64), _p(L), n, D, K, _p(qs), qs.size, _p(out), _p(keys),
                                   threads, cmp)
    if rc != OK:
        raise ValueError(f"oracle_bruteforce status {rc}")
    return out, keys


def should_stop(hits_prev, hits_cur, updates, rnd, max_rounds):
    return bool(_load().oracle_should_stop(hits_prev, hits_cur, updates, rnd, max_rounds))


STOP_FCR, STOP_FIXED_POINT, STOP_DELTA = 0, 1, 2


def stop_rule(rule, delta, n, K, hits_prev, hits_cur, updates, rnd, max_rounds):
    """(stop?, stopped only by the round cap?) under one of the stop rules."""
    capped = ctypes.c_int(0)
    s = _load().oracle_stop_rule(rule, delta, n, K, hits_prev, hits_cur, updates, rnd, max_rounds,
                                 ctypes.byref(capped))
    return bool(s), bool(capped.value)


class Result:
    """Outcome of a whole descent."""

    def __init__(self, status, idx, keys, updates, hits, evals, rounds, seconds):
        self.status, self.idx, self.keys = status, idx, keys
        self.updates, self.hits, self.evals = updates, hits, evals
        self.rounds, self.seconds = rounds, seconds


def build_graph(points, d, K, seed, M=0, max_rounds=100, threads=0, stop_rule=0, delta=0.0,
                cmp=CMP_KL):
    """Run the whole descent on points [n][d+1] (FP32 or FP64)."""
    points = np.ascontiguousarray(points)
    if points.dtype == np.float32:
        dtype = 0
    elif points.dtype == np.float64:
        dtype = 1
    else:
        raise TypeError("points must be float32 or float64")
    n = points.shape[0]
    idx = np.zeros((n, K), dtype=np.int32)
    keys = np.zeros((n, K), dtype=np.float64)
    R = max_rounds + 1
    upd = np.zeros(R, dtype=np.int64)
    hits = np.zeros(R, dtype=np.int64)
    evals = np.zeros(R, dtype=np.int64)
    secs = np.zeros(R, dtype=np.float64)
    rounds = ctypes.c_int32(0)
    st = _load().oracle_build(_p(points), dtype, n, d, K, seed, M, max_rounds, threads, _p(idx),
                              _p(keys), _p(upd), _p(hits), _p(evals), ctypes.byref(rounds),
                              _p(secs), stop_rule, delta, cmp)
    r = rounds.value
    return Result(st, idx, keys, upd[:r + 1], hits[:r + 1], evals[:r + 1], r, secs[:r + 1])
