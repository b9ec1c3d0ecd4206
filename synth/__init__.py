"""Seeded synthetic inputs (Dirichlet points on the simplex) shared by the GPU
library's tests/bench and the CPU oracle.  This package draws inputs only; it
contains none of the method's arithmetic.

The workloads follow the paper's experiments: i.i.d. Dirichlet(1,...,1) points
on the simplex (Section 4, scaling and dimension experiments, Tables 3-4),
clamped below at 1e-12 so every point is in the interior where the
Kullback-Leibler comparator is defined (Section 2.2).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dirichlet.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build():
    """Compile libsynth.so with gcc (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u64, i64, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32
    lib.synth_hash.restype = u64
    lib.synth_hash.argtypes = [u64, u64, u64, u64]
    lib.synth_bound.restype = u64
    lib.synth_bound.argtypes = [u64, u64]
    lib.synth_dirichlet_f64.restype = ctypes.c_int
    lib.synth_dirichlet_f64.argtypes = [u64, i64, ctypes.c_int, ctypes.c_void_p]
    lib.synth_dirichlet_f32.restype = ctypes.c_int
    lib.synth_dirichlet_f32.argtypes = [u64, i64, ctypes.c_int, ctypes.c_void_p]
    lib.synth_instance.restype = None
    lib.synth_instance.argtypes = [u64, i64] + [ctypes.c_void_p] * 5
    lib.synth_subsample.restype = ctypes.c_int
    lib.synth_subsample.argtypes = [u64, i64, i64, ctypes.c_void_p, ctypes.c_void_p]
    _lib = lib
    return lib


def hash64(s, t, a, b):
    return int(_load().synth_hash(s, t, a, b))


def bound(h, m):
    return int(_load().synth_bound(h, m))


def dirichlet(data_seed, n, d, dtype=np.float32):
    """n points with D = d+1 coordinates, row-major, FP32 or FP64."""
    D = d + 1
    lib = _load()
    if np.dtype(dtype) == np.float64:
        out = np.empty((n, D), dtype=np.float64)
        rc = lib.synth_dirichlet_f64(data_seed, n, D, out.ctypes.data)
    elif np.dtype(dtype) == np.float32:
        out = np.empty((n, D), dtype=np.float32)
        rc = lib.synth_dirichlet_f32(data_seed, n, D, out.ctypes.data)
    else:
        raise ValueError("dtype must be float32 or float64")
    if rc != 0:
        raise ValueError("bad generator arguments")
    return out


def instance(base, b):
    """Parameters of batched instance b: (n, d, K, data_seed, seed)."""
    n = ctypes.c_int64()
    d = ctypes.c_int32()
    K = ctypes.c_int32()
    ds = ctypes.c_uint64()
    s = ctypes.c_uint64()
    _load().synth_instance(base, b, ctypes.byref(n), ctypes.byref(d), ctypes.byref(K),
                           ctypes.byref(ds), ctypes.byref(s))
    return n.value, d.value, K.value, ds.value, s.value


def subsample(seed, n, m):
    """m distinct indices in [0, n), drawn by the counter hash with tag 7."""
    seen = np.empty(n, dtype=np.uint8)
    out = np.empty(m, dtype=np.int64)
    if _load().synth_subsample(seed, n, m, seen.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("m > n")
    return out


# The benchmark workloads, named by their sizes: (n, d, K, storage dtype, data
# seed, algorithm seed).
WORKLOADS = {
    "n2000_d5_k10": dict(n=2000, d=5, K=10, dtype=np.float64, data_seed=1001, seed=2001),
    "n100000_d10_k20": dict(n=100_000, d=10, K=20, dtype=np.float32, data_seed=1002, seed=2002),
    "n1000000_d20_k30": dict(n=1_000_000, d=20, K=30, dtype=np.float32, data_seed=1003, seed=2003),
    "n200000_d50_k20": dict(n=200_000, d=50, K=20, dtype=np.float32, data_seed=1004, seed=2004),
}
BATCH_WORKLOAD = "batch512"  # BATCH_INSTANCES instances drawn from BATCH_BASE_SEED
BATCH_BASE_SEED = 1005
BATCH_INSTANCES = 512
