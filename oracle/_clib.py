"""Loader of the oracle's own C routines (oracle/csrc), built with gcc.

TEST INFRASTRUCTURE ONLY.  The library is compiled in-tree (``build()``
here, also run by the repository's build entry point); a missing library is
built on first use.  Nothing here is shared with the HIP library.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "slab.c")
OUT = os.path.join(HERE, "lib", "liboracle_slab.so")
_LIB = None


def build():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    tmp = OUT + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", SRC, "-o", tmp, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gcc failed building the oracle's slab library:\n"
                           + res.stdout + res.stderr)
    os.replace(tmp, OUT)
    return OUT


def load():
    global _LIB
    if _LIB is None:
        if not os.path.exists(OUT):
            build()
        lib = ctypes.CDLL(OUT)
        u64, i64, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_philox_raw.argtypes = [vp, i64, u64, u64, vp]
        lib.oracle_philox_raw.restype = None
        lib.oracle_normal_slab.argtypes = [u64, u64, u64, i64, i64, vp, vp, vp, vp]
        lib.oracle_normal_slab.restype = None
        _LIB = lib
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox_raw(ctr, key):
    """Philox4x64-10 words of counters ctr[n, 4] under key (k0, k1)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64).reshape(-1, 4)
    out = np.empty_like(c)
    load().oracle_philox_raw(_p(c), len(c), int(key[0]), int(key[1]), _p(out))
    return out.reshape(np.shape(ctr))


def normal_slab(key, w2, n_rows, cols, w_row=None, w_col=None):
    """[n_rows, len(cols)]: (z * w_row[a]) * w_col[P] with z the Box-Muller
    normal of the block at counter (P, a, w2, 0) under key."""
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    wr = None if w_row is None else np.ascontiguousarray(w_row, dtype=np.float64)
    wc = None if w_col is None else np.ascontiguousarray(w_col, dtype=np.float64)
    out = np.empty((int(n_rows), len(cols)), dtype=np.float64)
    load().oracle_normal_slab(int(key[0]), int(key[1]), int(w2), int(n_rows), len(cols),
                              _p(cols), _p(wr), _p(wc), _p(out))
    return out
