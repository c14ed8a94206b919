"""CPU oracle for the exact sparse KNN join.  TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never calls it
and shares no code with it; the two meet only in the seeded inputs drawn by
the ``synth`` package.

* ``bf_topk`` -- the plain definition of the join (Sec. 3, Eq. 1) by brute
  force (Sec. 4.2, Algorithm 2), in single-threaded C (``knnj_oracle.c``):
  every pair's dot product by the two-pointer merge, neighbours are the pairs
  with score > 0 ordered by (score desc, id asc), first k kept, padding
  (-1, 0).  u8 inputs give exact int64 scores; f32 inputs give float64 scores
  (products of fp32 values widened to double, summed in ascending dimension
  order).
* ``models`` -- slow pure-Python walks of Algorithms 1-4 in the paper's
  order, used only to pin readings of the paper on small inputs.
* ``mlp`` -- float64 reference of the threshold-predicting MLP.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knnj_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile knnj_oracle.c with gcc (single-threaded, no OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            lib.oracle_bf_topk.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, ctypes.c_int64, P, P, P,
                                           ctypes.c_int, ctypes.c_int32, P, P, P]
            lib.oracle_bf_topk.restype = ctypes.c_int
            lib.oracle_scores_one.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int64, P, P, P, ctypes.c_int, P]
            lib.oracle_scores_one.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _arrays(m):
    indptr = np.ascontiguousarray(m.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(m.indices, dtype=np.int32)
    values = np.ascontiguousarray(m.values)
    if values.dtype not in (np.uint8, np.float32):
        raise TypeError("values must be uint8 or float32")
    return indptr, indices, values


def bf_topk(R, S, k: int, q_begin: int = 0, q_end=None):
    """Exact top-k of queries R[q_begin:q_end] against S.

    R, S: objects with indptr/indices/values (e.g. ``synth.CSR``), same value dtype.
    Returns (ids int32[n,k], scores int64|float64[n,k], count int32[n]).
    """
    lib = _load()
    rp, ri, rv = _arrays(R)
    sp, si, sv = _arrays(S)
    if rv.dtype != sv.dtype:
        raise TypeError("R and S value dtypes differ")
    dtype = 0 if rv.dtype == np.uint8 else 1
    n_r = rp.shape[0] - 1
    q_end = n_r if q_end is None else int(q_end)
    n = q_end - int(q_begin)
    ids = np.empty((n, k), dtype=np.int32)
    scores = np.empty((n, k), dtype=np.int64 if dtype == 0 else np.float64)
    count = np.empty(n, dtype=np.int32)
    rc = lib.oracle_bf_topk(int(q_begin), q_end, _p(rp), _p(ri), _p(rv), sp.shape[0] - 1, _p(sp), _p(si), _p(sv),
                            dtype, int(k), _p(ids), _p(scores), _p(count))
    if rc != 0:
        raise RuntimeError("oracle_bf_topk failed: %d" % rc)
    return ids, scores, count


def bf_topk_rows(R, S, k: int, rows):
    """Exact top-k for an arbitrary list of query rows (sampled checks)."""
    rows = np.asarray(rows, dtype=np.int64)
    ids = np.empty((len(rows), k), dtype=np.int32)
    count = np.empty(len(rows), dtype=np.int32)
    scores = None
    for i, q in enumerate(rows):
        a, b, c = bf_topk(R, S, k, int(q), int(q) + 1)
        if scores is None:
            scores = np.empty((len(rows), k), dtype=b.dtype)
        ids[i], scores[i], count[i] = a[0], b[0], c[0]
    if scores is None:
        scores = np.empty((0, k), dtype=np.int64)
    return ids, scores, count


def scores_one(R, S, q: int) -> np.ndarray:
    """dot(r_q, s_j) for every j (int64 for u8 inputs, float64 for f32)."""
    lib = _load()
    rp, ri, rv = _arrays(R)
    sp, si, sv = _arrays(S)
    dtype = 0 if rv.dtype == np.uint8 else 1
    out = np.empty(sp.shape[0] - 1, dtype=np.int64 if dtype == 0 else np.float64)
    rc = lib.oracle_scores_one(int(q), _p(rp), _p(ri), _p(rv), sp.shape[0] - 1, _p(sp), _p(si), _p(sv), dtype,
                               _p(out))
    if rc != 0:
        raise RuntimeError("oracle_scores_one failed")
    return out


def postings_walked(R, S) -> int:
    """Second term of Eq. 4: sum over r in R, d in r of |I_d| (IIB's postings walk)."""
    col = np.bincount(np.asarray(S.indices, dtype=np.int64), minlength=int(S.n_dims))
    return int(col[np.asarray(R.indices, dtype=np.int64)].sum())
