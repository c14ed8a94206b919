"""Seeded synthetic sparse inputs for the KNN join (CSR, numpy arrays).

This module only draws input vectors; it contains none of the join's
arithmetic.  Both sides of every parity test (the CPU oracle and the HIP
library) and the benchmark take their inputs from here.

A sparse vector is a list of features (d, w), ascending d, w > 0 (Problem
definition, Sec. 3); ids here are 0-based.  The five workload recipes below
stand in for the paper's data (its synthetic distribution is not stated in
Sec. 5 and its Yeast/Worm spectra are not available):

* ``tiny``    |R|=1,000  |S|=10,000   D=10,000  nnz U[20,100], uniform ids, u8 U[1,255], k=10
* ``medium``  |R|=100,000 |S|=1,000,000 D=10,000 nnz U[50,200], Zipf(1.1) ids over a seeded
              permutation of the dimensions, u8 U[1,255], k=10
* ``batched`` |R|=1,000,000 nnz round(lognormal(ln 100, 0.8)) clipped to [10,1000];
              |S|=4,000,000 nnz U[50,300]; D=20,000; Zipf(1.1); u8; k=1 and k=10
* ``learned`` the ``medium`` generator with |S|=4,000,000; 200,000 training queries and
              1,000,000 evaluation queries; k=10
* ``fp32``    |R|=500,000 |S|=10,000,000 D=100,000 nnz U[30,300], Zipf(1.05),
              fp32 lognormal(0,1) values L2-normalised per vector, k=50

Seeds: base = 20101 + 100*c for workload number c (tiny=1 ... fp32=5); S uses
base+1, R base+2, the dimension permutation base+3; ``learned`` draws its
training queries with base+4 and evaluation queries with base+5, and its S
with the ``medium`` permutation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lock = threading.Lock()
_lib = None

NNZ_UNIFORM, NNZ_LOGNORMAL = 0, 1
FEAT_UNIFORM, FEAT_ZIPF = 0, 1
VAL_U8, VAL_F32 = 0, 1


def build(force: bool = False) -> str:
    """Compile gen.c into libsynth.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            lib.synth_row_nnz.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_double, ctypes.c_double, P]
            lib.synth_row_nnz.restype = None
            lib.synth_permutation.argtypes = [ctypes.c_uint64, ctypes.c_int32, P]
            lib.synth_permutation.restype = None
            lib.synth_fill_rows.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int,
                                            ctypes.c_double, P, ctypes.c_int, P, P, P]
            lib.synth_fill_rows.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class CSR:
    """Host CSR matrix: indptr int64[n+1], indices int32[nnz], values uint8|float32[nnz]."""
    indptr: np.ndarray
    indices: np.ndarray
    values: np.ndarray
    n_dims: int

    @property
    def n_rows(self) -> int:
        return int(self.indptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    @property
    def dtype(self) -> str:
        return "u8" if self.values.dtype == np.uint8 else "f32"

    def row(self, i: int):
        b, e = int(self.indptr[i]), int(self.indptr[i + 1])
        return self.indices[b:e], self.values[b:e]

    def take_rows(self, rows) -> "CSR":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.indptr[rows + 1] - self.indptr[rows]
        indptr = np.zeros(len(rows) + 1, dtype=np.int64)
        np.cumsum(lens, out=indptr[1:])
        idx = np.concatenate([np.arange(self.indptr[r], self.indptr[r + 1]) for r in rows]) if len(rows) else \
            np.zeros(0, dtype=np.int64)
        return CSR(indptr, self.indices[idx].copy(), self.values[idx].copy(), self.n_dims)


def permutation(seed: int, n: int) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.int32)
    lib.synth_permutation(seed, n, _ptr(out))
    return out


def draw(seed: int, n_rows: int, n_dims: int, nnz: tuple, features: str = "uniform", zipf_s: float = 1.1,
         perm: Optional[np.ndarray] = None, values: str = "u8", nnz_kind: str = "uniform",
         mu: float = 0.0, sigma: float = 1.0) -> CSR:
    """Draw n_rows sparse vectors.

    nnz=(lo, hi): uniform on [lo, hi] (nnz_kind="uniform") or
    round(exp(N(mu, sigma))) clipped to [lo, hi] (nnz_kind="lognormal").
    features: "uniform" (without replacement) or "zipf" (Zipf(zipf_s) ranks mapped
    through perm, distinct ids).  values: "u8" (U[1,255]) or "f32" (lognormal(0,1),
    L2-normalised per row, normalised in double then stored as float).
    """
    lib = _load()
    lo, hi = int(nnz[0]), int(nnz[1])
    assert 1 <= lo <= hi <= min(n_dims, 4096)
    lens = np.empty(n_rows, dtype=np.int64)
    lib.synth_row_nnz(seed, n_rows, NNZ_LOGNORMAL if nnz_kind == "lognormal" else NNZ_UNIFORM, lo, hi,
                      float(mu), float(sigma), _ptr(lens))
    indptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    nnz_total = int(indptr[-1])
    indices = np.empty(nnz_total, dtype=np.int32)
    if values == "u8":
        vals = np.empty(nnz_total, dtype=np.uint8)
        vu8, vf = vals, None
    else:
        vals = np.empty(nnz_total, dtype=np.float32)
        vu8, vf = None, vals
    fk = FEAT_ZIPF if features == "zipf" else FEAT_UNIFORM
    if fk == FEAT_ZIPF and perm is not None:
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        assert perm.shape[0] == n_dims
    rc = lib.synth_fill_rows(seed, n_rows, n_dims, _ptr(indptr), fk, float(zipf_s),
                             _ptr(perm) if fk == FEAT_ZIPF and perm is not None else None,
                             VAL_U8 if values == "u8" else VAL_F32, _ptr(indices), _ptr(vu8), _ptr(vf))
    if rc != 0:
        raise ValueError("synth_fill_rows failed")
    return CSR(indptr, indices, vals, n_dims)


# name -> (number, dict of recipe parameters)
WORKLOADS = {
    "tiny": dict(c=1, n_r=1_000, n_s=10_000, d=10_000, nnz_r=(20, 100), nnz_s=(20, 100), features="uniform",
                 zipf=None, values="u8", k=(10,)),
    "medium": dict(c=2, n_r=100_000, n_s=1_000_000, d=10_000, nnz_r=(50, 200), nnz_s=(50, 200), features="zipf",
                   zipf=1.1, values="u8", k=(10,)),
    "batched": dict(c=3, n_r=1_000_000, n_s=4_000_000, d=20_000, nnz_r=(10, 1000), nnz_s=(50, 300),
                    r_lognormal=(float(np.log(100.0)), 0.8), features="zipf", zipf=1.1, values="u8", k=(1, 10)),
    "learned": dict(c=4, n_r=1_000_000, n_train=200_000, n_s=4_000_000, d=10_000, nnz_r=(50, 200),
                    nnz_s=(50, 200), features="zipf", zipf=1.1, values="u8", k=(10,)),
    "fp32": dict(c=5, n_r=500_000, n_s=10_000_000, d=100_000, nnz_r=(30, 300), nnz_s=(30, 300), features="zipf",
                 zipf=1.05, values="f32", k=(50,)),
}


def base_seed(name: str) -> int:
    return 20101 + 100 * WORKLOADS[name]["c"]


def workload_perm(name: str) -> Optional[np.ndarray]:
    w = WORKLOADS[name]
    if w["features"] != "zipf":
        return None
    if name == "learned":  # drawn on the medium workload's permutation
        return permutation(base_seed("medium") + 3, WORKLOADS["medium"]["d"])
    return permutation(base_seed(name) + 3, w["d"])


def make(name: str, part: str, n_rows: Optional[int] = None, perm: Optional[np.ndarray] = None) -> CSR:
    """Draw part "S", "R", "R_train" or "R_eval" of a workload.

    n_rows overrides the row count (same distribution, a prefix-independent draw
    of that many rows: row i is identical for every n_rows > i).
    """
    w = WORKLOADS[name]
    base = base_seed(name)
    if perm is None:
        perm = workload_perm(name)
    if part == "S":
        seed, n, nnz, lognorm = base + 1, w["n_s"], w["nnz_s"], None
    elif part in ("R", "R_eval"):
        seed, n, nnz, lognorm = (base + 5 if name == "learned" else base + 2), w["n_r"], w["nnz_r"], \
            w.get("r_lognormal")
    elif part == "R_train":
        seed, n, nnz, lognorm = base + 4, w["n_train"], w["nnz_r"], None
    else:
        raise ValueError(part)
    if n_rows is not None:
        n = int(n_rows)
    kw = {}
    if lognorm is not None:
        kw = dict(nnz_kind="lognormal", mu=lognorm[0], sigma=lognorm[1])
    return draw(seed, n, w["d"], nnz, features=w["features"], zipf_s=w["zipf"] or 1.0, perm=perm,
                values=w["values"], **kw)
