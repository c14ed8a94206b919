"""Python binding of libknnj.so (ctypes).  Argument marshalling only.

Every step of the join runs in the library's HIP kernels; PyTorch supplies
device memory and the current stream.  The binding fails loudly when the
library is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libknnj.so")

KNNJ_OK, KNNJ_EINVAL, KNNJ_ENOMEM, KNNJ_EDEVICE, KNNJ_EOVERFLOW, KNNJ_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
KNNJ_U8, KNNJ_F32 = 0, 1
KNNJ_IIB, KNNJ_IIIB = 0, 1
KNNJ_FLAG_NO_VALIDATE = 1
KNNJ_FLAG_IIIB_BOUND = 2
KNNJ_FLAG_PERSISTENT = 4
KNNJ_FLAG_NO_DENSE_HEAD = 8
STAT_POSTINGS, STAT_COMPLETION, STAT_CANDIDATES, STAT_FALLBACKS, STAT_COUNT = 0, 1, 2, 3, 8
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "EUNSUPPORTED"}


class KnnjError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("knnj %s: %s" % (_STATUS.get(code, str(code)), msg))
        self.code = code


class _CSR(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_dims", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("values", ctypes.c_void_p)]


class _IndexOpts(ctypes.Structure):
    _fields_ = [("tile_width", ctypes.c_int32), ("dense_head", ctypes.c_int32), ("reserved", ctypes.c_int32 * 6)]


class _JoinOpts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("flags", ctypes.c_uint32), ("r_block_rows", ctypes.c_int64),
                ("theta_seed", ctypes.c_void_p), ("stats", ctypes.c_void_p), ("fallback_out", ctypes.c_void_p),
                ("level_drop", ctypes.c_int32), ("r_max_row_nnz", ctypes.c_int32),
                ("tiles_per_launch", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class _BlockStats(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("copy_ms", ctypes.c_double), ("build_ms", ctypes.c_double),
                ("join_ms", ctypes.c_double), ("merge_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class _IndexInfo(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_dims", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("tile_width", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("max_row_nnz", ctypes.c_int32), ("dense_head", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libknnj.so and declare its C signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libknnj.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.knnj_build_index.argtypes = [ctypes.POINTER(_CSR), ctypes.POINTER(_IndexOpts), P, ctypes.POINTER(P)]
    lib.knnj_build_index.restype = I32
    lib.knnj_index_info_get.argtypes = [P, ctypes.POINTER(_IndexInfo)]
    lib.knnj_index_info_get.restype = I32
    lib.knnj_index_list_lengths.argtypes = [P, P, P]
    lib.knnj_index_list_lengths.restype = I32
    lib.knnj_index_free.argtypes = [P]
    lib.knnj_index_free.restype = None
    lib.knnj_join.argtypes = [P, ctypes.POINTER(_CSR), I32, ctypes.POINTER(_JoinOpts), P, P, P, P]
    lib.knnj_join.restype = I32
    lib.knnj_join_bf.argtypes = [ctypes.POINTER(_CSR), ctypes.POINTER(_CSR), I32, P, P, P, P]
    lib.knnj_join_bf.restype = I32
    lib.knnj_join_blocked.argtypes = [ctypes.POINTER(_CSR), I64, ctypes.POINTER(_IndexOpts), ctypes.POINTER(_CSR),
                                      I32, ctypes.POINTER(_JoinOpts), P, P, P, ctypes.POINTER(_BlockStats), P]
    lib.knnj_join_blocked.restype = I32
    lib.knnj_last_error.argtypes = []
    lib.knnj_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != KNNJ_OK:
        raise KnnjError(rc, _lib.knnj_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _require(t: Optional[torch.Tensor], name: str, dtype: torch.dtype, numel: int, at_least: bool = False):
    """Check a device array handed to the library: dtype, contiguity, the
    current device, and size (the kernels write exactly what the sizes say)."""
    if t is None:
        return
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (name, dtype))
    if t.device.type != "cuda" or t.device.index != torch.cuda.current_device():
        raise ValueError("%s must be on the current HIP device" % name)
    if (t.numel() < numel) if at_least else (t.numel() != numel):
        raise ValueError("%s has %d elements, %s %d" % (name, t.numel(), "needs at least" if at_least else "needs",
                                                         numel))


@dataclass
class DeviceCSR:
    """CSR matrix in device memory (torch tensors)."""
    indptr: torch.Tensor   # int64[n+1]
    indices: torch.Tensor  # int32[nnz]
    values: torch.Tensor   # uint8 or float32[nnz]
    n_dims: int

    @staticmethod
    def from_host(m, device="cuda") -> "DeviceCSR":
        """Copy a host CSR (numpy arrays indptr/indices/values, attribute n_dims)."""
        return DeviceCSR(torch.from_numpy(np.ascontiguousarray(m.indptr, dtype=np.int64)).to(device),
                         torch.from_numpy(np.ascontiguousarray(m.indices, dtype=np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(m.values)).to(device), int(m.n_dims))

    @property
    def n_rows(self) -> int:
        return int(self.indptr.shape[0]) - 1

    @property
    def dtype(self) -> int:
        return KNNJ_U8 if self.values.dtype == torch.uint8 else KNNJ_F32

    def _c(self) -> _CSR:
        if self.values.dtype not in (torch.uint8, torch.float32):
            raise TypeError("CSR values must be a uint8 or float32 device tensor")
        nnz = int(self.indices.numel())
        _require(self.indptr, "indptr", torch.int64, self.indptr.numel())
        _require(self.indices, "indices", torch.int32, nnz)
        _require(self.values, "values", self.values.dtype, nnz)
        if self.indptr.dim() != 1 or self.indptr.numel() < 1:
            raise ValueError("indptr must be a 1-d tensor of n_rows + 1 offsets")
        return _CSR(self.n_rows, self.n_dims, self.dtype, int(self.indices.shape[0]), _ptr(self.indptr),
                    _ptr(self.indices), _ptr(self.values))


class Index:
    """Inverted index of S (owned by the library; freed with the object)."""

    def __init__(self, handle: ctypes.c_void_p, S: DeviceCSR):
        self._h = handle
        self.n_dims = S.n_dims
        self.dtype = S.dtype
        info = _IndexInfo()
        _check(_lib.knnj_index_info_get(self._h, ctypes.byref(info)))
        self.info = info

    @property
    def n_rows(self) -> int:
        return int(self.info.n_rows)

    @property
    def tile_width(self) -> int:
        return int(self.info.tile_width)

    @property
    def n_tiles(self) -> int:
        return int(self.info.n_tiles)

    @property
    def dense_head(self) -> int:
        return int(self.info.dense_head)

    def list_lengths(self, stream=None) -> torch.Tensor:
        """|I_d| for every dimension (device int32)."""
        out = torch.empty(self.n_dims, dtype=torch.int32, device="cuda")
        _check(_lib.knnj_index_list_lengths(self._h, _ptr(out), _stream(stream)))
        return out

    def free(self):
        if self._h is not None and _lib is not None:
            _lib.knnj_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_index(S: DeviceCSR, tile_width: int = 0, dense_head: int = 0, stream=None) -> Index:
    """dense_head: keep that many (64, 128, 192 or 256) longest-list
    dimensions as dense per-tile blocks for the IIB join (0 = off)."""
    lib = load_library()
    h = ctypes.c_void_p()
    opts = _IndexOpts(int(tile_width), int(dense_head))
    c = S._c()
    _check(lib.knnj_build_index(ctypes.byref(c), ctypes.byref(opts), _stream(stream), ctypes.byref(h)))
    return Index(h, S)


def _outputs(n: int, k: int, dtype: int, out):
    sdt = torch.int32 if dtype == KNNJ_U8 else torch.float32
    if out is not None:
        ids, sc, cnt = out
        _require(ids, "out ids", torch.int32, n * k)
        _require(sc, "out scores", sdt, n * k)
        _require(cnt, "out count", torch.int32, n)
        return out
    return (torch.empty((n, k), dtype=torch.int32, device="cuda"), torch.empty((n, k), dtype=sdt, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda"))


def knn_join(index: Index, R: DeviceCSR, k: int, algo: str = "iib", r_block_rows: int = 0,
             theta_seed: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None,
             fallback_out: Optional[torch.Tensor] = None, validate: bool = True, bound_filter: bool = False,
             level_drop: int = 0, persistent: bool = False, r_max_row_nnz: int = 0, dense_head: bool = True,
             tiles_per_launch: int = 0, out=None, stream=None):
    """Exact top-k of every row of R against the indexed S.

    Returns (ids int32[n,k], scores int32|float32[n,k], count int32[n]) on the device.
    algo: "iib" or "iiib".  theta_seed: optional float32[n] device tensor of
    k-th score guesses (IIIB).  stats: optional int64[8] device tensor of
    counters (added to).  fallback_out: optional uint8[n] device tensor.
    bound_filter / level_drop: IIIB refinements (see knnj.h); results stay exact.
    persistent: one persistent launch per S tile with a device work queue (IIB).
    dense_head: use the index's dense head if it has one (IIB); False walks every list.
    tiles_per_launch: S tiles per launch of the dense-head join (0 = default).
    """
    lib = load_library()
    ids, sc, cnt = _outputs(R.n_rows, k, index.dtype, out)
    o = _JoinOpts()
    o.algo = KNNJ_IIIB if algo == "iiib" else KNNJ_IIB
    o.flags = ((0 if validate else KNNJ_FLAG_NO_VALIDATE) | (KNNJ_FLAG_IIIB_BOUND if bound_filter else 0) |
               (KNNJ_FLAG_PERSISTENT if persistent else 0) | (0 if dense_head else KNNJ_FLAG_NO_DENSE_HEAD))
    o.level_drop = int(level_drop)
    o.r_max_row_nnz = int(r_max_row_nnz)
    o.r_block_rows = int(r_block_rows)
    o.tiles_per_launch = int(tiles_per_launch)
    _require(theta_seed, "theta_seed", torch.float32, R.n_rows)
    _require(stats, "stats", torch.int64, STAT_COUNT, at_least=True)
    _require(fallback_out, "fallback_out", torch.uint8, R.n_rows)
    o.theta_seed = _ptr(theta_seed)
    o.stats = _ptr(stats)
    o.fallback_out = _ptr(fallback_out)
    c = R._c()
    _check(lib.knnj_join(index._h, ctypes.byref(c), int(k), ctypes.byref(o), _ptr(ids), _ptr(sc), _ptr(cnt),
                         _stream(stream)))
    return ids, sc, cnt


class HostCSR:
    """CSR matrix in host memory for the blocked join.  pin=True copies it into
    page-locked memory (torch pin_memory), so block copies run asynchronously."""

    def __init__(self, m, pin: bool = True):
        arrs = []
        for a, dt in ((m.indptr, torch.int64), (m.indices, torch.int32), (m.values, None)):
            t = torch.as_tensor(np.ascontiguousarray(a)) if isinstance(a, np.ndarray) else a
            if t.device.type != "cpu" or not t.is_contiguous() or (dt is not None and t.dtype != dt):
                raise TypeError("HostCSR arrays must be contiguous host arrays (indptr int64, indices int32)")
            arrs.append(t.pin_memory() if pin and not t.is_pinned() else t)
        self.indptr, self.indices, self.values = arrs
        if self.values.dtype not in (torch.uint8, torch.float32):
            raise TypeError("HostCSR values must be uint8 or float32")
        if self.indices.numel() != self.values.numel() or self.indptr.dim() != 1 or self.indptr.numel() < 1:
            raise ValueError("HostCSR: indptr must be 1-d with n_rows + 1 entries; indices and values of one size")
        self.n_dims = int(m.n_dims)

    @property
    def n_rows(self) -> int:
        return int(self.indptr.numel()) - 1

    def _c(self) -> _CSR:
        return _CSR(self.n_rows, self.n_dims, KNNJ_U8 if self.values.dtype == torch.uint8 else KNNJ_F32,
                    int(self.indices.numel()), _ptr(self.indptr), _ptr(self.indices), _ptr(self.values))


def knn_join_blocked(S: HostCSR, R: DeviceCSR, k: int, block_rows: int, tile_width: int = 0, dense_head: int = 0,
                     algo: str = "iib", bound_filter: bool = False, level_drop: int = 0, validate: bool = True,
                     stats: Optional[torch.Tensor] = None, out=None, stream=None):
    """Block nested loop with S in host memory (see knnj.h): S is copied to the
    device block_rows rows at a time, each block indexed (tile_width,
    dense_head) and joined; the result equals knn_join on all of S.
    Returns (ids, scores, count, phase times in ms)."""
    lib = load_library()
    if not isinstance(S, HostCSR):
        raise TypeError("S must be a HostCSR")
    ids, sc, cnt = _outputs(R.n_rows, k, KNNJ_U8 if S.values.dtype == torch.uint8 else KNNJ_F32, out)
    _require(stats, "stats", torch.int64, STAT_COUNT, at_least=True)
    io = _IndexOpts(int(tile_width), int(dense_head))
    o = _JoinOpts()
    o.algo = KNNJ_IIIB if algo == "iiib" else KNNJ_IIB
    o.flags = (0 if validate else KNNJ_FLAG_NO_VALIDATE) | (KNNJ_FLAG_IIIB_BOUND if bound_filter else 0)
    o.level_drop = int(level_drop)
    o.stats = _ptr(stats)
    bs = _BlockStats()
    cs, cr = S._c(), R._c()
    _check(lib.knnj_join_blocked(ctypes.byref(cs), int(block_rows), ctypes.byref(io), ctypes.byref(cr), int(k),
                                 ctypes.byref(o), _ptr(ids), _ptr(sc), _ptr(cnt), ctypes.byref(bs), _stream(stream)))
    times = {f: getattr(bs, f) for f, _ in _BlockStats._fields_}
    times["n_blocks"] = int(times["n_blocks"])
    return ids, sc, cnt, times


def knn_join_bf(S: DeviceCSR, R: DeviceCSR, k: int, out=None, stream=None):
    """Brute-force join (Algorithm 2); same outputs as knn_join."""
    lib = load_library()
    ids, sc, cnt = _outputs(R.n_rows, k, S.dtype, out)
    cs, cr = S._c(), R._c()
    _check(lib.knnj_join_bf(ctypes.byref(cs), ctypes.byref(cr), int(k), _ptr(ids), _ptr(sc), _ptr(cnt),
                            _stream(stream)))
    return ids, sc, cnt


# ---------------------------------------------------------------- learned seed
MLP_FEATURES, MLP_PARAMS, MLP_NORM = 64, 24961, 129


class _TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("tau", ctypes.c_float), ("seed", ctypes.c_uint64), ("reserved", ctypes.c_int32 * 8)]


def _load_mlp(lib):
    if getattr(lib, "_mlp_ready", False):
        return lib
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.knnj_mlp_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(P)]
    lib.knnj_mlp_create.restype = I32
    lib.knnj_mlp_free.argtypes = [P]
    lib.knnj_mlp_free.restype = None
    lib.knnj_mlp_features.argtypes = [P, ctypes.POINTER(_CSR), P, P]
    lib.knnj_mlp_features.restype = I32
    lib.knnj_mlp_train.argtypes = [P, P, P, I64, ctypes.POINTER(_TrainOpts), P, P]
    lib.knnj_mlp_train.restype = I32
    lib.knnj_mlp_predict.argtypes = [P, P, I64, P, P]
    lib.knnj_mlp_predict.restype = I32
    lib.knnj_mlp_grad.argtypes = [P, P, P, I64, ctypes.c_float, P, P, P]
    lib.knnj_mlp_grad.restype = I32
    lib.knnj_mlp_get_state.argtypes = [P, P, P]
    lib.knnj_mlp_get_state.restype = I32
    lib.knnj_mlp_set_state.argtypes = [P, P, P]
    lib.knnj_mlp_set_state.restype = I32
    lib._mlp_ready = True
    return lib


def _check_xy(X: torch.Tensor, y: Optional[torch.Tensor] = None):
    if X.dim() != 2 or X.shape[1] != MLP_FEATURES:
        raise ValueError("X must be [n, %d]" % MLP_FEATURES)
    _require(X, "X", torch.float32, X.numel())
    _require(y, "y", torch.float32, X.shape[0])


class Mlp:
    """Threshold-predicting MLP (64-128-128-1, bfloat16 weights) held by the library."""

    def __init__(self, seed: int = 0):
        self._lib = _load_mlp(load_library())
        h = ctypes.c_void_p()
        _check(self._lib.knnj_mlp_create(ctypes.c_uint64(seed), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def features(index: Index, R: DeviceCSR, stream=None) -> torch.Tensor:
        lib = _load_mlp(load_library())
        out = torch.empty((R.n_rows, MLP_FEATURES), dtype=torch.float32, device="cuda")
        c = R._c()
        _check(lib.knnj_mlp_features(index._h, ctypes.byref(c), _ptr(out), _stream(stream)))
        return out

    def train(self, X: torch.Tensor, y: torch.Tensor, epochs: int = 20, batch: int = 1024, lr: float = 1e-3,
              tau: float = 0.05, seed: int = 0, stream=None):
        _check_xy(X, y)
        o = _TrainOpts(int(epochs), int(batch), float(lr), float(tau), int(seed))
        losses = (ctypes.c_float * int(epochs))()
        _check(self._lib.knnj_mlp_train(self._h, _ptr(X), _ptr(y), int(X.shape[0]), ctypes.byref(o), losses,
                                        _stream(stream)))
        return list(losses)

    def predict(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        _check_xy(X)
        out = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        _check(self._lib.knnj_mlp_predict(self._h, _ptr(X), int(X.shape[0]), _ptr(out), _stream(stream)))
        return out

    def grad(self, X: torch.Tensor, y: torch.Tensor, tau: float, stream=None):
        _check_xy(X, y)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(self._lib.knnj_mlp_grad(self._h, _ptr(X), _ptr(y), int(X.shape[0]), float(tau), _ptr(g), _ptr(loss),
                                       _stream(stream)))
        return g, loss

    def get_state(self):
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        nrm = np.empty(MLP_NORM, dtype=np.float32)
        _check(self._lib.knnj_mlp_get_state(self._h, ctypes.c_void_p(p.ctypes.data), ctypes.c_void_p(nrm.ctypes.data)))
        return p, nrm

    def set_state(self, params: np.ndarray, norm: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        nrm = np.ascontiguousarray(norm, dtype=np.float32)
        if p.shape != (MLP_PARAMS,) or nrm.shape != (MLP_NORM,):
            raise ValueError("params must be [%d] and norm [%d]" % (MLP_PARAMS, MLP_NORM))
        _check(self._lib.knnj_mlp_set_state(self._h, ctypes.c_void_p(p.ctypes.data), ctypes.c_void_p(nrm.ctypes.data)))

    def free(self):
        if self._h is not None:
            self._lib.knnj_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
