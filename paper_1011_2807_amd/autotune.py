"""Autotuner for the join's launch parameters.

Times candidate settings on the device (HIP events around real joins of a
query sample) and keeps the fastest:

* tile width T (rows of S per tile: the LDS score array and the list split),
* for IIB, the dense head (0 = plain walk, or the number of longest-list
  dimensions kept as dense per-tile blocks) and, with a head, the S tiles per
  launch,
* schedule (one launch per tile, or the persistent work-queue launch),
* for IIIB, the level drop of the refined variant.

Results are cached in a JSON file keyed by the device architecture and a
signature of the workload (S size, dimensions, value type, k, algorithm,
query-sample cost), so a second call with the same signature does not time
anything.  Cache path: $KNNJ_TUNE_CACHE or ~/.cache/knnj/tune.json.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
from typing import Dict, Iterable, Optional

import torch

from . import knnj as kj

# candidates by value type: float32 score rows take twice the local memory, so
# narrower tiles and heads
DEFAULT_TILES = {"u8": (2048, 4096, 8192), "f32": (1024, 2048, 4096)}
DEFAULT_HEADS = {"u8": (0, 128, 192), "f32": (0, 64, 128)}
CACHE_VERSION = 4  # bumped when the candidate set changes


def _cache_path() -> str:
    return os.environ.get("KNNJ_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "knnj", "tune.json"))


def _load_cache() -> Dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(tab: Dict) -> None:
    p = _cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _arch() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def signature(S: kj.DeviceCSR, R_sample: kj.DeviceCSR, k: int, algo: str) -> str:
    nnz_s = int(S.indices.shape[0])
    nnz_r = int(R_sample.indices.shape[0])
    mean_r = nnz_r / max(1, R_sample.n_rows)
    return "v%d|%s|S%d|nnz%d|D%d|%s|k%d|%s|r%.0f" % (CACHE_VERSION, _arch(), S.n_rows, int(math.log2(max(1, nnz_s))),
                                                     S.n_dims, "u8" if S.dtype == kj.KNNJ_U8 else "f32", k, algo,
                                                     mean_r)


def candidates_key(tiles, heads, drops, tiles_per_launch) -> str:
    """Short stable name of a candidate set (part of the cache key)."""
    text = json.dumps([sorted(int(x) for x in c) for c in (tiles, heads, drops, tiles_per_launch)])
    return "c" + hashlib.sha256(text.encode()).hexdigest()[:12]


def _time(fn, reps: int = 2) -> float:
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(S: kj.DeviceCSR, R_sample: kj.DeviceCSR, k: int, algo: str = "iib", tiles: Optional[Iterable[int]] = None,
         drops: Iterable[int] = (0, 4, 8, 12, 16, 24), heads: Optional[Iterable[int]] = None,
         tiles_per_launch: Iterable[int] = (2, 4, 8), use_cache: bool = True, verbose: bool = False) -> Dict:
    """Fastest settings for joining queries like R_sample against S.

    Returns {"tile_width", "dense_head", "tiles_per_launch", "persistent",
    "level_drop", "ms", "timings"}; the index must then be built with
    tile_width and dense_head.
    R_sample should hold a few thousand queries drawn like the real ones.
    """
    vt = "u8" if S.dtype == kj.KNNJ_U8 else "f32"
    tiles = DEFAULT_TILES[vt] if tiles is None else tuple(tiles)
    heads = DEFAULT_HEADS[vt] if heads is None else tuple(heads)
    drops, tiles_per_launch = tuple(drops), tuple(tiles_per_launch)
    # the candidate set is part of the key: a cached choice is only reused for the same candidates
    key = signature(S, R_sample, k, algo) + "|" + candidates_key(tiles, heads, drops, tiles_per_launch)
    tab = _load_cache() if use_cache else {}
    if key in tab:
        return tab[key]
    timings = []
    best = None
    out = (torch.empty((R_sample.n_rows, k), dtype=torch.int32, device="cuda"),
           torch.empty((R_sample.n_rows, k), dtype=torch.int32 if S.dtype == kj.KNNJ_U8 else torch.float32,
                       device="cuda"),
           torch.empty(R_sample.n_rows, dtype=torch.int32, device="cuda"))
    hs = heads if algo == "iib" else (0,)
    for t in tiles:
        for h in hs:
            try:
                ix = kj.build_index(S, tile_width=t, dense_head=h)
            except kj.KnnjError:
                continue
            if algo == "iiib":
                cands = [dict(bound_filter=True, level_drop=d) for d in drops]
            elif h:
                cands = [dict(tiles_per_launch=g) for g in tiles_per_launch]
            else:
                cands = [dict(persistent=False), dict(persistent=True)]
            for c in cands:
                try:
                    ms = _time(lambda: kj.knn_join(ix, R_sample, k, algo=algo, validate=False, out=out, **c))
                except kj.KnnjError:
                    continue
                rec = {"tile_width": t, "dense_head": h, "ms": round(ms, 3), **c}
                timings.append(rec)
                if verbose:
                    print("autotune", rec, flush=True)
                if best is None or ms < best["ms"]:
                    best = rec
            ix.free()
    if best is None:
        raise RuntimeError("autotune: no candidate ran")
    res = {"tile_width": best["tile_width"], "dense_head": int(best.get("dense_head", 0)),
           "tiles_per_launch": int(best.get("tiles_per_launch", 0)),
           "persistent": bool(best.get("persistent", False)),
           "level_drop": int(best.get("level_drop", 0)), "bound_filter": bool(best.get("bound_filter", False)),
           "ms": best["ms"], "timings": timings, "signature": key}
    if use_cache:
        tab = _load_cache()
        tab[key] = res
        _store_cache(tab)
    return res
