"""Benchmark: exact sparse KNN join on one MI355X.

A step is one full join of every query of R against all of S (the whole hot
path: postings walk, score accumulation, per-query top-k), with S's inverted
index and both inputs already resident in device memory.  The default
workload is the medium one: |R| = 100,000, |S| = 1,000,000, D = 10,000,
nnz U[50,200], Zipf(1.1) feature ids, uint8 values, k = 10.

Prints one JSON line.  Extra keys beside the required ones:
  postings_entries_per_s, postings_GBps : posting entries walked per second and
      their algorithmic bytes (4 B per entry for uint8 data)
  roofline : dominant kernel (the tile join) against HBM peak
  cpu_baseline : the CPU oracle on a bounded query sample
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact KNN-join queries/s and postings GB/s vs HBM peak; learned vs plain IIIB"
HBM_PEAK_GBPS = 8000.0


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium")
    ap.add_argument("--algo", default="iib", choices=["iib", "iiib"])
    ap.add_argument("--bound", action="store_true", help="IIIB: bound-filtered completion")
    ap.add_argument("--drop", type=int, default=0, help="IIIB: level drop")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--k", type=int, default=0)
    ap.add_argument("--n-r", type=int, default=0, help="override |R| (quick runs only)")
    ap.add_argument("--n-s", type=int, default=0, help="override |S| (quick runs only)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--check", type=int, default=4, help="queries checked against the oracle after timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def _kernel_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1011_2807_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel_key: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    ent = tab.get(kernel_key)
    if not ent or ent.get("source_hash") != _kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def main():
    a = _args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md on sharding)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_MiB": a.copy_calibration}))
        return
    import synth
    import paper_1011_2807_amd as kj

    wl = synth.WORKLOADS[a.workload]
    k = a.k or wl["k"][-1]
    n_r = a.n_r or wl["n_r"]
    n_s = a.n_s or wl["n_s"]
    t0 = time.time()
    S = synth.make(a.workload, "S", n_rows=n_s)
    R = synth.make(a.workload, "R", n_rows=n_r)
    t_gen = time.time() - t0
    print("generated |S|=%d nnz=%d |R|=%d nnz=%d in %.1fs" % (S.n_rows, S.nnz, R.n_rows, R.nnz, t_gen),
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    torch.cuda.synchronize()
    tb = time.time()
    ix = kj.build_index(dS, tile_width=a.tile)
    torch.cuda.synchronize()
    t_build = time.time() - tb
    print("index built in %.3fs (T=%d, %d tiles)" % (t_build, ix.tile_width, ix.n_tiles), file=sys.stderr,
          flush=True)
    stream = torch.cuda.current_stream()
    sdt = torch.int32 if S.values.dtype == np.uint8 else torch.float32
    out = (torch.empty((n_r, k), dtype=torch.int32, device=dev), torch.empty((n_r, k), dtype=sdt, device=dev),
           torch.empty(n_r, dtype=torch.int32, device=dev))
    stats = torch.zeros(8, dtype=torch.int64, device=dev)
    # warmup (validated), also fills the counters
    for w in range(max(1, a.warmup)):
        kj.knn_join(ix, dR, k, algo=a.algo, stats=stats if w == 0 else None, validate=(w == 0), out=out,
                    bound_filter=a.bound, level_drop=a.drop)
        torch.cuda.synchronize()
        print("warmup %d done" % w, file=sys.stderr, flush=True)
    walked = int(stats[kj.STAT_POSTINGS].item())
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.time()
    ev0.record(stream)
    for s in range(a.steps):
        kj.knn_join(ix, dR, k, algo=a.algo, validate=False, out=out, stream=stream, bound_filter=a.bound,
                    level_drop=a.drop)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t_wall
    ms = ev0.elapsed_time(ev1) / a.steps
    print("timed %d steps: %.1f ms/step (wall %.2fs)" % (a.steps, ms, wall), file=sys.stderr, flush=True)
    qps = n_r / (ms / 1e3)
    entry_bytes = 4 if S.values.dtype == np.uint8 else 6
    eps = walked / (ms / 1e3)
    gbps = eps * entry_bytes / 1e9
    # dominant kernel: one launch per S tile; its average launch duration is the
    # step time over the launches (the only other launch per step is a tiny init)
    launches = ix.n_tiles
    avg_launch_ms = ms / launches
    bytes_per_launch = walked * entry_bytes / launches
    traffic = _traffic("k_iib_tile/%s/T%d" % (a.workload, ix.tile_width))
    roof = {"kernel": "k_iib_tile", "bound": "hbm", "achieved": round(bytes_per_launch / (avg_launch_ms / 1e3) / 1e9, 1),
            "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(bytes_per_launch / (avg_launch_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
            "traffic": traffic, "avg_launch_ms": round(avg_launch_ms, 4), "launches_per_step": launches,
            "algorithmic_bytes_per_launch": bytes_per_launch}

    # spot check against the oracle (not timed)
    import oracle
    ids, sc, cnt = [x.cpu().numpy() for x in out]
    rng = np.random.default_rng(0)
    rows = rng.choice(n_r, size=min(a.check, n_r), replace=False)
    tc = time.time()
    w_ids, w_sc, w_cnt = oracle.bf_topk_rows(R, S, k, rows)
    t_check = time.time() - tc
    ok = bool(np.array_equal(ids[rows], w_ids) and np.array_equal(cnt[rows], w_cnt) and
              (np.array_equal(sc[rows].astype(np.int64), w_sc) if sdt == torch.int32 else
               np.allclose(sc[rows], w_sc, rtol=1e-5)))
    cpu = None
    if not a.no_cpu:
        # oracle as it stands, single thread, on a bounded sample sized from the check's speed
        per_q = t_check / max(1, len(rows))
        n_cpu = int(max(1, min(n_r, a.cpu_seconds / max(per_q, 1e-6))))
        rows_cpu = rng.choice(n_r, size=n_cpu, replace=False)
        t1 = time.time()
        oracle.bf_topk_rows(R, S, k, rows_cpu)
        el = time.time() - t1
        cpu = {"value": round(n_cpu / el, 3), "unit": "queries/s", "cores": 1, "kind": "oracle",
               "sample": "%d random queries of the same workload, full S, single thread, %.1fs" % (n_cpu, el)}
    res = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8" if sdt == torch.int32 else "f32", "data": "synthetic",
        "config": {"workload": a.workload, "algo": a.algo, "bound_filter": a.bound, "level_drop": a.drop, "n_r": n_r, "n_s": n_s, "d": wl["d"], "k": k,
                   "tile_width": ix.tile_width, "nnz_s": S.nnz, "nnz_r": R.nnz},
        "iiib_counters": {"completion_entries": int(stats[kj.STAT_COMPLETION].item()),
                          "candidates": int(stats[kj.STAT_CANDIDATES].item())} if a.algo == "iiib" else None,
        "postings_entries_per_s": eps, "postings_GBps": round(gbps, 1), "postings_entries_per_step": walked,
        "index_build_s": round(t_build, 3), "oracle_spot_check": {"queries": len(rows), "exact": ok},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(res))
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
