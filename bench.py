"""Benchmark: exact sparse KNN join on one MI355X.

A step is one full join of every query of R against all of S (the whole hot
path: postings walk, score accumulation, per-query top-k), with S's inverted
index and both inputs already resident in device memory.  The default
workload is the medium one: |R| = 100,000, |S| = 1,000,000, D = 10,000,
nnz U[50,200], Zipf(1.1) feature ids, uint8 values, k = 10.

The headline `value` is the IIB join (Algorithm 3) on uint8 data with a dense
head: the 128 dimensions with the longest lists are kept as dense per-tile byte
blocks, scored with byte dot products, and only the other lists are walked
(exact; --dense-head 0 gives the plain list walk).  Beside it, on the same
queries and each checked identical to the headline output:
  iib_plain_walk  the same index walked list by list
  iiib.plain    Algorithm 4 as printed (split at the running threshold, every
                candidate completed)
  iiib.refined  the same plus the bound-filtered completion and a level drop
                picked by the autotuner on a query sample (beyond the paper;
                still exact)
  iiib.learned  iiib.refined seeded by the MLP's predicted k-th score (features
                + prediction + join timed together); miss rate = share of
                queries whose seed was too high and that were re-run
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact KNN-join queries/s and postings GB/s vs HBM peak; learned vs plain IIIB"
HBM_PEAK_GBPS = 8000.0
LDS_ATOMIC_PEAK = 256 * 2.4e9 * 16
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--k", type=int, default=0)
    ap.add_argument("--n-r", type=int, default=0, help="override |R| (quick runs only)")
    ap.add_argument("--n-s", type=int, default=0, help="override |S| (quick runs only)")
    ap.add_argument("--n-train", type=int, default=0, help="training queries of the learned seed")
    ap.add_argument("--no-iiib", action="store_true", help="skip the IIIB / learned-seed legs")
    ap.add_argument("--persistent", action="store_true", help="IIB: persistent per-tile launches with a work queue")
    ap.add_argument("--dense-head", type=int, default=-1,
                    help="dimensions kept as dense per-tile blocks (-1 = 128 for u8, 64 for f32; 0 = plain walk)")
    ap.add_argument("--tiles-per-launch", type=int, default=4, help="dense-head join: S tiles per launch")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--check", type=int, default=4, help="queries checked against the oracle after timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--print-kernel-hash", action="store_true")
    ap.add_argument("--sweep", choices=sorted(SWEEPS), default=None,
                    help="run one of the paper's experiment sweeps on synthetic data (one JSON line per point)")
    return ap.parse_args()


# The paper's experiment sweeps (Sec. 5) on synthetic stand-ins.  data_size and
# relative_size use the paper's own synthetic setting (10,000 dimensions; here
# the small workload's generator: uniform feature ids, nnz U[20,100], uint8
# values); k uses the sizes of the paper's Yeast (R) and Worm (S) spectra sets
# with the medium workload's skewed generator in place of the spectra.  k = 5 is
# the paper's default.  Every point times BF, IIB (list walk and dense head) and
# IIIB (as printed and refined) on the same queries.
SWEEPS = {
    # Fig. 1: data size, |R| = |S| = n
    "data_size": dict(figure="Fig. 1", gen="tiny",
                      points=[dict(n_r=n, n_s=n, k=5) for n in (10_000, 20_000, 30_000, 40_000, 50_000)]),
    # Fig. 2: relative size, |R| = 10,000 and |S| from 1,000 to 100,000 (R:S from 10:1 to 1:10)
    "relative_size": dict(figure="Fig. 2", gen="tiny",
                          points=[dict(n_r=10_000, n_s=n, k=5)
                                  for n in (1_000, 2_000, 5_000, 10_000, 20_000, 50_000, 100_000)]),
    # Fig. 3: k from 5 to 20, |R| = 35,236 and |S| = 207,804
    "k": dict(figure="Fig. 3", gen="medium", points=[dict(n_r=35_236, n_s=207_804, k=k) for k in (5, 10, 15, 20)]),
    # Fig. 4: buffer size.  The medium workload with S left in host memory and
    # read in blocks of 10% to 50% of its rows (the blocked join), beside the
    # join of an index of all of S in device memory
    "buffer": dict(figure="Fig. 4", gen="medium",
                   points=[dict(n_r=100_000, n_s=1_000_000, k=10, block_frac=f) for f in (0.1, 0.2, 0.3, 0.5)]),
}


KERNEL_SOURCES = ("common.hpp", "select.hpp", "walk.hpp", "join.hip", "head.hip")


def _strip_comments(src: str) -> str:
    """C++ source without comments and blank-space runs (so a comment edit does
    not count as a kernel change)."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def _kernel_hash() -> str:
    """Hash of the code (comments stripped) the IIB tile kernels are built from."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1011_2807_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(_strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def _counters(kernel_key: str):
    """Per-launch figures of a kernel from committed rocprofv3 counter runs
    (HBM bytes, VALU instructions), if they were taken on the current kernel
    sources; else {}."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        tab = json.load(f)
    ent = tab.get(kernel_key)
    if not ent or ent.get("source_hash") != _kernel_hash():
        return {}
    return ent


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline_leg(R, S, k, gpu_out, n_check, cpu_seconds, f32):
    """The cpu_baseline leg, the only place this script runs the oracle: the
    oracle as it stands (one thread) on random queries of the workload, against
    all of S, outside the timed region.  Its first n_check rows double as a
    spot check of the GPU result gpu_out (ids, scores, counts; u8 bit-exact,
    f32 counts equal and scores within 1e-5 relative); when cpu_seconds > 0 a
    further sample sized to about that much CPU time follows.  The rate over
    every row it ran is the reported baseline.  Returns (check, baseline)."""
    import oracle
    n_r = R.n_rows
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(n_r, size=max(1, min(n_check, n_r)), replace=False))
    ids, sc, cnt = [x.cpu().numpy() for x in gpu_out]
    t0 = time.time()
    w_ids, w_sc, w_cnt = oracle.bf_topk_rows(R, S, k, rows)
    el = time.time() - t0
    if not f32:
        ok = bool(np.array_equal(ids[rows], w_ids) and np.array_equal(cnt[rows], w_cnt) and
                  np.array_equal(sc[rows].astype(np.int64), w_sc))
    else:
        # float scores within 1e-5 of the fp64 oracle; ids may differ only on near-ties
        ok = bool(np.array_equal(cnt[rows], w_cnt) and np.allclose(sc[rows], w_sc, rtol=1e-5, atol=0))
    n_done = len(rows)
    if cpu_seconds > 0:
        per_q = el / n_done
        n_more = int(max(1, min(n_r, cpu_seconds / max(per_q, 1e-6))))
        more = rng.choice(n_r, size=n_more, replace=False)
        t1 = time.time()
        oracle.bf_topk_rows(R, S, k, more)
        el += time.time() - t1
        n_done += n_more
    cpu = {"value": round(n_done / el, 3), "unit": "queries/s", "cores": 1, "kind": "oracle",
           "sample": "%d random queries of the same workload against all of S, one thread, %.1fs"
                     " (the first %d also check the GPU result)" % (n_done, el, len(rows))}
    return {"queries": len(rows), "exact": ok}, cpu


def main():
    a = _args()
    if a.print_kernel_hash:
        print(_kernel_hash())
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the join has no multi-GPU path, so --gpus must be 1",
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

    if a.sweep:
        return run_sweep(a)
    if a.workload == "batched":
        return run_batched(a)
    wl = synth.WORKLOADS[a.workload]
    k = a.k or wl["k"][-1]
    n_r = a.n_r or wl["n_r"]
    n_s = a.n_s or wl["n_s"]
    n_train = a.n_train or wl.get("n_train", 20_000)
    t0 = time.time()
    perm = synth.workload_perm(a.workload)
    S = synth.make(a.workload, "S", n_rows=n_s, perm=perm)
    R = synth.make(a.workload, "R", n_rows=n_r, perm=perm)
    # training queries for the learned seed: the learned workload's own split, or
    # (other workloads) the same generator as R drawn with the learned workload's
    # training seed
    R_train = None
    if not a.no_iiib:
        if "n_train" in wl:
            R_train = synth.make(a.workload, "R_train", n_rows=n_train, perm=perm)
        else:
            kw = {}
            if wl.get("r_lognormal"):
                kw = dict(nnz_kind="lognormal", mu=wl["r_lognormal"][0], sigma=wl["r_lognormal"][1])
            R_train = synth.draw(synth.base_seed("learned") + 4, n_train, wl["d"], wl["nnz_r"],
                                 features=wl["features"], zipf_s=wl["zipf"] or 1.0, perm=perm, values=wl["values"],
                                 **kw)
    _log("generated |S|=%d nnz=%d |R|=%d nnz=%d in %.1fs" % (S.n_rows, S.nnz, R.n_rows, R.nnz, time.time() - t0))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    torch.cuda.synchronize()
    # dense head: 128 dimensions at T = 2048 for uint8 data, 64 at T = 1024 for float32
    # (their fastest settings on the medium and fp32 workloads)
    u8 = S.values.dtype == np.uint8
    head = a.dense_head if a.dense_head >= 0 else (128 if u8 else 64)
    if a.persistent:
        head = 0
    _log("building the index")
    tb = time.time()
    ix = kj.build_index(dS, tile_width=a.tile or ((2048 if u8 else 1024) if head else 0), dense_head=head)
    torch.cuda.synchronize()
    t_build = time.time() - tb
    _log("index built in %.3fs (T=%d, %d tiles, dense head %d)" % (t_build, ix.tile_width, ix.n_tiles, head))
    stream = torch.cuda.current_stream()
    sdt = torch.int32 if S.values.dtype == np.uint8 else torch.float32
    G = a.tiles_per_launch
    jkw = dict(persistent=a.persistent, tiles_per_launch=G)

    def outs():
        return (torch.empty((n_r, k), dtype=torch.int32, device=dev), torch.empty((n_r, k), dtype=sdt, device=dev),
                torch.empty(n_r, dtype=torch.int32, device=dev))

    out = outs()
    stats = torch.zeros(8, dtype=torch.int64, device=dev)
    for w in range(max(1, a.warmup)):
        kj.knn_join(ix, dR, k, stats=stats if w == 0 else None, validate=(w == 0), out=out, **jkw)
        torch.cuda.synchronize()
        _log("warmup %d done" % w)
    walked_tail = int(stats[kj.STAT_POSTINGS].item())
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for s in range(a.steps):
        kj.knn_join(ix, dR, k, validate=False, out=out, stream=stream, **jkw)
        _log("step %d launched" % s)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / a.steps
    _log("timed %d steps: %.1f ms/step" % (a.steps, ms))
    qps = n_r / (ms / 1e3)
    entry_bytes = 4 if S.values.dtype == np.uint8 else 6
    walk = None
    walked = walked_tail
    if head:
        # the same index walked list by list (Algorithm 3's accumulation with no
        # dense head): the comparison leg, and the count of every posting the
        # method processes per step
        o2 = outs()
        st2 = torch.zeros(8, dtype=torch.int64, device=dev)
        kj.knn_join(ix, dR, k, out=o2, stats=st2, validate=False, dense_head=False)
        torch.cuda.synchronize()
        walked = int(st2[kj.STAT_POSTINGS].item())
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        kj.knn_join(ix, dR, k, out=o2, validate=False, dense_head=False, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        walk = {"queries_per_s": round(n_r / (t / 1e3), 1), "ms": round(t, 2), "tile_width": ix.tile_width,
                "speedup_of_dense_head": round(t / ms, 3)}
        if sdt == torch.int32:
            walk["identical_to_dense_head"] = all(torch.equal(x, y) for x, y in zip(o2, out))
        else:
            # float sums in another order: counts equal, scores within the 1e-5 rule
            walk["counts_equal"] = bool(torch.equal(o2[2], out[2]))
            walk["max_rel_score_diff"] = float(((o2[1] - out[1]).abs() / out[1].abs().clamp_min(1e-30)).max())
        _log("plain walk", json.dumps(walk))
        del o2
    eps = walked / (ms / 1e3)
    gbps = eps * entry_bytes / 1e9
    # dominant kernel: the tile kernel, one launch per S tile (dense head: per
    # tiles_per_launch tiles); its average launch duration is the step time over
    # the launches (the other launches per step are small: output init, query
    # order, and for the dense head the per-join query preparation)
    launches = ix.n_tiles if not head else -(-ix.n_tiles // G)
    avg_launch_ms = ms / launches
    bytes_per_launch = walked * entry_bytes / launches
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    kname = "k_iibh_tiles" if head else "k_iib_tile"
    cnt = _counters("%s/%s/T%d" % (kname, a.workload, ix.tile_width))
    traffic = cnt.get("bytes_per_launch")
    tail_eps = walked_tail / (ms / 1e3)
    roof = {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "avg_launch_ms": round(avg_launch_ms, 4), "launches_per_step": launches,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            # every walked entry is one local-memory atomic add; gfx950 retires at most one
            # wave64 LDS atomic per 4 clocks per CU (16 lane-ops/clk): 256 CUs x 2.4 GHz x 16
            "onchip": {"unit": "LDS atomic lane-ops/s", "achieved": tail_eps, "peak": LDS_ATOMIC_PEAK,
                       "frac": round(tail_eps / LDS_ATOMIC_PEAK, 4)}}
    if cnt.get("valu_wave_instrs_per_launch"):
        # vector-ALU issue: the counted VALU wave instructions per launch over the live launch
        # time, against one wave64 VALU instruction per 4 clocks per SIMD (16 lanes), 4 SIMDs
        # per CU, 256 CUs, 2.4 GHz
        vi = cnt["valu_wave_instrs_per_launch"] / (avg_launch_ms / 1e3)
        roof["valu"] = {"unit": "VALU wave-instructions/s", "achieved": vi, "peak": VALU_ISSUE_PEAK,
                        "frac": round(vi / VALU_ISSUE_PEAK, 4)}
    if head:
        # bytes of dense head blocks read per launch (the four queries of a workgroup share each read)
        hb = -(-n_r // 4) * ix.tile_width * head * min(G, ix.n_tiles) * (1 if sdt == torch.int32 else 4)
        roof["head_block_bytes_per_launch"] = hb
        roof["head_block_GBps"] = round(hb / (avg_launch_ms / 1e3) / 1e9, 1)

    iiib = None
    if not a.no_iiib:
        iiib = {}
        # IIIB keeps a level table of n_tiles * D * 64 words per index: for float32 data over
        # 100,000 dimensions the dense head's narrow tile (T = 1024) would need 250 GB, so the
        # IIIB legs get an index of their own at T = 4096 (62.5 GB)
        iiib_tile = ix.tile_width if u8 else 4096
        iiib["tile_width"] = iiib_tile

        def timed_join(label, pre=None, **kw):
            o = outs()
            st = torch.zeros(8, dtype=torch.int64, device=dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            if pre is not None:
                kw["theta_seed"] = pre()
            kj.knn_join(ixi, dR, k, algo="iiib", validate=False, out=o, stats=st, stream=stream, **kw)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            if sdt == torch.int32:
                same = all(torch.equal(x, y) for x, y in zip(o, out))
            else:
                # float scores: summation order differs between algorithms
                same = bool(torch.equal(o[2], out[2]) and torch.allclose(o[1], out[1], rtol=1e-5, atol=0))
            res = {"queries_per_s": round(n_r / (t / 1e3), 1), "ms": round(t, 2), "identical_to_iib": same,
                   "postings_walked": int(st[kj.STAT_POSTINGS]), "candidates": int(st[kj.STAT_CANDIDATES]),
                   "completion_entries": int(st[kj.STAT_COMPLETION]), "fallbacks": int(st[kj.STAT_FALLBACKS])}
            _log(label, json.dumps(res))
            return res

        # level drop of the refined variants: the autotuner's choice on a 4,000-query sample.
        # It runs first: its own index and IIIB buffers are released before those of ixi
        # are allocated, so the two never hold device memory at once
        from paper_1011_2807_amd import autotune
        sample = kj.DeviceCSR.from_host(R.take_rows(range(min(4000, n_r))))
        drop = autotune.tune(dS, sample, k, algo="iiib", tiles=(iiib_tile,), drops=(4, 8, 12, 16, 24),
                             use_cache=False)["level_drop"]
        del sample
        _log("iiib level drop (autotuned): %d" % drop)
        iiib["level_drop"] = drop
        ixi = ix if u8 else kj.build_index(dS, tile_width=iiib_tile)
        # allocate the index-level IIIB buffers outside the timed legs
        _log("first IIIB join (IIIB buffers)")
        one = kj.DeviceCSR(dR.indptr[:2].contiguous(), dR.indices, dR.values, dR.n_dims)
        kj.knn_join(ixi, one, k, algo="iiib", validate=False)
        torch.cuda.synchronize()
        _log("first IIIB join done")
        iiib["plain"] = timed_join("iiib plain")
        iiib["refined"] = timed_join("iiib refined", bound_filter=True, level_drop=drop)
        # learned seed: labels are the exact k-th scores of the training queries
        tt = time.time()
        dT = kj.DeviceCSR.from_host(R_train)
        _, tsc, tcnt = kj.knn_join(ix, dT, k, validate=False)
        y = torch.where(tcnt == k, tsc[:, k - 1].float(), torch.zeros_like(tcnt, dtype=torch.float32)).contiguous()
        Xt = kj.Mlp.features(ixi, dT)
        mlp = kj.Mlp(seed=1)
        losses = mlp.train(Xt, y, epochs=8, batch=512, lr=2e-3, tau=0.05, seed=2)
        t_train = time.time() - tt
        _log("trained the seed MLP on %d queries in %.1fs, loss %.4f -> %.4f" % (n_train, t_train, losses[0],
                                                                                  losses[-1]))
        res = timed_join("iiib learned", bound_filter=True, level_drop=drop,
                         pre=lambda: mlp.predict(kj.Mlp.features(ixi, dR, stream=stream), stream=stream))
        res["miss_rate"] = round(res["fallbacks"] / n_r, 4)
        res["train_queries"] = n_train
        res["train_s"] = round(t_train, 2)
        res["train_loss"] = [round(losses[0], 5), round(losses[-1], 5)]
        iiib["learned"] = res
        iiib["learned_vs_refined_speedup"] = round(iiib["refined"]["ms"] / res["ms"], 3)
        iiib["learned_vs_plain_speedup"] = round(iiib["plain"]["ms"] / res["ms"], 3)

    check, cpu = cpu_baseline_leg(R, S, k, out, a.check, 0.0 if a.no_cpu else a.cpu_seconds,
                                  f32=sdt != torch.int32)
    ok = check["exact"]
    res = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8" if sdt == torch.int32 else "f32", "data": "synthetic",
        "config": {"workload": a.workload, "algo": "iib", "schedule": "persistent" if a.persistent else "tile launches",
                   "n_r": n_r, "n_s": n_s, "d": wl["d"], "k": k, "dense_head": head,
                   "tiles_per_launch": G if head else 1,
                   "tile_width": ix.tile_width, "nnz_s": S.nnz, "nnz_r": R.nnz},
        "postings_entries_per_s": eps, "postings_GBps": round(gbps, 1), "postings_entries_per_step": walked,
        "walked_entries_per_step": walked_tail, "iib_plain_walk": walk,
        "index_build_s": round(t_build, 3), "oracle_spot_check": check,
        "iiib": iiib, "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(res))
    bad = not ok or (iiib is not None and not all(iiib[v]["identical_to_iib"] for v in ("plain", "refined", "learned")))
    if walk is not None:
        bad = bad or not walk.get("identical_to_dense_head", True) or not walk.get("counts_equal", True) or \
            walk.get("max_rel_score_diff", 0.0) > 1e-5
    if bad:
        sys.exit(1)


def run_sweep(a):
    """One JSON line per point of a sweep: milliseconds per full join for each
    algorithm (mean of 3 timed runs after one untimed run, HIP events), every
    output identical to IIB's, and the oracle's rows (cpu_baseline leg)."""
    import torch
    import synth
    import paper_1011_2807_amd as kj
    sw = SWEEPS[a.sweep]
    gen = sw["gen"]
    perm = synth.workload_perm(gen)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if a.sweep == "buffer":
        return run_buffer_sweep(a, sw, perm, stream)
    bad = False
    for pt in sw["points"]:
        n_r, n_s, k = pt["n_r"], pt["n_s"], pt["k"]
        S = synth.make(gen, "S", n_rows=n_s, perm=perm)
        R = synth.make(gen, "R", n_rows=n_r, perm=perm)
        dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
        ix = kj.build_index(dS, tile_width=4096)
        ixh = kj.build_index(dS, tile_width=2048, dense_head=128)
        torch.cuda.synchronize()

        def outs():
            return (torch.empty((n_r, k), dtype=torch.int32, device="cuda"),
                    torch.empty((n_r, k), dtype=torch.int32, device="cuda"),
                    torch.empty(n_r, dtype=torch.int32, device="cuda"))

        runs = {
            "bf": lambda o: kj.knn_join_bf(dS, dR, k, out=o),
            "iib": lambda o: kj.knn_join(ix, dR, k, out=o, validate=False),
            "iib_dense_head": lambda o: kj.knn_join(ixh, dR, k, out=o, validate=False),
            "iiib": lambda o: kj.knn_join(ix, dR, k, algo="iiib", out=o, validate=False),
            "iiib_refined": lambda o: kj.knn_join(ix, dR, k, algo="iiib", bound_filter=True, level_drop=8, out=o,
                                                  validate=False),
        }
        ms, res = {}, {}
        for name, fn in runs.items():
            o = outs()
            reps = 0
            while True:
                # the first run is untimed unless it alone takes over 2 s
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(max(1, reps)):
                    fn(o)
                e1.record(stream)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1)
                if reps or t > 2000.0:
                    ms[name] = round(t / max(1, reps), 3)
                    break
                reps = 3
            res[name] = o
        same = {name: all(torch.equal(x, y) for x, y in zip(o, res["iib"])) for name, o in res.items()}
        check, cpu = cpu_baseline_leg(R, S, k, res["iib"], 2, 0.0, f32=False)
        bad |= not check["exact"] or not all(same.values())
        print(json.dumps({
            "sweep": a.sweep, "figure": sw["figure"], "data": "synthetic", "generator": gen,
            "n_r": n_r, "n_s": n_s, "d": synth.WORKLOADS[gen]["d"], "k": k, "nnz_r": R.nnz, "nnz_s": S.nnz,
            "ms_per_join": ms, "queries_per_s": {x: round(n_r / (v / 1e3), 1) for x, v in ms.items()},
            "identical_to_iib": same, "oracle_spot_check": check, "cpu_baseline": cpu,
            "notes": "mean of 3 timed joins after one untimed (one timed join where it takes over 2 s); bf includes "
                     "its input validation (a device check of R and S, one synchronisation); iib: T = 4096; "
                     "iib_dense_head: T = 2048, dense head 128; iiib_refined: bound filter, level drop 8",
        }), flush=True)
        del ix, ixh
    if bad:
        sys.exit(1)


def run_buffer_sweep(a, sw, perm, stream):
    """Fig. 4's buffer sweep: the blocked join (S in page-locked host memory,
    copied block by block on a stream of its own while the previous block is
    joined) at each block size, against the join of one index of all of S in
    device memory; IIB with the dense head (128, T = 2048), k = 10.  One JSON
    line per block size, phase times from the library (copy = I/O)."""
    import torch
    import synth
    import paper_1011_2807_amd as kj
    pt0 = sw["points"][0]
    n_r, n_s, k = pt0["n_r"], pt0["n_s"], pt0["k"]
    gen_name = sw["gen"]
    S = synth.make(gen_name, "S", n_rows=n_s, perm=perm)
    R = synth.make(gen_name, "R", n_rows=n_r, perm=perm)
    hS = kj.HostCSR(S)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    t0 = time.time()
    ix = kj.build_index(dS, tile_width=2048, dense_head=128)
    torch.cuda.synchronize()
    t_build = (time.time() - t0) * 1e3
    ref = kj.knn_join(ix, dR, k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    kj.knn_join(ix, dR, k, validate=False, out=ref)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_in = e0.elapsed_time(e1)
    del ix, dS
    s_bytes = int(S.indptr.nbytes + S.indices.nbytes + S.values.nbytes)
    check, cpu = cpu_baseline_leg(R, S, k, ref, 2, 0.0, f32=False)
    bad = not check["exact"]
    for pt in sw["points"]:
        block_rows = int(round(pt["block_frac"] * n_s))
        kj.knn_join_blocked(hS, dR, k, block_rows, tile_width=2048, dense_head=128)  # untimed
        ids, sc, cnt, t = kj.knn_join_blocked(hS, dR, k, block_rows, tile_width=2048, dense_head=128)
        same = all(torch.equal(x, y) for x, y in zip((ids, sc, cnt), ref))
        bad |= not same
        print(json.dumps({
            "sweep": "buffer", "figure": sw["figure"], "data": "synthetic", "generator": gen_name,
            "n_r": n_r, "n_s": n_s, "d": synth.WORKLOADS[gen_name]["d"], "k": k, "block_rows": block_rows,
            "block_share_of_S": pt["block_frac"], "n_blocks": t["n_blocks"],
            "phase_ms": {x: round(t[x], 3) for x in ("copy_ms", "build_ms", "join_ms", "merge_ms", "total_ms")},
            "queries_per_s": round(n_r / (t["total_ms"] / 1e3), 1),
            "copy_GBps": round(s_bytes / (t["copy_ms"] / 1e3) / 1e9, 2) if t["copy_ms"] > 0 else None,
            "in_memory": {"join_ms": round(ms_in, 3), "index_build_ms": round(t_build, 1),
                          "queries_per_s": round(n_r / (ms_in / 1e3), 1)},
            "identical_to_in_memory": same, "oracle_spot_check": check, "cpu_baseline": cpu,
            "notes": "IIB with dense head 128, T = 2048; one untimed blocked run first; S bytes %d" % s_bytes,
        }), flush=True)
    if bad:
        sys.exit(1)


def run_batched(a):
    """Batched workload: |R| = 1,000,000 queries of lognormal length, |S| =
    4,000,000, D = 20,000, k = 1 and k = 10.  Tile width and IIIB level drop come
    from the autotuner (timed on a 4,000-query sample); the IIIB joins for k = 1
    and k = 10 run as one captured HIP graph."""
    import torch
    import synth
    import paper_1011_2807_amd as kj
    from paper_1011_2807_amd import autotune

    wl = synth.WORKLOADS["batched"]
    n_r = a.n_r or wl["n_r"]
    n_s = a.n_s or wl["n_s"]
    t0 = time.time()
    perm = synth.workload_perm("batched")
    S = synth.make("batched", "S", n_rows=n_s, perm=perm)
    R = synth.make("batched", "R", n_rows=n_r, perm=perm)
    _log("generated |S|=%d nnz=%d |R|=%d nnz=%d in %.1fs" % (S.n_rows, S.nnz, R.n_rows, R.nnz, time.time() - t0))
    dev = torch.device("cuda:0")
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    sample = kj.DeviceCSR.from_host(R.take_rows(range(min(4000, n_r))))
    tt = time.time()
    tune_iib = autotune.tune(dS, sample, 10, algo="iib", tiles=(2048, 4096, 8192))
    tune_iiib = autotune.tune(dS, sample, 10, algo="iiib", tiles=(tune_iib["tile_width"],), drops=(4, 8, 12, 16, 24))
    _log("autotune %.1fs: IIB %s, IIIB %s" % (time.time() - tt,
                                             {x: tune_iib[x] for x in ("tile_width", "dense_head", "tiles_per_launch",
                                                                       "persistent")},
                                             {x: tune_iiib[x] for x in ("tile_width", "level_drop")}))
    ix = kj.build_index(dS, tile_width=tune_iib["tile_width"], dense_head=tune_iib["dense_head"])
    stream = torch.cuda.current_stream()

    def outs(k):
        return (torch.empty((n_r, k), dtype=torch.int32, device=dev), torch.empty((n_r, k), dtype=torch.int32, device=dev),
                torch.empty(n_r, dtype=torch.int32, device=dev))

    # IIB, k = 10 (validated warmup run, then one timed run)
    ref = outs(10)
    stats = torch.zeros(8, dtype=torch.int64, device=dev)
    jkw = dict(persistent=tune_iib["persistent"], tiles_per_launch=tune_iib["tiles_per_launch"])
    kj.knn_join(ix, dR, 10, out=ref, stats=stats, **jkw)
    torch.cuda.synchronize()
    # postings the method processes (Eq. 4's second term): sum over the queries'
    # features of |I_d| (with a dense head the walk counter sees only the tail)
    walked = int(ix.list_lengths().to(torch.int64)[dR.indices.long()].sum().item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    kj.knn_join(ix, dR, 10, out=ref, validate=False, stream=stream, **jkw)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_iib = e0.elapsed_time(e1)
    _log("IIB k=10: %.1f ms" % ms_iib)
    # IIIB k = 1 and k = 10 in one graph (eager run first: allocations, constants)
    o1, o10 = outs(1), outs(10)
    kw = dict(algo="iiib", bound_filter=True, level_drop=tune_iiib["level_drop"])
    kj.knn_join(ix, dR, 1, out=o1, **kw)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        kj.knn_join(ix, dR, 1, out=o1, validate=False, **kw)
        kj.knn_join(ix, dR, 10, out=o10, validate=False, **kw)
    torch.cuda.synchronize()
    e0.record(stream)
    g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1)
    _log("graph (IIIB k=1 + k=10): %.1f ms" % ms_graph)
    same10 = all(torch.equal(x, y) for x, y in zip(o10, ref))
    k1_prefix = bool(torch.equal(o1[0][:, 0], o10[0][:, 0]) and torch.equal(o1[1][:, 0], o10[1][:, 0]))
    check, cpu = cpu_baseline_leg(R, S, 10, ref, a.check, 0.0, f32=False)
    ok = check["exact"]
    qps = n_r / (ms_iib / 1e3)
    entry_bytes = 4
    head = tune_iib["dense_head"]
    launches = ix.n_tiles if not head else -(-ix.n_tiles // (tune_iib["tiles_per_launch"] or 4))
    achieved = walked * entry_bytes / (ms_iib / 1e3) / 1e9
    res = {
        "metric": METRIC, "value": round(qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(ms_iib, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "batched", "algo": "iib", "n_r": n_r, "n_s": n_s, "d": wl["d"], "k": 10,
                   "tile_width": ix.tile_width, "dense_head": tune_iib["dense_head"], "nnz_s": S.nnz,
                   "nnz_r": R.nnz},
        "postings_entries_per_s": walked / (ms_iib / 1e3), "postings_GBps": round(achieved, 1),
        "graph_iiib_k1_k10": {"ms": round(ms_graph, 2), "queries_per_s_per_k": round(2 * n_r / (ms_graph / 1e3), 1),
                              "k10_identical_to_iib": same10, "k1_is_first_column_of_k10": k1_prefix,
                              "level_drop": tune_iiib["level_drop"]},
        "autotune": {"iib": tune_iib["timings"], "iiib": tune_iiib["timings"]},
        "oracle_spot_check": check,
        "roofline": {"kernel": "k_iibh_tiles" if head else "k_iib_tile", "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                     "avg_launch_ms": round(ms_iib / launches, 4), "launches_per_step": launches},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))
    if not (ok and same10 and k1_prefix):
        sys.exit(1)


if __name__ == "__main__":
    main()
