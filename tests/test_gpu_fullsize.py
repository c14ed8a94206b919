"""Full-size runs in the configuration bench.py times (medium workload: 100,000
queries x 1,000,000 vectors, T = 2048, dense head of 128 dimensions, four tiles
per launch): sampled queries against the oracle one by one, and properties that
must hold for every query."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_exact

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1011_2807_amd as kj  # noqa: E402


def _invariants(ids, sc, cnt, k, n_s):
    ids = ids.cpu().numpy()
    sc = sc.cpu().numpy().astype(np.int64)
    cnt = cnt.cpu().numpy()
    assert np.all((cnt >= 0) & (cnt <= k))
    col = np.arange(k)[None, :]
    held = col < cnt[:, None]
    assert np.all(ids[held] >= 0) and np.all(ids[held] < n_s)
    assert np.all(sc[held] > 0)
    assert np.all(ids[~held] == -1) and np.all(sc[~held] == 0)
    # non-increasing scores, ascending ids among equal scores
    d = np.diff(sc, axis=1)
    both = held[:, 1:]
    assert np.all(d[both] <= 0)
    tie = both & (d == 0)
    assert np.all(np.diff(ids, axis=1)[tie] > 0)
    # no id twice in a row
    srt = np.sort(np.where(held, ids, -1 - col), axis=1)
    assert np.all(np.diff(srt, axis=1) != 0)


def test_medium_full_size_sampled_parity():
    S = synth.make("medium", "S")
    R = synth.make("medium", "R")
    k = 10
    print("medium full size generated", flush=True)
    ix = kj.build_index(kj.DeviceCSR.from_host(S), tile_width=2048, dense_head=128)
    dR = kj.DeviceCSR.from_host(R)
    got = kj.knn_join(ix, dR, k, tiles_per_launch=4)
    torch.cuda.synchronize()
    print("IIB (dense head) done", flush=True)
    _invariants(*got, k, S.n_rows)
    assert int(got[2].min()) == k          # every medium query has >= 10 positive scores
    # random queries plus the longest and the shortest one
    rng = np.random.default_rng(11)
    nnz = np.diff(R.indptr)
    rows = np.unique(np.concatenate([rng.choice(R.n_rows, 12, replace=False), [nnz.argmax(), nnz.argmin()]]))
    want = oracle.bf_topk_rows(R, S, k, rows)
    assert_exact(tuple(x[torch.from_numpy(rows).cuda()] for x in got), want, "medium full-size IIB")
    plain = kj.knn_join(ix, dR, k, dense_head=False)
    torch.cuda.synchronize()
    for a, b in zip(got, plain):
        assert torch.equal(a, b)
    print("plain walk identical", flush=True)
    ref = kj.knn_join(ix, dR, k, algo="iiib", bound_filter=True, level_drop=4)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    print("refined IIIB identical", flush=True)


def test_batched_full_S_sampled_parity():
    """The batched workload's full S (4,000,000 rows, 20,000 dimensions) with its
    longest and shortest queries (lognormal lengths up to 1,000 features) and a
    random sample, in the configurations its autotuner chooses between: plain
    walk at T = 4096, dense head 192; both exact on sampled rows and identical
    to each other and to refined IIIB."""
    S = synth.make("batched", "S")
    Rall = synth.make("batched", "R", n_rows=20_000)
    nnz = np.diff(Rall.indptr)
    rng = np.random.default_rng(5)
    pick = np.unique(np.concatenate([np.argsort(nnz)[-40:], np.argsort(nnz)[:20], rng.choice(20_000, 140, replace=False)]))
    R = Rall.take_rows(pick)
    k = 10
    print("batched full S generated; %d queries, longest %d features" % (R.n_rows, int(np.diff(R.indptr).max())),
          flush=True)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    ix = kj.build_index(dS, tile_width=4096)
    got = kj.knn_join(ix, dR, k)
    torch.cuda.synchronize()
    _invariants(*got, k, S.n_rows)
    nr = np.diff(R.indptr)
    rows = np.unique(np.concatenate([[nr.argmax(), nr.argmin()], rng.choice(R.n_rows, 6, replace=False)]))
    want = oracle.bf_topk_rows(R, S, k, rows)
    assert_exact(tuple(x[torch.from_numpy(rows).cuda()] for x in got), want, "batched full-S IIB")
    print("plain walk exact", flush=True)
    ref = kj.knn_join(ix, dR, k, algo="iiib", bound_filter=True, level_drop=6)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    ix.free()
    ixh = kj.build_index(dS, tile_width=4096, dense_head=192)
    head = kj.knn_join(ixh, dR, k)
    torch.cuda.synchronize()
    for a, b in zip(got, head):
        assert torch.equal(a, b)
    print("refined IIIB and dense head identical", flush=True)


def test_fp32_full_S_sampled_parity():
    """The fp32 workload's full S (10,000,000 rows, 100,000 dimensions; its IIIB
    level table exceeds 2^32 words): IIB and refined IIIB on a few hundred
    queries and the dense head at the settings bench.py times, sampled rows
    within the fp32 rule against the fp64 oracle."""
    from helpers import assert_f32_close
    S = synth.make("fp32", "S")
    R = synth.make("fp32", "R", n_rows=200)
    k = 50
    print("fp32 full S generated", flush=True)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    ix = kj.build_index(dS)
    got = kj.knn_join(ix, dR, k)
    torch.cuda.synchronize()
    print("IIB done", flush=True)
    assert_f32_close(got, R, S, [0, 57, 199], what="fp32 full-S IIB")
    ref = kj.knn_join(ix, dR, k, algo="iiib", bound_filter=True, level_drop=4)
    torch.cuda.synchronize()
    print("IIIB done", flush=True)
    assert torch.equal(got[2], ref[2])
    assert torch.allclose(got[1], ref[1], rtol=1e-5, atol=0)
    del ix
    # the launch configuration bench.py times for this workload: dense head 64 at T = 1024
    ixh = kj.build_index(dS, tile_width=1024, dense_head=64)
    head = kj.knn_join(ixh, dR, k)
    torch.cuda.synchronize()
    print("dense head done", flush=True)
    assert_f32_close(head, R, S, [0, 57, 199], what="fp32 full-S IIB dense head")
    assert torch.equal(got[2], head[2])
    assert torch.allclose(got[1], head[1], rtol=1e-5, atol=0)
