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
