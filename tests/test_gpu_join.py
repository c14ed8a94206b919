"""GPU parity of the HIP join (IIB and brute force) against the CPU oracle."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_exact, assert_f32_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1011_2807_amd as kj  # noqa: E402


def _dev(m):
    return kj.DeviceCSR.from_host(m)


def _csr(rows, n_dims, dtype=np.uint8):
    indptr = np.zeros(len(rows) + 1, dtype=np.int64)
    idx, val = [], []
    for i, r in enumerate(rows):
        r = sorted(r)
        indptr[i + 1] = indptr[i] + len(r)
        idx += [d for d, _ in r]
        val += [w for _, w in r]
    return synth.CSR(indptr, np.array(idx, dtype=np.int32), np.array(val, dtype=dtype), n_dims)


@pytest.fixture(scope="module")
def tiny():
    S = synth.make("tiny", "S")
    R = synth.make("tiny", "R")
    want = oracle.bf_topk(R, S, 10)
    return S, R, want


@pytest.mark.parametrize("tile", [256, 2048, 8192, 16384])
def test_tiny_iib_full_bit_exact(tiny, tile):
    S, R, want = tiny
    print("tiny IIB tile", tile, flush=True)
    try:
        ix = kj.build_index(_dev(S), tile_width=tile)
    except kj.KnnjError as e:
        if e.code == -5:
            pytest.skip("tile %d exceeds this device's workgroup local memory" % tile)
        raise
    got = kj.knn_join(ix, _dev(R), 10)
    torch.cuda.synchronize()
    assert_exact(got, want, "tiny IIB T=%d" % tile)


def test_tiny_bf_full_bit_exact(tiny):
    S, R, want = tiny
    print("tiny BF", flush=True)
    got = kj.knn_join_bf(_dev(S), _dev(R), 10)
    torch.cuda.synchronize()
    assert_exact(got, want, "tiny BF")


def test_postings_counter_equals_eq4(tiny):
    S, R, _ = tiny
    ix = kj.build_index(_dev(S))
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    kj.knn_join(ix, _dev(R), 10, stats=stats)
    torch.cuda.synchronize()
    assert int(stats[kj.STAT_POSTINGS]) == oracle.postings_walked(R, S)


def test_list_lengths(tiny):
    S, _, _ = tiny
    ix = kj.build_index(_dev(S), tile_width=1024)
    ll = ix.list_lengths().cpu().numpy()
    np.testing.assert_array_equal(ll, np.bincount(S.indices, minlength=S.n_dims))


@pytest.mark.parametrize("tile,k,per_tile", [(1024, 10, False), (4096, 1, True), (8192, 37, False), (2048, 10, True)])
def test_zipf_multi_tile_ragged(tile, k, per_tile):
    """Medium-workload recipe at 20,500 S rows (several tiles plus a ragged one),
    persistent schedule and one launch per tile."""
    S = synth.make("medium", "S", n_rows=20_500)
    R = synth.make("medium", "R", n_rows=120)
    print("zipf tile", tile, "k", k, "persistent", per_tile, flush=True)
    want = oracle.bf_topk(R, S, k)
    ix = kj.build_index(_dev(S), tile_width=tile)
    got = kj.knn_join(ix, _dev(R), k, persistent=per_tile)
    torch.cuda.synchronize()
    assert_exact(got, want, "zipf IIB T=%d k=%d" % (tile, k))


def test_uneven_queries_persistent_schedule():
    """Lognormal query lengths (batched-workload recipe): persistent schedule with
    the longest-first order equals persistent and the oracle."""
    S = synth.make("batched", "S", n_rows=12_000)
    R = synth.make("batched", "R", n_rows=300)
    ix = kj.build_index(_dev(S), tile_width=2048)
    want = oracle.bf_topk(R, S, 10)
    a = kj.knn_join(ix, _dev(R), 10)
    b = kj.knn_join(ix, _dev(R), 10, persistent=True)
    torch.cuda.synchronize()
    assert_exact(a, want, "batched per-tile launches")
    assert_exact(b, want, "batched persistent")


def test_edge_cases_empty_rows_padding_ties():
    # S: identical vectors (all tie), an empty row, a vector on unused dims
    rows_s = [[(1, 3), (5, 2)]] * 700 + [[]] + [[(9, 4)]] + [[(1, 1)]] * 300
    rows_r = [[(1, 2)], [], [(5, 1), (9, 1)], [(7, 200)], [(1, 255), (5, 255), (9, 255)]]
    S = _csr(rows_s, 12)
    R = _csr(rows_r, 12)
    for k in (1, 5, 1024):
        want = oracle.bf_topk(R, S, k)
        for tile in (256, 512):
            ix = kj.build_index(_dev(S), tile_width=tile)
            for per_tile in (False, True):
                got = kj.knn_join(ix, _dev(R), k, persistent=per_tile)
                torch.cuda.synchronize()
                assert_exact(got, want, "edge IIB k=%d T=%d per-tile=%s" % (k, tile, per_tile))
        got = kj.knn_join_bf(_dev(S), _dev(R), k)
        torch.cuda.synchronize()
        assert_exact(got, want, "edge BF k=%d" % k)


def test_empty_R_and_tiny_S():
    S = _csr([[(0, 1)], [(0, 2)], [(1, 1)]], 2)
    R = _csr([], 2)
    ix = kj.build_index(_dev(S))
    ids, sc, cnt = kj.knn_join(ix, _dev(R), 3)
    assert ids.shape == (0, 3)
    R1 = _csr([[(0, 5)]], 2)
    got = kj.knn_join(ix, _dev(R1), 3)
    torch.cuda.synchronize()
    assert_exact(got, oracle.bf_topk(R1, S, 3), "3-row S")


def test_validation_errors():
    S = _csr([[(0, 1), (3, 2)], [(2, 2)]], 4)
    ix = kj.build_index(_dev(S))
    bad_order = synth.CSR(np.array([0, 2], dtype=np.int64), np.array([3, 1], dtype=np.int32),
                          np.array([1, 1], dtype=np.uint8), 4)
    bad_zero = synth.CSR(np.array([0, 1], dtype=np.int64), np.array([1], dtype=np.int32),
                         np.array([0], dtype=np.uint8), 4)
    bad_range = synth.CSR(np.array([0, 1], dtype=np.int64), np.array([4], dtype=np.int32),
                          np.array([1], dtype=np.uint8), 4)
    for m in (bad_order, bad_zero, bad_range):
        with pytest.raises(kj.KnnjError) as e:
            kj.knn_join(ix, _dev(m), 2)
        assert e.value.code == -1
        with pytest.raises(kj.KnnjError) as e:
            kj.build_index(_dev(m))
        assert e.value.code == -1
    good = _csr([[(1, 1)]], 4)
    for k in (0, 1025):
        with pytest.raises(kj.KnnjError) as e:
            kj.knn_join(ix, _dev(good), k)
        assert e.value.code == -1
    other = _csr([[(1, 1)]], 5)
    with pytest.raises(kj.KnnjError):
        kj.knn_join(ix, _dev(other), 2)
    with pytest.raises(kj.KnnjError):
        kj.build_index(_dev(S), tile_width=1000)


def test_f32_iib_and_bf_within_tolerance():
    S = synth.draw(501, 9000, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    R = synth.draw(502, 40, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    ix = kj.build_index(_dev(S), tile_width=4096)
    got = kj.knn_join(ix, _dev(R), 50)
    torch.cuda.synchronize()
    assert_f32_close(got, R, S, range(R.n_rows), what="f32 IIB")
    got = kj.knn_join_bf(_dev(S), _dev(R), 50)
    torch.cuda.synchronize()
    assert_f32_close(got, R, S, range(R.n_rows), what="f32 BF")
