"""GPU parity of the IIB join with a dense head (the longest lists kept as dense
per-tile byte blocks and scored with dot products) against the CPU oracle."""
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
def zipf():
    # ragged last tile at every tile width used below
    S = synth.make("medium", "S", n_rows=20_500)
    R = synth.make("medium", "R", n_rows=150)
    return S, R, oracle.bf_topk(R, S, 10)


@pytest.mark.parametrize("tile,head,k", [(4096, 64, 10), (2048, 128, 10), (1024, 64, 1), (4096, 256, 100),
                                         (256, 64, 10), (1024, 128, 10), (1024, 192, 5), (512, 256, 1),
                                         (2048, 128, 60), (8192, 128, 10)])
def test_zipf_head_bit_exact(zipf, tile, head, k):
    S, R, want10 = zipf
    want = want10 if k == 10 else oracle.bf_topk(R, S, k)
    print("zipf head T", tile, "H", head, "k", k, flush=True)
    ix = kj.build_index(_dev(S), tile_width=tile, dense_head=head)
    assert ix.dense_head == head
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    got = kj.knn_join(ix, _dev(R), k, stats=stats)
    torch.cuda.synchronize()
    assert_exact(got, want, "zipf head T=%d H=%d k=%d" % (tile, head, k))
    # the head takes postings off the walk
    walked = int(stats[kj.STAT_POSTINGS])
    assert 0 <= walked < oracle.postings_walked(R, S)
    # the same index without the head walks every list
    stats.zero_()
    got = kj.knn_join(ix, _dev(R), k, stats=stats, dense_head=False)
    torch.cuda.synchronize()
    assert_exact(got, want, "zipf head off T=%d" % tile)
    assert int(stats[kj.STAT_POSTINGS]) == oracle.postings_walked(R, S)


def test_tiny_head_bit_exact():
    S = synth.make("tiny", "S")
    R = synth.make("tiny", "R")
    want = oracle.bf_topk(R, S, 10)
    for tile, head in ((1024, 64), (4096, 192), (2048, 256)):
        ix = kj.build_index(_dev(S), tile_width=tile, dense_head=head)
        got = kj.knn_join(ix, _dev(R), 10)
        torch.cuda.synchronize()
        assert_exact(got, want, "tiny head T=%d H=%d" % (tile, head))


def test_head_edge_cases():
    """Rows and queries with only head dimensions, only tail dimensions, none at
    all; fewer than k positive scores; ties at the cut; more head slots than
    dimensions; one query (a partly empty workgroup of four)."""
    rows_s = ([[(1, 3), (5, 2)]] * 700 + [[]] + [[(9, 4)]] + [[(1, 1)]] * 300 + [[(11, 255)]] * 3
              + [[(d, 1 + d) for d in range(12)]])
    S = _csr(rows_s, 12)
    queries = [[(1, 2)], [], [(5, 1), (9, 1)], [(7, 200)], [(1, 255), (5, 255), (9, 255)], [(11, 1), (0, 9)],
               [(d, 255) for d in range(12)]]
    for n_q in (len(queries), 1, 5):
        R = _csr(queries[:n_q], 12)
        for k in (1, 5, 1024):
            want = oracle.bf_topk(R, S, k)
            for tile, head in ((256, 64), (512, 128)):
                ix = kj.build_index(_dev(S), tile_width=tile, dense_head=head)
                got = kj.knn_join(ix, _dev(R), k)
                torch.cuda.synchronize()
                assert_exact(got, want, "edge head n_q=%d k=%d T=%d H=%d" % (n_q, k, tile, head))


def test_head_with_blocked_queries(zipf):
    S, R, want = zipf
    ix = kj.build_index(_dev(S), tile_width=2048, dense_head=64)
    got = kj.knn_join(ix, _dev(R), 10, r_block_rows=37)
    torch.cuda.synchronize()
    assert_exact(got, want, "zipf head B=37")


@pytest.fixture(scope="module")
def zipf_f32():
    # the float32 workload's distribution (Zipf 1.05, L2-normalised lognormal
    # values) at a size the oracle scores in seconds; ragged last tiles
    S = synth.draw(521, 9000, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    R = synth.draw(522, 48, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    return S, R


@pytest.mark.parametrize("tile,head,k", [(1024, 64, 50), (2048, 128, 50), (512, 256, 5), (4096, 192, 1),
                                         (256, 64, 100)])
def test_f32_head_within_tolerance(zipf_f32, tile, head, k):
    """float32 head blocks scored with fp64 products: every score within the
    1e-5 rule of the fp64 oracle, the same walk counter as the u8 head."""
    S, R = zipf_f32
    print("f32 head T", tile, "H", head, "k", k, flush=True)
    ix = kj.build_index(_dev(S), tile_width=tile, dense_head=head)
    assert ix.dense_head == head
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    got = kj.knn_join(ix, _dev(R), k, stats=stats)
    torch.cuda.synchronize()
    assert_f32_close(got, R, S, range(R.n_rows), what="f32 head T=%d H=%d k=%d" % (tile, head, k))
    assert 0 <= int(stats[kj.STAT_POSTINGS]) < oracle.postings_walked(R, S)
    plain = kj.knn_join(ix, _dev(R), k, dense_head=False)
    torch.cuda.synchronize()
    assert torch.equal(got[2], plain[2])
    torch.testing.assert_close(got[1], plain[1], rtol=1e-6, atol=0)


def test_f32_head_edge_cases():
    """Rows and queries with only head dimensions, only tail dimensions, none;
    fewer than k positive scores; equal vectors (ties within rounding); a
    partly empty workgroup of four queries."""
    rows_s = ([[(1, 0.5), (5, 0.25)]] * 700 + [[]] + [[(9, 1.0)]] + [[(1, 0.125)]] * 300 + [[(11, 2.0)]] * 3
              + [[(d, 0.1 * (1 + d)) for d in range(12)]])
    S = _csr(rows_s, 12, np.float32)
    queries = [[(1, 0.75)], [], [(5, 1.5), (9, 0.5)], [(7, 3.0)], [(1, 1.0), (5, 1.0), (9, 1.0)],
               [(11, 0.5), (0, 4.0)], [(d, 1.0) for d in range(12)]]
    for n_q in (len(queries), 1, 5):
        R = _csr(queries[:n_q], 12, np.float32)
        for k in (1, 5, 1024):
            for tile, head in ((256, 64), (512, 128)):
                ix = kj.build_index(_dev(S), tile_width=tile, dense_head=head)
                got = kj.knn_join(ix, _dev(R), k)
                torch.cuda.synchronize()
                assert_f32_close(got, R, S, range(R.n_rows), what="f32 edge n_q=%d k=%d T=%d H=%d" % (n_q, k, tile,
                                                                                                       head))


def test_head_rejections():
    u = synth.draw(12, 500, 300, (5, 20), features="uniform")
    for bad in (8, 16, 96, 320, -64):
        with pytest.raises(kj.KnnjError):
            kj.build_index(_dev(u), dense_head=bad)
