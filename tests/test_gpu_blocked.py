"""GPU parity of the blocked join (Algorithm 1's outer loop over S blocks with S
in host memory) against the CPU oracle: every block size, ragged last blocks,
ties split across blocks, both algorithms, the dense head, float32 data."""
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
    S = synth.make("medium", "S", n_rows=20_500)
    R = synth.make("medium", "R", n_rows=150)
    return S, R, oracle.bf_topk(R, S, 10)


@pytest.mark.parametrize("block_rows,tile,head", [(20_500, 4096, 0), (777, 1024, 0), (5000, 2048, 128),
                                                  (100_000, 4096, 0), (4096, 4096, 64)])
def test_blocked_iib_bit_exact(zipf, block_rows, tile, head):
    S, R, want = zipf
    print("blocked IIB B", block_rows, "T", tile, "H", head, flush=True)
    hS = kj.HostCSR(S)
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    ids, sc, cnt, times = kj.knn_join_blocked(hS, kj.DeviceCSR.from_host(R), 10, block_rows, tile_width=tile,
                                              dense_head=head, stats=stats)
    assert_exact((ids, sc, cnt), want, "blocked IIB B=%d T=%d H=%d" % (block_rows, tile, head))
    assert times["n_blocks"] == -(-S.n_rows // block_rows)
    assert times["total_ms"] > 0 and times["copy_ms"] > 0 and times["join_ms"] > 0
    if head == 0:
        # the blocks' walks add up to the walk of all of S (Eq. 4's second term)
        assert int(stats[kj.STAT_POSTINGS]) == oracle.postings_walked(R, S)


@pytest.mark.parametrize("block_rows,bound,drop", [(3000, False, 0), (6000, True, 8)])
def test_blocked_iiib_bit_exact(zipf, block_rows, bound, drop):
    S, R, want = zipf
    print("blocked IIIB B", block_rows, flush=True)
    got = kj.knn_join_blocked(kj.HostCSR(S), kj.DeviceCSR.from_host(R), 10, block_rows, tile_width=2048,
                              algo="iiib", bound_filter=bound, level_drop=drop)[:3]
    assert_exact(got, want, "blocked IIIB B=%d" % block_rows)


def test_blocked_ties_across_blocks_and_tiny_blocks():
    """700 identical rows split over several blocks (the lowest ids must win
    the ties), an empty row, rows on unused dimensions; block sizes down to one
    row; k above the number of positive scores."""
    rows_s = ([[(1, 3), (5, 2)]] * 700 + [[]] + [[(9, 4)]] + [[(1, 1)]] * 30 + [[(11, 255)]] * 3)
    S = _csr(rows_s, 12)
    R = _csr([[(1, 2)], [], [(5, 1), (9, 1)], [(7, 200)], [(1, 255), (5, 255), (9, 255)], [(11, 1)]], 12)
    dR = kj.DeviceCSR.from_host(R)
    for k in (1, 5, 1024):
        want = oracle.bf_topk(R, S, k)
        for block_rows in (1, 3, 256, 700, 701, 5000):
            if block_rows == 1 and k != 5:
                continue
            got = kj.knn_join_blocked(kj.HostCSR(S), dR, k, block_rows, tile_width=256)[:3]
            assert_exact(got, want, "ties k=%d B=%d" % (k, block_rows))


def test_blocked_f32_within_tolerance():
    S = synth.draw(511, 9000, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    R = synth.draw(512, 40, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    for block_rows in (2500, 9000):
        ids, sc, cnt, _ = kj.knn_join_blocked(kj.HostCSR(S), kj.DeviceCSR.from_host(R), 50, block_rows,
                                              tile_width=2048)
        assert_f32_close((ids, sc, cnt), R, S, range(R.n_rows), what="blocked f32 B=%d" % block_rows)


def test_blocked_empty_inputs_and_errors():
    S = _csr([[(0, 1)], [(0, 2)], [(1, 1)]], 2)
    R0 = kj.DeviceCSR.from_host(_csr([], 2))
    ids, sc, cnt, t = kj.knn_join_blocked(kj.HostCSR(S), R0, 3, 2)
    assert ids.shape == (0, 3) and t["n_blocks"] == 0
    R1 = kj.DeviceCSR.from_host(_csr([[(0, 5)]], 2))
    ids, sc, cnt, t = kj.knn_join_blocked(kj.HostCSR(_csr([], 2)), R1, 3, 2)
    torch.cuda.synchronize()
    assert cnt.tolist() == [0] and ids.tolist() == [[-1, -1, -1]] and sc.tolist() == [[0, 0, 0]]
    for bad in (0, -5):
        with pytest.raises(kj.KnnjError) as e:
            kj.knn_join_blocked(kj.HostCSR(S), R1, 3, bad)
        assert e.value.code == -1
    with pytest.raises(kj.KnnjError) as e:
        kj.knn_join_blocked(kj.HostCSR(S), kj.DeviceCSR.from_host(_csr([[(0, 5)]], 3)), 3, 2)
    assert e.value.code == -1
    with pytest.raises(kj.KnnjError) as e:      # a malformed block is refused by its index build
        bad = synth.CSR(np.array([0, 2], dtype=np.int64), np.array([1, 0], dtype=np.int32),
                        np.array([1, 1], dtype=np.uint8), 2)
        kj.knn_join_blocked(kj.HostCSR(bad), R1, 3, 1)
    assert e.value.code == -1
