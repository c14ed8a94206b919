"""GPU parity of the IIIB join (Algorithm 4) and of the seeded threshold with
its survivor check, against the CPU oracle."""
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
    return S, R, oracle.bf_topk(R, S, 10)


@pytest.fixture(scope="module")
def zipf():
    S = synth.make("medium", "S", n_rows=20_500)
    R = synth.make("medium", "R", n_rows=150)
    return S, R, oracle.bf_topk(R, S, 10)


@pytest.mark.parametrize("tile,r_block", [(1024, 0), (4096, 128), (2048, 1)])
def test_tiny_iiib_bit_exact(tiny, tile, r_block):
    S, R, want = tiny
    print("tiny IIIB tile", tile, "r_block", r_block, flush=True)
    ix = kj.build_index(_dev(S), tile_width=tile)
    got = kj.knn_join(ix, _dev(R), 10, algo="iiib", r_block_rows=r_block)
    torch.cuda.synchronize()
    assert_exact(got, want, "tiny IIIB T=%d B=%d" % (tile, r_block))


@pytest.mark.parametrize("tile,r_block,k", [(2048, 0, 10), (4096, 50, 3), (1024, 0, 1)])
def test_zipf_iiib_bit_exact(zipf, tile, r_block, k):
    S, R, want10 = zipf
    want = want10 if k == 10 else oracle.bf_topk(R, S, k)
    print("zipf IIIB tile", tile, "r_block", r_block, "k", k, flush=True)
    ix = kj.build_index(_dev(S), tile_width=tile)
    stats = torch.zeros(8, dtype=torch.int64, device="cuda")
    got = kj.knn_join(ix, _dev(R), k, algo="iiib", r_block_rows=r_block, stats=stats)
    torch.cuda.synchronize()
    assert_exact(got, want, "zipf IIIB T=%d B=%d k=%d" % (tile, r_block, k))
    st = stats.cpu().numpy()
    # the refinement never walks more postings than IIB, and completes candidates
    assert 0 < st[kj.STAT_POSTINGS] <= oracle.postings_walked(R, S)
    assert st[kj.STAT_CANDIDATES] > 0 and st[kj.STAT_COMPLETION] > 0


@pytest.mark.parametrize("bound,drop", [(True, 0), (True, 4), (False, 8)])
def test_zipf_iiib_refinement_options_exact(zipf, bound, drop):
    S, R, want = zipf
    ix = kj.build_index(_dev(S), tile_width=2048)
    got = kj.knn_join(ix, _dev(R), 10, algo="iiib", bound_filter=bound, level_drop=drop)
    torch.cuda.synchronize()
    assert_exact(got, want, "zipf IIIB bound=%s drop=%d" % (bound, drop))


def test_seeded_threshold_survivor_check(zipf):
    """Seeds at, below and above the true k-th score: results stay exact, and only
    seeds above the true k-th send a query to the fallback pass."""
    S, R, want = zipf
    ids, sc, cnt = want
    kth = np.where(cnt == 10, sc[:, 9], 0).astype(np.float64)
    ix = kj.build_index(_dev(S), tile_width=2048)
    rng = np.random.default_rng(5)
    cases = {
        "exact": kth,
        "low": 0.5 * kth,
        "high": 1.5 * kth + 1,
        "mixed": kth * rng.choice([0.7, 1.0, 1.3], size=len(kth)),
        "huge": np.full(len(kth), 1e30),
    }
    for name, seed in cases.items():
        print("seed case", name, flush=True)
        seed_t = torch.tensor(seed, dtype=torch.float32, device="cuda")
        fb = torch.zeros(R.n_rows, dtype=torch.uint8, device="cuda")
        stats = torch.zeros(8, dtype=torch.int64, device="cuda")
        got = kj.knn_join(ix, _dev(R), 10, algo="iiib", theta_seed=seed_t, fallback_out=fb, stats=stats)
        torch.cuda.synchronize()
        assert_exact(got, want, "seeded IIIB (%s)" % name)
        fbn = fb.cpu().numpy().astype(bool)
        s32 = seed.astype(np.float32).astype(np.float64)
        must = (np.ceil(s32) > kth) & (s32 > 0)     # seed above the true k-th: cannot be verified
        assert np.all(fbn[must]), name
        assert not np.any(fbn[np.ceil(s32) <= kth]), name
        assert int(stats[kj.STAT_FALLBACKS]) == int(fbn.sum())


def test_iiib_edge_cases():
    rows_s = [[(1, 3), (5, 2)]] * 700 + [[]] + [[(9, 4)]] + [[(1, 1)]] * 300
    rows_r = [[(1, 2)], [], [(5, 1), (9, 1)], [(7, 200)], [(1, 255), (5, 255), (9, 255)]]
    S = _csr(rows_s, 12)
    R = _csr(rows_r, 12)
    for k in (1, 5, 1024):
        want = oracle.bf_topk(R, S, k)
        for tile in (256, 512):
            ix = kj.build_index(_dev(S), tile_width=tile)
            got = kj.knn_join(ix, _dev(R), k, algo="iiib", r_block_rows=2)
            torch.cuda.synchronize()
            assert_exact(got, want, "edge IIIB k=%d T=%d" % (k, tile))


def test_f32_iiib_within_tolerance():
    S = synth.draw(501, 9000, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    R = synth.draw(502, 40, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    ix = kj.build_index(_dev(S), tile_width=2048)
    got = kj.knn_join(ix, _dev(R), 50, algo="iiib")
    torch.cuda.synchronize()
    assert_f32_close(got, R, S, range(R.n_rows), what="f32 IIIB")


@pytest.mark.parametrize("values,n_dims", [("f32", 20_000), ("u8", 50_000)])
def test_iiib_hashed_r_for_many_dimensions(values, n_dims):
    """Dimensions too many for a dense local copy of r: IIIB completes candidates
    through the local hash table of r's features."""
    S = synth.draw(601, 12_000, n_dims, (30, 300), features="zipf", zipf_s=1.05, values=values)
    R = synth.draw(602, 60, n_dims, (30, 300), features="zipf", zipf_s=1.05, values=values)
    ix = kj.build_index(_dev(S), tile_width=4096)
    for validate in (True, False):
        got = kj.knn_join(ix, _dev(R), 50 if values == "f32" else 10, algo="iiib", validate=validate)
        torch.cuda.synchronize()
        if values == "f32":
            assert_f32_close(got, R, S, range(R.n_rows), what="f32 hashed IIIB")
        else:
            assert_exact(got, oracle.bf_topk(R, S, 10), "u8 hashed IIIB")
