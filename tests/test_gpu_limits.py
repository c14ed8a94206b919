"""GPU parity at the library's size limits: rows of the longest accepted length
(4096 features) in both R and S, joined at the widest S tile the device's
workgroup local memory takes, with k up to its maximum (1024); one feature more,
or a tile wider than 65536 rows, is rejected."""
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

EINVAL, EUNSUPPORTED = -1, -5
N_DIMS = 8192


def _dev(m):
    return kj.DeviceCSR.from_host(m)


def _vstack(*ms):
    indptr, off = [np.zeros(1, dtype=np.int64)], 0
    for m in ms:
        indptr.append(m.indptr[1:] + off)
        off += m.nnz
    return synth.CSR(np.concatenate(indptr), np.concatenate([m.indices for m in ms]),
                     np.concatenate([m.values for m in ms]), ms[0].n_dims)


def _data(values):
    # Zipf rows around three rows of 4096 features (in the second S tile at the
    # narrower widths, the first at the wider), and two 4096-feature queries
    S = _vstack(synth.draw(901, 2500, N_DIMS, (20, 300), features="zipf", values=values),
                synth.draw(902, 3, N_DIMS, (4096, 4096), values=values),
                synth.draw(903, 600, N_DIMS, (20, 300), features="zipf", values=values))
    R = _vstack(synth.draw(904, 6, N_DIMS, (20, 300), features="zipf", values=values),
                synth.draw(905, 2, N_DIMS, (4096, 4096), values=values))
    return S, R


def _widest(run, **index_opts):
    """Run `run(ix)` on the widest power-of-two tile the device accepts for it;
    every wider tile must be refused as unsupported (local memory)."""
    for t in (65536, 32768, 16384, 8192, 4096, 2048):
        try:
            ix = kj.build_index(_dev(run.S), tile_width=t, **index_opts)
            got = run(ix)
            torch.cuda.synchronize()
            print("  widest tile", t, flush=True)
            return t, got
        except kj.KnnjError as e:
            assert e.code == EUNSUPPORTED, (t, e)
    raise AssertionError("no tile width accepted")


class _Join:
    def __init__(self, S, R, k, **join_opts):
        self.S, self.R, self.k, self.opts = S, R, k, join_opts

    def __call__(self, ix):
        return kj.knn_join(ix, _dev(self.R), self.k, **self.opts)


@pytest.mark.parametrize("k", [10, 1024])
def test_longest_rows_widest_tile_u8(k):
    S, R = _data("u8")
    want = oracle.bf_topk(R, S, k)
    for name, run, opts in (("IIB", _Join(S, R, k), {}),
                            ("IIB dense head", _Join(S, R, k), {"dense_head": 128}),
                            ("IIIB", _Join(S, R, k, algo="iiib"), {}),
                            ("refined IIIB", _Join(S, R, k, algo="iiib", bound_filter=True, level_drop=8), {})):
        print("limits u8", name, "k", k, flush=True)
        t, got = _widest(run, **opts)
        assert_exact(got, want, "%s k=%d T=%d" % (name, k, t))
    got = kj.knn_join_bf(_dev(S), _dev(R), k)
    torch.cuda.synchronize()
    assert_exact(got, want, "BF k=%d" % k)


def test_longest_rows_widest_tile_f32():
    S, R = _data("f32")
    k = 50
    for name, run in (("IIB", _Join(S, R, k)), ("IIIB", _Join(S, R, k, algo="iiib"))):
        print("limits f32", name, flush=True)
        t, got = _widest(run)
        assert_f32_close(got, R, S, range(R.n_rows), what="f32 %s T=%d" % (name, t))


def test_one_feature_too_many_and_too_wide_a_tile():
    S, _ = _data("u8")
    ix = kj.build_index(_dev(S), tile_width=4096)
    long_row = synth.CSR(np.array([0, 4097], dtype=np.int64), np.arange(4097, dtype=np.int32),
                         np.ones(4097, dtype=np.uint8), N_DIMS)
    with pytest.raises(kj.KnnjError) as e:
        kj.knn_join(ix, _dev(long_row), 10)
    assert e.value.code == EINVAL
    with pytest.raises(kj.KnnjError) as e:
        kj.build_index(_dev(long_row))
    assert e.value.code == EINVAL
    with pytest.raises(kj.KnnjError) as e:
        kj.build_index(_dev(S), tile_width=131072)
    assert e.value.code == EINVAL
