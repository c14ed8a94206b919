"""The autotuner times real joins, picks the fastest tile width (and dense head),
and caches it; the tuned join stays exact."""
import os

import pytest

import oracle
import synth
from helpers import assert_exact, assert_f32_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1011_2807_amd as kj  # noqa: E402
from paper_1011_2807_amd import autotune  # noqa: E402


def test_autotune_picks_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("KNNJ_TUNE_CACHE", str(tmp_path / "tune.json"))
    S = synth.make("medium", "S", n_rows=40_000)
    R = synth.make("medium", "R", n_rows=400)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    res = autotune.tune(dS, dR, 10, algo="iib", tiles=(1024, 4096), verbose=True)
    assert res["tile_width"] in (1024, 4096)
    # per tile: plain walk with tile launches and persistent, dense head 128 and 192
    # with 2, 4 and 8 tiles per launch
    assert len(res["timings"]) == 2 * (2 + 2 * 3)
    assert res["dense_head"] in (0, 128, 192)
    assert min(t["ms"] for t in res["timings"]) == res["ms"]
    assert os.path.exists(tmp_path / "tune.json")
    again = autotune.tune(dS, dR, 10, algo="iib", tiles=(1024, 4096))
    assert again == res                       # served from the cache
    ix = kj.build_index(dS, tile_width=res["tile_width"], dense_head=res["dense_head"])
    got = kj.knn_join(ix, dR, 10, persistent=res["persistent"], tiles_per_launch=res["tiles_per_launch"])
    torch.cuda.synchronize()
    assert_exact(got, oracle.bf_topk(R, S, 10), "tuned IIB")
    r2 = autotune.tune(dS, dR, 10, algo="iiib", tiles=(2048,), drops=(0, 4))
    ix2 = kj.build_index(dS, tile_width=r2["tile_width"])
    got = kj.knn_join(ix2, dR, 10, algo="iiib", bound_filter=r2["bound_filter"], level_drop=r2["level_drop"])
    torch.cuda.synchronize()
    assert_exact(got, oracle.bf_topk(R, S, 10), "tuned IIIB")


def test_autotune_float32_heads(tmp_path, monkeypatch):
    monkeypatch.setenv("KNNJ_TUNE_CACHE", str(tmp_path / "tune.json"))
    S = synth.draw(531, 12_000, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    R = synth.draw(532, 200, 4000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    res = autotune.tune(dS, dR, 50, algo="iib", tiles=(1024,), heads=(0, 64))
    # plain walk: two schedules; head 64: three launch groupings
    assert len(res["timings"]) == 2 + 3
    assert res["dense_head"] in (0, 64)
    ix = kj.build_index(dS, tile_width=res["tile_width"], dense_head=res["dense_head"])
    got = kj.knn_join(ix, dR, 50, persistent=res["persistent"], tiles_per_launch=res["tiles_per_launch"])
    torch.cuda.synchronize()
    assert_f32_close(got, R, S, range(R.n_rows), what="tuned f32 IIB")
