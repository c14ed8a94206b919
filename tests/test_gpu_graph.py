"""The IIB join captured into a HIP graph: k = 1 and k = 10 in one graph,
replayed several times with eager work between replays, every replay checked
against the eager result."""
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


def test_graph_k1_and_k10_replays():
    S = synth.make("batched", "S", n_rows=30_000)
    R = synth.make("batched", "R", n_rows=500)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    ix = kj.build_index(dS, tile_width=4096)
    n = R.n_rows
    outs = {}
    for k in (1, 10):
        outs[k] = (torch.empty((n, k), dtype=torch.int32, device="cuda"),
                   torch.empty((n, k), dtype=torch.int32, device="cuda"),
                   torch.empty(n, dtype=torch.int32, device="cuda"))
    # eager reference (also grows the library's join scratch outside the capture)
    eager = {k: [x.clone() for x in kj.knn_join(ix, dR, k)] for k in (1, 10)}
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for k in (1, 10):
            kj.knn_join(ix, dR, k, validate=False, out=outs[k])
    torch.cuda.synchronize()
    for rep in range(3):
        for k in (1, 10):
            for x in outs[k]:
                x.fill_(-7)
        # eager work between replays
        kj.knn_join(ix, dR, 3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in (1, 10):
            for a, b in zip(outs[k], eager[k]):
                assert torch.equal(a, b), (rep, k)
    # k = 1 is the first column of k = 10
    assert torch.equal(outs[1][0][:, 0], outs[10][0][:, 0])
    assert torch.equal(outs[1][1][:, 0], outs[10][1][:, 0])
    rows = list(range(0, n, 50))
    want = oracle.bf_topk_rows(R, S, 10, rows)
    assert_exact(tuple(x[rows] for x in outs[10]), want, "graph replay k=10")


def test_graph_learned_iiib_pipeline():
    """Features -> MLP prediction -> seeded IIIB (survivor check + fallback pass),
    with k = 1 and k = 10, all inside one captured graph; replays equal the
    eager IIB result."""
    S = synth.make("batched", "S", n_rows=30_000)
    R = synth.make("batched", "R", n_rows=400)
    T = synth.make("batched", "R", n_rows=3000)      # training queries (a larger draw; rows >= 400 unseen)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    ix = kj.build_index(dS, tile_width=4096)
    dT = kj.DeviceCSR.from_host(T.take_rows(range(400, 3000)))
    _, tsc, tcnt = kj.knn_join(ix, dT, 10)
    y = torch.where(tcnt == 10, tsc[:, 9].float(), torch.zeros_like(tcnt, dtype=torch.float32)).contiguous()
    m = kj.Mlp(seed=5)
    m.train(kj.Mlp.features(ix, dT), y, epochs=6, batch=256, lr=2e-3, tau=0.05, seed=3)
    n = R.n_rows
    ref = {k: [x.clone() for x in kj.knn_join(ix, dR, k)] for k in (1, 10)}
    outs = {k: (torch.empty((n, k), dtype=torch.int32, device="cuda"),
                torch.empty((n, k), dtype=torch.int32, device="cuda"),
                torch.empty(n, dtype=torch.int32, device="cuda")) for k in (1, 10)}
    feats = torch.empty((n, 64), dtype=torch.float32, device="cuda")
    theta = torch.empty(n, dtype=torch.float32, device="cuda")
    fb = torch.zeros(n, dtype=torch.uint8, device="cuda")
    # eager pass grows the library scratch and uploads constants before the capture
    for k in (1, 10):
        kj.knn_join(ix, dR, k, algo="iiib", theta_seed=m.predict(kj.Mlp.features(ix, dR)), bound_filter=True,
                    level_drop=4, fallback_out=fb)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        feats.copy_(kj.Mlp.features(ix, dR))
        theta.copy_(m.predict(feats))
        for k in (1, 10):
            kj.knn_join(ix, dR, k, algo="iiib", theta_seed=theta, bound_filter=True, level_drop=4, validate=False,
                        fallback_out=fb, out=outs[k])
    torch.cuda.synchronize()
    for rep in range(3):
        for k in (1, 10):
            for x in outs[k]:
                x.fill_(-7)
        kj.knn_join(ix, dR, 2)          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in (1, 10):
            for a, b in zip(outs[k], ref[k]):
                assert torch.equal(a, b), (rep, k)
    print("miss rate in the graph: %.3f" % float(fb.float().mean()), flush=True)


def test_graph_dense_head_replays():
    """The dense-head IIB join (per-join query preparation, group kernels over
    runs of tiles) captured with k = 1 and k = 10; replays with eager work in
    between equal the eager result and the oracle."""
    S = synth.make("medium", "S", n_rows=30_000)
    R = synth.make("medium", "R", n_rows=300)
    dS, dR = kj.DeviceCSR.from_host(S), kj.DeviceCSR.from_host(R)
    ix = kj.build_index(dS, tile_width=2048, dense_head=128)
    n = R.n_rows
    outs = {k: (torch.empty((n, k), dtype=torch.int32, device="cuda"),
                torch.empty((n, k), dtype=torch.int32, device="cuda"),
                torch.empty(n, dtype=torch.int32, device="cuda")) for k in (1, 10)}
    # eager reference (also grows the join scratch outside the capture)
    eager = {k: [x.clone() for x in kj.knn_join(ix, dR, k, tiles_per_launch=4)] for k in (1, 10)}
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for k in (1, 10):
            kj.knn_join(ix, dR, k, validate=False, out=outs[k], tiles_per_launch=4)
    torch.cuda.synchronize()
    for rep in range(3):
        for k in (1, 10):
            for x in outs[k]:
                x.fill_(-7)
        kj.knn_join(ix, dR, 3, dense_head=False)      # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in (1, 10):
            for a, b in zip(outs[k], eager[k]):
                assert torch.equal(a, b), (rep, k)
    assert torch.equal(outs[1][0][:, 0], outs[10][0][:, 0])
    rows = list(range(0, n, 30))
    want = oracle.bf_topk_rows(R, S, 10, rows)
    assert_exact(tuple(x[rows] for x in outs[10]), want, "graph replay, dense head, k=10")
