"""GPU parity of the learned-seed kernels (features, MLP forward/backward) against
the float64 reference, and what the trained seed gains inside IIIB."""
import numpy as np
import pytest

import oracle
import synth
from helpers import assert_exact
from oracle import mlp as ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1011_2807_amd as kj  # noqa: E402


def _dev(m):
    return kj.DeviceCSR.from_host(m)


@pytest.fixture(scope="module")
def small():
    S = synth.make("learned", "S", n_rows=40_000)
    R = synth.make("learned", "R_train", n_rows=3000)
    E = synth.make("learned", "R_eval", n_rows=600)
    ix = kj.build_index(_dev(S), tile_width=4096)
    return S, R, E, ix


def test_features_match_reference(small):
    S, R, _, ix = small
    X = kj.Mlp.features(ix, _dev(R)).cpu().numpy()
    ll = np.bincount(S.indices, minlength=S.n_dims)
    want = ref.features(R.take_rows(range(200)), ll)
    np.testing.assert_allclose(X[:200], want, rtol=2e-7, atol=1e-7)


def _state(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.1, ref.N_PARAMS).astype(np.float32)
    norm = np.concatenate([rng.normal(0, 0.2, 64), rng.uniform(0.3, 1.5, 64), [1000.0]]).astype(np.float32)
    return p, norm


def test_forward_and_grad_match_reference():
    m = kj.Mlp(seed=3)
    p, norm = _state(4)
    m.set_state(p, norm)
    pw, nw = m.get_state()
    np.testing.assert_array_equal(pw, ref.bf16_round(p))      # working weights are bf16-rounded
    rng = np.random.default_rng(5)
    n = 777
    X = rng.normal(0, 1, (n, 64)).astype(np.float32)
    y = rng.uniform(200, 1800, n).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    pred = m.predict(Xd).cpu().numpy().astype(np.float64)
    want = ref.predict(pw, nw, X)
    np.testing.assert_allclose(pred, want, rtol=1e-4, atol=1e-3 * float(nw[128]) * 1e-3)
    for tau in (0.05, 0.5):
        g, loss = m.grad(Xd, yd, tau)
        g = g.cpu().numpy().astype(np.float64)
        gw = ref.grad(pw, nw, X, y, tau)
        scale = np.abs(gw).max()
        err = np.abs(g - gw).max()
        print("tau", tau, "max |grad|", scale, "max err", err, flush=True)
        assert err <= 1e-4 * scale + 1e-7
        assert abs(float(loss.item()) - ref.pinball(pw, nw, X, y, tau)) <= 1e-5 * abs(ref.pinball(pw, nw, X, y, tau))


def test_training_lowers_the_loss_and_the_seed_gains(small):
    """Train on exact k-th scores from the join itself, then compare IIIB with and
    without the seed on fresh queries: identical exact results, fewer postings."""
    S, R, E, ix = small
    k = 10
    dR, dE = _dev(R), _dev(E)
    _, sc, cnt = kj.knn_join(ix, dR, k)
    y = torch.where(cnt == k, sc[:, k - 1], torch.zeros_like(cnt)).float().contiguous()
    X = kj.Mlp.features(ix, dR)
    m = kj.Mlp(seed=7)
    losses = m.train(X, y, epochs=12, batch=256, lr=2e-3, tau=0.05, seed=1)
    print("epoch losses", ["%.4f" % v for v in losses], flush=True)
    assert losses[-1] < 0.5 * losses[0]
    theta = m.predict(kj.Mlp.features(ix, dE))
    st_plain = torch.zeros(8, dtype=torch.int64, device="cuda")
    st_seed = torch.zeros(8, dtype=torch.int64, device="cuda")
    fb = torch.zeros(E.n_rows, dtype=torch.uint8, device="cuda")
    plain = kj.knn_join(ix, dE, k, algo="iiib", stats=st_plain)
    seeded = kj.knn_join(ix, dE, k, algo="iiib", theta_seed=theta, stats=st_seed, fallback_out=fb)
    torch.cuda.synchronize()
    for a, b in zip(plain, seeded):
        assert torch.equal(a, b)
    rows = list(range(0, E.n_rows, 60))
    want = oracle.bf_topk_rows(E, S, k, rows)
    assert_exact(tuple(x[rows] for x in seeded), want, "learned IIIB sample")
    walked_plain = int(st_plain[kj.STAT_POSTINGS])
    walked_seed = int(st_seed[kj.STAT_POSTINGS])
    miss = float(fb.float().mean())
    print("postings plain %d seeded %d (%.3f), candidates plain %d seeded %d, miss rate %.3f" % (
        walked_plain, walked_seed, walked_seed / walked_plain, int(st_plain[kj.STAT_CANDIDATES]),
        int(st_seed[kj.STAT_CANDIDATES]), miss), flush=True)
    assert walked_seed < walked_plain
    assert miss < 0.3
