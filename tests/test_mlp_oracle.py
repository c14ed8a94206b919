"""Pins for the float64 MLP reference (no GPU): the hand-written backward pass
against central finite differences, the feature definition on a worked case."""
import numpy as np

import synth
from oracle import mlp


def _rand_state(rng):
    p = rng.normal(0, 0.3, mlp.N_PARAMS)
    norm = np.concatenate([rng.normal(0, 0.1, 64), rng.uniform(0.5, 2.0, 64), [3.0]])
    return p, norm


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p, norm = _rand_state(rng)
    X = rng.normal(0, 1, (12, 64))
    yhat, _ = mlp.forward(p, norm, X)
    # targets away from the pinball kink so the loss is smooth near p
    y = (yhat + rng.choice([-1.0, 1.0], 12) * rng.uniform(0.5, 1.0, 12)) * norm[128]
    for tau in (0.05, 0.5):
        g = mlp.grad(p, norm, X, y, tau)
        idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False),
                              [mlp.OFF_B1, mlp.OFF_W2 + 5, mlp.OFF_B2 + 3, mlp.OFF_W3 + 7, mlp.OFF_B3]])
        eps = 1e-6
        for i in idx:
            pp, pm = p.copy(), p.copy()
            pp[i] += eps
            pm[i] -= eps
            fd = (mlp.pinball(pp, norm, X, y, tau) - mlp.pinball(pm, norm, X, y, tau)) / (2 * eps)
            assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(g[i]), (tau, i, fd, g[i])


def test_pinball_quantile_property():
    """Minimising the pinball loss over a constant gives the tau-quantile."""
    rng = np.random.default_rng(2)
    ys = rng.normal(0, 1, 2001)
    for tau in (0.05, 0.5, 0.9):
        cands = np.linspace(-3, 3, 2401)
        losses = [np.mean(np.where(ys - c >= 0, tau * (ys - c), (tau - 1) * (ys - c))) for c in cands]
        best = cands[int(np.argmin(losses))]
        assert abs(best - np.quantile(ys, tau)) < 0.02


def test_features_worked_case():
    # one query with weights 16, 17, 255 on dims 0, 1, 2; list lengths 0, 2, 1000
    R = synth.CSR(np.array([0, 3, 3], dtype=np.int64), np.array([0, 1, 2], dtype=np.int32),
                  np.array([16, 17, 255], dtype=np.uint8), 3)
    f = mlp.features(R, np.array([0, 2, 1000]))
    assert f.shape == (2, 64)
    assert abs(f[0, 0] - np.log(4.0)) < 1e-15
    # weight bins: 16>>4 = 1, 17>>4 = 1, 255>>4 = 15
    assert f[0, 1 + 1] == 2 / 3 and f[0, 1 + 15] == 1 / 3
    # length bins: 2 log2(1) = 0 -> 0; 2 log2(3) = 3.17 -> 3; 2 log2(1001) = 19.93 -> 19
    assert f[0, 17 + 0] == 1 / 3 and f[0, 17 + 3] == 1 / 3 and f[0, 17 + 19] == 1 / 3
    assert np.all(f[1] == 0)
    # the shares of each group sum to one
    assert abs(f[0, 1:17].sum() - 1) < 1e-15 and abs(f[0, 17:].sum() - 1) < 1e-15


def test_bf16_round():
    x = np.array([1.0, 1.00390625, 1.005859375, -2.5, 3.14159265], dtype=np.float32)
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0          # tie rounds to even
    assert r[2] == np.float32(1.0078125)        # above the tie rounds up
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-7
