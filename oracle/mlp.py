"""Float64 reference of the threshold-predicting MLP.  TEST INFRASTRUCTURE ONLY.

The learned seed is not part of the paper (its Sec. 6 asks for stronger
refinement of IIIB); what is fixed here is its definition:

* features of a query r (64 values): log(1 + |r|); the share of r's features in
  each of 16 weight bins (u8: w >> 4; f32: min(15, floor(16 w))); the share in
  each of 47 bins min(46, floor(2 log2(1 + |I_d|))) of posting-list length;
* network: x_std = (x - mean) / std; h1 = relu(W1 x_std + b1);
  h2 = relu(W2 h1 + b2); yhat = w3 . h2 + b3; prediction = yhat * label_scale;
* loss: mean pinball loss at quantile tau of (y / label_scale - yhat).

The backward pass is written out by hand and pinned against central finite
differences in tests/test_mlp_oracle.py.  Parameter layout (flat):
W1[128][64] b1[128] W2[128][128] b2[128] w3[128] b3.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 64, 128
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_HID * N_IN
OFF_W2 = OFF_B1 + N_HID
OFF_B2 = OFF_W2 + N_HID * N_HID
OFF_W3 = OFF_B2 + N_HID
OFF_B3 = OFF_W3 + N_HID
N_PARAMS = OFF_B3 + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(N_HID, N_IN), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(N_HID, N_HID),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def features(R, list_len) -> np.ndarray:
    """64 features per row of R (CSR with uint8 or float32 values)."""
    n = len(R.indptr) - 1
    out = np.zeros((n, N_IN), dtype=np.float64)
    ll = np.asarray(list_len, dtype=np.int64)
    for q in range(n):
        b, e = int(R.indptr[q]), int(R.indptr[q + 1])
        m = e - b
        out[q, 0] = np.log1p(m)
        if m == 0:
            continue
        w = R.values[b:e]
        if w.dtype == np.uint8:
            bw = w.astype(np.int64) >> 4
        else:
            bw = np.minimum(15, np.floor(16.0 * w.astype(np.float64))).astype(np.int64)
        x = ll[R.indices[b:e]] + 1
        # floor(2 log2 x) in integers: 2 * floor(log2 x) + [x^2 >= 2^(2 floor(log2 x) + 1)]
        fl = np.array([int(v).bit_length() - 1 for v in x], dtype=np.int64)
        half = np.array([int(v) * int(v) >= (1 << (2 * int(f) + 1)) for v, f in zip(x, fl)], dtype=np.int64)
        bl = np.minimum(46, 2 * fl + half)
        out[q, 1:17] = np.bincount(bw, minlength=16)[:16] / m
        out[q, 17:64] = np.bincount(bl, minlength=47)[:47] / m
    return out


def forward(p, norm, X):
    """Returns yhat (normalised units) and the cache for backward."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    norm = np.asarray(norm, dtype=np.float64)
    xs = (np.asarray(X, dtype=np.float64) - norm[:N_IN]) / norm[N_IN:2 * N_IN]
    a1 = xs @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    yhat = h2 @ w3 + b3
    return yhat, (xs, a1, h1, a2, h2)


def predict(p, norm, X):
    yhat, _ = forward(p, norm, X)
    return yhat * float(norm[2 * N_IN])


def pinball(p, norm, X, y, tau):
    yhat, _ = forward(p, norm, X)
    d = np.asarray(y, dtype=np.float64) / float(norm[2 * N_IN]) - yhat
    return float(np.mean(np.where(d >= 0, tau * d, (tau - 1.0) * d)))


def grad(p, norm, X, y, tau):
    """Gradient of the mean pinball loss with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    yhat, (xs, a1, h1, a2, h2) = forward(p, norm, X)
    n = len(yhat)
    d = np.asarray(y, dtype=np.float64) / float(norm[2 * N_IN]) - yhat
    g = np.where(d > 0, -tau, np.where(d < 0, 1.0 - tau, 0.0)) / n      # dL/dyhat
    g2 = np.outer(g, w3) * (a2 > 0)                                        # dL/da2
    g1 = (g2 @ W2) * (a1 > 0)                                              # dL/da1
    out = np.zeros(N_PARAMS)
    out[OFF_W1:OFF_B1] = (g1.T @ xs).ravel()
    out[OFF_B1:OFF_W2] = g1.sum(axis=0)
    out[OFF_W2:OFF_B2] = (g2.T @ h1).ravel()
    out[OFF_B2:OFF_W3] = g2.sum(axis=0)
    out[OFF_W3:OFF_B3] = g @ h2
    out[OFF_B3] = g.sum()
    return out


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even) and back."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (a >> 16) & 1
    r = ((a + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)
