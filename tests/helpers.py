"""Comparison helpers shared by the GPU parity tests."""
import numpy as np

import oracle


def assert_exact(got, want, what=""):
    """Bit-exact comparison of (ids, scores, count) for integer scores."""
    g_ids, g_sc, g_cnt = [np.asarray(x.cpu().numpy() if hasattr(x, "cpu") else x) for x in got]
    w_ids, w_sc, w_cnt = want
    bad = np.nonzero((g_ids != w_ids).any(axis=1) | (g_sc.astype(np.int64) != w_sc).any(axis=1) |
                     (g_cnt != w_cnt))[0]
    if len(bad):
        q = bad[0]
        raise AssertionError("%s: %d queries differ; first q=%d\n got ids %s sc %s cnt %d\nwant ids %s sc %s cnt %d" % (
            what, len(bad), q, g_ids[q].tolist(), g_sc[q].tolist(), g_cnt[q], w_ids[q].tolist(), w_sc[q].tolist(),
            w_cnt[q]))


def assert_f32_close(got, R, S, rows, rel=1e-5, what=""):
    """fp32 scores: every returned pair within rel of its fp64 oracle score; the id
    set may differ from the oracle's only on ids whose oracle score lies within rel
    of the oracle's k-th score; counts equal."""
    g_ids, g_sc, g_cnt = [np.asarray(x.cpu().numpy() if hasattr(x, "cpu") else x) for x in got]
    rows = list(rows)
    k = g_ids.shape[1]
    w_ids, w_sc, w_cnt = oracle.bf_topk_rows(R, S, k, rows)
    for i, q in enumerate(rows):
        gi = g_ids[i] if g_ids.shape[0] == len(rows) else g_ids[q]
        gs = g_sc[i] if g_sc.shape[0] == len(rows) else g_sc[q]
        gc = g_cnt[i] if g_cnt.shape[0] == len(rows) else g_cnt[q]
        assert gc == w_cnt[i], (what, q, gc, w_cnt[i])
        all_sc = oracle.scores_one(R, S, q)
        ids = gi[:gc]
        assert np.all(ids >= 0) and len(set(ids.tolist())) == gc, (what, q)
        np.testing.assert_allclose(gs[:gc], all_sc[ids], rtol=rel, atol=0, err_msg="%s q=%d" % (what, q))
        assert np.all(np.diff(gs[:gc].astype(np.float64)) <= 0), (what, q)
        if gc:
            kth = w_sc[i, gc - 1]
            diff = set(ids.tolist()) ^ set(w_ids[i, :gc].tolist())
            for j in diff:
                assert abs(all_sc[j] - kth) <= rel * kth, (what, q, j, all_sc[j], kth)
        assert np.all(gi[gc:] == -1) and np.all(gs[gc:] == 0), (what, q)
