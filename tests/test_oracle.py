"""Pins for the CPU oracle (no GPU).

The oracle is the brute-force definition of the join (Sec. 3 Eq. 1, Sec. 4.2
Algorithm 2).  Each test below checks it against something other than itself:
a hand-worked case, exhaustive enumeration against an independent dense
computation, planted maxima with a closed-form score, a scipy sparse product,
the paper's streaming selection form, and Theorem 1 (IIB and IIIB reach the
brute-force result).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import models

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _csr(rows, n_dims, dtype=np.uint8):
    indptr = np.zeros(len(rows) + 1, dtype=np.int64)
    idx, val = [], []
    for i, r in enumerate(rows):
        r = sorted(r)
        indptr[i + 1] = indptr[i] + len(r)
        idx += [d for d, _ in r]
        val += [w for _, w in r]
    return synth.CSR(indptr, np.array(idx, dtype=np.int32), np.array(val, dtype=dtype), n_dims)


def _dense(m):
    out = np.zeros((m.n_rows, m.n_dims), dtype=np.float64 if m.values.dtype == np.float32 else np.int64)
    for i in range(m.n_rows):
        d, w = m.row(i)
        out[i, d] = w
    return out


def _dense_topk(R, S, k):
    """Independent definition: dense score matrix + lexsort."""
    sc = _dense(R) @ _dense(S).T
    n_r, n_s = sc.shape
    ids = np.full((n_r, k), -1, dtype=np.int64)
    scores = np.zeros((n_r, k), dtype=sc.dtype)
    count = np.zeros(n_r, dtype=np.int64)
    for i in range(n_r):
        j = np.arange(n_s)
        order = np.lexsort((j, -sc[i]))
        order = order[sc[i][order] > 0][:k]
        ids[i, :len(order)] = order
        scores[i, :len(order)] = sc[i][order]
        count[i] = len(order)
    return ids, scores, count


@pytest.fixture(scope="module")
def hand():
    with open(os.path.join(GOLD, "hand_worked.json")) as f:
        return json.load(f)


def test_hand_worked_case(hand):
    S = _csr(hand["S"], hand["n_dims"])
    R = _csr(hand["R"], hand["n_dims"])
    for k, key in ((2, "k2"), (4, "k4")):
        ids, scores, count = oracle.bf_topk(R, S, k)
        assert ids.tolist() == hand[key]["ids"]
        assert scores.tolist() == hand[key]["scores"]
        assert count.tolist() == hand[key]["count"]


def test_hand_worked_iiib_walk(hand):
    S = models.csr_to_lists(_csr(hand["S"], hand["n_dims"]))
    R = models.csr_to_lists(_csr(hand["R"], hand["n_dims"]))
    ex = hand["iiib_r0_theta7_gt"]
    # MinPruneScore 7 supplied as a seed on a single-query block
    res, st = models.bnl_join([R[0]], S, 2, "iiib", rule="gt", seed=[7])
    assert st["indexed"] == ex["indexed"]
    assert st["postings_walked"] == ex["postings_walked"]
    assert st["completion_entries"] == ex["completion_entries"]
    assert [list(t) for t in res[0]] == ex["result"]
    _, st_iib = models.bnl_join([R[0]], S, 2, "iib")
    assert st_iib["postings_walked"] == ex["iib_postings_walked"]
    sd = hand["iiib_r0_seed8"]
    res_gt, st_gt = models.bnl_join([R[0]], S, 2, "iiib", rule="gt", seed=[8])
    res_ge, st_ge = models.bnl_join([R[0]], S, 2, "iiib", rule="ge", seed=[8])
    assert (len(st_gt["fallbacks"]) == 1) == sd["gt_fallback"]
    assert (len(st_ge["fallbacks"]) == 1) == sd["ge_fallback"]
    assert [list(t) for t in res_gt[0]] == sd["result"] == [list(t) for t in res_ge[0]]


def _universe():
    rows = []
    for states in itertools.product((0, 1, 2), repeat=3):
        r = [(d, w) for d, w in enumerate(states) if w > 0]
        if r:
            rows.append(r)
    return rows


def test_exhaustive_universe_all_k():
    """All 26 non-empty vectors over 3 dims with values {1,2}, as both R and S, every k."""
    U = _csr(_universe(), 3)
    assert U.n_rows == 26
    for k in range(1, 28):
        ids, scores, count = oracle.bf_topk(U, U, k)
        e_ids, e_scores, e_count = _dense_topk(U, U, k)
        np.testing.assert_array_equal(ids, e_ids)
        np.testing.assert_array_equal(scores, e_scores)
        np.testing.assert_array_equal(count, e_count)


def test_streaming_form_equals_sort_form():
    """Algorithm 2's streaming insert (strict > pruneScore, ascending scan) == sort form."""
    U = models.csr_to_lists(_csr(_universe(), 3))
    for k in (1, 2, 3, 5, 9, 26, 30):
        stream, _ = models.bnl_join(U, U, k, "bf", r_block=4, s_block=5)
        assert stream == models.brute_force_sorted(U, U, k)


@pytest.mark.parametrize("r_block,s_block", [(1, 1), (3, 4), (26, 7), (100, 100)])
def test_theorem1_iib_iiib_equal_bf_every_order(r_block, s_block):
    """Theorem 1: IIB and IIIB give the brute-force result, for every dimension order."""
    U = models.csr_to_lists(_csr(_universe(), 3))
    for k in (1, 3, 8):
        ref = models.brute_force_sorted(U, U, k)
        res, st = models.bnl_join(U, U, k, "iib", r_block, s_block)
        assert res == ref
        for perm in itertools.permutations(range(3)):
            rank = {d: i for i, d in enumerate(perm)}
            for rule in ("gt", "ge"):
                res, st = models.bnl_join(U, U, k, "iiib", r_block, s_block, rule=rule,
                                          order_key=lambda d, f, rank=rank: (rank[d],))
                assert res == ref, (k, perm, rule)
                assert not st["fallbacks"]


def test_seeded_threshold_ge_rule_exact_for_every_theta():
    """Any seed: result exact after the survivor check; seeds <= true k-th never fall back."""
    U = models.csr_to_lists(_csr(_universe(), 3))
    for k in (1, 4):
        ref = models.brute_force_sorted(U, U, k)
        kth = [r[-1][0] if len(r) == k else 0 for r in ref]
        for theta in range(0, 11):
            seed = [theta] * len(U)
            for r_block in (1, 5):
                res, st = models.bnl_join(U, U, k, "iiib", r_block, 6, rule="ge", seed=seed)
                assert res == ref
                expect_fb = {i for i in range(len(U)) if theta > kth[i] or len(ref[i]) < k}
                assert set(st["fallbacks"]) <= expect_fb
                if r_block == 1:
                    assert set(st["fallbacks"]) == {i for i in expect_fb if theta > 0}
        # an unreachable seed sends every query with a non-empty result to fallback
        res, st = models.bnl_join(U, U, k, "iiib", 3, 6, rule="ge", seed=[10 ** 9] * len(U))
        assert res == ref and len(st["fallbacks"]) == len(U)


def test_eq4_and_eq3_work_terms():
    rng = np.random.default_rng(7)
    R = synth.draw(11, 30, 40, (1, 9))
    S = synth.draw(12, 50, 40, (1, 9))
    Rl, Sl = models.csr_to_lists(R), models.csr_to_lists(S)
    _, st = models.bnl_join(Rl, Sl, 3, "iib", 7, 11)
    assert st["postings_walked"] == oracle.postings_walked(R, S)
    _, st = models.bnl_join(Rl, Sl, 3, "bf", 7, 11)
    c2 = sum(len(r) + len(s) for r in Rl for s in Sl)
    assert st["merge_steps"] == c2
    del rng


def test_planted_maximum_u8():
    """s* = support(r) with every value 255 is top-1 with score 255 * sum_d r[d]."""
    S = synth.make("tiny", "S", n_rows=3000)
    R = synth.make("tiny", "R", n_rows=40)
    rng = np.random.default_rng(3)
    for q in range(R.n_rows):
        d, w = R.row(q)
        pos = int(rng.integers(0, S.n_rows + 1))
        rows = [list(zip(*S.row(j))) for j in range(S.n_rows)]
        rows.insert(pos, [(int(x), 255) for x in d])
        S2 = _csr(rows, S.n_dims)
        ids, scores, count = oracle.bf_topk(R, S2, 3, q, q + 1)
        assert ids[0, 0] == pos
        assert scores[0, 0] == 255 * int(w.astype(np.int64).sum())
        if q > 4:
            break


def test_planted_self_cosine_f32():
    """L2-normalised values: a copy of r in S scores 1 (Cauchy-Schwarz), and is top-1."""
    S = synth.draw(5, 2000, 3000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    R = synth.draw(6, 5, 3000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    for q in range(R.n_rows):
        rows = [list(zip(*S.row(j))) for j in range(S.n_rows)]
        rows.insert(17, list(zip(*R.row(q))))
        S2 = _csr(rows, S.n_dims, dtype=np.float32)
        ids, scores, count = oracle.bf_topk(R, S2, 5, q, q + 1)
        assert ids[0, 0] == 17
        assert abs(scores[0, 0] - 1.0) < 1e-6
        assert np.all(np.diff(scores[0]) <= 0)


def test_scipy_cross_check_tiny_prefix():
    sp = pytest.importorskip("scipy.sparse")
    S = synth.make("tiny", "S", n_rows=4000)
    R = synth.make("tiny", "R", n_rows=60)
    k = 10
    ids, scores, count = oracle.bf_topk(R, S, k)
    Sm = sp.csr_matrix((S.values.astype(np.int64), S.indices, S.indptr), shape=(S.n_rows, S.n_dims))
    Rm = sp.csr_matrix((R.values.astype(np.int64), R.indices, R.indptr), shape=(R.n_rows, R.n_dims))
    sc = (Rm @ Sm.T).toarray()
    for i in range(R.n_rows):
        order = np.lexsort((np.arange(S.n_rows), -sc[i]))
        order = order[sc[i][order] > 0][:k]
        assert count[i] == len(order)
        np.testing.assert_array_equal(ids[i, :len(order)], order)
        np.testing.assert_array_equal(scores[i, :len(order)], sc[i][order])
        assert np.all(ids[i, len(order):] == -1)


def test_scipy_cross_check_f32():
    sp = pytest.importorskip("scipy.sparse")
    S = synth.draw(15, 3000, 5000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    R = synth.draw(16, 20, 5000, (30, 300), features="zipf", zipf_s=1.05, values="f32")
    ids, scores, count = oracle.bf_topk(R, S, 50)
    Sm = sp.csr_matrix((S.values.astype(np.float64), S.indices, S.indptr), shape=(S.n_rows, S.n_dims))
    Rm = sp.csr_matrix((R.values.astype(np.float64), R.indices, R.indptr), shape=(R.n_rows, R.n_dims))
    sc = (Rm @ Sm.T).toarray()
    for i in range(R.n_rows):
        np.testing.assert_allclose(scores[i], sc[i][ids[i]], rtol=1e-12)
        assert scores[i, -1] >= np.sort(sc[i])[::-1][49] * (1 - 1e-12)


def test_scores_one_matches_topk():
    S = synth.make("tiny", "S", n_rows=2000)
    R = synth.make("tiny", "R", n_rows=5)
    ids, scores, count = oracle.bf_topk(R, S, 10)
    for q in range(R.n_rows):
        all_sc = oracle.scores_one(R, S, q)
        np.testing.assert_array_equal(all_sc[ids[q, :count[q]]], scores[q, :count[q]])
        assert (all_sc > scores[q, count[q] - 1]).sum() < 10
