"""Slow pure-Python walks of the paper's algorithms.  TEST INFRASTRUCTURE ONLY.

These follow Algorithms 1-4 (Sec. 4) step by step, in the paper's order, on
small inputs.  They exist to pin readings of the paper (tie order, the
selection rule, the IIIB split condition, the learned-seed survivor rule)
against the brute-force definition, and to count the work terms of Eq. 2-4.

Vectors are lists of (d, w) pairs in ascending d with w > 0 (Sec. 3).
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional, Sequence, Tuple

Vec = List[Tuple[int, float]]


def csr_to_lists(m) -> List[Vec]:
    out = []
    for i in range(len(m.indptr) - 1):
        b, e = int(m.indptr[i]), int(m.indptr[i + 1])
        vals = m.values[b:e]
        cast = int if getattr(vals, "dtype", None) is not None and vals.dtype.kind in "iu" else float
        out.append([(int(d), cast(w)) for d, w in zip(m.indices[b:e], vals)])
    return out


def dot(r: Vec, s: Vec):
    """dot(r, s) by the two-pointer merge of Algorithm 2 (its dot() routine)."""
    ret = 0
    a = b = 0
    while a < len(r) and b < len(s):
        if r[a][0] == s[b][0]:
            ret += r[a][1] * s[b][1]
            a += 1
            b += 1
        elif r[a][0] > s[b][0]:
            b += 1
        else:
            a += 1
    return ret


class Candidates:
    """The KNN candidate set of one r with its pruneScore (the candidate step of
    Algorithm 2).

    pruneScore is the score of the k-th candidate once k are held, else 0
    (Algorithm 1 initialises it to 0).  A vector enters only if its
    score is strictly greater; the set keeps the k best by (score desc, id asc).
    """

    def __init__(self, k: int):
        self.k = k
        self.items: List[Tuple[float, int]] = []  # (score, id)

    def prune_score(self):
        return self.items[-1][0] if len(self.items) == self.k else 0

    def offer(self, s: int, v) -> None:
        if v > self.prune_score():
            self.items.append((v, s))
            self.items.sort(key=lambda t: (-t[0], t[1]))
            del self.items[self.k:]


def brute_force_sorted(R: List[Vec], S: List[Vec], k: int):
    """The definition in 'sort form': all scores, keep > 0, sort (score desc, id asc), take k."""
    out = []
    for r in R:
        sc = [(dot(r, s), j) for j, s in enumerate(S)]
        sc = [t for t in sc if t[0] > 0]
        sc.sort(key=lambda t: (-t[0], t[1]))
        out.append(sc[:k])
    return out


def _blocks(n: int, size: int):
    size = max(1, size)
    return [range(i, min(n, i + size)) for i in range(0, n, size)]


def bnl_join(R: List[Vec], S: List[Vec], k: int, algo: str = "bf", r_block: int = 1 << 30, s_block: int = 1 << 30,
             rule: str = "ge", order_key: Optional[Callable[[int, Dict[int, int]], tuple]] = None,
             seed: Optional[Sequence[float]] = None, max_weight: Optional[Callable[[int], float]] = None):
    """Block nested loop join (Algorithm 1) with BF, IIB or IIIB as the in-memory join.

    algo: "bf" (Algorithm 2), "iib" (Algorithm 3) or "iiib" (Algorithm 4).
    rule: IIIB split condition, "gt" (index once t > MinPruneScore, as printed in
      Algorithm 4) or "ge" (index once t >= threshold).
    order_key(d, freq): sort key for the dimension order in Create_Inverted_List_IIIB;
      default (-freq_d(B_r), d), i.e. most frequent in B_r first.
    seed: optional per-query threshold guesses; the IIIB block threshold is then
      min over B_r of max(pruneScore(r), seed(r)), and a query whose final list
      has fewer than k entries or a k-th score below the largest threshold
      applied to its block is recomputed without the seed (fallback).
    max_weight(d): optional replacement for maxWeight_d(B_r) (any upper bound
      of the block's weights).

    Returns (results, stats) where results[i] is a list of (score, id) and stats
    counts postings walked, entries indexed, completion entries and fallbacks.
    """
    stats = dict(postings_walked=0, indexed=0, completion_entries=0, candidates=0, merge_steps=0,
                 fallbacks=[])
    results: List[List[Tuple[float, int]]] = [None] * len(R)  # type: ignore
    for rb in _blocks(len(R), r_block):                       # Alg. 1: outer loop over R blocks
        cand = {i: Candidates(k) for i in rb}                  # empty lists, pruneScore 0
        theta_max = {i: 0 for i in rb}
        for sb in _blocks(len(S), s_block):                    # inner loop over S blocks
            _join_blocks(R, S, rb, sb, cand, algo, rule, order_key, seed, max_weight, stats, theta_max)
        for i in rb:                                           # output of the block
            res = cand[i].items
            if seed is not None and (len(res) < k or res[-1][0] < theta_max[i]):
                stats["fallbacks"].append(i)
                sub, _ = bnl_join([R[i]], S, k, algo, 1, s_block, rule, order_key, None, max_weight)
                res = sub[0]
            results[i] = [(v, s) for (v, s) in res]
    return results, stats


def _join_blocks(R, S, rb, sb, cand, algo, rule, order_key, seed, max_weight, stats, theta_max):
    if algo == "bf":                                           # Algorithm 2
        for i in rb:
            for j in sb:
                stats["merge_steps"] += len(R[i]) + len(S[j])
                cand[i].offer(j, dot(R[i], S[j]))
        return
    if algo == "iib":                                          # Algorithm 3
        inv: Dict[int, List[Tuple[int, float]]] = {}
        for j in sb:                                           # Create_Inverted_List_IIB
            for d, w in S[j]:
                inv.setdefault(d, []).append((j, w))
        for i in rb:                                           # Find_Matches_IIB
            A: Dict[int, float] = {}
            for d, rw in R[i]:
                for j, w in inv.get(d, []):
                    A[j] = A.get(j, 0) + rw * w
                    stats["postings_walked"] += 1
            for j in sorted(A):
                if A[j] != 0:
                    stats["candidates"] += 1
                    cand[i].offer(j, A[j])
        return
    assert algo == "iiib"                                      # Algorithm 4
    # MinPruneScore over the block (Sec. 4.4), optionally raised by per-query seeds
    thr = []
    for i in rb:
        p = cand[i].prune_score()
        if seed is not None:
            p = max(p, seed[i])
        thr.append(p)
    theta = min(thr)
    for i in rb:
        theta_max[i] = max(theta_max[i], theta)
    # Create_Inverted_List_IIIB: dimension order and maxWeight_d(B_r)
    freq: Dict[int, int] = {}
    maxw: Dict[int, float] = {}
    for i in rb:
        for d, w in R[i]:
            freq[d] = freq.get(d, 0) + 1
            maxw[d] = max(maxw.get(d, 0), w)
    key = order_key if order_key is not None else (lambda d, f: (-f.get(d, 0), d))
    inv = {}
    rest: Dict[int, Vec] = {}
    for j in sb:
        t = 0
        kept: Vec = []
        for d, w in sorted(S[j], key=lambda f: key(f[0], freq)):
            mw = max_weight(d) if max_weight is not None else maxw.get(d, 0)
            t += mw * w
            if (t > theta) if rule == "gt" else (t >= theta):
                inv.setdefault(d, []).append((j, w))           # index, and remove from s
                stats["indexed"] += 1
            else:
                kept.append((d, w))
        rest[j] = sorted(kept)
    for i in rb:                                               # Find_Matches_IIIB
        A = {}
        for d, rw in R[i]:
            for j, w in inv.get(d, []):
                A[j] = A.get(j, 0) + rw * w
                stats["postings_walked"] += 1
        for j in sorted(A):
            if A[j] != 0:
                stats["candidates"] += 1
                stats["completion_entries"] += len(rest[j])
                A[j] = A[j] + dot(R[i], rest[j])               # unindexed features
                cand[i].offer(j, A[j])
