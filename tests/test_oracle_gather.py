"""Pins of the gather-phase oracle (Sect. 2.2): a hand-worked example with a
tie at the centroid cut, a brute force over a document x centroid incidence
matrix, and invariants of the definition."""
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hand_example():
    fx = json.load(open(os.path.join(HERE, "golden", "gather_example.json")))
    ids, sims = oracle.top_centroids(fx["Q"], fx["C"], fx["kc"])
    assert ids.tolist() == fx["top_ids"] and sims.tolist() == fx["top_sims"]
    docs, scores = oracle.gather(fx["Q"], fx["C"], fx["list_off"], fx["list_docs"], fx["kc"], fx["kd"])
    assert docs.tolist() == fx["docs"] and scores.tolist() == fx["scores"]


def _index(seed, K=60, D=40, dim=8, nq=5, per_doc=6):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((K, dim))
    Q = rng.standard_normal((nq, dim))
    assign = rng.integers(0, K, D * per_doc)
    doc = np.repeat(np.arange(D), per_doc)
    off, docs = oracle.inverted_lists(assign, doc, K)
    return Q, C, off, docs, D


def _brute(Q, C, off, docs, D, kc):
    """S over all documents from an incidence matrix: A[d, j] = d in L_j."""
    K = C.shape[0]
    A = np.zeros((D, K), bool)
    for j in range(K):
        A[docs[off[j]:off[j + 1]], j] = True
    sims = Q @ C.T
    S = np.zeros(D)
    reached = np.zeros(D, bool)
    for i in range(Q.shape[0]):
        order = np.argsort(-sims[i], kind="stable")[:kc]     # stable: equal sims keep the lower id first
        keep = np.zeros(K, bool)
        keep[order] = True
        M = np.where(A & keep[None, :], sims[i][None, :], -np.inf)
        best = M.max(axis=1)
        hit = np.isfinite(best)
        S[hit] += best[hit]
        reached |= hit
    return S, reached


@pytest.mark.parametrize("seed,kc", [(0, 3), (1, 10), (2, 1)])
def test_matches_incidence_brute_force(seed, kc):
    Q, C, off, docs, D = _index(seed)
    S = oracle.document_scores(Q, C, off, docs, kc)
    ref, reached = _brute(Q, C, off, docs, D, kc)
    assert sorted(S) == np.nonzero(reached)[0].tolist()
    for d, s in S.items():
        assert abs(s - ref[d]) <= 1e-12 * (1 + abs(ref[d]))
    kd = 7
    got_d, got_s = oracle.gather(Q, C, off, docs, kc, kd)
    order = sorted(np.nonzero(reached)[0].tolist(), key=lambda d: (-ref[d], d))[:kd]
    assert got_d[:len(order)].tolist() == order


def test_all_centroids_reach_every_listed_document():
    Q, C, off, docs, D = _index(3)
    K = C.shape[0]
    S = oracle.document_scores(Q, C, off, docs, K)
    assert sorted(S) == sorted(set(docs.tolist()))
    sims = Q @ C.T
    for d in list(S)[:10]:
        cents = [j for j in range(K) if d in docs[off[j]:off[j + 1]].tolist()]
        assert abs(S[d] - sum(max(sims[i, j] for j in cents) for i in range(Q.shape[0]))) <= 1e-12


def test_scaling_list_order_and_padding():
    Q, C, off, docs, D = _index(4)
    d0, s0 = oracle.gather(Q, C, off, docs, 4, 10)
    d1, s1 = oracle.gather(3.0 * Q, C, off, docs, 4, 10)
    assert d0.tolist() == d1.tolist() and np.allclose(s1, 3.0 * s0, rtol=1e-12)
    rev = np.concatenate([docs[off[j]:off[j + 1]][::-1] for j in range(C.shape[0])])   # lists in any order
    d2, s2 = oracle.gather(Q, C, off, rev, 4, 10)
    assert d2.tolist() == d0.tolist() and np.array_equal(s2, s0)
    dn, sn = oracle.gather(Q, C, off, docs, 1, 10_000)
    n = len(oracle.document_scores(Q, C, off, docs, 1))
    assert np.all(dn[n:] == -1) and np.all(np.isneginf(sn[n:])) and np.all(dn[:n] >= 0)
    assert np.all(np.diff(sn[:n]) <= 0)


def test_score_bounds_exact_without_tolerance():
    """With no rounding allowance and distinct similarities the admissible
    interval collapses to the oracle's score, and every document is sure."""
    for seed, kc in ((0, 3), (1, 10), (5, 1)):
        Q, C, off, docs, D = _index(seed)
        S = oracle.document_scores(Q, C, off, docs, kc)
        sure, lo, hi = oracle.document_score_bounds(Q, C, off, docs, kc, 0.0)
        assert sure == set(S) and set(lo) == set(S) and set(hi) == set(S)
        for d, s in S.items():
            assert lo[d] == hi[d] and abs(lo[d] - s) <= 1e-12 * (1 + abs(s))


def _near_tie_index(seed, nq=2, dim=6, K=14, D=12):
    """Centroid pairs whose similarities to every query token differ by about
    1e-4, so that a tolerance of 1e-3 makes the centroids at the cut optional."""
    rng = np.random.default_rng(seed)
    base = rng.standard_normal((K // 2, dim))
    C = np.concatenate([base, base * (1 + 1e-4 * rng.standard_normal((K // 2, 1)))])
    Q = rng.standard_normal((nq, dim))
    assign = rng.integers(0, K, D * 3)
    doc = np.repeat(np.arange(D), 3)
    off, docs = oracle.inverted_lists(assign, doc, K)
    return Q, C, off, docs, D


@pytest.mark.parametrize("seed,kc", [(10, 3), (11, 4), (12, 2)])
def test_score_bounds_cover_every_admissible_choice(seed, kc):
    """Brute force over every centroid choice an implementation with similarity
    error up to tol may make: each choice takes the kc centroids of largest
    perturbed similarity, so it keeps every centroid above v + 2 tol, none below
    v - 2 tol, and exactly kc in all.  Every document score of every choice lies
    in [lo, hi], every sure document is reached by every choice, and every
    document some choice reaches has bounds."""
    import itertools
    tol = 1e-3
    Q, C, off, docs, D = _near_tie_index(seed)
    sure, lo, hi = oracle.document_score_bounds(Q, C, off, docs, kc, tol)
    sims = Q @ C.T
    K = C.shape[0]
    per_token = []
    for i in range(Q.shape[0]):
        v = np.sort(sims[i])[::-1][kc - 1]
        must = [j for j in range(K) if sims[i, j] > v + 2 * tol]
        maybe = [j for j in range(K) if v - 2 * tol <= sims[i, j] <= v + 2 * tol]
        assert len(maybe) >= 2, "the fixture must leave a choice at the cut"
        choices = [set(must) | set(a) for a in itertools.combinations(maybe, kc - len(must))]
        per_token.append(choices)
    seen = set()
    for combo in itertools.product(*per_token):
        S = {}
        for i, chosen in enumerate(combo):
            best = {}
            for j in chosen:
                for d in docs[off[j]:off[j + 1]].tolist():
                    best[d] = max(best.get(d, -np.inf), sims[i, j])
            for d, s in best.items():
                S[d] = S.get(d, 0.0) + s
        assert sure <= set(S)
        for d, s in S.items():
            seen.add(d)
            assert lo[d] - 1e-12 <= s <= hi[d] + 1e-12, (d, s, lo[d], hi[d])
    assert seen == set(lo) == set(hi)
