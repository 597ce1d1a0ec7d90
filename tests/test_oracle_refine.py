"""Pins of the refine (MaxSim over PQ-coded documents) oracle (Sect. 2.2): a
hand-worked example, a brute-force decode of every token vector, and
invariants that hold for the definition."""
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixture():
    return json.load(open(os.path.join(HERE, "golden", "maxsim_example.json")))


def test_hand_example():
    fx = _fixture()
    T = oracle.distance_tables(np.asarray(fx["Q"], float), np.asarray(fx["codebooks"], float))
    assert T.tolist() == fx["tables"]
    s = oracle.maxsim_scores(fx["Q"], fx["C"], np.asarray(fx["codebooks"], float),
                             np.asarray(fx["layout"], np.uint8), fx["doc_off"], fx["rnorm"], fx["cand"])
    assert s.tolist() == fx["scores"]
    # candidate ids that name no document score NaN
    s = oracle.maxsim_scores(fx["Q"], fx["C"], np.asarray(fx["codebooks"], float),
                             np.asarray(fx["layout"], np.uint8), fx["doc_off"], fx["rnorm"], [4, -1, 0])
    assert np.isnan(s[0]) and np.isnan(s[1]) and s[2] == 10.0


def _problem(seed, dim=16, M=4, ksub=8, K=10, nq=5, D=12, maxlen=6, bad_ids=False):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((K, dim))
    B = rng.standard_normal((M, ksub, dim // M))
    Q = rng.standard_normal((nq, dim))
    lens = rng.integers(0, maxlen + 1, D)
    doc_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    N = int(doc_off[-1])
    assign = rng.integers(-2 if bad_ids else 0, K + (2 if bad_ids else 0), N)
    codes = rng.integers(0, ksub, (N, M)).astype(np.uint8)
    rnorm = rng.uniform(0.0, 2.0, N)
    return C, B, Q, doc_off, assign, codes, rnorm


def _layout(assign, codes, doc_off):
    return oracle.doc_layout(np.asarray(assign, np.int32), codes, doc_off)


def _brute(C, B, Q, doc_off, assign, codes, rnorm, cand):
    """The definition with every token vector decoded: x = c_a + rho * concat_m B[m, code_m]."""
    K, M = C.shape[0], B.shape[0]
    out = []
    for d in cand:
        best = [None] * Q.shape[0]
        for t in range(int(doc_off[d]), int(doc_off[d + 1])):
            if not 0 <= assign[t] < K:
                continue
            u = np.concatenate([B[m, codes[t, m]] for m in range(M)])
            x = C[assign[t]] + rnorm[t] * u
            for i in range(Q.shape[0]):
                v = float(sum(Q[i, k] * x[k] for k in range(x.size)))
                best[i] = v if best[i] is None else max(best[i], v)
        out.append(-np.inf if best[0] is None else sum(best))
    return np.asarray(out)


@pytest.mark.parametrize("seed,bad", [(0, False), (1, False), (2, True)])
def test_matches_brute_force_decode(seed, bad):
    C, B, Q, doc_off, assign, codes, rnorm = _problem(seed, bad_ids=bad)
    cand = np.arange(doc_off.size - 1)[::-1]
    got = oracle.maxsim_scores(Q, C, B, _layout(assign, codes, doc_off), doc_off, rnorm, cand)
    ref = _brute(C, B, Q, doc_off, assign, codes, rnorm, cand)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    assert np.allclose(got[fin], ref[fin], rtol=1e-12, atol=1e-12)


def test_token_order_does_not_matter():
    C, B, Q, doc_off, assign, codes, rnorm = _problem(3)
    rng = np.random.default_rng(30)
    perm = np.arange(assign.size)
    for d in range(doc_off.size - 1):                 # shuffle tokens inside every document
        a, b = int(doc_off[d]), int(doc_off[d + 1])
        perm[a:b] = a + rng.permutation(b - a)
    cand = np.arange(doc_off.size - 1)
    s0 = oracle.maxsim_scores(Q, C, B, _layout(assign, codes, doc_off), doc_off, rnorm, cand)
    s1 = oracle.maxsim_scores(Q, C, B, _layout(assign[perm], codes[perm], doc_off), doc_off, rnorm[perm], cand)
    assert np.allclose(s0, s1, rtol=1e-12, atol=1e-12)


def test_zero_norms_give_the_centroid_only_score():
    C, B, Q, doc_off, assign, codes, rnorm = _problem(4)
    cand = np.arange(doc_off.size - 1)
    s = oracle.maxsim_scores(Q, C, B, _layout(assign, codes, doc_off), doc_off, np.zeros_like(rnorm), cand)
    for j, d in enumerate(cand):
        a = assign[int(doc_off[d]):int(doc_off[d + 1])]
        if a.size == 0:
            assert s[j] == -np.inf
        else:
            assert np.isclose(s[j], (Q @ C[a].T).max(axis=1).sum(), rtol=1e-12, atol=1e-12)


def test_one_query_token_is_a_maximum_and_scaling_is_linear():
    C, B, Q, doc_off, assign, codes, rnorm = _problem(5, nq=1)
    lay = _layout(assign, codes, doc_off)
    cand = np.arange(doc_off.size - 1)
    s = oracle.maxsim_scores(Q, C, B, lay, doc_off, rnorm, cand)
    s2 = oracle.maxsim_scores(2.5 * Q, C, B, lay, doc_off, rnorm, cand)
    fin = np.isfinite(s)
    assert np.allclose(s2[fin], 2.5 * s[fin], rtol=1e-12, atol=1e-12)
    # a single-token document scores the plain inner product
    for j, d in enumerate(cand):
        if doc_off[d + 1] - doc_off[d] == 1:
            t = int(doc_off[d])
            x = C[assign[t]] + rnorm[t] * np.concatenate([B[m, codes[t, m]] for m in range(B.shape[0])])
            assert np.isclose(s[j], float(Q[0] @ x), rtol=1e-12, atol=1e-12)


def test_candidates_are_independent():
    C, B, Q, doc_off, assign, codes, rnorm = _problem(6)
    lay = _layout(assign, codes, doc_off)
    all_s = oracle.maxsim_scores(Q, C, B, lay, doc_off, rnorm, np.arange(doc_off.size - 1))
    cand = np.asarray([3, 3, 0, 7, 3])
    s = oracle.maxsim_scores(Q, C, B, lay, doc_off, rnorm, cand)
    assert np.array_equal(s, all_s[cand])
