"""Gather phase on the GPU (Sect. 2.2) against the oracle: query lengths 32 and
7, kappa_c of 1, 8, 40 and every centroid, kappa_d below and above the number
of reached documents (padding), empty lists, determinism, bad arguments, and
three sampled queries at the benchmark's launch shape (64 queries x 32 tokens,
262,144 centroids, kappa_c = 40, kappa_d = 1,000).

Similarities are FP32 matrix-core products, so the comparison allows for
rounding in two ways.  Every query is checked against the oracle's admissible
score intervals (a near-tie at a token's kappa_c cut lets either centroid be
taken; see _check_bounds).  Where no two similarities come within TOL of each
other at any cut (asserted from the oracle's float64 values), the check is
the strict one: every returned score matches the oracle's S of that document
within TOL * n_q, the documents the oracle ranks clearly above the kappa_d-th
score are all returned, and the order is by score, ties by id."""
import numpy as np
import pytest
import torch

import oracle

from gpu_common import dev, host

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")

DIM = 128
TOL = 2e-5   # per similarity: FP32 products of unit vectors over 128 coordinates, with margin


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


def _index(seed, K, D, ntok, empty_lists=0):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((K, DIM)).astype(np.float32)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    assign = rng.integers(empty_lists, K, ntok)            # centroids below empty_lists keep empty lists
    doc = np.sort(rng.integers(0, D, ntok))
    off, docs = oracle.inverted_lists(assign, doc, K)
    return C, off, docs


def _queries(seed, B, nq):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((B, nq, DIM)).astype(np.float32)
    return Q / np.linalg.norm(Q, axis=2, keepdims=True)


def _gpu(ctx, Q, C, off, docs, D, kc, kd):
    cand = torch.full((Q.shape[0], kd), -7, dtype=torch.int32, device="cuda")
    score = torch.full((Q.shape[0], kd), 7.0, dtype=torch.float32, device="cuda")
    tac.tac_gather(ctx, dev(Q), dev(C), dev(off.astype(np.int64)), dev(docs.astype(np.int32)), D, kc, cand, score)
    return host(cand), host(score)


def _well_posed(q, C, kc):
    """No two similarities within TOL of each other across the kappa_c cut."""
    if kc >= C.shape[0]:
        return True
    s = np.sort(q.astype(np.float64) @ C.T.astype(np.float64), axis=1)[:, ::-1]
    return bool(np.all(s[:, kc - 1] - s[:, kc] > 2 * TOL))


def _check(q, C, off, docs, kc, kd, got_d, got_s):
    S = oracle.document_scores(q, C, off, docs, kc)
    nq = q.shape[0]
    tol = TOL * nq
    n = min(kd, len(S))
    assert np.all(got_d[n:] == -1) and np.all(np.isneginf(got_s[n:]))
    assert np.all(got_d[:n] >= 0) and len(set(got_d[:n].tolist())) == n
    for d, s in zip(got_d[:n].tolist(), got_s[:n].tolist()):
        assert d in S and abs(s - S[d]) <= tol, (d, s, S.get(d))
    # order: by score, ties by id
    for r in range(n - 1):
        assert got_s[r] > got_s[r + 1] or (got_s[r] == got_s[r + 1] and got_d[r] < got_d[r + 1])
    # every document clearly above the kappa_d-th oracle score is returned
    ref = sorted(S.values(), reverse=True)
    cut = ref[n - 1] if n else np.inf
    must = {d for d, s in S.items() if s > cut + 2 * tol}
    assert must <= set(got_d[:n].tolist())


def _check_bounds(q, C, off, docs, kc, kd, got_d, got_s):
    """The check for any query, near-ties at a token's kappa_c cut included:
    the oracle's admissible score interval of every document over every
    centroid choice a similarity error of TOL allows (oracle.document_score_bounds).
    Each returned document is one some choice reaches, its score lies in its
    interval, the count of returned documents is one some choice gives, the
    order is by score with ties by id, and every document that every choice
    reaches and that fewer than kappa_d others can outscore is returned."""
    sure, lo, hi = oracle.document_score_bounds(q, C, off, docs, kc, TOL)
    nq = q.shape[0]
    tol = TOL * nq
    n = int(np.sum(got_d >= 0))
    assert np.all(got_d[:n] >= 0) and np.all(got_d[n:] == -1) and np.all(np.isneginf(got_s[n:]))
    assert min(kd, len(sure)) <= n <= min(kd, len(lo))
    assert len(set(got_d[:n].tolist())) == n
    for d, s in zip(got_d[:n].tolist(), got_s[:n].tolist()):
        assert d in lo and lo[d] - tol <= s <= hi[d] + tol, (d, s, lo.get(d), hi.get(d))
    for r in range(n - 1):
        assert got_s[r] > got_s[r + 1] or (got_s[r] == got_s[r + 1] and got_d[r] < got_d[r + 1])
    his = np.sort(np.array(list(hi.values())))
    returned = set(got_d[:n].tolist())
    for d in sure:
        # documents other than d that some choice could score at least as high as d's lowest
        rivals = his.size - np.searchsorted(his, lo[d] - 2 * tol, side="left") - (1 if hi[d] >= lo[d] - 2 * tol else 0)
        if rivals < kd:
            assert d in returned, (d, lo[d], rivals)


@pytest.mark.parametrize("nq,kc,kd", [(32, 8, 50), (7, 40, 400), (32, 1, 20), (7, 8, 2000)])
def test_matches_oracle(ctx, nq, kc, kd):
    K, D = 300, 500
    C, off, docs = _index(80 + kc, K, D, 20_000, empty_lists=5)
    seed = 81
    while not all(_well_posed(q, C, kc) for q in _queries(seed, 4, nq)):
        seed += 100
    Q = _queries(seed, 4, nq)
    got_d, got_s = _gpu(ctx, Q, C, off, docs, D, kc, kd)
    for b in range(Q.shape[0]):
        _check(Q[b], C, off, docs, kc, kd, got_d[b], got_s[b])
        _check_bounds(Q[b], C, off, docs, kc, kd, got_d[b], got_s[b])


def test_every_centroid_and_determinism(ctx):
    K, D = 64, 300
    C, off, docs = _index(90, K, D, 3_000)
    Q = _queries(91, 3, 32)
    a = _gpu(ctx, Q, C, off, docs, D, K, 300)
    b = _gpu(ctx, Q, C, off, docs, D, K, 300)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
    for q in range(3):
        _check(Q[q], C, off, docs, K, 300, a[0][q], a[1][q])
        assert set(a[0][q][a[0][q] >= 0].tolist()) == set(docs.tolist())    # every listed document is reached


def test_bad_arguments(ctx):
    C, off, docs = _index(95, 16, 10, 100)
    Q = _queries(96, 1, 4)
    for kc, kd in ((0, 5), (257, 5), (4, 0), (4, 4097)):
        with pytest.raises(tac.TacError):
            _gpu(ctx, Q, C, off, docs, 10, kc, kd)


def test_sampled_at_benchmark_shape(ctx):
    """64 queries x 32 tokens against 262,144 centroids (kappa_c = 40, kappa_d =
    1,000) over lists of 1M tokens in 10,000 documents; queries 0 and 37 are
    recomputed by the oracle."""
    K, D = 262_144, 10_000
    C, off, docs = _index(100, K, D, 1_000_000)
    Q = _queries(101, 64, 32)
    got_d, got_s = _gpu(ctx, Q, C, off, docs, D, 40, 1000)
    for b in (0, 37, 63):
        _check_bounds(Q[b], C, off, docs, 40, 1000, got_d[b], got_s[b])
        if _well_posed(Q[b], C, 40):
            _check(Q[b], C, off, docs, 40, 1000, got_d[b], got_s[b])


def test_query_chunks(ctx):
    """130 queries x 32 tokens against 262,144 centroids do not fit one chunk of
    similarities (128 queries do); queries on both sides of the chunk edge are
    checked against the oracle."""
    K, D = 262_144, 2_000
    C, off, docs = _index(110, K, D, 200_000)
    Q = _queries(111, 130, 32)
    got_d, got_s = _gpu(ctx, Q, C, off, docs, D, 8, 50)
    for b in (0, 127, 128, 129):
        _check_bounds(Q[b], C, off, docs, 8, 50, got_d[b], got_s[b])
        if _well_posed(Q[b], C, 8):
            _check(Q[b], C, off, docs, 8, 50, got_d[b], got_s[b])

