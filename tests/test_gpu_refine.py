"""Refine-phase MaxSim on the GPU (Sect. 2.2) against the oracle: ragged and
empty documents, tokens without a centroid, out-of-range candidates, query
lengths 1, 17 and 32, repeated candidates, determinism, and sampled scores at
the launch shape the benchmark times (64 queries x 1,000 candidates, documents
of 30-180 tokens, 262,144 centroids).

Scores are FP32 matrix-core dot products compared with the float64 oracle
within a bound derived from the arithmetic: each score's error is at most
sum_i gamma * max_t sum_k |q_ik| |x_tk| (the maximum moves by no more than
the largest error of the dots it compares; gamma = 140 u covers the rounding
of x = c + rho * u and the accumulation of 128 products) plus the rounding of
the final sum over the query tokens."""
import numpy as np
import pytest
import torch

import oracle

from gpu_common import dev, host

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")

U = 2.0 ** -24
DIM, M = 128, 32


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


def _index(seed, K, lens, ksub=256, bad_frac=0.0):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((K, DIM)).astype(np.float32)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    B = (0.2 * rng.standard_normal((M, ksub, DIM // M))).astype(np.float32)
    doc_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    N = int(doc_off[-1])
    assign = rng.integers(0, K, N).astype(np.int32)
    if bad_frac:
        bad = rng.random(N) < bad_frac
        assign[bad] = rng.choice(np.array([-1, K, K + 7], np.int32), int(bad.sum()))
    codes = rng.integers(0, ksub, (N, M)).astype(np.uint8)
    rnorm = rng.uniform(0.0, 0.6, N).astype(np.float32)
    layout = oracle.doc_layout(assign, codes, doc_off)
    return dict(C=C, B=B, doc_off=doc_off, assign=assign, codes=codes, rnorm=rnorm, layout=layout)


def _queries(seed, nb, nq):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((nb, nq, DIM)).astype(np.float32)
    return Q / np.linalg.norm(Q, axis=2, keepdims=True)


def _gpu(ctx, ix, Q, cand):
    scores = torch.full(cand.shape, 12345.0, dtype=torch.float32, device="cuda")
    tac.tac_maxsim(ctx, dev(Q), dev(ix["C"]), dev(ix["B"]), dev(ix["layout"]), dev(ix["doc_off"]),
                   dev(ix["rnorm"]), dev(cand.astype(np.int32)), scores)
    return host(scores)


def _tolerance(ix, q, d):
    """Error bound of one score (see the module docstring)."""
    t0, t1 = int(ix["doc_off"][d]), int(ix["doc_off"][d + 1])
    K = ix["C"].shape[0]
    a = ix["assign"][t0:t1]
    keep = (a >= 0) & (a < K)
    if not keep.any():
        return 0.0
    a = a[keep].astype(np.int64)
    codes = ix["codes"][t0:t1][keep]
    u = np.concatenate([ix["B"][m][codes[:, m]] for m in range(M)], axis=1).astype(np.float64)
    x = ix["C"][a].astype(np.float64) + ix["rnorm"][t0:t1][keep][:, None].astype(np.float64) * u
    bound = np.abs(q.astype(np.float64)) @ np.abs(x).T          # [nq, tokens]
    best = (q.astype(np.float64) @ x.T).max(axis=1)
    return 140 * U * bound.max(axis=1).sum() + 2 * q.shape[0] * U * np.abs(best).sum()


def _check(ix, Q, cand, got):
    for b in range(Q.shape[0]):
        ref = oracle.maxsim_scores(Q[b], ix["C"], ix["B"], ix["layout"], ix["doc_off"], ix["rnorm"], cand[b])
        for j, d in enumerate(cand[b].tolist()):
            D = ix["doc_off"].size - 1
            if not 0 <= d < D:
                assert np.isnan(got[b, j]), (b, j, d)
            elif np.isinf(ref[j]):
                assert got[b, j] == ref[j], (b, j, d)
            else:
                tol = _tolerance(ix, Q[b], d)
                assert abs(float(got[b, j]) - ref[j]) <= tol, (b, j, d, float(got[b, j]), ref[j], tol)


@pytest.mark.parametrize("nq", [32, 17, 1])
def test_matches_oracle_ragged_documents(ctx, nq):
    rng = np.random.default_rng(40 + nq)
    lens = rng.integers(0, 70, 60)
    lens[[3, 11]] = 0                               # empty documents
    lens[[5, 6, 7]] = [1, 16, 17]                   # one token, a full block, a block and one
    ix = _index(41 + nq, 300, lens, bad_frac=0.05)
    D = lens.size
    ix["assign"][ix["doc_off"][20]:ix["doc_off"][21]] = -1          # a document with no scored token
    ix["layout"] = oracle.doc_layout(ix["assign"], ix["codes"], ix["doc_off"])
    Q = _queries(42 + nq, 3, nq)
    cand = np.stack([rng.permutation(D)[:45] for _ in range(3)]).astype(np.int64)
    cand[0, :4] = [3, 20, D, -1]                     # empty, nothing scored, out of range twice
    cand[1, 10:14] = cand[1, 0]                      # repeats
    got = _gpu(ctx, ix, Q, cand)
    _check(ix, Q, cand, got)
    assert np.isneginf(got[0, 0]) and np.isneginf(got[0, 1]) and np.isnan(got[0, 2]) and np.isnan(got[0, 3])
    assert np.all(got[1, 10:14] == got[1, 0])


def test_small_codebooks_and_determinism(ctx):
    rng = np.random.default_rng(50)
    lens = rng.integers(1, 200, 40)
    ix = _index(51, 64, lens, ksub=16)
    Q = _queries(52, 5, 32)
    cand = np.stack([rng.integers(0, lens.size, 37) for _ in range(5)]).astype(np.int64)
    a = _gpu(ctx, ix, Q, cand)
    b = _gpu(ctx, ix, Q, cand)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    _check(ix, Q, cand, a)


def test_bad_arguments(ctx):
    ix = _index(60, 8, np.array([3, 4]))
    cand = np.zeros((1, 2), np.int64)
    for nq in (0, 33):
        Q = np.zeros((1, max(nq, 1), DIM), np.float32) if nq else np.zeros((1, 0, DIM), np.float32)
        with pytest.raises(tac.TacError):
            _gpu(ctx, ix, Q, cand)


def test_sampled_at_benchmark_shape(ctx):
    """64 queries x 1,000 candidates (the benchmark's launch shape) over 20,000
    documents of 30-180 tokens and 262,144 centroids; one sampled candidate per
    query is recomputed by the oracle."""
    rng = np.random.default_rng(70)
    lens = rng.integers(30, 181, 20_000)
    K = 262_144
    ix = _index(71, K, lens)
    Q = _queries(72, 64, 32)
    cand = np.stack([rng.choice(lens.size, 1000, replace=False) for _ in range(64)]).astype(np.int64)
    got = _gpu(ctx, ix, Q, cand)
    assert np.all(np.isfinite(got))
    pick = rng.integers(0, 1000, 64)
    for b in range(64):
        d = int(cand[b, pick[b]])
        ref = oracle.maxsim_scores(Q[b], ix["C"], ix["B"], ix["layout"], ix["doc_off"], ix["rnorm"], [d])[0]
        assert abs(float(got[b, pick[b]]) - ref) <= _tolerance(ix, Q[b], d), (b, d)
