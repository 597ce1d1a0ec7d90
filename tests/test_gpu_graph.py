"""GPU centroid graph and its search (the gather's step 1 in place of the
paper's HNSW, Sect. 2.2) against the oracle: the built neighbour table, the
beam search (agreement with the oracle's search on the same graph, validity of
every returned similarity, recall of the exact top-kappa_c), steps 2-4 from
given top lists, and bad arguments.

Similarities are float32 on the GPU and float64 in the oracle, so lists are
compared up to near-ties (two similarities within TOL may come in either
order) and the search must agree with the oracle's on nearly every query
token (a near-tie can send the two walks different ways)."""
import numpy as np
import pytest
import torch

import oracle
from oracle.gather import beam_search, gather_from_top, knn_graph

from gpu_common import dev, host

pytestmark = pytest.mark.gpu

tac = pytest.importorskip("paper_2604_28142_amd")

DIM, DEG = 128, 32
TOL = 2e-5


@pytest.fixture(scope="module")
def ctx():
    c = tac.Context(0)
    yield c
    c.close()


def clustered_centroids(seed, groups, per_group, spread=0.25):
    """Unit vectors around `groups` random centres (a token's centroids sit
    together); returns (C float32 [K, 128], first centroid of every group)."""
    rng = np.random.default_rng(seed)
    cen = rng.standard_normal((groups, DIM))
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    sizes = rng.integers(1, 2 * per_group, groups)
    C = np.concatenate([cen[g] + spread / np.sqrt(DIM) * rng.standard_normal((n, DIM)) for g, n in enumerate(sizes)])
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    first = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    return C.astype(np.float32), first.astype(np.int32), cen


def gpu_graph(ctx, C):
    nbr = torch.full((C.shape[0], 2 * DEG), -7, dtype=torch.int32, device="cuda")
    tac.tac_graph_build(ctx, dev(C), nbr)
    return host(nbr)


def test_graph_build_matches_oracle(ctx):
    rng = np.random.default_rng(4)
    C = rng.standard_normal((1500, DIM)).astype(np.float32)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    g = gpu_graph(ctx, C)
    ref = knn_graph(C.astype(np.float64), DEG)
    S = C.astype(np.float64) @ C.T.astype(np.float64)
    np.fill_diagonal(S, -np.inf)
    for i in range(C.shape[0]):
        f, fo = g[i, :DEG], ref[i, :DEG]
        cut = S[i, fo[-1]]
        # the same set up to near-ties at the cut, in order up to near-ties
        assert np.all(S[i, f] >= cut - TOL) and len(set(f.tolist())) == DEG and i not in f
        if np.sum(np.abs(S[i] - cut) < TOL) == 1:
            assert set(f.tolist()) == set(fo.tolist()), i
        assert np.all(np.diff(S[i, f]) <= TOL)
    # reverse edges follow the GPU's own forward lists exactly (structure), by similarity up to near-ties
    fwd = [set(g[j, :DEG].tolist()) for j in range(C.shape[0])]
    for i in range(C.shape[0]):
        r = g[i, DEG:]
        r = r[r >= 0]
        cand = [j for j in range(C.shape[0]) if i in fwd[j] and j not in fwd[i]]
        assert set(r.tolist()) <= set(cand) and len(r) == min(DEG, len(cand))
        if len(cand) > DEG:
            dropped = set(cand) - set(r.tolist())
            assert S[i, r].min() >= max(S[i, list(dropped)]) - TOL
        assert np.all(np.diff(S[i, r]) <= TOL)
        assert np.all(g[i, DEG + len(r):] == -1)


def _search(ctx, Q, C, nbr_d, entry, ef, kc):
    top_id = torch.full((Q.shape[0], kc), -7, dtype=torch.int32, device="cuda")
    top_sim = torch.full((Q.shape[0], kc), 7.0, dtype=torch.float32, device="cuda")
    tac.tac_graph_search(ctx, dev(Q), dev(C), nbr_d, dev(entry), ef, kc, top_id, top_sim)
    return host(top_id), host(top_sim)


def test_search_agrees_with_oracle_and_finds_the_exact_set(ctx):
    C, first, cen = clustered_centroids(5, groups=300, per_group=40)
    K = C.shape[0]
    nbr_d = torch.empty((K, 2 * DEG), dtype=torch.int32, device="cuda")
    tac.tac_graph_build(ctx, dev(C), nbr_d)
    nbr = host(nbr_d)
    rng = np.random.default_rng(6)
    groups = rng.integers(0, cen.shape[0], 200)
    Q = cen[groups] + 0.3 / np.sqrt(DIM) * rng.standard_normal((200, DIM))
    Q = (Q / np.linalg.norm(Q, axis=1, keepdims=True)).astype(np.float32)
    ef, kc = 60, 40
    ids, sims = _search(ctx, Q, C, nbr_d, first, ef, kc)
    ei, es = oracle.top_centroids(Q, C, kc)
    Cd = C.astype(np.float64)
    agree, recall = 0, []
    for r in range(Q.shape[0]):
        v = ids[r][ids[r] >= 0]
        assert len(set(v.tolist())) == len(v) and np.all(ids[r][len(v):] == -1)
        exact = Cd[v] @ Q[r].astype(np.float64)
        assert np.allclose(sims[r][:len(v)], exact, atol=TOL)          # every similarity is the centroid's own
        assert np.all(np.diff(sims[r][:len(v)]) <= 0)
        oi, _ = beam_search(Q[r], C, nbr, first, ef, kc)
        agree += np.array_equal(oi, ids[r])
        recall.append(len(set(v.tolist()) & set(ei[r].tolist())) / kc)
    assert agree >= 0.98 * Q.shape[0], agree
    assert np.mean(recall) >= 0.95, np.mean(recall)
    # deterministic
    ids2, sims2 = _search(ctx, Q, C, nbr_d, first, ef, kc)
    assert np.array_equal(ids, ids2) and np.array_equal(sims.view(np.uint32), sims2.view(np.uint32))


def test_gather_lists_matches_oracle(ctx):
    rng = np.random.default_rng(7)
    K, D, nq, B, kc, kd = 3000, 400, 8, 6, 20, 50
    C = rng.standard_normal((K, DIM)).astype(np.float32)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    assign = rng.integers(0, K, 20000)
    doc = np.sort(rng.integers(0, D, 20000))
    off, docs = oracle.inverted_lists(assign, doc, K)
    Q = rng.standard_normal((B, nq, DIM)).astype(np.float32)
    Q /= np.linalg.norm(Q, axis=2, keepdims=True)
    ids = np.empty((B, nq, kc), np.int32)
    sims = np.empty((B, nq, kc), np.float32)
    for b in range(B):
        i, s = oracle.top_centroids(Q[b], C, kc)
        ids[b], sims[b] = i, s
    ids[0, 0, -3:] = -1                      # empty slots add nothing
    cand = torch.full((B, kd), -7, dtype=torch.int32, device="cuda")
    score = torch.full((B, kd), 7.0, dtype=torch.float32, device="cuda")
    tac.tac_gather_lists(ctx, dev(ids), dev(sims), dev(off.astype(np.int64)), dev(docs.astype(np.int32)), K, D, kd,
                         cand, score)
    cand, score = host(cand), host(score)
    for b in range(B):
        d, s = gather_from_top(ids[b], sims[b].astype(np.float64), off, docs, kd)
        assert np.allclose(score[b], s, atol=TOL * nq) or np.array_equal(cand[b], d)
        ok = np.abs(s - s[-1]) > TOL * nq                    # clear of the kappa_d-th score
        assert set(d[ok & (d >= 0)].tolist()) <= set(cand[b].tolist())
        got = {int(x): float(y) for x, y in zip(cand[b], score[b]) if x >= 0}
        ref = dict(zip(d.tolist(), s.tolist()))
        for x, y in got.items():
            if x in ref:
                assert abs(ref[x] - y) <= TOL * nq


def test_exact_topk_matches_oracle(ctx):
    rng = np.random.default_rng(8)
    C = rng.standard_normal((5000, DIM)).astype(np.float32)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    Q = rng.standard_normal((70, DIM)).astype(np.float32)
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    top_id = torch.empty((70, 40), dtype=torch.int32, device="cuda")
    top_sim = torch.empty((70, 40), dtype=torch.float32, device="cuda")
    tac.tac_centroid_topk(ctx, dev(Q), dev(C), 40, top_id, top_sim)
    ti, ts = host(top_id), host(top_sim)
    ei, es = oracle.top_centroids(Q, C, 40)
    assert np.allclose(ts, es, atol=TOL)
    for r in range(70):
        if np.min(np.abs(np.diff(es[r]))) > TOL:
            assert np.array_equal(ti[r], ei[r])


def test_graph_bad_arguments(ctx):
    C = np.eye(4, DIM, dtype=np.float32)
    nbr = torch.empty((4, 2 * DEG), dtype=torch.int32, device="cuda")
    tac.tac_graph_build(ctx, dev(C), nbr)
    Q = np.eye(2, DIM, dtype=np.float32)
    for ef, kc in ((65, 10), (10, 11), (0, 1)):
        with pytest.raises(tac.TacError):
            _search(ctx, Q, C, nbr, np.array([0, 1], np.int32), ef, kc)
    ids, sims = _search(ctx, Q, C, nbr, np.array([2, 3], np.int32), 4, 4)   # K < ef: the beam holds every centroid
    assert ids[0, 0] == 0 and ids[1, 0] == 1 and sorted(ids[0].tolist()) == [0, 1, 2, 3]
