"""Pins of the oracle's centroid graph, its best-first search and steps 2-4 of
the gather from given top lists (oracle/gather.py): hand-worked graphs, the
search reaching the exact set when its beam covers every centroid, greedy walks
on a path graph (including a stop at a local maximum), and agreement with the
whole gather."""
import numpy as np

import oracle
from oracle.gather import beam_search, gather_from_top, knn_graph


def test_knn_graph_hand_worked():
    # 1-d "centroids" 3, 1, 2, -1: <c_i, c_j> = c_i c_j
    C = np.array([[3.0], [1.0], [2.0], [-1.0]])
    assert knn_graph(C, deg=1).tolist() == [[2, 1], [0, 3], [0, -1], [1, -1]]
    assert knn_graph(C, deg=2).tolist() == [[2, 1, -1, -1], [0, 2, 3, -1], [0, 1, 3, -1], [1, 2, -1, -1]]


def test_knn_graph_ties_to_lower_id():
    C = np.ones((3, 1))
    assert knn_graph(C, deg=1).tolist() == [[1, 2], [0, -1], [0, -1]]


def test_knn_graph_invariants():
    rng = np.random.default_rng(1)
    C = rng.standard_normal((60, 8))
    deg = 5
    g = knn_graph(C, deg)
    S = C @ C.T
    for i in range(60):
        f = g[i, :deg]
        others = np.delete(np.arange(60), i)
        assert np.allclose(np.sort(S[i, f])[::-1], np.sort(S[i, others])[::-1][:deg])
        assert np.all(np.diff(S[i, f]) <= 0)
        r = g[i, deg:][g[i, deg:] >= 0]
        for j in r:
            assert i in g[j, :deg] and j not in f
        cand = [j for j in range(60) if i in g[j, :deg] and j not in f]
        assert len(r) == min(deg, len(cand))


def test_beam_covering_every_centroid_is_exact():
    rng = np.random.default_rng(2)
    C = rng.standard_normal((50, 16))
    g = knn_graph(C, 4)
    for t in range(5):
        q = rng.standard_normal(16)
        ids, sims = beam_search(q, C, g, np.arange(50), ef=50, kc=7)
        ei, es = oracle.top_centroids(q[None], C, 7)
        assert np.array_equal(ids, ei[0]) and np.allclose(sims, es[0])
        # a complete graph: one expansion sees every centroid
        full = np.array([[j for j in range(50) if j != i] for i in range(50)])
        ids2, _ = beam_search(q, C, full, np.array([t]), ef=7, kc=7)
        assert np.array_equal(ids2, ei[0])


def test_greedy_walk_on_a_path():
    path = np.array([[-1, 1]] + [[i - 1, i + 1] for i in range(1, 9)] + [[8, -1]])
    C = np.arange(10, dtype=np.float64)[:, None]
    ids, sims = beam_search(np.array([1.0]), C, path, np.array([0]), ef=1, kc=1)
    assert ids.tolist() == [9] and sims.tolist() == [9.0]
    # a local maximum stops a one-entry beam: 10 is never reached
    C2 = np.array([[0.0], [5.0], [1.0], [10.0]])
    path2 = np.array([[-1, 1], [0, 2], [1, 3], [2, -1]])
    ids, _ = beam_search(np.array([1.0]), C2, path2, np.array([0]), ef=1, kc=1)
    assert ids.tolist() == [1]
    ids, _ = beam_search(np.array([1.0]), C2, path2, np.array([0]), ef=2, kc=2)   # a wider beam walks past it
    assert ids.tolist() == [3, 1]
    ids, sims = beam_search(np.array([1.0]), C2, path2, np.array([0]), ef=4, kc=5)
    assert ids.tolist() == [3, 1, 2, 0, -1] and sims[-1] == -np.inf


def test_gather_from_top_agrees_with_gather():
    rng = np.random.default_rng(3)
    K, D = 40, 12
    C = rng.standard_normal((K, 16))
    assign = rng.integers(0, K, 300)
    doc = np.sort(rng.integers(0, D, 300))
    off, docs = oracle.inverted_lists(assign, doc, K)
    for kc, kd in ((1, 3), (5, 12), (40, 20)):
        Q = rng.standard_normal((6, 16))
        ids, sims = oracle.top_centroids(Q, C, kc)
        d0, s0 = oracle.gather(Q, C, off, docs, kc, kd)
        d1, s1 = gather_from_top(ids, sims, off, docs, kd)
        assert np.array_equal(d0, d1) and np.allclose(s0, s1)
    # an empty slot adds nothing
    ids[:, -1] = -1
    d2, _ = gather_from_top(ids, sims, off, docs, 20)
    d3, _ = oracle.gather(Q, C, off, docs, kc - 1, 20) if kc > 1 else (d2, None)
    assert np.array_equal(d2, d3)
