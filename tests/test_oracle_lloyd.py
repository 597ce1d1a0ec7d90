"""Pins for the oracle's per-token Lloyd iteration and the canonical FP32 distance."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import dist32
from oracle.budget import BudgetParams


def _tiny_index(K=300, name="tiny"):
    x, tok = datagen.make(name)
    w = datagen.WORKLOADS[name]
    perm, seg_off, counts = oracle.group_by_token(tok, w.vocab)
    xs = x[perm]
    s = oracle.spreads(xs, seg_off)
    kappa = oracle.budget(counts, s, K, BudgetParams(mu=20, tau=60, eps=2, theta=10.0))
    cent_off = oracle.cent_offsets(kappa)
    picks = datagen.init_picks(counts, kappa, 0)
    C0 = oracle.init_centroids(xs, seg_off, cent_off, picks)
    return xs, seg_off, counts, s, kappa, cent_off, C0


def test_dist32_exact_on_dyadic():
    rng = np.random.default_rng(0)
    X = (rng.integers(-64, 65, (50, 128)) / 8).astype(np.float32)
    C = (rng.integers(-64, 65, (30, 128)) / 8).astype(np.float32)
    exact = ((X[:, None, :].astype(np.float64) - C[None].astype(np.float64)) ** 2).sum(-1)
    assert np.array_equal(dist32.pairwise(X, C).astype(np.float64), exact)


def test_dist32_rounding_bound():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((200, 128)).astype(np.float32)
    C = rng.standard_normal((40, 128)).astype(np.float32)
    exact = ((X[:, None, :].astype(np.float64) - C[None].astype(np.float64)) ** 2).sum(-1)
    err = np.abs(dist32.pairwise(X, C) - exact)
    assert np.all(err <= 130 * 2.0 ** -24 * exact)
    assert np.array_equal(dist32.rowwise(X[:40], C), np.diagonal(dist32.pairwise(X[:40], C)))


def test_assign_matches_direct_definition():
    """The float64 matrix-product form agrees with sum_i (x_i - c_i)^2 loops."""
    xs, seg_off, counts, s, kappa, cent_off, C0 = _tiny_index()
    r = oracle.assign(xs, seg_off, C0, cent_off, topk=3)
    rng = np.random.default_rng(2)
    for i in rng.choice(xs.shape[0], 60, replace=False):
        j = np.searchsorted(seg_off, i, side="right") - 1
        best, bestd = -1, np.inf
        for k in range(cent_off[j], cent_off[j + 1]):
            dd = sum((float(xs[i, t]) - float(C0[k, t])) ** 2 for t in range(128))
            if dd < bestd:
                best, bestd = k, dd
        assert r["a"][i] == best
        assert abs(r["D"][i] - bestd) <= 1e-12
        assert r["top_idx"][i, 0] == best


def test_fp32_decision_pruned_equals_full():
    xs, seg_off, counts, s, kappa, cent_off, C0 = _tiny_index()
    a = oracle.assign(xs, seg_off, C0, cent_off, decide="fp32")
    b = oracle.assign(xs, seg_off, C0, cent_off, decide="fp32", full_fp32=True)
    assert np.array_equal(a["a"], b["a"])
    assert np.array_equal(a["d32"], b["d32"])
    # every fp32 decision is a float64 tie at worst
    c = oracle.assign(xs, seg_off, C0, cent_off, decide="fp64")
    assert np.all(a["D"] - c["D"] < 1e-5)


def test_one_centroid_per_token_closed_form():
    """kappa_j = 1 for every present token: one update gives the token means, and
    the inertia after it is sum_j n_j s_j (spread of Sect. 2.1)."""
    x, tok = datagen.make("tiny")
    perm, seg_off, counts = oracle.group_by_token(tok, 40)
    xs = x[perm]
    s = oracle.spreads(xs, seg_off)
    kappa = (counts > 0).astype(np.int64)
    cent_off = oracle.cent_offsets(kappa)
    rng = np.random.default_rng(3)
    C0 = rng.standard_normal((int(kappa.sum()), 128)).astype(np.float32)
    r0 = oracle.assign(xs, seg_off, C0, cent_off)
    C1, cnt = oracle.update(xs, r0["a"], C0)
    r1 = oracle.assign(xs, seg_off, C1, cent_off)
    present = np.nonzero(counts)[0]
    assert np.array_equal(cnt, counts[present])
    for c, j in enumerate(present):
        mean = xs[seg_off[j]:seg_off[j + 1]].astype(np.float64).mean(axis=0)
        assert np.array_equal(C1[c], mean.astype(np.float32))
    expect = float((counts * s).sum())
    assert abs(r1["J"] - expect) <= 1e-9 * expect


def test_every_row_its_own_centroid():
    rng = np.random.default_rng(4)
    xs = rng.standard_normal((90, 128)).astype(np.float32)
    seg_off = np.array([0, 30, 90])
    cent_off = np.array([0, 30, 90])
    r = oracle.assign(xs, seg_off, xs.copy(), cent_off)
    assert r["J"] == 0.0 and np.array_equal(r["a"], np.arange(90))
    C1, cnt = oracle.update(xs, r["a"], xs)
    assert np.array_equal(C1, xs) and np.all(cnt == 1)


def test_inertia_non_increasing_and_empty_keep():
    xs, seg_off, counts, s, kappa, cent_off, C0 = _tiny_index()
    steps = oracle.lloyd(xs, seg_off, cent_off, C0, iters=10)
    J = [st["J"] for st in steps]
    for a, b in zip(J, J[1:]):
        assert b <= a * (1 + 1e-12)
    for st in steps[:-1]:
        empty = st["counts"] == 0
        assert np.array_equal(st["C_new"][empty], st["C"][empty])
        # assignments stay inside the row's own token
        seg = np.searchsorted(seg_off, np.arange(xs.shape[0]), side="right") - 1
        assert np.all(st["a"] >= cent_off[seg]) and np.all(st["a"] < cent_off[seg + 1])


def test_single_token_matches_textbook_lloyd():
    """T = 1 is plain Lloyd: scikit-learn's Lloyd from the same start agrees."""
    sk = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(5)
    centers = rng.standard_normal((6, 128)) * 3
    X = (centers[rng.integers(0, 6, 1200)] + rng.standard_normal((1200, 128)) * 0.3).astype(np.float32)
    init = X[rng.choice(1200, 6, replace=False)]
    steps = oracle.lloyd(X, np.array([0, 1200]), np.array([0, 6]), init, iters=10)
    km = sk.KMeans(6, init=init.astype(np.float64), n_init=1, max_iter=10, tol=0.0,
                   algorithm="lloyd").fit(X.astype(np.float64))
    assert np.array_equal(km.labels_, steps[-1]["a"])
    assert np.allclose(km.cluster_centers_, steps[-1]["C"], rtol=0, atol=1e-6)


def test_empty_cluster_keeps_previous_centroid():
    x = np.zeros((3, 128), dtype=np.float32)
    x[:, 0] = [0.0, 0.125, 10.0]
    C = np.zeros((2, 128), dtype=np.float32)
    C[:, 0] = [0.0, 100.0]
    r = oracle.assign(x, np.array([0, 3]), C, np.array([0, 2]))
    C1, cnt = oracle.update(x, r["a"], C)
    assert cnt.tolist() == [3, 0]
    assert C1[1, 0] == 100.0 and C1[0, 0] == np.float32((0.0 + 0.125 + 10.0) / 3)


def test_inertia_closed_forms():
    """oracle.inertia (the within-cluster sum of squares of Sect. 2.1) against
    values fixed independently of it: at the token means it equals sum_j n_j s_j
    built from the two-pass spreads, on dyadic 1-D points it equals the
    hand-computed sum, and a row that is its own centroid adds nothing."""
    x, tok = datagen.make("tiny")
    perm, seg_off, counts = oracle.group_by_token(tok, 40)
    xs = x[perm]
    s = oracle.spreads(xs, seg_off)
    present = np.nonzero(counts)[0]
    means = np.stack([xs[seg_off[j]:seg_off[j + 1]].astype(np.float64).mean(axis=0) for j in present])
    a = np.repeat(np.arange(present.size), counts[present])
    # the means kept in float64 (inertia promotes, so no rounding enters the comparison)
    J = oracle.inertia(xs, a, means)
    expect = float((counts * s).sum())
    assert abs(J - expect) <= 1e-10 * expect
    # 1-D dyadic points 0, 1/2, 3 against centroids 1/4 and 3: (1/4)^2 + (1/4)^2 + 0 = 1/8 exactly
    X = np.zeros((3, 128), np.float32)
    X[:, 0] = [0.0, 0.5, 3.0]
    Cd = np.zeros((2, 128), np.float32)
    Cd[:, 0] = [0.25, 3.0]
    assert oracle.inertia(X, np.array([0, 0, 1]), Cd) == 0.125
    # a wrong assignment costs the squared gap: point 3 to centroid 1/4 adds (11/4)^2
    assert oracle.inertia(X, np.array([0, 0, 0]), Cd) == 0.125 + (2.75 ** 2)
    rng = np.random.default_rng(6)
    R = rng.standard_normal((20, 128)).astype(np.float32)
    assert oracle.inertia(R, np.arange(20), R) == 0.0


def test_smallest_k_is_stable_argsort_prefix():
    """The top-k selection used for the float64 tie report equals the first k
    entries of a stable argsort, including ties across the k-th position."""
    from oracle.lloyd import _smallest_k
    rng = np.random.default_rng(7)
    D = rng.integers(0, 40, (300, 500)).astype(np.float64)   # many equal values
    for kk in (1, 8, 37):
        assert np.array_equal(_smallest_k(D, kk), np.argsort(D, axis=1, kind="stable")[:, :kk])
    D2 = rng.standard_normal((50, 70))
    assert np.array_equal(_smallest_k(D2, 8), np.argsort(D2, axis=1, kind="stable")[:, :8])
