"""Brute-force pins of the oracle's per-token Lloyd on tiny 1-D inputs.

Values are dyadic (k/8, |k| <= 64), embedded as coordinate 0 of a 128-d
zero vector, so every float operation on them is exact.  For each token the
test enumerates all kappa^n labelings to find the optimal within-cluster sum
of squares (Sect. 2.1) and its optimal partitions.
"""
import itertools

import numpy as np

import oracle

D = 128


def embed(vals):
    x = np.zeros((len(vals), D), dtype=np.float32)
    x[:, 0] = vals
    return x


def wcss(vals, labels, k):
    tot = 0.0
    for c in range(k):
        m = [v for v, l in zip(vals, labels) if l == c]
        if m:
            mu = sum(m) / len(m)
            tot += sum((v - mu) ** 2 for v in m)
    return tot


def optimal(vals, k):
    best, parts = np.inf, []
    for lab in itertools.product(range(k), repeat=len(vals)):
        if len(set(lab)) < k:          # every centroid used (n >= k)
            continue
        j = wcss(vals, lab, k)
        if j < best - 1e-12:
            best, parts = j, [lab]
        elif abs(j - best) <= 1e-12:
            parts.append(lab)
    return best, parts


def canonical(vals, lab):
    """Partition as a frozenset of frozensets of positions."""
    groups = {}
    for i, l in enumerate(lab):
        groups.setdefault(l, set()).add(i)
    return frozenset(frozenset(g) for g in groups.values())


def cases(seed, ntok=4):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(ntok):
        n = int(rng.integers(3, 9))
        k = int(rng.integers(1, min(3, n) + 1))
        vals = [float(v) / 8 for v in rng.integers(-64, 65, n)]
        out.append((vals, k))
    return out


def build(tok_cases):
    vals = [v for vs, _ in tok_cases for v in vs]
    seg_off = np.cumsum([0] + [len(vs) for vs, _ in tok_cases])
    cent_off = np.cumsum([0] + [k for _, k in tok_cases])
    return embed(vals), seg_off, cent_off


def test_optimal_partitions_contiguous_and_fixed_points():
    for seed in range(12):
        for vals, k in cases(seed):
            best, parts = optimal(vals, k)
            order = np.argsort(vals, kind="stable")
            for lab in parts:
                # contiguous in sorted order (ties of equal values may interleave)
                sv = [vals[i] for i in order]
                sl = [lab[i] for i in order]
                for c in set(sl):
                    pos = [p for p, l in enumerate(sl) if l == c]
                    lo, hi = pos[0], pos[-1]
                    assert all(sl[p] == c or sv[p] in (sv[lo], sv[hi]) for p in range(lo, hi + 1))
                # a Lloyd fixed point: every point is (weakly) nearest to its own mean
                means = np.zeros((k, D))
                for c in range(k):
                    m = [v for v, l in zip(vals, lab) if l == c]
                    means[c, 0] = sum(m) / len(m)
                x = embed(vals)
                r = oracle.assign(x, np.array([0, len(vals)]), means, np.array([0, k]))
                own = np.array([(vals[i] - means[lab[i], 0]) ** 2 for i in range(len(vals))])
                assert np.allclose(r["D"], own, rtol=0, atol=1e-12)


def test_lloyd_never_beats_optimum_and_planted_groups_reach_it():
    for seed in range(12):
        tc = cases(seed)
        x, seg_off, cent_off = build(tc)
        rng = np.random.default_rng(100 + seed)
        init = []
        for j, (vals, k) in enumerate(tc):
            pick = rng.choice(len(vals), k, replace=False)
            init.extend(x[seg_off[j] + pick])
        steps = oracle.lloyd(x, seg_off, cent_off, np.array(init), iters=10)
        Jstar = sum(optimal(vals, k)[0] for vals, k in tc)
        assert steps[-1]["J"] >= Jstar - 1e-12
    # planted groups: gaps larger than k * (widest group) -> Lloyd from one point
    # per group finds the optimum exactly
    groups = [[-6.0, -5.875, -5.75], [0.0, 0.125], [5.0, 5.25, 5.125, 5.0]]
    vals = [v for g in groups for v in g]
    x = embed(vals)
    init = embed([g[0] for g in groups])
    steps = oracle.lloyd(x, np.array([0, len(vals)]), np.array([0, 3]), init, iters=10)
    Jstar, parts = optimal(vals, 3)
    assert abs(steps[-1]["J"] - Jstar) <= 1e-12
    assert canonical(vals, steps[-1]["a"].tolist()) in {canonical(vals, p) for p in parts}


def test_exact_ties_go_to_lowest_index():
    x = embed([1.0, 3.0, 2.0])
    C = embed([1.0, 3.0])              # 2.0 is equidistant from both centroids
    r = oracle.assign(x, np.array([0, 3]), C, np.array([0, 2]))
    assert r["a"].tolist() == [0, 1, 0]
    r32 = oracle.assign(x, np.array([0, 3]), C, np.array([0, 2]), decide="fp32")
    assert r32["a"].tolist() == [0, 1, 0]
