"""Pins for the oracle's per-token budget (Sect. 2.1, Phases 1-4)."""
import json
import math
import os

import numpy as np
import pytest

from oracle.budget import (BudgetParams, Infeasible, POLICY_SOFT, budget)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "budget_examples.json")


def _params(case):
    return BudgetParams(mu=case.get("mu", 128), tau=case.get("tau", 256), eps=case.get("eps", 4),
                        theta=float(case.get("theta", 39)), policy=case["policy"])


def test_hand_worked_examples():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        k = budget(c["counts"], c["spread"], c["K"], _params(c))
        assert k.tolist() == c["kappa"], c["steps"]


def _random_case(rng, T=300):
    counts = np.where(rng.random(T) < 0.1, 0, np.floor(20000 * (np.arange(1, T + 1) ** -1.1))).astype(np.int64)
    rng.shuffle(counts)
    spread = rng.uniform(0.01, 0.5, T)
    return counts, spread


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("policy", [0, 1])
def test_invariants(seed, policy):
    rng = np.random.default_rng(seed)
    counts, spread = _random_case(rng)
    p = BudgetParams(policy=policy)
    active = counts >= p.tau
    tail = int(((counts > 0) & (counts < p.mu)).sum() + 2 * ((counts >= p.mu) & (counts < p.tau)).sum())
    lo_K = tail + p.eps * int(active.sum())
    hi_K = tail + int(counts[active].sum())
    for K in np.linspace(lo_K, hi_K, 7).astype(int):
        info = {}
        k = budget(counts, spread, int(K), p, info=info)
        assert k.sum() == K
        assert np.all(k[counts == 0] == 0)
        assert np.all(k[(counts > 0) & (counts < p.mu)] == 1)
        assert np.all(k[(counts >= p.mu) & (counts < p.tau)] == 2)
        assert np.all(k[active] >= p.eps)
        assert np.all(k <= counts)
        assert np.all(k[counts > 0] >= 1)
        caps = np.maximum(p.eps, np.floor(counts / p.theta)).astype(np.int64)
        if policy == 0 and info["tier2"] == 0:
            assert np.all(k[active] <= caps[active])
        if policy == 0 and info["tier2"] > 0:
            # theta is relaxed only once every active token sits at its cap
            assert np.all(k[active] >= caps[active])


def test_infeasible():
    counts = [1000, 400, 300, 200, 100, 50]
    spread = [0.5] * 6
    with pytest.raises(Infeasible):
        budget(counts, spread, 4 + 3 * 4 - 1)      # below tail + eps per active token
    with pytest.raises(Infeasible):
        budget(counts, spread, 4 + 1700 + 1)        # more centroids than active vectors
    budget(counts, spread, 4 + 12)
    budget(counts, spread, 4 + 1700)


def test_no_bounds_closed_form():
    """Without tail, floor or cap, kappa_j = floor(w_j / W * B) whenever the
    floors already sum to B; and the speed-up bound of Sect. 2.1 holds:
    N * K / sum n_j kappa_j >= W / max w."""
    p = BudgetParams(mu=0, tau=0, eps=0, theta=0.0)
    n = np.array([4, 16, 4, 64, 256])           # sqrt: 2, 4, 2, 8, 16 -> W = 32
    s = np.ones(5)
    K = 32
    k = budget(n, s, K, p)
    assert k.tolist() == [2, 4, 2, 8, 16]
    w = np.sqrt(n) * s
    assert n.sum() * K / (n * k).sum() >= w.sum() / w.max()


@pytest.mark.parametrize("lam", [0.25, 2.0, 1024.0])
def test_scale_invariance(lam):
    """w_j / W does not change when every spread is scaled (powers of two keep it exact)."""
    rng = np.random.default_rng(7)
    counts, spread = _random_case(rng)
    for K in (3000, 9000):
        assert np.array_equal(budget(counts, spread, K), budget(counts, spread * lam, K))


def test_zero_spread_falls_back_to_sqrt_n():
    k = budget([1024, 256], [0.0, 0.0], 12, BudgetParams(theta=0.0))
    # w = sqrt(n) = [32, 16], q = [8, 4]
    assert k.tolist() == [8, 4]


def test_soft_policy_differs_only_when_caps_cannot_hold_B():
    counts = [1000, 400, 300, 200, 100, 50]
    spread = [0.5, 0.5, 0.8, 0.3, 0.9, 0.2]
    # sum of caps 42 >= B = 36: both policies agree
    assert np.array_equal(budget(counts, spread, 40), budget(counts, spread, 40, BudgetParams(policy=POLICY_SOFT)))


def test_damping_favours_rare_tokens():
    """sqrt damping: a token 4x more frequent with equal spread gets 2x the share."""
    k = budget([40000, 10000], [0.5, 0.5], 3000, BudgetParams(theta=0.0))
    assert k.tolist() == [2000, 1000]
    assert math.isclose(k[0] / k[1], 2.0)
