"""The speed-up of token-aware clustering over global k-means (Sect. 2.1,
"Theoretical Lower Bound for Speed-up") on the real budget of the 10M-row
workload: N = 10,000,000 rows over 30,522 Zipf(1.0) token ids, K = 262,144.

One Lloyd iteration of global k-means computes N * K distances; the
token-aware one computes sum_j n_j * kappa_j.  Their ratio is the speed-up in
work.  The paper bounds it from below by sum_j w_j / max_j w_j for the
proportional allocation kappa_j = w_j / W * K (floors and tail handling set
aside): sum_j n_j kappa_j <= K / W * max_j w_j * sum_j n_j.

The counts come from the seeded token generator; the spreads of the active
tokens (n_j >= 256, the only ones the budget weighs) from a fixture the oracle
wrote (tests/golden/make_c1_token_stats.py)."""
import os

import numpy as np
import pytest

import datagen
import oracle
from oracle.budget import BudgetParams

FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "c1_token_stats.txt")
P = BudgetParams()          # mu 128, tau 256, eps 4, theta 39


@pytest.fixture(scope="module")
def c1_stats():
    w = datagen.WORKLOADS["c1"]
    counts = np.bincount(datagen.tokens(w.n, w.vocab, w.zipf_s, w.seed), minlength=w.vocab).astype(np.int64)
    with open(FIXTURE) as f:
        rows = np.array([ln.split() for ln in f if not ln.startswith("#")])
    ids = rows[:, 0].astype(np.int64)
    assert np.array_equal(rows[:, 1].astype(np.int64), counts[ids]), "fixture counts differ from the generator"
    assert np.array_equal(ids, np.nonzero(counts >= P.tau)[0]), "fixture must hold exactly the active tokens"
    spread = np.zeros(w.vocab)
    spread[ids] = rows[:, 2].astype(np.float64)
    return w, counts, spread


def test_bound_holds_for_the_proportional_allocation(c1_stats):
    """The paper's inequality on the real counts and spreads: the active tokens
    share what Phase 1 leaves (B) in proportion to w_j = sqrt(n_j) s_j, with no
    floor and no bound; their work ratio is at least W / max w."""
    w, counts, spread = c1_stats
    act = counts >= P.tau
    n = counts[act].astype(np.float64)
    wj = np.sqrt(n) * spread[act]
    tail = int(((counts > 0) & (counts < P.mu)).sum() + 2 * ((counts >= P.mu) & (counts < P.tau)).sum())
    B = w.k - tail
    kappa = wj / wj.sum() * B
    ratio = n.sum() * B / float((n * kappa).sum())
    bound = wj.sum() / wj.max()
    assert ratio >= bound * (1 - 1e-12)
    # the inequality is tight only when every row sits in the heaviest token; here it has slack
    assert ratio > 1.5 * bound


def test_real_budget_work_ratio(c1_stats):
    """The reconciled budget (Phases 1-4) under the default theta policy is not
    proportional.  This workload has N / K = 38.1 rows per centroid, below
    theta = 39, so the caps floor(n_j / theta) of the active tokens hold only
    204,393 of the B = 231,613 units Phase 1 leaves: Phase 4 fills every active
    token to its cap before it relaxes the caps for the remaining 27,220 units,
    and the largest token gets 23,485 = floor(915,946 / 39) centroids instead of
    its proportional 1,841.  The work ratio (73.95) then falls below W / max w
    (125.8): the paper's bound assumes the proportional allocation.  What the
    same derivation gives for any allocation, N K / sum n_j kappa_j >=
    K / max kappa_j, holds."""
    w, counts, spread = c1_stats
    info = {}
    kappa = oracle.budget(counts, spread, w.k, P, info=info)
    assert kappa.sum() == w.k and kappa.max() == 23_485
    assert info["B"] == 231_613 and info["tier2"] == 27_220
    act = counts >= P.tau
    caps = np.maximum(P.eps, np.floor(counts / P.theta)).astype(np.int64)
    assert caps[act].sum() == 204_393
    assert np.all(kappa[act] >= caps[act])
    N = int(counts.sum())
    ratio = N * w.k / float((counts * kappa).sum())
    assert ratio >= w.k / kappa.max()
    wj = np.sqrt(counts[act].astype(np.float64)) * spread[act]
    assert ratio < wj.sum() / wj.max()
    assert 73.9 < ratio < 74.0


def test_soft_policy_keeps_the_bound(c1_stats):
    """With the soft theta policy (theta dropped when its caps cannot hold B)
    the allocation stays close to proportional, the largest token gets its
    proportional 1,841 centroids, and the work ratio (583.5) clears W / max w."""
    w, counts, spread = c1_stats
    kappa = oracle.budget(counts, spread, w.k, BudgetParams(policy=1))
    assert kappa.sum() == w.k and kappa.max() == 1_841
    act = counts >= P.tau
    ratio = int(counts.sum()) * w.k / float((counts * kappa).sum())
    wj = np.sqrt(counts[act].astype(np.float64)) * spread[act]
    assert ratio >= wj.sum() / wj.max()


def test_host_budget_matches_oracle_on_c1(c1_stats):
    """The library's host budget gives the oracle's allocation on the real statistics."""
    tac = pytest.importorskip("paper_2604_28142_amd")
    w, counts, spread = c1_stats
    for policy in (0, 1):
        got, tier2 = tac.tac_budget_from_stats(counts, spread, w.k, tac.BudgetParams(theta_policy=policy))
        assert np.array_equal(got, oracle.budget(counts, spread, w.k, BudgetParams(policy=policy)))
        assert tier2 == (27_220 if policy == 0 else 0)
