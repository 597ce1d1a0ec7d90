"""Per-token centroid budget, Phases 1-4 of Sect. 2.1 (oracle; test infrastructure only).

Phase 1 (tail handling): micro tokens (n < mu) get 1 centroid, small tokens
(mu <= n < tau) get 2, active tokens (n >= tau) are allocated dynamically.
Phase 2 (damped scoring): w_j = sqrt(n_j) * s_j and kappa_j = floor(w_j / W * B),
with B the budget left after Phase 1.
Phase 3 (bounding): kappa_j >= eps for active tokens and n_j / kappa_j >= theta.
Phase 4 (reconciliation): move surplus or deficit units so the total is K.

Readings where the paper is silent or loose (each listed in the design notes):
* W sums the weights of the *active* tokens only, since B is what is left for
  them after Phase 1.  If every active spread is 0, w_j = sqrt(n_j).
* The theta cap is hi_j = max(eps, floor(n_j / theta)), never above n_j;
  theta <= 0 means no theta cap (hi_j = n_j).
* Tail tokens get min(1, n_j) / min(2, n_j) so that no token gets more
  centroids than vectors.
* Phase 4 rule: while units are missing, add one to the eligible active token
  (kappa_j < cap_j) with the largest remaining quota p_j = q_j - kappa_j
  (ties: larger w_j, then smaller j).  When no token is below its theta cap the
  caps are relaxed to n_j ("tier 2") and the same rule continues.  While units
  are in excess, remove one from the active token with kappa_j > eps and the
  smallest p_j (ties: smaller w_j, then larger j).
* Policy "soft": if the theta caps cannot hold B at all (sum of caps < B),
  theta is dropped from the start (caps n_j) instead of being filled first.
* Infeasible budgets (K below the tail plus eps per active token, or above the
  number of vectors) raise ``Infeasible``.

All arithmetic is float64 evaluated as written, with sums taken sequentially
in ascending token id, so the result is a deterministic function of
(counts, spreads, K, params).

Pinned by: hand-worked examples, the closed form kappa_j = floor(q_j) when no
bound binds, the invariants (sum = K, tail sizes, floors, caps, kappa <= n),
scale invariance in s, and the speed-up bound of Sect. 2.1
(tests/test_oracle_budget.py).
"""
from __future__ import annotations

import heapq
import math
from dataclasses import dataclass

import numpy as np

POLICY_FILL_THEN_RELAX = 0
POLICY_SOFT = 1


class Infeasible(ValueError):
    pass


@dataclass(frozen=True)
class BudgetParams:
    mu: int = 128
    tau: int = 256
    eps: int = 4
    theta: float = 39.0
    policy: int = POLICY_FILL_THEN_RELAX


def budget(counts, spread, K: int, p: BudgetParams = BudgetParams(), info: dict | None = None):
    """int64[T] centroids per token, summing to K exactly."""
    counts = [int(c) for c in counts]
    spread = [float(s) for s in spread]
    T = len(counts)
    kappa = [0] * T
    active = []
    tail = 0
    for j in range(T):
        n = counts[j]
        if n == 0:
            continue
        if n < p.mu:
            kappa[j] = min(1, n)
            tail += kappa[j]
        elif n < p.tau:
            kappa[j] = min(2, n)
            tail += kappa[j]
        else:
            active.append(j)
    B = K - tail
    cap_total = 0
    for j in active:
        cap_total += counts[j]
    if B < p.eps * len(active) or B > cap_total or (not active and B != 0):
        raise Infeasible(f"K={K}: tail={tail}, active={len(active)}, B={B}, vectors in active={cap_total}")
    if not active:
        return np.asarray(kappa, dtype=np.int64)

    # Phase 2: damped weights and proportional share of B.
    w = {}
    W = 0.0
    for j in active:
        w[j] = math.sqrt(float(counts[j])) * spread[j]
        W += w[j]
    if not W > 0.0:
        W = 0.0
        for j in active:
            w[j] = math.sqrt(float(counts[j]))
            W += w[j]
    q = {}
    for j in active:
        q[j] = w[j] / W * float(B)
        kappa[j] = int(math.floor(q[j]))

    # Phase 3: floor eps, theta cap.
    hi = {}
    for j in active:
        n = counts[j]
        if p.theta > 0:
            hi[j] = min(n, max(p.eps, int(math.floor(float(n) / p.theta))))
        else:
            hi[j] = n
    if p.policy == POLICY_SOFT:
        total_hi = 0
        for j in active:
            total_hi += hi[j]
        if total_hi < B:
            for j in active:
                hi[j] = counts[j]
    for j in active:
        kappa[j] = min(max(kappa[j], p.eps), hi[j])

    # Phase 4: reconcile to exactly B.
    D = B
    for j in active:
        D -= kappa[j]
    tier2 = 0
    if D > 0:
        relaxed = False
        while D > 0:
            heap = [(-(q[j] - float(kappa[j])), -w[j], j) for j in active if kappa[j] < hi[j]]
            heapq.heapify(heap)
            while D > 0 and heap:
                _, _, j = heapq.heappop(heap)
                kappa[j] += 1
                D -= 1
                if relaxed:
                    tier2 += 1
                if kappa[j] < hi[j]:
                    heapq.heappush(heap, (-(q[j] - float(kappa[j])), -w[j], j))
            if D > 0:
                if relaxed:
                    raise Infeasible("no active token can take another centroid")
                relaxed = True
                for j in active:
                    hi[j] = counts[j]
    elif D < 0:
        heap = [((q[j] - float(kappa[j])), w[j], -j) for j in active if kappa[j] > p.eps]
        heapq.heapify(heap)
        while D < 0:
            if not heap:
                raise Infeasible("no active token can give up a centroid")
            _, _, nj = heapq.heappop(heap)
            j = -nj
            kappa[j] -= 1
            D += 1
            if kappa[j] > p.eps:
                heapq.heappush(heap, ((q[j] - float(kappa[j])), w[j], -j))
    if info is not None:
        info.update(tail=tail, B=B, W=W, tier2=tier2, active=len(active))
    return np.asarray(kappa, dtype=np.int64)


def cent_offsets(kappa) -> np.ndarray:
    """int64[T+1] exclusive prefix sum: token j owns centroids [off[j], off[j+1])."""
    off = np.zeros(len(kappa) + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.asarray(kappa, dtype=np.int64))
    return off
