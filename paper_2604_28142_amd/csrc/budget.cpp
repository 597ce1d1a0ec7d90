// Host side of tac_budget: the per-token centroid budget of Sect. 2.1.
//
// Phase 1 (tail handling): n < mu -> 1 centroid, mu <= n < tau -> 2, n >= tau active.
// Phase 2 (damped scoring): w_j = sqrt(n_j) * s_j, kappa_j = floor(w_j / W * B), where
//   B = K - tail and W sums the active weights (all-zero spreads fall back to sqrt(n_j)).
// Phase 3 (bounding): kappa_j >= eps, and the theta cap hi_j = max(eps, floor(n_j / theta)),
//   never above n_j (theta <= 0: no cap).
// Phase 4 (reconciliation, rule not given in the paper): hand missing units one at a time to
//   the token below its cap with the largest remaining quota p_j = q_j - kappa_j (ties: larger
//   w_j, then smaller j); once every token sits at its theta cap, relax the caps to n_j and go
//   on.  Excess units are taken one at a time from the token above eps with the smallest p_j
//   (ties: smaller w_j, then larger j).
// All arithmetic is IEEE double evaluated as written, sums in ascending token order, so the
// result is a deterministic function of the inputs.
#include <cmath>
#include <queue>
#include <vector>

#include "tac_internal.h"

namespace tac {

namespace {

struct Entry {
    double p;
    double w;
    int32_t j;
};

struct SurplusOrder {  // top of the heap: largest p, then larger w, then smaller j
    bool operator()(const Entry& a, const Entry& b) const {
        if (a.p != b.p) return a.p < b.p;
        if (a.w != b.w) return a.w < b.w;
        return a.j > b.j;
    }
};

struct DeficitOrder {  // top of the heap: smallest p, then smaller w, then larger j
    bool operator()(const Entry& a, const Entry& b) const {
        if (a.p != b.p) return a.p > b.p;
        if (a.w != b.w) return a.w > b.w;
        return a.j < b.j;
    }
};

}  // namespace

tac_status host_budget(const int64_t* counts, const double* spread, int32_t T, int64_t K,
                       const tac_budget_params& prm, int64_t* kappa, int64_t* tier2_units) {
    std::vector<int32_t> active;
    int64_t tail = 0;
    for (int32_t j = 0; j < T; ++j) {
        const int64_t n = counts[j];
        kappa[j] = 0;
        if (n == 0) continue;
        if (n < prm.mu) {
            kappa[j] = n < 1 ? n : 1;
            tail += kappa[j];
        } else if (n < prm.tau) {
            kappa[j] = n < 2 ? n : 2;
            tail += kappa[j];
        } else {
            active.push_back(j);
        }
    }
    const int64_t B = K - tail;
    int64_t cap_total = 0;
    for (int32_t j : active) cap_total += counts[j];
    if (B < prm.eps * (int64_t)active.size() || B > cap_total || (active.empty() && B != 0))
        return set_error(TAC_E_INFEASIBLE,
                         "budget infeasible: K=" + std::to_string(K) + ", tail=" + std::to_string(tail) +
                             ", active tokens=" + std::to_string(active.size()) + ", B=" + std::to_string(B) +
                             ", active vectors=" + std::to_string(cap_total));
    if (tier2_units) *tier2_units = 0;
    if (active.empty()) return TAC_OK;

    std::vector<double> w(T, 0.0), q(T, 0.0);
    std::vector<int64_t> hi(T, 0);
    double W = 0.0;
    for (int32_t j : active) {
        w[j] = std::sqrt((double)counts[j]) * spread[j];
        W += w[j];
    }
    if (!(W > 0.0)) {
        W = 0.0;
        for (int32_t j : active) {
            w[j] = std::sqrt((double)counts[j]);
            W += w[j];
        }
    }
    for (int32_t j : active) {
        q[j] = w[j] / W * (double)B;
        kappa[j] = (int64_t)std::floor(q[j]);
    }
    for (int32_t j : active) {
        const int64_t n = counts[j];
        if (prm.theta > 0) {
            int64_t c = (int64_t)std::floor((double)n / prm.theta);
            if (c < prm.eps) c = prm.eps;
            hi[j] = c < n ? c : n;
        } else {
            hi[j] = n;
        }
    }
    if (prm.theta_policy == TAC_THETA_SOFT) {
        int64_t total_hi = 0;
        for (int32_t j : active) total_hi += hi[j];
        if (total_hi < B)
            for (int32_t j : active) hi[j] = counts[j];
    }
    for (int32_t j : active) {
        int64_t k = kappa[j] < prm.eps ? prm.eps : kappa[j];
        kappa[j] = k < hi[j] ? k : hi[j];
    }

    int64_t D = B;
    for (int32_t j : active) D -= kappa[j];
    int64_t tier2 = 0;
    if (D > 0) {
        bool relaxed = false;
        while (D > 0) {
            std::priority_queue<Entry, std::vector<Entry>, SurplusOrder> heap;
            for (int32_t j : active)
                if (kappa[j] < hi[j]) heap.push({q[j] - (double)kappa[j], w[j], j});
            while (D > 0 && !heap.empty()) {
                Entry e = heap.top();
                heap.pop();
                const int32_t j = e.j;
                kappa[j] += 1;
                D -= 1;
                if (relaxed) ++tier2;
                if (kappa[j] < hi[j]) heap.push({q[j] - (double)kappa[j], w[j], j});
            }
            if (D > 0) {
                if (relaxed) return set_error(TAC_E_INFEASIBLE, "budget: no active token can take another centroid");
                relaxed = true;
                for (int32_t j : active) hi[j] = counts[j];
            }
        }
    } else if (D < 0) {
        std::priority_queue<Entry, std::vector<Entry>, DeficitOrder> heap;
        for (int32_t j : active)
            if (kappa[j] > prm.eps) heap.push({q[j] - (double)kappa[j], w[j], j});
        while (D < 0) {
            if (heap.empty()) return set_error(TAC_E_INFEASIBLE, "budget: no active token can give up a centroid");
            Entry e = heap.top();
            heap.pop();
            const int32_t j = e.j;
            kappa[j] -= 1;
            D += 1;
            if (kappa[j] > prm.eps) heap.push({q[j] - (double)kappa[j], w[j], j});
        }
    }
    if (tier2_units) *tier2_units = tier2;
    return TAC_OK;
}

}  // namespace tac

using namespace tac;

extern "C" tac_status tac_budget_from_stats(const int64_t* counts_h, const double* spread_h, int32_t T, int64_t K,
                                            const tac_budget_params* params, int64_t* kappa_h, int64_t* tier2_h) {
    if (T < 1 || K < 0) return set_error(TAC_E_INVAL, "tac_budget_from_stats: bad T or K");
    if (!counts_h || !spread_h || !kappa_h) return set_error(TAC_E_INVAL, "tac_budget_from_stats: NULL pointer");
    tac_budget_params prm = {128, 256, 4, 39.0, TAC_THETA_FILL_THEN_RELAX};
    if (params) prm = *params;
    if (prm.mu < 0 || prm.tau < 0 || prm.eps < 0 || prm.mu > prm.tau ||
        (prm.theta_policy != TAC_THETA_FILL_THEN_RELAX && prm.theta_policy != TAC_THETA_SOFT))
        return set_error(TAC_E_INVAL, "tac_budget_from_stats: bad budget parameters");
    for (int32_t j = 0; j < T; ++j)
        if (counts_h[j] < 0) return set_error(TAC_E_INVAL, "tac_budget_from_stats: negative count");
    return host_budget(counts_h, spread_h, T, K, prm, kappa_h, tier2_h);
}
