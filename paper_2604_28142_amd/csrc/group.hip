// Grouping by token, per-token spread and the budget entry point (Sect. 2.1).
//
// Rows are stably sorted by token id (a radix sort over the id bits), the
// segment offsets are read off the sorted ids, rows are gathered into
// token-sorted order, and the spread s_j = (1/n_j) sum ||x - mean_j||^2 of
// Phase 2 is computed in two float64 passes over the sorted rows: per-chunk
// partial sums in a fixed order, then per-token combinations in chunk order,
// so results are bitwise reproducible.
#include <algorithm>
#include <vector>

#include "tac_internal.h"

namespace tac {

namespace {

constexpr int kChunkRows = 4096;  // rows per partial sum of the spread passes

__global__ void copy_tokens(const int32_t* __restrict__ tok, int64_t n, int32_t T, uint32_t* __restrict__ keys,
                            unsigned int* __restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t t = tok[i];
        if (t < 0 || t >= T) {
            atomicOr(bad, 1u);
            keys[i] = 0;
        } else {
            keys[i] = (uint32_t)t;
        }
    }
}

// seg_off[t] = first sorted position whose id is >= t, for t in [0, T].
__global__ void offsets_from_sorted(const uint32_t* __restrict__ keys, int64_t n, int32_t T,
                                    int64_t* __restrict__ seg_off) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t prev = i == 0 ? -1 : (int64_t)keys[i - 1];
        const int64_t cur = i == n ? (int64_t)T : (int64_t)keys[i];
        for (int64_t t = prev + 1; t <= cur; ++t) seg_off[t] = i;
    }
}

// dst[i] = src[idx[i]] for rows of 128 floats; 32 lanes move one row as float4s.
__global__ void gather_rows(const float* __restrict__ src, const int32_t* __restrict__ idx, int64_t n,
                            float* __restrict__ dst) {
    const int sub = threadIdx.x & 31;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5; r < n;
         r += ((int64_t)gridDim.x * blockDim.x) >> 5) {
        const float4* s = reinterpret_cast<const float4*>(src + (int64_t)idx[r] * kDim);
        float4* d = reinterpret_cast<float4*>(dst + r * kDim);
        d[sub] = s[sub];
    }
}

struct Item {
    int32_t tok;
    int32_t rows;
    int64_t row0;
};

// Pass 1: per item, float64 column sums over its rows (two half-blocks, then combined).
__global__ void __launch_bounds__(256) spread_sum(const float* __restrict__ xs, const int32_t* __restrict__ perm,
                                                  const Item* __restrict__ items, double* __restrict__ part) {
    __shared__ double lds[256];
    const Item it = items[blockIdx.x];
    const int dim = threadIdx.x & 127;
    const int half = threadIdx.x >> 7;
    double acc = 0.0;
    for (int r = half; r < it.rows; r += 2) {
        const int64_t row = it.row0 + r;
        const int64_t src = perm ? (int64_t)perm[row] : row;
        acc += (double)xs[src * kDim + dim];
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    if (half == 0) part[(int64_t)blockIdx.x * kDim + dim] = lds[dim] + lds[dim + 128];
}

__global__ void __launch_bounds__(128) spread_mean(const double* __restrict__ part, const int32_t* __restrict__ first,
                                                   const int64_t* __restrict__ seg_off, int32_t T,
                                                   double* __restrict__ mean) {
    const int32_t j = blockIdx.x;
    const int64_t n = seg_off[j + 1] - seg_off[j];
    double s = 0.0;
    for (int32_t i = first[j]; i < first[j + 1]; ++i) s += part[(int64_t)i * kDim + threadIdx.x];
    mean[(int64_t)j * kDim + threadIdx.x] = n > 0 ? s / (double)n : 0.0;
}

// Pass 2: per item, sum over rows and dimensions of (x - mean)^2 in float64.
__global__ void __launch_bounds__(256) spread_dev(const float* __restrict__ xs, const int32_t* __restrict__ perm,
                                                  const Item* __restrict__ items, const double* __restrict__ mean,
                                                  double* __restrict__ part) {
    __shared__ double lds[256];
    const Item it = items[blockIdx.x];
    const int dim = threadIdx.x & 127;
    const int half = threadIdx.x >> 7;
    const double m = mean[(int64_t)it.tok * kDim + dim];
    double acc = 0.0;
    for (int r = half; r < it.rows; r += 2) {
        const int64_t row = it.row0 + r;
        const int64_t src = perm ? (int64_t)perm[row] : row;
        const double v = (double)xs[src * kDim + dim] - m;
        acc += v * v;
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

__global__ void spread_final(const double* __restrict__ part, const int32_t* __restrict__ first,
                             const int64_t* __restrict__ seg_off, int32_t T, double* __restrict__ spread) {
    const int32_t j = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= T) return;
    const int64_t n = seg_off[j + 1] - seg_off[j];
    double s = 0.0;
    for (int32_t i = first[j]; i < first[j + 1]; ++i) s += part[i];
    spread[j] = n > 0 ? s / (double)n : 0.0;
}

__global__ void init_gather(const float* __restrict__ xs, const int64_t* __restrict__ seg_off,
                            const int64_t* __restrict__ cent_off, int32_t T, const int32_t* __restrict__ picks,
                            int64_t K, float* __restrict__ C, unsigned int* __restrict__ bad) {
    const int sub = threadIdx.x & 31;
    for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5; k < K;
         k += ((int64_t)gridDim.x * blockDim.x) >> 5) {
        int32_t lo = 0, hi = T;  // largest j with cent_off[j] <= k
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (cent_off[mid] <= k) lo = mid; else hi = mid;
        }
        const int64_t n = seg_off[lo + 1] - seg_off[lo];
        const int32_t p = picks[k];
        float4* d = reinterpret_cast<float4*>(C + k * kDim);
        if (p < 0 || p >= n) {
            if (sub == 0) atomicOr(bad, 1u);
            d[sub] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        const float4* s = reinterpret_cast<const float4*>(xs + (seg_off[lo] + p) * kDim);
        d[sub] = s[sub];
    }
}

unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

}  // namespace

}  // namespace tac

using namespace tac;

extern "C" tac_status tac_budget(tac_ctx ctx, const float* x_d, const int32_t* tok_d, int64_t N, int32_t d,
                                 int32_t T, int64_t K, const tac_budget_params* params,
                                 const double* spread_override_h, int32_t* perm_d, float* xs_d,
                                 int64_t* seg_off_d, int64_t* seg_off_h, int64_t* count_h, double* spread_h,
                                 int64_t* kappa_h, int64_t* cent_off_d, int64_t* cent_off_h) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_budget: ctx is NULL");
    if (d != kDim) return set_error(TAC_E_INVAL, "tac_budget: d must be 128");
    if (N < 0 || N > INT32_MAX) return set_error(TAC_E_INVAL, "tac_budget: N out of range");
    if (T < 1 || T > (1 << 24)) return set_error(TAC_E_INVAL, "tac_budget: T must be in [1, 2^24]");
    if (K < 0) return set_error(TAC_E_INVAL, "tac_budget: K < 0");
    if (N > 0 && (!x_d || !tok_d)) return set_error(TAC_E_INVAL, "tac_budget: x_d / tok_d is NULL");
    if (!perm_d && N > 0) return set_error(TAC_E_INVAL, "tac_budget: perm_d is NULL");
    tac_budget_params prm = {128, 256, 4, 39.0, TAC_THETA_FILL_THEN_RELAX};
    if (params) prm = *params;
    if (prm.mu < 0 || prm.tau < 0 || prm.eps < 0 || prm.mu > prm.tau ||
        (prm.theta_policy != TAC_THETA_FILL_THEN_RELAX && prm.theta_policy != TAC_THETA_SOFT))
        return set_error(TAC_E_INVAL, "tac_budget: bad budget parameters");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;

    const int64_t max_items = (N + kChunkRows - 1) / kChunkRows + T + 1;
    Carve cv;
    const size_t o_k0 = cv.take<uint32_t>(N + 1), o_v0 = cv.take<int32_t>(N + 1);
    const size_t o_k1 = cv.take<uint32_t>(N + 1), o_v1 = cv.take<int32_t>(N + 1);
    const size_t o_sort = cv.take<char>(radix_sort_scratch_bytes(N));
    const size_t o_flag = cv.take<unsigned int>(4);
    const size_t o_seg = cv.take<int64_t>(T + 1);
    const size_t o_items = cv.take<Item>(max_items);
    const size_t o_first = cv.take<int32_t>(T + 1);
    const size_t o_part1 = cv.take<double>(max_items * kDim);
    const size_t o_part2 = cv.take<double>(max_items);
    const size_t o_mean = cv.take<double>((int64_t)T * kDim);
    const size_t o_spread = cv.take<double>(T);
    const size_t o_cent = cv.take<int64_t>(T + 1);
    tac_status st = ws_reserve(ctx, cv.off);
    if (st != TAC_OK) return st;
    uint32_t* k0 = ws_at<uint32_t>(ctx, o_k0);
    int32_t* v0 = ws_at<int32_t>(ctx, o_v0);
    uint32_t* k1 = ws_at<uint32_t>(ctx, o_k1);
    int32_t* v1 = ws_at<int32_t>(ctx, o_v1);
    unsigned int* flag = ws_at<unsigned int>(ctx, o_flag);
    int64_t* seg = seg_off_d ? seg_off_d : ws_at<int64_t>(ctx, o_seg);

    TAC_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned int), s));
    if (N > 0) {
        copy_tokens<<<grid_for(N, 256), 256, 0, s>>>(tok_d, N, T, k0, flag);
        TAC_LAUNCH_CHECK("copy_tokens");
    }
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < T) ++bits;
    int in1 = 0;
    st = radix_sort(s, N, bits, k0, v0, k1, v1, nullptr, ws_at<void>(ctx, o_sort), &in1);
    if (st != TAC_OK) return st;
    const uint32_t* sk = in1 ? k1 : k0;
    const int32_t* sv = in1 ? v1 : v0;
    if (N > 0) TAC_HIP(hipMemcpyAsync(perm_d, sv, (size_t)N * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    offsets_from_sorted<<<grid_for(N + 1, 256), 256, 0, s>>>(sk, N, T, seg);
    TAC_LAUNCH_CHECK("offsets_from_sorted");
    if (xs_d && N > 0) {
        gather_rows<<<grid_for(N * 32, 256), 256, 0, s>>>(x_d, perm_d, N, xs_d);
        TAC_LAUNCH_CHECK("gather_rows");
    }
    std::vector<int64_t> off(T + 1);
    unsigned int bad = 0;
    TAC_HIP(hipMemcpyAsync(off.data(), seg, (size_t)(T + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TAC_HIP(hipMemcpyAsync(&bad, flag, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    TAC_HIP(hipStreamSynchronize(s));
    if (bad) return set_error(TAC_E_INVAL, "tac_budget: token id outside [0, T)");

    // chunk list for the spread passes
    std::vector<Item> items;
    std::vector<int32_t> first(T + 1);
    for (int32_t j = 0; j < T; ++j) {
        first[j] = (int32_t)items.size();
        for (int64_t r = off[j]; r < off[j + 1]; r += kChunkRows)
            items.push_back({j, (int32_t)std::min<int64_t>(kChunkRows, off[j + 1] - r), r});
    }
    first[T] = (int32_t)items.size();
    Item* items_d = ws_at<Item>(ctx, o_items);
    int32_t* first_d = ws_at<int32_t>(ctx, o_first);
    double* part1 = ws_at<double>(ctx, o_part1);
    double* part2 = ws_at<double>(ctx, o_part2);
    double* mean = ws_at<double>(ctx, o_mean);
    double* spread_d = ws_at<double>(ctx, o_spread);
    if (!items.empty())
        TAC_HIP(hipMemcpyAsync(items_d, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, s));
    TAC_HIP(hipMemcpyAsync(first_d, first.data(), (size_t)(T + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    const float* src = xs_d ? xs_d : x_d;
    const int32_t* via = xs_d ? nullptr : perm_d;
    if (!items.empty()) {
        spread_sum<<<(unsigned)items.size(), 256, 0, s>>>(src, via, items_d, part1);
        TAC_LAUNCH_CHECK("spread_sum");
    }
    spread_mean<<<(unsigned)T, 128, 0, s>>>(part1, first_d, seg, T, mean);
    TAC_LAUNCH_CHECK("spread_mean");
    if (!items.empty()) {
        spread_dev<<<(unsigned)items.size(), 256, 0, s>>>(src, via, items_d, mean, part2);
        TAC_LAUNCH_CHECK("spread_dev");
    }
    spread_final<<<(unsigned)((T + 255) / 256), 256, 0, s>>>(part2, first_d, seg, T, spread_d);
    TAC_LAUNCH_CHECK("spread_final");
    std::vector<double> spread(T);
    TAC_HIP(hipMemcpyAsync(spread.data(), spread_d, (size_t)T * sizeof(double), hipMemcpyDeviceToHost, s));
    TAC_HIP(hipStreamSynchronize(s));

    std::vector<int64_t> counts(T), kappa(T), coff(T + 1);
    for (int32_t j = 0; j < T; ++j) counts[j] = off[j + 1] - off[j];
    st = host_budget(counts.data(), spread_override_h ? spread_override_h : spread.data(), T, K, prm, kappa.data(),
                     nullptr);
    if (st != TAC_OK) return st;
    coff[0] = 0;
    for (int32_t j = 0; j < T; ++j) coff[j + 1] = coff[j] + kappa[j];
    if (seg_off_h) std::copy(off.begin(), off.end(), seg_off_h);
    if (count_h) std::copy(counts.begin(), counts.end(), count_h);
    if (spread_h) std::copy(spread.begin(), spread.end(), spread_h);
    if (kappa_h) std::copy(kappa.begin(), kappa.end(), kappa_h);
    if (cent_off_h) std::copy(coff.begin(), coff.end(), cent_off_h);
    if (cent_off_d) {
        TAC_HIP(hipMemcpyAsync(cent_off_d, coff.data(), (size_t)(T + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        TAC_HIP(hipStreamSynchronize(s));
    }
    return TAC_OK;
}

extern "C" tac_status tac_init_centroids(tac_ctx ctx, const float* xs_d, const int64_t* seg_off_d,
                                         const int64_t* cent_off_d, int32_t T, int32_t d, const int32_t* picks_d,
                                         int64_t K, float* C_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_init_centroids: ctx is NULL");
    if (d != kDim) return set_error(TAC_E_INVAL, "tac_init_centroids: d must be 128");
    if (T < 1 || K < 0) return set_error(TAC_E_INVAL, "tac_init_centroids: bad T or K");
    if (K == 0) return TAC_OK;
    if (!xs_d || !seg_off_d || !cent_off_d || !picks_d || !C_d)
        return set_error(TAC_E_INVAL, "tac_init_centroids: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    Carve cv;
    const size_t o_flag = cv.take<unsigned int>(4);
    tac_status st = ws_reserve(ctx, cv.off);
    if (st != TAC_OK) return st;
    unsigned int* flag = ws_at<unsigned int>(ctx, o_flag);
    hipStream_t s = ctx->stream;
    TAC_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned int), s));
    init_gather<<<grid_for(K * 32, 256), 256, 0, s>>>(xs_d, seg_off_d, cent_off_d, T, picks_d, K, C_d, flag);
    TAC_LAUNCH_CHECK("init_gather");
    unsigned int bad = 0;
    TAC_HIP(hipMemcpyAsync(&bad, flag, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    TAC_HIP(hipStreamSynchronize(s));
    if (bad) return set_error(TAC_E_INVAL, "tac_init_centroids: a pick is outside its token's rows");
    return TAC_OK;
}
