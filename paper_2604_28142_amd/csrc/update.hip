// Update step of per-token Lloyd (Sect. 2.1): each centroid becomes the mean of
// its rows; a centroid with no rows keeps its previous value.
//
// Determinism without float atomics: rows are stably sorted by assigned
// centroid (radix sort on the assignment), so every centroid's members form a
// contiguous run in ascending row order, and one wavefront sums each run in
// that fixed order (two dimensions per lane).  Runs longer than kChunk members
// are cut into chunks of kChunk that separate wavefronts sum, and the chunk
// sums are then added in chunk order, so one large cluster does not hold the
// whole update up; the cut points depend only on the counts.  Tokens with more
// than 65,536 rows sum in float64; smaller ones use compensated (Kahan)
// float32 sums, chunk sums included.
#include "tac_internal.h"

namespace tac {

namespace {

__global__ void update_keys(const int32_t* __restrict__ assign, int64_t n, int64_t K, uint32_t* __restrict__ keys) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = assign[i];
        keys[i] = (a < 0 || a >= K) ? (uint32_t)K : (uint32_t)a;
    }
}

// off[k] = first sorted position with key >= k, for k in [0, K].
__global__ void member_offsets(const uint32_t* __restrict__ keys, int64_t n, int64_t K, int64_t* __restrict__ off) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t prev = i == 0 ? -1 : (int64_t)keys[i - 1];
        int64_t cur = i == n ? K : (int64_t)keys[i];
        if (cur > K) cur = K;
        for (int64_t t = prev + 1; t <= cur; ++t) off[t] = i;
    }
}

constexpr int kUnroll = 16;
constexpr int64_t kChunk = 256;  // members per chunk of a long run

// wide[k] = 1 when centroid k's token has more than kFp64Rows rows (the token is
// found from the centroid's first member); one thread per centroid, so the
// dependent searches of all centroids overlap.
__global__ void centroid_flags(const int64_t* __restrict__ seg_off, int32_t T, const int32_t* __restrict__ rows,
                               const int64_t* __restrict__ off, int64_t K, uint8_t* __restrict__ wide) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = off[k];
        if (b == off[k + 1]) {
            wide[k] = 0;
            continue;
        }
        const int64_t r0 = rows[b];
        int32_t lo = 0, hi = T;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (seg_off[mid] <= r0) lo = mid; else hi = mid;
        }
        wide[k] = seg_off[lo + 1] - seg_off[lo] > kFp64Rows ? 1 : 0;
    }
}

// Sum of members [b, e) of a run (b, e wave-uniform; two dimensions per lane,
// lane's pair of x columns), in member order.  The run's row indices come in
// with one coalesced load per 64 members and are read out lane by lane, so that
// the kUnroll row loads of a round depend on no other load and are in flight
// together; a short round reloads its last row (a cache hit) instead of
// branching around loads.  Wide: float64; else a compensated float32 sum,
// returned as its corrected value.
template <bool Wide>
__device__ __forceinline__ double2 run_sum(const float* __restrict__ xs, const int32_t* __restrict__ rows, int64_t b,
                                           int64_t e, int lane) {
    const float2* xv = reinterpret_cast<const float2*>(xs) + lane;
    double d0 = 0.0, d1 = 0.0;
    float s0 = 0.f, s1 = 0.f, c0 = 0.f, c1 = 0.f;
    for (int64_t g = b; g < e; g += 64) {
        const int n = (int)(e - g < 64 ? e - g : 64);
        const int32_t mine = lane < n ? rows[g + lane] : 0;
        for (int q = 0; q < n; q += kUnroll) {
            float2 v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int src = q + u < n ? q + u : n - 1;
                v[u] = xv[(int64_t)__builtin_amdgcn_readlane(mine, src) * (kDim / 2)];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (q + u >= n) continue;
                if (Wide) {
                    d0 += (double)v[u].x;
                    d1 += (double)v[u].y;
                } else {
                    float y = __fsub_rn(v[u].x, c0);
                    float t = __fadd_rn(s0, y);
                    c0 = __fsub_rn(__fsub_rn(t, s0), y);
                    s0 = t;
                    y = __fsub_rn(v[u].y, c1);
                    t = __fadd_rn(s1, y);
                    c1 = __fsub_rn(__fsub_rn(t, s1), y);
                    s1 = t;
                }
            }
        }
    }
    if (Wide) return make_double2(d0, d1);
    return make_double2((double)__fsub_rn(s0, c0), (double)__fsub_rn(s1, c1));
}

__device__ __forceinline__ double2 run_sum(const float* __restrict__ xs, const int32_t* __restrict__ rows, int64_t b,
                                           int64_t e, bool wide, int lane) {
    return wide ? run_sum<true>(xs, rows, b, e, lane) : run_sum<false>(xs, rows, b, e, lane);
}

// wave index, known to the compiler as wave-uniform (scalar loads of off[k])
__device__ __forceinline__ int64_t wave_id() {
    return __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
}

__device__ __forceinline__ float2 run_mean(double2 sum, int64_t cnt, bool wide) {
    if (wide) return make_float2((float)(sum.x / (double)cnt), (float)(sum.y / (double)cnt));
    const float fc = (float)cnt;
    return make_float2(__fdiv_rn((float)sum.x, fc), __fdiv_rn((float)sum.y, fc));
}

// Centroids with at most kChunk members: one wave each.  Longer runs are left
// to chunk_sums / chunk_means.
__global__ void __launch_bounds__(256) centroid_means(const float* __restrict__ xs, const uint8_t* __restrict__ wide_k,
                                                      const int32_t* __restrict__ rows,
                                                      const int64_t* __restrict__ off, int64_t K,
                                                      const float* __restrict__ C_old, float* __restrict__ C_new,
                                                      int64_t* __restrict__ count) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = wave_id();
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t k = wave0; k < K; k += nwaves) {
        const int64_t b = off[k], e = off[k + 1];
        const int64_t cnt = e - b;
        if (count && lane == 0) count[k] = cnt;
        if (cnt > kChunk) continue;
        float2* out = reinterpret_cast<float2*>(C_new + k * kDim);
        if (cnt == 0) {
            out[lane] = reinterpret_cast<const float2*>(C_old + k * kDim)[lane];
            continue;
        }
        const bool wide = wide_k[k] != 0;
        out[lane] = run_mean(run_sum(xs, rows, b, e, wide, lane), cnt, wide);
    }
}

// chunk slots of the long runs: nch[k] = number of kChunk chunks of centroid k
// when it has more than kChunk members, else 0 (exclusive-scanned afterwards)
__global__ void chunk_count(const int64_t* __restrict__ off, int64_t K, int64_t* __restrict__ nch) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cnt = off[k + 1] - off[k];
        nch[k] = cnt > kChunk ? (cnt + kChunk - 1) / kChunk : 0;
    }
}

// one wave per chunk of a long run: its sum into part[chunk] (128 values)
__global__ void __launch_bounds__(256) chunk_sums(const float* __restrict__ xs, const uint8_t* __restrict__ wide_k,
                                                  const int32_t* __restrict__ rows, const int64_t* __restrict__ off,
                                                  int64_t K, const int64_t* __restrict__ choff,
                                                  double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = wave_id();
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t total = choff[K];
    for (int64_t c = wave0; c < total; c += nwaves) {
        int64_t lo = 0, hi = K;  // centroid: the last k with choff[k] <= c
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (choff[mid] <= c) lo = mid; else hi = mid;
        }
        const int64_t k = lo;
        const int64_t b = off[k] + (c - choff[k]) * kChunk;
        const int64_t e = min(off[k + 1], b + kChunk);
        reinterpret_cast<double2*>(part + c * kDim)[lane] = run_sum(xs, rows, b, e, wide_k[k] != 0, lane);
    }
}

// one wave per long run: its chunk sums added in chunk order (float64 for wide
// tokens, compensated float32 otherwise), then the mean
__global__ void __launch_bounds__(256) chunk_means(const uint8_t* __restrict__ wide_k, const int64_t* __restrict__ off,
                                                   int64_t K, const int64_t* __restrict__ choff,
                                                   const double* __restrict__ part, float* __restrict__ C_new) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t k = wave0; k < K; k += nwaves) {
        const int64_t c0 = choff[k], c1 = choff[k + 1];
        if (c0 == c1) continue;
        const bool wide = wide_k[k] != 0;
        double2 sum;
        if (wide) {
            double s0 = 0.0, s1 = 0.0;
            for (int64_t c = c0; c < c1; ++c) {
                const double2 v = reinterpret_cast<const double2*>(part + c * kDim)[lane];
                s0 += v.x;
                s1 += v.y;
            }
            sum = make_double2(s0, s1);
        } else {
            float s0 = 0.f, s1 = 0.f, e0 = 0.f, e1 = 0.f;
            for (int64_t c = c0; c < c1; ++c) {
                const double2 v = reinterpret_cast<const double2*>(part + c * kDim)[lane];
                float y = __fsub_rn((float)v.x, e0);
                float t = __fadd_rn(s0, y);
                e0 = __fsub_rn(__fsub_rn(t, s0), y);
                s0 = t;
                y = __fsub_rn((float)v.y, e1);
                t = __fadd_rn(s1, y);
                e1 = __fsub_rn(__fsub_rn(t, s1), y);
                s1 = t;
            }
            sum = make_double2((double)__fsub_rn(s0, e0), (double)__fsub_rn(s1, e1));
        }
        reinterpret_cast<float2*>(C_new + k * kDim)[lane] = run_mean(sum, off[k + 1] - off[k], wide);
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

extern "C" tac_status tac_update(tac_ctx ctx, const float* xs_d, const int64_t* seg_off_d, int32_t T, int64_t N,
                                 int32_t d, const int32_t* assign_d, const float* C_old_d, int64_t K, float* C_new_d,
                                 int64_t* count_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_update: ctx is NULL");
    if (d != kDim) return set_error(TAC_E_INVAL, "tac_update: d must be 128");
    if (N < 0 || N > INT32_MAX || K < 0 || K >= INT32_MAX || T < 1)
        return set_error(TAC_E_INVAL, "tac_update: bad sizes");
    if (K == 0) return TAC_OK;
    if (!seg_off_d || !C_old_d || !C_new_d || (N > 0 && (!xs_d || !assign_d)))
        return set_error(TAC_E_INVAL, "tac_update: NULL pointer");
    if (C_old_d == C_new_d) return set_error(TAC_E_INVAL, "tac_update: C_old_d and C_new_d must not alias");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    Carve cv;
    const size_t o_k0 = cv.take<uint32_t>(N + 1), o_v0 = cv.take<int32_t>(N + 1);
    const size_t o_k1 = cv.take<uint32_t>(N + 1), o_v1 = cv.take<int32_t>(N + 1);
    const size_t o_sort = cv.take<char>(radix_sort_scratch_bytes(N));
    const size_t o_off = cv.take<int64_t>(K + 1);
    const size_t o_wide = cv.take<uint8_t>(K + 1);
    const size_t o_choff = cv.take<int64_t>(K + 1);
    const size_t o_cscan = cv.take<char>(scan_scratch_bytes(K));
    // chunks of the long runs: each has more than kChunk members, so there are at most 2 N / kChunk
    const size_t o_part = cv.take<double>((2 * N / kChunk + 1) * kDim);
    tac_status st = ws_reserve(ctx, cv.off);
    if (st != TAC_OK) return st;
    uint32_t* k0 = ws_at<uint32_t>(ctx, o_k0);
    int32_t* v0 = ws_at<int32_t>(ctx, o_v0);
    uint32_t* k1 = ws_at<uint32_t>(ctx, o_k1);
    int32_t* v1 = ws_at<int32_t>(ctx, o_v1);
    int64_t* off = ws_at<int64_t>(ctx, o_off);
    if (N > 0) {
        update_keys<<<grid_for(N, 256), 256, 0, s>>>(assign_d, N, K, k0);
        TAC_LAUNCH_CHECK("update_keys");
    }
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) <= K) ++bits;
    int in1 = 0;
    st = radix_sort(s, N, bits, k0, v0, k1, v1, nullptr, ws_at<void>(ctx, o_sort), &in1);
    if (st != TAC_OK) return st;
    member_offsets<<<grid_for(N + 1, 256), 256, 0, s>>>(in1 ? k1 : k0, N, K, off);
    TAC_LAUNCH_CHECK("member_offsets");
    time_start(ctx, TAC_SLOT_UPDATE);
    uint8_t* wide = ws_at<uint8_t>(ctx, o_wide);
    centroid_flags<<<grid_for(K, 256), 256, 0, s>>>(seg_off_d, T, in1 ? v1 : v0, off, K, wide);
    TAC_LAUNCH_CHECK("centroid_flags");
    const int32_t* srows = in1 ? v1 : v0;
    centroid_means<<<grid_for(K * 64, 256), 256, 0, s>>>(xs_d, wide, srows, off, K, C_old_d, C_new_d, count_d);
    TAC_LAUNCH_CHECK("centroid_means");
    int64_t* choff = ws_at<int64_t>(ctx, o_choff);
    double* part = ws_at<double>(ctx, o_part);
    chunk_count<<<grid_for(K, 256), 256, 0, s>>>(off, K, choff);
    TAC_LAUNCH_CHECK("chunk_count");
    st = exclusive_scan_i64(s, choff, choff, K, ws_at<void>(ctx, o_cscan));
    if (st != TAC_OK) return st;
    chunk_sums<<<(unsigned)ctx->props_cu * 32, 256, 0, s>>>(xs_d, wide, srows, off, K, choff, part);
    TAC_LAUNCH_CHECK("chunk_sums");
    chunk_means<<<grid_for(K * 64, 256), 256, 0, s>>>(wide, off, K, choff, part, C_new_d);
    TAC_LAUNCH_CHECK("chunk_means");
    time_stop(ctx, TAC_SLOT_UPDATE);
    return TAC_OK;
}
