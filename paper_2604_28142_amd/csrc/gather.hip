// Gather phase of retrieval (Sect. 2.2, "Gather Phase: Centroid-based
// Document Scoring"): for each query token the kappa_c centroids of largest
// inner product, the documents of their inverted lists with the largest
// similarity per (token, document), the sum over the query's tokens, and the
// kappa_d documents of largest sum.
//
// The paper finds the centroids with an HNSW graph over them; on gfx950 the
// exact set costs one dense product per query token, so it is computed:
// * sim_kernel: <q, c> for a block of query tokens and every centroid on the
//   matrix cores (v_mfma_f32_16x16x4f32), written to the workspace;
// * topk_rows: one work-group per query token selects the kappa_c largest
//   (ties to the lower centroid id): the kappa_c-th largest of 1024 block
//   maxima bounds the cut from below, the few similarities above that bound
//   are sorted in LDS (a three-digit radix select on the order-preserving bit
//   pattern of the similarity when too many reach it);
// * the lists of the selected centroids expand into (query, document) keys
//   carrying the token and the similarity (counts, a scan, emission), one
//   stable radix sort groups them by (query, document) with the tokens in
//   increasing order, and one thread per group takes the largest similarity
//   of each token and adds them up in token order;
// * topk_docs: one work-group per query selects the kappa_d documents of
//   largest sum (ties to the lower document id) the same way.
// Queries run in chunks so that the similarity matrix stays within 4 GiB.
#include <algorithm>
#include <cmath>

#include "tac_internal.h"

namespace tac {

namespace {

constexpr int kGDim = 128;
constexpr int kSelThreads = 256;
constexpr int kMaxKc = 256;
constexpr int kMaxKd = 4096;
constexpr int64_t kSimBudget = (int64_t)4 << 30;  // bytes of similarities per chunk of queries

typedef float f4 __attribute__((ext_vector_type(4)));

unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

// Order-preserving key of a float (larger float, larger key); NaN ranks lowest.
__device__ __forceinline__ uint32_t fkey(float f) {
    if (f != f) return 0u;
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ---- similarities: 64 query-token rows x 256 centroids per wave ----------------
// Lane (g, col) supplies coordinates 16 i + 4 g + k of centroid k0 + col (A) and
// of query row 16 rb + col (B); D[centroid 4 g + r][row col].
__global__ void __launch_bounds__(256) sim_kernel(const float* __restrict__ Q, int64_t R,
                                                  const float* __restrict__ C, int64_t K, float* __restrict__ S,
                                                  int64_t ldS) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.y * 64;
    const int64_t kbase = ((int64_t)blockIdx.x * 4 + wave) * 256;
    if (kbase >= K) return;
    float qf[4][32];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int64_t row = r0 + 16 * rb + col;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (row < R) v = reinterpret_cast<const float4*>(Q + row * kGDim)[4 * i + g];
            qf[rb][4 * i + 0] = v.x;
            qf[rb][4 * i + 1] = v.y;
            qf[rb][4 * i + 2] = v.z;
            qf[rb][4 * i + 3] = v.w;
        }
    }
    for (int t = 0; t < 16; ++t) {
        const int64_t k0 = kbase + 16 * t;
        if (k0 >= K) break;
        const int64_t kr = k0 + col;
        float cf[32];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (kr < K) v = reinterpret_cast<const float4*>(C + kr * kGDim)[4 * i + g];
            cf[4 * i + 0] = v.x;
            cf[4 * i + 1] = v.y;
            cf[4 * i + 2] = v.z;
            cf[4 * i + 3] = v.w;
        }
        f4 acc[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) acc[rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 32; ++s)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(cf[s], qf[rb][s], acc[rb], 0, 0, 0);
        const int64_t kk = k0 + 4 * g;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            const int64_t row = r0 + 16 * rb + col;
            if (row >= R) continue;
            float* dst = S + row * ldS + kk;
            if (kk + 3 < K) {
                *reinterpret_cast<float4*>(dst) = make_float4(acc[rb][0], acc[rb][1], acc[rb][2], acc[rb][3]);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (kk + r < K) dst[r] = acc[rb][r];
            }
        }
    }
}

// ---- exact top-k of one list in one work-group ---------------------------------
struct SelShared {
    unsigned hist[2048];
    unsigned cnt_gt[kSelThreads];
    unsigned cnt_eq[kSelThreads];
    unsigned long long sortbuf[kMaxKd];
    unsigned sel_digit, sel_above;
};

// The k largest (key, index) of n elements, larger key first and, among equal
// keys, lower index first; GET(t) returns the key of element t.  Results (key,
// index) land sorted in sh.sortbuf[0 .. min(k, n)) as ((~key) << 32) | index.
// Returns min(k, n).  k <= kMaxKd.
template <class GET>
__device__ int select_topk(GET get, int64_t n, int k, SelShared& sh) {
    const int tid = threadIdx.x;
    const int kk = (int)std::min<int64_t>(k, n);
    uint32_t prefix = 0u, pmask = 0u;
    unsigned remaining = (unsigned)kk;  // elements still to take among those matching the prefix
    if (kk > 0 && kk < n) {
        const int shifts[3] = {21, 10, 0};
        const int widths[3] = {11, 11, 10};
        for (int dgt = 0; dgt < 3; ++dgt) {
            const int sh_ = shifts[dgt];
            const uint32_t dmask = (1u << widths[dgt]) - 1u;
            for (int b = tid; b < 2048; b += kSelThreads) sh.hist[b] = 0u;
            __syncthreads();
            for (int64_t t = tid; t < n; t += kSelThreads) {
                const uint32_t key = get(t);
                if ((key & pmask) == prefix) atomicAdd(&sh.hist[(key >> sh_) & dmask], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                unsigned above = 0u;
                int v = (int)dmask;
                for (; v > 0; --v) {
                    if (above + sh.hist[v] >= remaining) break;
                    above += sh.hist[v];
                }
                sh.sel_digit = (unsigned)v;
                sh.sel_above = above;
            }
            __syncthreads();
            prefix |= sh.sel_digit << sh_;
            pmask |= dmask << sh_;
            remaining -= sh.sel_above;
            __syncthreads();
        }
    }
    // collect: every key above the threshold, then the lowest-index keys equal to it
    const bool all = kk >= n;
    const int64_t chunk = (n + kSelThreads - 1) / kSelThreads;
    const int64_t t0 = std::min<int64_t>(n, tid * chunk), t1 = std::min<int64_t>(n, t0 + chunk);
    unsigned ngt = 0u, neq = 0u;
    for (int64_t t = t0; t < t1; ++t) {
        const uint32_t key = get(t);
        if (all || key > prefix) ++ngt;
        else if (key == prefix) ++neq;
    }
    sh.cnt_gt[tid] = ngt;
    sh.cnt_eq[tid] = neq;
    __syncthreads();
    if (tid == 0) {
        unsigned a = 0u, e = 0u;
        for (int i = 0; i < kSelThreads; ++i) {
            const unsigned x = sh.cnt_gt[i], y = sh.cnt_eq[i];
            sh.cnt_gt[i] = a;
            sh.cnt_eq[i] = e;
            a += x;
            e += y;
        }
        sh.sel_above = a;  // number of keys above the threshold
    }
    __syncthreads();
    const unsigned nabove = sh.sel_above;
    unsigned pg = sh.cnt_gt[tid], pe = sh.cnt_eq[tid];
    for (int64_t t = t0; t < t1; ++t) {
        const uint32_t key = get(t);
        const unsigned long long packed = ((unsigned long long)(~key) << 32) | (unsigned long long)(uint32_t)t;
        if (all || key > prefix) {
            sh.sortbuf[pg++] = packed;
        } else if (key == prefix) {
            if (pe < remaining) sh.sortbuf[nabove + pe] = packed;
            ++pe;
        }
    }
    // pad to a power of two and sort ascending (bitonic)
    int np2 = 1;
    while (np2 < kk) np2 <<= 1;
    for (int i = kk + tid; i < np2; i += kSelThreads) sh.sortbuf[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= np2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < np2; i += kSelThreads) {
                const int p = i ^ stride;
                if (p > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = sh.sortbuf[i], b = sh.sortbuf[p];
                    if ((a > b) == up) {
                        sh.sortbuf[i] = b;
                        sh.sortbuf[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    return kk;
}

// Ascending bitonic sort of np2 (a power of two, <= 2048) 32-bit keys in LDS.
__device__ void bitonic_u32(unsigned* a, int np2) {
    const int tid = threadIdx.x;
    for (int size = 2; size <= np2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < np2; i += kSelThreads) {
                const int p = i ^ stride;
                if (p > i) {
                    const bool up = (i & size) == 0;
                    const unsigned x = a[i], y = a[p];
                    if ((x > y) == up) {
                        a[i] = y;
                        a[p] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// The same selection for small k out of a long float row.  The maxima of
// 1024 blocks of the row (block b holds the elements t with t mod 1024 = b,
// so that thread i owns blocks 4 i .. 4 i + 3 and both passes read the row
// coalesced, four elements per load) give a lower bound for the k-th largest
// key (the k-th largest block maximum: at least k elements reach it), every
// element at or above that bound is collected, and the candidates are sorted
// like select_topk's.  When more candidates than the sort buffer holds reach
// the bound, select_topk runs instead.  The candidate set, and so the result,
// does not depend on the order of the collection.  n >= 1024, n % 4 == 0, row
// 16-byte aligned.
template <class GET>
__device__ int select_topk_blocks(const float* __restrict__ row, GET get, int64_t n, int k, SelShared& sh) {
    constexpr int kBlocks = 1024;
    static_assert(kBlocks == 4 * kSelThreads, "each thread owns four blocks");
    const int tid = threadIdx.x;
    const float4* r4 = reinterpret_cast<const float4*>(row);
    const int64_t n4 = n / 4;
    uint32_t m0 = 0u, m1 = 0u, m2 = 0u, m3 = 0u;
    for (int64_t v = tid; v < n4; v += kSelThreads) {
        const float4 x = r4[v];
        m0 = max(m0, fkey(x.x));
        m1 = max(m1, fkey(x.y));
        m2 = max(m2, fkey(x.z));
        m3 = max(m3, fkey(x.w));
    }
    sh.hist[4 * tid + 0] = m0;
    sh.hist[4 * tid + 1] = m1;
    sh.hist[4 * tid + 2] = m2;
    sh.hist[4 * tid + 3] = m3;
    if (tid == 0) sh.sel_above = 0u;
    __syncthreads();
    bitonic_u32(sh.hist, kBlocks);
    const uint32_t bound = sh.hist[kBlocks - k];  // k-th largest block maximum
    auto take = [&](uint32_t key, int64_t t) {
        if (key >= bound) {
            const unsigned slot = atomicAdd(&sh.sel_above, 1u);
            if (slot < (unsigned)kMaxKd)
                sh.sortbuf[slot] = ((unsigned long long)(~key) << 32) | (unsigned long long)(uint32_t)t;
        }
    };
    for (int64_t v = tid; v < n4; v += kSelThreads) {
        const float4 x = r4[v];
        take(fkey(x.x), 4 * v + 0);
        take(fkey(x.y), 4 * v + 1);
        take(fkey(x.z), 4 * v + 2);
        take(fkey(x.w), 4 * v + 3);
    }
    __syncthreads();
    const unsigned nc = sh.sel_above;
    __syncthreads();
    if (nc > (unsigned)kMaxKd) return select_topk(get, n, k, sh);
    int np2 = 1;
    while (np2 < (int)nc) np2 <<= 1;
    for (int i = (int)nc + tid; i < np2; i += kSelThreads) sh.sortbuf[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= np2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < np2; i += kSelThreads) {
                const int p = i ^ stride;
                if (p > i) {
                    const bool up = (i & size) == 0;
                    const unsigned long long a = sh.sortbuf[i], b = sh.sortbuf[p];
                    if ((a > b) == up) {
                        sh.sortbuf[i] = b;
                        sh.sortbuf[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    return k;
}

__device__ __forceinline__ float key_float(uint32_t key) {
    const uint32_t u = (key & 0x80000000u) ? (key & 0x7FFFFFFFu) : ~key;
    return __uint_as_float(u);
}

// kappa_c largest similarities of every query-token row
__global__ void __launch_bounds__(kSelThreads) topk_rows(const float* __restrict__ S, int64_t ldS, int64_t K, int kc,
                                                         int32_t* __restrict__ top_id, float* __restrict__ top_sim) {
    __shared__ SelShared sh;
    const int64_t row = blockIdx.x;
    const float* s = S + row * ldS;
    auto get = [&](int64_t t) { return fkey(s[t]); };
    // the block bound needs at least kc non-empty blocks
    const int kk = (K >= 4 * 1024 && K % 4 == 0 && ldS % 4 == 0 && kc <= 256) ? select_topk_blocks(s, get, K, kc, sh)
                                                                             : select_topk(get, K, kc, sh);
    for (int r = threadIdx.x; r < kc; r += kSelThreads) {
        const int64_t o = row * kc + r;
        if (r < kk) {
            const unsigned long long p = sh.sortbuf[r];
            top_id[o] = (int32_t)(uint32_t)p;
            top_sim[o] = key_float(~(uint32_t)(p >> 32));
        } else {
            top_id[o] = -1;
            top_sim[o] = -INFINITY;
        }
    }
}

// entries (row, rank): the length of the selected centroid's list
__global__ void emit_count(const int32_t* __restrict__ top_id, int64_t n, const int64_t* __restrict__ list_off,
                           int64_t K, int64_t* __restrict__ cnt) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = top_id[e];
        cnt[e] = (j >= 0 && j < K) ? std::max<int64_t>(0, list_off[j + 1] - list_off[j]) : 0;
    }
}

// one wave per entry: its list's documents become keys q * D + d carrying (token, similarity)
__global__ void emit_kernel(const int32_t* __restrict__ top_id, const float* __restrict__ top_sim, int64_t n, int kc,
                            int nq, const int64_t* __restrict__ list_off, const int32_t* __restrict__ list_docs,
                            int64_t K, int64_t D, const int64_t* __restrict__ eoff, uint32_t* __restrict__ keys,
                            int32_t* __restrict__ tok, float* __restrict__ sim) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    const uint32_t sentinel = (uint32_t)((n / kc / nq) * D);  // past every valid key of the chunk
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); e < n; e += waves) {
        const int32_t j = top_id[e];
        if (j < 0 || j >= K) continue;
        const int64_t row = e / kc;
        const int64_t q = row / nq;
        const int i = (int)(row - q * nq);
        const float s = top_sim[e];
        const int64_t base = list_off[j], len = eoff[e + 1] - eoff[e];
        for (int64_t t = lane; t < len; t += 64) {
            const int64_t pos = eoff[e] + t;
            const int32_t d = list_docs[base + t];
            keys[pos] = (d >= 0 && d < D) ? (uint32_t)(q * D + d) : sentinel;
            tok[pos] = i;
            sim[pos] = s;
        }
    }
}

// group heads of the sorted keys (valid keys only)
__global__ void seg_flags(const uint32_t* __restrict__ keys, int64_t n, uint32_t limit, int64_t* __restrict__ flag) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        flag[p] = (keys[p] < limit && (p == 0 || keys[p] != keys[p - 1])) ? 1 : 0;
}

__global__ void seg_compact(const int64_t* __restrict__ flag, const int64_t* __restrict__ idx, int64_t n,
                            int64_t* __restrict__ start) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        if (flag[p]) start[idx[p]] = p;
}

// One thread per (query, document) group: the largest similarity of each token,
// summed over the tokens in increasing order (the sort kept emission order).
__global__ void seg_reduce(const uint32_t* __restrict__ keys, const int32_t* __restrict__ pos, int64_t n,
                           const int32_t* __restrict__ tok, const float* __restrict__ sim,
                           const int64_t* __restrict__ start, const int64_t* __restrict__ nseg_p,
                           uint32_t* __restrict__ seg_key, float* __restrict__ seg_score) {
    const int64_t nseg = *nseg_p;
    for (int64_t sg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sg < nseg;
         sg += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p0 = start[sg];
        const uint32_t key = keys[p0];
        double sum = 0.0;
        int cur = -1;
        float mx = -INFINITY;
        for (int64_t p = p0; p < n && keys[p] == key; ++p) {
            const int32_t e = pos[p];
            const int i = tok[e];
            const float v = sim[e];
            if (i != cur) {
                if (cur >= 0) sum += (double)mx;
                cur = i;
                mx = v;
            } else {
                mx = fmaxf(mx, v);
            }
        }
        if (cur >= 0) sum += (double)mx;
        seg_key[sg] = key;
        seg_score[sg] = (float)sum;
    }
}

// qoff[q] = first group with key >= q * D, q in [0, QC]
__global__ void seg_qoff(const uint32_t* __restrict__ seg_key, const int64_t* __restrict__ nseg_p, int64_t QC,
                         int64_t D, int64_t* __restrict__ qoff) {
    const int64_t nseg = *nseg_p;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= QC; q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t target = (uint64_t)q * (uint64_t)D;
        int64_t lo = 0, hi = nseg;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((uint64_t)seg_key[mid] < target) lo = mid + 1;
            else hi = mid;
        }
        qoff[q] = lo;
    }
}

// kappa_d documents of largest score per query (ties: lower id, which is the lower group index)
__global__ void __launch_bounds__(kSelThreads) topk_docs(const uint32_t* __restrict__ seg_key,
                                                         const float* __restrict__ seg_score,
                                                         const int64_t* __restrict__ qoff, int64_t D, int kd,
                                                         int32_t* __restrict__ out_doc, float* __restrict__ out_score) {
    __shared__ SelShared sh;
    const int64_t q = blockIdx.x;
    const int64_t s0 = qoff[q], n = qoff[q + 1] - s0;
    const int kk = select_topk([&](int64_t t) { return fkey(seg_score[s0 + t]); }, n, kd, sh);
    for (int r = threadIdx.x; r < kd; r += kSelThreads) {
        const int64_t o = q * kd + r;
        if (r < kk) {
            const unsigned long long p = sh.sortbuf[r];
            const int64_t t = (int64_t)(uint32_t)p;
            out_doc[o] = (int32_t)((int64_t)seg_key[s0 + t] - q * D);
            out_score[o] = seg_score[s0 + t];
        } else {
            out_doc[o] = -1;
            out_score[o] = -INFINITY;
        }
    }
}

// ---- proximity graph over the centroids (the gather's centroid search) ---------
// The paper searches the centroids with an HNSW graph (Sect. 2.2, "Index
// Structure"; built with M = 32 and ef_c = 1500, searched with ef_s = 1.5
// kappa_c, Sect. 3).  Here the graph is built on the matrix cores and searched
// one wave per query token:
// * build: each centroid's kGraphDeg nearest centroids by inner product
//   (exact: the similarity and top-k kernels above, the centroids as queries,
//   itself dropped), then up to kGraphDeg reverse edges per centroid (the
//   centroids that list it, largest similarity first, lower id on ties,
//   without those it already lists), so that a centroid listed by many keeps
//   its best in-links and one listed by none is still reachable;
// * entry: an exhaustive scan of a set of router centroids (the caller's:
//   e.g. one per token segment) picks the ef best as the starting beam;
// * search: best-first expansion of a beam of ef <= 64 entries, one per lane,
//   kept sorted by (similarity descending, id ascending); a visited set in LDS
//   (open addressing) keeps every centroid from being scored twice; it stops
//   when every beam entry has been expanded.  Similarities are float32 dot
//   products accumulated in a fixed order, so the search is deterministic.
constexpr int kGraphDeg = 32;
constexpr int kGraphCols = 2 * kGraphDeg;
constexpr int kSearchWaves = 4;
constexpr int kHashSlots = 8192;     // visited-set slots per wave (32 KiB of LDS)
constexpr int kHashProbes = 32;
constexpr int kMaxEf = 64;

// forward lists from the rows' kGraphDeg + 1 nearest: the centroid itself dropped
__global__ void graph_forward(const int32_t* __restrict__ top_id, const float* __restrict__ top_sim, int64_t r0,
                              int64_t R, int32_t* __restrict__ nbr, float* __restrict__ fsim) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int64_t i = r0 + r;
    int w = 0;
    for (int t = 0; t <= kGraphDeg && w < kGraphDeg; ++t) {
        const int32_t j = top_id[r * (kGraphDeg + 1) + t];
        if (j < 0 || j == i) continue;
        nbr[i * kGraphCols + w] = j;
        fsim[i * kGraphDeg + w] = top_sim[r * (kGraphDeg + 1) + t];
        ++w;
    }
    for (; w < kGraphDeg; ++w) {
        nbr[i * kGraphCols + w] = -1;
        fsim[i * kGraphDeg + w] = -INFINITY;
    }
}

__global__ void rev_count(const int32_t* __restrict__ nbr, int64_t K, int64_t* __restrict__ cnt) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < K * kGraphDeg;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = nbr[(e / kGraphDeg) * kGraphCols + e % kGraphDeg];
        if (j >= 0) atomicAdd(reinterpret_cast<unsigned long long*>(cnt + j), 1ull);
    }
}

__global__ void rev_fill(const int32_t* __restrict__ nbr, const float* __restrict__ fsim, int64_t K,
                         const int64_t* __restrict__ off, int64_t* __restrict__ cur, int32_t* __restrict__ rsrc,
                         float* __restrict__ rsim) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < K * kGraphDeg;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / kGraphDeg;
        const int32_t j = nbr[i * kGraphCols + e % kGraphDeg];
        if (j < 0) continue;
        const int64_t p = off[j] + (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(cur + j), 1ull);
        rsrc[p] = (int32_t)i;
        rsim[p] = fsim[e];
    }
}

// Packed order key of a candidate: larger similarity first, then lower id.
__device__ __forceinline__ unsigned long long cand_key(float sim, int32_t id) {
    return ((unsigned long long)fkey(sim) << 32) | (unsigned long long)(~(uint32_t)id);
}

// One wave per centroid j: its reverse entries (the centroids listing it), those
// it lists itself excluded, the kGraphDeg best by (similarity, lower id) into
// columns kGraphDeg .. kGraphCols - 1, -1 where fewer.  The fill order of the
// entries (atomic) does not matter: the selection is by key.
__global__ void __launch_bounds__(256) rev_select(const int64_t* __restrict__ off, const int32_t* __restrict__ rsrc,
                                                  const float* __restrict__ rsim, int64_t K,
                                                  int32_t* __restrict__ nbr) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= K) return;
    const int64_t s0 = off[j], n = off[j + 1] - s0;
    const int32_t mine = lane < kGraphDeg ? nbr[j * kGraphCols + lane] : -1;
    unsigned long long prev = ~0ull;
    for (int r = 0; r < kGraphDeg; ++r) {
        unsigned long long best = 0ull;
        // whole-wave passes over the entries (lane t0 + lane), so that every lane
        // takes part in the shuffles that compare a source with j's own list
        for (int64_t t0 = 0; t0 < n; t0 += 64) {
            const int64_t t = t0 + lane;
            const int32_t src = t < n ? rsrc[s0 + t] : -1;
            bool listed = false;
            for (int u = 0; u < kGraphDeg; ++u) listed |= __shfl(mine, u) == src;
            const unsigned long long k = (t >= n || listed) ? 0ull : cand_key(rsim[s0 + t], src);
            if (k < prev && k > best) best = k;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long ob = __shfl_xor(best, o);
            best = ob > best ? ob : best;
        }
        if (lane == 0) nbr[j * kGraphCols + kGraphDeg + r] = best ? (int32_t)~(uint32_t)best : -1;
        if (!best) {
            for (int q = r + 1 + lane; q < kGraphDeg; q += 64) nbr[j * kGraphCols + kGraphDeg + q] = -1;
            break;
        }
        prev = best;
    }
}

// router picks -> centroid ids
__global__ void map_ids(const int32_t* __restrict__ pick, int64_t n, const int32_t* __restrict__ entry,
                        int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = pick[i] >= 0 ? entry[pick[i]] : -1;
}

// router rows; an id outside [0, K) gets a zero row (and its picks are dropped by the search)
__global__ void gather_rows128(const float* __restrict__ C, int64_t K, const int32_t* __restrict__ ids, int64_t n,
                               float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 8 + (threadIdx.x >> 5);
    if (i >= n) return;
    const int32_t id = ids[i];
    reinterpret_cast<float4*>(out + i * kGDim)[threadIdx.x & 31] =
        id >= 0 && id < K ? reinterpret_cast<const float4*>(C + (int64_t)id * kGDim)[threadIdx.x & 31]
                          : make_float4(0.f, 0.f, 0.f, 0.f);
}

// <q, c> in float32, four interleaved partial sums over the coordinates (i mod 4), then (s0 + s1) + (s2 + s3)
__device__ __forceinline__ float dot128(const float4 (&q)[32], const float* __restrict__ c) {
    const float4* cv = reinterpret_cast<const float4*>(c);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const float4 v = cv[i];
        s0 = fmaf(q[i].x, v.x, s0);
        s1 = fmaf(q[i].y, v.y, s1);
        s2 = fmaf(q[i].z, v.z, s2);
        s3 = fmaf(q[i].w, v.w, s3);
    }
    return (s0 + s1) + (s2 + s3);
}

struct SearchShared {
    int32_t hash[kSearchWaves][kHashSlots];
    unsigned long long all[kSearchWaves][2 * kMaxEf];
    unsigned long long beam[kSearchWaves][kMaxEf];
    int32_t done[kSearchWaves][kMaxEf];
};

// Visited-set insertion: true when `id` was not in the set (and now is).  A
// full probe sequence counts as visited, so the search skips that centroid.
__device__ __forceinline__ bool visit(int32_t* __restrict__ H, int32_t id) {
    unsigned h = ((unsigned)id * 2654435761u) >> (32 - 13);
    static_assert(kHashSlots == 1 << 13, "13-bit hash");
    for (int p = 0; p < kHashProbes; ++p) {
        const int32_t old = atomicCAS(&H[h], -1, id);
        if (old == -1) return true;
        if (old == id) return false;
        h = (h + 1) & (kHashSlots - 1);
    }
    return false;
}

// One wave per query-token row.  Lane l < ef holds beam entry l (sorted); `done`
// marks expanded entries.  Each step expands the best entry not expanded yet:
// its kGraphCols neighbours (one per lane) not visited before are scored, and
// the ef best of beam and new entries become the beam (every one of the 2 * 64
// keys is ranked against the others, each lands at its rank).
__global__ void __launch_bounds__(64 * kSearchWaves) graph_search(const float* __restrict__ Q, int64_t R,
                                                                   const float* __restrict__ C, int64_t K,
                                                                   const int32_t* __restrict__ nbr,
                                                                   const int32_t* __restrict__ init, int ef, int kc,
                                                                   int max_steps, int32_t* __restrict__ top_id,
                                                                   float* __restrict__ top_sim,
                                                                   int32_t* __restrict__ steps_out) {
    extern __shared__ __attribute__((aligned(16))) unsigned char search_lds[];
    SearchShared& sh = *reinterpret_cast<SearchShared*>(search_lds);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t row = (int64_t)blockIdx.x * kSearchWaves + w;
    if (row >= R) return;  // waves are independent: no work-group barrier follows
    int32_t* H = sh.hash[w];
    unsigned long long* all = sh.all[w];
    unsigned long long* bm = sh.beam[w];
    int32_t* dn = sh.done[w];
    for (int i = lane; i < kHashSlots; i += 64) H[i] = -1;
    float4 q[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) q[i] = reinterpret_cast<const float4*>(Q + row * kGDim)[i];
    // an empty slot's key: below every real key, distinct per position
    const unsigned long long empty_lo = (unsigned long long)lane, empty_hi = 64ull + lane;
    // starting beam: the router picks, scored like every other centroid
    unsigned long long mykey = empty_lo;
    if (lane < ef) {
        const int32_t id = init[row * ef + lane];
        if (id >= 0 && id < K && visit(H, id)) mykey = cand_key(dot128(q, C + (int64_t)id * kGDim), id);
    }
    int mydone = 0;
    // sort by ranking: position = number of larger keys
    auto rank_merge = [&](unsigned long long a, int da, unsigned long long b) {
        all[lane] = a;
        all[64 + lane] = b;
        __builtin_amdgcn_wave_barrier();
        int ra = 0, rb = 0;
        for (int t = 0; t < 128; ++t) {
            const unsigned long long v = all[t];
            ra += v > a;
            rb += v > b;
        }
        __builtin_amdgcn_wave_barrier();
        if (ra < ef) { bm[ra] = a; dn[ra] = da; }
        if (rb < ef) { bm[rb] = b; dn[rb] = 0; }
        __builtin_amdgcn_wave_barrier();
        mykey = lane < ef ? bm[lane] : empty_lo;
        mydone = lane < ef ? dn[lane] : 1;
        __builtin_amdgcn_wave_barrier();
    };
    rank_merge(mykey, 0, empty_hi);
    int step = 0;
    for (; step < max_steps; ++step) {
        const unsigned long long open = __ballot(lane < ef && mykey > 127ull && !mydone);
        if (!open) break;
        const int p = __ffsll((long long)open) - 1;
        const int32_t node = (int32_t)~(uint32_t)__shfl((unsigned)(mykey & 0xFFFFFFFFull), p);
        if (lane == p) mydone = 1;
        const int32_t nid = nbr[(int64_t)node * kGraphCols + lane];
        unsigned long long nk = empty_hi;
        if (nid >= 0 && nid < K && visit(H, nid)) nk = cand_key(dot128(q, C + (int64_t)nid * kGDim), nid);
        // the beam's last key: a new key at or below it cannot enter a full beam
        const unsigned long long worst = __shfl(mykey, ef - 1);
        if (!__ballot(nk > worst)) continue;
        rank_merge(mykey, mydone, nk);
    }
    if (lane < kc) {
        const bool ok = mykey > 127ull;
        top_id[row * kc + lane] = ok ? (int32_t)~(uint32_t)mykey : -1;
        top_sim[row * kc + lane] = ok ? key_float((uint32_t)(mykey >> 32)) : -INFINITY;
    }
    if (steps_out && lane == 0) steps_out[row] = step;
}

int bits_for(uint64_t maxkey) {
    int b = 1;
    while (b < 32 && (uint64_t(1) << b) <= maxkey) ++b;
    return b;
}

}  // namespace

}  // namespace tac

using namespace tac;

extern "C" tac_status tac_gather(tac_ctx ctx, const float* Q_d, int64_t B, int32_t nq, int32_t d, const float* C_d,
                                 int64_t K, const int64_t* list_off_d, const int32_t* list_docs_d, int64_t D,
                                 int32_t kc, int32_t kd, int32_t* cand_d, float* score_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_gather: ctx is NULL");
    if (d != kGDim) return set_error(TAC_E_INVAL, "tac_gather: d must be 128");
    if (B < 0 || nq < 1 || nq > 1024 || K < 1 || K > INT32_MAX || D < 1 || D > INT32_MAX)
        return set_error(TAC_E_INVAL, "tac_gather: bad sizes");
    if (kc < 1 || kc > kMaxKc) return set_error(TAC_E_INVAL, "tac_gather: kappa_c must be in [1, 256]");
    if (kd < 1 || kd > kMaxKd) return set_error(TAC_E_INVAL, "tac_gather: kappa_d must be in [1, 4096]");
    if (B == 0) return TAC_OK;
    if (!Q_d || !C_d || !list_off_d || !list_docs_d || !cand_d || !score_d)
        return set_error(TAC_E_INVAL, "tac_gather: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t ldS = (K + 3) / 4 * 4;
    // queries per chunk: the similarity matrix within kSimBudget, the keys q * D + d within 32 bits
    int64_t QC = std::max<int64_t>(1, kSimBudget / ((int64_t)nq * ldS * 4));
    QC = std::min<int64_t>(QC, ((int64_t)UINT32_MAX - 1) / D);
    QC = std::min<int64_t>(QC, B);
    if (QC < 1) return set_error(TAC_E_INVAL, "tac_gather: too many documents for 32-bit keys");
    size_t need_b = 0;  // size of the expansion stage seen so far
    for (int64_t q0 = 0; q0 < B; q0 += QC) {
        const int64_t qc = std::min<int64_t>(QC, B - q0);
        const int64_t R = qc * nq;
        const int64_t nent = R * kc;
        // stage A: top lists and list-length scan, then the similarity matrix
        Carve ca;
        const size_t o_id = ca.take<int32_t>(nent), o_sim = ca.take<float>(nent);
        const size_t o_eoff = ca.take<int64_t>(nent + 1);
        const size_t o_scan = ca.take<char>(scan_scratch_bytes(nent));
        const size_t base_b = ca.off;
        const size_t o_S = ca.take<float>(R * ldS);
        tac_status st = ws_reserve(ctx, std::max(ca.off, need_b));
        if (st != TAC_OK) return st;
        int64_t E = 0;
        for (int attempt = 0; attempt < 2; ++attempt) {
            int32_t* top_id = ws_at<int32_t>(ctx, o_id);
            float* top_sim = ws_at<float>(ctx, o_sim);
            int64_t* eoff = ws_at<int64_t>(ctx, o_eoff);
            float* S = ws_at<float>(ctx, o_S);
            const dim3 sg((unsigned)((K + 1023) / 1024), (unsigned)((R + 63) / 64));
            if (sg.y > 65535) return set_error(TAC_E_INVAL, "tac_gather: too many query tokens per chunk");
            sim_kernel<<<sg, 256, 0, s>>>(Q_d + q0 * nq * kGDim, R, C_d, K, S, ldS);
            TAC_LAUNCH_CHECK("sim_kernel");
            topk_rows<<<(unsigned)R, kSelThreads, 0, s>>>(S, ldS, K, kc, top_id, top_sim);
            TAC_LAUNCH_CHECK("topk_rows");
            emit_count<<<grid_for(nent, 256), 256, 0, s>>>(top_id, nent, list_off_d, K, eoff);
            TAC_LAUNCH_CHECK("emit_count");
            st = exclusive_scan_i64(s, eoff, eoff, nent, ws_at<void>(ctx, o_scan));
            if (st != TAC_OK) return st;
            TAC_HIP(hipMemcpyAsync(&E, eoff + nent, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            TAC_HIP(hipStreamSynchronize(s));
            // stage B sizes (it reuses the similarity matrix's memory)
            Carve cb;
            cb.off = base_b;
            const int64_t En = std::max<int64_t>(E, 1);
            cb.take<uint32_t>(En);
            cb.take<uint32_t>(En);
            cb.take<int32_t>(En);
            cb.take<int32_t>(En);
            cb.take<int32_t>(En);
            cb.take<float>(En);
            cb.take<char>(radix_sort_scratch_bytes(En));
            cb.take<int64_t>(En + 1);
            cb.take<int64_t>(En + 1);
            cb.take<char>(scan_scratch_bytes(En + 1));
            cb.take<int64_t>(En + 1);
            cb.take<uint32_t>(En);
            cb.take<float>(En);
            cb.take<int64_t>(qc + 1);
            need_b = std::max(need_b, cb.off);
            if (need_b <= ctx->ws_cap) break;
            // the workspace must grow, which drops its contents: grow, then redo stage A
            st = ws_reserve(ctx, std::max(ca.off, need_b));
            if (st != TAC_OK) return st;
        }
        int32_t* top_id = ws_at<int32_t>(ctx, o_id);
        float* top_sim = ws_at<float>(ctx, o_sim);
        int64_t* eoff = ws_at<int64_t>(ctx, o_eoff);
        int32_t* cand = cand_d + q0 * kd;
        float* score = score_d + q0 * kd;
        if (E == 0) {
            Carve cq;
            cq.off = base_b;
            int64_t* qoff = ws_at<int64_t>(ctx, cq.take<int64_t>(qc + 1));
            TAC_HIP(hipMemsetAsync(qoff, 0, (qc + 1) * sizeof(int64_t), s));
            topk_docs<<<(unsigned)qc, kSelThreads, 0, s>>>(nullptr, nullptr, qoff, D, kd, cand, score);
            TAC_LAUNCH_CHECK("topk_docs");
            continue;
        }
        Carve cb;
        cb.off = base_b;
        uint32_t* keys = ws_at<uint32_t>(ctx, cb.take<uint32_t>(E));
        uint32_t* k1 = ws_at<uint32_t>(ctx, cb.take<uint32_t>(E));
        int32_t* v0 = ws_at<int32_t>(ctx, cb.take<int32_t>(E));
        int32_t* v1 = ws_at<int32_t>(ctx, cb.take<int32_t>(E));
        int32_t* tok = ws_at<int32_t>(ctx, cb.take<int32_t>(E));
        float* simv = ws_at<float>(ctx, cb.take<float>(E));
        void* sort_scr = ws_at<void>(ctx, cb.take<char>(radix_sort_scratch_bytes(E)));
        int64_t* flag = ws_at<int64_t>(ctx, cb.take<int64_t>(E + 1));
        int64_t* fidx = ws_at<int64_t>(ctx, cb.take<int64_t>(E + 1));
        void* scan2 = ws_at<void>(ctx, cb.take<char>(scan_scratch_bytes(E + 1)));
        int64_t* start = ws_at<int64_t>(ctx, cb.take<int64_t>(E + 1));
        uint32_t* seg_key = ws_at<uint32_t>(ctx, cb.take<uint32_t>(E));
        float* seg_score = ws_at<float>(ctx, cb.take<float>(E));
        int64_t* qoff = ws_at<int64_t>(ctx, cb.take<int64_t>(qc + 1));
        {
            const int waves_per_block = 4;
            emit_kernel<<<grid_for(nent, waves_per_block), 64 * waves_per_block, 0, s>>>(
                top_id, top_sim, nent, kc, nq, list_off_d, list_docs_d, K, D, eoff, keys, tok, simv);
            TAC_LAUNCH_CHECK("emit_kernel");
        }
        const uint32_t limit = (uint32_t)(qc * D);
        int in1 = 0;
        st = radix_sort(s, E, bits_for(limit), keys, v0, k1, v1, nullptr, sort_scr, &in1);
        if (st != TAC_OK) return st;
        const uint32_t* sk = in1 ? k1 : keys;
        const int32_t* sv = in1 ? v1 : v0;
        seg_flags<<<grid_for(E, 256), 256, 0, s>>>(sk, E, limit, flag);
        TAC_LAUNCH_CHECK("seg_flags");
        st = exclusive_scan_i64(s, flag, fidx, E, scan2);  // fidx[E] = number of groups
        if (st != TAC_OK) return st;
        seg_compact<<<grid_for(E, 256), 256, 0, s>>>(flag, fidx, E, start);
        TAC_LAUNCH_CHECK("seg_compact");
        seg_reduce<<<grid_for(E, 256), 256, 0, s>>>(sk, sv, E, tok, simv, start, fidx + E, seg_key, seg_score);
        TAC_LAUNCH_CHECK("seg_reduce");
        seg_qoff<<<grid_for(qc + 1, 256), 256, 0, s>>>(seg_key, fidx + E, qc, D, qoff);
        TAC_LAUNCH_CHECK("seg_qoff");
        topk_docs<<<(unsigned)qc, kSelThreads, 0, s>>>(seg_key, seg_score, qoff, D, kd, cand, score);
        TAC_LAUNCH_CHECK("topk_docs");
    }
    return TAC_OK;
}

namespace {

// Steps 2-4 of the gather for qc queries of nq tokens whose top lists (kc
// centroids and similarities per token, -1 for an empty slot) are given:
// list expansion, the per-(query, document) maxima and sums, the kd best
// documents.  The workspace from `base` on is this function's.
tac_status gather_from_top(tac_ctx ctx, const int32_t* top_id, const float* top_sim, int64_t qc, int32_t nq,
                           int32_t kc, const int64_t* list_off_d, const int32_t* list_docs_d, int64_t K, int64_t D,
                           int32_t kd, int32_t* cand, float* score, size_t base) {
    hipStream_t s = ctx->stream;
    const int64_t nent = qc * nq * kc;
    Carve ca;
    ca.off = base;
    const size_t o_eoff = ca.take<int64_t>(nent + 1);
    const size_t o_scan = ca.take<char>(scan_scratch_bytes(nent));
    const size_t base_b = ca.off;
    size_t need = ca.off;
    int64_t E = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        tac_status st = ws_reserve(ctx, need);
        if (st != TAC_OK) return st;
        int64_t* eoff = ws_at<int64_t>(ctx, o_eoff);
        emit_count<<<grid_for(nent, 256), 256, 0, s>>>(top_id, nent, list_off_d, K, eoff);
        TAC_LAUNCH_CHECK("emit_count");
        st = exclusive_scan_i64(s, eoff, eoff, nent, ws_at<void>(ctx, o_scan));
        if (st != TAC_OK) return st;
        TAC_HIP(hipMemcpyAsync(&E, eoff + nent, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        TAC_HIP(hipStreamSynchronize(s));
        Carve cb;
        cb.off = base_b;
        const int64_t En = std::max<int64_t>(E, 1);
        cb.take<uint32_t>(En);
        cb.take<uint32_t>(En);
        cb.take<int32_t>(En);
        cb.take<int32_t>(En);
        cb.take<int32_t>(En);
        cb.take<float>(En);
        cb.take<char>(radix_sort_scratch_bytes(En));
        cb.take<int64_t>(En + 1);
        cb.take<int64_t>(En + 1);
        cb.take<char>(scan_scratch_bytes(En + 1));
        cb.take<int64_t>(En + 1);
        cb.take<uint32_t>(En);
        cb.take<float>(En);
        cb.take<int64_t>(qc + 1);
        if (cb.off <= ctx->ws_cap) break;
        need = cb.off;  // growing drops the workspace's contents: count again after it
    }
    int64_t* eoff = ws_at<int64_t>(ctx, o_eoff);
    Carve cb;
    cb.off = base_b;
    if (E == 0) {
        int64_t* qoff = ws_at<int64_t>(ctx, cb.take<int64_t>(qc + 1));
        TAC_HIP(hipMemsetAsync(qoff, 0, (qc + 1) * sizeof(int64_t), s));
        topk_docs<<<(unsigned)qc, kSelThreads, 0, s>>>(nullptr, nullptr, qoff, D, kd, cand, score);
        TAC_LAUNCH_CHECK("topk_docs");
        return TAC_OK;
    }
    uint32_t* keys = ws_at<uint32_t>(ctx, cb.take<uint32_t>(E));
    uint32_t* k1 = ws_at<uint32_t>(ctx, cb.take<uint32_t>(E));
    int32_t* v0 = ws_at<int32_t>(ctx, cb.take<int32_t>(E));
    int32_t* v1 = ws_at<int32_t>(ctx, cb.take<int32_t>(E));
    int32_t* tok = ws_at<int32_t>(ctx, cb.take<int32_t>(E));
    float* simv = ws_at<float>(ctx, cb.take<float>(E));
    void* sort_scr = ws_at<void>(ctx, cb.take<char>(radix_sort_scratch_bytes(E)));
    int64_t* flag = ws_at<int64_t>(ctx, cb.take<int64_t>(E + 1));
    int64_t* fidx = ws_at<int64_t>(ctx, cb.take<int64_t>(E + 1));
    void* scan2 = ws_at<void>(ctx, cb.take<char>(scan_scratch_bytes(E + 1)));
    int64_t* start = ws_at<int64_t>(ctx, cb.take<int64_t>(E + 1));
    uint32_t* seg_key = ws_at<uint32_t>(ctx, cb.take<uint32_t>(E));
    float* seg_score = ws_at<float>(ctx, cb.take<float>(E));
    int64_t* qoff = ws_at<int64_t>(ctx, cb.take<int64_t>(qc + 1));
    {
        const int waves_per_block = 4;
        emit_kernel<<<grid_for(nent, waves_per_block), 64 * waves_per_block, 0, s>>>(
            top_id, top_sim, nent, kc, nq, list_off_d, list_docs_d, K, D, eoff, keys, tok, simv);
        TAC_LAUNCH_CHECK("emit_kernel");
    }
    const uint32_t limit = (uint32_t)(qc * D);
    int in1 = 0;
    tac_status st = radix_sort(s, E, bits_for(limit), keys, v0, k1, v1, nullptr, sort_scr, &in1);
    if (st != TAC_OK) return st;
    const uint32_t* sk = in1 ? k1 : keys;
    const int32_t* sv = in1 ? v1 : v0;
    seg_flags<<<grid_for(E, 256), 256, 0, s>>>(sk, E, limit, flag);
    TAC_LAUNCH_CHECK("seg_flags");
    st = exclusive_scan_i64(s, flag, fidx, E, scan2);
    if (st != TAC_OK) return st;
    seg_compact<<<grid_for(E, 256), 256, 0, s>>>(flag, fidx, E, start);
    TAC_LAUNCH_CHECK("seg_compact");
    seg_reduce<<<grid_for(E, 256), 256, 0, s>>>(sk, sv, E, tok, simv, start, fidx + E, seg_key, seg_score);
    TAC_LAUNCH_CHECK("seg_reduce");
    seg_qoff<<<grid_for(qc + 1, 256), 256, 0, s>>>(seg_key, fidx + E, qc, D, qoff);
    TAC_LAUNCH_CHECK("seg_qoff");
    topk_docs<<<(unsigned)qc, kSelThreads, 0, s>>>(seg_key, seg_score, qoff, D, kd, cand, score);
    TAC_LAUNCH_CHECK("topk_docs");
    return TAC_OK;
}

bool g_attr_search = false;

}  // namespace

extern "C" tac_status tac_graph_build(tac_ctx ctx, const float* C_d, int64_t K, int32_t d, int32_t* nbr_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_graph_build: ctx is NULL");
    if (d != kGDim) return set_error(TAC_E_INVAL, "tac_graph_build: d must be 128");
    if (K < 2 || K > INT32_MAX) return set_error(TAC_E_INVAL, "tac_graph_build: K must be in [2, 2^31)");
    if (!C_d || !nbr_d) return set_error(TAC_E_INVAL, "tac_graph_build: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t ldS = (K + 3) / 4 * 4;
    const int kk = kGraphDeg + 1;
    // rows per pass: the similarity block within kSimBudget
    const int64_t RC = std::max<int64_t>(64, std::min<int64_t>(K, kSimBudget / (ldS * 4)));
    Carve cw;
    const size_t o_fsim = cw.take<float>(K * kGraphDeg);
    const size_t o_id = cw.take<int32_t>(RC * kk), o_sim = cw.take<float>(RC * kk);
    const size_t o_S = cw.take<float>(RC * ldS);
    // the reverse-edge stage reuses the similarity block's memory
    Carve cr;
    cr.off = o_S;
    const size_t o_cnt = cr.take<int64_t>(K + 1), o_off = cr.take<int64_t>(K + 1), o_cur = cr.take<int64_t>(K + 1);
    const size_t o_scan = cr.take<char>(scan_scratch_bytes(K + 1));
    const size_t o_rsrc = cr.take<int32_t>(K * kGraphDeg), o_rsim = cr.take<float>(K * kGraphDeg);
    tac_status st = ws_reserve(ctx, std::max(cw.off, cr.off));
    if (st != TAC_OK) return st;
    float* fsim = ws_at<float>(ctx, o_fsim);
    int32_t* tid = ws_at<int32_t>(ctx, o_id);
    float* tsim = ws_at<float>(ctx, o_sim);
    float* S = ws_at<float>(ctx, o_S);
    for (int64_t r0 = 0; r0 < K; r0 += RC) {
        const int64_t R = std::min<int64_t>(RC, K - r0);
        const dim3 sg((unsigned)((K + 1023) / 1024), (unsigned)((R + 63) / 64));
        sim_kernel<<<sg, 256, 0, s>>>(C_d + r0 * kGDim, R, C_d, K, S, ldS);
        TAC_LAUNCH_CHECK("sim_kernel");
        topk_rows<<<(unsigned)R, kSelThreads, 0, s>>>(S, ldS, K, kk, tid, tsim);
        TAC_LAUNCH_CHECK("topk_rows");
        graph_forward<<<grid_for(R, 256), 256, 0, s>>>(tid, tsim, r0, R, nbr_d, fsim);
        TAC_LAUNCH_CHECK("graph_forward");
    }
    int64_t* cnt = ws_at<int64_t>(ctx, o_cnt);
    int64_t* off = ws_at<int64_t>(ctx, o_off);
    int64_t* cur = ws_at<int64_t>(ctx, o_cur);
    TAC_HIP(hipMemsetAsync(cnt, 0, (K + 1) * sizeof(int64_t), s));
    TAC_HIP(hipMemsetAsync(cur, 0, (K + 1) * sizeof(int64_t), s));
    const unsigned eg = grid_for(K * kGraphDeg, 256);
    rev_count<<<eg, 256, 0, s>>>(nbr_d, K, cnt);
    TAC_LAUNCH_CHECK("rev_count");
    st = exclusive_scan_i64(s, cnt, off, K + 1, ws_at<void>(ctx, o_scan));
    if (st != TAC_OK) return st;
    rev_fill<<<eg, 256, 0, s>>>(nbr_d, fsim, K, off, cur, ws_at<int32_t>(ctx, o_rsrc), ws_at<float>(ctx, o_rsim));
    TAC_LAUNCH_CHECK("rev_fill");
    rev_select<<<grid_for(K, 4), 256, 0, s>>>(off, ws_at<int32_t>(ctx, o_rsrc), ws_at<float>(ctx, o_rsim), K, nbr_d);
    TAC_LAUNCH_CHECK("rev_select");
    return TAC_OK;
}

extern "C" tac_status tac_graph_search(tac_ctx ctx, const float* Q_d, int64_t R, int32_t d, const float* C_d,
                                       int64_t K, const int32_t* nbr_d, const int32_t* entry_d, int64_t nentry,
                                       int32_t ef, int32_t kc, int32_t* top_id_d, float* top_sim_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_graph_search: ctx is NULL");
    if (d != kGDim) return set_error(TAC_E_INVAL, "tac_graph_search: d must be 128");
    if (R < 0 || K < 2 || K > INT32_MAX || nentry < 1 || nentry > K)
        return set_error(TAC_E_INVAL, "tac_graph_search: bad sizes");
    if (ef < 1 || ef > kMaxEf || kc < 1 || kc > ef)
        return set_error(TAC_E_INVAL, "tac_graph_search: need 1 <= kappa_c <= ef <= 64");
    if (R == 0) return TAC_OK;
    if (!Q_d || !C_d || !nbr_d || !entry_d || !top_id_d || !top_sim_d)
        return set_error(TAC_E_INVAL, "tac_graph_search: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t ldE = (nentry + 3) / 4 * 4;
    // query rows per pass: the router similarities within kSimBudget
    const int64_t RC = std::max<int64_t>(64, std::min<int64_t>(R, kSimBudget / (ldE * 4)));
    Carve cw;
    const size_t o_er = cw.take<float>(nentry * kGDim);
    const size_t o_pick = cw.take<int32_t>(RC * ef), o_psim = cw.take<float>(RC * ef), o_init = cw.take<int32_t>(RC * ef);
    const size_t o_S = cw.take<float>(RC * ldE);
    tac_status st = ws_reserve(ctx, cw.off);
    if (st != TAC_OK) return st;
    float* Er = ws_at<float>(ctx, o_er);
    gather_rows128<<<grid_for(nentry, 8), 256, 0, s>>>(C_d, K, entry_d, nentry, Er);
    TAC_LAUNCH_CHECK("gather_rows128");
    if (!g_attr_search) {
        TAC_HIP(hipFuncSetAttribute((const void*)graph_search, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)sizeof(SearchShared)));
        g_attr_search = true;
    }
    for (int64_t r0 = 0; r0 < R; r0 += RC) {
        const int64_t Rc = std::min<int64_t>(RC, R - r0);
        const dim3 sg((unsigned)((nentry + 1023) / 1024), (unsigned)((Rc + 63) / 64));
        sim_kernel<<<sg, 256, 0, s>>>(Q_d + r0 * kGDim, Rc, Er, nentry, ws_at<float>(ctx, o_S), ldE);
        TAC_LAUNCH_CHECK("sim_kernel");
        topk_rows<<<(unsigned)Rc, kSelThreads, 0, s>>>(ws_at<float>(ctx, o_S), ldE, nentry, ef,
                                                       ws_at<int32_t>(ctx, o_pick), ws_at<float>(ctx, o_psim));
        TAC_LAUNCH_CHECK("topk_rows");
        map_ids<<<grid_for(Rc * ef, 256), 256, 0, s>>>(ws_at<int32_t>(ctx, o_pick), Rc * ef, entry_d,
                                                      ws_at<int32_t>(ctx, o_init));
        TAC_LAUNCH_CHECK("map_ids");
        graph_search<<<(unsigned)((Rc + kSearchWaves - 1) / kSearchWaves), 64 * kSearchWaves, sizeof(SearchShared),
                       s>>>(Q_d + r0 * kGDim, Rc, C_d, K, nbr_d, ws_at<int32_t>(ctx, o_init), ef, kc, 64 * ef,
                            top_id_d + r0 * kc, top_sim_d + r0 * kc, nullptr);
        TAC_LAUNCH_CHECK("graph_search");
    }
    return TAC_OK;
}

extern "C" tac_status tac_gather_lists(tac_ctx ctx, const int32_t* top_id_d, const float* top_sim_d, int64_t B,
                                       int32_t nq, int32_t kc, const int64_t* list_off_d, const int32_t* list_docs_d,
                                       int64_t K, int64_t D, int32_t kd, int32_t* cand_d, float* score_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_gather_lists: ctx is NULL");
    if (B < 0 || nq < 1 || nq > 1024 || K < 1 || K > INT32_MAX || D < 1 || D > INT32_MAX)
        return set_error(TAC_E_INVAL, "tac_gather_lists: bad sizes");
    if (kc < 1 || kc > kMaxKc) return set_error(TAC_E_INVAL, "tac_gather_lists: kappa_c must be in [1, 256]");
    if (kd < 1 || kd > kMaxKd) return set_error(TAC_E_INVAL, "tac_gather_lists: kappa_d must be in [1, 4096]");
    if (B == 0) return TAC_OK;
    if (!top_id_d || !top_sim_d || !list_off_d || !list_docs_d || !cand_d || !score_d)
        return set_error(TAC_E_INVAL, "tac_gather_lists: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    // queries per pass: the keys q * D + d within 32 bits
    const int64_t QC = std::min<int64_t>(B, ((int64_t)UINT32_MAX - 1) / D);
    if (QC < 1) return set_error(TAC_E_INVAL, "tac_gather_lists: too many documents for 32-bit keys");
    for (int64_t q0 = 0; q0 < B; q0 += QC) {
        const int64_t qc = std::min<int64_t>(QC, B - q0);
        const tac_status st = gather_from_top(ctx, top_id_d + q0 * nq * kc, top_sim_d + q0 * nq * kc, qc, nq, kc,
                                              list_off_d, list_docs_d, K, D, kd, cand_d + q0 * kd, score_d + q0 * kd, 0);
        if (st != TAC_OK) return st;
    }
    return TAC_OK;
}

extern "C" tac_status tac_centroid_topk(tac_ctx ctx, const float* Q_d, int64_t R, int32_t d, const float* C_d,
                                        int64_t K, int32_t kc, int32_t* top_id_d, float* top_sim_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_centroid_topk: ctx is NULL");
    if (d != kGDim) return set_error(TAC_E_INVAL, "tac_centroid_topk: d must be 128");
    if (R < 0 || K < 1 || K > INT32_MAX) return set_error(TAC_E_INVAL, "tac_centroid_topk: bad sizes");
    if (kc < 1 || kc > kMaxKc) return set_error(TAC_E_INVAL, "tac_centroid_topk: kappa_c must be in [1, 256]");
    if (R == 0) return TAC_OK;
    if (!Q_d || !C_d || !top_id_d || !top_sim_d) return set_error(TAC_E_INVAL, "tac_centroid_topk: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t ldS = (K + 3) / 4 * 4;
    const int64_t RC = std::max<int64_t>(64, std::min<int64_t>(R, kSimBudget / (ldS * 4)));
    Carve cw;
    const size_t o_S = cw.take<float>(RC * ldS);
    tac_status st = ws_reserve(ctx, cw.off);
    if (st != TAC_OK) return st;
    for (int64_t r0 = 0; r0 < R; r0 += RC) {
        const int64_t Rc = std::min<int64_t>(RC, R - r0);
        const dim3 sg((unsigned)((K + 1023) / 1024), (unsigned)((Rc + 63) / 64));
        sim_kernel<<<sg, 256, 0, s>>>(Q_d + r0 * kGDim, Rc, C_d, K, ws_at<float>(ctx, o_S), ldS);
        TAC_LAUNCH_CHECK("sim_kernel");
        topk_rows<<<(unsigned)Rc, kSelThreads, 0, s>>>(ws_at<float>(ctx, o_S), ldS, K, kc, top_id_d + r0 * kc,
                                                       top_sim_d + r0 * kc);
        TAC_LAUNCH_CHECK("topk_rows");
    }
    return TAC_OK;
}
