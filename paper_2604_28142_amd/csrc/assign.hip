// Assignment step of per-token Lloyd (Sect. 2.1): every vector of token j goes
// to the nearest of token j's centroids.
//
// One persistent launch serves every token.  The work list holds one item per
// (token, row tile); items of tokens with many centroids come first, so the
// longest items start early.  Each item takes one of two routes, split at a
// tunable kappa limit (default 4, at most 16):
//
// * direct (few centroids): every centroid is a candidate, so each row computes
//   the canonical FP32 distance to all of them;
// * screen (more centroids): the distance contraction ||c||^2 - 2 x.c runs on the
//   matrix cores (FP32 v_mfma_f32_16x16x4f32, or BF16 v_mfma_f32_16x16x32_bf16
//   on hi/lo splits of both operands), centroid tiles are staged through LDS,
//   and every lane keeps a running top-k (4 for FP32, 3 for BF16) of packed
//   (screen value, index) keys with one min and k - 1 med3 per distance.  At
//   the end of an item each row's candidates (the lists of its four lanes) are
//   rescored with the canonical FP32 distance where the screen bound cannot
//   exclude them; a rigorous bound on the screen error certifies that no other
//   centroid can win, and rows whose certificate fails are queued for a batched
//   exhaustive rescoring kernel.
//
// The canonical distance is acc = 0; for i: t = x_i - c_i; acc = acc + t*t,
// each operation rounded to float32 without fusion, so the result is the same
// for the FP32 and BF16 screens and independent of tile shapes.
#include <algorithm>
#include <cfloat>
#include <mutex>
#include <type_traits>

#include "tac_internal.h"

namespace tac {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kNB = 4;                          // 16-row column blocks per wave
constexpr int kTileRows = kWaves * kNB * 16;    // rows per screened work item
constexpr int kStage = 64;                      // centroids per LDS stage
constexpr int kRowWords = 132;                  // LDS row stride (512 B + 16 B pad)
constexpr int kEpochBlocks = 64;                // 16-centroid blocks per packed-index epoch
constexpr int kDirectCap = 16;                  // most centroids a direct (screen-free) token may have
constexpr float kInvalid = 3.0e38f;             // screen value of padding centroids
constexpr unsigned kCntRows = 0, kCntScreened = 1, kCntFallback = 2, kCntUnassigned = 3;
// dynamic LDS of the assignment kernel: two centroid stages, their norms, then the
// per-lane merged top-4 lists (value and index words) of every wave
constexpr size_t kGlistOffsetWords = (size_t)2 * kStage * kRowWords + (size_t)2 * kStage;
constexpr size_t kLdsBytes = (kGlistOffsetWords + (size_t)kWaves * kNB * 8 * 64) * 4;

__device__ __forceinline__ float dist32_rows(const float* __restrict__ x, const float* __restrict__ c, float* xx) {
    const float4* xv = reinterpret_cast<const float4*>(x);
    const float4* cv = reinterpret_cast<const float4*>(c);
    float acc = 0.f, sx = 0.f;
    // sixteen iterations' loads are issued together: two latency rounds per row
#pragma unroll 16
    for (int i = 0; i < kDim / 4; ++i) {
        const float4 a = xv[i];
        const float4 b = cv[i];
        float t;
        t = __fsub_rn(a.x, b.x); acc = __fadd_rn(acc, __fmul_rn(t, t)); sx = __fadd_rn(sx, __fmul_rn(a.x, a.x));
        t = __fsub_rn(a.y, b.y); acc = __fadd_rn(acc, __fmul_rn(t, t)); sx = __fadd_rn(sx, __fmul_rn(a.y, a.y));
        t = __fsub_rn(a.z, b.z); acc = __fadd_rn(acc, __fmul_rn(t, t)); sx = __fadd_rn(sx, __fmul_rn(a.z, a.z));
        t = __fsub_rn(a.w, b.w); acc = __fadd_rn(acc, __fmul_rn(t, t)); sx = __fadd_rn(sx, __fmul_rn(a.w, a.w));
    }
    if (xx) *xx = sx;
    return acc;
}

// The same canonical distance with the x row already in registers (a row
// rescored against several candidates is loaded once, all of it in flight at
// once); the loop is fully unrolled so that the row stays in registers.
__device__ __forceinline__ float dist32_xreg(const float4 (&xv)[kDim / 4], const float* __restrict__ c, float* xx) {
    const float4* cv = reinterpret_cast<const float4*>(c);
    float acc = 0.f, sx = 0.f;
#pragma unroll
    for (int i = 0; i < kDim / 4; ++i) {
        const float4 a = xv[i];
        const float4 b = cv[i];
        float t;
        t = __fsub_rn(a.x, b.x); acc = __fadd_rn(acc, __fmul_rn(t, t)); sx = __fadd_rn(sx, __fmul_rn(a.x, a.x));
        t = __fsub_rn(a.y, b.y); acc = __fadd_rn(acc, __fmul_rn(t, t)); sx = __fadd_rn(sx, __fmul_rn(a.y, a.y));
        t = __fsub_rn(a.z, b.z); acc = __fadd_rn(acc, __fmul_rn(t, t)); sx = __fadd_rn(sx, __fmul_rn(a.z, a.z));
        t = __fsub_rn(a.w, b.w); acc = __fadd_rn(acc, __fmul_rn(t, t)); sx = __fadd_rn(sx, __fmul_rn(a.w, a.w));
    }
    if (xx) *xx = sx;
    return acc;
}

__device__ __forceinline__ unsigned short bf16_rne(float v) {
    return __builtin_bit_cast(unsigned short, (__bf16)v);  // v_cvt_pk_bf16_f32: round to nearest even
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// ---- per-call reset of the work counter, statistics and max centroid norm ----
__global__ void reset_call(unsigned long long* __restrict__ work, unsigned long long* __restrict__ counters,
                           unsigned* __restrict__ cstat, const unsigned* __restrict__ cstat_static) {
    work[0] = 0;
    for (int i = 0; i < 4; ++i) counters[i] = 0;
    // the centroid bounds come from prep_centroids, or from the prepared static centroids
    cstat[0] = cstat_static ? cstat_static[0] : 0;
    cstat[1] = 0;
    cstat[2] = cstat_static ? cstat_static[2] : 0;
}

// ---- plan: item counts per (class, token) ----
// Split route (16-bit screens): a token of at most kSplitMaxRows rows and at
// least kSplitMinKappa centroids -- the shape of a serving batch's frequent
// tokens; a clustering budget gives such a kappa only to tokens with far more
// rows -- is cut into (row tile, chunk of kSplitChunk centroids) work items of a second
// launch spread over the device, where the persistent kernel would screen all
// of the token's centroids for a row tile on one CU.  Each item's exact per-row
// minimum over its chunk (with its own certificate) meets the other chunks' in
// a 64-bit (distance bits, index) atomicMin slot per row; a row whose
// certificate fails in any chunk goes, once, to the token's fallback queue,
// which rescores every centroid of the token.
constexpr int kSplitMaxRows = 8192;
constexpr int kSplitMinKappa = 2048;
constexpr int kSplitChunk = 1024;

// work items per (class, token): class 0 heavy screen, 1 screen, 2 direct,
// 3 split (row tiles x centroid chunks); after them, at 4T + j, the split
// token's row count (its scan gives the token's first row slot)
__global__ void plan_count(const int64_t* __restrict__ seg_off, const int64_t* __restrict__ cent_off, int32_t T,
                           int direct_max, int heavy, int split_min, int screen_rows, int direct_rows,
                           int64_t* __restrict__ cnt, unsigned* __restrict__ kmax) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= T) return;
    const int64_t n = seg_off[j + 1] - seg_off[j];
    const int64_t k = cent_off[j + 1] - cent_off[j];
    if (n > 0 && k > 0) atomicMax(kmax, (unsigned)k);
    int cls;
    if (k == 0 || k <= direct_max)
        cls = 2;
    else if (split_min > 0 && n > 0 && n <= kSplitMaxRows && k >= split_min)
        cls = 3;
    else
        cls = k >= heavy ? 0 : 1;
    const int64_t rows = cls == 2 ? direct_rows : screen_rows;
    const int64_t tiles = (n + rows - 1) / rows;
    const int64_t items = cls == 3 ? tiles * ((k + kSplitChunk - 1) / kSplitChunk) : tiles;
    for (int c = 0; c < 4; ++c) cnt[(int64_t)c * T + j] = c == cls ? items : 0;
    cnt[4 * (int64_t)T + j] = cls == 3 ? n : 0;
}

// Everything a work item needs, in one 32-byte record, so that an item's first
// memory access is its x rows (the persistent loop fetches the next item's
// record while the current item runs).
struct ItemDesc {
    int64_t row0;  // first sorted row of the item
    int64_t s1;    // end of the token's rows
    int64_t k0;    // first centroid of the token
    int32_t kc;    // centroids of the token
    int32_t jc;    // class << 24 | token
};
static_assert(sizeof(ItemDesc) == 32, "one 32-byte record per item");

// item descriptors from the scanned item offsets: items of (class, token) pair
// idx = class * T + token cut the token's rows into tiles of the class's size,
// split-route items (class 3) into (row tile, centroid chunk) pairs.  One
// thread per item, which finds its (class, token) by binary search over the
// offsets, so that a token of thousands of items does not fall to one thread.
__global__ void plan_fill(const int64_t* __restrict__ item_off, const int64_t* __restrict__ seg_off,
                          const int64_t* __restrict__ cent_off, int32_t T, int screen_rows, int direct_rows,
                          ItemDesc* __restrict__ desc) {
    const int64_t ncls = 4 * (int64_t)T;
    const int64_t total = item_off[ncls];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = ncls;  // the last idx with item_off[idx] <= t (a non-empty range)
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (item_off[mid] <= t) lo = mid; else hi = mid;
        }
        const int64_t idx = lo, b = item_off[idx];
        const int cls = (int)(idx / T);
        const int32_t j = (int32_t)(idx - (int64_t)cls * T);
        const int64_t rows = cls == 2 ? direct_rows : screen_rows;
        ItemDesc d;
        d.s1 = seg_off[j + 1];
        d.k0 = cent_off[j];
        d.kc = (int32_t)(cent_off[j + 1] - d.k0);
        d.jc = (cls << 24) | j;
        const int64_t s0 = seg_off[j];
        if (cls == 3) {
            const int64_t k0 = d.k0, kc = d.kc;
            const int64_t chunks = (kc + kSplitChunk - 1) / kSplitChunk;
            const int64_t tile = (t - b) / chunks, c = (t - b) - tile * chunks;
            d.row0 = s0 + tile * rows;
            d.k0 = k0 + c * kSplitChunk;
            d.kc = (int32_t)min((int64_t)kSplitChunk, kc - c * kSplitChunk);
        } else {
            d.row0 = s0 + (t - b) * rows;
        }
        desc[t] = d;
    }
}

// the split route's per-row slots (best candidate, queued flag), one thread per
// (split token, row)
__global__ void plan_split_slots(const int64_t* __restrict__ item_off, const int64_t* __restrict__ seg_off,
                                 int32_t T, unsigned long long* __restrict__ sslot, int32_t* __restrict__ sflag) {
    const int64_t base = item_off[4 * (int64_t)T];
    for (int64_t j = blockIdx.x; j < T; j += gridDim.x) {
        if (item_off[3 * (int64_t)T + j] == item_off[3 * (int64_t)T + j + 1]) continue;
        const int64_t sb = item_off[4 * (int64_t)T + j] - base;
        const int64_t n = seg_off[j + 1] - seg_off[j];
        for (int64_t q = threadIdx.x; q < n; q += blockDim.x) {
            sslot[sb + q] = ~0ull;
            sflag[sb + q] = 0;
        }
    }
}

// ---- centroid preparation: squared norms, max norm, 16-bit staging rows ----
// BF16: hi/lo splits (hi = bf16(c), lo = bf16(c - hi)), 512 B per centroid.
// FP16: one rounding c16 = f16(c), 256 B per centroid, and the largest
// ||c - c16||^2 over all centroids into cstat[2] (the FP16 certificate's
// operand-rounding bound).
__global__ void __launch_bounds__(256) prep_centroids(const float* __restrict__ C, int64_t K, float* __restrict__ cn,
                                                      unsigned* __restrict__ cstat, unsigned short* __restrict__ chl,
                                                      int prec) {
    __shared__ unsigned red[256];
    __shared__ unsigned redd[256];
    const int sub = threadIdx.x & 31;
    unsigned mx = 0, mxd = 0;
    for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5; k < K;
         k += ((int64_t)gridDim.x * blockDim.x) >> 5) {
        const float4 v = reinterpret_cast<const float4*>(C + k * kDim)[sub];
        float s = v.x * v.x;
        s = s + v.y * v.y;
        s = s + v.z * v.z;
        s = s + v.w * v.w;
        for (int m = 16; m > 0; m >>= 1) s += __shfl_xor(s, m, 32);
        if (sub == 0) cn[k] = s;
        mx = max(mx, __float_as_uint(s));  // non-negative floats order like their bit patterns
        if (chl && prec == TAC_F16) {
            const float e[4] = {v.x, v.y, v.z, v.w};
            unsigned short h[4];
            float dd = 0.f;
            for (int i = 0; i < 4; ++i) {
                const _Float16 q = (_Float16)e[i];
                h[i] = __builtin_bit_cast(unsigned short, q);
                const float r = e[i] - (float)q;  // exact: q is e rounded to a coarser grid
                dd = dd + r * r;
            }
            for (int m = 16; m > 0; m >>= 1) dd += __shfl_xor(dd, m, 32);
            // a non-finite residual (|c| beyond the FP16 range) becomes +inf, so that the bound disables the screen
            mxd = max(mxd, dd <= FLT_MAX ? __float_as_uint(dd) : 0x7F800000u);
            uint2 hv;
            hv.x = h[0] | ((unsigned)h[1] << 16);
            hv.y = h[2] | ((unsigned)h[3] << 16);
            reinterpret_cast<uint2*>(chl + k * kDim)[sub] = hv;
        } else if (chl) {
            const float e[4] = {v.x, v.y, v.z, v.w};
            unsigned short hi[4], lo[4];
            for (int i = 0; i < 4; ++i) {
                hi[i] = bf16_rne(e[i]);
                lo[i] = bf16_rne(e[i] - bf16_to_f(hi[i]));
            }
            unsigned short* row = chl + k * (2 * kDim);
            uint2 h, l;
            h.x = hi[0] | ((unsigned)hi[1] << 16);
            h.y = hi[2] | ((unsigned)hi[3] << 16);
            l.x = lo[0] | ((unsigned)lo[1] << 16);
            l.y = lo[2] | ((unsigned)lo[3] << 16);
            reinterpret_cast<uint2*>(row)[sub] = h;
            reinterpret_cast<uint2*>(row + kDim)[sub] = l;
        }
    }
    red[threadIdx.x] = mx;
    redd[threadIdx.x] = mxd;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + off]);
            redd[threadIdx.x] = max(redd[threadIdx.x], redd[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicMax(cstat, red[0]);
    if (threadIdx.x == 0 && redd[0]) atomicMax(cstat + 2, redd[0]);
}

struct Params {
    const float* x;
    const int32_t* rowmap;       // sorted position -> physical row (NULL: identity)
    const int64_t* seg_off;
    const int64_t* cent_off;
    int32_t T;
    const float* C;
    const void* cstage;          // rows staged into LDS: C (FP32), hi/lo BF16 pairs or FP16 rows
    const float* cn;
    const unsigned* cstat;       // [0] = bits of max ||c||^2, [1] = max kappa, [2] = bits of max ||c - f16(c)||^2
    const int64_t* item_off;     // [4T + 1]: items of classes 0-2, then the split items
    const ItemDesc* desc;        // per item
    unsigned long long* work;
    int32_t* assign;
    float* dist;
    // Fallback queue, grouped by token: the k-th failed row of token j sits at
    // index seg_off[j] + k (k < fbcnt[j]) with its physical row, its canonical
    // ||x||^2 and a 64-bit (distance bits, index) slot holding its best exact
    // candidate so far.
    int32_t* fbq;
    float* fbxx;
    unsigned long long* fbslot;
    int32_t* fbcnt;
    unsigned long long* counters;
};

// Per-row state of the split route's rows (see kSplitMaxRows): the best exact
// candidate over the chunks so far, and whether the row is already queued.
struct SplitArgs {
    unsigned long long* slot;
    int32_t* flag;
};

__device__ __forceinline__ unsigned med3u(unsigned a, unsigned b, unsigned c) {
    unsigned r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Running top-4 of packed keys (bit pattern of a non-negative float with its low
// 8 bits replaced by a lane-local candidate index): one min and three med3.
__device__ __forceinline__ void list_insert(unsigned (&l)[4], unsigned p) {
    l[3] = med3u(l[2], l[3], p);
    l[2] = med3u(l[1], l[2], p);
    l[1] = med3u(l[0], l[1], p);
    l[0] = min(l[0], p);
}

// The same running top-LK (LK <= 4) on keys held as floats: the keys are
// non-negative finite floats, which order like their bit patterns, and med3 of
// floats selects one of its inputs exactly.  The empty slot is FLT_MAX.
template <int LK>
__device__ __forceinline__ void list_insert(float (&l)[4], float p) {
#pragma unroll
    for (int e = LK - 1; e >= 1; --e) l[e] = __builtin_amdgcn_fmed3f(l[e - 1], l[e], p);
    l[0] = __builtin_amdgcn_fmed3f(l[0], p, -FLT_MAX);  // min without an IEEE canonicalisation
}
__device__ __forceinline__ unsigned key_bits(unsigned k) { return k; }
__device__ __forceinline__ unsigned key_bits(float k) { return __float_as_uint(k); }
template <class K>
__device__ __forceinline__ K key_empty();
template <>
__device__ __forceinline__ unsigned key_empty<unsigned>() { return 0xFFFFFFFFu; }
template <>
__device__ __forceinline__ float key_empty<float>() { return FLT_MAX; }

// Insert (t, i) into the ascending list (G, I) of length L; `lex` breaks value
// ties by index.
template <int L>
__device__ __forceinline__ void glist_insert(float (&G)[4], int (&I)[4], float t, int i, bool lex) {
    bool c[L];
#pragma unroll
    for (int e = 0; e < L; ++e) c[e] = t < G[e] || (lex && t == G[e] && (unsigned)i < (unsigned)I[e]);
#pragma unroll
    for (int e = L - 1; e >= 1; --e) {
        G[e] = c[e - 1] ? G[e - 1] : (c[e] ? t : G[e]);
        I[e] = c[e - 1] ? I[e - 1] : (c[e] ? i : I[e]);
    }
    G[0] = c[0] ? t : G[0];
    I[0] = c[0] ? i : I[0];
}

// x fragments of the NB column blocks (16 rows each) a wave owns for a whole
// item: FP32 keeps -2x, BF16 keeps hi/lo BF16 splits of -2x.  Lane group g
// holds coordinates [32g, 32g + 32) of row `col` of each block.
template <int PREC, int NB>
struct Frag;

template <int NB>
struct Frag<TAC_FP32, NB> {
    float x[NB][32];
};

template <int NB>
struct Frag<TAC_BF16, NB> {
    bf8 xh[NB][4];
    bf8 xl[NB][4];
};

template <int NB>
struct Frag<TAC_F16, NB> {
    h8 xh[NB][4];
};

typedef unsigned short us8 __attribute__((ext_vector_type(8)));

// Move a 16-bit fragment into accumulation registers (AGPRs).  The 16-bit
// screens' x operands stay there for a whole item and feed the matrix cores
// directly, which leaves the VGPRs to the accumulators, lists and centroid fragments.
template <class V>
__device__ __forceinline__ V to_agpr(V v) {
    const u4 u = __builtin_bit_cast(u4, v);
    unsigned a0, a1, a2, a3;
    asm("v_accvgpr_write_b32 %0, %1" : "=a"(a0) : "v"(u[0]));
    asm("v_accvgpr_write_b32 %0, %1" : "=a"(a1) : "v"(u[1]));
    asm("v_accvgpr_write_b32 %0, %1" : "=a"(a2) : "v"(u[2]));
    asm("v_accvgpr_write_b32 %0, %1" : "=a"(a3) : "v"(u[3]));
    const u4 r = {a0, a1, a2, a3};
    return __builtin_bit_cast(V, r);
}

// hi = bf16(v), lo = bf16(v - hi) for 8 consecutive values (round to nearest even)
__device__ __forceinline__ void split_bf8(const float* v, bf8& hi, bf8& lo) {
    us8 h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const unsigned short a = bf16_rne(v[e]);
        h[e] = a;
        l[e] = bf16_rne(v[e] - bf16_to_f(a));
    }
    hi = __builtin_bit_cast(bf8, h);
    lo = __builtin_bit_cast(bf8, l);
}

// Direct route: one row per thread, every centroid of the token a candidate.
template <int ROWS>
__device__ __forceinline__ void direct_item(const Params& P, const ItemDesc& D) {
    const int64_t s1 = D.s1;
    const int64_t k0 = D.k0;
    const int kc = D.kc;
    const int64_t row0 = D.row0;
    const int64_t v = row0 + threadIdx.x;
    const bool valid = v < s1;
    if (valid) {
        const int64_t r = P.rowmap ? (int64_t)P.rowmap[v] : v;
        if (kc == 0) {
            P.assign[r] = -1;
            P.dist[r] = 0.f;
        } else {
            // centroid by centroid, each a canonical distance with eight float4
            // iterations' loads in flight; the first minimum wins ties
            const float* xr = P.x + r * kDim;
            float bd = INFINITY;
            int best = 0;
            for (int k = 0; k < kc; ++k) {
                const float d = dist32_rows(xr, P.C + (k0 + k) * kDim, nullptr);
                if (d < bd) {
                    bd = d;
                    best = k;
                }
            }
            P.assign[r] = (int32_t)(k0 + best);
            P.dist[r] = bd;
        }
    }
    const unsigned long long nval = __popcll(__ballot(valid));
    if ((threadIdx.x & 63) == 0 && nval) {
        atomicAdd(&P.counters[kCntRows], nval);
        if (kc == 0) atomicAdd(&P.counters[kCntUnassigned], nval);
    }
}

// Load and convert the wave's x fragments (rows row0 .. row0 + 16 NB - 1, those
// at or past s1 as zeros); returns the largest ||x||^2 over the wave's rows.
// FP16 also stores each row's ||-2x - f16(-2x)||^2 at sdx[16 nb + col].  The
// 16-bit screens pass xt, the wave's transpose area (16 rows of kXtStride words).
constexpr int kXtStride = kDim + 4;
template <int PREC, int NB, int GROUP = NB, bool AGPR = true>
__device__ __forceinline__ float load_x_frags(const Params& P, int64_t row0, int64_t s1, int g, int col,
                                              Frag<PREC, NB>& F, float* sdx = nullptr, float* xt = nullptr) {
    float xxmax = 0.f;
    if constexpr (PREC == TAC_FP32) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            __builtin_amdgcn_sched_barrier(0);  // one column block at a time (bounded live registers)
            const int64_t v = row0 + nb * 16 + col;
            const bool valid = v < s1;
            const int64_t r = valid ? (P.rowmap ? (int64_t)P.rowmap[v] : v) : 0;
            const float4* xv = reinterpret_cast<const float4*>(P.x + r * kDim + 32 * g);
            float xx = 0.f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 a = valid ? xv[q] : make_float4(0.f, 0.f, 0.f, 0.f);
                xx += a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w;
                F.x[nb][4 * q + 0] = -2.0f * a.x;
                F.x[nb][4 * q + 1] = -2.0f * a.y;
                F.x[nb][4 * q + 2] = -2.0f * a.z;
                F.x[nb][4 * q + 3] = -2.0f * a.w;
            }
            xx += __shfl_xor(xx, 16);
            xx += __shfl_xor(xx, 32);
            xxmax = fmaxf(xxmax, xx);
        }
    } else {
        // The rows of GROUP column blocks are loaded before any is converted, so
        // that their loads are in flight together (all NB blocks at once when a
        // wave has the SIMD's registers to itself).  Each load instruction reads
        // 1 KiB of contiguous memory (lane l: 16 bytes of row 2 i + l / 32), and
        // each 16-row block is turned into the fragment layout through the
        // wave's transpose area in LDS (rows padded to 528 bytes); a
        // fragment-layout load straight from memory would touch 64 cache lines
        // per instruction.  Row numbers fit in 32 bits (N <= INT32_MAX).
        static_assert(NB % GROUP == 0, "whole groups of column blocks");
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int nb0 = 0; nb0 < NB; nb0 += GROUP) {
            float4 ld[GROUP][8];
            // physical rows first (the serving path's row map), all lookups in flight together
            int32_t rr[GROUP][8];
#pragma unroll
            for (int q = 0; q < GROUP; ++q)
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int64_t v = row0 + (nb0 + q) * 16 + 2 * i + (lane >> 5);
                    rr[q][i] = v < s1 ? (int32_t)v : -1;
                }
            if (P.rowmap) {  // unconditional lookups (rows past s1 read the last row's entry) keep them in flight together
                int32_t m[GROUP][8];
#pragma unroll
                for (int q = 0; q < GROUP; ++q)
#pragma unroll
                    for (int i = 0; i < 8; ++i) m[q][i] = P.rowmap[rr[q][i] >= 0 ? (int64_t)rr[q][i] : s1 - 1];
#pragma unroll
                for (int q = 0; q < GROUP; ++q)
#pragma unroll
                    for (int i = 0; i < 8; ++i) rr[q][i] = rr[q][i] >= 0 ? m[q][i] : -1;
            }
#pragma unroll
            for (int q = 0; q < GROUP; ++q)
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    ld[q][i] = rr[q][i] >= 0 ? reinterpret_cast<const float4*>(P.x + (int64_t)rr[q][i] * kDim)[lane & 31]
                                             : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int q = 0; q < GROUP; ++q) {
                const int nb = nb0 + q;
                float xx = 0.f, dyy = 0.f;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    *reinterpret_cast<float4*>(xt + (2 * i + (lane >> 5)) * kXtStride + 4 * (lane & 31)) = ld[q][i];
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                float4 fr[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) fr[c] = *reinterpret_cast<const float4*>(xt + col * kXtStride + 32 * g + 4 * c);
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the next block rewrites the area
                // eight coordinates at a time straight into the 16-bit fragments
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const float4 a = fr[2 * s];
                    const float4 b = fr[2 * s + 1];
                    xx += a.x * a.x + a.y * a.y + a.z * a.z + a.w * a.w + b.x * b.x + b.y * b.y + b.z * b.z + b.w * b.w;
                    const float v8[8] = {-2.0f * a.x, -2.0f * a.y, -2.0f * a.z, -2.0f * a.w,
                                         -2.0f * b.x, -2.0f * b.y, -2.0f * b.z, -2.0f * b.w};
                    if constexpr (PREC == TAC_BF16) {
                        bf8 hi, lo;
                        split_bf8(v8, hi, lo);
                        F.xh[nb][s] = AGPR ? to_agpr(hi) : hi;
                        F.xl[nb][s] = AGPR ? to_agpr(lo) : lo;
                    } else {
                        h8 h;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            h[e] = (_Float16)v8[e];
                            const float r = v8[e] - (float)h[e];  // exact: h is v rounded to a coarser grid
                            dyy = dyy + r * r;
                        }
                        F.xh[nb][s] = AGPR ? to_agpr(h) : h;
                    }
                }
                xx += __shfl_xor(xx, 16);
                xx += __shfl_xor(xx, 32);
                xxmax = fmaxf(xxmax, xx);
                if constexpr (PREC == TAC_F16) {
                    dyy += __shfl_xor(dyy, 16);
                    dyy += __shfl_xor(dyy, 32);
                    if (g == 0) sdx[nb * 16 + col] = dyy;
                }
            }
        }
    }
    // keep every fragment write far above the first matrix-core read
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) xxmax = fmaxf(xxmax, __shfl_xor(xxmax, m));
    return xxmax;
}

// The merged (value, index) top-k list of each lane lives in wave-private LDS,
// touched only at epoch ends and once per item: slot (nb, e) of a lane is
// glist[(nb * 8 + e) * 64], values for e < 4 and indices for e >= 4.
template <int NB>
__device__ __forceinline__ void glist_init(unsigned* glist) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            glist[(nb * 8 + e) * 64] = __float_as_uint(kInvalid);
            glist[(nb * 8 + 4 + e) * 64] = 0xFFFFFFFFu;
        }
}

// Fold the epoch's packed keys into the merged lists and reset them.  A key's
// low 8 bits are (16-block within the epoch) * 4 + r; ebase is the global index
// of the epoch's first centroid plus 4g, kend one past the token's last centroid.
// Padding columns past kend carry huge screen values and never enter the merged
// list; the index check also holds when non-finite operands made them small.
template <int NB, int LK, class Key>
__device__ __forceinline__ void epoch_flush(Key (&el)[NB][4], unsigned* glist, int64_t ebase, int64_t kend) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        float G[4];
        int I[4];
#pragma unroll
        for (int e = 0; e < LK; ++e) {
            G[e] = __uint_as_float(glist[(nb * 8 + e) * 64]);
            I[e] = (int)glist[(nb * 8 + 4 + e) * 64];
        }
#pragma unroll
        for (int e = 0; e < LK; ++e) {
            const unsigned bits = key_bits(el[nb][e]);
            const float t = __uint_as_float(bits & ~0xFFu);
            const unsigned loc = bits & 0xFFu;
            const int gi = (int)(ebase + (int64_t)(loc >> 2) * 16 + (loc & 3u));
            if (t < 1.0e38f && gi < kend) glist_insert<LK>(G, I, t, gi, false);
            el[nb][e] = key_empty<Key>();
        }
#pragma unroll
        for (int e = 0; e < LK; ++e) {
            glist[(nb * 8 + e) * 64] = __float_as_uint(G[e]);
            glist[(nb * 8 + 4 + e) * 64] = (unsigned)I[e];
        }
    }
}

// End of a screened item: every lane takes whole rows.  A row's candidates
// are the entries of its four lane groups' top-LK lists (the lists of lane
// (g, c) hold the best screen values among the columns that lane saw).  The
// lane computes the canonical distance of the best-screened candidate, then of
// every other candidate whose screen lower bound does not exclude it, keeps
// the lexicographic (distance, index) minimum, and certifies it against every
// candidate a list dropped: a dropped value is at least its list's last entry.
// Rows whose certificate fails are queued for exhaustive rescoring.
//
// The screen error bound E covers, per screen value:
// * FP32 accumulation: every product and partial sum rounded, the sum of
//   |terms| at most 2(||c||^2 + beta) + 2 ||x|| ||c|| (with a 10% margin on the
//   norms); gamma_130 for the FP32 screen, gamma_386 for BF16's three products
//   per coordinate, gamma_260 for FP16 (one product, doubled for the unknown
//   summation order inside the matrix core);
// * operand rounding: BF16 hi/lo splits leave at most 3 * 2^-16 |x_i| |c_i| per
//   coordinate (6.2 * 2^-16 ||x|| ||c|| after the -2 factor and margin); FP16
//   rounds y = -2x and c once, and with dy = y - f16(y), dc = c - f16(c) the
//   dot error y.c - f16(y).f16(c) = f16(y).dc + dy.f16(c) + dy.dc is bounded by
//   Cauchy-Schwarz with the measured norms ||dy|| (per row) and max ||dc||.
template <int PREC, int NB, int LK, bool SPLIT = false, bool XREG = PREC != TAC_FP32>
__device__ __forceinline__ void finish_item(const Params& P, int32_t j, int64_t row0, int64_t s1, int64_t klo,
                                            int64_t khi, const unsigned* glist, float beta, float cnmax, float cmax,
                                            int lane, const float* sdx = nullptr, SplitArgs S = {}) {
    const double u = 5.9604644775390625e-8;  // 2^-24
    const double g130 = 130.0 * u / (1.0 - 130.0 * u);
    const double g260 = 260.0 * u / (1.0 - 260.0 * u);
    const double g386 = 386.0 * u / (1.0 - 386.0 * u);
    // FP16: largest ||c - f16(c)|| over the centroids (upper bound of the FP32 sum)
    const double dcm = PREC == TAC_F16 ? sqrt((double)__uint_as_float(P.cstat[2]) * (1.0 + 1e-4)) : 0.0;
    const double bt = (double)beta;
    const double cm = (double)cmax, cn2 = (double)cnmax;
    const unsigned* wlist = glist - lane;  // this wave's list slots: lane L's slot (nb, e) at (nb * 8 + e) * 64 + L
    int nscreen = 0;
    for (int q = lane; q < NB * 16; q += 64) {
        const int nb = q >> 4, c = q & 15;
        const int64_t v = row0 + q;
        if (v >= s1) continue;
        ++nscreen;
        // best screen value and the dropped-value bound over the four lane groups
        float g0 = FLT_MAX, tau = FLT_MAX;
        int i0 = -1;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const unsigned* sl = wlist + nb * 8 * 64 + 16 * g + c;
            const float G0 = __uint_as_float(sl[0]);
            const int I0 = (int)sl[4 * 64];
            // a candidate outside the item's centroids (an empty slot) is no candidate
            if (I0 >= klo && I0 < khi && (G0 < g0 || (G0 == g0 && I0 < i0))) {
                g0 = G0;
                i0 = I0;
            }
            tau = fminf(tau, __uint_as_float(sl[(LK - 1) * 64]));
        }
        const int64_t r = P.rowmap ? (int64_t)P.rowmap[v] : v;
        const float* xr = P.x + r * kDim;
        // XREG: the row in registers, loaded once for all of its candidates (a
        // wave with the SIMD's registers to itself); with two waves per SIMD
        // there is no room for it and each candidate reads the row again
        float4 xv[XREG ? kDim / 4 : 1];
        if constexpr (XREG) {
#pragma unroll
            for (int i = 0; i < kDim / 4; ++i) xv[i] = reinterpret_cast<const float4*>(xr)[i];
        }
        auto dist = [&](int64_t k, float* xx) {
            if constexpr (!XREG)
                return dist32_rows(xr, P.C + k * kDim, xx);
            else
                return dist32_xreg(xv, P.C + k * kDim, xx);
        };
        bool ok = false;
        float bd = INFINITY, xxq = INFINITY;
        int bi = INT32_MAX;
        if (i0 >= 0) {
            float xxc;
            bd = dist((int64_t)i0, &xxc);
            xxq = xxc;
            bi = i0;
            // canonical ||x - c||^2 >= (screen - E - beta + ||x||^2) (1 - g130) for every candidate
            const double xx_hi = (double)xxc * (1.0 + g130);
            const double xx_lo = (double)xxc * (1.0 - g130);
            const double xn = sqrt(xx_hi);
            double E;
            if constexpr (PREC == TAC_FP32) {
                E = 1.1 * (g130 * (2.0 * (cn2 + bt) + 2.0 * xn * cm));
            } else if constexpr (PREC == TAC_BF16) {
                E = 1.1 * (g386 * (2.0 * (cn2 + bt) + 2.2 * xn * cm) + 6.2 * 1.52587890625e-5 * xn * cm);
            } else {
                const double dyn = sqrt((double)sdx[q] * (1.0 + 1e-4));  // ||-2x - f16(-2x)||, upper bound
                const double yn = 2.0 * xn + dyn;                         // ||f16(-2x)||
                E = 1.1 * (g260 * (2.0 * (cn2 + bt) + 2.2 * xn * cm) + yn * dcm + dyn * (cm + dcm) + dyn * dcm);
            }
            E += 1e-30;
            // a non-finite bound (operands beyond the 16-bit range, infinite
            // inputs) proves nothing: the row goes to exhaustive rescoring
            const bool bounded = E < 1e30;
            const double shift = -E - bt + xx_lo;
            for (int g = 0; g < (bounded ? 4 : 0); ++g) {
                const unsigned* sl = wlist + nb * 8 * 64 + 16 * g + c;
#pragma unroll
                for (int e = 0; e < LK; ++e) {
                    const int I = (int)sl[(4 + e) * 64];
                    const double G = (double)__uint_as_float(sl[e * 64]);
                    if (I < klo || I >= khi || I == i0 || (G + shift) * (1.0 - g130) > (double)bd) continue;
                    const float d = dist((int64_t)I, nullptr);
                    if (d < bd || (d == bd && I < bi)) {
                        bd = d;
                        bi = I;
                    }
                }
            }
            ok = bounded && ((double)tau >= 1.0e38 || ((double)tau + shift) * (1.0 - g130) > (double)bd);
        }
        if constexpr (SPLIT) {
            // this chunk's exact minimum joins the row's slot; a failed
            // certificate queues the row once, with this chunk's best as its
            // starting bound
            const int64_t si = P.item_off[4 * (int64_t)P.T + j] - P.item_off[4 * (int64_t)P.T] + (v - P.seg_off[j]);
            if (ok) {
                atomicMin(&S.slot[si], ((unsigned long long)__float_as_uint(bd) << 32) | (unsigned)bi);
            } else if (atomicExch(&S.flag[si], 1) == 0) {
                const int64_t qi = P.seg_off[j] + atomicAdd(&P.fbcnt[j], 1);
                P.fbq[qi] = (int32_t)r;
                P.fbxx[qi] = xxq;
                P.fbslot[qi] =
                    bi < INT32_MAX ? ((unsigned long long)__float_as_uint(bd) << 32) | (unsigned)bi : ~0ull;
                atomicAdd(&P.counters[kCntFallback], 1ull);
            }
        } else if (ok) {
            P.assign[r] = bi;
            P.dist[r] = bd;
        } else {
            const int64_t qi = P.seg_off[j] + atomicAdd(&P.fbcnt[j], 1);
            P.fbq[qi] = (int32_t)r;
            P.fbxx[qi] = xxq;
            P.fbslot[qi] = bi < INT32_MAX ? ((unsigned long long)__float_as_uint(bd) << 32) | (unsigned)bi : ~0ull;
            atomicAdd(&P.counters[kCntFallback], 1ull);
        }
    }
    if constexpr (SPLIT) return;  // the split route's rows are counted once, when their slots are read
    for (int m = 32; m > 0; m >>= 1) nscreen += __shfl_xor(nscreen, m);
    if (lane == 0 && nscreen) {
        atomicAdd(&P.counters[kCntRows], (unsigned long long)nscreen);
        atomicAdd(&P.counters[kCntScreened], (unsigned long long)nscreen);
    }
}

// ---- FP32 screen: 8 waves x 4 column blocks of 16 rows = 512 rows per item ----
// Centroid stages of 64 rows are staged through registers into padded LDS rows.
__device__ __forceinline__ void screen_item_fp32(const Params& P, const ItemDesc& D, unsigned* lds) {
    constexpr int NB = kNB;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int col = lane & 15;
    const int32_t j = D.jc & 0xFFFFFF;
    const int64_t s1 = D.s1;
    const int64_t k0 = D.k0;
    const int kc = D.kc;
    const int64_t row0 = D.row0 + wave * (NB * 16);
    const float cnmax = __uint_as_float(P.cstat[0]) * (1.0f + 1e-5f);
    const float cmax = sqrtf(cnmax) * (1.0f + 1e-6f);

    // LDS: two stages of kStage rows (kRowWords words each) and their norms
    unsigned* stage_rows = lds;                                  // [2][kStage][kRowWords]
    float* stage_cn = reinterpret_cast<float*>(lds + 2 * kStage * kRowWords);  // [2][kStage]

    Frag<TAC_FP32, NB> F;
    const float xxmax = load_x_frags<TAC_FP32, NB>(P, row0, s1, g, col, F);
    // One shift for the whole wave makes every screen value positive:
    // beta >= ||x||^2 + (screen error) for each of its rows, so that
    // beta + ||c||^2 - 2 x.c >= ||x - c||^2 + margin > 0 and packed keys order as floats.
    const float beta = xxmax * (1.0f + 0.00390625f) + 0.00390625f * cnmax + 1e-30f;

    unsigned el[NB][4];
    unsigned* glist = lds + kGlistOffsetWords + (unsigned)wave * (NB * 8 * 64) + lane;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) el[nb][e] = 0xFFFFFFFFu;
    glist_init<NB>(glist);

    const char* csrc = static_cast<const char*>(P.cstage);
    const int nst = (kc + kStage - 1) / kStage;
    // stage loader: 64 rows x 512 B = 2048 float4; each thread moves kStageVec of them
    constexpr int kStageVec = kStage * 32 / kThreads;
    auto load_stage = [&](int st, u4 (&reg)[kStageVec], float& rcn) {
#pragma unroll
        for (int it = 0; it < kStageVec; ++it) {
            const int chunk = it * kThreads + threadIdx.x;
            const int row = chunk >> 5;
            const int c16 = chunk & 31;
            const int kk = st * kStage + row;
            reg[it] = kk < kc ? reinterpret_cast<const u4*>(csrc + (k0 + kk) * 512)[c16] : u4{0u, 0u, 0u, 0u};
        }
        const int kk = st * kStage + (threadIdx.x & 63);
        rcn = kk < kc ? P.cn[k0 + kk] : kInvalid;
    };
    auto store_stage = [&](int buf, const u4 (&reg)[kStageVec], float rcn) {
#pragma unroll
        for (int it = 0; it < kStageVec; ++it) {
            const int chunk = it * kThreads + threadIdx.x;
            const int row = chunk >> 5;
            const int c16 = chunk & 31;
            *reinterpret_cast<u4*>(stage_rows + (buf * kStage + row) * kRowWords + c16 * 4) = reg[it];
        }
        if (threadIdx.x < kStage) stage_cn[buf * kStage + threadIdx.x] = rcn;
    };

    u4 pf[kStageVec];
    float pcn;
    load_stage(0, pf, pcn);
    store_stage(0, pf, pcn);
    __syncthreads();

    int epoch_first = 0;  // first 16-block of the current epoch (segment-relative)
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        if (st + 1 < nst) load_stage(st + 1, pf, pcn);
#pragma unroll 1
        for (int b = 0; b < kStage / 16; ++b) {
            const int blk16 = st * (kStage / 16) + b;  // segment-relative 16-block
            if (blk16 * 16 >= kc) break;
            const unsigned* crow = stage_rows + (buf * kStage + b * 16 + col) * kRowWords;
            const f4 cinit = *reinterpret_cast<const f4*>(stage_cn + buf * kStage + b * 16 + 4 * g);
            f4 acc[NB];
            const f4 cb4 = cinit + beta;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb] = cb4;
            // centroid fragments stream from LDS one k-step group at a time
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const f4 c4 = *reinterpret_cast<const f4*>(crow + 32 * g + 4 * q);
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(c4[e], F.x[nb][4 * q + e], acc[nb], 0, 0, 0);
            }
            const unsigned lb = (unsigned)(blk16 - epoch_first) * 4u;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) list_insert(el[nb], (__float_as_uint(acc[nb][r]) & ~0xFFu) | (lb + r));
            const bool last = (blk16 + 1) * 16 >= kc;
            if (blk16 - epoch_first == kEpochBlocks - 1 || last) {
                epoch_flush<NB, 4, unsigned>(el, glist, k0 + (int64_t)epoch_first * 16 + 4 * g, k0 + kc);
                epoch_first = blk16 + 1;
            }
        }
        if (st + 1 < nst) store_stage(buf ^ 1, pf, pcn);
        __syncthreads();
    }
    finish_item<TAC_FP32, NB, 4>(P, j, row0, s1, k0, k0 + kc, glist, beta, cnmax, cmax, lane);
}

// ---- 16-bit screens: 4 waves (one per SIMD) x 5 column blocks of 16 rows = 320 rows per item ----
// The wave's x operands (16-bit fragments of -2x: hi and lo BF16 splits, or
// one FP16 rounding) stay in AGPRs for the whole item.  Centroid stages of
// 32 KiB (64 centroids of hi/lo BF16 rows, 512 B each, or 128 centroids of
// FP16 rows, 256 B each) go straight from global memory into LDS
// (global_load_lds_dwordx4, no registers), three buffers deep, with the
// 16-byte chunks of row r stored at chunk ^ (r & 15) so that the fragment
// reads of 16 consecutive rows hit distinct banks without padding.  The
// 16-centroid block loop is software pipelined: while the matrix cores run
// block b, the wave reads block b + 1's fragments from LDS and folds block
// b - 1's screen values into its top-3 lists, so the three streams (matrix,
// LDS, vector) overlap.
constexpr int kBThreads = 256;
constexpr int kBWaves = kBThreads / 64;
// column blocks (16 rows each) per wave: the item's row tile is 64 * NB rows.
// Each NB in [kBNBMin, kBNB] is compiled; the launch takes the context's
// tuning (tile_blocks), which the autotuner chooses by measurement.
constexpr int kBNB = 5;
constexpr int kBNBMin = 3;
// Per-lane list length of the 16-bit screens.  For BF16 a top-3 costs one med3
// less per screen value than a top-4 and its certificate rarely fails either
// way; the FP16 screen's wider error bound makes a top-3 fail about five times
// as often as a top-4, and the rescoring of those rows costs more than the
// extra med3.
template <int PREC>
constexpr int kBLK = PREC == TAC_F16 ? 4 : 3;
constexpr int kBBufs = 3;                                 // stage buffers
constexpr int kBCnStride = 128;                           // norms per stage buffer (room for FP16's 128)
// after the tiles: the persistent loop's work-item slots (two descriptors, two indices)
constexpr size_t kSlotBytes = 80;

// LDS layout of a 16-bit screen work-group when OCC of them share a CU (one or
// two waves per SIMD), in words: the norms of the three stage buffers, the
// stage buffers, the waves' merged lists (room for kMaxNB column blocks), then
// the FP16 screen's per-row rounding norms.  One work-group per CU stages
// 32 KiB at a time and holds column blocks up to kBNB; two per CU stage 16 KiB
// and hold three column blocks, so that both fit in the 160 KiB of LDS and in
// half of the SIMD's registers each.
template <int OCC>
struct BLayout {
    static constexpr int kStageWords = OCC == 1 ? 8192 : 4096;
    static constexpr int kMaxNB = OCC == 1 ? kBNB : kBNBMin;
    static constexpr size_t kCn = 0;
    static constexpr size_t kStage = (size_t)kBBufs * kBCnStride;
    static constexpr size_t kGlist = kStage + (size_t)kBBufs * kStageWords;
    static constexpr size_t kDx = kGlist + (size_t)kBWaves * kMaxNB * 8 * 64;
    static constexpr size_t kBytes = (kDx + (size_t)kBWaves * kMaxNB * 16) * 4;
    // vector-memory instructions each wave issues per stage: its 1 KiB row
    // transfers and one transfer of norms
    static constexpr int kStageOps = kStageWords / 256 / kBWaves + 1;
    static_assert(kStageWords / 256 % kBWaves == 0, "transfers split evenly over the waves");
    static_assert(OCC * (kBytes + kSlotBytes) <= 160 * 1024, "fits the LDS of a CU");
};

// Stage geometry of a 16-bit screen: bytes per centroid row and centroids per stage.
template <int PREC, int OCC>
struct StageGeom {
    static constexpr int kRowBytes = PREC == TAC_BF16 ? 512 : 256;
    static constexpr int kCents = BLayout<OCC>::kStageWords * 4 / kRowBytes;  // 64 / 128, or 32 / 64
    static constexpr int kBlocks = kCents / 16;                                // 16-centroid blocks per stage
};

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// Issue the DMA of stage `st` (centroids st*S .. st*S+S-1 of the token) into
// `buf` and its norms into `bcn`: the rows as wave-wide transfers of 1 KiB
// (two BF16 or four FP16 rows), an equal share per wave, and the norms as one
// 4-byte transfer per wave (S / 4 lanes each), so that every wave issues
// exactly kStageOps vector-memory instructions per stage.  Lane l moves 16
// bytes of row (1 KiB group) * rows + l / chunks into physical chunk l % chunks.
// Rows past the token's last centroid repeat it, and their norms come from
// g_invalid_norm, which makes their screen values huge.
__device__ const float g_invalid_norm = kInvalid;
template <int PREC, int OCC>
__device__ __forceinline__ void bf_stage_issue(const char* __restrict__ chl, const float* __restrict__ cn, int64_t k0,
                                               int kc, int st, unsigned* buf, float* bcn, int wave, int lane) {
    constexpr int RB = StageGeom<PREC, OCC>::kRowBytes;
    constexpr int SC = StageGeom<PREC, OCC>::kCents;
    constexpr int RPI = 1024 / RB;  // rows per transfer
    constexpr int CPR = RB / 16;    // chunks per row
    constexpr int PER = BLayout<OCC>::kStageWords / 256 / kBWaves;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int grp = wave * PER + i;
        const int row = RPI * grp + lane / CPR;
        int kk = st * SC + row;
        kk = kk < kc ? kk : kc - 1;
        const int chunk = (lane % CPR) ^ (row & 15);
        const char* src = chl + (k0 + kk) * RB + chunk * 16;
        __builtin_amdgcn_global_load_lds(src, (lds_void_ptr)(buf + grp * 256), 16, 0, 0);
    }
    constexpr int NPW = SC / kBWaves;  // norms per wave
    if (lane < NPW) {
        const int kk = st * SC + wave * NPW + lane;
        const float* src = kk < kc ? cn + k0 + kk : &g_invalid_norm;
        __builtin_amdgcn_global_load_lds(src, (lds_void_ptr)(bcn + wave * NPW), 4, 0, 0);
    }
}

// Workgroup barrier without a memory fence: the stage pipeline waits for its
// own transfers with counted vmcnt waits, which a fenced barrier would turn
// into waits for every transfer in flight.  The empty asm statements keep the
// compiler from moving memory accesses across it.
__device__ __forceinline__ void bare_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One 16-centroid block's operands in registers: the fragments for the four
// k-steps (hi and lo for BF16) and the accumulator start (norms + beta) of the
// lane's four columns.
template <int PREC>
struct BBlock;
template <>
struct BBlock<TAC_BF16> {
    bf8 ch[4];
    bf8 cl[4];
    f4 cb;
};
template <>
struct BBlock<TAC_F16> {
    h8 ch[4];
    f4 cb;
};

template <int PREC, int NB, int OCC, bool SPLIT = false>
__device__ __forceinline__ void screen_item_mx(const Params& P, const ItemDesc& D, unsigned* lds, SplitArgs S = {}) {
    using LY = BLayout<OCC>;
    static_assert(NB >= kBNBMin && NB <= LY::kMaxNB, "a compiled tile");
    constexpr int SW = LY::kStageWords;
    constexpr int SC = StageGeom<PREC, OCC>::kCents;
    constexpr int BPS = StageGeom<PREC, OCC>::kBlocks;
    constexpr int RW = StageGeom<PREC, OCC>::kRowBytes / 4;  // words per staged row
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int col = lane & 15;
    // the item's fields are the same on every lane: held as scalars
    auto uni64 = [](int64_t v) {
        const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(uint64_t)v);
        const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)v >> 32));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    const int32_t j = __builtin_amdgcn_readfirstlane(D.jc & 0xFFFFFF);
    const int64_t s1 = uni64(D.s1);
    const int64_t k0 = uni64(D.k0);
    const int kc = __builtin_amdgcn_readfirstlane(D.kc);
    const int64_t row0 = uni64(D.row0) + wave * (NB * 16);
    const float cnmax = __uint_as_float(P.cstat[0]) * (1.0f + 1e-5f);
    const float cmax = sqrtf(cnmax) * (1.0f + 1e-6f);

    unsigned* stage = lds + LY::kStage;                                  // [3][SW]
    float* stage_cn = reinterpret_cast<float*>(lds + LY::kCn);           // [3][kBCnStride]
    unsigned* glist = lds + LY::kGlist + (unsigned)wave * (NB * 8 * 64) + lane;
    float* sdx = reinterpret_cast<float*>(lds + LY::kDx) + wave * (NB * 16);
    const char* chl = static_cast<const char*>(P.cstage);
    const int nst = (kc + SC - 1) / SC;
    const int nblk = (kc + 15) / 16;

    // stage 0 first, so that its latency overlaps the x prologue
    bf_stage_issue<PREC, OCC>(chl, P.cn, k0, kc, 0, stage, stage_cn, wave, lane);

    Frag<PREC, NB> F;
    // the x transpose areas start at stage buffer 1: buffers 1 and 2 (whose DMAs
    // start after the prologue) and, with 16 KiB stages, the merged lists (set
    // up after it) hold them
    float* xt = reinterpret_cast<float*>(stage + SW) + wave * (16 * kXtStride);
    static_assert(LY::kStage + SW + kBWaves * 16 * kXtStride <= LY::kDx, "transpose areas end before the row norms");
    // one wave per SIMD: the x operands in AGPRs; two: in VGPRs, since the
    // compiler splits a half register file evenly between the two kinds
    const float xxmax = load_x_frags<PREC, NB, OCC == 1 ? NB : 1, OCC == 1>(P, row0, s1, g, col, F, sdx, xt);
    // One shift for the whole wave makes every screen value positive (see the FP32 screen).
    const float beta = xxmax * (1.0f + 0.00390625f) + 0.00390625f * cnmax + 1e-30f;
    float el[NB][4];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) el[nb][e] = FLT_MAX;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    // the merged lists only now: with 16 KiB stages the last waves' transpose
    // areas reach into the first waves' lists, so every prologue must be done
    glist_init<NB>(glist);
    // stages 1 and 2 in flight: the pipeline keeps two stages ahead of the one being read
    if (nst > 1) bf_stage_issue<PREC, OCC>(chl, P.cn, k0, kc, 1, stage + SW, stage_cn + kBCnStride, wave, lane);
    if (nst > 2) bf_stage_issue<PREC, OCC>(chl, P.cn, k0, kc, 2, stage + 2 * SW, stage_cn + 2 * kBCnStride, wave, lane);

    int epoch_first = 0;
    auto load_block = [&](int blk, BBlock<PREC>& B) {
        const int buf = (blk / BPS) % kBBufs;
        const int b = blk % BPS;
        const unsigned* srow = stage + buf * SW + (b * 16 + col) * RW;
#pragma unroll
        for (int st4 = 0; st4 < 4; ++st4) {
            if constexpr (PREC == TAC_BF16) {
                B.ch[st4] = *reinterpret_cast<const bf8*>(srow + 4 * ((4 * g + st4) ^ col));
                B.cl[st4] = *reinterpret_cast<const bf8*>(srow + 4 * ((16 + 4 * g + st4) ^ col));
            } else {
                B.ch[st4] = *reinterpret_cast<const h8*>(srow + 4 * ((4 * g + st4) ^ col));
            }
        }
        B.cb = *reinterpret_cast<const f4*>(stage_cn + buf * kBCnStride + b * 16 + 4 * g) + beta;
    };
    // the matrix-core products of one k-step term: BF16 has three (hi.hi, hi.lo, lo.hi), FP16 one
    constexpr int NPR = PREC == TAC_BF16 ? 3 : 1;
    auto mfma1 = [&](const BBlock<PREC>& B, int st4, int pr, int nb, const f4& c) -> f4 {
        if constexpr (PREC == TAC_BF16) {
            const bf8 av = pr == 2 ? B.cl[st4] : B.ch[st4];
            const bf8 bv = pr == 1 ? F.xl[nb][st4] : F.xh[nb][st4];
            return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
        } else {
            return __builtin_amdgcn_mfma_f32_16x16x32_f16(B.ch[st4], F.xh[nb][st4], c, 0, 0, 0);
        }
    };
    auto mfmas = [&](const BBlock<PREC>& B, f4 (&acc)[NB]) {
#pragma unroll
        for (int st4 = 0; st4 < 4; ++st4)
#pragma unroll
            for (int pr = 0; pr < NPR; ++pr)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[nb] = mfma1(B, st4, pr, nb, (st4 == 0 && pr == 0) ? B.cb : acc[nb]);
    };
    // top-k inserts of block blk's screen values; the key's low byte becomes
    // the value's position in the epoch ((block in epoch) * 4 + r)
    auto inserts = [&](int blk, const f4 (&acc)[NB]) {
        const unsigned lb = (unsigned)(blk - epoch_first) * 4u;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                list_insert<kBLK<PREC>>(el[nb], __uint_as_float(__builtin_amdgcn_perm(__float_as_uint(acc[nb][r]), lb + r,
                                                                          0x07060500u)));
    };
    // Steady-state block: the MFMAs of block B interleaved by hand with the
    // top-k inserts of the previous block (one insert after every third BF16
    // MFMA, after every FP16 MFMA); scheduling barriers keep that order, so the
    // vector work fills the matrix pipeline's gaps instead of bunching up.  The
    // inserts visit the NB lists round-robin (value v goes to list v % NB), and
    // each key is packed one group ahead of its insert, so no vector
    // instruction waits on the one issued just before it.
    auto mfmas_inserts = [&](const BBlock<PREC>& B, f4 (&acc)[NB], int pblk, const f4 (&prev)[NB]) {
        const unsigned lb = (unsigned)(pblk - epoch_first) * 4u;
        auto key = [&](int v) {
            return __uint_as_float(
                __builtin_amdgcn_perm(__float_as_uint(prev[v % NB][v / NB]), lb + (unsigned)(v / NB), 0x07060500u));
        };
        float kcur = key(0);
#pragma unroll
        for (int st4 = 0; st4 < 4; ++st4)
#pragma unroll
            for (int pr = 0; pr < NPR; ++pr)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    acc[nb] = mfma1(B, st4, pr, nb, (st4 == 0 && pr == 0) ? B.cb : acc[nb]);
                    const int i = (st4 * NPR + pr) * NB + nb;
                    if (i % NPR == NPR - 1) {
                        const int v = i / NPR;
                        if (v < 4 * NB) {
                            const float knext = v + 1 < 4 * NB ? key(v + 1) : 0.f;
                            list_insert<kBLK<PREC>>(el[v % NB], kcur);
                            kcur = knext;
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
    };
    auto flush_if = [&](int blk) {
        if (blk - epoch_first == kEpochBlocks - 1 || blk + 1 == nblk) {
            epoch_flush<NB, kBLK<PREC>, float>(el, glist, k0 + (int64_t)epoch_first * 16 + 4 * g, k0 + kc);
            epoch_first = blk + 1;
        }
    };
    // Before the last block of stage s (its region reads the first block of
    // stage s + 1's operands): wait until stage s + 1 has landed (each wave
    // waits for its own transfers, counting out stage s + 2's, which stay in
    // flight), make sure no wave still reads stage s's buffer (its last
    // operand reads were issued in the previous region), then start the DMA of
    // stage s + 3 into that buffer.  Two stages of transfers are thus always
    // in flight behind the one being read.
    auto stage_turn = [&](int blk) {
        if (blk % BPS != BPS - 1) return;
        const int sn = blk / BPS + 1;
        if (sn >= nst) return;
        // the count of one stage's transfers: stage s + 2's stay in flight
        if (sn + 1 < nst)
            asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(LY::kStageOps) : "memory");
        else
            asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
        bare_barrier();
        if (sn + 2 < nst)
            bf_stage_issue<PREC, OCC>(chl, P.cn, k0, kc, sn + 2, stage + ((sn + 2) % kBBufs) * SW,
                                      stage_cn + ((sn + 2) % kBBufs) * kBCnStride, wave, lane);
    };

    if constexpr (OCC == 1) {
        // Pipeline over the blocks: region(b) = MFMAs of b, operands of b + 1,
        // inserts of b - 1.  Unrolled by two so that operand and accumulator
        // sets alternate without copies.
        BBlock<PREC> BA, BB;
        f4 accA[NB], accB[NB];
        load_block(0, BA);
        if (nblk == 1) {
            mfmas(BA, accA);
            inserts(0, accA);
            flush_if(0);
        } else {
            load_block(1, BB);
            mfmas(BA, accA);
            for (int blk = 1;; ++blk) {
                // odd block: operands BB -> accB, previous block in accA
                stage_turn(blk);
                if (blk + 1 >= nblk) {
                    mfmas(BB, accB);
                    inserts(blk - 1, accA);
                    flush_if(blk - 1);
                    inserts(blk, accB);
                    flush_if(blk);
                    break;
                }
                load_block(blk + 1, BA);
                mfmas_inserts(BB, accB, blk - 1, accA);
                flush_if(blk - 1);
                ++blk;
                // even block: operands BA -> accA, previous block in accB
                stage_turn(blk);
                if (blk + 1 >= nblk) {
                    mfmas(BA, accA);
                    inserts(blk - 1, accB);
                    flush_if(blk - 1);
                    inserts(blk, accA);
                    flush_if(blk);
                    break;
                }
                load_block(blk + 1, BB);
                mfmas_inserts(BA, accA, blk - 1, accB);
                flush_if(blk - 1);
            }
        }
    } else {
        // Two waves per SIMD leave half the registers.  A block's operands are
        // read one k-step ahead instead of one block ahead; two accumulator
        // sets let the previous block's inserts run between this block's
        // products.  Since a block's
        // operands are read while its own MFMAs run, a stage's buffer is free
        // only once its last block is done: the turn comes before the first
        // block of the next stage (wait for that stage, barrier, then the DMA
        // of the stage after the next one into the buffer just finished).
        struct KOps {
            typename std::conditional<PREC == TAC_BF16, bf8, h8>::type ch;
            typename std::conditional<PREC == TAC_BF16, bf8, h8>::type cl;  // BF16 only
        };
        auto load_k = [&](int blk, int st4, KOps& K) {
            const int buf = (blk / BPS) % kBBufs;
            const unsigned* srow = stage + buf * SW + ((blk % BPS) * 16 + col) * RW;
            const unsigned* hp = srow + 4 * ((4 * g + st4) ^ col);
            if constexpr (PREC == TAC_BF16) {
                // chunk (16 + c) ^ col = 16 + (c ^ col) for c, col < 16: the lo half
                // sits 64 words after the hi half, one address for both
                K.ch = *reinterpret_cast<const bf8*>(hp);
                K.cl = *reinterpret_cast<const bf8*>(hp + 64);
            } else {
                K.ch = *reinterpret_cast<const h8*>(hp);
            }
        };
        auto load_cb = [&](int blk) {
            const int buf = (blk / BPS) % kBBufs;
            return *reinterpret_cast<const f4*>(stage_cn + buf * kBCnStride + (blk % BPS) * 16 + 4 * g) + beta;
        };
        auto turn_before = [&](int blk) {
            if (blk == 0 || blk % BPS != 0) return;
            const int sn = blk / BPS;  // the stage about to be read
            if (sn + 1 < nst)
                asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(LY::kStageOps) : "memory");
            else
                asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
            bare_barrier();
            if (sn + 2 < nst)
                bf_stage_issue<PREC, OCC>(chl, P.cn, k0, kc, sn + 2, stage + ((sn + 2) % kBBufs) * SW,
                                          stage_cn + ((sn + 2) % kBBufs) * kBCnStride, wave, lane);
        };
        KOps KA, KB;
        // The MFMAs of block blk into acc; after the i-th product, between(i).
        auto block_mfmas = [&](int blk, f4 (&acc)[NB], auto&& between) {
            load_k(blk, 0, KA);
            const f4 cb = load_cb(blk);
#pragma unroll
            for (int st4 = 0; st4 < 4; ++st4) {
                KOps& K = st4 % 2 == 0 ? KA : KB;
                KOps& Kn = st4 % 2 == 0 ? KB : KA;
                if (st4 < 3) load_k(blk, st4 + 1, Kn);
                // FP16: the next step's reads stay ahead of this step's products
                // (measured faster; BF16's longer steps measured faster without)
                if constexpr (PREC == TAC_F16) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int pr = 0; pr < NPR; ++pr) {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        if constexpr (PREC == TAC_BF16) {
                            const bf8 av = pr == 2 ? K.cl : K.ch;
                            const bf8 bv = pr == 1 ? F.xl[nb][st4] : F.xh[nb][st4];
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, (st4 == 0 && pr == 0) ? cb : acc[nb],
                                                                             0, 0, 0);
                        } else {
                            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(K.ch, F.xh[nb][st4],
                                                                            st4 == 0 ? cb : acc[nb], 0, 0, 0);
                        }
                        between((st4 * NPR + pr) * NB + nb);
                    }
                }
            }
        };
        // The vector work of block pblk's inserts spread over the next block's
        // products: one insert after every NPR-th product (the matrix core hides
        // about two vector instructions per product issued from the same wave,
        // but none issued from the SIMD's other wave), each key packed one
        // insert ahead so that no vector instruction waits on the one before.
        auto pipelined = [&](int blk, f4 (&acc)[NB], int pblk, const f4 (&prev)[NB]) {
            const unsigned lb = (unsigned)(pblk - epoch_first) * 4u;
            auto key = [&](int v) {
                return __uint_as_float(
                    __builtin_amdgcn_perm(__float_as_uint(prev[v % NB][v / NB]), lb + (unsigned)(v / NB), 0x07060500u));
            };
            float kcur = key(0);
            block_mfmas(blk, acc, [&](int i) {
                if (i % NPR == NPR - 1) {
                    const int v = i / NPR;
                    if (v < 4 * NB) {
                        const float knext = v + 1 < 4 * NB ? key(v + 1) : 0.f;
                        list_insert<kBLK<PREC>>(el[v % NB], kcur);
                        kcur = knext;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            });
        };
        // unrolled by two so that the two accumulator sets alternate without copies
        f4 accA[NB], accB[NB];
        turn_before(0);
        block_mfmas(0, accA, [](int) {});
        for (int blk = 1;; ++blk) {
            if (blk >= nblk) {
                inserts(blk - 1, accA);
                flush_if(blk - 1);
                break;
            }
            turn_before(blk);
            pipelined(blk, accB, blk - 1, accA);
            flush_if(blk - 1);
            ++blk;
            if (blk >= nblk) {
                inserts(blk - 1, accB);
                flush_if(blk - 1);
                break;
            }
            turn_before(blk);
            pipelined(blk, accA, blk - 1, accB);
            flush_if(blk - 1);
        }
    }
    finish_item<PREC, NB, kBLK<PREC>, SPLIT, OCC == 1>(P, j, row0, s1, k0, k0 + kc, glist, beta, cnmax, cmax, lane,
                                                      sdx, S);
}

// OCC: persistent work-groups per CU that the 16-bit screens are compiled for
// (the register budget of a wave is the SIMD's file over OCC).
template <int PREC, int NB = kBNB, int OCC = 1>
__global__ void __launch_bounds__(PREC == TAC_FP32 ? kThreads : kBThreads, OCC) assign_main(Params P) {
    // All shared memory is dynamic so that it starts 16-byte aligned (a static
    // variable in front of it would shift every 16-byte LDS access off alignment).
    extern __shared__ __attribute__((aligned(16))) unsigned lds[];
    // the work-item slots after the kernel's tiles: descriptors of the current
    // and next item (by parity), then the indices of the next two items
    ItemDesc* s_desc = reinterpret_cast<ItemDesc*>(lds + (PREC == TAC_FP32 ? kLdsBytes : BLayout<OCC>::kBytes) / 4);
    long long* s_idx = reinterpret_cast<long long*>(s_desc + 2);
    const int64_t total = P.item_off[3 * (int64_t)P.T];
    if (threadIdx.x == 0) {
        const long long a = (long long)atomicAdd(P.work, 1ull);
        const long long b = (long long)atomicAdd(P.work, 1ull);
        s_idx[0] = a;
        s_idx[1] = b;
        if (a < total) s_desc[0] = P.desc[a];
    }
    __syncthreads();
    for (int par = 0;; par ^= 1) {
        const int64_t item = s_idx[0];
        if (item >= total) break;
        const int64_t nxt = s_idx[1];
        const ItemDesc D = s_desc[par];
        // one item of look-ahead: the item after next is claimed and the next
        // item's descriptor copied into its slot (LDS DMA, no registers held)
        // now, so both latencies overlap this item
        long long nn = 0;
        if (threadIdx.x < 2) {
            if (threadIdx.x == 0) nn = (long long)atomicAdd(P.work, 1ull);
            if (nxt < total)
                __builtin_amdgcn_global_load_lds(reinterpret_cast<const char*>(P.desc + nxt) + 16 * threadIdx.x,
                                                 (lds_void_ptr)(s_desc + (par ^ 1)), 16, 0, 0);
        }
        const int cls = D.jc >> 24;
        if constexpr (PREC != TAC_FP32) {
            if (cls == 2)
                direct_item<kBThreads>(P, D);
            else
                screen_item_mx<PREC, NB, OCC>(P, D, lds);
        } else {
            if (cls == 2)
                direct_item<kThreads>(P, D);
            else
                screen_item_fp32(P, D, lds);
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the descriptor copy has landed
        __syncthreads();  // every thread has read this item's slots
        if (threadIdx.x == 0) {
            s_idx[0] = nxt;
            s_idx[1] = nn;
        }
        __syncthreads();
    }
}

// The split route's work items (items item_off[3T] .. item_off[4T]), one per
// work-group at a time in a grid-stride loop: the same 16-bit screen and
// finish as the persistent kernel, on one row tile and one centroid chunk.
template <int PREC, int NB, int OCC>
__global__ void __launch_bounds__(kBThreads, OCC) assign_split(Params P, SplitArgs S) {
    extern __shared__ __attribute__((aligned(16))) unsigned lds[];
    const int64_t b = P.item_off[3 * (int64_t)P.T], e = P.item_off[4 * (int64_t)P.T];
    for (int64_t t = b + blockIdx.x; t < e; t += gridDim.x) {
        const ItemDesc D = P.desc[t];
        screen_item_mx<PREC, NB, OCC, true>(P, D, lds, S);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();  // every wave is done with this item's LDS
    }
}

// The split route's results: each split token's first item writes the slots
// of all of the token's rows to assign / dist, except rows queued for
// exhaustive rescoring (the fallback writes those), and counts the rows.
__global__ void split_resolve(const int64_t* __restrict__ item_off, const ItemDesc* __restrict__ desc, int32_t T,
                              const int32_t* __restrict__ rowmap, const unsigned long long* __restrict__ slot,
                              const int32_t* __restrict__ flag, int32_t* __restrict__ assign,
                              float* __restrict__ dist, unsigned long long* __restrict__ counters) {
    const int64_t b = item_off[3 * (int64_t)T], e = item_off[4 * (int64_t)T];
    for (int64_t t = b + blockIdx.x; t < e; t += gridDim.x) {
        const ItemDesc D = desc[t];
        const int32_t j = D.jc & 0xFFFFFF;
        if (t != item_off[3 * (int64_t)T + j]) continue;  // not the token's first chunk
        const int n = (int)(D.s1 - D.row0);  // the first item's tile starts at the token's first row
        const int64_t sb = item_off[4 * (int64_t)T + j] - item_off[4 * (int64_t)T];
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int64_t si = sb + q;
            const int64_t v = D.row0 + q;
            const int64_t r = rowmap ? (int64_t)rowmap[v] : v;
            if (!flag[si]) {
                const unsigned long long sv = slot[si];
                assign[r] = (int32_t)(unsigned)sv;
                dist[r] = __uint_as_float((unsigned)(sv >> 32));
            }
        }
        if (threadIdx.x == 0) {
            atomicAdd(&counters[kCntRows], (unsigned long long)n);
            atomicAdd(&counters[kCntScreened], (unsigned long long)n);
        }
    }
}

// Rescoring of the rows whose certificate failed, on the matrix cores.  The
// queue holds each token's failed rows together (see Params), so a work item
// is (token j, batch of kFbRows of its failed rows, chunk c of its
// centroids): the chunk's centroid rows stream once for the whole batch, the
// screen value cn - 2 x.c of every (row, centroid) pair goes to LDS, and each
// row rescores exactly every centroid of the chunk whose screen lower bound
// (screen - E + ||x||^2) (1 - g130) does not exceed the distance in its slot.
// The screen is the split-BF16 one of the assignment (three products per
// coordinate, error bound E as in finish_item); with the FP32 matrix-core
// product instead, the fallback of the 10M-row workload's second Lloyd
// assignment took 4.85 ms (FP16 screen, 110,837 rows) and 0.53 ms (BF16,
// 12,945 rows) against 3.76 and 0.45 ms, with bitwise the same results.  The slot starts
// at the row's best exact candidate from the screen and takes the 64-bit
// atomicMin over chunks: non-negative float bits in the high word order like
// the distances, so it ends at the exact lexicographic (distance, index)
// minimum whatever the order of the work items.  32-row batches and 256-centroid
// chunks (52 KiB of LDS) let three work-groups share a CU; 64 x 128 (71 KiB, two
// per CU) measured 12% slower, 16 x 256 (five per CU) 6% slower.
constexpr int kFbRows = 32;
constexpr int kFbChunk = 256;
constexpr int kFbGroupsPerCu = 3;
constexpr int kFbBStride = kDim + 8;         // LDS row stride (16-bit values) of the x splits
constexpr int kFbSStride = kFbChunk + 16;    // LDS row stride of the screen values

__global__ void fb_zero(int32_t* __restrict__ fbcnt, int32_t T) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < T; j += (int64_t)gridDim.x * blockDim.x)
        fbcnt[j] = 0;
}

// work items per token: (batches of its failed rows) x (chunks of its centroids)
__global__ void fb_plan(const int32_t* __restrict__ fbcnt, const int64_t* __restrict__ cent_off, int32_t T,
                        int64_t* __restrict__ wcnt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= T) return;
    const int64_t c = fbcnt[j];
    const int64_t k = cent_off[j + 1] - cent_off[j];
    wcnt[j] = c > 0 ? ((c + kFbRows - 1) / kFbRows) * ((k + kFbChunk - 1) / kFbChunk) : 0;
}

__device__ __forceinline__ unsigned long long min_u64(unsigned long long a, unsigned long long b) { return a < b ? a : b; }

__global__ void __launch_bounds__(256) fb_screen(const float* __restrict__ x, const int64_t* __restrict__ seg_off,
                                                 const int64_t* __restrict__ cent_off, int32_t T,
                                                 const float* __restrict__ C, const float* __restrict__ cn,
                                                 const unsigned* __restrict__ cstat, const int64_t* __restrict__ woff,
                                                 const int32_t* __restrict__ fbcnt, const int32_t* __restrict__ fbq,
                                                 const float* __restrict__ fbxx,
                                                 unsigned long long* __restrict__ fbslot) {
    // the batch's rows as BF16 hi / lo splits of -2x (the matrix-core operand), and the screen values
    __shared__ __attribute__((aligned(16))) unsigned short xb[2 * kFbRows * kFbBStride];
    __shared__ __attribute__((aligned(16))) float sv[kFbRows * kFbSStride];
    const double u = 5.9604644775390625e-8;  // 2^-24
    const double g130 = 130.0 * u / (1.0 - 130.0 * u);
    const double g386 = 386.0 * u / (1.0 - 386.0 * u);
    const float cnmax = __uint_as_float(cstat[0]) * (1.0f + 1e-5f);
    const double cn2 = (double)cnmax, cm = (double)(sqrtf(cnmax) * (1.0f + 1e-6f));
    const int64_t total = woff[T];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    constexpr int kTpr = 256 / kFbRows;  // row phase: threads per row
    const int rr = threadIdx.x / kTpr, sub = threadIdx.x % kTpr;
    unsigned short* xbh = xb;
    unsigned short* xbl = xb + kFbRows * kFbBStride;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        // token: the last j with woff[j] <= w
        int lo_j = 0, hi_j = T;
        while (hi_j - lo_j > 1) {
            const int mid = (lo_j + hi_j) >> 1;
            if (woff[mid] <= w) lo_j = mid; else hi_j = mid;
        }
        const int j = lo_j;
        const int64_t k0 = cent_off[j];
        const int64_t kc = cent_off[j + 1] - k0;
        const int64_t nch = (kc + kFbChunk - 1) / kFbChunk;
        const int64_t local = w - woff[j];
        const int64_t e0 = (local / nch) * kFbRows;
        const int64_t lo = k0 + (local % nch) * kFbChunk;
        const int n = (int)min((int64_t)kFbChunk, k0 + kc - lo);
        const int nr = (int)min((int64_t)kFbRows, (int64_t)fbcnt[j] - e0);
        const int64_t qb = seg_off[j] + e0;
        __syncthreads();  // the previous work item is done with xb and sv
        for (int e = threadIdx.x; e < kFbRows * (kDim / 8); e += blockDim.x) {
            const int r = e / (kDim / 8), c8 = e % (kDim / 8);
            float v8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (r < nr) {
                const float4* xr = reinterpret_cast<const float4*>(x + (int64_t)fbq[qb + r] * kDim) + 2 * c8;
                const float4 a = xr[0], b = xr[1];
                v8[0] = -2.0f * a.x; v8[1] = -2.0f * a.y; v8[2] = -2.0f * a.z; v8[3] = -2.0f * a.w;
                v8[4] = -2.0f * b.x; v8[5] = -2.0f * b.y; v8[6] = -2.0f * b.z; v8[7] = -2.0f * b.w;
            }
            bf8 hi, lo8;
            split_bf8(v8, hi, lo8);
            *reinterpret_cast<bf8*>(xbh + r * kFbBStride + 8 * c8) = hi;
            *reinterpret_cast<bf8*>(xbl + r * kFbBStride + 8 * c8) = lo8;
        }
        __syncthreads();
        // screen: wave w takes 16-centroid blocks w, w + 4, ...; lane (g, col) holds
        // the BF16 hi / lo splits of the block's centroid row col at coordinates
        // 32 s + 8 g + [0, 8) for the four k-steps s, and runs three products per
        // k-step (hi.hi, hi.lo, lo.hi) against every 16-row block of the batch
        const int nrb = (nr + 15) / 16;
        for (int cb = wave; cb * 16 < n; cb += 4) {
            const int64_t kb = lo + cb * 16;
            const float* cr = C + min(kb + col, lo + n - 1) * kDim + 8 * g;
            bf8 ch[4], cl[4];
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const float4 a = *reinterpret_cast<const float4*>(cr + 32 * st);
                const float4 b = *reinterpret_cast<const float4*>(cr + 32 * st + 4);
                const float v8[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
                split_bf8(v8, ch[st], cl[st]);
            }
            f4 cinit;
#pragma unroll
            for (int r = 0; r < 4; ++r) cinit[r] = cb * 16 + 4 * g + r < n ? cn[kb + 4 * g + r] : 0.f;
            for (int rb = 0; rb < nrb; ++rb) {
                const int xo = (rb * 16 + col) * kFbBStride + 8 * g;
                f4 acc = cinit;
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const bf8 xh = *reinterpret_cast<const bf8*>(xbh + xo + 32 * st);
                    const bf8 xl = *reinterpret_cast<const bf8*>(xbl + xo + 32 * st);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[st], xh, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[st], xl, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cl[st], xh, acc, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int kl = cb * 16 + 4 * g + r;
                    if (kl < n) sv[(rb * 16 + col) * kFbSStride + kl] = acc[r];
                }
            }
        }
        __syncthreads();
        if (rr < nr) {  // whole kTpr-lane groups
            const int64_t qi = qb + rr;
            const unsigned long long s0 = fbslot[qi];
            float bd = s0 == ~0ull ? INFINITY : __uint_as_float((unsigned)(s0 >> 32));
            const double xx = (double)fbxx[qi];
            // the split-BF16 screen's error bound (as in the screen of the item)
            const double xn = sqrt(xx * (1.0 + g130));
            const double E = 1.1 * (g386 * (2.0 * cn2 + 2.2 * xn * cm) + 6.2 * 1.52587890625e-5 * xn * cm) + 1e-30;
            const double shift = -E + xx * (1.0 - g130);
            const float* srow = sv + rr * kFbSStride;
            const float* xrow = x + (int64_t)fbq[qi] * kDim;
            float lbd = INFINITY;
            int lbk = INT32_MAX;
            // A centroid is a candidate when ((double)s + shift) (1 - g130) <= bd.  The
            // same test as one float comparison against that bound on s, rounded up
            // with a margin for the double roundings: its candidates are a superset,
            // and rescoring more of them changes no result.  A NaN screen value stays
            // a candidate, as before.
            const double T0 = (double)bd / (1.0 - g130) - shift;
            const float thr = __double2float_ru(T0 + fabs(T0) * 1e-12 + 1e-30);
            for (int k4 = 4 * sub; k4 < n; k4 += 4 * kTpr) {
                const float4 s4 = *reinterpret_cast<const float4*>(srow + k4);
                const float sk[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = k4 + e;
                    if (k >= n || sk[e] > thr) continue;
                    const float d = dist32_rows(xrow, C + (lo + k) * kDim, nullptr);
                    if (d < lbd || (d == lbd && k < lbk)) {
                        lbd = d;
                        lbk = k;
                    }
                }
            }
            unsigned long long key = lbk < n ? ((unsigned long long)__float_as_uint(lbd) << 32) | (unsigned)(lo + lbk)
                                             : ~0ull;
            for (int m = kTpr / 2; m > 0; m >>= 1) {
                const unsigned lo32 = __shfl_xor((unsigned)(key & 0xFFFFFFFFull), m, kTpr);
                const unsigned hi32 = __shfl_xor((unsigned)(key >> 32), m, kTpr);
                key = min_u64(key, ((unsigned long long)hi32 << 32) | lo32);
            }
            if (sub == 0 && key < s0) atomicMin(&fbslot[qi], key);
        }
    }
}

// the queued rows take their slots' exact minima
__global__ void fb_final(const int64_t* __restrict__ seg_off, int32_t T, const int32_t* __restrict__ fbcnt,
                         const int32_t* __restrict__ fbq, const unsigned long long* __restrict__ fbslot,
                         int32_t* __restrict__ assign, float* __restrict__ dist) {
    for (int64_t j = blockIdx.x; j < T; j += gridDim.x) {
        const int c = fbcnt[j];
        for (int e = threadIdx.x; e < c; e += blockDim.x) {
            const int64_t qi = seg_off[j] + e;
            const unsigned long long key = fbslot[qi];
            const int32_t r = fbq[qi];
            assign[r] = (int32_t)(unsigned)(key & 0xFFFFFFFFull);
            dist[r] = __uint_as_float((unsigned)(key >> 32));
        }
    }
}

constexpr int kRedThreads = 256;
constexpr int kRedItems = 16;

__global__ void __launch_bounds__(kRedThreads) inertia_partial(const float* __restrict__ dist, int64_t n,
                                                               double* __restrict__ part) {
    __shared__ double lds[kRedThreads];
    const int64_t base = (int64_t)blockIdx.x * kRedThreads * kRedItems;
    double s = 0.0;
    for (int i = 0; i < kRedItems; ++i) {
        const int64_t k = base + (int64_t)i * kRedThreads + threadIdx.x;
        if (k < n) s += (double)dist[k];
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

__global__ void __launch_bounds__(kRedThreads) inertia_final(const double* __restrict__ part, int64_t nb,
                                                             double* __restrict__ out) {
    __shared__ double lds[kRedThreads];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += kRedThreads) s += part[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int off = kRedThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) lds[threadIdx.x] += lds[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = lds[0];
}

// serving path: token ids -> sort keys; invalid ids sort last (key T) and are marked unassigned
__global__ void serve_keys(const int32_t* __restrict__ tok, int64_t n, int32_t T, uint32_t* __restrict__ keys,
                           int32_t* __restrict__ assign, float* __restrict__ dist,
                           unsigned long long* __restrict__ counters) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t t = tok[i];
        if (t < 0 || t >= T) {
            keys[i] = (uint32_t)T;
            assign[i] = -1;
            dist[i] = 0.f;
            atomicAdd(&counters[kCntUnassigned], 1ull);
        } else {
            keys[i] = (uint32_t)t;
        }
    }
}

// The grouping of a small serving batch in one work group: the same stable
// order and offsets as serve_keys + the radix sort + serve_offsets, without
// their dozen launches.  Keys (token << 16 | row, rows out of range taking
// token T) are unique, so an ascending bitonic sort in LDS gives the stable
// order; offset t is the number of keys below t (a binary search per token).
constexpr int kSmallGroupThreads = 1024;
constexpr int kSmallGroupRows = 4096;  // N at most this, T + 1 below 2^16
__global__ void __launch_bounds__(kSmallGroupThreads) serve_group_small(const int32_t* __restrict__ tok, int32_t n,
                                                                         int32_t T, int32_t* __restrict__ rowmap,
                                                                         int64_t* __restrict__ seg_off,
                                                                         int32_t* __restrict__ assign,
                                                                         float* __restrict__ dist,
                                                                         unsigned long long* __restrict__ counters) {
    __shared__ uint32_t key[kSmallGroupRows];
    int p2 = 1;
    while (p2 < n) p2 <<= 1;
    unsigned bad = 0;
    for (int i = threadIdx.x; i < p2; i += blockDim.x) {
        uint32_t k = 0xFFFFFFFFu;  // padding sorts last
        if (i < n) {
            const int32_t t = tok[i];
            const bool ok = t >= 0 && t < T;
            if (!ok) {
                assign[i] = -1;
                dist[i] = 0.f;
                ++bad;
            }
            k = ((uint32_t)(ok ? t : T) << 16) | (uint32_t)i;
        }
        key[i] = k;
    }
    if (bad) atomicAdd(&counters[kCntUnassigned], (unsigned long long)bad);
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = threadIdx.x; q < (p2 >> 1); q += blockDim.x) {
                const int lo = 2 * q - (q & (stride - 1));  // pairs (lo, lo + stride)
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint32_t a = key[lo], b = key[hi];
                if ((a > b) == up) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) rowmap[i] = (int32_t)(key[i] & 0xFFFFu);
    for (int t = threadIdx.x; t <= T + 1; t += blockDim.x) {
        int a = 0, b = n;  // the first sorted position whose token is >= t
        while (a < b) {
            const int m = (a + b) >> 1;
            if ((int)(key[m] >> 16) < t) a = m + 1; else b = m;
        }
        seg_off[t] = a;
    }
}

__global__ void serve_offsets(const uint32_t* __restrict__ keys, int64_t n, int32_t T, int64_t* __restrict__ seg_off) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t prev = i == 0 ? -1 : (int64_t)keys[i - 1];
        const int64_t cur = i == n ? (int64_t)T + 1 : (int64_t)keys[i];
        for (int64_t t = prev + 1; t <= cur; ++t) seg_off[t] = i;
    }
}

unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}


// The compiled 16-bit screen kernels of one precision, row tile and
// occupancy, with the dynamic LDS their tiles take.
struct Kernels16 {
    void (*main)(Params);
    void (*split)(Params, SplitArgs);
    size_t lds;  // tile bytes (the persistent kernel adds kSlotBytes)
    int nb;      // column blocks of 16 rows per wave
};
template <int PREC>
Kernels16 kernels16_of(int nb, int occ) {
    static_assert(kBNBMin == 3 && kBNB == 5 && BLayout<2>::kMaxNB == 3, "one case per compiled tile");
    if (occ == 2) return {assign_main<PREC, 3, 2>, assign_split<PREC, 3, 2>, BLayout<2>::kBytes, 3};
    switch (nb) {
        case 3: return {assign_main<PREC, 3, 1>, assign_split<PREC, 3, 1>, BLayout<1>::kBytes, 3};
        case 4: return {assign_main<PREC, 4, 1>, assign_split<PREC, 4, 1>, BLayout<1>::kBytes, 4};
        default: return {assign_main<PREC, 5, 1>, assign_split<PREC, 5, 1>, BLayout<1>::kBytes, 5};
    }
}
Kernels16 kernels16(int precision, int nb, int occ) {
    return precision == TAC_BF16 ? kernels16_of<TAC_BF16>(nb, occ) : kernels16_of<TAC_F16>(nb, occ);
}
// The 16-bit screen variant a context's tuning selects: two work-groups per CU
// (three column blocks) for waves_per_simd 2, and by default unless
// tile_blocks asks for a tile only one work-group per CU holds (4 or 5);
// otherwise one work-group per CU with tile_blocks column blocks (default 5).
int occupancy_of(const tac_tuning& t) {
    if (t.waves_per_simd == 1 || t.waves_per_simd == 2) return t.waves_per_simd;
    return t.tile_blocks == 4 || t.tile_blocks == 5 ? 1 : 2;
}
Kernels16 kernels16_for(const tac_tuning& t, int precision) {
    const int occ = occupancy_of(t);
    const int nb = occ == 2 ? 3 : t.tile_blocks >= kBNBMin && t.tile_blocks <= kBNB ? t.tile_blocks : kBNB;
    return kernels16(precision, nb, occ);
}

}  // namespace

}  // namespace tac

using namespace tac;

namespace {
// Layout of a prepared-centroid buffer: the bounds (4 words), the norms (K + 1
// floats), then the 16-bit staging rows, each part 256-byte aligned.
struct StaticLayout {
    size_t cn, chl, bytes;
    StaticLayout(int64_t K, int32_t precision) {
        cn = 256;
        chl = cn + (((size_t)(K + 1) * sizeof(float) + 255) / 256) * 256;
        const size_t rows = precision == TAC_FP32 ? 0 : (size_t)(K + 1) * (precision == TAC_BF16 ? 2 : 1) * kDim;
        bytes = chl + rows * sizeof(unsigned short);
    }
};
}  // namespace

extern "C" tac_status tac_ctx_set_static_centroids(tac_ctx ctx, const float* C_d, int64_t K, int32_t precision) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_ctx_set_static_centroids: ctx is NULL");
    if (C_d && (K < 1 || K > INT32_MAX))
        return set_error(TAC_E_INVAL, "tac_ctx_set_static_centroids: K out of range");
    if (C_d && precision != TAC_FP32 && precision != TAC_BF16 && precision != TAC_F16)
        return set_error(TAC_E_INVAL, "tac_ctx_set_static_centroids: bad precision");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TAC_HIP(hipStreamIsCapturing(ctx->stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return set_error(TAC_E_INVAL, "tac_ctx_set_static_centroids: not allowed during stream capture");
    if (ctx->sc_buf) {
        // retired, not freed: a graph captured on this context may still address
        // it; it keeps counting against the context's limit
        ctx->ws_retired.push_back(ctx->sc_buf);
        ctx->ws_retired_bytes += ctx->sc_bytes;
        ctx->sc_buf = nullptr;
        ctx->sc_bytes = 0;
    }
    ctx->sc_C = nullptr;
    ctx->sc_K = 0;
    ctx->sc_prec = -1;
    if (!C_d) return TAC_OK;
    const StaticLayout L(K, precision);
    const size_t held = ctx->ws_retired_bytes + ctx->ws_cap;
    if (ctx->max_ws && held + L.bytes > ctx->max_ws)
        return set_error(TAC_E_NOMEM, "prepared centroids of " + std::to_string(L.bytes) + " bytes (with " +
                                          std::to_string(held) + " bytes already held) exceed the context limit of " +
                                          std::to_string(ctx->max_ws));
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, L.bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(TAC_E_NOMEM, "hipMalloc of " + std::to_string(L.bytes) + " prepared-centroid bytes failed");
    }
    // from here on every failure frees the new buffer before returning
    auto fail = [&](hipError_t err, const char* what) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(p);
        return hip_error(err, what);
    };
    char* base = static_cast<char*>(p);
    unsigned* cstat = reinterpret_cast<unsigned*>(base);
    e = hipMemsetAsync(cstat, 0, 4 * sizeof(unsigned), ctx->stream);
    if (e != hipSuccess) return fail(e, "hipMemsetAsync(prepared bounds)");
    const unsigned pgrid = std::min<unsigned>(grid_for(K * 32, 256), (unsigned)ctx->props_cu * 16);
    prep_centroids<<<pgrid, 256, 0, ctx->stream>>>(
        C_d, K, reinterpret_cast<float*>(base + L.cn), cstat,
        precision == TAC_FP32 ? nullptr : reinterpret_cast<unsigned short*>(base + L.chl), precision);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(e, "prep_centroids");
    // synchronous: later calls may run on another stream of the context
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(e, "hipStreamSynchronize(prepared centroids)");
    ctx->sc_buf = p;
    ctx->sc_bytes = L.bytes;
    ctx->sc_C = C_d;
    ctx->sc_K = K;
    ctx->sc_prec = precision;
    return TAC_OK;
}

namespace {

// Where each part of tac_assign's workspace sits (byte offsets from its base),
// and the bytes it needs; the same plan serves the context's arena and the
// no-allocation entry point's static scratch.
struct AssignPlan {
    bool serve = false, mx16 = false, prepared = false;
    int64_t ncls = 0, nsplit_rows = 0, nred = 0;
    size_t o_cnt = 0, o_scan = 0, o_table = 0, o_work = 0, o_cstat = 0, o_cn = 0, o_chl = 0;
    size_t o_fbq = 0, o_fbxx = 0, o_slot = 0, o_fbcnt = 0, o_sslot = 0, o_sflag = 0, o_dist = 0, o_red = 0;
    size_t o_k0 = 0, o_v0 = 0, o_k1 = 0, o_v1 = 0, o_sort = 0, o_seg = 0;
    size_t bytes = 0;
};

tac_status assign_check(tac_ctx ctx, const char* fn, const float* x_d, const int64_t* seg_off_d,
                        const int32_t* tok_d, int64_t N, int32_t d, int32_t T, const float* C_d,
                        const int64_t* cent_off_d, int64_t K, int32_t precision, const int32_t* assign_d) {
    const std::string f = fn;
    if (!ctx) return set_error(TAC_E_INVAL, f + ": ctx is NULL");
    if (d != kDim) return set_error(TAC_E_INVAL, f + ": d must be 128");
    if (N < 0 || N > INT32_MAX) return set_error(TAC_E_INVAL, f + ": N out of range");
    if (T < 1 || T > (1 << 24)) return set_error(TAC_E_INVAL, f + ": T must be in [1, 2^24]");
    if (K < 0 || K > INT32_MAX) return set_error(TAC_E_INVAL, f + ": K out of range");
    if ((seg_off_d == nullptr) == (tok_d == nullptr))
        return set_error(TAC_E_INVAL, f + ": pass exactly one of seg_off_d and tok_d");
    if (precision != TAC_FP32 && precision != TAC_BF16 && precision != TAC_F16)
        return set_error(TAC_E_INVAL, f + ": bad precision");
    if (!cent_off_d || (N > 0 && (!x_d || !assign_d)) || (K > 0 && !C_d))
        return set_error(TAC_E_INVAL, f + ": NULL pointer");
    return TAC_OK;
}

AssignPlan assign_plan(tac_ctx ctx, const int32_t* tok_d, int64_t N, int32_t T, const float* C_d, int64_t K,
                       int32_t precision, const float* dist_d) {
    AssignPlan p;
    p.serve = tok_d != nullptr;
    p.ncls = 4 * (int64_t)T;  // item counts of the four classes; the split rows follow
    p.mx16 = precision != TAC_FP32;
    // centroids declared unchanging for exactly this call's (C, K, precision): prepared once
    p.prepared = ctx->sc_buf && ctx->sc_C == C_d && ctx->sc_K == K && ctx->sc_prec == precision;
    Carve cv;
    p.o_cnt = cv.take<int64_t>(p.ncls + T + 1);
    p.o_scan = cv.take<char>(scan_scratch_bytes(p.ncls + T));
    // items: at most one partial tile per token, plus the split route's (tile, chunk) items
    constexpr int64_t kMinTileRows = kBWaves * kBNBMin * 16;
    constexpr int64_t kSplitTiles = (kSplitMaxRows + kMinTileRows - 1) / kMinTileRows;
    p.o_table = cv.take<ItemDesc>(N / 256 + (int64_t)T + kSplitTiles * (K / kSplitChunk + K / kSplitMinKappa) + 1);
    p.o_work = cv.take<unsigned long long>(1);
    p.o_cstat = cv.take<unsigned>(4);
    p.o_cn = p.prepared ? 0 : cv.take<float>(K + 1);
    p.o_chl = p.mx16 && !p.prepared ? cv.take<unsigned short>((K + 1) * (precision == TAC_BF16 ? 2 : 1) * kDim) : 0;
    p.o_fbq = cv.take<int32_t>(N + 1);
    p.o_fbxx = cv.take<float>(N + 1);
    p.o_slot = cv.take<unsigned long long>(N + 1);
    p.o_fbcnt = cv.take<int32_t>((int64_t)T + 1);
    // split-route row slots: each split token has at most kSplitMaxRows rows and kSplitMinKappa centroids
    p.nsplit_rows = p.mx16 ? std::min<int64_t>(N, (K / kSplitMinKappa) * kSplitMaxRows) : 0;
    p.o_sslot = cv.take<unsigned long long>(p.nsplit_rows + 1);
    p.o_sflag = cv.take<int32_t>(p.nsplit_rows + 1);
    p.o_dist = dist_d ? 0 : cv.take<float>(N + 1);
    p.nred = (N + kRedThreads * kRedItems - 1) / (kRedThreads * kRedItems);
    p.o_red = cv.take<double>(p.nred + 1);
    if (p.serve) {
        p.o_k0 = cv.take<uint32_t>(N + 1);
        p.o_v0 = cv.take<int32_t>(N + 1);
        p.o_k1 = cv.take<uint32_t>(N + 1);
        p.o_v1 = cv.take<int32_t>(N + 1);
        p.o_sort = cv.take<char>(radix_sort_scratch_bytes(N));
        p.o_seg = cv.take<int64_t>((int64_t)T + 2);
    }
    p.bytes = cv.off;
    return p;
}

template <class T>
T* at(char* base, size_t off) {
    return reinterpret_cast<T*>(base + off);
}

// Everything tac_assign enqueues, with its workspace at `ws` (laid out by `pl`).
// Every part of the workspace that a kernel reads is written earlier in the
// same call, so the workspace may hold anything on entry.
tac_status assign_run(tac_ctx ctx, char* ws, const AssignPlan& pl, const float* x_d, const int64_t* seg_off_d,
                      const int32_t* tok_d, int64_t N, int32_t T, const float* C_d, const int64_t* cent_off_d,
                      int64_t K, int32_t precision, int32_t* assign_d, float* dist_d, double* inertia_d) {
    hipStream_t s = ctx->stream;
    const bool serve = pl.serve, mx16 = pl.mx16, prepared = pl.prepared;
    const int64_t ncls = pl.ncls;
    tac_status st = TAC_OK;
    float* dist = dist_d ? dist_d : at<float>(ws, pl.o_dist);
    unsigned* cstat = at<unsigned>(ws, pl.o_cstat);
    float* cn = at<float>(ws, pl.o_cn);
    unsigned short* chl = mx16 ? at<unsigned short>(ws, pl.o_chl) : nullptr;
    const unsigned* cstat_static = nullptr;
    if (prepared) {
        const StaticLayout L(K, precision);
        char* base = static_cast<char*>(ctx->sc_buf);
        cstat_static = reinterpret_cast<const unsigned*>(base);
        cn = reinterpret_cast<float*>(base + L.cn);
        chl = mx16 ? reinterpret_cast<unsigned short*>(base + L.chl) : nullptr;
    }
    int64_t* cnt = at<int64_t>(ws, pl.o_cnt);
    unsigned long long* work = at<unsigned long long>(ws, pl.o_work);

    const int64_t* seg = seg_off_d;
    const int32_t* rowmap = nullptr;
    reset_call<<<1, 1, 0, s>>>(work, ctx->counters, cstat, cstat_static);
    TAC_LAUNCH_CHECK("reset_call");
    if (serve) {
        int64_t* sseg = at<int64_t>(ws, pl.o_seg);
        uint32_t* k0 = at<uint32_t>(ws, pl.o_k0);
        int32_t* v0 = at<int32_t>(ws, pl.o_v0);
        uint32_t* k1 = at<uint32_t>(ws, pl.o_k1);
        int32_t* v1 = at<int32_t>(ws, pl.o_v1);
        if (N <= kSmallGroupRows && (int64_t)T + 1 < 65536) {
            // a small batch: one work group groups it
            serve_group_small<<<1, kSmallGroupThreads, 0, s>>>(tok_d, (int32_t)N, T, v0, sseg, assign_d, dist,
                                                               ctx->counters);
            TAC_LAUNCH_CHECK("serve_group_small");
            seg = sseg;
            rowmap = v0;
        } else {
            if (N > 0) {
                serve_keys<<<grid_for(N, 256), 256, 0, s>>>(tok_d, N, T, k0, assign_d, dist, ctx->counters);
                TAC_LAUNCH_CHECK("serve_keys");
            }
            int bits = 1;
            while (bits < 31 && (int64_t(1) << bits) < (int64_t)T + 1) ++bits;
            int in1 = 0;
            st = radix_sort(s, N, bits, k0, v0, k1, v1, nullptr, at<void>(ws, pl.o_sort), &in1);
            if (st != TAC_OK) return st;
            serve_offsets<<<grid_for(N + 1, 256), 256, 0, s>>>(in1 ? k1 : k0, N, T, sseg);
            TAC_LAUNCH_CHECK("serve_offsets");
            seg = sseg;
            rowmap = in1 ? v1 : v0;
        }
    }
    const int threads = mx16 ? kBThreads : kThreads;
    // the 16-bit screens' kernels and row tile (column blocks of 16 rows per wave)
    const Kernels16 k16 = kernels16_for(ctx->tuning, mx16 ? precision : TAC_BF16);
    const int screen_rows = mx16 ? kBWaves * k16.nb * 16 : kTileRows;
    // dynamic LDS: the kernel's tiles plus the work-item slots
    const size_t lds_bytes = (mx16 ? k16.lds : kLdsBytes) + kSlotBytes;
    plan_count<<<grid_for(T, 256), 256, 0, s>>>(seg, cent_off_d, T, ctx->tuning.direct_max_kappa,
                                                  ctx->tuning.heavy_kappa, mx16 ? kSplitMinKappa : 0,
                                                  screen_rows, threads, cnt, cstat + 1);
    TAC_LAUNCH_CHECK("plan_count");
    st = exclusive_scan_i64(s, cnt, cnt, ncls + T, at<void>(ws, pl.o_scan));
    if (st != TAC_OK) return st;
    ItemDesc* table = at<ItemDesc>(ws, pl.o_table);
    SplitArgs S;
    S.slot = at<unsigned long long>(ws, pl.o_sslot);
    S.flag = at<int32_t>(ws, pl.o_sflag);
    // one thread per item: the grid covers the largest item count a call can have
    plan_fill<<<grid_for(N / 64 + 4 * (int64_t)T, 256), 256, 0, s>>>(cnt, seg, cent_off_d, T, screen_rows, threads,
                                                                      table);
    TAC_LAUNCH_CHECK("plan_fill");
    if (mx16) {
        plan_split_slots<<<std::min<unsigned>(grid_for(T, 1), 1024u), 256, 0, s>>>(cnt, seg, T, S.slot, S.flag);
        TAC_LAUNCH_CHECK("plan_split_slots");
    }
    if (K > 0 && !prepared) {
        // a grid-stride launch of a few blocks per CU keeps the per-block atomicMax on the norm bound cheap
        const unsigned pgrid = std::min<unsigned>(grid_for(K * 32, 256), (unsigned)ctx->props_cu * 16);
        prep_centroids<<<pgrid, 256, 0, s>>>(C_d, K, cn, cstat, chl, precision);
        TAC_LAUNCH_CHECK("prep_centroids");
    }
    Params P;
    P.x = x_d;
    P.rowmap = rowmap;
    P.seg_off = seg;
    P.cent_off = cent_off_d;
    P.T = T;
    P.C = C_d;
    P.cstage = mx16 ? (const void*)chl : (const void*)C_d;
    P.cn = cn;
    P.cstat = cstat;
    P.item_off = cnt;
    P.desc = table;
    P.work = work;
    P.assign = assign_d;
    P.dist = dist;
    P.fbq = at<int32_t>(ws, pl.o_fbq);
    P.fbxx = at<float>(ws, pl.o_fbxx);
    P.fbslot = at<unsigned long long>(ws, pl.o_slot);
    P.fbcnt = at<int32_t>(ws, pl.o_fbcnt);
    fb_zero<<<grid_for(T, 256), 256, 0, s>>>(P.fbcnt, T);
    TAC_LAUNCH_CHECK("fb_zero");
    P.counters = ctx->counters;
    // persistent grid: as many work-group slots as the device holds at once
    // (occupancy per kernel: FP32, then each 16-bit precision's tiles 3-5 at
    // one work-group per CU and tile 3 at two)
    static int occ[1 + 2 * 4] = {0};
    auto occ_slot = [](int prec, int nb, int wps) { return 1 + (prec - TAC_BF16) * 4 + (wps == 2 ? 3 : nb - kBNBMin); };
    if (!occ[0]) {
        TAC_HIP(hipFuncSetAttribute((const void*)assign_main<TAC_FP32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(kLdsBytes + kSlotBytes)));
        TAC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[0], assign_main<TAC_FP32>, kThreads,
                                                             kLdsBytes + kSlotBytes));
        for (int pr = TAC_BF16; pr <= TAC_F16; ++pr)
            for (int v = 0; v < 4; ++v) {
                const int wps = v == 3 ? 2 : 1, nb = v == 3 ? kBNBMin : kBNBMin + v;
                const Kernels16 k = kernels16(pr, nb, wps);
                TAC_HIP(hipFuncSetAttribute((const void*)k.main, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)(k.lds + kSlotBytes)));
                TAC_HIP(hipFuncSetAttribute((const void*)k.split, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)k.lds));
                TAC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ[occ_slot(pr, nb, wps)], k.main, kBThreads,
                                                                     k.lds + kSlotBytes));
            }
        for (int& o : occ) o = o < 1 ? 1 : o;
    }
    const int occ16 = occupancy_of(ctx->tuning);
    int per_cu = mx16 ? occ[occ_slot(precision, k16.nb, occ16)] : occ[0];
    if (ctx->tuning.groups_per_cu > 0 && ctx->tuning.groups_per_cu < per_cu) per_cu = ctx->tuning.groups_per_cu;
    const unsigned grid = (unsigned)ctx->props_cu * (unsigned)per_cu;
    const unsigned sgrid = (unsigned)ctx->props_cu;
    if (mx16) {
        // The split route (no work items outside serving-sized batches: then
        // the launch finds an empty item range and returns) on the context's
        // second stream, beside the persistent kernel: its work groups take the
        // CUs the persistent kernel's tail frees.  The two write disjoint rows
        // (a split token's rows have only split items) and count fallbacks
        // with atomics.
        TAC_HIP(hipEventRecord(ctx->fork_ev, s));
        TAC_HIP(hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
        k16.split<<<sgrid * (unsigned)occ16, kBThreads, k16.lds, ctx->aux>>>(P, S);
        TAC_LAUNCH_CHECK("assign_split");
        TAC_HIP(hipEventRecord(ctx->join_ev, ctx->aux));
    }
    time_start(ctx, TAC_SLOT_ASSIGN);
    if (precision == TAC_FP32) {
        assign_main<TAC_FP32><<<grid, threads, lds_bytes, s>>>(P);
        TAC_LAUNCH_CHECK("assign_main<fp32>");
    } else {
        k16.main<<<grid, threads, lds_bytes, s>>>(P);
        TAC_LAUNCH_CHECK(precision == TAC_BF16 ? "assign_main<bf16>" : "assign_main<f16>");
    }
    time_stop(ctx, TAC_SLOT_ASSIGN);
    if (mx16) {
        TAC_HIP(hipStreamWaitEvent(s, ctx->join_ev, 0));
        split_resolve<<<sgrid, 128, 0, s>>>(cnt, table, T, rowmap, S.slot, S.flag, assign_d, dist, ctx->counters);
        TAC_LAUNCH_CHECK("split_resolve");
    }
    // rows whose certificate failed: per-token work plan (the item plan's
    // buffers are free again), matrix-core rescoring, write-back
    int64_t* woff = cnt;
    fb_plan<<<grid_for(T, 256), 256, 0, s>>>(P.fbcnt, cent_off_d, T, woff);
    TAC_LAUNCH_CHECK("fb_plan");
    st = exclusive_scan_i64(s, woff, woff, T, at<void>(ws, pl.o_scan));
    if (st != TAC_OK) return st;
    fb_screen<<<(unsigned)ctx->props_cu * kFbGroupsPerCu, 256, 0, s>>>(x_d, seg, cent_off_d, T, C_d, cn, cstat, woff, P.fbcnt, P.fbq,
                                                        P.fbxx, P.fbslot);
    TAC_LAUNCH_CHECK("fb_screen");
    fb_final<<<std::min<unsigned>((unsigned)T, (unsigned)ctx->props_cu * 8), 256, 0, s>>>(seg, T, P.fbcnt, P.fbq,
                                                                                        P.fbslot, assign_d, dist);
    TAC_LAUNCH_CHECK("fb_final");
    if (inertia_d) {
        double* part = at<double>(ws, pl.o_red);
        if (pl.nred > 0) {
            inertia_partial<<<(unsigned)pl.nred, kRedThreads, 0, s>>>(dist, N, part);
            TAC_LAUNCH_CHECK("inertia_partial");
        }
        inertia_final<<<1, kRedThreads, 0, s>>>(part, pl.nred, inertia_d);
        TAC_LAUNCH_CHECK("inertia_final");
    }
    return TAC_OK;
}

// ---- the no-allocation entry point's scratch --------------------------------
// One fixed array per device (each device that loads the library holds its own
// copy until the process ends).  Host code never passes the array's name to a
// kernel or a copy: it is a host-side stand-in there, and the device address
// comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

tac_status scratch_ptr(int device, char** out) {
    if (device < 0 || device >= kMaxDevices) return set_error(TAC_E_INVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        TAC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));  // the caller made `device` current
        if (!p) return set_error(TAC_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[device] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[device];
    return TAC_OK;
}

}  // namespace

extern "C" tac_status tac_assign(tac_ctx ctx, const float* x_d, const int64_t* seg_off_d, const int32_t* tok_d,
                                 int64_t N, int32_t d, int32_t T, const float* C_d, const int64_t* cent_off_d,
                                 int64_t K, int32_t precision, int32_t* assign_d, float* dist_d, double* inertia_d) {
    tac_status st = assign_check(ctx, "tac_assign", x_d, seg_off_d, tok_d, N, d, T, C_d, cent_off_d, K, precision,
                                 assign_d);
    if (st != TAC_OK) return st;
    TAC_HIP(hipSetDevice(ctx->device));
    const AssignPlan pl = assign_plan(ctx, tok_d, N, T, C_d, K, precision, dist_d);
    st = ws_reserve(ctx, pl.bytes);
    if (st != TAC_OK) return st;
    return assign_run(ctx, static_cast<char*>(ctx->ws), pl, x_d, seg_off_d, tok_d, N, T, C_d, cent_off_d, K,
                      precision, assign_d, dist_d, inertia_d);
}

extern "C" tac_status tac_assign_noalloc(tac_ctx ctx, const float* x_d, const int64_t* seg_off_d,
                                         const int32_t* tok_d, int64_t N, int32_t d, int32_t T, const float* C_d,
                                         const int64_t* cent_off_d, int64_t K, int32_t precision, int32_t* assign_d,
                                         float* dist_d, double* inertia_d) {
    tac_status st = assign_check(ctx, "tac_assign_noalloc", x_d, seg_off_d, tok_d, N, d, T, C_d, cent_off_d, K,
                                 precision, assign_d);
    if (st != TAC_OK) return st;
    TAC_HIP(hipSetDevice(ctx->device));
    const AssignPlan pl = assign_plan(ctx, tok_d, N, T, C_d, K, precision, dist_d);
    if (pl.bytes > kScratchBytes)
        return set_error(TAC_E_NOMEM, "tac_assign_noalloc: this call needs " + std::to_string(pl.bytes) +
                                          " bytes of scratch, more than the fixed " + std::to_string(kScratchBytes) +
                                          " (fewer rows, fewer tokens, or centroids prepared with "
                                          "tac_ctx_set_static_centroids lower the need)");
    char* base = nullptr;
    st = scratch_ptr(ctx->device, &base);
    if (st != TAC_OK) return st;
    return assign_run(ctx, base, pl, x_d, seg_off_d, tok_d, N, T, C_d, cent_off_d, K, precision, assign_d, dist_d,
                      inertia_d);
}

extern "C" tac_status tac_assign_workspace_bytes(tac_ctx ctx, int64_t N, int32_t T, const float* C_d, int64_t K,
                                                 int32_t precision, int with_tok, int with_dist, size_t* bytes) {
    if (!ctx || !bytes) return set_error(TAC_E_INVAL, "tac_assign_workspace_bytes: NULL argument");
    if (N < 0 || N > INT32_MAX || T < 1 || T > (1 << 24) || K < 0 || K > INT32_MAX)
        return set_error(TAC_E_INVAL, "tac_assign_workspace_bytes: sizes out of range");
    if (precision != TAC_FP32 && precision != TAC_BF16 && precision != TAC_F16)
        return set_error(TAC_E_INVAL, "tac_assign_workspace_bytes: bad precision");
    // the plan only tests the token-id pointer and the dist pointer for NULL
    static const int32_t tok_marker = 0;
    static float dist_marker = 0.f;
    const AssignPlan pl = assign_plan(ctx, with_tok ? &tok_marker : nullptr, N, T, C_d, K, precision,
                                      with_dist ? &dist_marker : nullptr);
    *bytes = pl.bytes;
    return TAC_OK;
}

extern "C" tac_status tac_assign_stats(tac_ctx ctx, tac_assign_counters* out) {
    if (!ctx || !out) return set_error(TAC_E_INVAL, "tac_assign_stats: NULL argument");
    TAC_HIP(hipSetDevice(ctx->device));
    unsigned long long c[4];
    TAC_HIP(hipMemcpyAsync(c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
    TAC_HIP(hipStreamSynchronize(ctx->stream));
    out->rows = (int64_t)c[0];
    out->screened = (int64_t)c[1];
    out->fallback = (int64_t)c[2];
    out->unassigned = (int64_t)c[3];
    return TAC_OK;
}
