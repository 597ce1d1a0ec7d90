// Residual compression with product quantisation (Sect. 2.1, "Residuals
// Compression"; M = 32 subspaces with 8-bit codes in Sect. 3.1).
//
// r = x - c_{a(x)}, rho = ||r||, u = r / rho (u = 0 for rho = 0), then for each
// subspace m (coordinates 4m..4m+3) the code is the argmin over the codebook
// of the canonical FP32 distance, lowest code on ties.  The codebooks
// (M x 256 x 4 floats = 128 KiB) stay resident in LDS while a block encodes
// its rows.  Training runs Lloyd per subspace: encode, stably sort the rows of
// each subspace by code, and average every code's members in float64 in that
// fixed order (codes with no member keep their value).  All subspaces are
// sorted together, keyed by (subspace, code), which keeps that order.
#include <algorithm>
#include <cfloat>

#include "tac_internal.h"

namespace tac {

namespace {

constexpr int kDsub = 4;
constexpr int kMaxCodebookFloats = 32 * 256 * kDsub;
constexpr size_t kMaxCodebookLds = (size_t)32 * 256 * (kDsub + 1) * sizeof(float);  // codes + norms

// Canonical residual of one row: r_i = x_i - c_i, rho = sqrt(sum r_i * r_i), each op rounded.
__device__ __forceinline__ float residual_norm(const float* __restrict__ x, const float* __restrict__ c) {
    const float4* xv = reinterpret_cast<const float4*>(x);
    const float4* cv = reinterpret_cast<const float4*>(c);
    float acc = 0.f;
    for (int i = 0; i < kDim / 4; ++i) {
        const float4 a = xv[i], b = cv[i];
        float t;
        t = __fsub_rn(a.x, b.x); acc = __fadd_rn(acc, __fmul_rn(t, t));
        t = __fsub_rn(a.y, b.y); acc = __fadd_rn(acc, __fmul_rn(t, t));
        t = __fsub_rn(a.z, b.z); acc = __fadd_rn(acc, __fmul_rn(t, t));
        t = __fsub_rn(a.w, b.w); acc = __fadd_rn(acc, __fmul_rn(t, t));
    }
    return sqrtf(acc);  // correctly rounded (HIP default for sqrtf); __fsqrt_rn may map to the native approximation
}

// Canonical 4-d distance: t = u_i - b_i, acc = acc + t * t, each op rounded, no fusion.
__device__ __forceinline__ float dist4(const float4 u, const float4 b) {
    float t = __fsub_rn(u.x, b.x);
    float acc = __fmul_rn(t, t);
    t = __fsub_rn(u.y, b.y);
    acc = __fadd_rn(acc, __fmul_rn(t, t));
    t = __fsub_rn(u.z, b.z);
    acc = __fadd_rn(acc, __fmul_rn(t, t));
    t = __fsub_rn(u.w, b.w);
    return __fadd_rn(acc, __fmul_rn(t, t));
}

__device__ __forceinline__ unsigned med3u(unsigned a, unsigned b, unsigned c) {
    unsigned r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Canonical argmin over the ksub codes (LDS cb / cn = squared norms) of one 4-d
// subvector u, lowest code on ties.  A fused-FMA screen ||b||^2 + beta - 2 u.b,
// shifted by beta >= ||u||^2 + margin so that it is positive, keeps a top-2 of
// keys (screen bits with the code in the low 8 bits: one min and one med3 per
// code); both nominees are rescored with the canonical distance, and a rigorous
// bound on the screen error shows that no other code can win.  If it cannot,
// the lane scans every code with the canonical distance.
__device__ __forceinline__ int code_argmin(const float4 u, const float4* cb, const float* cn, int ksub, float cnmax) {
    const float uu = u.x * u.x + u.y * u.y + u.z * u.z + u.w * u.w;
    const float beta = uu * (1.0f + 0.00390625f) + 0.00390625f * cnmax + 1e-30f;
    const float m0 = -2.0f * u.x, m1 = -2.0f * u.y, m2 = -2.0f * u.z, m3 = -2.0f * u.w;
    unsigned k1 = 0xFFFFFFFFu, k2 = 0xFFFFFFFFu;
#pragma unroll 8
    for (int b = 0; b < ksub; ++b) {
        const float4 v = cb[b];
        float t = cn[b] + beta;
        t = fmaf(m0, v.x, t);
        t = fmaf(m1, v.y, t);
        t = fmaf(m2, v.z, t);
        t = fmaf(m3, v.w, t);
        const unsigned key = (__float_as_uint(t) & ~0xFFu) | (unsigned)b;
        k2 = med3u(k1, k2, key);
        k1 = min(k1, key);
    }
    const int n1 = (int)(k1 & 0xFFu);
    const float d1 = dist4(u, cb[n1]);
    if (ksub == 1) return n1;
    const int n2 = (int)(k2 & 0xFFu);
    const float d2 = dist4(u, cb[n2]);
    const bool second = d2 < d1 || (d2 == d1 && n2 < n1);
    const int win = second ? n2 : n1;
    const float dw = second ? d2 : d1;
    if (ksub == 2) return win;
    // every other code has screen >= tau (its key is >= k2, and truncation only lowers tau)
    const double uc = 5.9604644775390625e-8;  // 2^-24
    const double g6 = 6.0 * uc / (1.0 - 6.0 * uc);
    float ucan = __fmul_rn(u.x, u.x);
    ucan = __fadd_rn(ucan, __fmul_rn(u.y, u.y));
    ucan = __fadd_rn(ucan, __fmul_rn(u.z, u.z));
    ucan = __fadd_rn(ucan, __fmul_rn(u.w, u.w));
    const double tau = (double)__uint_as_float(k2 & ~0xFFu);
    const double un = sqrt((double)ucan * (1.0 + g6));
    const double bt = (double)beta, cm2 = (double)cnmax * (1.0 + 1e-5);
    const double E = 1.1 * g6 * (2.0 * (cm2 + bt) + 2.0 * un * sqrt(cm2)) + 1e-30;
    const double L = (tau - E - bt + (double)ucan * (1.0 - g6)) * (1.0 - g6);
    if (L > (double)dw) return win;
    float best = INFINITY;
    int bi = 0;
    for (int b = 0; b < ksub; ++b) {
        const float d = dist4(u, cb[b]);
        if (d < best) {
            best = d;
            bi = b;
        }
    }
    return bi;
}

// Codebooks (float4 per code) and their squared norms into LDS; returns the max norm^2.
__device__ float load_codebooks_norms(const float* __restrict__ cbg, int M, int ksub, float4* lcb, float* lcn) {
    const int n = M * ksub;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float4 v = reinterpret_cast<const float4*>(cbg)[i];
        lcb[i] = v;
        lcn[i] = v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
    }
    __syncthreads();
    float mx = 0.f;
    for (int i = threadIdx.x & 63; i < n; i += 64) mx = fmaxf(mx, lcn[i]);
    for (int m = 32; m > 0; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
    return mx;
}

__global__ void __launch_bounds__(256) residuals_kernel(const float* __restrict__ x, const int32_t* __restrict__ assign,
                                                        const float* __restrict__ C, int64_t K,
                                                        const int64_t* __restrict__ rows, int64_t n, int normalize,
                                                        float* __restrict__ R, float* __restrict__ rnorm) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = rows ? rows[i] : i;
        const int32_t a = assign[row];
        float4* out = reinterpret_cast<float4*>(R + i * kDim);
        if (a < 0 || a >= K) {
            for (int q = 0; q < kDim / 4; ++q) out[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (rnorm) rnorm[i] = 0.f;
            continue;
        }
        const float* xr = x + row * kDim;
        const float* cr = C + (int64_t)a * kDim;
        const float rho = residual_norm(xr, cr);
        const bool scale = normalize && rho > 0.f;
        for (int q = 0; q < kDim / 4; ++q) {
            const float4 xa = reinterpret_cast<const float4*>(xr)[q];
            const float4 cb = reinterpret_cast<const float4*>(cr)[q];
            float4 r;
            r.x = __fsub_rn(xa.x, cb.x);
            r.y = __fsub_rn(xa.y, cb.y);
            r.z = __fsub_rn(xa.z, cb.z);
            r.w = __fsub_rn(xa.w, cb.w);
            if (scale) {
                r.x = __fdiv_rn(r.x, rho);
                r.y = __fdiv_rn(r.y, rho);
                r.z = __fdiv_rn(r.z, rho);
                r.w = __fdiv_rn(r.w, rho);
            } else if (normalize) {
                r = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            out[q] = r;
        }
        if (rnorm) rnorm[i] = rho;
    }
}

// Fused residual + normalisation + encoding, one row per thread; codebooks and
// their norms resident in LDS (32 x 256 x 16 B + 32 x 256 x 4 B = 160 KiB).
__global__ void __launch_bounds__(512) encode_kernel(const float* __restrict__ x, const int32_t* __restrict__ assign,
                                                     const float* __restrict__ C, int64_t K, int64_t n, int normalize,
                                                     const float* __restrict__ cb, int M, int ksub,
                                                     uint8_t* __restrict__ codes, float* __restrict__ rnorm) {
    extern __shared__ float4 lds4[];
    float4* lcb = lds4;
    float* lcn = reinterpret_cast<float*>(lds4 + M * ksub);
    const float cnmax = load_codebooks_norms(cb, M, ksub, lcb, lcn);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = assign[i];
        uint32_t* out = reinterpret_cast<uint32_t*>(codes + i * M);
        if (a < 0 || a >= K) {
            for (int m = 0; m < M / 4; ++m) out[m] = 0u;
            if (rnorm) rnorm[i] = 0.f;
            continue;
        }
        const float* xr = x + i * kDim;
        const float* cr = C + (int64_t)a * kDim;
        const float rho = residual_norm(xr, cr);
        const bool scale = normalize && rho > 0.f;
        uint32_t word = 0;
        for (int m = 0; m < M; ++m) {
            const float4 xa = reinterpret_cast<const float4*>(xr)[m];
            const float4 cv = reinterpret_cast<const float4*>(cr)[m];
            float4 u;
            u.x = __fsub_rn(xa.x, cv.x);
            u.y = __fsub_rn(xa.y, cv.y);
            u.z = __fsub_rn(xa.z, cv.z);
            u.w = __fsub_rn(xa.w, cv.w);
            if (scale) {
                u.x = __fdiv_rn(u.x, rho);
                u.y = __fdiv_rn(u.y, rho);
                u.z = __fdiv_rn(u.z, rho);
                u.w = __fdiv_rn(u.w, rho);
            } else if (normalize) {
                u = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            const unsigned c = (unsigned)code_argmin(u, lcb + m * ksub, lcn + m * ksub, ksub, cnmax);
            word |= c << (8 * (m & 3));
            if ((m & 3) == 3) {
                out[m >> 2] = word;
                word = 0;
            }
        }
        if (rnorm) rnorm[i] = rho;
    }
}

// Codes of training rows R (already normalised residuals), one row per thread.
__global__ void __launch_bounds__(512) train_encode(const float* __restrict__ R, int64_t n,
                                                    const float* __restrict__ cb, int M, int ksub,
                                                    uint32_t* __restrict__ codes /* [M][n] */) {
    extern __shared__ float4 lds4[];
    float4* lcb = lds4;
    float* lcn = reinterpret_cast<float*>(lds4 + M * ksub);
    const float cnmax = load_codebooks_norms(cb, M, ksub, lcb, lcn);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int m = 0; m < M; ++m) {
            const float4 u = reinterpret_cast<const float4*>(R + i * kDim)[m];
            codes[(int64_t)m * n + i] = (uint32_t)code_argmin(u, lcb + m * ksub, lcn + m * ksub, ksub, cnmax);
        }
    }
}

// ---- matrix-core PQ encoding (M = 32 subspaces, ksub a multiple of 16) ----
// For subspace m the screen values ||b||^2 + beta - 2 u.b of 16 codes x 16 rows
// come from one v_mfma_f32_16x16x16_f16.  Its contraction holds three products
// of 16-bit splits: with w = -2u = wh + wl + ew and b = bh + bl + eb (wh, bh
// the FP16 roundings, wl, bl the FP16 roundings of what is left), the
// sixteen terms are bh.wh + bl.wh + bh.wl (+ four zeros), so the screen misses
// only bl.wl, bh.ew, bl.ew and eb.w, a few 2^-22 of ||b|| ||w||.  (On this
// chip the FP32 matrix instruction and vector instructions do not overlap,
// while a 16-bit one hides about two vector instructions issued beside it,
// and costs half the cycles.)  Lane (g, col) supplies k-slice 4g..4g+3: of code
// 16 t + col (bh, bl, bh, bh) and of row col (wh, wh, wl, 0), and receives
// codes 16 t + 4 g + r of row col.  Each lane keeps a top-2 of packed keys over
// its ksub / 4 codes; the four lanes of a row then rescore their first entries
// with the canonical distance, take the lexicographic minimum and certify it
// against every other code, whose screen value is at least the smallest
// second entry of the four lists (so a second entry can never beat a certified
// winner and is not rescored); once all four row blocks of the wave are
// certified, a row that failed screens its codes again and rescores every
// code the bound admits (rows without a finite bound scan every code).  The
// four lanes of a row
// exchange values with the two lane-swap instructions (rows of 16 lanes
// swapped in pairs, halves of the wave swapped), not through LDS.
// Codes are bitwise those of the scalar screen.
// Work split: the 32 subspaces are encoded by two work-groups per block of
// 512 rows (16 subspaces each, 80 KiB of split codebooks and norms in LDS), so
// two work-groups share a CU and hide each other's load latency.  An input of
// few row blocks (a serving batch) is split into eight work-groups of 4
// subspaces per block instead, so that it spreads over more CUs.
constexpr int kEThreads = 512;
constexpr int kENB = 4;
constexpr int kERows = (kEThreads / 64) * kENB * 16;
constexpr int kEHalf = 16;  // subspaces per work-group
static_assert(kENB * 16 == 64, "one prologue row per lane");

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));

// Top-2 (l0 <= l1) of packed keys after two more keys a and b.  The keys are
// bit patterns of positive floats, so unsigned order is value order.  The new
// minimum is min(l0, a, b); the new second is min(l1, med3(l0, a, b)), since
// the second smallest of {l0, l1, a, b} is the smallest of what is left once
// the overall minimum (which lies in {l0, a, b}) is taken out.
__device__ __forceinline__ void top2_insert2(unsigned& l0, unsigned& l1, unsigned a, unsigned b) {
    l1 = min(l1, med3u(l0, a, b));
    l0 = min(min(l0, a), b);
}

// Maximum over each row of 16 lanes of non-negative floats (compared as their
// bit patterns), through DPP lane permutations: swap neighbours, swap pairs,
// mirror each half row, mirror the row.
template <int kCtrl>
__device__ __forceinline__ unsigned dpp_max(unsigned v) {
    return max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_max(float v) {
    unsigned b = __float_as_uint(v);
    b = dpp_max<0xB1>(b);   // quad_perm [1, 0, 3, 2]
    b = dpp_max<0x4E>(b);   // quad_perm [2, 3, 0, 1]
    b = dpp_max<0x141>(b);  // row_half_mirror
    b = dpp_max<0x140>(b);  // row_mirror
    return __uint_as_float(b);
}

// Packed key: the screen value's bits with the low byte replaced by byte r of
// `codes` (four consecutive codes, one per byte).
template <int r>
__device__ __forceinline__ unsigned screen_key(float v, unsigned codes) {
    return __builtin_amdgcn_perm(__float_as_uint(v), codes, 0x07060500u + r);
}

// The four lanes (g, col), g = 0..3, of one row exchange one 32-bit value v:
// afterwards every one of them holds the values of rows g = 0, 1, 2, 3 of the
// wave's 16-lane rows, in that order.  A swap of odd and even 16-lane rows
// gives each lane rows (g & ~1, g | 1); a swap of the wave's halves then
// spreads those over all four rows.
__device__ __forceinline__ void gather4(unsigned v, unsigned (&o)[4]) {
    const u2v p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    const u2v q0 = __builtin_amdgcn_permlane32_swap(p[0], p[0], false, false);
    const u2v q1 = __builtin_amdgcn_permlane32_swap(p[1], p[1], false, false);
    o[0] = q0[0];
    o[1] = q1[0];
    o[2] = q0[1];
    o[3] = q1[1];
}

// The value of lane (g ^ 1, col) and of lane (g ^ 2, col) next to the lane's
// own: the two swaps each return the own value and the partner's, in an order
// that depends on g, which a symmetric combination does not see.
__device__ __forceinline__ u2v pair16(unsigned v) { return __builtin_amdgcn_permlane16_swap(v, v, false, false); }
__device__ __forceinline__ u2v pair32(unsigned v) { return __builtin_amdgcn_permlane32_swap(v, v, false, false); }

// Split FP16 codebook fragments: per code bh = f16(b) and bl = f16(b - bh)
// (8 bytes each, bh first) and ||b||^2 into LDS; returns the largest ||b||^2,
// or +inf when a coordinate lies outside the FP16 range (no screen bound then
// holds and every row is scanned exhaustively).
__device__ float load_split_codebooks(const float* __restrict__ cbg, int M, int ksub, uint2* lfr, float* lcn) {
    const int n = M * ksub;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float4 v = reinterpret_cast<const float4*>(cbg)[i];
        h4 hi, lo;
        hi[0] = (_Float16)v.x;
        hi[1] = (_Float16)v.y;
        hi[2] = (_Float16)v.z;
        hi[3] = (_Float16)v.w;
        lo[0] = (_Float16)(v.x - (float)hi[0]);
        lo[1] = (_Float16)(v.y - (float)hi[1]);
        lo[2] = (_Float16)(v.z - (float)hi[2]);
        lo[3] = (_Float16)(v.w - (float)hi[3]);
        lfr[2 * i] = __builtin_bit_cast(uint2, hi);
        lfr[2 * i + 1] = __builtin_bit_cast(uint2, lo);
        const float nn = v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
        const float am = fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w)));
        lcn[i] = am < 32768.f ? nn : INFINITY;  // fails for NaN too
    }
    __syncthreads();
    float mx = 0.f;
    for (int i = threadIdx.x & 63; i < n; i += 64) mx = fmaxf(mx, lcn[i]);
    for (int m = 32; m > 0; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
    return mx;
}

template <bool RESID, int SUB = kEHalf>
__global__ void __launch_bounds__(kEThreads) __attribute__((amdgpu_waves_per_eu(4))) encode_screen(const float* __restrict__ x,
                                                              const int32_t* __restrict__ assign,
                                                              const float* __restrict__ C, int64_t K, int64_t n,
                                                              int normalize, const float* __restrict__ cbg, int ksub,
                                                              uint8_t* __restrict__ codes_rows,
                                                              uint32_t* __restrict__ codes_sub,
                                                              float* __restrict__ rnorm) {
    constexpr int M = kDim / kDsub;
    static_assert(M % SUB == 0 && SUB % 4 == 0, "whole 4-code words per work-group");
    constexpr int G = M / SUB;  // work-groups per row block
    constexpr unsigned kNoKey = 0x7F7FFFFFu;  // FLT_MAX: an empty list entry
    extern __shared__ uint2 lds2[];
    const int m0 = (int)(blockIdx.x % G) * SUB;
    uint2* lfr = lds2;
    float* lcn = reinterpret_cast<float*>(lds2 + 2 * SUB * ksub);
    const float cnmax = load_split_codebooks(cbg + (size_t)m0 * ksub * kDsub, SUB, ksub, lfr, lcn);
    const float4* cbv4 = reinterpret_cast<const float4*>(cbg);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
    const double uc = 5.9604644775390625e-8;  // 2^-24
    const double g6 = 6.0 * uc / (1.0 - 6.0 * uc);
    const double g44 = 44.0 * uc / (1.0 - 44.0 * uc);
    const double cm2 = (double)cnmax * (1.0 + 1e-5);
    const double scm = sqrt(cm2);
    const int nt = ksub / 16;
    // lane g's fragment of a code: bh for g = 0, 2, 3 (zero rows of w face g = 3), bl for g = 1
    const int fsel = g == 1 ? 1 : 0;
    // bytes of the gathered (wh, wl) pairs that form lane g's k-slice of w: the
    // four wh, the four wl, or zeros
    const unsigned wsel = g < 2 ? 0x05040100u : (g == 2 ? 0x07060302u : 0x0C0C0C0Cu);
    const int64_t nblk = gridDim.x / G;
    for (int64_t base = (int64_t)(blockIdx.x / G) * kERows; base < n; base += nblk * kERows) {
        const int64_t wbase = base + wave * (kENB * 16);
        // lane-per-row prologue: validity, centroid and canonical residual norm
        const int64_t myrow = wbase + lane;
        int a = -1;
        float rho = 0.f;
        int ok_row = 0;
        if (myrow < n) {
            if constexpr (RESID) {
                a = assign[myrow];
                ok_row = a >= 0 && a < K;
                if (ok_row) rho = residual_norm(x + myrow * kDim, C + (int64_t)a * kDim);
                if (rnorm && m0 == 0) rnorm[myrow] = rho;
            } else {
                ok_row = 1;
            }
        }
        // per row block: the centroid row's offset (32-bit; the host keeps K * 128 below 2^32), the norm, validity
        unsigned coff[kENB];
        int vrow[kENB];
        float rrow[kENB];
        uint32_t word[kENB];
#pragma unroll
        for (int nb = 0; nb < kENB; ++nb) {
            const int ar = __shfl(a, nb * 16 + col);
            rrow[nb] = __shfl(rho, nb * 16 + col);
            vrow[nb] = __shfl(ok_row, nb * 16 + col);
            coff[nb] = vrow[nb] && RESID ? (unsigned)ar * (unsigned)kDim + (unsigned)g : 0u;
            word[nb] = 0u;
        }
        // coordinate 4 m + g of every row block, one subspace ahead of its use
        // (addresses from the wave's first row and 32-bit lane offsets, so that
        // no 64-bit address stays live across the subspaces)
        const float* xw = x + wbase * kDim;
        const unsigned xl = (unsigned)(col * kDim + g);
        float xs[kENB] = {}, cs[kENB] = {};
        auto fetch = [&](int m) {
#pragma unroll
            for (int nb = 0; nb < kENB; ++nb) {
                if (vrow[nb]) {
                    xs[nb] = xw[(unsigned)(nb * 16 * kDim + kDsub * m) + xl];
                    if constexpr (RESID) cs[nb] = C[coff[nb] + (unsigned)(kDsub * m)];
                }
            }
        };
        fetch(m0);
        for (int mi = 0; mi < SUB; ++mi) {
            const int m = m0 + mi;
            // coordinate g of the row's subvector u (canonical residual,
            // normalised), the FP16 split of w = -2u as this lane's k-slice of
            // the row (the row's w gathered from its four lanes), and ||u||^2;
            // the whole u is gathered again where the rescoring needs it
            float ug[kENB];
            h4 wk[kENB];
            float sq[kENB], um = 0.f;
            bool wok = true;
#pragma unroll
            for (int nb = 0; nb < kENB; ++nb) {
                float v;
                if constexpr (RESID) {
                    // without branches: a row out of range has xs = cs = 0
                    const float dlt = __fsub_rn(xs[nb], cs[nb]);
                    const float r = rrow[nb];
                    const float q = __fdiv_rn(dlt, r > 0.f ? r : 1.0f);
                    v = normalize ? (r > 0.f ? q : 0.f) : dlt;
                } else {
                    v = xs[nb];
                }
                v = vrow[nb] ? v : 0.f;
                ug[nb] = v;
                const float w = -2.0f * v;
                const _Float16 wh = (_Float16)w;
                const _Float16 wl = (_Float16)(w - (float)wh);
                // |w| within the FP16 range (NaN fails too)
                wok = wok && fabsf(w) < 32768.f;
                unsigned dw[4];
                gather4((unsigned)__builtin_bit_cast(unsigned short, wh) |
                            ((unsigned)__builtin_bit_cast(unsigned short, wl) << 16),
                        dw);
                u2v k2;
                k2[0] = __builtin_amdgcn_perm(dw[1], dw[0], wsel);
                k2[1] = __builtin_amdgcn_perm(dw[3], dw[2], wsel);
                wk[nb] = __builtin_bit_cast(h4, k2);
                // the row's ||u||^2 (the four lanes' squares summed in pairs),
                // within a relative 3 u of the exact value
                const float v2 = __fmul_rn(v, v);
                const u2v s1 = pair16(__float_as_uint(v2));
                const float h = __fadd_rn(__uint_as_float(s1[0]), __uint_as_float(s1[1]));
                const u2v s2 = pair32(__float_as_uint(h));
                const float s = __fadd_rn(__uint_as_float(s2[0]), __uint_as_float(s2[1]));
                sq[nb] = s;
                um = fmaxf(um, s);
            }
            if (mi + 1 < SUB) fetch(m + 1);
            um = row16_max(um);
            // one shift per wave and subspace: beta >= ||u||^2 + (screen error) for each of its rows
            const float beta = um * (1.0f + 0.00390625f) + 0.00390625f * cnmax + 1e-30f;
            unsigned l0[kENB], l1[kENB];
#pragma unroll
            for (int nb = 0; nb < kENB; ++nb) {
                l0[nb] = kNoKey;
                l1[nb] = kNoKey;
            }
            const uint2* frm = lfr + (size_t)mi * ksub * 2 + fsel;
            const float* cnm = lcn + (size_t)mi * ksub;
            // codes 16 t + 4 g + r, r = 0..3, one per byte (at most 255: no carry between bytes)
            unsigned cb4 = (unsigned)(4 * g) * 0x01010101u + 0x03020100u;
            for (int t = 0; t < nt; ++t) {
                const h4 af = __builtin_bit_cast(h4, frm[(16 * t + col) * 2]);
                const f4 ci = *reinterpret_cast<const f4*>(cnm + 16 * t + 4 * g) + beta;
#pragma unroll
                for (int nb = 0; nb < kENB; ++nb) {
                    const f4 acc = __builtin_amdgcn_mfma_f32_16x16x16f16(af, wk[nb], ci, 0, 0, 0);
                    top2_insert2(l0[nb], l1[nb], screen_key<0>(acc[0], cb4), screen_key<1>(acc[1], cb4));
                    top2_insert2(l0[nb], l1[nb], screen_key<2>(acc[2], cb4), screen_key<3>(acc[3], cb4));
                }
                cb4 += 0x10101010u;
            }
            // The first entries' codes, their FP32 codebook rows (from global
            // memory) requested for all row blocks before any is used.
            const float4* cbm = cbv4 + (size_t)m * ksub;
            float4 bv[kENB];
#pragma unroll
            for (int nb = 0; nb < kENB; ++nb) bv[nb] = cbm[min((int)(l0[nb] & 0xFFu), ksub - 1)];
            const double bt = (double)beta;
            // The screen's error bound for a row with ||u|| <= xn is E0 + E1 xn
            // (see the split above): FP32 accumulation of the norm, the shift
            // and sixteen products (doubled for the matrix core's unknown
            // summation order), the dropped split terms, and the FP16
            // roundings' absolute floor, with a 10% margin.
            const double E0 = 1.1 * (g44 * 2.0 * (cm2 + bt) + 1.1920928955078125e-7 * scm) + 1e-12;
            const double E1 = 1.1 * (g44 * 2.02 * 2.0 * scm + 6.1 * 2.384185791015625e-7 * 2.0 * scm +
                                     1.1920928955078125e-7 * 2.02);
            // xn >= sqrt(||u||^2 (1 + g6)): the hardware square root (within an
            // ulp or two; a flushed tiny input only drops a term far below E0's
            // absolute floor) with a relative 2^-19 margin
            auto xnorm = [](float q) { return (double)(__builtin_amdgcn_sqrtf(q) * (1.0f + 1.9073486328125e-6f)); };
            float4 uv[kENB];
#pragma unroll
            for (int nb = 0; nb < kENB; ++nb) {
                unsigned uo[4];
                gather4(__float_as_uint(ug[nb]), uo);
                uv[nb] = make_float4(__uint_as_float(uo[0]), __uint_as_float(uo[1]), __uint_as_float(uo[2]),
                                     __uint_as_float(uo[3]));
            }
            int code[kENB];
            float bdr[kENB];
            unsigned fail = 0u;
            // a w outside the FP16 range anywhere in the wave: no screen bound holds there
            const bool wave_bounded = __ballot(!wok) == 0ull;
#pragma unroll
            for (int nb = 0; nb < kENB; ++nb) {
                const unsigned k0 = l0[nb];
                const int i0 = min((int)(k0 & 0xFFu), ksub - 1);
                const float e0 = dist4(uv[nb], bv[nb]);
                float bd = k0 != kNoKey ? e0 : INFINITY;
                int bi = k0 != kNoKey ? i0 : INT32_MAX;
                float tau = __uint_as_float(l1[nb] & ~0xFFu);
                // lexicographic minimum of (distance, code) and the smallest
                // second entry over the row's four lanes
                {
                    const u2v pd = pair16(__float_as_uint(bd)), pi = pair16((unsigned)bi);
                    const bool t1 = __uint_as_float(pd[1]) < __uint_as_float(pd[0]) ||
                                    (pd[1] == pd[0] && (int)pi[1] < (int)pi[0]);
                    bd = __uint_as_float(t1 ? pd[1] : pd[0]);
                    bi = (int)(t1 ? pi[1] : pi[0]);
                    const u2v pt = pair16(__float_as_uint(tau));
                    tau = fminf(__uint_as_float(pt[0]), __uint_as_float(pt[1]));
                }
                {
                    const u2v pd = pair32(__float_as_uint(bd)), pi = pair32((unsigned)bi);
                    const bool t1 = __uint_as_float(pd[1]) < __uint_as_float(pd[0]) ||
                                    (pd[1] == pd[0] && (int)pi[1] < (int)pi[0]);
                    bd = __uint_as_float(t1 ? pd[1] : pd[0]);
                    bi = (int)(t1 ? pi[1] : pi[0]);
                    const u2v pt = pair32(__float_as_uint(tau));
                    tau = fminf(__uint_as_float(pt[0]), __uint_as_float(pt[1]));
                }
                const double E = E0 + E1 * xnorm(sq[nb]);
                // every code no list kept has screen >= tau; L bounds its canonical distance from below
                const double L = ((double)tau - E - bt + (double)sq[nb] * (1.0 - g6)) * (1.0 - g6);
                code[nb] = bi;
                bdr[nb] = bd;
                const bool bounded = wave_bounded && E < 1e30;
                if (!(bounded && bi != INT32_MAX && L > (double)bd)) fail |= 1u << nb;
            }
            // A failed row (every lane of a row has the same verdict) screens
            // its codes again, bitwise the same values, and rescores every code
            // whose screen value admits a canonical distance within its best so
            // far (the certificate's bound read the other way round); rows with
            // no bound (non-finite or out-of-range operands) scan every code.
            if (__ballot(fail != 0u) != 0ull) {
#pragma unroll
                for (int nb = 0; nb < kENB; ++nb) {
                    if (__ballot((fail >> nb) & 1u) == 0ull) continue;
                    const bool mine = (fail >> nb) & 1u;
                    const double E = E0 + E1 * xnorm(sq[nb]);
                    const bool bounded = wave_bounded && E < 1e30 && bdr[nb] < INFINITY;
                    float best = mine ? bdr[nb] : INFINITY;
                    int bc = mine ? code[nb] : INT32_MAX;
                    if (mine && !bounded) {
                        best = INFINITY;
                        bc = 0;
                        for (int b = 0; b < ksub; ++b) {
                            const float d = dist4(uv[nb], cbm[b]);
                            if (d < best) {
                                best = d;
                                bc = b;
                            }
                        }
                    }
                    // canonical distance <= best requires screen <= thr
                    const float thr = mine && bounded
                                          ? __double2float_ru((double)best / (1.0 - g6) + E + bt -
                                                              (double)sq[nb] * (1.0 - g6))
                                          : -INFINITY;
                    unsigned cb4 = (unsigned)(4 * g) * 0x01010101u + 0x03020100u;
                    for (int t = 0; t < nt; ++t) {
                        const h4 af = __builtin_bit_cast(h4, frm[(16 * t + col) * 2]);
                        const f4 ci = *reinterpret_cast<const f4*>(cnm + 16 * t + 4 * g) + beta;
                        const f4 acc = __builtin_amdgcn_mfma_f32_16x16x16f16(af, wk[nb], ci, 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            if (acc[r] <= thr) {
                                const int k = (int)((cb4 >> (8 * r)) & 0xFFu);
                                const float d = dist4(uv[nb], cbm[k]);
                                if (d < best || (d == best && k < bc)) {
                                    best = d;
                                    bc = k;
                                }
                            }
                        }
                        cb4 += 0x10101010u;
                    }
                    // the row's lexicographic minimum over its four lanes
                    {
                        const u2v pd = pair16(__float_as_uint(best)), pi = pair16((unsigned)bc);
                        const bool t1 = __uint_as_float(pd[1]) < __uint_as_float(pd[0]) ||
                                        (pd[1] == pd[0] && (int)pi[1] < (int)pi[0]);
                        best = __uint_as_float(t1 ? pd[1] : pd[0]);
                        bc = (int)(t1 ? pi[1] : pi[0]);
                    }
                    {
                        const u2v pd = pair32(__float_as_uint(best)), pi = pair32((unsigned)bc);
                        const bool t1 = __uint_as_float(pd[1]) < __uint_as_float(pd[0]) ||
                                        (pd[1] == pd[0] && (int)pi[1] < (int)pi[0]);
                        bc = (int)(t1 ? pi[1] : pi[0]);
                    }
                    if (mine) code[nb] = bc;
                }
            }
#pragma unroll
            for (int nb = 0; nb < kENB; ++nb) {
                const int cv = vrow[nb] ? code[nb] : 0;
                const int64_t row = wbase + nb * 16 + col;
                if constexpr (RESID) {
                    word[nb] |= (uint32_t)cv << (8 * (m & 3));
                    if ((m & 3) == 3) {
                        if (g == 0 && row < n) reinterpret_cast<uint32_t*>(codes_rows + row * M)[m >> 2] = word[nb];
                        word[nb] = 0u;
                    }
                } else {
                    if (g == 0 && row < n) codes_sub[(int64_t)m * n + row] = (uint32_t)cv;
                }
            }
        }
    }
}

bool g_attr_screen[2] = {false, false};

// LDS of one encode_screen work-group: split codebook fragments (16 bytes per
// code) and norms (4 bytes) of its subspaces.
size_t screen_lds(int ksub, int sub = kEHalf) { return (size_t)sub * ksub * (4 * sizeof(uint16_t) * 2 + sizeof(float)); }
bool g_attr_screen4 = false;

// off[t] = first sorted position with key >= t, t in [0, nkeys]
__global__ void code_offsets(const uint32_t* __restrict__ keys, int64_t n, int nkeys, int64_t* __restrict__ off) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t prev = i == 0 ? -1 : (int64_t)keys[i - 1];
        const int64_t cur = i == n ? nkeys : (int64_t)keys[i];
        for (int64_t t = prev + 1; t <= cur; ++t) off[t] = i;
    }
}

// Training keys of subspaces m0 .. m0 + G - 1, in place over their m-major
// codes: entry (m, row) becomes (m - m0) * ksub + code, so that one stable sort
// orders every subspace's rows by code, ascending row within a code.
__global__ void train_keys(uint32_t* __restrict__ codes, int64_t n, int G, int ksub) {
    const int64_t total = (int64_t)G * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        codes[i] += (uint32_t)(i / n) * (uint32_t)ksub;
}

// New code vectors of subspaces m0 .. m0 + G - 1: one wavefront per (subspace,
// code), lanes stride over its members in sorted order (the sorted values are
// positions (m - m0) * n + row), float64 partials combined by a fixed butterfly.
__global__ void __launch_bounds__(256) code_means(const float* __restrict__ R, const int32_t* __restrict__ pos,
                                                  const int64_t* __restrict__ off, int64_t n, int m0, int G,
                                                  int ksub, const float* __restrict__ cb_old,
                                                  float* __restrict__ cb_new) {
    const int lane = threadIdx.x & 63;
    const int w = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (w >= G * ksub) return;
    const int ml = w / ksub, b = w - ml * ksub, m = m0 + ml;
    const int64_t s = off[w], e = off[w + 1];
    const int64_t pbase = (int64_t)ml * n;
    double acc[kDsub] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = s + lane; p < e; p += 64) {
        const float4 v = reinterpret_cast<const float4*>(R + ((int64_t)pos[p] - pbase) * kDim)[m];
        acc[0] += (double)v.x;
        acc[1] += (double)v.y;
        acc[2] += (double)v.z;
        acc[3] += (double)v.w;
    }
    for (int k = 32; k > 0; k >>= 1)
        for (int i = 0; i < kDsub; ++i) acc[i] += __shfl_xor(acc[i], k);
    if (lane == 0) {
        float4* out = reinterpret_cast<float4*>(cb_new) + (int64_t)m * ksub + b;
        const int64_t cnt = e - s;
        if (cnt == 0) {
            *out = reinterpret_cast<const float4*>(cb_old)[(int64_t)m * ksub + b];
        } else {
            float4 r;
            r.x = (float)(acc[0] / (double)cnt);
            r.y = (float)(acc[1] / (double)cnt);
            r.z = (float)(acc[2] / (double)cnt);
            r.w = (float)(acc[3] / (double)cnt);
            *out = r;
        }
    }
}

unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

tac_status check_pq(int32_t d, int32_t M, int32_t ksub, const char* who) {
    if (d != kDim) return set_error(TAC_E_INVAL, std::string(who) + ": d must be 128");
    if (M <= 0 || d % M != 0 || d / M != kDsub)
        return set_error(TAC_E_INVAL, std::string(who) + ": subspaces of 4 coordinates are required (M = 32)");
    if (ksub < 1 || ksub > 256) return set_error(TAC_E_INVAL, std::string(who) + ": ksub must be in [1, 256]");
    return TAC_OK;
}

bool g_attr_encode = false, g_attr_train = false;

}  // namespace

}  // namespace tac

using namespace tac;

extern "C" tac_status tac_residuals(tac_ctx ctx, const float* x_d, const int32_t* assign_d, const float* C_d, int64_t K,
                                    const int64_t* rows_d, int64_t n, int32_t d, int normalize, float* R_d,
                                    float* rnorm_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_residuals: ctx is NULL");
    if (d != kDim) return set_error(TAC_E_INVAL, "tac_residuals: d must be 128");
    if (n < 0 || K < 0) return set_error(TAC_E_INVAL, "tac_residuals: bad sizes");
    if (n == 0) return TAC_OK;
    if (!x_d || !assign_d || !R_d || (K > 0 && !C_d)) return set_error(TAC_E_INVAL, "tac_residuals: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    residuals_kernel<<<grid_for(n, 256), 256, 0, ctx->stream>>>(x_d, assign_d, C_d, K, rows_d, n, normalize, R_d,
                                                                 rnorm_d);
    TAC_LAUNCH_CHECK("residuals_kernel");
    return TAC_OK;
}

extern "C" tac_status pq_encode(tac_ctx ctx, const float* x_d, const int32_t* assign_d, const float* C_d, int64_t K,
                                int64_t n, int32_t d, const float* codebooks_d, int32_t M, int32_t ksub,
                                int normalize, uint8_t* codes_d, float* rnorm_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "pq_encode: ctx is NULL");
    tac_status st = check_pq(d, M, ksub, "pq_encode");
    if (st != TAC_OK) return st;
    if (n < 0 || K < 0) return set_error(TAC_E_INVAL, "pq_encode: bad sizes");
    if (K >= ((int64_t)1 << 32) / kDim) return set_error(TAC_E_INVAL, "pq_encode: K * 128 must stay below 2^32");
    if (n == 0) return TAC_OK;
    if (!x_d || !assign_d || !codebooks_d || !codes_d || (K > 0 && !C_d))
        return set_error(TAC_E_INVAL, "pq_encode: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    const size_t lds = (size_t)M * ksub * (kDsub + 1) * sizeof(float);
    if (!g_attr_encode) {
        TAC_HIP(hipFuncSetAttribute((const void*)encode_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kMaxCodebookLds));
        g_attr_encode = true;
    }
    time_start(ctx, TAC_SLOT_ENCODE);
    if (ksub % 16 == 0) {
        if (!g_attr_screen[0]) {
            TAC_HIP(hipFuncSetAttribute((const void*)encode_screen<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)kMaxCodebookLds));
            g_attr_screen[0] = true;
        }
        const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + kERows - 1) / kERows, (int64_t)ctx->props_cu));
        if (4 * blocks <= (int64_t)ctx->props_cu) {
            // few row blocks: eight work-groups of 4 subspaces per block
            if (!g_attr_screen4) {
                TAC_HIP(hipFuncSetAttribute((const void*)encode_screen<true, 4>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxCodebookLds));
                g_attr_screen4 = true;
            }
            encode_screen<true, 4><<<(unsigned)(8 * blocks), kEThreads, screen_lds(ksub, 4), ctx->stream>>>(
                x_d, assign_d, C_d, K, n, normalize, codebooks_d, ksub, codes_d, nullptr, rnorm_d);
        } else {
            encode_screen<true><<<(unsigned)(2 * blocks), kEThreads, screen_lds(ksub), ctx->stream>>>(
                x_d, assign_d, C_d, K, n, normalize, codebooks_d, ksub, codes_d, nullptr, rnorm_d);
        }
        TAC_LAUNCH_CHECK("encode_screen");
    } else {
        const unsigned grid =
            (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 511) / 512, (int64_t)ctx->props_cu));
        encode_kernel<<<grid, 512, lds, ctx->stream>>>(x_d, assign_d, C_d, K, n, normalize, codebooks_d, M, ksub,
                                                       codes_d, rnorm_d);
        TAC_LAUNCH_CHECK("encode_kernel");
    }
    time_stop(ctx, TAC_SLOT_ENCODE);
    return TAC_OK;
}

extern "C" tac_status pq_train(tac_ctx ctx, const float* R_d, int64_t n, int32_t d, int32_t M, int32_t ksub,
                               int32_t iters, const float* init_d, float* codebooks_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "pq_train: ctx is NULL");
    tac_status st = check_pq(d, M, ksub, "pq_train");
    if (st != TAC_OK) return st;
    if (n < 0 || n > INT32_MAX || iters < 0) return set_error(TAC_E_INVAL, "pq_train: bad sizes");
    if (!init_d || !codebooks_d || (n > 0 && !R_d)) return set_error(TAC_E_INVAL, "pq_train: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const size_t cb_bytes = (size_t)M * ksub * kDsub * sizeof(float);
    // subspaces sorted together per batch: G * n sort positions must fit int32
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(M, n > 0 ? (int64_t)INT32_MAX / n : M));
    const int64_t gn = (int64_t)G * n;
    Carve cv;
    const size_t o_codes = cv.take<uint32_t>((int64_t)M * n + 1);
    const size_t o_k1 = cv.take<uint32_t>(gn + 1);
    const size_t o_v0 = cv.take<int32_t>(gn + 1), o_v1 = cv.take<int32_t>(gn + 1);
    const size_t o_sort = cv.take<char>(radix_sort_scratch_bytes(gn));
    const size_t o_off = cv.take<int64_t>((int64_t)G * ksub + 1);
    const size_t o_cb = cv.take<char>(cb_bytes);
    st = ws_reserve(ctx, cv.off);
    if (st != TAC_OK) return st;
    uint32_t* codes = ws_at<uint32_t>(ctx, o_codes);
    uint32_t* k1 = ws_at<uint32_t>(ctx, o_k1);
    int32_t* v0 = ws_at<int32_t>(ctx, o_v0);
    int32_t* v1 = ws_at<int32_t>(ctx, o_v1);
    int64_t* off = ws_at<int64_t>(ctx, o_off);
    float* cur = ws_at<float>(ctx, o_cb);
    if (init_d != codebooks_d)
        TAC_HIP(hipMemcpyAsync(codebooks_d, init_d, cb_bytes, hipMemcpyDeviceToDevice, s));
    if (!g_attr_train) {
        TAC_HIP(hipFuncSetAttribute((const void*)train_encode, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kMaxCodebookLds));
        TAC_HIP(hipFuncSetAttribute((const void*)encode_screen<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kMaxCodebookLds));
        g_attr_train = true;
    }
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 511) / 512, (int64_t)ctx->props_cu));
    const size_t lds = (size_t)M * ksub * (kDsub + 1) * sizeof(float);
    for (int it = 0; it < iters && n > 0; ++it) {
        TAC_HIP(hipMemcpyAsync(cur, codebooks_d, cb_bytes, hipMemcpyDeviceToDevice, s));
        if (ksub % 16 == 0) {
            const unsigned sgrid = 2u * (unsigned)std::max<int64_t>(
                                            1, std::min<int64_t>((n + kERows - 1) / kERows, (int64_t)ctx->props_cu));
            encode_screen<false><<<sgrid, kEThreads, screen_lds(ksub), s>>>(R_d, nullptr, nullptr, 0, n, 0, cur, ksub,
                                                                             nullptr, codes, nullptr);
            TAC_LAUNCH_CHECK("encode_screen");
        } else {
            train_encode<<<grid, 512, lds, s>>>(R_d, n, cur, M, ksub, codes);
            TAC_LAUNCH_CHECK("train_encode");
        }
        for (int m0 = 0; m0 < M; m0 += G) {
            const int g = std::min(G, M - m0);
            const int64_t tot = (int64_t)g * n;
            const int nkeys = g * ksub;
            int bits = 1;
            while ((1 << bits) < nkeys) ++bits;
            uint32_t* keys = codes + (int64_t)m0 * n;  // sorted in place (ping-pong with k1)
            train_keys<<<grid_for(tot, 256), 256, 0, s>>>(keys, n, g, ksub);
            TAC_LAUNCH_CHECK("train_keys");
            int in1 = 0;
            st = radix_sort(s, tot, bits, keys, v0, k1, v1, nullptr, ws_at<void>(ctx, o_sort), &in1);
            if (st != TAC_OK) return st;
            code_offsets<<<grid_for(tot + 1, 256), 256, 0, s>>>(in1 ? k1 : keys, tot, nkeys, off);
            TAC_LAUNCH_CHECK("code_offsets");
            code_means<<<(unsigned)(((int64_t)nkeys * 64 + 255) / 256), 256, 0, s>>>(
                R_d, in1 ? v1 : v0, off, n, m0, g, ksub, cur, codebooks_d);
            TAC_LAUNCH_CHECK("code_means");
        }
    }
    return TAC_OK;
}
