// Refine phase of retrieval (Sect. 2.2, "Refine Phase: PQ-Optimized MaxSim
// Computation"): the MaxSim score of candidate documents for a query,
//   S(q, d) = sum_i max_{t in d} <q_i, x_t>,  x_t = c_{a_t} + rho_t * u_t,
// read from the document layout (centroid ids, then PQ codes) with the
// residual norms stored apart and u_t the concatenated codewords of the
// token's 32 codes.
//
// Design on gfx950.  A persistent work-group of 8 waves keeps the codebooks
// (32 x ksub codewords, at most 128 KiB) in LDS; each wave scores a contiguous
// range of (query, document) pairs and keeps the current query's operand
// fragments in registers.  For every block of 16 document tokens it decodes
// x = c_a + rho * u straight into the A operand of v_mfma_f32_16x16x4f32 and
// contracts it with two blocks of 16 query tokens: 64 matrix instructions per
// token block.  Lane group g supplies coordinates 16 i + 4 g + k (i = 0..7,
// k = 0..3), so the four lanes of a token read 64 contiguous bytes of its
// centroid per load and each lane reads whole codewords (subspace 4 i + g)
// from LDS.  The paper's per-query distance tables (M x 256 x n_q floats,
// 1 MiB at n_q = 32, laid out so that one code fetches the values of all query
// tokens) exist to share one lookup among the query tokens on a CPU; here the
// decoded coordinate is shared by all query tokens in the matrix instruction
// instead, and only the codebooks have to fit in LDS.
#include <algorithm>
#include <cmath>

#include "tac_internal.h"

namespace tac {

namespace {

constexpr int kRThreads = 512;
constexpr int kRDim = 128;
constexpr int kRM = 32;     // PQ subspaces of 4 coordinates
constexpr int kRMaxQ = 32;  // query tokens: two blocks of 16

typedef float f4 __attribute__((ext_vector_type(4)));

// B fragments of query b: token 16 jb + col, coordinates 16 i + 4 g + k (zero past nq)
__device__ __forceinline__ void load_query(const float* __restrict__ Q, int64_t b, int nq, int g, int col,
                                           float (&qf)[2][32]) {
    const float* qb = Q + b * (int64_t)nq * kRDim;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        const int j = jb * 16 + col;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < nq) v = reinterpret_cast<const float4*>(qb + (int64_t)j * kRDim)[4 * i + g];
            qf[jb][4 * i + 0] = v.x;
            qf[jb][4 * i + 1] = v.y;
            qf[jb][4 * i + 2] = v.z;
            qf[jb][4 * i + 3] = v.w;
        }
    }
}

// One block of 16 document tokens as lane (g, col) needs it: token col's
// validity, norm, 32 codes and the 32 centroid coordinates 16 i + 4 g + k.
struct Stage {
    bool ok;
    float rho;
    uint32_t cw[8];
    float4 cv[8];
    __device__ __forceinline__ void load(int a, int64_t K, const float* __restrict__ C,
                                         const uint8_t* __restrict__ codes, const float* __restrict__ rnorm,
                                         int64_t t0, int64_t blk, int col, int g) {
        ok = a >= 0 && a < K;
        rho = 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            cw[i] = 0u;
            cv[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (ok) {
            const int64_t t = blk + col;
            rho = rnorm[t0 + t];
            const uint32_t* cr = reinterpret_cast<const uint32_t*>(codes + 32 * t);
            const float4* crow = reinterpret_cast<const float4*>(C + (int64_t)a * kRDim);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                cw[i] = cr[i];
                cv[i] = crow[4 * i + g];
            }
        }
    }
};

__global__ void __launch_bounds__(kRThreads) maxsim_kernel(const float* __restrict__ Q, int64_t nb, int nq,
                                                           const float* __restrict__ C, int64_t K,
                                                           const float* __restrict__ cbg, int ksub,
                                                           const uint8_t* __restrict__ layout,
                                                           const int64_t* __restrict__ doc_off, int64_t D,
                                                           int64_t N, const float* __restrict__ rnorm,
                                                           const int32_t* __restrict__ cand, int64_t nc,
                                                           float* __restrict__ scores) {
    extern __shared__ float4 lcb[];  // codeword (m, b) at m * ksub + b
    for (int i = threadIdx.x; i < kRM * ksub; i += kRThreads) lcb[i] = reinterpret_cast<const float4*>(cbg)[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
    const int64_t items = nb * nc;
    const int64_t waves = (int64_t)gridDim.x * (kRThreads / 64);
    const int64_t per = (items + waves - 1) / waves;
    const int64_t w = (int64_t)blockIdx.x * (kRThreads / 64) + wave;
    const int64_t it0 = w * per, it1 = min(items, it0 + per);
    float qf[2][32];
    int64_t qcur = -1;
    for (int64_t it = it0; it < it1; ++it) {
        const int64_t b = it / nc;
        if (b != qcur) {
            load_query(Q, b, nq, g, col, qf);
            qcur = b;
        }
        const int64_t d = cand[it];
        float score = NAN;
        if (d >= 0 && d < D) {
            const int64_t t0 = min(max(doc_off[d], (int64_t)0), N);
            const int64_t t1 = min(max(doc_off[d + 1], t0), N);
            const int64_t nd = t1 - t0;
            const uint8_t* base = layout + t0 * (4 + kRM);
            const int32_t* ids = reinterpret_cast<const int32_t*>(base);
            const uint8_t* codes = base + 4 * nd;
            float mx0 = -INFINITY, mx1 = -INFINITY;
            // Software pipeline over blocks of 16 tokens: the centroid ids run two
            // blocks ahead, the centroid row, codes and norm of the next block one
            // block ahead, so their memory latency overlaps the matrix work.
            auto id_of = [&](int64_t blk) { return blk + col < nd ? ids[blk + col] : -1; };
            Stage cur, nxt;
            int a1 = id_of(16);
            cur.load(id_of(0), K, C, codes, rnorm, t0, 0, col, g);
            for (int64_t blk = 0; blk < nd; blk += 16) {
                if (blk + 16 < nd) {
                    nxt.load(a1, K, C, codes, rnorm, t0, blk + 16, col, g);
                    a1 = id_of(blk + 32);
                }
                f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < 8; ++i) {  // subspace 4 i + g: coordinates 16 i + 4 g .. 16 i + 4 g + 3
                    const int code = min((int)((cur.cw[i] >> (8 * g)) & 0xFFu), ksub - 1);
                    const float4 bv = lcb[(4 * i + g) * ksub + code];
                    const float4 cv = cur.cv[i];
                    const float x[4] = {fmaf(cur.rho, bv.x, cv.x), fmaf(cur.rho, bv.y, cv.y),
                                        fmaf(cur.rho, bv.z, cv.z), fmaf(cur.rho, bv.w, cv.w)};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[k], qf[0][4 * i + k], acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[k], qf[1][4 * i + k], acc1, 0, 0, 0);
                    }
                }
                // acc[r] = <x of token blk + 4 g + r, q_{16 jb + col}>; tokens without a centroid are left out
                const uint64_t okm = __ballot(cur.ok);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if ((okm >> (4 * g + r)) & 1ull) {
                        mx0 = fmaxf(mx0, acc0[r]);
                        mx1 = fmaxf(mx1, acc1[r]);
                    }
                }
                cur = nxt;
            }
            // maximum over the four lane groups, then the sum over query tokens in a fixed order
#pragma unroll
            for (int o = 16; o <= 32; o <<= 1) {
                mx0 = fmaxf(mx0, __shfl_xor(mx0, o));
                mx1 = fmaxf(mx1, __shfl_xor(mx1, o));
            }
            float s = (col < nq ? mx0 : 0.f) + (16 + col < nq ? mx1 : 0.f);
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) s += __shfl_xor(s, o);
            score = s;
        }
        if (lane == 0) scores[it] = score;
    }
}

bool g_attr_maxsim = false;

}  // namespace

}  // namespace tac

using namespace tac;

extern "C" tac_status tac_maxsim(tac_ctx ctx, const float* Q_d, int64_t B, int32_t nq, int32_t d,
                                 const float* C_d, int64_t K, const float* codebooks_d, int32_t M, int32_t ksub,
                                 const uint8_t* layout_d, const int64_t* doc_off_d, int64_t D, int64_t N,
                                 const float* rnorm_d, const int32_t* cand_d, int64_t nc, float* scores_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_maxsim: ctx is NULL");
    if (d != kRDim) return set_error(TAC_E_INVAL, "tac_maxsim: d must be 128");
    if (M != kRM) return set_error(TAC_E_INVAL, "tac_maxsim: M must be 32 (subspaces of 4 coordinates)");
    if (ksub < 1 || ksub > 256) return set_error(TAC_E_INVAL, "tac_maxsim: ksub must be in [1, 256]");
    if (nq < 1 || nq > kRMaxQ) return set_error(TAC_E_INVAL, "tac_maxsim: nq must be in [1, 32]");
    if (B < 0 || B > 65535 || K < 0 || D < 0 || N < 0 || nc < 0)
        return set_error(TAC_E_INVAL, "tac_maxsim: bad sizes");
    if (B == 0 || nc == 0) return TAC_OK;
    if (!Q_d || !codebooks_d || !doc_off_d || !cand_d || !scores_d || (K > 0 && !C_d) ||
        (N > 0 && (!layout_d || !rnorm_d)))
        return set_error(TAC_E_INVAL, "tac_maxsim: NULL pointer");
    if ((reinterpret_cast<uintptr_t>(layout_d) & 3u) != 0u)
        return set_error(TAC_E_INVAL, "tac_maxsim: layout must be 4-byte aligned");
    TAC_HIP(hipSetDevice(ctx->device));
    const size_t lds = (size_t)kRM * ksub * sizeof(float4);
    if (!g_attr_maxsim) {
        TAC_HIP(hipFuncSetAttribute((const void*)maxsim_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(kRM * 256 * sizeof(float4))));
        g_attr_maxsim = true;
    }
    // one persistent work-group per CU (the codebooks fill its LDS), fewer for small calls
    const int64_t items = B * nc;
    const int64_t wgs = std::max<int64_t>(1, std::min<int64_t>((int64_t)ctx->props_cu,
                                                                (items + 8 * (kRThreads / 64) - 1) /
                                                                    (8 * (kRThreads / 64))));
    maxsim_kernel<<<(unsigned)wgs, kRThreads, lds, ctx->stream>>>(Q_d, B, nq, C_d, K, codebooks_d, ksub, layout_d,
                                                                   doc_off_d, D, N, rnorm_d, cand_d, nc, scores_d);
    TAC_LAUNCH_CHECK("maxsim_kernel");
    return TAC_OK;
}
