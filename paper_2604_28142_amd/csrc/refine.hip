// Refine phase of retrieval (Sect. 2.3, "Refine Phase: PQ-Optimized MaxSim
// Computation"): the MaxSim score of candidate documents for a query,
//   S(q, d) = sum_i max_{t in d} <q_i, x_t>,  x_t = c_{a_t} + rho_t * u_t,
// read from the document layout (centroid ids, then PQ codes) with the
// residual norms stored apart and u_t the concatenated codewords of the
// token's 32 codes.
//
// Design on gfx950.  One wave scores one (query, document) pair at a time and
// keeps the query's operand fragments in registers for all of its documents.
// For every block of 16 document tokens it decodes x = c_a + rho * u straight
// into the A operand of v_mfma_f32_16x16x4f32 and contracts it with two
// blocks of 16 query tokens: 64 matrix instructions per token block.  The
// contraction visits coordinate 32 g + s at step s in lane group g, so a lane
// reads 128 contiguous bytes of its token's centroid and the whole 16-byte
// codewords of subspaces 8 g .. 8 g + 7.  The paper's per-query distance
// tables (M x 256 x n_q floats, 1 MiB at n_q = 32, laid out so that one code
// fetches the values of all query tokens) exist to share one lookup among the
// query tokens on a CPU; here the decoded coordinate is shared by all query
// tokens in the matrix instruction instead, and nothing per query has to fit
// in LDS.
#include <cmath>

#include "tac_internal.h"

namespace tac {

namespace {

constexpr int kRThreads = 256;
constexpr int kRDocsPerWave = 8;
constexpr int kRDim = 128;
constexpr int kRM = 32;     // PQ subspaces of 4 coordinates
constexpr int kRMaxQ = 32;  // query tokens: two blocks of 16

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kRThreads) maxsim_kernel(const float* __restrict__ Q, int nq,
                                                           const float* __restrict__ C, int64_t K,
                                                           const float* __restrict__ cb, int ksub,
                                                           const uint8_t* __restrict__ layout,
                                                           const int64_t* __restrict__ doc_off, int64_t D,
                                                           int64_t N, const float* __restrict__ rnorm,
                                                           const int32_t* __restrict__ cand, int64_t nc,
                                                           float* __restrict__ scores) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, col = lane & 15;
    const int64_t b = blockIdx.y;
    const int64_t c0 = ((int64_t)blockIdx.x * (kRThreads / 64) + wave) * kRDocsPerWave;
    if (c0 >= nc) return;
    // B fragments: query token 16 jb + col, coordinates 32 g + s (zero past nq)
    float qf[2][32];
    const float* qb = Q + b * (int64_t)nq * kRDim;
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        const int j = jb * 16 + col;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < nq) v = reinterpret_cast<const float4*>(qb + (int64_t)j * kRDim + 32 * g)[i];
            qf[jb][4 * i + 0] = v.x;
            qf[jb][4 * i + 1] = v.y;
            qf[jb][4 * i + 2] = v.z;
            qf[jb][4 * i + 3] = v.w;
        }
    }
    for (int k = 0; k < kRDocsPerWave; ++k) {
        const int64_t ci = c0 + k;
        if (ci >= nc) break;
        const int64_t d = cand[b * nc + ci];
        float score = NAN;
        if (d >= 0 && d < D) {
            const int64_t t0 = min(max(doc_off[d], (int64_t)0), N);
            const int64_t t1 = min(max(doc_off[d + 1], t0), N);
            const int64_t nd = t1 - t0;
            const uint8_t* base = layout + t0 * (4 + kRM);
            const int32_t* ids = reinterpret_cast<const int32_t*>(base);
            const uint8_t* codes = base + 4 * nd;
            float mx0 = -INFINITY, mx1 = -INFINITY;
            for (int64_t blk = 0; blk < nd; blk += 16) {
                const int64_t t = blk + col;
                const int a = t < nd ? ids[t] : -1;
                const bool ok = a >= 0 && a < K;
                f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
                float rho = 0.f;
                uint32_t w0 = 0u, w1 = 0u;
                const float* crow = C;
                if (ok) {
                    rho = rnorm[t0 + t];
                    const uint32_t* cw = reinterpret_cast<const uint32_t*>(codes + 32 * t + 8 * g);
                    w0 = cw[0];
                    w1 = cw[1];
                    crow = C + (int64_t)a * kRDim + 32 * g;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {  // subspace 8 g + i, coordinates 32 g + 4 i .. 32 g + 4 i + 3
                    const int code = min((int)(((i < 4 ? w0 : w1) >> (8 * (i & 3))) & 0xFFu), ksub - 1);
                    float4 cv = make_float4(0.f, 0.f, 0.f, 0.f), bv = cv;
                    if (ok) {
                        cv = reinterpret_cast<const float4*>(crow)[i];
                        bv = reinterpret_cast<const float4*>(cb)[(int64_t)(8 * g + i) * ksub + code];
                    }
                    const float x[4] = {fmaf(rho, bv.x, cv.x), fmaf(rho, bv.y, cv.y), fmaf(rho, bv.z, cv.z),
                                        fmaf(rho, bv.w, cv.w)};
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[kk], qf[0][4 * i + kk], acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x[kk], qf[1][4 * i + kk], acc1, 0, 0, 0);
                    }
                }
                // acc[r] = <x of token blk + 4 g + r, q_{16 jb + col}>; tokens without a centroid are left out
                const uint64_t okm = __ballot(ok);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if ((okm >> (4 * g + r)) & 1ull) {
                        mx0 = fmaxf(mx0, acc0[r]);
                        mx1 = fmaxf(mx1, acc1[r]);
                    }
                }
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
        if (lane == 0) scores[b * nc + ci] = score;
    }
}

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
    const int64_t per_block = (int64_t)(kRThreads / 64) * kRDocsPerWave;
    const int64_t gx = (nc + per_block - 1) / per_block;
    if (gx > INT32_MAX) return set_error(TAC_E_INVAL, "tac_maxsim: too many candidates");
    TAC_HIP(hipSetDevice(ctx->device));
    maxsim_kernel<<<dim3((unsigned)gx, (unsigned)B), kRThreads, 0, ctx->stream>>>(
        Q_d, nq, C_d, K, codebooks_d, ksub, layout_d, doc_off_d, D, N, rnorm_d, cand_d, nc, scores_d);
    TAC_LAUNCH_CHECK("maxsim_kernel");
    return TAC_OK;
}
