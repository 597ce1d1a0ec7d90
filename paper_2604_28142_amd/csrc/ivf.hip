// Index structures built from the clustering (Sect. 2.2): the inverted list of
// every centroid (the ids of the documents whose tokens it holds) and the
// per-document layout (all centroid ids of a document's tokens, then all of
// their PQ codes).
//
// Inverted lists: rows are stably sorted by document id, then by centroid
// (LSD radix sorts), so each centroid's rows form a run with non-decreasing
// document ids; the first row of every distinct (centroid, document) pair is
// kept (flags and an exclusive scan), which gives each list its ids once and
// in increasing order.  Everything is integer work, so the result is exact.
#include "tac_internal.h"

namespace tac {

namespace {

unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

int key_bits(int64_t max_key) {
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) <= max_key) ++bits;
    return bits;
}

// keys for the first sort: the document id (D for ids outside [0, D))
__global__ void ivf_doc_keys(const int32_t* __restrict__ doc, int64_t n, int64_t D, uint32_t* __restrict__ keys) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = doc[i];
        keys[i] = (d < 0 || d >= D) ? (uint32_t)D : (uint32_t)d;
    }
}

// keys for the second sort, in document order: the centroid (K when the row
// has no centroid or no valid document), carrying the document id
__global__ void ivf_cent_keys(const int32_t* __restrict__ assign, const int32_t* __restrict__ doc,
                              const int32_t* __restrict__ rows, int64_t n, int64_t K, int64_t D,
                              uint32_t* __restrict__ keys, int32_t* __restrict__ vals) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rows[i];
        const int32_t a = assign[r];
        const int32_t d = doc[r];
        const bool valid = a >= 0 && a < K && d >= 0 && d < D;
        keys[i] = valid ? (uint32_t)a : (uint32_t)K;
        vals[i] = valid ? d : 0;
    }
}

// flag[i] = 1 for the first row of each distinct (centroid, document) pair
__global__ void ivf_flags(const uint32_t* __restrict__ k, const int32_t* __restrict__ v, int64_t n, int64_t K,
                          int64_t* __restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = k[i] < (uint32_t)K && (i == 0 || k[i] != k[i - 1] || v[i] != v[i - 1]) ? 1 : 0;
}

__global__ void ivf_compact(const int32_t* __restrict__ v, const int64_t* __restrict__ pos, int64_t n,
                            int32_t* __restrict__ docs) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (pos[i + 1] != pos[i]) docs[pos[i]] = v[i];
}

// off[c] = the compacted position of the first row whose centroid key is >= c
__global__ void ivf_offsets(const uint32_t* __restrict__ k, const int64_t* __restrict__ pos, int64_t n, int64_t K,
                            int64_t* __restrict__ off) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t prev = i == 0 ? -1 : (int64_t)min(k[i - 1], (uint32_t)K);
        const int64_t cur = i == n ? K : (int64_t)min(k[i], (uint32_t)K);
        for (int64_t t = prev + 1; t <= cur; ++t) off[t] = pos[i];
    }
}

__global__ void fill_i64(int64_t* __restrict__ p, int64_t n, int64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One wave per document: its centroid ids (4-byte little-endian), then its
// PQ codes in token order.  Offsets are clamped to [0, N], so malformed ones
// cannot address memory outside the layout.
__global__ void __launch_bounds__(256) doc_layout_kernel(const int32_t* __restrict__ assign,
                                                         const uint8_t* __restrict__ codes, int M,
                                                         const int64_t* __restrict__ doc_off, int64_t D, int64_t N,
                                                         uint8_t* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t d = wave0; d < D; d += nwaves) {
        const int64_t b = min(max(doc_off[d], (int64_t)0), N);
        const int64_t e = min(max(doc_off[d + 1], b), N);
        const int64_t n = e - b;
        uint8_t* base = out + b * (4 + (int64_t)M);
        if (M % 4 == 0) {  // word copies: the layout keeps 4-byte alignment
            uint32_t* ids = reinterpret_cast<uint32_t*>(base);
            for (int64_t i = lane; i < n; i += 64) ids[i] = (uint32_t)assign[b + i];
            const uint32_t* src = reinterpret_cast<const uint32_t*>(codes + b * M);
            uint32_t* dst = reinterpret_cast<uint32_t*>(base + 4 * n);
            const int64_t words = n * M / 4;
            for (int64_t w = lane; w < words; w += 64) dst[w] = src[w];
        } else {
            for (int64_t i = lane; i < 4 * n; i += 64) base[i] = (uint8_t)((uint32_t)assign[b + i / 4] >> (8 * (i % 4)));
            const uint8_t* src = codes + b * M;
            uint8_t* dst = base + 4 * n;
            for (int64_t i = lane; i < n * M; i += 64) dst[i] = src[i];
        }
    }
}

}  // namespace

}  // namespace tac

using namespace tac;

extern "C" tac_status tac_ivf_build(tac_ctx ctx, const int32_t* assign_d, const int32_t* doc_d, int64_t N, int64_t K,
                                    int64_t D, int64_t* list_off_d, int32_t* list_docs_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_ivf_build: ctx is NULL");
    if (N < 0 || N > INT32_MAX || K < 1 || K >= INT32_MAX || D < 1 || D >= INT32_MAX)
        return set_error(TAC_E_INVAL, "tac_ivf_build: bad sizes");
    if (!list_off_d || (N > 0 && (!assign_d || !doc_d || !list_docs_d)))
        return set_error(TAC_E_INVAL, "tac_ivf_build: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    if (N == 0) {
        fill_i64<<<grid_for(K + 1, 256), 256, 0, s>>>(list_off_d, K + 1, 0);
        TAC_LAUNCH_CHECK("fill_i64");
        return TAC_OK;
    }
    Carve cv;
    const size_t o_k0 = cv.take<uint32_t>(N + 1), o_v0 = cv.take<int32_t>(N + 1);
    const size_t o_k1 = cv.take<uint32_t>(N + 1), o_v1 = cv.take<int32_t>(N + 1);
    const size_t o_k2 = cv.take<uint32_t>(N + 1), o_v2 = cv.take<int32_t>(N + 1);
    const size_t o_sort = cv.take<char>(radix_sort_scratch_bytes(N));
    const size_t o_pos = cv.take<int64_t>(N + 1);
    const size_t o_scan = cv.take<char>(scan_scratch_bytes(N));
    tac_status st = ws_reserve(ctx, cv.off);
    if (st != TAC_OK) return st;
    uint32_t* k0 = ws_at<uint32_t>(ctx, o_k0);
    int32_t* v0 = ws_at<int32_t>(ctx, o_v0);
    uint32_t* k1 = ws_at<uint32_t>(ctx, o_k1);
    int32_t* v1 = ws_at<int32_t>(ctx, o_v1);
    uint32_t* k2 = ws_at<uint32_t>(ctx, o_k2);
    int32_t* v2 = ws_at<int32_t>(ctx, o_v2);
    int64_t* pos = ws_at<int64_t>(ctx, o_pos);
    // rows in document order
    ivf_doc_keys<<<grid_for(N, 256), 256, 0, s>>>(doc_d, N, D, k0);
    TAC_LAUNCH_CHECK("ivf_doc_keys");
    int in1 = 0;
    st = radix_sort(s, N, key_bits(D), k0, v0, k1, v1, nullptr, ws_at<void>(ctx, o_sort), &in1);
    if (st != TAC_OK) return st;
    // then by centroid (stable: document order is kept within a centroid)
    ivf_cent_keys<<<grid_for(N, 256), 256, 0, s>>>(assign_d, doc_d, in1 ? v1 : v0, N, K, D, k2, v2);
    TAC_LAUNCH_CHECK("ivf_cent_keys");
    st = radix_sort(s, N, key_bits(K), k2, v2, k0, v0, v2, ws_at<void>(ctx, o_sort), &in1);
    if (st != TAC_OK) return st;
    const uint32_t* ks = in1 ? k0 : k2;
    const int32_t* vs = in1 ? v0 : v2;
    ivf_flags<<<grid_for(N, 256), 256, 0, s>>>(ks, vs, N, K, pos);
    TAC_LAUNCH_CHECK("ivf_flags");
    st = exclusive_scan_i64(s, pos, pos, N, ws_at<void>(ctx, o_scan));
    if (st != TAC_OK) return st;
    ivf_compact<<<grid_for(N, 256), 256, 0, s>>>(vs, pos, N, list_docs_d);
    TAC_LAUNCH_CHECK("ivf_compact");
    ivf_offsets<<<grid_for(N + 1, 256), 256, 0, s>>>(ks, pos, N, K, list_off_d);
    TAC_LAUNCH_CHECK("ivf_offsets");
    return TAC_OK;
}

extern "C" tac_status tac_doc_layout(tac_ctx ctx, const int32_t* assign_d, const uint8_t* codes_d, int32_t M,
                                     const int64_t* doc_off_d, int64_t D, int64_t N, uint8_t* layout_d) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_doc_layout: ctx is NULL");
    if (N < 0 || D < 0 || M < 1 || M > 4096) return set_error(TAC_E_INVAL, "tac_doc_layout: bad sizes");
    if (D == 0 || N == 0) return TAC_OK;
    if (!assign_d || !codes_d || !doc_off_d || !layout_d) return set_error(TAC_E_INVAL, "tac_doc_layout: NULL pointer");
    TAC_HIP(hipSetDevice(ctx->device));
    doc_layout_kernel<<<grid_for(D * 64, 256), 256, 0, ctx->stream>>>(assign_d, codes_d, M, doc_off_d, D, N, layout_d);
    TAC_LAUNCH_CHECK("doc_layout_kernel");
    return TAC_OK;
}
