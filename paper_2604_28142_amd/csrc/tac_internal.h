// Internal declarations shared by the libtac translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "tac.h"

namespace tac {

constexpr int kDim = 128;          // vector dimension supported by the kernels
constexpr int64_t kFp64Rows = 65536;  // update sums switch to float64 above this many rows per token

// ---- errors ---------------------------------------------------------------
tac_status set_error(tac_status st, const std::string& msg);
tac_status hip_error(hipError_t e, const char* what);

#define TAC_HIP(call)                                               \
    do {                                                            \
        hipError_t _e = (call);                                     \
        if (_e != hipSuccess) return ::tac::hip_error(_e, #call);   \
    } while (0)

#define TAC_LAUNCH_CHECK(what)                                          \
    do {                                                                \
        hipError_t _e = hipGetLastError();                              \
        if (_e != hipSuccess) return ::tac::hip_error(_e, what);        \
    } while (0)

// ---- workspace arena ------------------------------------------------------
// A bump allocator over one device buffer owned by the context.  Every call
// first sums what it needs (plan), reserves it once, then carves it.
struct Carve {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        size_t at = (off + 255) & ~size_t(255);
        off = at + count * sizeof(T);
        return at;
    }
};

}  // namespace tac

struct tac_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t max_ws = 0;
    void* ws = nullptr;
    size_t ws_cap = 0;
    // workspaces replaced by a larger one: kept until the context is destroyed,
    // because HIP graphs captured earlier still address them
    std::vector<void*> ws_retired;
    size_t ws_retired_bytes = 0;
    // per-context device counters of the last tac_assign (rows, screened, fallback, unassigned)
    unsigned long long* counters = nullptr;
    int props_cu = 256;
    tac_tuning tuning = {4, 1024, 0, 0, 0};
    // centroids declared unchanging (tac_ctx_set_static_centroids): the
    // assignment's per-call preparation (norms, bounds, 16-bit staging rows),
    // done once into sc_buf; replaced buffers are retired like workspaces
    const float* sc_C = nullptr;
    int64_t sc_K = 0;
    int32_t sc_prec = -1;
    void* sc_buf = nullptr;
    size_t sc_bytes = 0;
    // a second stream (default priority) and two events: the assignment runs
    // its split route's kernel there, beside the persistent kernel
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // optional HIP-event timing of each entry point's dominant kernel
    bool timing = false;
    hipEvent_t ev[TAC_KERNEL_SLOTS][2] = {};
    bool ev_recorded[TAC_KERNEL_SLOTS] = {};
};

namespace tac {
// Record the start / stop event of a timing slot when timing is enabled.
inline void time_start(tac_ctx ctx, int slot) {
    if (ctx->timing) (void)hipEventRecord(ctx->ev[slot][0], ctx->stream);
}
inline void time_stop(tac_ctx ctx, int slot) {
    if (ctx->timing) {
        (void)hipEventRecord(ctx->ev[slot][1], ctx->stream);
        ctx->ev_recorded[slot] = true;
    }
}
}  // namespace tac

namespace tac {

// Make sure the workspace holds `bytes`; grows (synchronously) when needed.
tac_status ws_reserve(tac_ctx ctx, size_t bytes);
template <class T>
inline T* ws_at(tac_ctx ctx, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ctx->ws) + off);
}

// ---- budget (host) --------------------------------------------------------
tac_status host_budget(const int64_t* counts, const double* spread, int32_t T, int64_t K,
                       const tac_budget_params& p, int64_t* kappa, int64_t* tier2_units);

// ---- device building blocks (launchers enqueue on `s`) --------------------
// Stable LSD radix sort of 32-bit keys by bits [0, bits); values travel with
// the keys (vals_in == nullptr means the identity 0..n-1).  Buffers: keys and
// values ping-pong between (k0,v0) and (k1,v1); the sorted result ends in the
// returned pair index (0 or 1).
size_t radix_sort_scratch_bytes(int64_t n);
tac_status radix_sort(hipStream_t s, int64_t n, int bits, uint32_t* k0, int32_t* v0, uint32_t* k1,
                      int32_t* v1, const int32_t* vals_in, void* scratch, int* result_in_1);

// Exclusive prefix sum of n int64 values (in may equal out); out[n] = total.
size_t scan_scratch_bytes(int64_t n);
tac_status exclusive_scan_i64(hipStream_t s, const int64_t* in, int64_t* out, int64_t n, void* scratch);

}  // namespace tac
