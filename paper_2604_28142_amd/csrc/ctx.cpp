// Context, workspace arena and error reporting of libtac.
#include <cstring>
#include <new>

#include "tac_internal.h"

namespace tac {

static thread_local std::string g_last_error;

tac_status set_error(tac_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

tac_status hip_error(hipError_t e, const char* what) {
    std::string m = what;
    m += ": ";
    m += hipGetErrorName(e);
    m += " (";
    m += hipGetErrorString(e);
    m += ")";
    return set_error(TAC_E_HIP, m);
}

tac_status ws_reserve(tac_ctx ctx, size_t bytes) {
    if (bytes <= ctx->ws_cap) return TAC_OK;
    // the limit bounds every allocation the context holds, replaced workspaces included
    const size_t held = ctx->ws_retired_bytes + ctx->ws_cap + ctx->sc_bytes;
    if (ctx->max_ws && held + bytes > ctx->max_ws)
        return set_error(TAC_E_NOMEM, "workspace of " + std::to_string(bytes) + " bytes (with " +
                                          std::to_string(held) + " bytes already held) exceeds the context limit of " +
                                          std::to_string(ctx->max_ws));
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TAC_HIP(hipStreamIsCapturing(ctx->stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return set_error(TAC_E_NOMEM, "workspace must grow to " + std::to_string(bytes) +
                                          " bytes, which is not allowed during stream capture; "
                                          "run one eager call of the same sizes first");
    // round up to limit regrowth
    size_t cap = bytes + bytes / 8 + (size_t(1) << 20);
    if (ctx->max_ws && held + cap > ctx->max_ws) cap = ctx->max_ws - held;
    TAC_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->ws) {
        // not freed: a graph captured on this context may still address it
        ctx->ws_retired.push_back(ctx->ws);
        ctx->ws_retired_bytes += ctx->ws_cap;
        ctx->ws = nullptr;
        ctx->ws_cap = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cap);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(TAC_E_NOMEM, "hipMalloc of " + std::to_string(cap) + " workspace bytes failed");
    }
    ctx->ws = p;
    ctx->ws_cap = cap;
    return TAC_OK;
}

}  // namespace tac

using namespace tac;

extern "C" const char* tac_last_error(void) { return g_last_error.c_str(); }

extern "C" tac_status tac_ctx_create(int device, void* hip_stream, size_t max_workspace_bytes, tac_ctx* out) {
    if (!out) return set_error(TAC_E_INVAL, "tac_ctx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    TAC_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n)
        return set_error(TAC_E_INVAL, "tac_ctx_create: device " + std::to_string(device) + " out of range");
    TAC_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    TAC_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(TAC_E_INVAL, std::string("libtac is built for gfx950, device is ") + prop.gcnArchName);
    tac_ctx c = new (std::nothrow) tac_ctx_s();
    if (!c) return set_error(TAC_E_NOMEM, "tac_ctx_create: out of host memory");
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->max_ws = max_workspace_bytes;
    c->props_cu = prop.multiProcessorCount;
    hipError_t e = hipMalloc(&c->counters, 8 * sizeof(unsigned long long));
    if (e != hipSuccess) {
        delete c;
        return hip_error(e, "hipMalloc(counters)");
    }
    e = hipMemset(c->counters, 0, 8 * sizeof(unsigned long long));
    if (e != hipSuccess) {
        (void)hipFree(c->counters);
        delete c;
        return hip_error(e, "hipMemset(counters)");
    }
    e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (c->join_ev) (void)hipEventDestroy(c->join_ev);
        if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
        if (c->aux) (void)hipStreamDestroy(c->aux);
        (void)hipFree(c->counters);
        delete c;
        return hip_error(e, "tac_ctx_create: auxiliary stream");
    }
    *out = c;
    return TAC_OK;
}

extern "C" tac_status tac_ctx_set_stream(tac_ctx ctx, void* hip_stream) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_ctx_set_stream: ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return TAC_OK;
}

extern "C" tac_status tac_ctx_set_tuning(tac_ctx ctx, const tac_tuning* t) {
    if (!ctx || !t) return set_error(TAC_E_INVAL, "tac_ctx_set_tuning: NULL argument");
    if (t->direct_max_kappa < 0 || t->direct_max_kappa > 16 || t->heavy_kappa < 1 || t->groups_per_cu < 0 ||
        (t->tile_blocks != 0 && (t->tile_blocks < 3 || t->tile_blocks > 5)) || t->waves_per_simd < 0 ||
        t->waves_per_simd > 2 || (t->waves_per_simd == 2 && t->tile_blocks != 0 && t->tile_blocks != 3))
        return set_error(TAC_E_INVAL, "tac_ctx_set_tuning: direct_max_kappa in [0, 16], heavy_kappa >= 1, "
                                      "groups_per_cu >= 0, tile_blocks 0 or in [3, 5], waves_per_simd in [0, 2] "
                                      "(with 2, tile_blocks 0 or 3)");
    ctx->tuning = *t;
    return TAC_OK;
}

extern "C" tac_status tac_ctx_get_tuning(tac_ctx ctx, tac_tuning* t) {
    if (!ctx || !t) return set_error(TAC_E_INVAL, "tac_ctx_get_tuning: NULL argument");
    *t = ctx->tuning;
    return TAC_OK;
}

extern "C" tac_status tac_ctx_enable_timing(tac_ctx ctx, int enable) {
    if (!ctx) return set_error(TAC_E_INVAL, "tac_ctx_enable_timing: ctx is NULL");
    TAC_HIP(hipSetDevice(ctx->device));
    if (enable && !ctx->ev[0][0]) {
        for (int s = 0; s < TAC_KERNEL_SLOTS; ++s)
            for (int k = 0; k < 2; ++k) TAC_HIP(hipEventCreate(&ctx->ev[s][k]));
    }
    ctx->timing = enable != 0;
    return TAC_OK;
}

extern "C" tac_status tac_kernel_ms(tac_ctx ctx, int slot, float* ms) {
    if (!ctx || !ms || slot < 0 || slot >= TAC_KERNEL_SLOTS)
        return set_error(TAC_E_INVAL, "tac_kernel_ms: bad argument");
    if (!ctx->ev_recorded[slot]) return set_error(TAC_E_INVAL, "tac_kernel_ms: slot never recorded");
    TAC_HIP(hipSetDevice(ctx->device));
    TAC_HIP(hipEventSynchronize(ctx->ev[slot][1]));
    TAC_HIP(hipEventElapsedTime(ms, ctx->ev[slot][0], ctx->ev[slot][1]));
    return TAC_OK;
}

extern "C" void tac_ctx_destroy(tac_ctx ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int s = 0; s < TAC_KERNEL_SLOTS; ++s)
        for (int k = 0; k < 2; ++k)
            if (ctx->ev[s][k]) (void)hipEventDestroy(ctx->ev[s][k]);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->sc_buf) (void)hipFree(ctx->sc_buf);
    for (void* p : ctx->ws_retired) (void)hipFree(p);
    if (ctx->counters) (void)hipFree(ctx->counters);
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        (void)hipStreamDestroy(ctx->aux);
    }
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    delete ctx;
}
