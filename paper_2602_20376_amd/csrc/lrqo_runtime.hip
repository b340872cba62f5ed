// Host runtime of liblrqo: error text, stream, per-device scratch.
#include "lrqo_runtime.h"

#include <cstdlib>
#include <cstring>
#include <memory>

namespace lrqo {

namespace {
thread_local std::string t_error;
thread_local hipStream_t t_stream = nullptr;

constexpr int kMaxDevices = 64;
std::mutex g_ctx_mu;
DeviceCtx* g_ctx[kMaxDevices] = {};
}  // namespace

lrqo_status fail(lrqo_status st, const std::string& msg) {
    t_error = msg;
    return st;
}

void clear_error() { t_error.clear(); }

hipStream_t current_stream() { return t_stream; }

DeviceCtx* device_ctx() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        fail(LRQO_EDEVICE, std::string("hipGetDevice failed: ") + hipGetErrorString(e));
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if (!g_ctx[dev]) {
        auto* c = new DeviceCtx();
        c->device = dev;
        if (hipEventCreate(&c->ev_start) != hipSuccess || hipEventCreate(&c->ev_stop) != hipSuccess ||
            hipEventCreate(&c->ev_score0) != hipSuccess || hipEventCreate(&c->ev_score1) != hipSuccess) {
            delete c;
            fail(LRQO_EDEVICE, "hipEventCreate failed");
            return nullptr;
        }
        g_ctx[dev] = c;
    }
    return g_ctx[dev];
}

// Upper bound on one call's device scratch, from LRQO_ARENA_LIMIT (bytes; a
// positive integer, read at every call); 0 means none.
size_t arena_limit() {
    const char* e = std::getenv("LRQO_ARENA_LIMIT");
    if (!e || !*e) return 0;
    const long long v = std::atoll(e);
    return v > 0 ? (size_t)v : 0;
}

lrqo_status reserve_arena(DeviceCtx* ctx, size_t bytes) {
    const size_t limit = arena_limit();
    if (limit && bytes > limit)
        return fail(LRQO_ENOMEM, "device scratch of " + std::to_string(bytes) + " bytes exceeds LRQO_ARENA_LIMIT (" +
                                     std::to_string(limit) + " bytes)");
    if (bytes <= ctx->arena_bytes) return LRQO_OK;
    if (ctx->arena) {
        LRQO_HIP(hipDeviceSynchronize());
        LRQO_HIP(hipFree(ctx->arena));
        ctx->arena = nullptr;
        ctx->arena_bytes = 0;
    }
    // grow geometrically to avoid a reallocation per size step
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&ctx->arena, want) != hipSuccess) {
        (void)hipGetLastError();
        ctx->arena = nullptr;
        if (hipMalloc(&ctx->arena, bytes) != hipSuccess) {
            (void)hipGetLastError();
            ctx->arena = nullptr;
            return fail(LRQO_ENOMEM, "device scratch allocation of " + std::to_string(bytes) +
                                         " bytes failed");
        }
        want = bytes;
    }
    ctx->arena_bytes = want;
    return LRQO_OK;
}

lrqo_status reserve_host(DeviceCtx* ctx, size_t bytes) {
    if (bytes <= ctx->host_bytes) return LRQO_OK;
    if (ctx->host) {
        LRQO_HIP(hipHostFree(ctx->host));
        ctx->host = nullptr;
        ctx->host_bytes = 0;
    }
    if (hipHostMalloc(&ctx->host, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ctx->host = nullptr;
        return fail(LRQO_ENOMEM, "pinned host allocation failed");
    }
    ctx->host_bytes = bytes;
    return LRQO_OK;
}

bool is_device_pointer(const void* p) {
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

}  // namespace lrqo

extern "C" {

int32_t lrqo_version(void) { return 20000; }

const char* lrqo_last_error(void) { return lrqo::t_error.c_str(); }

lrqo_status lrqo_set_stream(void* hip_stream) {
    lrqo::t_stream = static_cast<hipStream_t>(hip_stream);
    return LRQO_OK;
}

lrqo_status lrqo_shutdown(void) {
    std::lock_guard<std::mutex> lk(lrqo::g_ctx_mu);
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (int d = 0; d < lrqo::kMaxDevices; ++d) {
        lrqo::DeviceCtx* c = lrqo::g_ctx[d];
        if (!c) continue;
        {
            std::lock_guard<std::mutex> dl(c->mu);
            if (hipSetDevice(d) == hipSuccess) {
                (void)hipDeviceSynchronize();
                if (c->arena) (void)hipFree(c->arena);
                if (c->host) (void)hipHostFree(c->host);
                (void)hipEventDestroy(c->ev_start);
                (void)hipEventDestroy(c->ev_stop);
                (void)hipEventDestroy(c->ev_score0);
                (void)hipEventDestroy(c->ev_score1);
            }
        }
        lrqo::g_ctx[d] = nullptr;
        delete c;
    }
    if (cur >= 0) (void)hipSetDevice(cur);
    return LRQO_OK;
}

}  // extern "C"
