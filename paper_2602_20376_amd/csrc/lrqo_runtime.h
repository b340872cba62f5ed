// Host runtime of liblrqo: per-thread stream and error text, per-device
// scratch arena, HIP error checking.  Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "../../include/lrqo.h"

namespace lrqo {

// Sets the calling thread's error text and returns `st`.
lrqo_status fail(lrqo_status st, const std::string& msg);
void clear_error();
hipStream_t current_stream();

// Device scratch: one grow-only arena per device, plus a pinned host block
// for results.  Callers take the device lock for the duration of a solve,
// which serialises solves on one device across host threads.
struct DeviceCtx {
    int device = -1;
    std::mutex mu;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    void* host = nullptr;  // pinned
    size_t host_bytes = 0;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    hipEvent_t ev_score0 = nullptr, ev_score1 = nullptr;  // bracket the scoring kernels
    void* static_scratch = nullptr;  // this device's copy of the allocation-free entry point's array
};

// Context of the current device (created on first use).  nullptr on failure
// (error text set).
DeviceCtx* device_ctx();

// Ensures the arena holds at least `bytes`; the old contents are dropped.
lrqo_status reserve_arena(DeviceCtx* ctx, size_t bytes);
lrqo_status reserve_host(DeviceCtx* ctx, size_t bytes);

// Bump allocator over a reserved block (256-byte alignment).
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    static size_t round(size_t x) { return (x + 255) & ~size_t(255); }
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + off);
        off += round(sizeof(T) * count);
        return p;
    }
};
// Size a carve would need: same rounding.
struct CarveSize {
    size_t bytes = 0;
    template <class T>
    void add(size_t count) { bytes += Carve::round(sizeof(T) * count); }
};

// Is `p` device memory usable on the current device (or managed)?
bool is_device_pointer(const void* p);

}  // namespace lrqo

#define LRQO_HIP(call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::lrqo::fail(LRQO_EDEVICE, std::string(#call " failed: ") +             \
                                                 hipGetErrorString(e_));                    \
    } while (0)

#define LRQO_TRY(expr)                 \
    do {                                \
        lrqo_status s_ = (expr);        \
        if (s_ != LRQO_OK) return s_;   \
    } while (0)
