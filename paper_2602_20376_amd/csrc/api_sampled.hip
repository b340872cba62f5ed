// C-ABI entry points of the sampled solver: argument checks, scratch,
// launch, synchronisation, result delivery.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "lrqo_runtime.h"
#include "sampled_internal.h"

namespace {

lrqo_status check_sampled_args(const float* V, int64_t n, int32_t r, int32_t K, int64_t S,
                               const lrqo_sampled_options* opt, const uint8_t* z) {
    using lrqo::fail;
    if (!V) return fail(LRQO_EINVAL, "V is null");
    if (!z) return fail(LRQO_EINVAL, "z is null");
    if (n < 1 || n > INT32_MAX) return fail(LRQO_EINVAL, "n must be in [1, 2^31-1]");
    if (r < 1 || r > LRQO_MAX_R) return fail(LRQO_EINVAL, "r must be in [1, 8]");
    if (K < 2 || K > LRQO_MAX_K) return fail(LRQO_EINVAL, "K must be in [2, 255]");
    if (S < 1 || S > (int64_t)0xFFFFFFFFll) return fail(LRQO_EINVAL, "S must be in [1, 2^32-1]");
    if (opt) {
        if (opt->real_v != 0 && opt->real_v != 1) return fail(LRQO_EINVAL, "real_v must be 0 or 1");
        if (opt->precision != 0 && opt->precision != 1)
            return fail(LRQO_EINVAL, "precision must be 0 (FP32) or 1 (BF16 MFMA)");
        if (opt->rescore_topk < 0 || opt->rescore_topk > LRQO_MAX_TOPK)
            return fail(LRQO_EINVAL, "rescore_topk must be in [0, 64]");
        if (opt->first_index > UINT64_MAX - (uint64_t)S)
            return fail(LRQO_EINVAL, "first_index + S overflows");
        if (opt->directions && opt->first_index != 0)
            return fail(LRQO_EINVAL, "first_index must be 0 with a direction list");
        if (opt->probe_count < 0 || opt->probe_count > LRQO_MAX_TOPK)
            return fail(LRQO_EINVAL, "probe_count must be in [0, 64]");
        if (opt->probe_count > 0) {
            if (!opt->probe || !opt->probe_labels)
                return fail(LRQO_EINVAL, "probe and probe_labels are needed with probe_count > 0");
            for (int t = 0; t < opt->probe_count; ++t)
                if (opt->probe[t] < 0 || opt->probe[t] >= S)
                    return fail(LRQO_EINVAL, "probe positions must be in [0, S)");
        }
    }
    return LRQO_OK;
}

// Scratch of lrqo_solve_sampled_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes this name to a kernel (on the host it
// is a stand-in, not a device address): the device address comes from
// hipGetSymbolAddress, once per device, and is kept in the device context.
static __device__ __align__(256) char scratch[LRQO_NOALLOC_SCRATCH_BYTES];

lrqo_status static_scratch_ptr(lrqo::DeviceCtx* ctx, void** out) {
    if (!ctx->static_scratch) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return lrqo::fail(LRQO_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                                hipGetErrorString(e));
        ctx->static_scratch = ptr;
    }
    *out = ctx->static_scratch;
    return LRQO_OK;
}

// Arguments of a sampled call as a job, after the checks that need no device.
lrqo_status make_job(const float* V, int64_t n, int32_t r, int32_t K, int64_t S, uint64_t seed,
                     const lrqo_sampled_options* opt, uint8_t* z, lrqo::SampledJob& job) {
    using namespace lrqo;
    LRQO_TRY(check_sampled_args(V, n, r, K, S, opt, z));
    lrqo_sampled_options o{};
    if (opt) o = *opt;
    if (o.rescore_topk == 0) o.rescore_topk = LRQO_MAX_TOPK;
    if (o.precision == 1 && r > 4) return fail(LRQO_EINVAL, "the precision form (BF16 MFMA) needs r <= 4");
    if (!is_device_pointer(V)) return fail(LRQO_EINVAL, "V is not device memory");
    if (!is_device_pointer(z)) return fail(LRQO_EINVAL, "z is not device memory");
    if (o.f_out && !is_device_pointer(o.f_out)) return fail(LRQO_EINVAL, "f_out is not device memory");
    if (o.directions && !is_device_pointer(o.directions))
        return fail(LRQO_EINVAL, "directions is not device memory");
    if (o.dirs_out && !is_device_pointer(o.dirs_out)) return fail(LRQO_EINVAL, "dirs_out is not device memory");
    if (o.probe_count > 0 && !is_device_pointer(o.probe_labels))
        return fail(LRQO_EINVAL, "probe_labels is not device memory");
    job = SampledJob{};
    job.V = V;
    job.n = n;
    job.r = r;
    job.K = K;
    job.S = S;
    job.seed = seed;
    job.instance = o.instance;
    job.first = o.first_index;
    job.real = o.real_v == 1;
    job.precision = o.precision;
    job.topk = o.rescore_topk;
    job.f_out = o.f_out;
    job.dirs = o.directions;
    job.dirs_out = o.dirs_out;
    job.probe_out = o.probe_labels;
    job.probe_count = o.probe_count;
    for (int t = 0; t < o.probe_count; ++t) job.probe_idx[t] = (uint32_t)o.probe[t];
    job.z = z;
    return LRQO_OK;
}

void fill_result(const lrqo::DevResult& h, const lrqo::ScratchPlan& plan, float ms, float score_ms,
                 lrqo_sampled_result* res) {
    if (!res) return;
    std::memset(res, 0, sizeof *res);
    res->best_index = h.best_index;
    res->obj = h.obj;
    res->fp32_obj = h.fp32_obj;
    for (int j = 0; j < 2 * LRQO_MAX_R; ++j) res->best_c[j] = h.c[j];
    res->flagged_rows = (int64_t)h.flagged_rows;
    res->device_ms = ms;
    res->score_ms = score_ms;
    res->rescored = plan.topk;
    res->slices = plan.slices;
}

}  // namespace

extern "C" {

lrqo_status lrqo_solve_sampled_noalloc(const float* V, int64_t n, int32_t r, int32_t K, int64_t S,
                                       uint64_t seed, const lrqo_sampled_options* opt, uint8_t* z,
                                       lrqo_sampled_result* res) {
    using namespace lrqo;
    clear_error();
    LRQO_TRY(check_sampled_args(V, n, r, K, S, opt, z));
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    SampledJob job;
    LRQO_TRY(make_job(V, n, r, K, S, seed, opt, z, job));
    ScratchPlan plan;
    plan_sampled(job, plan);
    if (plan.bytes > (size_t)LRQO_NOALLOC_SCRATCH_BYTES)
        return fail(LRQO_ETOOBIG, "scratch of " + std::to_string(plan.bytes) + " bytes exceeds the " +
                                      std::to_string((size_t)LRQO_NOALLOC_SCRATCH_BYTES) +
                                      "-byte static array of the allocation-free entry point");
    job.ev_score0 = ctx->ev_score0;
    job.ev_score1 = ctx->ev_score1;

    std::lock_guard<std::mutex> lk(ctx->mu);
    void* ptr = nullptr;
    LRQO_TRY(static_scratch_ptr(ctx, &ptr));
    hipStream_t st = current_stream();
    DevResult h{};
    LRQO_HIP(hipEventRecord(ctx->ev_start, st));
    LRQO_TRY(launch_sampled(job, plan, ptr, st));
    // the result block sits first in the scratch (pageable host copy)
    LRQO_HIP(hipMemcpyAsync(&h, ptr, sizeof(DevResult), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipEventRecord(ctx->ev_stop, st));
    LRQO_HIP(hipStreamSynchronize(st));
    float ms = 0.0f, score_ms = 0.0f;
    LRQO_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
    LRQO_HIP(hipEventElapsedTime(&score_ms, ctx->ev_score0, ctx->ev_score1));
    if (h.nonfinite) return fail(LRQO_ENOTFINITE, "V holds a NaN or an infinity");
    fill_result(h, plan, ms, score_ms, res);
    return LRQO_OK;
}

lrqo_status lrqo_solve_sampled_ex(const float* V, int64_t n, int32_t r, int32_t K, int64_t S,
                                  uint64_t seed, const lrqo_sampled_options* opt, uint8_t* z,
                                  lrqo_sampled_result* res) {
    using namespace lrqo;
    clear_error();
    LRQO_TRY(check_sampled_args(V, n, r, K, S, opt, z));
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    SampledJob job;
    LRQO_TRY(make_job(V, n, r, K, S, seed, opt, z, job));
    job.ev_score0 = ctx->ev_score0;
    job.ev_score1 = ctx->ev_score1;

    std::lock_guard<std::mutex> lk(ctx->mu);
    ScratchPlan plan;
    plan_sampled(job, plan);
    LRQO_TRY(reserve_arena(ctx, plan.bytes));
    LRQO_TRY(reserve_host(ctx, sizeof(DevResult)));
    hipStream_t st = current_stream();
    DevResult* hres = static_cast<DevResult*>(ctx->host);

    LRQO_HIP(hipEventRecord(ctx->ev_start, st));
    LRQO_TRY(launch_sampled(job, plan, ctx->arena, st));
    // the result block sits first in the arena
    LRQO_HIP(hipMemcpyAsync(hres, ctx->arena, sizeof(DevResult), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipEventRecord(ctx->ev_stop, st));
    LRQO_HIP(hipStreamSynchronize(st));
    float ms = 0.0f, score_ms = 0.0f;
    LRQO_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
    LRQO_HIP(hipEventElapsedTime(&score_ms, ctx->ev_score0, ctx->ev_score1));

    if (hres->nonfinite) return fail(LRQO_ENOTFINITE, "V holds a NaN or an infinity");
    fill_result(*hres, plan, ms, score_ms, res);
    return LRQO_OK;
}

lrqo_status lrqo_solve_sampled(const float* V, int64_t n, int32_t r, int32_t K, int64_t S,
                               uint64_t seed, uint8_t* z, double* obj) {
    if (!obj) return lrqo::fail(LRQO_EINVAL, "obj is null");
    lrqo_sampled_result res;
    lrqo_status st = lrqo_solve_sampled_ex(V, n, r, K, S, seed, nullptr, z, &res);
    if (st == LRQO_OK) *obj = res.obj;
    return st;
}

}  // extern "C"
