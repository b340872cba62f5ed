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
    }
    return LRQO_OK;
}

}  // namespace

extern "C" {

lrqo_status lrqo_solve_sampled_ex(const float* V, int64_t n, int32_t r, int32_t K, int64_t S,
                                  uint64_t seed, const lrqo_sampled_options* opt, uint8_t* z,
                                  lrqo_sampled_result* res) {
    using namespace lrqo;
    clear_error();
    LRQO_TRY(check_sampled_args(V, n, r, K, S, opt, z));
    lrqo_sampled_options o{};
    if (opt) o = *opt;
    if (o.rescore_topk == 0) o.rescore_topk = LRQO_MAX_TOPK;
    if (o.precision == 1 && r > 4) return fail(LRQO_EINVAL, "the precision form (BF16 MFMA) needs r <= 4");

    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    if (!is_device_pointer(V)) return fail(LRQO_EINVAL, "V is not device memory");
    if (!is_device_pointer(z)) return fail(LRQO_EINVAL, "z is not device memory");
    if (o.f_out && !is_device_pointer(o.f_out)) return fail(LRQO_EINVAL, "f_out is not device memory");
    if (o.directions && !is_device_pointer(o.directions))
        return fail(LRQO_EINVAL, "directions is not device memory");

    SampledJob job{};
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
    job.z = z;
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
    if (res) {
        std::memset(res, 0, sizeof *res);
        res->best_index = hres->best_index;
        res->obj = hres->obj;
        res->fp32_obj = hres->fp32_obj;
        for (int j = 0; j < 2 * LRQO_MAX_R; ++j) res->best_c[j] = hres->c[j];
        res->flagged_rows = (int64_t)hres->flagged_rows;
        res->device_ms = ms;
        res->score_ms = score_ms;
        res->rescored = plan.topk;
        res->slices = plan.slices;
    }
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
