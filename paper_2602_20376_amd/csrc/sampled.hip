// Sampled maximisation (Sec. 4.2): fused FP32 scorer over uniform sphere
// directions, top-T selection, FP64 rescore of the T best, label write-out.
//
// Kernels, in launch order:
//   k_prologue      roots of unity and the zeroed result record (block 0);
//                   per block, whether its share of V holds a NaN or an
//                   infinity (k_pick gathers the blocks' flags)
//   k_score*        fused candidate generation + scoring (sampled_kernels.h):
//                   each lane owns CPL directions in registers; row tiles of V
//                   stream through LDS; per row-candidate w = V_i c, the
//                   nearest K-th root of arg(w), s += conj(V_i) z_i.  With
//                   several row slices (gridDim.y > 1) partial sums instead.
//                   The precision form's scorers are in sampled_bf16.h.
//   k_finalize      sums the slice partials in a fixed order -> f = ||s||^2,
//                   and sorts each wave's 64 keys for the selection
//   topk_select     best T packed (f, index) keys (select.hip)
//   k_rescore       FP64 re-evaluation of each kept direction, row-sliced
//   k_pick          FP64 arg-max of the rescored candidates (ties -> lowest index)
//   k_labels        FP64 decision rule of the winner -> uint8 labels
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "lrqo_device.h"
#include "lrqo_runtime.h"
#include "sampled_internal.h"
#include "sampled_kernels.h"
#include "sampled_bf16.h"
#include "select.h"

#ifndef LRQO_SCORE_BLOCKS
#define LRQO_SCORE_BLOCKS 2048
#endif

namespace lrqo {

namespace {

// ------------------------------------------------------------ set-up and checks
// Block 0: roots of unity omega^k = (cos, sin)(2 pi k / K) in FP64 and their
// FP32 roundings, and the zeroed result record.  Every block: whether its
// share of V holds a NaN or an infinity, into bad[blockIdx.x] (so that no
// block writes the record while block 0 clears it; k_pick gathers them), and
// the largest finite |V| entry of the share, into vmax[blockIdx.x] (the real
// K = 3 scorer sizes its quantiser scale from it).
__global__ __launch_bounds__(kBlock) void k_prologue(int K, double2* __restrict__ roots64,
                                                     float2* __restrict__ roots32, DevResult* __restrict__ res,
                                                     const float* __restrict__ V, int64_t count,
                                                     int* __restrict__ bad, float* __restrict__ vmax) {
    __shared__ float wmax[kBlock / kWave];
    if (blockIdx.x == 0) {
        for (int k = threadIdx.x; k < K; k += blockDim.x) {
            double sn, cs;
            sincospi(2.0 * (double)k / (double)K, &sn, &cs);
            roots64[k] = make_double2(cs, sn);
            roots32[k] = make_float2((float)cs, (float)sn);
        }
        if (threadIdx.x == 0) *res = DevResult{};
    }
    bool b = false;
    float m = 0.0f;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float x = V[e];
        const bool fin = isfinite(x);
        b |= !fin;
        m = fin ? fmaxf(m, fabsf(x)) : m;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = m;
    const int any = __syncthreads_or(b);
    if (threadIdx.x == 0) {
        bad[blockIdx.x] = any;
        float mm = 0.0f;
        for (int w = 0; w < kBlock / kWave; ++w) mm = fmaxf(mm, wmax[w]);
        vmax[blockIdx.x] = mm;
    }
}

// Slice sums: f of each candidate from the scorer's per-slice partial sums
// (slices in order, then the components in order).  Each wave also sorts its
// 64 keys across its lanes, so the first top-T pass merges sorted lists.
template <int R>
__global__ __launch_bounds__(kBlock) void k_finalize(const float* __restrict__ partial, int P,
                                                     uint32_t S, float* __restrict__ f_out,
                                                     unsigned long long* __restrict__ lists) {
    constexpr int U = R <= 4 ? 8 : 4;      // slices loaded together
    const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    unsigned long long key = 0;
    if (idx < S) {
        float acc[2 * R];
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) acc[j] = 0.0f;
        int p0 = 0;
        for (; p0 + U <= P; p0 += U) {          // whole groups: every load issued before the adds
            float v[U][2 * R];
#pragma unroll
            for (int q = 0; q < U; ++q)
#pragma unroll
                for (int j = 0; j < 2 * R; ++j) v[q][j] = partial[((size_t)(p0 + q) * (2 * R) + j) * S + idx];
#pragma unroll
            for (int q = 0; q < U; ++q)
#pragma unroll
                for (int j = 0; j < 2 * R; ++j) acc[j] += v[q][j];
        }
        for (; p0 < P; ++p0)
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) acc[j] += partial[((size_t)p0 * (2 * R) + j) * S + idx];
        float f = 0.0f;
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) f = fmaf(acc[j], acc[j], f);
        f_out[idx] = f;
        key = pack_key(f, idx);
    }
    lists[idx] = wave_sort_desc(key, lane);
}

// ------------------------------------------------------------ FP64 rescore
template <int R, bool REAL, int KS>
__global__ __launch_bounds__(kBlock) void k_rescore(RescoreParams p) {
    __shared__ double2 roots_s[LRQO_MAX_K];
    __shared__ double red[kBlock / kWave][2 * R];
    for (int k = threadIdx.x; k < p.K; k += kBlock) roots_s[k] = p.roots64[k];
    __syncthreads();
    const int t = blockIdx.x;
    const uint32_t idx = key_index(p.keys[t]);
    float cf[2 * R];
    direction_any<R>(p.dirs, p.seed, p.first + idx, p.instance, cf);
    double c[2 * R], acc[2 * R];
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
        c[j] = (double)cf[j];
        acc[j] = 0.0;
    }
    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    constexpr int RF = Row<R, REAL>::F;
    // one row's FP64 terms, added to acc
    // (a real V leaves out the products with Im V: half the FP64 work)
    auto add_row = [&](const float (&row)[RF]) {
        double wr = 0.0, wi = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if constexpr (REAL) {
                const double vr = (double)row[j];
                wr += vr * c[2 * j];
                wi += vr * c[2 * j + 1];
            } else {
                const double vr = (double)row[2 * j], vi = (double)row[2 * j + 1];
                wr += vr * c[2 * j] - vi * c[2 * j + 1];
                wi += vr * c[2 * j + 1] + vi * c[2 * j];
            }
        }
        double zr, zi;
        nearest_root64<KS>(wr, wi, p.K, roots_s, zr, zi);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if constexpr (REAL) {
                const double vr = (double)row[j];
                acc[2 * j] += vr * zr;
                acc[2 * j + 1] += vr * zi;
            } else {
                const double vr = (double)row[2 * j], vi = (double)row[2 * j + 1];
                acc[2 * j] += vr * zr + vi * zi;
                acc[2 * j + 1] += vr * zi - vi * zr;
            }
        }
    };
    // four rows' loads in flight; the rows are still added in order
    int64_t i = r0 + threadIdx.x;
    for (; i + 3 * kBlock < r1; i += 4 * kBlock) {
        float rows[4][RF];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < RF; ++e) rows[u][e] = p.V[(i + (int64_t)u * kBlock) * RF + e];
#pragma unroll
        for (int u = 0; u < 4; ++u) add_row(rows[u]);
    }
    for (; i < r1; i += kBlock) {
        float row[RF];
#pragma unroll
        for (int e = 0; e < RF; ++e) row[e] = p.V[i * RF + e];
        add_row(row);
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
        const double s = wave_sum_f64(acc[j]);
        if (lane == 0) red[wave][j] = s;
    }
    __syncthreads();
    if (threadIdx.x < 2 * R) {
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += red[w][threadIdx.x];
        p.partial[((size_t)t * gridDim.y + blockIdx.y) * (2 * R) + threadIdx.x] = s;
    }
}

// Thread (t, j) sums component j of kept candidate t over the slices
// (fixed order, eight loads in flight); lane t of wave 0 forms f_t, and a
// butterfly over the wave takes the FP64 arg-max, ties to the lowest index.
template <int R>
__global__ __launch_bounds__(64 * 2 * R) void k_pick(const double* __restrict__ partial, int T, int P,
                                                     const unsigned long long* __restrict__ keys,
                                                     uint64_t seed, uint32_t instance, uint64_t first,
                                                     const float* dirs, const int* __restrict__ bad, int nbad,
                                                     DevResult* res) {
    __shared__ double comp[64][2 * R];
    const int t = threadIdx.x / (2 * R), j = threadIdx.x % (2 * R);
    if (t < T) {
        const double* src = partial + (size_t)t * P * (2 * R) + j;
        double a = 0.0;
        int q = 0;
        for (; q + 8 <= P; q += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src[(size_t)(q + u) * (2 * R)];
#pragma unroll
            for (int u = 0; u < 8; ++u) a += v[u];
        }
        for (; q < P; ++q) a += src[(size_t)q * (2 * R)];
        comp[t][j] = a;
    }
    int b = 0;                                   // the prologue's finiteness flags
    for (int q = threadIdx.x; q < nbad; q += blockDim.x) b |= bad[q];
    const int any_bad = __syncthreads_or(b);
    if (threadIdx.x >= kWave) return;
    const int lane = threadIdx.x;
    double f = -1.0;
    unsigned long long key = 0ull;
    uint32_t idx = 0xFFFFFFFFu;
    if (lane < T) {
        double s = 0.0;
        for (int jj = 0; jj < 2 * R; ++jj) s += comp[lane][jj] * comp[lane][jj];
        key = keys[lane];
        idx = key_index(key);
        f = s >= 0.0 ? s : -1.0;      // a non-finite score is never picked
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const double fo = __shfl_xor(f, off, kWave);
        const uint32_t io = __shfl_xor(idx, off, kWave);
        const unsigned long long ko = __shfl_xor(key, off, kWave);
        if (fo > f || (fo == f && io < idx)) {
            f = fo;
            idx = io;
            key = ko;
        }
    }
    if (lane != 0) return;
    if (f < 0.0) {  // only with non-finite scores; the host reports the error
        key = keys[0];
        idx = key_index(key);
    }
    float cf[2 * R];
    direction_any<R>(dirs, seed, first + idx, instance, cf);
    res->nonfinite = any_bad ? 1 : 0;
    res->best_index = (int64_t)(first + idx);
    res->obj = f;
    res->fp32_obj = (double)key_value(key);
    for (int jj = 0; jj < 2 * LRQO_MAX_R; ++jj) res->c[jj] = jj < 2 * R ? (double)cf[jj] : 0.0;
}

template <int R, bool REAL>
__global__ __launch_bounds__(kBlock) void k_labels(const float* __restrict__ V, int64_t n, int K,
                                                   const DevResult* __restrict__ res,
                                                   uint8_t* __restrict__ z) {
    constexpr int RF = Row<R, REAL>::F;
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    const float* row = V + i * RF;
    double wr = 0.0, wi = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const double vr = REAL ? (double)row[j] : (double)row[2 * j];
        const double vi = REAL ? 0.0 : (double)row[2 * j + 1];
        wr += vr * res->c[2 * j] - vi * res->c[2 * j + 1];
        wi += vr * res->c[2 * j + 1] + vi * res->c[2 * j];
    }
    z[i] = (uint8_t)label_f64(wr, wi, K);
}

// ------------------------------------------------------------ host driver
// Candidates per lane, and per block (the MFMA scorer's 4 waves share one
// set of 64*CPL candidates; the vector-ALU scorer's 256 lanes hold distinct ones).
int cands_per_lane(int R) { return R <= 4 ? LRQO_SCORE_CPL : 1; }
int cands_per_block(int R) { return R <= 4 ? kWave * cands_per_lane(R) : kBlock * cands_per_lane(R); }
int cands_per_block(const SampledJob& job) {
    const bool mfma = job.precision == 1 && job.r <= 4 && (job.K == 2 || job.K == 3 || job.K == 4) && bf16_form() == 0;
    return mfma ? kBf16xCands : cands_per_block(job.r);
}

template <int R, bool REAL, int KS>
void launch_score(const ScoreParams& p, dim3 grid, hipStream_t st) {
    constexpr int CPL = R <= 4 ? LRQO_SCORE_CPL : 1;
    if constexpr (R <= 4) {
        hipLaunchKernelGGL((k_score_rows<R, CPL, REAL, KS, false>), grid, dim3(kBlock), 0, st, p);
    } else {
        hipLaunchKernelGGL((k_score<R, CPL, REAL, KS, false>), grid, dim3(kBlock), 0, st, p);
    }
}

template <int R, bool REAL, int KS>
void launch_score_bf16(const ScoreParams& p, dim3 grid, hipStream_t st) {
    if constexpr (R <= 4) {
        if constexpr (KS == 2 || KS == 3 || KS == 4) {
            if (bf16_form() == 0) {
                hipLaunchKernelGGL((k_score_bf16x<R, REAL, KS, false>), grid, dim3(kBlock), 0, st, p);
                return;
            }
        }
        hipLaunchKernelGGL((k_score_bf16<R, LRQO_SCORE_CPL, REAL, KS, LRQO_BF16_SPLIT, false>), grid, dim3(kBlock), 0,
                           st, p);
    }
}

template <int R, bool REAL>
void launch_score_k(const ScoreParams& p, dim3 grid, hipStream_t st, int precision) {
    if (p.probe_count > 0) {   // the same scorers with the probed candidates' labels written out
        launch_score_probe(p, grid, st, R, REAL, precision);
        return;
    }
    if (precision == 1) {
        switch (p.K) {
            case 2: launch_score_bf16<R, REAL, 2>(p, grid, st); break;
            case 3: launch_score_bf16<R, REAL, 3>(p, grid, st); break;
            case 4: launch_score_bf16<R, REAL, 4>(p, grid, st); break;
            default: launch_score_bf16<R, REAL, 0>(p, grid, st); break;
        }
        return;
    }
    switch (p.K) {
        case 2: launch_score<R, REAL, 2>(p, grid, st); break;
        case 3: launch_score<R, REAL, 3>(p, grid, st); break;
        case 4: launch_score<R, REAL, 4>(p, grid, st); break;
        case 8: launch_score<R, REAL, 8>(p, grid, st); break;
        case 16: launch_score<R, REAL, 16>(p, grid, st); break;
        default: launch_score<R, REAL, 0>(p, grid, st); break;
    }
}

template <int R, bool REAL>
lrqo_status run_sampled(const SampledJob& job, Scratch& sc, hipStream_t st) {
    const uint32_t S = (uint32_t)job.S;
    const int64_t cand_blocks = ((int64_t)S + cands_per_block(job) - 1) / cands_per_block(job);

    // ---- fused scorer
    ScoreParams p{};
    p.V = job.V;
    p.n = job.n;
    p.K = job.K;
    p.seed = job.seed;
    p.instance = job.instance;
    p.first = job.first;
    p.S = S;
    p.f_out = sc.f32;
    p.partial = sc.partial;
    p.roots32 = sc.roots32;
    p.rows_per_slice = sc.rows_per_slice;
    LRQO_HIP(hipEventRecord(job.ev_score0, st));
    p.flagged = &sc.result->flagged_rows;
    p.dirs = job.dirs;
    p.dirs_out = job.dirs_out;
    p.probe_out = job.probe_out;
    p.probe_count = job.probe_count;
    for (int t = 0; t < job.probe_count; ++t) p.probe_idx[t] = job.probe_idx[t];
    p.vmax = sc.vmax;
    p.vmax_count = kCheckBlocks;
    launch_score_k<R, REAL>(p, dim3((unsigned)cand_blocks, (unsigned)sc.slices), st, job.precision);
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipEventRecord(job.ev_score1, st));
    // ---- top-T
    const int T = sc.topk;
    const unsigned long long* keys = nullptr;
    if (sc.slices > 1) {
        const uint32_t fblocks = (S + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((k_finalize<R>), dim3(fblocks), dim3(kBlock), 0, st, sc.partial, sc.slices, S, sc.f32,
                           sc.lists);
        LRQO_HIP(hipGetLastError());
        LRQO_TRY(topk_select_lists(sc.lists, fblocks * kBlock, T, sc.keys_a, sc.keys_b, st, &keys));
    } else {
        LRQO_TRY(topk_select(sc.f32, S, T, sc.keys_a, sc.keys_b, st, &keys));
    }

    // ---- FP64 rescore of the T kept keys
    RescoreParams rp{};
    rp.V = job.V;
    rp.n = job.n;
    rp.K = job.K;
    rp.seed = job.seed;
    rp.instance = job.instance;
    rp.first = job.first;
    rp.keys = keys;
    rp.roots64 = sc.roots64;
    rp.partial = sc.rescore;
    rp.rows_per_slice = sc.rescore_rows;
    rp.dirs = job.dirs;
    const dim3 rgrid(T, sc.rescore_slices);
    switch (k_special(job.K)) {
        case 2: hipLaunchKernelGGL((k_rescore<R, REAL, 2>), rgrid, dim3(kBlock), 0, st, rp); break;
        case 3: hipLaunchKernelGGL((k_rescore<R, REAL, 3>), rgrid, dim3(kBlock), 0, st, rp); break;
        case 4: hipLaunchKernelGGL((k_rescore<R, REAL, 4>), rgrid, dim3(kBlock), 0, st, rp); break;
        case 8: hipLaunchKernelGGL((k_rescore<R, REAL, 8>), rgrid, dim3(kBlock), 0, st, rp); break;
        case 16: hipLaunchKernelGGL((k_rescore<R, REAL, 16>), rgrid, dim3(kBlock), 0, st, rp); break;
        default: hipLaunchKernelGGL((k_rescore<R, REAL, 0>), rgrid, dim3(kBlock), 0, st, rp); break;
    }
    LRQO_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_pick<R>), dim3(1), dim3(64 * 2 * R), 0, st, sc.rescore, T, sc.rescore_slices, keys,
                       job.seed, job.instance, job.first, job.dirs, sc.bad_blocks, kCheckBlocks, sc.result);
    LRQO_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_labels<R, REAL>), dim3((unsigned)((job.n + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, job.V, job.n, job.K, sc.result, job.z);
    LRQO_HIP(hipGetLastError());
    return LRQO_OK;
}

template <bool REAL>
lrqo_status dispatch_r(const SampledJob& job, Scratch& sc, hipStream_t st) {
    switch (job.r) {
        case 1: return run_sampled<1, REAL>(job, sc, st);
        case 2: return run_sampled<2, REAL>(job, sc, st);
        case 3: return run_sampled<3, REAL>(job, sc, st);
        case 4: return run_sampled<4, REAL>(job, sc, st);
        case 5: return run_sampled<5, REAL>(job, sc, st);
        case 6: return run_sampled<6, REAL>(job, sc, st);
        case 7: return run_sampled<7, REAL>(job, sc, st);
        case 8: return run_sampled<8, REAL>(job, sc, st);
        default: return fail(LRQO_EINVAL, "r out of range");
    }
}

}  // namespace

// Plans the launch shapes and the scratch layout of one sampled solve.
void plan_sampled(const SampledJob& job, ScratchPlan& plan) {
    const int R = job.r;
    const int64_t cand_blocks = (job.S + cands_per_block(job) - 1) / cands_per_block(job);
    // enough blocks to fill 256 CUs several times over, slices of >= 1024 rows
    int64_t slices = std::max<int64_t>(1, (LRQO_SCORE_BLOCKS + cand_blocks - 1) / cand_blocks);
    slices = std::min<int64_t>(slices, std::max<int64_t>(1, job.n / 1024));
    int64_t rows = (job.n + slices - 1) / slices;
    rows = ((rows + 63) / 64) * 64;
    slices = (job.n + rows - 1) / rows;
    plan.slices = (int)slices;
    plan.rows_per_slice = rows;
    plan.topk = (int)std::min<int64_t>(job.topk, job.S);
    int64_t rrows = std::max<int64_t>(4096, (job.n + 127) / 128);
    plan.rescore_rows = rrows;
    plan.rescore_slices = (int)((job.n + rrows - 1) / rrows);
    CarveSize cs;
    cs.add<DevResult>(1);
    cs.add<float2>(LRQO_MAX_K);
    cs.add<double2>(LRQO_MAX_K);
    cs.add<float>(job.f_out ? 0 : job.S);
    cs.add<float>(slices > 1 ? (size_t)slices * 2 * R * job.S : 0);
    cs.add<unsigned long long>(topk_buffer_keys((uint32_t)job.S, plan.topk));
    cs.add<unsigned long long>(topk_buffer_keys((uint32_t)job.S, plan.topk));
    cs.add<unsigned long long>(slices > 1 ? (size_t)(job.S + kBlock - 1) / kBlock * kBlock : 0);
    cs.add<double>((size_t)plan.topk * plan.rescore_slices * 2 * R);
    cs.add<int>(kCheckBlocks);
    cs.add<float>(kCheckBlocks);
    plan.bytes = cs.bytes;
}

lrqo_status launch_sampled(const SampledJob& job, const ScratchPlan& plan, void* arena, hipStream_t st) {
    Carve cv(arena);
    Scratch sc{};
    sc.result = cv.take<DevResult>(1);
    sc.roots32 = cv.take<float2>(LRQO_MAX_K);
    sc.roots64 = cv.take<double2>(LRQO_MAX_K);
    sc.f32 = job.f_out ? job.f_out : cv.take<float>(job.S);
    sc.slices = plan.slices;
    sc.rows_per_slice = plan.rows_per_slice;
    sc.partial = plan.slices > 1 ? cv.take<float>((size_t)plan.slices * 2 * job.r * job.S) : nullptr;
    sc.topk = plan.topk;
    sc.keys_a = cv.take<unsigned long long>(topk_buffer_keys((uint32_t)job.S, plan.topk));
    sc.keys_b = cv.take<unsigned long long>(topk_buffer_keys((uint32_t)job.S, plan.topk));
    sc.lists = plan.slices > 1 ? cv.take<unsigned long long>((size_t)(job.S + kBlock - 1) / kBlock * kBlock)
                               : nullptr;
    sc.rescore_slices = plan.rescore_slices;
    sc.rescore_rows = plan.rescore_rows;
    sc.rescore = cv.take<double>((size_t)plan.topk * plan.rescore_slices * 2 * job.r);

    sc.bad_blocks = cv.take<int>(kCheckBlocks);
    sc.vmax = cv.take<float>(kCheckBlocks);

    const int64_t vcount = job.n * job.r * (job.real ? 1 : 2);
    hipLaunchKernelGGL(k_prologue, dim3(kCheckBlocks), dim3(kBlock), 0, st, job.K, sc.roots64, sc.roots32,
                       sc.result, job.V, vcount, sc.bad_blocks, sc.vmax);
    LRQO_HIP(hipGetLastError());
    return job.real ? dispatch_r<true>(job, sc, st) : dispatch_r<false>(job, sc, st);
}

}  // namespace lrqo
