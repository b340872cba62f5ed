// Internal interfaces of the sampled solver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lrqo.h"

#ifndef LRQO_BF16_SPLIT
#define LRQO_BF16_SPLIT 2      // bf16 hi + lo parts of V and c in the precision form
#endif
#ifndef LRQO_SCORE_CPL
#define LRQO_SCORE_CPL 4       // candidates per lane of the r <= 4 scorers
#endif

namespace lrqo {

constexpr int kMaxProbe = 64;   // probed candidates of one call, at most

// Result block written by the device and copied to pinned host memory.
struct DevResult {
    int64_t best_index;
    double obj;
    double fp32_obj;
    double c[2 * LRQO_MAX_R];
    int32_t nonfinite;
    int32_t pad;
    unsigned long long flagged_rows;
};

struct ScoreParams {
    const float* V;
    int64_t n;
    int K;
    uint64_t seed;
    uint32_t instance;
    uint64_t first;
    uint32_t S;
    int64_t rows_per_slice;
    float* f_out;
    float* partial;
    const float2* roots32;
    unsigned long long* flagged;   // precision form: row-candidates recomputed in FP32
    const float* dirs;             // optional [S][2r] directions in place of the stream
    float* dirs_out;               // optional [S][2r]: the FP32 direction each candidate was scored with
    uint16_t* probe_out;           // [probe_count][n] labels of the probed candidates (| 0x100: recomputed)
    int probe_count;
    uint32_t probe_idx[kMaxProbe]; // positions (0..S-1) of the probed candidates
    const float* vmax;             // [vmax_count] largest |V| entry of each prologue block's share
    int vmax_count;
};

struct RescoreParams {
    const float* V;
    int64_t n;
    int K;
    uint64_t seed;
    uint32_t instance;
    uint64_t first;
    const unsigned long long* keys;
    const double2* roots64;
    double* partial;
    int64_t rows_per_slice;
    const float* dirs;
};

struct SampledJob {
    const float* V;
    int64_t n;
    int r;
    int K;
    int64_t S;
    uint64_t seed;
    uint32_t instance;
    uint64_t first;
    bool real;
    int precision;
    int topk;
    float* f_out;
    const float* dirs;
    float* dirs_out;
    uint16_t* probe_out;
    int probe_count;
    uint32_t probe_idx[kMaxProbe];
    uint8_t* z;
    hipEvent_t ev_score0;   // recorded before / after the scoring kernels
    hipEvent_t ev_score1;
};

struct ScratchPlan {
    int slices = 1;
    int64_t rows_per_slice = 0;
    int topk = 64;
    int rescore_slices = 1;
    int64_t rescore_rows = 0;
    size_t bytes = 0;
};

struct Scratch {
    DevResult* result;
    float2* roots32;
    double2* roots64;
    float* f32;
    float* partial;
    int slices;
    int64_t rows_per_slice;
    int topk;
    unsigned long long* keys_a;
    unsigned long long* keys_b;
    unsigned long long* lists;  // per-wave sorted keys from the slice sum
    double* rescore;
    int rescore_slices;
    int64_t rescore_rows;
    int* bad_blocks;            // [kCheckBlocks] finiteness flags of the prologue's blocks
    float* vmax;                // [kCheckBlocks] largest finite |V| entry of each prologue block's share
};

constexpr int kCheckBlocks = 256;   // blocks of the prologue's finiteness check

void plan_sampled(const SampledJob& job, ScratchPlan& plan);
// The scorers with per-row label output for p.probe_count candidates
// (sampled_probe.hip); same arithmetic as the plain launches.
void launch_score_probe(const ScoreParams& p, dim3 grid, hipStream_t st, int r, bool real, int precision);

// Layout of the precision form's scorer: 0 = both products on MFMA
// (k_score_bf16x; K = 2, 3, 4, other K take 1), 1 = V c on 4x4x4 MFMA tiles
// with V^H z on the vector ALU (k_score_bf16).  LRQO_BF16_FORM = "w4" selects
// 1 (read once per process).
int bf16_form();
lrqo_status launch_sampled(const SampledJob& job, const ScratchPlan& plan, void* arena, hipStream_t st);

}  // namespace lrqo
