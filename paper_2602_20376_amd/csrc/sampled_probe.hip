// The sampled scorers with per-row label output for a few probed candidates
// (inspection of the decision rule as the scorer applies it).  The kernels
// are those of sampled_kernels.h with PROBE = true: the same arithmetic, plus
// a store of each probed candidate's label for every row.
#include <cstdlib>
#include <cstring>

#include "lrqo_device.h"
#include "sampled_internal.h"
#include "sampled_kernels.h"
#include "sampled_bf16.h"

namespace lrqo {

namespace {

template <int R, bool REAL, int KS>
void probe_fp32(const ScoreParams& p, dim3 grid, hipStream_t st) {
    constexpr int CPL = R <= 4 ? LRQO_SCORE_CPL : 1;
    if constexpr (R <= 4) {
        hipLaunchKernelGGL((k_score_rows<R, CPL, REAL, KS, true>), grid, dim3(kBlock), 0, st, p);
    } else {
        hipLaunchKernelGGL((k_score<R, CPL, REAL, KS, true>), grid, dim3(kBlock), 0, st, p);
    }
}

template <int R, bool REAL, int KS>
void probe_bf16(const ScoreParams& p, dim3 grid, hipStream_t st) {
    if constexpr (R <= 4) {
        if constexpr (KS == 2 || KS == 3 || KS == 4) {
            if (bf16_form() == 0) {
                hipLaunchKernelGGL((k_score_bf16x<R, REAL, KS, true>), grid, dim3(kBlock), 0, st, p);
                return;
            }
        }
        hipLaunchKernelGGL((k_score_bf16<R, LRQO_SCORE_CPL, REAL, KS, LRQO_BF16_SPLIT, true>), grid, dim3(kBlock), 0,
                           st, p);
    }
}

template <int R, bool REAL>
void probe_k(const ScoreParams& p, dim3 grid, hipStream_t st, int precision) {
    if (precision == 1) {
        switch (p.K) {
            case 2: probe_bf16<R, REAL, 2>(p, grid, st); break;
            case 3: probe_bf16<R, REAL, 3>(p, grid, st); break;
            case 4: probe_bf16<R, REAL, 4>(p, grid, st); break;
            default: probe_bf16<R, REAL, 0>(p, grid, st); break;
        }
        return;
    }
    switch (p.K) {
        case 2: probe_fp32<R, REAL, 2>(p, grid, st); break;
        case 3: probe_fp32<R, REAL, 3>(p, grid, st); break;
        case 4: probe_fp32<R, REAL, 4>(p, grid, st); break;
        case 8: probe_fp32<R, REAL, 8>(p, grid, st); break;
        case 16: probe_fp32<R, REAL, 16>(p, grid, st); break;
        default: probe_fp32<R, REAL, 0>(p, grid, st); break;
    }
}

template <bool REAL>
void probe_r(const ScoreParams& p, dim3 grid, hipStream_t st, int r, int precision) {
    switch (r) {
        case 1: probe_k<1, REAL>(p, grid, st, precision); break;
        case 2: probe_k<2, REAL>(p, grid, st, precision); break;
        case 3: probe_k<3, REAL>(p, grid, st, precision); break;
        case 4: probe_k<4, REAL>(p, grid, st, precision); break;
        case 5: probe_k<5, REAL>(p, grid, st, precision); break;
        case 6: probe_k<6, REAL>(p, grid, st, precision); break;
        case 7: probe_k<7, REAL>(p, grid, st, precision); break;
        case 8: probe_k<8, REAL>(p, grid, st, precision); break;
        default: break;
    }
}

}  // namespace

int bf16_form() {
    static const int form = [] {
        const char* e = std::getenv("LRQO_BF16_FORM");
        return e && std::strcmp(e, "w4") == 0 ? 1 : 0;
    }();
    return form;
}

void launch_score_probe(const ScoreParams& p, dim3 grid, hipStream_t st, int r, bool real, int precision) {
    if (real) probe_r<true>(p, grid, st, r, precision);
    else probe_r<false>(p, grid, st, r, precision);
}

}  // namespace lrqo
