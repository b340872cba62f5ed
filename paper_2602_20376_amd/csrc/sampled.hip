// Sampled maximisation (Sec. 4.2): fused FP32 scorer over uniform sphere
// directions, top-T selection, FP64 rescore of the T best, label write-out.
//
// Kernels, in launch order:
//   k_prologue      roots of unity and the zeroed result record (block 0);
//                   per block, whether its share of V holds a NaN or an
//                   infinity (k_pick gathers the blocks' flags)
//   k_score         fused candidate generation + scoring (A1, A3-A6): each
//                   lane owns CPL directions in registers; the block streams
//                   row tiles of V through LDS (every lane of a wave reads the
//                   same row: an LDS broadcast); per row-candidate it forms
//                   w = V_i c, rounds arg(w) to the nearest K-th root and
//                   accumulates s += conj(V_i) z_i.  With several row slices
//                   (gridDim.y > 1) it writes partial sums instead.
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
#include "select.h"

#ifndef LRQO_BF16_SPLIT
#define LRQO_BF16_SPLIT 2
#endif
#ifndef LRQO_SCORE_BLOCKS
#define LRQO_SCORE_BLOCKS 2048
#endif
#ifndef LRQO_SCORE_CPL
#define LRQO_SCORE_CPL 4
#endif

namespace lrqo {

namespace {

constexpr int kBlock = 256;
constexpr int kTile = 256;        // rows per LDS tile

template <int R, bool REAL>
struct Row {
    static constexpr int F = REAL ? R : 2 * R;  // floats per row of V
};

// ------------------------------------------------------------ set-up and checks
// Block 0: roots of unity omega^k = (cos, sin)(2 pi k / K) in FP64 and their
// FP32 roundings, and the zeroed result record.  Every block: whether its
// share of V holds a NaN or an infinity, into bad[blockIdx.x] (so that no
// block writes the record while block 0 clears it; k_pick gathers them).
__global__ __launch_bounds__(kBlock) void k_prologue(int K, double2* __restrict__ roots64,
                                                     float2* __restrict__ roots32, DevResult* __restrict__ res,
                                                     const float* __restrict__ V, int64_t count,
                                                     int* __restrict__ bad) {
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
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        b |= !isfinite(V[e]);
    const int any = __syncthreads_or(b);
    if (threadIdx.x == 0) bad[blockIdx.x] = any;
}

// ------------------------------------------------------------ fused scorer
template <int R, int CPL, bool REAL, int KS>
__global__ __launch_bounds__(kBlock) void k_score(ScoreParams p) {
    constexpr int RF = Row<R, REAL>::F;
    __shared__ __align__(16) float tile[kTile * RF];
    __shared__ float2 roots_s[KS == 0 ? LRQO_MAX_K : 1];
    const int tid = threadIdx.x;
    if constexpr (KS == 0) {
        for (int k = tid; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
    }

    float c[CPL][2 * R], acc[CPL][2 * R];
    const uint32_t base = blockIdx.x * (uint32_t)(kBlock * CPL) + tid;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const uint32_t idx = base + q * kBlock;
        if (idx < p.S) {
            direction_any<R>(p.dirs, p.seed, p.first + idx, p.instance, c[q]);
        } else {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) c[q][j] = 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) acc[q][j] = 0.0f;
    }

    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, r1 - t0);
        __syncthreads();
        const float* __restrict__ src = p.V + t0 * RF;
        for (int e = tid; e < cnt * RF; e += kBlock) tile[e] = src[e];
        __syncthreads();
        for (int i = 0; i < cnt; ++i) {
            float v[RF];
#pragma unroll
            for (int e = 0; e < RF; ++e) v[e] = tile[i * RF + e];
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                float wr = 0.0f, wi = 0.0f;
                if constexpr (REAL) {
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        wr = fmaf(v[j], c[q][2 * j], wr);
                        wi = fmaf(v[j], c[q][2 * j + 1], wi);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const float vr = v[2 * j], vi = v[2 * j + 1];
                        wr = fmaf(vr, c[q][2 * j], fmaf(-vi, c[q][2 * j + 1], wr));
                        wi = fmaf(vr, c[q][2 * j + 1], fmaf(vi, c[q][2 * j], wi));
                    }
                }
                float zr, zi;
                nearest_root<KS>(wr, wi, p.K, roots_s, zr, zi);
                if constexpr (REAL) {
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        acc[q][2 * j] = fmaf(v[j], zr, acc[q][2 * j]);
                        acc[q][2 * j + 1] = fmaf(v[j], zi, acc[q][2 * j + 1]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const float vr = v[2 * j], vi = v[2 * j + 1];
                        // conj(V_ij) z_i
                        acc[q][2 * j] = fmaf(vr, zr, fmaf(vi, zi, acc[q][2 * j]));
                        acc[q][2 * j + 1] = fmaf(vr, zi, fmaf(-vi, zr, acc[q][2 * j + 1]));
                    }
                }
            }
        }
    }

    if (gridDim.y == 1) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const uint32_t idx = base + q * kBlock;
            if (idx < p.S) {
                float f = 0.0f;
#pragma unroll
                for (int j = 0; j < 2 * R; ++j) f = fmaf(acc[q][j], acc[q][j], f);
                p.f_out[idx] = f;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const uint32_t idx = base + q * kBlock;
            if (idx < p.S) {
#pragma unroll
                for (int j = 0; j < 2 * R; ++j)
                    p.partial[((size_t)blockIdx.y * (2 * R) + j) * p.S + idx] = acc[q][j];
            }
        }
    }
}

// ------------------------------------------------------------ fused scorer, r <= 4
// Per row every lane forms w = V_i c and the nearest root z on the vector
// ALU for its CPL candidates and accumulates s += conj(V_i) z.  The four
// waves of a block hold the same 64*CPL candidates and split the rows of the
// block's slice; their partial sums are added through LDS at the end (fixed
// order).  Rows reach the waves as LDS broadcasts of a staged row tile.
typedef float v4f __attribute__((ext_vector_type(4)));

// K = 3 with the real part of w pre-scaled by sqrt(3): label 0 iff
// |Im w| <= sqrt(3) Re w; otherwise the sign of Im w picks omega or omega^2.
__device__ __forceinline__ void nearest_root_k3s(float wr3, float wi, float& zr, float& zi) {
    const bool k0 = fabsf(wi) <= wr3;
    zr = k0 ? 1.0f : -0.5f;
    zi = k0 ? 0.0f : copysignf(0.8660254037844386f, wi);
}

// One row (values v, in registers or SGPRs) against the lane's candidates;
// dr[q][j] / di[q][j] accumulate the real / imaginary part of s_j (for
// complex r <= 2 the packed form keeps Re V and Im V products apart).
template <int R, int CPL, bool REAL, int KS>
__device__ __forceinline__ void score_vals(const float (&v)[Row<R, REAL>::F],
                                          const float (&c)[CPL][2 * R], const float (&c3)[CPL][2 * R],
                                          int K, const float2* roots, v4f (&dr)[CPL], v4f (&di)[CPL]) {
    constexpr bool PACK = !REAL && R <= 2;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        float wr = 0.0f, wi = 0.0f;
        if constexpr (REAL) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                wr = fmaf(v[j], c3[q][2 * j], wr);
                wi = fmaf(v[j], c[q][2 * j + 1], wi);
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const float vr = v[2 * j], vi = v[2 * j + 1];
                wr = fmaf(vr, c3[q][2 * j], fmaf(-vi, c3[q][2 * j + 1], wr));
                wi = fmaf(vr, c[q][2 * j + 1], fmaf(vi, c[q][2 * j], wi));
            }
        }
        float zr, zi;
        if constexpr (KS == 3) nearest_root_k3s(wr, wi, zr, zi);
        else nearest_root<KS>(wr, wi, K, roots, zr, zi);
        if constexpr (REAL) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                dr[q][j] = fmaf(v[j], zr, dr[q][j]);
                di[q][j] = fmaf(v[j], zi, di[q][j]);
            }
        } else if constexpr (PACK) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const float vr = v[2 * j], vi = v[2 * j + 1];
                dr[q][j] = fmaf(vr, zr, dr[q][j]);
                dr[q][2 + j] = fmaf(vi, zr, dr[q][2 + j]);
                di[q][j] = fmaf(vr, zi, di[q][j]);
                di[q][2 + j] = fmaf(vi, zi, di[q][2 + j]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const float vr = v[2 * j], vi = v[2 * j + 1];
                dr[q][j] = fmaf(vr, zr, fmaf(vi, zi, dr[q][j]));
                di[q][j] = fmaf(vr, zi, fmaf(-vi, zr, di[q][j]));
            }
        }
    }
}

template <int R, int CPL, bool REAL, int KS>
__device__ __forceinline__ void score_row(const float* __restrict__ row, const float (&c)[CPL][2 * R],
                                         const float (&c3)[CPL][2 * R], int K, const float2* roots,
                                         v4f (&dr)[CPL], v4f (&di)[CPL]) {
    constexpr int RF = Row<R, REAL>::F;
    float v[RF];
#pragma unroll
    for (int e = 0; e < RF; ++e) v[e] = row[e];
    score_vals<R, CPL, REAL, KS>(v, c, c3, K, roots, dr, di);
}

template <int R, int CPL, bool REAL, int KS>
__global__ __launch_bounds__(kBlock) void k_score_rows(ScoreParams p) {
    static_assert(R <= 4, "the packed accumulators hold r <= 4");
    constexpr int RF = Row<R, REAL>::F;
    constexpr bool PACK = !REAL && R <= 2;
    constexpr int NW = kBlock / kWave;
    __shared__ __align__(16) float tile[kTile * RF];
    __shared__ float2 roots_s[KS == 0 ? LRQO_MAX_K : 1];
    __shared__ float red[NW - 1][CPL * 2 * R][kWave];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if constexpr (KS == 0) {
        for (int k = tid; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
        __syncthreads();
    }

    float c[CPL][2 * R], c3[CPL][2 * R];
    v4f dr[CPL], di[CPL];
    const uint32_t base = blockIdx.x * (uint32_t)(kWave * CPL) + lane;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const uint32_t idx = base + q * kWave;
        if (idx < p.S) {
            direction_any<R>(p.dirs, p.seed, p.first + idx, p.instance, c[q]);
        } else {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) c[q][j] = 0.0f;
        }
        // K = 3: the real part of w is formed with sqrt(3) c
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) c3[q][j] = (KS == 3) ? 1.7320508075688772f * c[q][j] : c[q][j];
        dr[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        di[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    }

    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, r1 - t0);
        __syncthreads();
        const float* __restrict__ src = p.V + t0 * RF;
        for (int e = tid; e < cnt * RF; e += kBlock) tile[e] = src[e];
        __syncthreads();
        if (cnt == kTile) {
#pragma unroll 4
            for (int ii = 0; ii < kTile / NW; ++ii)
                score_row<R, CPL, REAL, KS>(tile + (wave + NW * ii) * RF, c, c3, p.K, roots_s, dr, di);
        } else {
            for (int i = wave; i < cnt; i += NW)
                score_row<R, CPL, REAL, KS>(tile + i * RF, c, c3, p.K, roots_s, dr, di);
        }
    }

    // per-lane sums s_j (re, im) of this lane's candidates, then across waves
    float acc[CPL][2 * R];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if constexpr (PACK) {
                // dr = [Re V zr, Im V zr], di = [Re V zi, Im V zi] per column
                acc[q][2 * j] = dr[q][j] + di[q][2 + j];       // Re: Re V zr + Im V zi
                acc[q][2 * j + 1] = di[q][j] - dr[q][2 + j];   // Im: Re V zi - Im V zr
            } else {
                acc[q][2 * j] = dr[q][j];
                acc[q][2 * j + 1] = di[q][j];
            }
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int q = 0; q < CPL; ++q)
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) red[wave - 1][q * 2 * R + j][lane] = acc[q][j];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < NW - 1; ++w)
#pragma unroll
        for (int q = 0; q < CPL; ++q)
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) acc[q][j] += red[w][q * 2 * R + j][lane];

    if (gridDim.y == 1) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const uint32_t idx = base + q * kWave;
            if (idx < p.S) {
                float f = 0.0f;
#pragma unroll
                for (int j = 0; j < 2 * R; ++j) f = fmaf(acc[q][j], acc[q][j], f);
                p.f_out[idx] = f;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const uint32_t idx = base + q * kWave;
            if (idx < p.S) {
#pragma unroll
                for (int j = 0; j < 2 * R; ++j)
                    p.partial[((size_t)blockIdx.y * (2 * R) + j) * p.S + idx] = acc[q][j];
            }
        }
    }
}

// ------------------------------------------------------------ precision form (BF16 MFMA for V c)
// For r <= 4.  w = V_i c comes from v_mfma_f32_4x4x4bf16_1k: block b holds
// lanes 4b..4b+3; lane 4b+m supplies row m of A (4 bf16 along k), lane 4b+n
// supplies column n of B (4 bf16 along k) and register m of lane 4b+n gets
// sum_k A[m][k] B[k][n].  A = four consecutive rows of V (k = component of the
// row), B = the lane's own direction, so register m is w of row m for the
// lane's own candidate.  With SPLIT = 2, V and c are written as hi + lo bf16
// pairs and hi*hi + hi*lo + lo*hi is accumulated (about 16 bits of mantissa).
// Every row whose distance to the nearest decision-boundary line is not above
// its error bound kappa ||V_i|| is recomputed in FP32 on the vector ALU
// before it is labelled; s += conj(V_i) z stays FP32 on the vector ALU.
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __uint_as_float((uint32_t)h << 16);
}

// Relative error bound of the BF16 products plus FP32 accumulation (unit c).
template <int SPLIT>
constexpr float bf16_kappa() {
    // SPLIT 1: both operands rounded once (2 u_bf + u_bf^2), u_bf = 2^-9,
    //          plus FP32 accumulation of at most 8 products (8 * 2^-24);
    // SPLIT 2: lo parts rounded (2 * 2^-18), lo*lo dropped (2^-18), FP32
    //          accumulation of 3 x 8 products (24 * 2^-24).
    return SPLIT == 1 ? (0x1p-8f + 0x1p-18f + 8.0f * 0x1p-24f) * 1.01f
                      : (3.0f * 0x1p-18f + 24.0f * 0x1p-24f) * 1.01f;
}

// Distance from w to the nearest decision-boundary line, and the nearest root.
template <int KS>
__device__ __forceinline__ float root_and_margin(float wr, float wi, int K, const float2* roots,
                                                 float& zr, float& zi) {
    if constexpr (KS == 3) {
        const float t = fmaf(1.7320508075688772f, wr, -fabsf(wi));
        const bool k0 = t >= 0.0f;
        zr = k0 ? 1.0f : -0.5f;
        zi = k0 ? 0.0f : copysignf(0.8660254037844386f, wi);
        return k0 ? 0.5f * t : fminf(-0.5f * t, fabsf(wi));
    } else if constexpr (KS == 2) {
        zr = copysignf(1.0f, wr);
        zi = 0.0f;
        return fabsf(wr);
    } else if constexpr (KS == 4) {
        const bool horiz = fabsf(wr) >= fabsf(wi);
        zr = horiz ? copysignf(1.0f, wr) : 0.0f;
        zi = horiz ? 0.0f : copysignf(1.0f, wi);
        return fabsf(fabsf(wr) - fabsf(wi)) * 0.70710678118654752f;
    } else {
        const float x = static_cast<float>(K) * (atan2f(wi, wr) * 0.15915494309189535f) + 0.5f;
        const int k = label_f32_generic(wr, wi, K);
        const float2 t = roots[k < K ? k : 0];
        zr = t.x;
        zi = t.y;
        const float fr = x - floorf(x);
        const float d = fminf(fr, 1.0f - fr) * (6.283185307179586f / static_cast<float>(K));
        return sqrtf(wr * wr + wi * wi) * __sinf(d) * 0.999f;
    }
}

template <int R, int CPL, bool REAL, int KS, int SPLIT>
__global__ __launch_bounds__(kBlock) void k_score_bf16(ScoreParams p) {
    static_assert(R <= 4, "precision form covers r <= 4");
    static_assert(kBlock == kTile, "one thread prepares one row of the tile");
    constexpr int RF = Row<R, REAL>::F;
    constexpr int NCH = (REAL || R <= 2) ? 1 : 2;     // k-chunks of 4
    constexpr int NW = kBlock / kWave;
    constexpr float kappa = bf16_kappa<SPLIT>();
    __shared__ __align__(16) float tile[kTile * RF];
    __shared__ __align__(16) v4s apack[SPLIT][NCH][kTile];
    __shared__ float bound[kTile];
    __shared__ float2 roots_s[KS == 0 ? LRQO_MAX_K : 1];
    __shared__ float red[NW - 1][CPL * 2 * R][kWave];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if constexpr (KS == 0) {
        for (int k = tid; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
    }

    float c[CPL][2 * R], acc[CPL][2 * R];
    v4s bre[SPLIT][CPL][NCH], bim[SPLIT][CPL][NCH];
    const uint32_t base = blockIdx.x * (uint32_t)(kWave * CPL) + lane;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const uint32_t idx = base + q * kWave;
        if (idx < p.S) {
            direction_any<R>(p.dirs, p.seed, p.first + idx, p.instance, c[q]);
        } else {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) c[q][j] = 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) acc[q][j] = 0.0f;
        // B columns (k-vectors) for the real and imaginary part of w
        float br[NCH * 4], bi[NCH * 4];
#pragma unroll
        for (int k = 0; k < NCH * 4; ++k) br[k] = bi[k] = 0.0f;
        if constexpr (REAL) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                br[j] = c[q][2 * j];
                bi[j] = c[q][2 * j + 1];
            }
        } else if constexpr (R <= 2) {     // A = [Re V_0, Re V_1, Im V_0, Im V_1]
#pragma unroll
            for (int j = 0; j < R; ++j) {
                br[j] = c[q][2 * j];
                br[2 + j] = -c[q][2 * j + 1];
                bi[j] = c[q][2 * j + 1];
                bi[2 + j] = c[q][2 * j];
            }
        } else {                           // A1 = Re V, A2 = Im V
#pragma unroll
            for (int j = 0; j < R; ++j) {
                br[j] = c[q][2 * j];
                br[4 + j] = -c[q][2 * j + 1];
                bi[j] = c[q][2 * j + 1];
                bi[4 + j] = c[q][2 * j];
            }
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const unsigned short hr = bf16_rne(br[4 * ch + k]), hi = bf16_rne(bi[4 * ch + k]);
                bre[0][q][ch][k] = (short)hr;
                bim[0][q][ch][k] = (short)hi;
                if constexpr (SPLIT == 2) {
                    bre[SPLIT - 1][q][ch][k] = (short)bf16_rne(br[4 * ch + k] - bf16_to_f32(hr));
                    bim[SPLIT - 1][q][ch][k] = (short)bf16_rne(bi[4 * ch + k] - bf16_to_f32(hi));
                }
            }
        }
    }

    unsigned flagged = 0;
    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, r1 - t0);
        __syncthreads();
        const float* __restrict__ src = p.V + t0 * RF;
        for (int e = tid; e < kTile * RF; e += kBlock) tile[e] = e < cnt * RF ? src[e] : 0.0f;
        __syncthreads();
        // A operands (bf16, k-chunks of 4) and the error bound of every row
        {
            const int i = tid;    // kBlock == kTile
            float a[NCH * 4];
#pragma unroll
            for (int k = 0; k < NCH * 4; ++k) a[k] = 0.0f;
            float nrm2 = 0.0f;
            if constexpr (REAL) {
#pragma unroll
                for (int j = 0; j < R; ++j) a[j] = tile[i * RF + j];
            } else if constexpr (R <= 2) {
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    a[j] = tile[i * RF + 2 * j];
                    a[2 + j] = tile[i * RF + 2 * j + 1];
                }
            } else {
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    a[j] = tile[i * RF + 2 * j];
                    a[4 + j] = tile[i * RF + 2 * j + 1];
                }
            }
#pragma unroll
            for (int k = 0; k < NCH * 4; ++k) nrm2 = fmaf(a[k], a[k], nrm2);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                v4s h, l;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const unsigned short hb = bf16_rne(a[4 * ch + k]);
                    h[k] = (short)hb;
                    l[k] = (short)bf16_rne(a[4 * ch + k] - bf16_to_f32(hb));
                }
                apack[0][ch][i] = h;
                if constexpr (SPLIT == 2) apack[SPLIT - 1][ch][i] = l;
            }
            // padding rows beyond the tile end and zero rows (they add
            // nothing to s whatever their label) are never flagged
            bound[i] = (i < cnt && nrm2 > 0.0f) ? kappa * sqrtf(nrm2) : -1.0f;
        }
        __syncthreads();
        const int groups = (cnt + 3) / 4;
        for (int g = wave; g < groups; g += NW) {
            const int i0 = 4 * g;
            v4s ah[NCH], al[NCH];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                ah[ch] = apack[0][ch][i0 + (lane & 3)];
                if constexpr (SPLIT == 2) al[ch] = apack[SPLIT - 1][ch][i0 + (lane & 3)];
            }
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                v4f wre = {0.0f, 0.0f, 0.0f, 0.0f}, wim = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    wre = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah[ch], bre[0][q][ch], wre, 0, 0, 0);
                    wim = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah[ch], bim[0][q][ch], wim, 0, 0, 0);
                    if constexpr (SPLIT == 2) {
                        wre = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah[ch], bre[1][q][ch], wre, 0, 0, 0);
                        wre = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(al[ch], bre[0][q][ch], wre, 0, 0, 0);
                        wim = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah[ch], bim[1][q][ch], wim, 0, 0, 0);
                        wim = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(al[ch], bim[0][q][ch], wim, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int i = i0 + m;
                    float zr, zi;
                    const float margin = root_and_margin<KS>(wre[m], wim[m], p.K, roots_s, zr, zi);
                    const bool flag = margin <= bound[i];
                    const unsigned long long bal = __ballot(flag);
                    float v[RF];
#pragma unroll
                    for (int e = 0; e < RF; ++e) v[e] = tile[i * RF + e];
                    if (bal) {
                        flagged += (unsigned)__popcll(bal);
                        if (flag) {   // FP32 recompute of w for this row-candidate
                            float wr = 0.0f, wi = 0.0f;
                            if constexpr (REAL) {
#pragma unroll
                                for (int j = 0; j < R; ++j) {
                                    wr = fmaf(v[j], c[q][2 * j], wr);
                                    wi = fmaf(v[j], c[q][2 * j + 1], wi);
                                }
                            } else {
#pragma unroll
                                for (int j = 0; j < R; ++j) {
                                    const float vr = v[2 * j], vi = v[2 * j + 1];
                                    wr = fmaf(vr, c[q][2 * j], fmaf(-vi, c[q][2 * j + 1], wr));
                                    wi = fmaf(vr, c[q][2 * j + 1], fmaf(vi, c[q][2 * j], wi));
                                }
                            }
                            nearest_root<KS>(wr, wi, p.K, roots_s, zr, zi);
                        }
                    }
                    if constexpr (REAL) {
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            acc[q][2 * j] = fmaf(v[j], zr, acc[q][2 * j]);
                            acc[q][2 * j + 1] = fmaf(v[j], zi, acc[q][2 * j + 1]);
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            const float vr = v[2 * j], vi = v[2 * j + 1];
                            acc[q][2 * j] = fmaf(vr, zr, fmaf(vi, zi, acc[q][2 * j]));
                            acc[q][2 * j + 1] = fmaf(vr, zi, fmaf(-vi, zr, acc[q][2 * j + 1]));
                        }
                    }
                }
            }
        }
    }
    if (lane == 0 && flagged) atomicAdd(p.flagged, (unsigned long long)flagged);

    if (wave > 0) {
#pragma unroll
        for (int q = 0; q < CPL; ++q)
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) red[wave - 1][q * 2 * R + j][lane] = acc[q][j];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < NW - 1; ++w)
#pragma unroll
        for (int q = 0; q < CPL; ++q)
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) acc[q][j] += red[w][q * 2 * R + j][lane];

    if (gridDim.y == 1) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const uint32_t idx = base + q * kWave;
            if (idx < p.S) {
                float f = 0.0f;
#pragma unroll
                for (int j = 0; j < 2 * R; ++j) f = fmaf(acc[q][j], acc[q][j], f);
                p.f_out[idx] = f;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const uint32_t idx = base + q * kWave;
            if (idx < p.S) {
#pragma unroll
                for (int j = 0; j < 2 * R; ++j)
                    p.partial[((size_t)blockIdx.y * (2 * R) + j) * p.S + idx] = acc[q][j];
            }
        }
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

template <int R, bool REAL, int KS>
void launch_score(const ScoreParams& p, dim3 grid, hipStream_t st) {
    constexpr int CPL = R <= 4 ? LRQO_SCORE_CPL : 1;
    if constexpr (R <= 4) {
        hipLaunchKernelGGL((k_score_rows<R, CPL, REAL, KS>), grid, dim3(kBlock), 0, st, p);
    } else {
        hipLaunchKernelGGL((k_score<R, CPL, REAL, KS>), grid, dim3(kBlock), 0, st, p);
    }
}

template <int R, bool REAL, int KS>
void launch_score_bf16(const ScoreParams& p, dim3 grid, hipStream_t st) {
    if constexpr (R <= 4) {
        constexpr int CPL = LRQO_SCORE_CPL;
        hipLaunchKernelGGL((k_score_bf16<R, CPL, REAL, KS, LRQO_BF16_SPLIT>), grid, dim3(kBlock), 0, st, p);
    }
}

template <int R, bool REAL>
void launch_score_k(const ScoreParams& p, dim3 grid, hipStream_t st, int precision) {
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
    const int64_t cand_blocks = ((int64_t)S + cands_per_block(R) - 1) / cands_per_block(R);

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
    const int64_t cand_blocks = (job.S + cands_per_block(R) - 1) / cands_per_block(R);
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

    const int64_t vcount = job.n * job.r * (job.real ? 1 : 2);
    hipLaunchKernelGGL(k_prologue, dim3(kCheckBlocks), dim3(kBlock), 0, st, job.K, sc.roots64, sc.roots32,
                       sc.result, job.V, vcount, sc.bad_blocks);
    LRQO_HIP(hipGetLastError());
    return job.real ? dispatch_r<true>(job, sc, st) : dispatch_r<false>(job, sc, st);
}

}  // namespace lrqo
