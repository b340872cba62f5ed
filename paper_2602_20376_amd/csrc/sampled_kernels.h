// Fused scoring kernels of the sampled solver (Sec. 4.2): direction
// generation, w = V c, the decision rule and the accumulation of V^H z.
// Internal header, included by sampled.hip (the plain launches) and
// sampled_probe.hip (the same kernels with per-row label output for a few
// probed candidates, for inspection).
//
//   k_score        r > 4: each lane owns CPL directions; the block streams
//                  row tiles of V through LDS (every lane of a wave reads the
//                  same row: an LDS broadcast).
//   k_score_rows   r <= 4: the four waves of a block hold the same 64*CPL
//                  candidates and split the rows of the block's slice;
//                  their sums are added through LDS at the end (fixed order).
//   k_score_bf16   the precision form: w = V c from BF16 MFMAs, rows inside
//                  the BF16 error margin recomputed in FP32.
// With several row slices (gridDim.y > 1) a scorer writes per-slice partial
// sums instead of f.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lrqo_device.h"
#include "sampled_internal.h"

namespace lrqo {
namespace {

constexpr int kBlock = 256;
constexpr int kTile = 256;        // rows per LDS tile

template <int R, bool REAL>
struct Row {
    static constexpr int F = REAL ? R : 2 * R;  // floats per row of V
};

// Label of an FP32 root of unity (cos, sin)(2 pi k / K): the integer nearest
// to K arg / 2 pi.  Only the inspection output uses it.
__device__ __forceinline__ int root_index(float zr, float zi, int K) {
    int k = static_cast<int>(rintf(static_cast<float>(K) * (atan2f(zi, zr) * 0.15915494309189535f)));
    k = k < 0 ? k + K : k;
    return k >= K ? k - K : k;
}

// Candidate directions of one lane (position idx = base + q * stride) and,
// when asked, their FP32 values written once (first row slice, first wave),
// plus the probe slot of each candidate (-1: not probed).
template <int R, int CPL, bool PROBE>
__device__ __forceinline__ void lane_directions(const ScoreParams& p, uint32_t base, uint32_t stride, bool writer,
                                                float (&c)[CPL][2 * R], int (&slot)[CPL]) {
    // generation alone in its loop, so that it unrolls and c stays in registers
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const uint32_t idx = base + q * stride;
        if (idx < p.S) {
            direction_any<R>(p.dirs, p.seed, p.first + idx, p.instance, c[q]);
        } else {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) c[q][j] = 0.0f;
        }
    }
    if (p.dirs_out && writer) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            const uint32_t idx = base + q * stride;
            if (idx < p.S) {
#pragma unroll
                for (int j = 0; j < 2 * R; ++j) p.dirs_out[(size_t)idx * (2 * R) + j] = c[q][j];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        slot[q] = -1;
        if constexpr (PROBE) {
            const uint32_t idx = base + q * stride;
            for (int t = 0; t < p.probe_count; ++t)
                if (idx < p.S && p.probe_idx[t] == idx) slot[q] = t;
        }
    }
}

// ------------------------------------------------------------ fused scorer, r > 4
template <int R, int CPL, bool REAL, int KS, bool PROBE>
__global__ __launch_bounds__(kBlock) void k_score(ScoreParams p) {
    constexpr int RF = Row<R, REAL>::F;
    __shared__ __align__(16) float tile[kTile * RF];
    __shared__ float2 roots_s[KS == 0 ? LRQO_MAX_K : 1];
    const int tid = threadIdx.x;
    if constexpr (KS == 0) {
        for (int k = tid; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
    }

    float c[CPL][2 * R], acc[CPL][2 * R];
    int slot[CPL];
    const uint32_t base = blockIdx.x * (uint32_t)(kBlock * CPL) + tid;
    lane_directions<R, CPL, PROBE>(p, base, kBlock, blockIdx.y == 0, c, slot);
#pragma unroll
    for (int q = 0; q < CPL; ++q)
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) acc[q][j] = 0.0f;

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
                if constexpr (PROBE) {
                    if (slot[q] >= 0) p.probe_out[(size_t)slot[q] * p.n + t0 + i] = (uint16_t)root_index(zr, zi, p.K);
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

// One row (values v) against the lane's candidates; dr[q][j] / di[q][j]
// accumulate the real / imaginary part of s_j (for complex r <= 2 the packed
// form keeps Re V and Im V products apart).  PROBE: probed candidates write
// the row's label at probe_row[slot * n].
template <int R, int CPL, bool REAL, int KS, bool PROBE>
__device__ __forceinline__ void score_vals(const float (&v)[Row<R, REAL>::F],
                                          const float (&c)[CPL][2 * R], const float (&c3)[CPL][2 * R],
                                          int K, const float2* roots, v4f (&dr)[CPL], v4f (&di)[CPL],
                                          const int (&slot)[CPL], uint16_t* probe_row, int64_t n) {
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
        else if constexpr (KS == 8) nearest_root_k8t(wr, wi, zr, zi);
        else nearest_root<KS>(wr, wi, K, roots, zr, zi);
        if constexpr (PROBE) {
            if (slot[q] >= 0) probe_row[(size_t)slot[q] * n] = (uint16_t)root_index(zr, zi, K);
        }
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

template <int R, int CPL, bool REAL, int KS, bool PROBE>
__device__ __forceinline__ void score_row(const float* __restrict__ row, const float (&c)[CPL][2 * R],
                                         const float (&c3)[CPL][2 * R], int K, const float2* roots,
                                         v4f (&dr)[CPL], v4f (&di)[CPL], const int (&slot)[CPL],
                                         uint16_t* probe_row, int64_t n) {
    constexpr int RF = Row<R, REAL>::F;
    float v[RF];
#pragma unroll
    for (int e = 0; e < RF; ++e) v[e] = row[e];
    score_vals<R, CPL, REAL, KS, PROBE>(v, c, c3, K, roots, dr, di, slot, probe_row, n);
}

// Sums of the four waves of a block added in wave order; wave 0 writes f
// (one slice) or the slice's partial sums.
template <int R, int CPL>
__device__ __forceinline__ void block_sums_out(const ScoreParams& p, float (&acc)[CPL][2 * R], uint32_t base,
                                               float (*red)[CPL * 2 * R][kWave], int wave, int lane) {
    constexpr int NW = kBlock / kWave;
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

template <int R, int CPL, bool REAL, int KS, bool PROBE>
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
    int slot[CPL];
    v4f dr[CPL], di[CPL];
    const uint32_t base = blockIdx.x * (uint32_t)(kWave * CPL) + lane;
    lane_directions<R, CPL, PROBE>(p, base, kWave, blockIdx.y == 0 && wave == 0, c, slot);
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        // K = 3 and 8: the real part of w is formed with a pre-scaled c
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) c3[q][j] = re_prescale(KS) * c[q][j];
        dr[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        di[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    }

    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    uint16_t* probe_base = PROBE ? p.probe_out : nullptr;
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, r1 - t0);
        __syncthreads();
        const float* __restrict__ src = p.V + t0 * RF;
        for (int e = tid; e < cnt * RF; e += kBlock) tile[e] = src[e];
        __syncthreads();
        if (cnt == kTile) {
#pragma unroll 4
            for (int ii = 0; ii < kTile / NW; ++ii) {
                const int i = wave + NW * ii;
                score_row<R, CPL, REAL, KS, PROBE>(tile + i * RF, c, c3, p.K, roots_s, dr, di, slot,
                                                   probe_base + t0 + i, p.n);
            }
        } else {
            for (int i = wave; i < cnt; i += NW)
                score_row<R, CPL, REAL, KS, PROBE>(tile + i * RF, c, c3, p.K, roots_s, dr, di, slot,
                                                   probe_base + t0 + i, p.n);
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
    block_sums_out<R, CPL>(p, acc, base, red, wave, lane);
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
// its error bound is recomputed in FP32 on the vector ALU before it is
// labelled; s += conj(V_i) z stays FP32 on the vector ALU.
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __uint_as_float((uint32_t)h << 16);
}

// Bound on |Re w - Re w~| and on |Im w - Im w~| relative to ||V_i|| (unit c):
// each is a dot product of a row of norm ||V_i|| with a unit vector.
template <int SPLIT>
constexpr float bf16_kappa() {
    // SPLIT 1: both operands rounded once (2 u_bf + u_bf^2), u_bf = 2^-9,
    //          plus FP32 accumulation of at most 8 products (8 * 2^-24);
    // SPLIT 2: lo parts rounded (2 * 2^-18), lo*lo dropped (2^-18), FP32
    //          accumulation of 3 x 8 products (24 * 2^-24).
    return SPLIT == 1 ? (0x1p-8f + 0x1p-18f + 8.0f * 0x1p-24f) * 1.01f
                      : (3.0f * 0x1p-18f + 24.0f * 0x1p-24f) * 1.01f;
}

// Nearest root of the BF16-formed w and whether the row must be recomputed
// in FP32.  b = kappa ||V_i|| bounds the error of each of Re w and Im w
// (bf16_kappa).  wr arrives pre-scaled by sqrt(3) for K = 3 (the MFMA's B
// column for Re w is sqrt(3) Re c), so that the K = 3 test needs no multiply.
//   K = 3: t = sqrt(3) Re w - |Im w| decides label 0 (t >= 0); its error is at
//          most sqrt(3)|dRe w| + |dIm w|, i.e. 2b for a real V (the two
//          errors come from one row against Re c and Im c, ||c|| = 1) and
//          (1 + sqrt(3)) b for a complex one; between labels 1 and 2 the sign
//          of Im w decides (error b).  Flag |t| <= that bound or |Im w| <= b.
//   K = 2: the sign of Re w (flag |Re w| <= b).
//   K = 4: the sign of |Re w| - |Im w| (flag |.| <= 2b), then the signs.
//   other: atan2 and the root table; flag when the Euclidean distance to the
//          nearest boundary line is within the bound on |dw| (b for a real V,
//          sqrt(2) b for a complex one).
template <int KS, bool REAL>
__device__ __forceinline__ bool bf16_root(float wr, float wi, float b, int K, const float2* roots, float& zr,
                                          float& zi) {
    if constexpr (KS == 3) {
        constexpr float tb = REAL ? 2.0f : 2.7320508075688772f;
        const float t = wr - fabsf(wi);
        const bool k0 = t >= 0.0f;
        zr = k0 ? 1.0f : -0.5f;
        zi = k0 ? 0.0f : copysignf(0.8660254037844386f, wi);
        return (fabsf(t) <= tb * b) | (fabsf(wi) <= b);
    } else if constexpr (KS == 2) {
        zr = copysignf(1.0f, wr);
        zi = 0.0f;
        return fabsf(wr) <= b;
    } else if constexpr (KS == 4) {
        const float d = fabsf(wr) - fabsf(wi);
        const bool horiz = d >= 0.0f;
        zr = horiz ? copysignf(1.0f, wr) : 0.0f;
        zi = horiz ? 0.0f : copysignf(1.0f, wi);
        return fabsf(d) <= 2.0f * b;
    } else {
        const float x = static_cast<float>(K) * (atan2f(wi, wr) * 0.15915494309189535f) + 0.5f;
        const int k = label_f32_generic(wr, wi, K);
        const float2 r2 = roots[k < K ? k : 0];
        zr = r2.x;
        zi = r2.y;
        const float fr = x - floorf(x);
        const float dist = sqrtf(wr * wr + wi * wi) * __sinf(fminf(fr, 1.0f - fr) * (6.283185307179586f / K)) * 0.999f;
        return dist <= (REAL ? 1.0f : 1.4142136f) * b;
    }
}

// One row's FP32 w for a candidate (the precision form's recompute).
template <int R, bool REAL>
__device__ __forceinline__ void w_f32(const float (&v)[Row<R, REAL>::F], const float (&c)[2 * R], float& wr,
                                      float& wi) {
    wr = 0.0f;
    wi = 0.0f;
    if constexpr (REAL) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            wr = fmaf(v[j], c[2 * j], wr);
            wi = fmaf(v[j], c[2 * j + 1], wi);
        }
    } else {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float vr = v[2 * j], vi = v[2 * j + 1];
            wr = fmaf(vr, c[2 * j], fmaf(-vi, c[2 * j + 1], wr));
            wi = fmaf(vr, c[2 * j + 1], fmaf(vi, c[2 * j], wi));
        }
    }
}

// s += conj(V_i) (zr + i zi) for one row and one candidate.
template <int R, bool REAL>
__device__ __forceinline__ void acc_row(const float (&v)[Row<R, REAL>::F], float zr, float zi, float (&acc)[2 * R]) {
    if constexpr (REAL) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            acc[2 * j] = fmaf(v[j], zr, acc[2 * j]);
            acc[2 * j + 1] = fmaf(v[j], zi, acc[2 * j + 1]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const float vr = v[2 * j], vi = v[2 * j + 1];
            acc[2 * j] = fmaf(vr, zr, fmaf(vi, zi, acc[2 * j]));
            acc[2 * j + 1] = fmaf(vr, zi, fmaf(-vi, zr, acc[2 * j + 1]));
        }
    }
}

template <int R, int CPL, bool REAL, int KS, int SPLIT, bool PROBE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_score_bf16(ScoreParams p) {
    static_assert(R <= 4, "precision form covers r <= 4");
    static_assert(kBlock == kTile, "one thread prepares one row of the tile");
    constexpr int RF = Row<R, REAL>::F;
    constexpr int NCH = (REAL || R <= 2) ? 1 : 2;     // k-chunks of 4
    constexpr int NW = kBlock / kWave;
    constexpr float kappa = bf16_kappa<SPLIT>() * 1.0001f;
    constexpr float s3 = KS == 3 ? 1.7320508075688772f : 1.0f;   // K = 3: Re w pre-scaled
    __shared__ __align__(16) float tile[kTile * RF];
    __shared__ __align__(16) v4s apack[SPLIT][NCH][kTile];
    __shared__ __align__(16) float bound[kTile];
    __shared__ float2 roots_s[KS == 0 ? LRQO_MAX_K : 1];
    __shared__ float red[NW - 1][CPL * 2 * R][kWave];
    __shared__ float cdir[CPL][2 * R][kWave];   // the directions, for the rare FP32 recompute
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if constexpr (KS == 0) {
        for (int k = tid; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
    }

    float acc[CPL][2 * R];
    int slot[CPL];
    v4s bre[SPLIT][CPL][NCH], bim[SPLIT][CPL][NCH];
    const uint32_t base = blockIdx.x * (uint32_t)(kWave * CPL) + lane;
    {
    float c[CPL][2 * R];
    lane_directions<R, CPL, PROBE>(p, base, kWave, blockIdx.y == 0 && wave == 0, c, slot);
    if (wave == 0) {   // every wave holds the same candidates
#pragma unroll
        for (int q = 0; q < CPL; ++q)
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) cdir[q][j][lane] = c[q][j];
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) acc[q][j] = 0.0f;
        // B columns (k-vectors) for the real (times s3) and imaginary part of w
        float br[NCH * 4], bi[NCH * 4];
#pragma unroll
        for (int k = 0; k < NCH * 4; ++k) br[k] = bi[k] = 0.0f;
        if constexpr (REAL) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                br[j] = s3 * c[q][2 * j];
                bi[j] = c[q][2 * j + 1];
            }
        } else if constexpr (R <= 2) {     // A = [Re V_0, Re V_1, Im V_0, Im V_1]
#pragma unroll
            for (int j = 0; j < R; ++j) {
                br[j] = s3 * c[q][2 * j];
                br[2 + j] = -s3 * c[q][2 * j + 1];
                bi[j] = c[q][2 * j + 1];
                bi[2 + j] = c[q][2 * j];
            }
        } else {                           // A1 = Re V, A2 = Im V
#pragma unroll
            for (int j = 0; j < R; ++j) {
                br[j] = s3 * c[q][2 * j];
                br[4 + j] = -s3 * c[q][2 * j + 1];
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
    }   // c leaves the registers: the recompute reads cdir

    unsigned flagged = 0;
    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, r1 - t0);
        __syncthreads();
        const float* __restrict__ src = p.V + t0 * RF;
        for (int e = tid; e < kTile * RF; e += kBlock) tile[e] = e < cnt * RF ? src[e] : 0.0f;
        __syncthreads();
        // A operands (bf16, k-chunks of 4) and the per-component error bound of every row
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
            // the group's four rows and bounds, read once for every candidate
            float v[4][RF];
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int e = 0; e < RF; ++e) v[m][e] = tile[(i0 + m) * RF + e];
            const v4f bnd = *reinterpret_cast<const v4f*>(&bound[i0]);
            // every candidate's w first (24 independent MFMA chains), so that
            // the matrix core runs ahead of the quantiser's VALU work
            v4f wre[CPL], wim[CPL];
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                wre[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
                wim[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    wre[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah[ch], bre[0][q][ch], wre[q], 0, 0, 0);
                    wim[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah[ch], bim[0][q][ch], wim[q], 0, 0, 0);
                    if constexpr (SPLIT == 2) {
                        wre[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah[ch], bre[1][q][ch], wre[q], 0, 0, 0);
                        wre[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(al[ch], bre[0][q][ch], wre[q], 0, 0, 0);
                        wim[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah[ch], bim[1][q][ch], wim[q], 0, 0, 0);
                        wim[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(al[ch], bim[0][q][ch], wim[q], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                // labels from the BF16 values, accumulated at once; a row
                // inside its bound (rare) is fixed up after the group
                float zr[4], zi[4];
                bool fl[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    fl[m] = bf16_root<KS, REAL>(wre[q][m], wim[q][m], bnd[m], p.K, roots_s, zr[m], zi[m]) &&
                            bnd[m] >= 0.0f;
                    acc_row<R, REAL>(v[m], zr[m], zi[m], acc[q]);
                }
                if (__ballot(fl[0] | fl[1] | fl[2] | fl[3])) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        if (fl[m]) {   // FP32 w, its label, s corrected by conj(V_i)(z' - z)
                            ++flagged;
                            float cq[2 * R], wr, wi, nr, ni;
#pragma unroll
                            for (int j = 0; j < 2 * R; ++j) cq[j] = cdir[q][j][lane];
                            w_f32<R, REAL>(v[m], cq, wr, wi);
                            nearest_root<KS>(wr, wi, p.K, roots_s, nr, ni);
                            acc_row<R, REAL>(v[m], nr - zr[m], ni - zi[m], acc[q]);
                            zr[m] = nr;
                            zi[m] = ni;
                        }
                    }
                }
                if constexpr (PROBE) {
                    if (slot[q] >= 0) {
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            if (i0 + m < cnt)
                                p.probe_out[(size_t)slot[q] * p.n + t0 + i0 + m] =
                                    (uint16_t)(root_index(zr[m], zi[m], p.K) | (fl[m] ? 0x100 : 0));
                    }
                }
            }
        }
    }
    // flagged row-candidates: a wave sum, one atomic per wave that has any
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) flagged += __shfl_xor(flagged, off, kWave);
    if (lane == 0 && flagged) atomicAdd(p.flagged, (unsigned long long)flagged);

    block_sums_out<R, CPL>(p, acc, base, red, wave, lane);
}

}  // namespace
}  // namespace lrqo
