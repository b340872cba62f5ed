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
// The precision form's scorer (BF16 MFMA for V c) is in sampled_bf16.h.
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

// Scale B = 2^e of the real K = 3 quantiser, from the largest |V| entry M
// (the prologue's per-block maxima, reduced by each wave): e = 118 -
// floor(log2 M) keeps B |w| below 2^122 for r <= 4 and unit directions, so
// B (|Im w| - sqrt(3) Re w) cannot overflow; it reaches [0, 1) without being
// 0 only for rows whose |w| is below about 2^-95 M (where it stands for a
// tie), and is at least 1 otherwise.  Any B when M is 0 or not finite (the
// call then fails on the finiteness check).
__device__ __forceinline__ float q3_scale(const float* vmax, int count) {
    float m = 0.0f;
    for (int k = (int)(threadIdx.x & (kWave - 1)); k < count; k += kWave) m = fmaxf(m, vmax[k]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    if (!(m > 0.0f) || !isfinite(m)) return 1.0f;
    const int e = min(126, max(-126, 118 - ilogbf(m)));
    return ldexpf(1.0f, e);
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
        if constexpr (REAL && KS == 3) {
            // real V, K = 3: z = 1 - 3/2 q + i (sqrt(3)/2) q sigma with
            // q = [label != 0] and sigma = sign(Im w); dr accumulates
            // sum_i V_i q_i and di sum_i V_i q_i sigma_i, and the caller
            // forms s = sum_i V_i - 3/2 dr + i (sqrt(3)/2) di.  Here
            // wi = B Im w and wr = -B sqrt(3) Re w (B a power of two, see
            // q3_scale), so |wi| + wr = B (|Im w| - sqrt(3) Re w) has the
            // sign of the label test exactly, and clamped to [0, 1] it is q
            // (one add with the clamp modifier); q sigma takes the sign of wi
            const float qf = __builtin_amdgcn_fmed3f(fabsf(wi) + wr, 0.0f, 1.0f);
            const float qs = copysignf(qf, wi);
            if constexpr (PROBE) {
                if (slot[q] >= 0)
                    probe_row[(size_t)slot[q] * n] = (uint16_t)(qf == 0.0f ? 0 : ((__float_as_uint(wi) >> 31) ? 2 : 1));
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                dr[q][j] = fmaf(v[j], qf, dr[q][j]);
                di[q][j] = fmaf(v[j], qs, di[q][j]);
            }
            continue;
        }
        float zr, zi;
        if constexpr (KS == 3) nearest_root_k3s(wr, wi, zr, zi);
        else if constexpr (KS == 8) bisector_k8(wr, wi, zr, zi);     // root turned by e^{-i pi/8}
        else if constexpr (KS == 16) bisector_k16(wr, wi, zr, zi);   // root turned by e^{-i pi/16}
        else nearest_root<KS>(wr, wi, K, roots, zr, zi);
        if constexpr (PROBE) {
            if (slot[q] >= 0) {
                float lr = zr, li = zi;
                if constexpr (KS == 8 || KS == 16) {   // the label of the root itself
                    constexpr float co = KS == 8 ? kCos8 : kCos16, si = KS == 8 ? kSin8 : kSin16;
                    lr = zr * co - zi * si;
                    li = zr * si + zi * co;
                }
                probe_row[(size_t)slot[q] * n] = (uint16_t)root_index(lr, li, K);
            }
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
template <int R, int CPL, bool Q3 = false>
__device__ __forceinline__ void block_sums_out(const ScoreParams& p, float (&acc)[CPL][2 * R], uint32_t base,
                                               float (*red)[CPL * 2 * R][kWave], int wave, int lane,
                                               const float* tsum = nullptr) {
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
    if constexpr (Q3) {   // (sum_i V_i q_i, sum_i V_i q_i sigma_i) -> s (score_vals, real V, K = 3);
                          // tsum[w * R + j]: wave w's share of sum_i V_ij over the slice
        float t[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            t[j] = tsum[j];
#pragma unroll
            for (int w = 1; w < NW; ++w) t[j] += tsum[w * R + j];
        }
#pragma unroll
        for (int q = 0; q < CPL; ++q)
#pragma unroll
            for (int j = 0; j < R; ++j) {
                acc[q][2 * j] = fmaf(-1.5f, acc[q][2 * j], t[j]);
                acc[q][2 * j + 1] *= 0.8660254037844386f;
            }
    }

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
    constexpr bool Q3 = REAL && KS == 3;   // score_vals' real K = 3 form needs sum_i V_i
    __shared__ float tsum[Q3 ? NW * R : 1];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    if constexpr (KS == 0) {
        for (int k = tid; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
        __syncthreads();
    }
    float tp[R];   // Q3: this thread's rows (row tid of every tile) summed
#pragma unroll
    for (int j = 0; j < R; ++j) tp[j] = 0.0f;

    float c[CPL][2 * R], c3[CPL][2 * R];
    int slot[CPL];
    v4f dr[CPL], di[CPL];
    float qscale = 1.0f;
    if constexpr (Q3) qscale = q3_scale(p.vmax, p.vmax_count);
    const uint32_t base = blockIdx.x * (uint32_t)(kWave * CPL) + lane;
    lane_directions<R, CPL, PROBE>(p, base, kWave, blockIdx.y == 0 && wave == 0, c, slot);
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        // K = 3: the real part of w is formed with a pre-scaled c (real V:
        // -B sqrt(3) c, and B c for the imaginary part); K = 8 and 16: w is
        // formed with c turned by e^{-i pi/K} (the stored directions are
        // the unturned ones)
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) c3[q][j] = re_prescale(KS) * c[q][j];
        if constexpr (Q3) {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) {
                c3[q][j] *= -qscale;
                c[q][j] *= qscale;
            }
        }
        if constexpr (KS == 8 || KS == 16) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                turn_direction<KS>(c[q][2 * j], c[q][2 * j + 1]);
                c3[q][2 * j] = c[q][2 * j];
                c3[q][2 * j + 1] = c[q][2 * j + 1];
            }
        }
        dr[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        di[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    }

    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    uint16_t* probe_base = PROBE ? p.probe_out : nullptr;
    // each thread stages RF values of a tile (kTile == kBlock); the next
    // tile's values are loaded into registers while the current one is scored
    static_assert(kTile == kBlock, "one row's worth of values per thread");
    float pre[RF];
    auto fetch = [&](int64_t t0n) {
        const int64_t lim = (min((int64_t)kTile, r1 - t0n)) * RF;
        const float* __restrict__ src = p.V + t0n * RF;
#pragma unroll
        for (int k = 0; k < RF; ++k) {
            const int e = tid + k * kBlock;
            pre[k] = e < lim ? src[e] : 0.0f;
        }
    };
    fetch(r0);
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, r1 - t0);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RF; ++k) tile[tid + k * kBlock] = pre[k];
        __syncthreads();
        if (t0 + kTile < r1) fetch(t0 + kTile);
        if constexpr (Q3) {
            if (tid < cnt) {
#pragma unroll
                for (int j = 0; j < R; ++j) tp[j] += tile[tid * RF + j];
            }
        }
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
    if constexpr (Q3) {   // wave sums of tp, in a fixed order
#pragma unroll
        for (int j = 0; j < R; ++j) {
            float t = tp[j];
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) t += __shfl_xor(t, off, kWave);
            if (lane == 0) tsum[wave * R + j] = t;
        }
    }
    block_sums_out<R, CPL, Q3>(p, acc, base, red, wave, lane, tsum);
}

}  // namespace
}  // namespace lrqo
