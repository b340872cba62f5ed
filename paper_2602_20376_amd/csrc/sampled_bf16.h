// The precision form's fused scorers.  K = 2, 3, 4: k_score_bf16x, both
// w = V c and s = V^H z on BF16 MFMA from three-part splits (FP32-grade w,
// no recompute).  Other K: k_score_bf16, w = V c on BF16 MFMA from hi + lo
// parts, rows inside the BF16 error margin recomputed in FP32, V^H z
// accumulated in FP32 on the vector ALU.  Internal header, included after
// sampled_kernels.h by sampled.hip and sampled_probe.hip.
#pragma once

#include "sampled_kernels.h"

namespace lrqo {
namespace {

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
// each is a dot product of a row of norm ||V_i|| with a unit vector.  BF16
// keeps 8 significant bits, so rounding to it errs by at most u_bf = 2^-8
// relative.  SPLIT 1: both operands rounded once (2 u_bf + u_bf^2).  SPLIT 2:
// x = hi + lo + e with |e| <= u_bf^2 |x| = 2^-16 |x| for both operands, and
// lo*lo is dropped: 3 * 2^-16.  Products of BF16 values are exact in FP32;
// their sum (at most 3 x 8 products and the accumulator) is charged one FP32
// ulp (2^-23) per addition, which also covers an adder that truncates.
template <int SPLIT>
constexpr float bf16_kappa() {
    return SPLIT == 1 ? (0x1p-7f + 0x1p-16f + 9.0f * 0x1p-23f) * 1.01f
                      : (3.0f * 0x1p-16f + 25.0f * 0x1p-23f) * 1.01f;
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

namespace lrqo {
namespace {

// ------------------------------------------------------------ precision form, both products on MFMA
// For K = 2, 3, 4 and r <= 4.  V and c enter as three BF16 parts each (hi,
// mid, lo: an FP32 value is their sum to within 2^-24 of itself), and w is
// formed from the six products of order up to 2^-16,
//   hi.hi + mid.hi + hi.mid + lo.hi + hi.lo + mid.mid,
// so w carries FP32-grade error (the dropped products are of order 2^-24).
// The labels are taken from w directly, with no recomputation: away from a
// decision boundary they are the FP64 rule's.  Every K-th root has
// coordinates in {0, +-1, -1/2} once Im z is divided by sqrt(3)/2 for K = 3,
// so the labels are exact in BF16 and s = V^H z runs on the matrix core too.
//
// Both products are v_mfma_f32_16x16x32_bf16 (gfx950 layout: lane l supplies
// row (A) / column (B) l % 16 and k-slots 8 (l / 16) .. + 7; register g of the
// result is row 4 (l / 16) + g, column l % 16).  A wave holds 32 candidates
// (two column halves n) and takes the rows of a tile 32 at a time (two
// 16-row blocks b).
//   w: for each (n, b) and part (Re w, Im w), the 16 rows x 16 candidates with
//      the C components (C = r for a real V; 2r for a complex one, Re V then
//      Im V) times the six products on k: slot kappa = tau C + x holds
//      product tau of component x (one instruction when 6C <= 32).
//   s: D_r += A2 Z_r and D_i += A2 Z_i: A2 row m = p C + x holds part p of
//      component x of the rows; k-slot (G, t) is row 16 (t / 4) + 4 G + t % 4
//      of the 32, which is where lane l (G = l / 16) holds the labels it
//      computed (block t / 4, register t % 4), so they go into the second
//      product without leaving their lanes.  D stays in registers for the
//      whole slice; each candidate's parts are added once at the end.
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int R, bool REAL>
struct Split16 {
    static constexpr int C = REAL ? R : 2 * R;      // values per row
    static constexpr int N = 6 * C;                 // k-slots of the split product
    static constexpr int NCH = (N + 31) / 32;       // chunks of 32 slots
    static constexpr int NMB = (3 * C + 15) / 16;   // 16-row blocks of A2
};
// The parts (0 hi, 1 mid, 2 lo) of V and of c in product tau.
__host__ __device__ constexpr int part_v(int tau) { return tau == 1 || tau == 5 ? 1 : (tau == 3 ? 2 : 0); }
__host__ __device__ constexpr int part_c(int tau) { return tau == 2 || tau == 5 ? 1 : (tau == 4 ? 2 : 0); }

__device__ __forceinline__ v8bf as_bf(v8s x) { return __builtin_bit_cast(v8bf, x); }

// Candidates per block (four waves of 32).
constexpr int kBf16xCands = (kBlock / kWave) * 32;

// Upper halves of two FP32 values in one dword (first in the low half), and
// their sign bits spread over the halves (v_perm_b32 selectors 9 and 11
// replicate the top bit of bytes 3 and 7).
__device__ __forceinline__ uint32_t hi_pair(float lo, float hi) {
    return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
}
__device__ __forceinline__ uint32_t sign_pair(float lo, float hi) {
    return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x0B0B0909u);
}

// Three BF16 parts of x: hi = rn(x), mid = rn(x - hi), lo = rn(x - hi - mid)
// (both differences exact in FP32).
__device__ __forceinline__ void bf16_split3(float x, unsigned short (&pt)[3]) {
    pt[0] = bf16_rne(x);
    const float r1 = x - bf16_to_f32(pt[0]);
    pt[1] = bf16_rne(r1);
    pt[2] = bf16_rne(r1 - bf16_to_f32(pt[1]));
}

template <int R, bool REAL, int KS, bool PROBE>
__global__ __launch_bounds__(kBlock) void k_score_bf16x(ScoreParams p) {
    static_assert(R <= 4, "precision form covers r <= 4");
    static_assert(KS == 2 || KS == 3 || KS == 4, "labels exact in BF16 for K = 2, 3, 4");
    static_assert(kBlock == kTile, "one thread prepares one row of the tile");
    using SP = Split16<R, REAL>;
    constexpr int RF = Row<R, REAL>::F;
    constexpr int C = SP::C, NCH = SP::NCH, NMB = SP::NMB;
    constexpr bool IM = KS != 2;    // K = 2: neither Im w nor Im z is needed
    // The quantiser's test value u: K = 3 u = sqrt(3) Re w - |Im w| (label 0
    // iff u >= 0, else the sign of Im w), with Re w taken from sqrt(3) c;
    // K = 4 u = |Re w| - |Im w| (a horizontal root iff u >= 0, its sign from
    // Re w, else from Im w); K = 2 u = Re w.
    constexpr float s3 = re_prescale(KS);
    constexpr float zs = KS == 3 ? 0.8660254037844386f : 1.0f;   // Im z = zs * (packed Im label)
    __shared__ __align__(16) v8s apk[NCH][kTile / 16][16][4];
    __shared__ __align__(16) unsigned short a2s[kTile / 32][16 * NMB][4][8];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int G = lane >> 4, col = lane & 15;
    {   // A2 rows 3C.. stay zero
        unsigned short* z = &a2s[0][0][0][0];
        for (int e = tid; e < (kTile / 32) * 16 * NMB * 32; e += kBlock) z[e] = 0;
    }

    // candidates: wave w, half n, column j -> base + 32 w + 16 n + j
    const uint32_t wbase = blockIdx.x * (uint32_t)kBf16xCands + (uint32_t)wave * 32;
    float c[2][2 * R];
    int slot[2];
    lane_directions<R, 2, PROBE>(p, wbase + col, 16, blockIdx.y == 0 && G == 0, c, slot);
    v8s bre[2][NCH], bim[2][NCH];
    v4f dr[2][NMB], di[2][NMB];
#pragma unroll
    for (int n = 0; n < 2; ++n) {
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
            dr[n][mb] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            di[n][mb] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        }
        unsigned short brp[C][3], bip[C][3];
#pragma unroll
        for (int x = 0; x < C; ++x) {
            float br, bi;
            if (REAL || x < R) {
                br = s3 * c[n][2 * (x % R)];
                bi = c[n][2 * (x % R) + 1];
            } else {
                br = -s3 * c[n][2 * (x - R) + 1];
                bi = c[n][2 * (x - R)];
            }
            bf16_split3(br, brp[x]);
            bf16_split3(bi, bip[x]);
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                short vr = 0, vi = 0;
#pragma unroll
                for (int gg = 0; gg < 4; ++gg) {   // the slot index at compile time
                    const int kap = 32 * ch + 8 * gg + t;
                    if (gg == G && kap < SP::N) {
                        const int tau = kap / C, x = kap % C;
                        vr = (short)brp[x][part_c(tau)];
                        vi = (short)bip[x][part_c(tau)];
                    }
                }
                bre[n][ch][t] = vr;
                bim[n][ch][t] = vi;
            }
        }
    }

    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    // row tid of each tile straight from HBM (each thread needs exactly its
    // own row), the next tile's loads in flight while the current one is scored
    float v[RF];
#pragma unroll
    for (int e = 0; e < RF; ++e) v[e] = r0 + tid < r1 ? p.V[(r0 + tid) * RF + e] : 0.0f;
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, r1 - t0);
        __syncthreads();   // the previous tile's operands are consumed
        {   // row tid: A of the first product and its k-slot in A2
            const int i = tid;
            unsigned short ap[C][3];
#pragma unroll
            for (int x = 0; x < C; ++x) {
                const float a = REAL ? v[x] : (x < R ? v[2 * x] : v[2 * (x - R) + 1]);
                bf16_split3(a, ap[x]);
            }
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int gg = 0; gg < 4; ++gg) {
                    v8s e;
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int kap = 32 * ch + 8 * gg + t;
                        e[t] = kap < SP::N ? (short)ap[kap % C][part_v(kap / C)] : (short)0;
                    }
                    apk[ch][i >> 4][i & 15][gg] = e;
                }
            const int rho = i & 31;
            const int tt = 4 * (rho >> 4) + (rho & 3), gi = (rho >> 2) & 3;
#pragma unroll
            for (int x = 0; x < C; ++x)
#pragma unroll
                for (int pp = 0; pp < 3; ++pp) a2s[i >> 5][pp * C + x][gi][tt] = ap[x][pp];
        }
        __syncthreads();
        {
            const int64_t nx = t0 + kTile + tid;
#pragma unroll
            for (int e = 0; e < RF; ++e) v[e] = nx < r1 ? p.V[nx * RF + e] : 0.0f;
        }
        for (int sub = 0; sub * 32 < cnt; ++sub) {
            v8s a[2][NCH], a2[NMB];
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) a[b][ch] = apk[ch][2 * sub + b][col][G];
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
                a2[mb] = *reinterpret_cast<const v8s*>(&a2s[sub][16 * mb + col][G][0]);
            // w for both halves and both row blocks: independent instructions
            v4f wre[2][2], wim[2][2];
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    wre[n][b] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
                    wim[n][b] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        wre[n][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a[b][ch]), as_bf(bre[n][ch]), wre[n][b], 0, 0, 0);
                        if constexpr (IM)
                            wim[n][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a[b][ch]), as_bf(bim[n][ch]), wim[n][b], 0, 0, 0);
                    }
                }
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                // values t = 4 b + g: row 16 b + 4 G + g
                float u[8], wr[8], wi[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    wr[t] = wre[n][t >> 2][t & 3];
                    wi[t] = wim[n][t >> 2][t & 3];
                    if constexpr (KS == 3) u[t] = wr[t] - fabsf(wi[t]);
                    else if constexpr (KS == 4) u[t] = fabsf(wr[t]) - fabsf(wi[t]);
                    else u[t] = wr[t];
                }
                if constexpr (PROBE) {
                    if (slot[n] >= 0) {
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            const int row = sub * 32 + 16 * (t >> 2) + 4 * G + (t & 3);
                            if (row >= cnt) continue;
                            const bool neg = __float_as_uint(u[t]) >> 31;   // the sign bits, as packed below
                            const bool wneg = __float_as_uint(wi[t]) >> 31, rneg = __float_as_uint(wr[t]) >> 31;
                            int k;
                            if constexpr (KS == 3) k = neg ? (wneg ? 2 : 1) : 0;
                            else if constexpr (KS == 4) k = neg ? (wneg ? 3 : 1) : (rneg ? 2 : 0);
                            else k = neg ? 1 : 0;
                            p.probe_out[(size_t)slot[n] * p.n + t0 + row] = (uint16_t)k;
                        }
                    }
                }
                // labels to BF16, two rows per dword, from sign bits
                // (m = 0xFFFF in each half whose u is negative)
                uint32_t ur[4], ui[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t m = sign_pair(u[2 * e], u[2 * e + 1]);
                    const uint32_t isg = (hi_pair(wi[2 * e], wi[2 * e + 1]) & 0x80008000u) | 0x3F803F80u;
                    if constexpr (KS == 3) {
                        ur[e] = (m & 0xBF00BF00u) | (~m & 0x3F803F80u);   // -1/2 : 1
                        ui[e] = isg & m;                                     // +-1 : 0
                    } else if constexpr (KS == 4) {
                        ur[e] = ((hi_pair(wr[2 * e], wr[2 * e + 1]) & 0x80008000u) | 0x3F803F80u) & ~m;
                        ui[e] = isg & m;
                    } else {
                        ur[e] = (m & 0x80008000u) | 0x3F803F80u;           // +-1 from the sign of Re w
                        ui[e] = 0;
                    }
                }
                const v8s zr = __builtin_bit_cast(v8s, ur);
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
                    dr[n][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a2[mb]), as_bf(zr), dr[n][mb], 0, 0, 0);
                if constexpr (IM) {
                    const v8s zi = __builtin_bit_cast(v8s, ui);
#pragma unroll
                    for (int mb = 0; mb < NMB; ++mb)
                        di[n][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a2[mb]), as_bf(zi), di[n][mb], 0, 0, 0);
                }
            }
        }
    }

    // register g of lane l in (n, mb) is A2 row 16 mb + 4 (l / 16) + g, i.e.
    // part m / C of component m % C, of candidate 16 n + l % 16: gather the
    // four lane groups, add the parts; lanes 0..31 write candidate l
    float pr[2][C], pi[2][C];
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int x = 0; x < C; ++x) pr[n][x] = pi[n][x] = 0.0f;
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int gg = 0; gg < 4; ++gg)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int m = 16 * mb + 4 * gg + g;
                    if (m >= 3 * C) continue;
                    const int srcl = col + 16 * gg;
                    pr[n][m % C] += __shfl(dr[n][mb][g], srcl, kWave);
                    if constexpr (IM) pi[n][m % C] += __shfl(di[n][mb][g], srcl, kWave);
                }
    const uint32_t idx = wbase + lane;
    if (lane >= 32 || idx >= p.S) return;
    const int n = lane >> 4;
    float s[2 * R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const float prj = n ? pr[1][j] : pr[0][j];
        const float pij = n ? pi[1][j] : pi[0][j];
        if constexpr (REAL) {
            s[2 * j] = prj;
            s[2 * j + 1] = IM ? zs * pij : 0.0f;
        } else {
            const float prR = n ? pr[1][R + j] : pr[0][R + j];
            const float piR = n ? pi[1][R + j] : pi[0][R + j];
            s[2 * j] = IM ? prj + zs * piR : prj;
            s[2 * j + 1] = IM ? zs * pij - prR : -prR;
        }
    }
    if (gridDim.y == 1) {
        float f = 0.0f;
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) f = fmaf(s[j], s[j], f);
        p.f_out[idx] = f;
    } else {
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) p.partial[((size_t)blockIdx.y * (2 * R) + j) * p.S + idx] = s[j];
    }
}

}  // namespace
}  // namespace lrqo
