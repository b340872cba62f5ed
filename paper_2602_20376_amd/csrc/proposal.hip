// Learned direction proposal for the sampled maximiser (rank r = 3).
//
// A permutation-invariant network reads the rows of V in a canonical gauge
// and returns a mixture of von Mises-Fisher densities on the unit sphere of
// C^3 = R^6; directions drawn from it (with a share of uniform directions
// kept as fallback) are scored by the sampled solver like any other
// candidates, and its objective is always the FP64 rescore.
//
//   gauge     M = sum_i |v_i|^2 v_i^H v_i (FP64); G = eigenvectors of M in
//             descending order, column phases fixed so that sum_i (V G)_ij^K
//             is real positive and arg sum_i (V G)_ij lies in [-pi/K, pi/K);
//             features x_i = s v_i G, s = sqrt(n / ||V||_F^2)
//   network   h1 = relu(W1 x + b1) (64), h2 = relu(W2 h1 + b2) (64),
//             m = mean_i h2, y = W3 m + b3 (32 x (6 + 2)): component k has
//             mean direction mu_k = y_k[0:6]/|.|, logit a_k, kappa_k = exp(y_k[7])
//   density   vMF on S^5: C_6(kappa) exp(kappa mu . x),
//             C_6 = kappa^2 / ((2 pi)^3 I_2(kappa))
//   loss      -log( (1/K) sum_t p(omega^t c*) ) for the canonical target c*
//   training  hand-written backward (row MLP gradients accumulated over LDS
//             row tiles), fixed-order reduction, Adam
//   sampling  Wood's rejection sampler (Beta(5/2, 5/2) from Gamma(2) and
//             Gamma(1/2) variates), Philox-driven, bounded retries
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lrqo_device.h"
#include "lrqo_runtime.h"

namespace lrqo {

namespace {

constexpr int DIN = 6, H = 64, NC = 32, OUT = NC * (DIN + 2);
constexpr int NP = H * DIN + H + H * H + H + OUT * H + OUT;   // 21,248 parameters
constexpr int OFF_W1 = 0, OFF_B1 = H * DIN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + OUT * H;
constexpr int kBlock = 256;
constexpr int kRowTile = 64;   // rows per backward tile (one per lane)
static_assert(kRowTile == kWave, "the backward maps lane l to row l of the tile");
constexpr int kMaxRetry = 32;  // rejection-sampler attempts before falling back to the mean

struct Frame {                 // canonical gauge of one instance
    double g[18];              // G (3x3 complex, row-major, (re, im))
    double s;
    double pad;
};

// ---------------------------------------------------------------- Bessel
// log I_nu(k): power series below 30, four-term asymptotic expansion above.
__device__ float log_bessel_i(int nu, float k) {
    if (k < 30.0f) {
        const float h2 = 0.25f * k * k;
        float term = nu == 2 ? 0.125f * k * k : k * k * k / 48.0f;   // (k/2)^nu / nu!
        float tot = term;
        for (int m = 1; m < 120; ++m) {
            term *= h2 / (float)(m * (m + nu));
            tot += term;
            if (term < 1e-9f * tot) break;
        }
        return logf(tot);
    }
    const float mu = 4.0f * nu * nu;
    float a = 1.0f, ser = 1.0f, kp = 1.0f, sg = -1.0f;
    for (int j = 1; j <= 4; ++j) {
        a *= (mu - (float)((2 * j - 1) * (2 * j - 1))) / (8.0f * j);
        kp *= k;
        ser += sg * a / kp;
        sg = -sg;
    }
    return k - 0.5f * logf(6.283185307179586f * k) + logf(ser);
}

__device__ float log_vmf_norm(float k) {
    return 2.0f * logf(k) - 3.0f * 1.8378770664093453f - log_bessel_i(2, k);   // 3 log(2 pi)
}

__device__ float mean_resultant(float k) {   // I_3 / I_2 = -d log C_6 / d kappa
    return expf(log_bessel_i(3, k) - log_bessel_i(2, k));
}

// ---------------------------------------------------------------- gauge
// Eigenvectors of a 3x3 Hermitian M through the 6x6 real symmetric form
// [[Re M, -Im M], [Im M, Re M]] (cyclic Jacobi), each eigenvalue appearing
// twice; complex vectors are taken in descending eigenvalue order and
// orthogonalised (complex Gram-Schmidt), keeping three.
__device__ void hermitian_eig3(const double (&Mr)[3][3], const double (&Mi)[3][3],
                               double (&Ur)[3][3], double (&Ui)[3][3]) {
    double A[6][6], Q[6][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            A[i][j] = Mr[i][j];
            A[i + 3][j + 3] = Mr[i][j];
            A[i][j + 3] = -Mi[i][j];
            A[i + 3][j] = Mi[i][j];
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) Q[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, dia = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            dia += A[i][i] * A[i][i];
#pragma unroll
            for (int j = i + 1; j < 6; ++j) off += A[i][j] * A[i][j];
        }
        // converged when the off-diagonal part is at FP64 rounding of the
        // diagonal (an absolute bound would never be met for large M)
        if (off <= 1e-32 * dia || off < 1e-300) break;
        // fully unrolled: every index is a constant, so A and Q stay in registers
#pragma unroll
        for (int p = 0; p < 6; ++p)
#pragma unroll
            for (int q = p + 1; q < 6; ++q) {
                if (fabs(A[p][q]) < 1e-300) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const double qkp = Q[k][p], qkq = Q[k][q];
                    Q[k][p] = c * qkp - s * qkq;
                    Q[k][q] = s * qkp + c * qkq;
                }
            }
    }
    // Everything below indexes A, Q, U only with constants (unrolled loops
    // and selects), so that they stay in registers.
    double ev[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) ev[c] = A[c][c];
    auto pick6 = [](const double (&a)[6], int idx) {
        double v = a[0];
#pragma unroll
        for (int c = 1; c < 6; ++c) v = idx == c ? a[c] : v;
        return v;
    };
    int order[6] = {0, 1, 2, 3, 4, 5};
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j)
            if (pick6(ev, order[j]) > pick6(ev, order[i])) {
                const int t = order[i];
                order[i] = order[j];
                order[j] = t;
            }
    int got = 0;
#pragma unroll
    for (int oi = 0; oi < 6; ++oi) {
        if (got >= 3) break;
        const int col = order[oi];
        double ur[3], ui[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ur[k] = Q[k][0];
            ui[k] = Q[k + 3][0];
#pragma unroll
            for (int c = 1; c < 6; ++c) {
                ur[k] = col == c ? Q[k][c] : ur[k];
                ui[k] = col == c ? Q[k + 3][c] : ui[k];
            }
        }
#pragma unroll
        for (int prev = 0; prev < 3; ++prev) {     // remove <u_prev, u> u_prev
            if (prev >= got) break;
            double dr = 0.0, di = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                dr += Ur[k][prev] * ur[k] + Ui[k][prev] * ui[k];
                di += Ur[k][prev] * ui[k] - Ui[k][prev] * ur[k];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ur[k] -= dr * Ur[k][prev] - di * Ui[k][prev];
                ui[k] -= dr * Ui[k][prev] + di * Ur[k][prev];
            }
        }
        double nrm = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) nrm += ur[k] * ur[k] + ui[k] * ui[k];
        nrm = sqrt(nrm);
        if (nrm < 0.5) continue;                   // the i * u twin of an earlier vector
#pragma unroll
        for (int g = 0; g < 3; ++g)
            if (g == got) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Ur[k][g] = ur[k] / nrm;
                    Ui[k][g] = ui[k] / nrm;
                }
            }
        ++got;
    }
}

__device__ double block_sum(double x, double* red) {
    x = wave_sum_f64(x);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[w] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kBlock / kWave; ++i) t += red[i];
    return t;
}

// Canonical frame of each instance in four stages, the two row passes split
// over `splits` blocks per instance (row range q of ceil(n / splits) rows),
// their partial sums added in split order (FP64):
//   k_frame_m    per split: sum_i |v_i|^2 conj(v_ia) v_ib and sum_i |v_i|^2
//   k_frame_eig  per instance: M, its eigenvectors (descending) -> g, scale s
//   k_frame_p    per split: sum_i (s V U)_ib^K (binary exponentiation of the
//                complex number) and sum_i (s V U)_ib
//   k_frame_fin  per instance: column phases from the two sums -> g
constexpr int kFrameM = 19, kFrameP = 12;

__device__ __forceinline__ void split_rows(int64_t n, int q, int splits, int64_t& r0, int64_t& r1) {
    const int64_t per = (n + splits - 1) / splits;
    r0 = min(n, (int64_t)q * per);
    r1 = min(n, r0 + per);
}

__global__ __launch_bounds__(kBlock) void k_frame_m(const float* __restrict__ V, const int64_t* voff,
                                                   const int64_t* nrows, int splits, double* __restrict__ work) {
    __shared__ double red[kBlock / kWave];
    const int t = blockIdx.x, q = blockIdx.y;
    const float* Vt = V + voff[t];
    int64_t r0, r1;
    split_rows(nrows[t], q, splits, r0, r1);
    double acc[kFrameM] = {0};   // 9 complex entries of M, then sum |v|^2
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        double vr[3], vi[3], w = 0.0;
        for (int j = 0; j < 3; ++j) {
            vr[j] = Vt[i * 6 + 2 * j];
            vi[j] = Vt[i * 6 + 2 * j + 1];
            w += vr[j] * vr[j] + vi[j] * vi[j];
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {   // conj(v_a) v_b
                acc[2 * (3 * a + b)] += w * (vr[a] * vr[b] + vi[a] * vi[b]);
                acc[2 * (3 * a + b) + 1] += w * (vr[a] * vi[b] - vi[a] * vr[b]);
            }
        acc[18] += w;
    }
    for (int e = 0; e < kFrameM; ++e) {
        const double v = block_sum(acc[e], red);
        if (threadIdx.x == 0) work[((size_t)t * splits + q) * kFrameM + e] = v;
    }
}

// One wave sums each entry e < W of instance t over the splits into tot[e]:
// lane l adds splits l, l + 64, ... in order (all W entries' loads in flight
// together), then the 64 lane sums are added by a butterfly (a fixed order).
template <int W>
__device__ __forceinline__ void sum_splits(const double* __restrict__ work, int t, int splits, double* tot) {
    const int l = threadIdx.x;              // blockDim.x == kWave
    const double* src = work + (size_t)t * splits * W;
    double a[W];
#pragma unroll
    for (int e = 0; e < W; ++e) a[e] = 0.0;
    for (int q = l; q < splits; q += kWave) {
#pragma unroll
        for (int e = 0; e < W; ++e) a[e] += src[(size_t)q * W + e];
    }
#pragma unroll
    for (int e = 0; e < W; ++e) {
        const double x = wave_sum_f64(a[e]);
        if (l == 0) tot[e] = x;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kWave) void k_frame_eig(const double* __restrict__ work, const int64_t* nrows, int splits,
                            Frame* __restrict__ frames) {
    __shared__ double tot[kFrameM];
    const int t = blockIdx.x;
    sum_splits<kFrameM>(work, t, splits, tot);
    if (threadIdx.x != 0) return;
    double Mr[3][3], Mi[3][3], Ur[3][3], Ui[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            Mr[a][b] = tot[2 * (3 * a + b)];
            Mi[a][b] = tot[2 * (3 * a + b) + 1];
        }
    hermitian_eig3(Mr, Mi, Ur, Ui);
    Frame f;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            f.g[2 * (3 * a + b)] = Ur[a][b];
            f.g[2 * (3 * a + b) + 1] = Ui[a][b];
        }
    f.s = sqrt((double)nrows[t] / tot[18]);
    f.pad = 0.0;
    frames[t] = f;
}

// w^K for an integer K >= 1 by binary exponentiation
__device__ __forceinline__ void cpow_int(double wr, double wi, int K, double& pr, double& pi) {
    double rr = 1.0, ri = 0.0, br = wr, bi = wi;
    for (int e = K; e > 0; e >>= 1) {
        if (e & 1) {
            const double x = rr * br - ri * bi;
            ri = rr * bi + ri * br;
            rr = x;
        }
        if (e > 1) {
            const double x = br * br - bi * bi;
            bi = 2.0 * br * bi;
            br = x;
        }
    }
    pr = rr;
    pi = ri;
}

__global__ __launch_bounds__(kBlock) void k_frame_p(const float* __restrict__ V, const int64_t* voff,
                                                   const int64_t* nrows, int splits, int K,
                                                   const Frame* __restrict__ frames, double* __restrict__ work) {
    __shared__ double red[kBlock / kWave];
    __shared__ double Us[18];
    const int t = blockIdx.x, q = blockIdx.y;
    if (threadIdx.x < 18) Us[threadIdx.x] = frames[t].g[threadIdx.x];
    __syncthreads();
    const double s = frames[t].s;
    const float* Vt = V + voff[t];
    int64_t r0, r1;
    split_rows(nrows[t], q, splits, r0, r1);
    double pk[6] = {0}, p1[6] = {0};
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        double vr[3], vi[3];
        for (int j = 0; j < 3; ++j) {
            vr[j] = s * Vt[i * 6 + 2 * j];
            vi[j] = s * Vt[i * 6 + 2 * j + 1];
        }
        for (int b = 0; b < 3; ++b) {
            double wr = 0.0, wi = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double ur = Us[2 * (3 * a + b)], ui = Us[2 * (3 * a + b) + 1];
                wr += vr[a] * ur - vi[a] * ui;
                wi += vr[a] * ui + vi[a] * ur;
            }
            p1[2 * b] += wr;
            p1[2 * b + 1] += wi;
            double pr, pim;
            cpow_int(wr, wi, K, pr, pim);
            pk[2 * b] += pr;
            pk[2 * b + 1] += pim;
        }
    }
    for (int e = 0; e < 6; ++e) {
        const double a = block_sum(pk[e], red);
        const double b = block_sum(p1[e], red);
        if (threadIdx.x == 0) {
            work[((size_t)t * splits + q) * kFrameP + e] = a;
            work[((size_t)t * splits + q) * kFrameP + 6 + e] = b;
        }
    }
}

__global__ __launch_bounds__(kWave) void k_frame_fin(const double* __restrict__ work, int splits, int K, Frame* __restrict__ frames) {
    __shared__ double tot[kFrameP];
    const int t = blockIdx.x;
    sum_splits<kFrameP>(work, t, splits, tot);
    if (threadIdx.x != 0) return;
    double PK[6], P1[6];
    for (int e = 0; e < 6; ++e) {
        PK[e] = tot[e];
        P1[e] = tot[6 + e];
    }
    Frame f = frames[t];
    double Us[18];
    for (int e = 0; e < 18; ++e) Us[e] = f.g[e];
    const double two_pi = 6.283185307179586476925286766559;
    for (int b = 0; b < 3; ++b) {
        const double phi = atan2(PK[2 * b + 1], PK[2 * b]) / K;
        // first moment after the K-th-moment phase: rotate into [-pi/K, pi/K)
        const double c1 = cos(-phi), s1 = sin(-phi);
        const double fr = P1[2 * b] * c1 - P1[2 * b + 1] * s1;
        const double fi = P1[2 * b] * s1 + P1[2 * b + 1] * c1;
        const double psi = atan2(fi, fr);
        const double m = floor(psi * K / two_pi + 0.5);
        const double ang = -phi - two_pi * m / K;
        const double cr = cos(ang), ci = sin(ang);
        for (int a = 0; a < 3; ++a) {
            const double ur = Us[2 * (3 * a + b)], ui = Us[2 * (3 * a + b) + 1];
            f.g[2 * (3 * a + b)] = ur * cr - ui * ci;
            f.g[2 * (3 * a + b) + 1] = ur * ci + ui * cr;
        }
    }
    frames[t] = f;
}

// Row splits for frames of `count` instances of at most max_n rows: about
// 1024 blocks in all, at least 1024 rows per split.
int frame_splits(int count, int64_t max_n) {
    int64_t sp = (1024 + count - 1) / count;
    sp = std::min<int64_t>(sp, std::max<int64_t>(1, max_n / 1024));
    return (int)std::max<int64_t>(1, std::min<int64_t>(sp, 256));
}

// Work doubles the frame stages need.
size_t frame_work(int count, int splits) { return (size_t)count * splits * (kFrameM + kFrameP); }

void launch_frames(const float* V, const int64_t* voff, const int64_t* n, int count, int splits, int K,
                   Frame* frames, double* work, hipStream_t st) {
    double* wm = work;
    double* wp = work + (size_t)count * splits * kFrameM;
    hipLaunchKernelGGL(k_frame_m, dim3(count, splits), dim3(kBlock), 0, st, V, voff, n, splits, wm);
    hipLaunchKernelGGL(k_frame_eig, dim3(count), dim3(64), 0, st, wm, n, splits, frames);
    hipLaunchKernelGGL(k_frame_p, dim3(count, splits), dim3(kBlock), 0, st, V, voff, n, splits, K, frames, wp);
    hipLaunchKernelGGL(k_frame_fin, dim3(count), dim3(64), 0, st, wp, splits, K, frames);
}

__device__ __forceinline__ void feature_row(const float* Vt, int64_t i, const Frame& f, float (&x)[DIN]) {
    float vr[3], vi[3];
    for (int j = 0; j < 3; ++j) {
        vr[j] = Vt[i * 6 + 2 * j];
        vi[j] = Vt[i * 6 + 2 * j + 1];
    }
    for (int b = 0; b < 3; ++b) {
        float wr = 0.0f, wi = 0.0f;
        for (int a = 0; a < 3; ++a) {
            const float gr = (float)f.g[2 * (3 * a + b)], gi = (float)f.g[2 * (3 * a + b) + 1];
            wr += vr[a] * gr - vi[a] * gi;
            wi += vr[a] * gi + vi[a] * gr;
        }
        x[2 * b] = (float)f.s * wr;
        x[2 * b + 1] = (float)f.s * wi;
    }
}

// ---------------------------------------------------------------- forward
// Blocks of 256 rows; item j covers rows [start, start+256) of instance inst.
struct RowItems {
    const int32_t* inst;
    const int64_t* start;
    int32_t count;
};

__global__ __launch_bounds__(kBlock) void k_mlp_fwd(const float* __restrict__ V, const int64_t* voff,
                                                   const int64_t* nrows, const Frame* frames,
                                                   const float* __restrict__ theta, RowItems items,
                                                   float* __restrict__ partial /*[items][H]*/) {
    __shared__ float W1[H * DIN], b1[H], W2[H * H], b2[H];
    __shared__ float hs[kBlock / kWave][H];
    for (int e = threadIdx.x; e < H * DIN; e += kBlock) W1[e] = theta[OFF_W1 + e];
    for (int e = threadIdx.x; e < H * H; e += kBlock) W2[e] = theta[OFF_W2 + e];
    for (int e = threadIdx.x; e < H; e += kBlock) {
        b1[e] = theta[OFF_B1 + e];
        b2[e] = theta[OFF_B2 + e];
    }
    __syncthreads();
    const int it = blockIdx.x;
    const int t = items.inst[it];
    const int64_t i = items.start[it] + threadIdx.x;
    const int64_t n = nrows[t];
    const bool live = i < n;
    float x[DIN], h1[H];
#pragma unroll
    for (int k = 0; k < DIN; ++k) x[k] = 0.0f;
    if (live) feature_row(V + voff[t], i, frames[t], x);
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float a = b1[o];
#pragma unroll
        for (int k = 0; k < DIN; ++k) a = fmaf(W1[o * DIN + k], x[k], a);
        h1[o] = fmaxf(a, 0.0f);
    }
    // each output of the second layer is summed over the block as it is made
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int o = 0; o < H; ++o) {
        float a = b2[o];
#pragma unroll
        for (int k = 0; k < H; ++k) a = fmaf(W2[o * H + k], h1[k], a);
        float v = live ? fmaxf(a, 0.0f) : 0.0f;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
        if (lane == 0) hs[w][o] = v;
    }
    __syncthreads();
    if (threadIdx.x < H) {
        float v = 0.0f;
        for (int q = 0; q < kBlock / kWave; ++q) v += hs[q][threadIdx.x];
        partial[(size_t)it * H + threadIdx.x] = v;
    }
}

// Mean embedding per instance from its items' partial sums (items of one
// instance are consecutive).  kPoolGroups groups of H threads each add a
// contiguous run of the items (in item order, sixteen loads in flight); the
// group sums are then added in group order.
constexpr int kPoolGroups = 16;

__global__ __launch_bounds__(H * kPoolGroups) void k_pool(const float* __restrict__ partial, const int32_t* first_item,
                                                          const int64_t* nrows, int count, float* __restrict__ mvec) {
    __shared__ float gsum[kPoolGroups][H];
    const int t = blockIdx.x;
    const int o = threadIdx.x % H, grp = threadIdx.x / H;
    if (t >= count) return;                  // the same in every thread of the block
    const int first = first_item[t], end = first_item[t + 1];
    const int per = (end - first + kPoolGroups - 1) / kPoolGroups;
    int it = min(end, first + grp * per);
    const int stop = min(end, it + per);
    float v = 0.0f;
    for (; it + 16 <= stop; it += 16) {
        float p[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) p[u] = partial[(size_t)(it + u) * H + o];
#pragma unroll
        for (int u = 0; u < 16; ++u) v += p[u];
    }
    for (; it < stop; ++it) v += partial[(size_t)it * H + o];
    gsum[grp][o] = v;
    __syncthreads();
    if (grp == 0) {
        float sum = 0.0f;
        for (int g = 0; g < kPoolGroups; ++g) sum += gsum[g][o];
        mvec[(size_t)t * H + o] = sum / (float)nrows[t];
    }
}

// Head: mixture parameters of one instance.
struct Mixture {
    float mu[NC][DIN];
    float logpi[NC];
    float kappa[NC];
    float logc[NC];
    float nrm[NC];
};

__device__ void head(const float* theta, const float* m, Mixture& mx, float* y /*[OUT]*/) {
    for (int o = threadIdx.x; o < OUT; o += blockDim.x) {
        float a = theta[OFF_B3 + o];
        for (int k = 0; k < H; ++k) a = fmaf(theta[OFF_W3 + o * H + k], m[k], a);
        y[o] = a;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        const int k = threadIdx.x;
        float nrm = 0.0f;
        for (int d = 0; d < DIN; ++d) nrm += y[k * (DIN + 2) + d] * y[k * (DIN + 2) + d];
        nrm = sqrtf(nrm);
        mx.nrm[k] = nrm;
        for (int d = 0; d < DIN; ++d) mx.mu[k][d] = y[k * (DIN + 2) + d] / nrm;
        const float kap = expf(y[k * (DIN + 2) + DIN + 1]);
        mx.kappa[k] = kap;
        mx.logc[k] = log_vmf_norm(kap);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float amax = -INFINITY;
        for (int k = 0; k < NC; ++k) amax = fmaxf(amax, y[k * (DIN + 2) + DIN]);
        float se = 0.0f;
        for (int k = 0; k < NC; ++k) se += expf(y[k * (DIN + 2) + DIN] - amax);
        const float lse = amax + logf(se);
        for (int k = 0; k < NC; ++k) mx.logpi[k] = y[k * (DIN + 2) + DIN] - lse;
    }
    __syncthreads();
}

// Per instance: loss, d loss / d y, d loss / d m (for the row backward), and
// this instance's share of dW3, db3.  One block of 256 threads.
__global__ __launch_bounds__(kBlock) void k_head_loss(const float* __restrict__ theta,
                                                     const float* __restrict__ mvec,
                                                     const float* __restrict__ target /*[count][6] canonical c**/,
                                                     int K, float* __restrict__ loss,
                                                     float* __restrict__ dmvec, float* __restrict__ gW3 /*[count][OUT*H+OUT]*/) {
    __shared__ Mixture mx;
    __shared__ float y[OUT], dy[OUT], m[H];
    __shared__ float lg[256][NC + 1];   // K <= 255 rotations
    __shared__ float Q[NC], Xb[NC][DIN];
    const int t = blockIdx.x;
    if (threadIdx.x < H) m[threadIdx.x] = mvec[(size_t)t * H + threadIdx.x];
    __syncthreads();
    head(theta, m, mx, y);
    const float* c = target + (size_t)t * DIN;
    // log(pi_k) + log f_k(omega^r c*) for every rotation r and component k
    for (int e = threadIdx.x; e < K * NC; e += kBlock) {
        const int r = e / NC, k = e % NC;
        const float ang = 6.283185307179586f * (float)r / (float)K;
        const float cs = cosf(ang), sn = sinf(ang);
        float dot = 0.0f;
        for (int j = 0; j < 3; ++j) {
            const float xr = cs * c[2 * j] - sn * c[2 * j + 1];
            const float xi = sn * c[2 * j] + cs * c[2 * j + 1];
            dot += mx.mu[k][2 * j] * xr + mx.mu[k][2 * j + 1] * xi;
        }
        lg[r][k] = mx.logpi[k] + mx.logc[k] + mx.kappa[k] * dot;
    }
    __syncthreads();
    __shared__ float lse_s;
    if (threadIdx.x == 0) {
        float mxv = -INFINITY;
        for (int r = 0; r < K; ++r)
            for (int k = 0; k < NC; ++k) mxv = fmaxf(mxv, lg[r][k]);
        float se = 0.0f;
        for (int r = 0; r < K; ++r)
            for (int k = 0; k < NC; ++k) se += expf(lg[r][k] - mxv);
        lse_s = mxv + logf(se);
        loss[t] = -(lse_s - logf((float)K));
    }
    __syncthreads();
    // posterior q_{rk}: component mass Q_k and weighted mean X̄_k
    if (threadIdx.x < NC) {
        const int k = threadIdx.x;
        float qk = 0.0f, xb[DIN] = {0};
        for (int r = 0; r < K; ++r) {
            const float q = expf(lg[r][k] - lse_s);
            qk += q;
            const float ang = 6.283185307179586f * (float)r / (float)K;
            const float cs = cosf(ang), sn = sinf(ang);
            for (int j = 0; j < 3; ++j) {
                xb[2 * j] += q * (cs * c[2 * j] - sn * c[2 * j + 1]);
                xb[2 * j + 1] += q * (sn * c[2 * j] + cs * c[2 * j + 1]);
            }
        }
        Q[k] = qk;
        for (int d = 0; d < DIN; ++d) Xb[k][d] = xb[d];
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        const int k = threadIdx.x;
        const float kap = mx.kappa[k];
        float mux = 0.0f;
        for (int d = 0; d < DIN; ++d) mux += mx.mu[k][d] * Xb[k][d];
        const float dkappa = -(Q[k] * (-mean_resultant(kap)) + mux);
        dy[k * (DIN + 2) + DIN + 1] = dkappa * kap;
        dy[k * (DIN + 2) + DIN] = -Q[k] + expf(mx.logpi[k]);
        float dmu[DIN], proj = 0.0f;
        for (int d = 0; d < DIN; ++d) {
            dmu[d] = -kap * Xb[k][d];
            proj += dmu[d] * mx.mu[k][d];
        }
        for (int d = 0; d < DIN; ++d) dy[k * (DIN + 2) + d] = (dmu[d] - proj * mx.mu[k][d]) / mx.nrm[k];
    }
    __syncthreads();
    float* g = gW3 + (size_t)t * (OUT * H + OUT);
    for (int e = threadIdx.x; e < OUT * H; e += kBlock) g[e] = dy[e / H] * m[e % H];
    for (int o = threadIdx.x; o < OUT; o += kBlock) g[OUT * H + o] = dy[o];
    if (threadIdx.x < H) {
        float a = 0.0f;
        for (int o = 0; o < OUT; ++o) a = fmaf(theta[OFF_W3 + o * H + threadIdx.x], dy[o], a);
        dmvec[(size_t)t * H + threadIdx.x] = a;
    }
}

// Row backward: item j covers kRowTile rows of one instance; gradients of
// W1, b1, W2, b2 over those rows into partial[j][...] (H*DIN + H + H*H + H).
__global__ __launch_bounds__(kBlock) void k_mlp_bwd(const float* __restrict__ V, const int64_t* voff,
                                                   const int64_t* nrows, const Frame* frames,
                                                   const float* __restrict__ theta,
                                                   const float* __restrict__ dmvec, RowItems items,
                                                   float* __restrict__ partial) {
    constexpr int NG = H * DIN + H + H * H + H;
    __shared__ float W1[H * DIN], b1[H], W2[H * H], b2[H];
    // rows padded to H + 1 floats: lanes that hold different rows of one
    // column fall in different LDS banks
    __shared__ float X[kRowTile][DIN + 1], A1[kRowTile][H + 1], D2[kRowTile][H + 1], D1[kRowTile][H + 1];
    __shared__ float dh2[H];
    for (int e = threadIdx.x; e < H * DIN; e += kBlock) W1[e] = theta[OFF_W1 + e];
    for (int e = threadIdx.x; e < H * H; e += kBlock) W2[e] = theta[OFF_W2 + e];
    const int it = blockIdx.x;
    const int t = items.inst[it];
    const int64_t n = nrows[t];
    for (int e = threadIdx.x; e < H; e += kBlock) {
        b1[e] = theta[OFF_B1 + e];
        b2[e] = theta[OFF_B2 + e];
        dh2[e] = dmvec[(size_t)t * H + e] / (float)n;   // mean pooling
    }
    __syncthreads();
    const int64_t i0 = items.start[it];
    // forward recompute and d pre-activations: thread (row rr = lane, part =
    // wave) takes neurons 16 part .. 16 part + 15 of each layer
    constexpr int HP = H / (kBlock / kWave);
    const int rr = threadIdx.x & (kWave - 1), o0 = (threadIdx.x / kWave) * HP;
    const int64_t i = i0 + rr;
    const bool live = i < n;
    {
        float x[DIN];
#pragma unroll
        for (int k = 0; k < DIN; ++k) x[k] = 0.0f;
        if (live) feature_row(V + voff[t], i, frames[t], x);
        if (o0 == 0) {
#pragma unroll
            for (int k = 0; k < DIN; ++k) X[rr][k] = x[k];
        }
#pragma unroll
        for (int oo = 0; oo < HP; ++oo) {
            const int o = o0 + oo;
            float a = b1[o];
#pragma unroll
            for (int k = 0; k < DIN; ++k) a = fmaf(W1[o * DIN + k], x[k], a);
            A1[rr][o] = live ? fmaxf(a, 0.0f) : 0.0f;
        }
    }
    __syncthreads();
    for (int oo = 0; oo < HP; ++oo) {
        const int o = o0 + oo;
        float a = b2[o];
#pragma unroll 16
        for (int k = 0; k < H; ++k) a = fmaf(W2[o * H + k], A1[rr][k], a);
        D2[rr][o] = (live && a > 0.0f) ? dh2[o] : 0.0f;
    }
    __syncthreads();
    for (int kk = 0; kk < HP; ++kk) {
        const int k = o0 + kk;
        float a = 0.0f;
#pragma unroll 16
        for (int o = 0; o < H; ++o) a = fmaf(W2[o * H + k], D2[rr][o], a);
        D1[rr][k] = A1[rr][k] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    // weight gradients over the tile's rows, each entry summed over the rows
    // in order.  dW2[o][k] = sum_r D2[r][o] A1[r][k]: thread (to, tk) of a
    // 16 x 16 grid owns the 4 x 4 block o in 4to.., k in 4tk.. (eight LDS
    // reads per sixteen FMAs)
    float* out = partial + (size_t)it * NG;
    static_assert(kBlock == 256 && H == 64, "the dW2 tiling assumes 256 threads and H = 64");
    {
        const int to = threadIdx.x / 16, tk = threadIdx.x % 16;
        float acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
        for (int r = 0; r < kRowTile; ++r) {
            float d[4], h[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                d[a] = D2[r][4 * to + a];
                h[a] = A1[r][4 * tk + a];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(d[a], h[b], acc[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) out[H * DIN + H + (4 * to + a) * H + 4 * tk + b] = acc[a][b];
    }
    // dW1, db1 and db2: thread e owns entries e, e + 256 of those 512
    for (int e = threadIdx.x; e < H * DIN + 2 * H; e += kBlock) {
        float a = 0.0f;
        if (e < H * DIN) {                       // dW1[o][k] = sum_r D1[r][o] X[r][k]
            const int o = e / DIN, k = e % DIN;
            for (int r = 0; r < kRowTile; ++r) a = fmaf(D1[r][o], X[r][k], a);
            out[e] = a;
        } else if (e < H * DIN + H) {            // db1
            const int o = e - H * DIN;
            for (int r = 0; r < kRowTile; ++r) a += D1[r][o];
            out[e] = a;
        } else {                                 // db2
            const int o = e - H * DIN - H;
            for (int r = 0; r < kRowTile; ++r) a += D2[r][o];
            out[H * DIN + H + H * H + o] = a;
        }
    }
}

// grad[p] = (1/B) * (sum over row items of the MLP partials + sum over
// instances of the head partials), fixed order.
// Gradient = (sum of the row-tile partials of the MLP parameters, sum of
// the per-instance head partials) / count, in two fixed-order levels:
// chunk c of the partials -> gpart[c][p], then the chunks in order.
constexpr int kGradChunks = 64;

__global__ void k_grad_partial(const float* __restrict__ mlp_partial, int nitems,
                               const float* __restrict__ head_partial, int count,
                               float* __restrict__ gpart) {
    constexpr int NG = H * DIN + H + H * H + H;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (p >= NP) return;
    float a = 0.0f;
    if (p < NG) {
        const int per = (nitems + kGradChunks - 1) / kGradChunks;
        const int lo = c * per, hi = min(nitems, lo + per);
        for (int it = lo; it < hi; ++it) a += mlp_partial[(size_t)it * NG + p];
    } else {
        const int q = p - NG;
        const int per = (count + kGradChunks - 1) / kGradChunks;
        const int lo = c * per, hi = min(count, lo + per);
        for (int t = lo; t < hi; ++t) a += head_partial[(size_t)t * (OUT * H + OUT) + q];
    }
    gpart[(size_t)c * NP + p] = a;
}

__global__ void k_grad_reduce(const float* __restrict__ gpart, int count, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    float a = 0.0f;
    for (int c = 0; c < kGradChunks; ++c) a += gpart[(size_t)c * NP + p];
    grad[p] = a / (float)count;
}

__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    theta[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// ---------------------------------------------------------------- sampling
__device__ __forceinline__ float u01(uint32_t x) { return ((float)(x >> 9) + 0.5f) * 0x1p-23f; }

struct Rng {             // Philox-driven stream of uniforms for one sample
    uint64_t seed;
    uint32_t inst, s;
    uint32_t blk;
    uint32_t buf[4];
    int used;
    __device__ float next() {
        if (used == 4) {
            const U4 o = philox4x32_10(U4{s, 0x5EEDu, inst, 0x40000000u | blk},
                                       (uint32_t)seed, (uint32_t)(seed >> 32));
            buf[0] = o.x; buf[1] = o.y; buf[2] = o.z; buf[3] = o.w;
            ++blk;
            used = 0;
        }
        return u01(buf[used++]);
    }
    __device__ float normal() {
        const float a = next(), b = next();
        return sqrtf(-2.0f * logf(a)) * cospif(2.0f * b);
    }
    __device__ float gamma25() {   // Gamma(2) + Gamma(1/2) = Gamma(5/2)
        const float z = normal();
        return -logf(next() * next()) + 0.5f * z * z;
    }
};

// One thread per proposed direction.  Index s is uniform (the plain stream's
// direction s) when s % period == 0 with period = round(1/uniform_fraction),
// otherwise drawn from the mixture: component by its weight, w by Wood's
// rejection, a uniform tangent direction; c = G c_can.
__global__ __launch_bounds__(kBlock) void k_sample(const float* __restrict__ theta, const float* __restrict__ mvec,
                                                  const Frame* frames, int64_t S, uint64_t seed, uint32_t inst,
                                                  int period, float* __restrict__ dirs) {
    __shared__ Mixture mx;
    __shared__ float y[OUT], m[H];
    if (threadIdx.x < H) m[threadIdx.x] = mvec[threadIdx.x];
    __syncthreads();
    head(theta, m, mx, y);
    const Frame f = frames[0];
    for (int64_t s = blockIdx.x * (int64_t)kBlock + threadIdx.x; s < S; s += (int64_t)gridDim.x * kBlock) {
        float c[6];
        if (period > 0 && s % period == 0) {
            direction_f32<3>(seed, (uint64_t)s, inst, c);
        } else {
            Rng rng{seed, inst, (uint32_t)s, 0u, {0, 0, 0, 0}, 4};
            const float u = rng.next();
            int k = 0;
            float cum = expf(mx.logpi[0]);
            while (k < NC - 1 && u > cum) {
                ++k;
                cum += expf(mx.logpi[k]);
            }
            const float kap = mx.kappa[k];
            const float b = 5.0f / (2.0f * kap + sqrtf(4.0f * kap * kap + 25.0f));
            const float x0 = (1.0f - b) / (1.0f + b);
            const float cc = kap * x0 + 5.0f * logf(1.0f - x0 * x0);
            float w = 1.0f;
            for (int a = 0; a < kMaxRetry; ++a) {
                const float g1 = rng.gamma25(), g2 = rng.gamma25();
                const float z = g1 / (g1 + g2);
                const float ww = (1.0f - (1.0f + b) * z) / (1.0f - (1.0f - b) * z);
                const float uu = rng.next();
                if (kap * ww + 5.0f * logf(1.0f - x0 * ww) - cc >= logf(uu)) {
                    w = ww;
                    break;
                }
            }
            float tv[6], dot = 0.0f;
            for (int d = 0; d < 6; ++d) {
                tv[d] = rng.normal();
                dot += tv[d] * mx.mu[k][d];
            }
            float nt = 0.0f;
            for (int d = 0; d < 6; ++d) {
                tv[d] -= dot * mx.mu[k][d];
                nt += tv[d] * tv[d];
            }
            nt = nt > 0.0f ? 1.0f / sqrtf(nt) : 0.0f;
            const float sw = sqrtf(fmaxf(0.0f, 1.0f - w * w));
            float xc[6];
            for (int d = 0; d < 6; ++d) xc[d] = w * mx.mu[k][d] + sw * tv[d] * nt;
            // c = G c_can
            float nrm = 0.0f;
            for (int a2 = 0; a2 < 3; ++a2) {
                float re = 0.0f, im = 0.0f;
                for (int b2 = 0; b2 < 3; ++b2) {
                    const float gr = (float)f.g[2 * (3 * a2 + b2)], gi = (float)f.g[2 * (3 * a2 + b2) + 1];
                    re += gr * xc[2 * b2] - gi * xc[2 * b2 + 1];
                    im += gr * xc[2 * b2 + 1] + gi * xc[2 * b2];
                }
                c[2 * a2] = re;
                c[2 * a2 + 1] = im;
                nrm += re * re + im * im;
            }
            const float inv = 1.0f / sqrtf(nrm);
            for (int d = 0; d < 6; ++d) c[d] *= inv;
        }
        for (int d = 0; d < 6; ++d) dirs[s * 6 + d] = c[d];
    }
}

// Canonical targets: c_can = G^H c* (unit), written as 6 floats.
__global__ void k_targets(const float* __restrict__ cstar, const Frame* frames, int count,
                          float* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const Frame f = frames[t];
    float nrm = 0.0f, o[6];
    for (int b = 0; b < 3; ++b) {
        float re = 0.0f, im = 0.0f;
        for (int a = 0; a < 3; ++a) {
            const float gr = (float)f.g[2 * (3 * a + b)], gi = -(float)f.g[2 * (3 * a + b) + 1];
            const float cr = cstar[t * 6 + 2 * a], ci = cstar[t * 6 + 2 * a + 1];
            re += gr * cr - gi * ci;
            im += gr * ci + gi * cr;
        }
        o[2 * b] = re;
        o[2 * b + 1] = im;
        nrm += re * re + im * im;
    }
    const float inv = 1.0f / sqrtf(nrm);
    for (int d = 0; d < 6; ++d) out[t * 6 + d] = o[d] * inv;
}

}  // namespace
}  // namespace lrqo

// ---------------------------------------------------------------- C ABI
struct lrqo_proposal {
    int device;
    int K;
    float* theta = nullptr;   // device parameters
    float* m = nullptr;       // Adam first moment
    float* v = nullptr;       // Adam second moment
    float* grad = nullptr;
    int64_t step = 0;
    // per-call scratch (grown on demand)
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
};

namespace {

using lrqo::fail;

lrqo_status ensure_scratch(lrqo_proposal* p, size_t bytes) {
    if (bytes <= p->scratch_bytes) return LRQO_OK;
    if (p->scratch) {
        LRQO_HIP(hipDeviceSynchronize());
        LRQO_HIP(hipFree(p->scratch));
        p->scratch = nullptr;
        p->scratch_bytes = 0;
    }
    if (hipMalloc(&p->scratch, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->scratch = nullptr;
        return fail(LRQO_ENOMEM, "proposal scratch allocation failed");
    }
    p->scratch_bytes = bytes;
    return LRQO_OK;
}

struct RowPlan {
    std::vector<int32_t> inst;
    std::vector<int64_t> start;
    std::vector<int32_t> first;   // first item of each instance (+ end)
};

void plan_rows(int count, const int64_t* n, int tile, RowPlan& rp) {
    rp.inst.clear();
    rp.start.clear();
    rp.first.assign(count + 1, 0);
    for (int t = 0; t < count; ++t) {
        rp.first[t] = (int32_t)rp.inst.size();
        for (int64_t s = 0; s < n[t]; s += tile) {
            rp.inst.push_back(t);
            rp.start.push_back(s);
        }
    }
    rp.first[count] = (int32_t)rp.inst.size();
}

// The host-to-device data of one call in one copy: its pieces are carved one
// after another, so their device offsets (alignment padding included) lay
// out one host image of the whole range.
struct Upload {
    char* base = nullptr;
    std::vector<char> img;
    template <class T>
    T* take(lrqo::Carve& cv, const T* src, size_t count) {
        T* d = cv.take<T>(count);
        if (!base) base = reinterpret_cast<char*>(d);
        const size_t off = (size_t)(reinterpret_cast<char*>(d) - base), bytes = sizeof(T) * count;
        if (img.size() < off + bytes) img.resize(off + bytes);
        if (bytes) std::memcpy(img.data() + off, src, bytes);
        return d;
    }
    lrqo_status send(hipStream_t st) {
        using namespace lrqo;
        if (base && !img.empty())
            LRQO_HIP(hipMemcpyAsync(base, img.data(), img.size(), hipMemcpyHostToDevice, st));
        return LRQO_OK;
    }
};

// Shared by training and inference: frames, pooled embeddings.
struct FwdBufs {
    int64_t* voff;
    int64_t* n;
    lrqo::Frame* frames;
    int32_t* inst;
    int64_t* start;
    int32_t* first;
    float* partial;
    float* mvec;
    double* fwork;              // frame stages' partial sums
    int fsplits;
};

// b's descriptors (offsets, sizes, the row plan) are on the device already.
lrqo_status run_embed(lrqo_proposal* P, const float* V, int count, const RowPlan& rp, FwdBufs& b, hipStream_t st) {
    using namespace lrqo;
    launch_frames(V, b.voff, b.n, count, b.fsplits, P->K, b.frames, b.fwork, st);
    LRQO_HIP(hipGetLastError());
    RowItems items{b.inst, b.start, (int32_t)rp.inst.size()};
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)rp.inst.size()), dim3(kBlock), 0, st, V, b.voff, b.n,
                       b.frames, P->theta, items, b.partial);
    LRQO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pool, dim3(count), dim3(H * kPoolGroups), 0, st, b.partial, b.first, b.n, count, b.mvec);
    LRQO_HIP(hipGetLastError());
    return LRQO_OK;
}

}  // namespace

extern "C" {

int32_t lrqo_proposal_param_count(void) { return lrqo::NP; }

lrqo_status lrqo_proposal_create(const double* init, int32_t K, lrqo_proposal** out) {
    using namespace lrqo;
    clear_error();
    if (!init || !out) return fail(LRQO_EINVAL, "null pointer argument");
    if (K < 2 || K > LRQO_MAX_K) return fail(LRQO_EINVAL, "K must be in [2, 255]");
    auto* P = new lrqo_proposal();
    P->K = K;
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return fail(LRQO_EDEVICE, "hipGetDevice failed");
    }
    std::vector<float> h(NP);
    for (int i = 0; i < NP; ++i) h[i] = (float)init[i];
    if (hipMalloc(&P->theta, sizeof(float) * NP) != hipSuccess || hipMalloc(&P->m, sizeof(float) * NP) != hipSuccess ||
        hipMalloc(&P->v, sizeof(float) * NP) != hipSuccess || hipMalloc(&P->grad, sizeof(float) * NP) != hipSuccess) {
        (void)hipGetLastError();
        lrqo_proposal_destroy(P);
        return fail(LRQO_ENOMEM, "proposal allocation failed");
    }
    LRQO_HIP(hipMemcpy(P->theta, h.data(), sizeof(float) * NP, hipMemcpyHostToDevice));
    LRQO_HIP(hipMemset(P->m, 0, sizeof(float) * NP));
    LRQO_HIP(hipMemset(P->v, 0, sizeof(float) * NP));
    LRQO_HIP(hipMemset(P->grad, 0, sizeof(float) * NP));
    *out = P;
    return LRQO_OK;
}

lrqo_status lrqo_proposal_destroy(lrqo_proposal* P) {
    if (!P) return LRQO_OK;
    (void)hipDeviceSynchronize();
    if (P->theta) (void)hipFree(P->theta);
    if (P->m) (void)hipFree(P->m);
    if (P->v) (void)hipFree(P->v);
    if (P->grad) (void)hipFree(P->grad);
    if (P->scratch) (void)hipFree(P->scratch);
    delete P;
    return LRQO_OK;
}

lrqo_status lrqo_proposal_get_state(lrqo_proposal* P, float* theta, float* m, float* v, int64_t* step) {
    using namespace lrqo;
    clear_error();
    if (!P || !theta) return fail(LRQO_EINVAL, "null pointer argument");
    LRQO_HIP(hipDeviceSynchronize());
    LRQO_HIP(hipMemcpy(theta, P->theta, sizeof(float) * NP, hipMemcpyDeviceToHost));
    if (m) LRQO_HIP(hipMemcpy(m, P->m, sizeof(float) * NP, hipMemcpyDeviceToHost));
    if (v) LRQO_HIP(hipMemcpy(v, P->v, sizeof(float) * NP, hipMemcpyDeviceToHost));
    if (step) *step = P->step;
    return LRQO_OK;
}

lrqo_status lrqo_proposal_set_state(lrqo_proposal* P, const float* theta, const float* m, const float* v,
                                    int64_t step) {
    using namespace lrqo;
    clear_error();
    if (!P || !theta) return fail(LRQO_EINVAL, "null pointer argument");
    if (step < 0) return fail(LRQO_EINVAL, "step must be >= 0");
    LRQO_HIP(hipMemcpy(P->theta, theta, sizeof(float) * NP, hipMemcpyHostToDevice));
    if (m) LRQO_HIP(hipMemcpy(P->m, m, sizeof(float) * NP, hipMemcpyHostToDevice));
    if (v) LRQO_HIP(hipMemcpy(P->v, v, sizeof(float) * NP, hipMemcpyHostToDevice));
    P->step = step;
    return LRQO_OK;
}

lrqo_status lrqo_proposal_train_step(lrqo_proposal* P, const float* V, int32_t count, const int64_t* v_offset,
                                     const int64_t* n, const float* targets, float lr, int32_t update,
                                     double* mean_loss, float* grad_out) {
    using namespace lrqo;
    clear_error();
    if (!P || !V || !v_offset || !n || !targets) return fail(LRQO_EINVAL, "null pointer argument");
    if (count < 1 || count > 65536) return fail(LRQO_EINVAL, "count must be in [1, 65536]");
    if (!(lr >= 0.0f) || lr > 1.0f) return fail(LRQO_EINVAL, "lr must be in [0, 1]");
    for (int t = 0; t < count; ++t)
        if (n[t] < 1 || n[t] > (1 << 24) || v_offset[t] < 0) return fail(LRQO_EINVAL, "bad n or v_offset");
    if (!is_device_pointer(V)) return fail(LRQO_EINVAL, "V is not device memory");
    RowPlan fp, bp;
    plan_rows(count, n, kBlock, fp);
    plan_rows(count, n, kRowTile, bp);
    constexpr int NG = H * DIN + H + H * H + H;
    CarveSize cs;
    cs.add<int64_t>(count);                  // uploaded: offsets, sizes,
    cs.add<int64_t>(count);
    cs.add<int32_t>(fp.inst.size());         // forward row plan,
    cs.add<int64_t>(fp.start.size());
    cs.add<int32_t>(count + 1);
    cs.add<float>((size_t)count * 6);        // host targets,
    cs.add<int32_t>(bp.inst.size());         // backward row plan
    cs.add<int64_t>(bp.start.size());
    cs.add<Frame>(count);
    cs.add<float>(fp.inst.size() * H);
    cs.add<float>((size_t)count * H);        // m
    cs.add<float>((size_t)count * H);        // dm
    cs.add<float>((size_t)count * 6);        // canonical targets
    cs.add<float>(count);                    // loss
    cs.add<float>((size_t)count * (OUT * H + OUT));
    cs.add<float>(bp.inst.size() * NG);
    cs.add<float>((size_t)kGradChunks * NP);
    const int fsplits = frame_splits(count, *std::max_element(n, n + count));
    cs.add<double>(frame_work(count, fsplits));
    LRQO_TRY(ensure_scratch(P, cs.bytes));
    Carve cv(P->scratch);
    FwdBufs b{};
    Upload up;
    b.voff = up.take(cv, v_offset, count);
    b.n = up.take(cv, n, count);
    b.inst = up.take(cv, fp.inst.data(), fp.inst.size());
    b.start = up.take(cv, fp.start.data(), fp.start.size());
    b.first = up.take(cv, fp.first.data(), fp.first.size());
    float* tin = up.take(cv, targets, (size_t)count * 6);
    int32_t* inst_b = up.take(cv, bp.inst.data(), bp.inst.size());
    int64_t* start_b = up.take(cv, bp.start.data(), bp.start.size());
    b.frames = cv.take<Frame>(count);
    b.partial = cv.take<float>(fp.inst.size() * H);
    b.mvec = cv.take<float>((size_t)count * H);
    float* dm = cv.take<float>((size_t)count * H);
    float* tcan = cv.take<float>((size_t)count * 6);
    float* loss = cv.take<float>(count);
    float* headp = cv.take<float>((size_t)count * (OUT * H + OUT));
    float* mlpp = cv.take<float>(bp.inst.size() * NG);
    float* gpart = cv.take<float>((size_t)kGradChunks * NP);
    b.fwork = cv.take<double>(frame_work(count, fsplits));
    b.fsplits = fsplits;
    hipStream_t st = current_stream();
    LRQO_TRY(up.send(st));
    LRQO_TRY(run_embed(P, V, count, fp, b, st));
    hipLaunchKernelGGL(k_targets, dim3((count + 255) / 256), dim3(256), 0, st, tin, b.frames, count, tcan);
    hipLaunchKernelGGL(k_head_loss, dim3(count), dim3(kBlock), 0, st, P->theta, b.mvec, tcan, P->K, loss, dm, headp);
    LRQO_HIP(hipGetLastError());
    RowItems items{inst_b, start_b, (int32_t)bp.inst.size()};
    hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)bp.inst.size()), dim3(kBlock), 0, st, V, b.voff, b.n, b.frames,
                       P->theta, dm, items, mlpp);
    LRQO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_grad_partial, dim3((NP + 255) / 256, kGradChunks), dim3(256), 0, st, mlpp,
                       (int)bp.inst.size(), headp, count, gpart);
    hipLaunchKernelGGL(k_grad_reduce, dim3((NP + 255) / 256), dim3(256), 0, st, gpart, count, P->grad);
    LRQO_HIP(hipGetLastError());
    if (update) {
        P->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - powf(b1, (float)P->step), c2 = 1.0f - powf(b2, (float)P->step);
        hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, st, P->theta, P->grad, P->m, P->v, lr, b1,
                           b2, 1e-8f, c1, c2);
        LRQO_HIP(hipGetLastError());
    }
    std::vector<float> hl(count);
    LRQO_HIP(hipMemcpyAsync(hl.data(), loss, sizeof(float) * count, hipMemcpyDeviceToHost, st));
    if (grad_out) LRQO_HIP(hipMemcpyAsync(grad_out, P->grad, sizeof(float) * NP, hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipStreamSynchronize(st));
    if (mean_loss) {
        double s = 0.0;
        for (float x : hl) s += x;
        *mean_loss = s / count;
    }
    return LRQO_OK;
}

lrqo_status lrqo_proposal_sample(lrqo_proposal* P, const float* V, int64_t n, int64_t S, uint64_t seed,
                                 uint32_t instance, float uniform_fraction, float* dirs) {
    using namespace lrqo;
    clear_error();
    if (!P || !V || !dirs) return fail(LRQO_EINVAL, "null pointer argument");
    if (n < 1 || n > (1 << 24)) return fail(LRQO_EINVAL, "n must be in [1, 2^24]");
    if (S < 1 || S > (int64_t)0xFFFFFFFFll) return fail(LRQO_EINVAL, "S must be in [1, 2^32-1]");
    if (!(uniform_fraction >= 0.0f && uniform_fraction <= 1.0f))
        return fail(LRQO_EINVAL, "uniform_fraction must be in [0, 1]");
    if (!is_device_pointer(V) || !is_device_pointer(dirs)) return fail(LRQO_EINVAL, "V and dirs must be device memory");
    RowPlan fp;
    const int64_t zero = 0;
    plan_rows(1, &n, kBlock, fp);
    CarveSize cs;
    cs.add<int64_t>(1);                      // uploaded: offset, size, row plan
    cs.add<int64_t>(1);
    cs.add<int32_t>(fp.inst.size());
    cs.add<int64_t>(fp.start.size());
    cs.add<int32_t>(2);
    cs.add<Frame>(1);
    cs.add<float>(fp.inst.size() * H);
    cs.add<float>(H);
    const int fsplits = frame_splits(1, n);
    cs.add<double>(frame_work(1, fsplits));
    LRQO_TRY(ensure_scratch(P, cs.bytes));
    Carve cv(P->scratch);
    FwdBufs b{};
    Upload up;
    b.voff = up.take(cv, &zero, 1);
    b.n = up.take(cv, &n, 1);
    b.inst = up.take(cv, fp.inst.data(), fp.inst.size());
    b.start = up.take(cv, fp.start.data(), fp.start.size());
    b.first = up.take(cv, fp.first.data(), fp.first.size());
    b.frames = cv.take<Frame>(1);
    b.partial = cv.take<float>(fp.inst.size() * H);
    b.mvec = cv.take<float>(H);
    b.fwork = cv.take<double>(frame_work(1, fsplits));
    b.fsplits = fsplits;
    hipStream_t st = current_stream();
    LRQO_TRY(up.send(st));
    LRQO_TRY(run_embed(P, V, 1, fp, b, st));
    const int period = uniform_fraction > 0.0f ? std::max(1, (int)lrintf(1.0f / uniform_fraction)) : 0;
    const unsigned blocks = (unsigned)std::min<int64_t>((S + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_sample, dim3(blocks), dim3(kBlock), 0, st, P->theta, b.mvec, b.frames, S, seed, instance,
                       period, dirs);
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipStreamSynchronize(st));
    return LRQO_OK;
}

lrqo_status lrqo_proposal_frame(lrqo_proposal* P, const float* V, int64_t n, double* frame_out) {
    using namespace lrqo;
    clear_error();
    if (!P || !V || !frame_out) return fail(LRQO_EINVAL, "null pointer argument");
    if (n < 1 || n > (1 << 24)) return fail(LRQO_EINVAL, "n must be in [1, 2^24]");
    if (!is_device_pointer(V)) return fail(LRQO_EINVAL, "V is not device memory");
    const int fsplits = frame_splits(1, n);
    CarveSize cs;
    cs.add<int64_t>(2);
    cs.add<Frame>(1);
    cs.add<double>(frame_work(1, fsplits));
    LRQO_TRY(ensure_scratch(P, cs.bytes));
    Carve cv(P->scratch);
    int64_t* d = cv.take<int64_t>(2);
    Frame* fr = cv.take<Frame>(1);
    double* work = cv.take<double>(frame_work(1, fsplits));
    const int64_t h[2] = {0, n};
    hipStream_t st = current_stream();
    LRQO_HIP(hipMemcpyAsync(d, h, sizeof h, hipMemcpyHostToDevice, st));
    launch_frames(V, d, d + 1, 1, fsplits, P->K, fr, work, st);
    LRQO_HIP(hipGetLastError());
    Frame hf;
    LRQO_HIP(hipMemcpyAsync(&hf, fr, sizeof hf, hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipStreamSynchronize(st));
    for (int e = 0; e < 18; ++e) frame_out[e] = hf.g[e];
    frame_out[18] = hf.s;
    return LRQO_OK;
}

}  // extern "C"
