// Spectral truncation (the step before the path): the r largest eigenpairs of
// a Hermitian operator by Lanczos with full reorthogonalisation in FP64, and
// the factor V = U diag(sqrt(lambda)) the solvers take.
//
// Operators:
//   Laplacian    L = D - A of a CSR graph (as for Max-K-Cut, Sec. 5):
//                y_i = sum_j w_ij (x_i - x_j)
//   phase sync   Q = U U^H + sigma W with W Hermitian Gaussian regenerated
//                on the fly from a counter-based definition (for i <= j,
//                Philox4x32-10 with key seed and counter (i, j >> 1,
//                0x57484D41, 0); words (x, y) for even j, (z, w) for odd j;
//                off-diagonal sqrt(-log u0) e^{2 pi i u1}, conjugated below
//                the diagonal; diagonal sqrt(-2 log u0) cos 2 pi u1), so the
//                n x n matrix is never stored; each upper-triangle entry is
//                generated once per product and serves its row and column
//
// Per Lanczos step j (basis columns q_0..q_j in HBM, column-major):
//   w = A q_j; h = Q^H w (alpha_j = Re h_j); w -= Q h; a second pass of the
//   same (classical Gram-Schmidt, twice); beta_j = ||w||; q_{j+1} = w/beta_j.
// alpha and beta are written on the device; the host reads them only at the
// checks.  Every check interval one block finds the r largest eigenvalues of the
// tridiagonal T_j by Sturm bisection and their vectors by inverse iteration;
// |beta_j s_{j,k}| bounds the residual of Ritz pair k.  At convergence the
// Ritz vectors U = Q S are formed, each is rotated so that its
// largest-modulus entry is real positive, and scaled by sqrt(max(theta, 0)).
// All sums are fixed-order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "graph_internal.h"
#include "lrqo_device.h"
#include "lrqo_runtime.h"

namespace lrqo {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kWStream = 0x57484D41u;
constexpr int kMaxIter = 2000;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) b
__device__ __forceinline__ double2 cdot1(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ void block_sum2(double& a, double& b) {
    __shared__ double sa[kBlock], sb[kBlock];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (unsigned h = kBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sa[threadIdx.x] += sa[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
    __syncthreads();
}

// ---------------------------------------------------------------- operators
struct LapOp {
    const int64_t* row_ptr;
    const int32_t* col;
    const double* w;
    int64_t n;
};

// The entries [e, e1) of a row in chunks of U: the U column and weight
// loads, then the U gathers of x, are issued together; the additions keep
// entry order.  Leaves e at the first entry of an incomplete chunk.
template <int U>
__device__ __forceinline__ void lap_chunk(const LapOp& g, const double2* __restrict__ x, int64_t& e, int64_t e1,
                                          double& ar, double& ai, double& deg) {
    for (; e + U <= e1; e += U) {
        int32_t c[U];
        double w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = g.col[e + u];
            w[u] = g.w ? g.w[e + u] : 1.0;
        }
        double2 xj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xj[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ar += w[u] * xj[u].x;
            ai += w[u] * xj[u].y;
            deg += w[u];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_apply_lap(LapOp g, const double2* __restrict__ x, double2* __restrict__ y) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= g.n) return;
    const double2 xi = x[i];
    double ar = 0.0, ai = 0.0, deg = 0.0;
    int64_t e = g.row_ptr[i];
    const int64_t e1 = g.row_ptr[i + 1];
    lap_chunk<8>(g, x, e, e1, ar, ai, deg);
    lap_chunk<4>(g, x, e, e1, ar, ai, deg);
    for (; e < e1; ++e) {
        const double w = g.w ? g.w[e] : 1.0;
        const double2 xj = x[g.col[e]];
        ar += w * xj.x;
        ai += w * xj.y;
        deg += w;
    }
    y[i] = make_double2(deg * xi.x - ar, deg * xi.y - ai);
}

struct PhaseOp {
    const double2* U;      // n x p row-major
    int p;
    double sigma;
    uint64_t seed;
    int64_t n;
};

// W entries in FP32 from the words of one Philox call, with the hardware
// transcendentals: v_log_f32 is log2, v_sin_f32 / v_cos_f32 take the angle in
// turns (sin 2 pi u).  u >= 2^-24 is never denormal, so none of the library
// range reductions is needed.
constexpr float kLn2 = 0.693147180559945309f;

__device__ __forceinline__ float unit_from_bits(uint32_t x) {
    // ((x >> 9) + 1/2) 2^-23, exact: one rounding of an exact value
    return __builtin_fmaf(static_cast<float>(x >> 9), 0x1p-23f, 0x1p-24f);
}
// sqrt(-log u0) e^{2 pi i u1}
__device__ __forceinline__ float2 w_off(uint32_t a, uint32_t b) {
    const float u0 = unit_from_bits(a), u1 = unit_from_bits(b);
    const float rad = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(u0) * -kLn2);
    return make_float2(rad * __builtin_amdgcn_cosf(u1), rad * __builtin_amdgcn_sinf(u1));
}
// sqrt(-2 log u0) cos 2 pi u1
__device__ __forceinline__ float w_diag(uint32_t a, uint32_t b) {
    const float u0 = unit_from_bits(a), u1 = unit_from_bits(b);
    return __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(u0) * (-2.0f * kLn2)) * __builtin_amdgcn_cosf(u1);
}

// One entry (row i, column j, i <= j) of the upper triangle against the
// tile's x_j (row use) and, off the diagonal, conj(W_ij) x_i into the
// column accumulator ca.
__device__ __forceinline__ void w_use(float2 e, double2 xj, double2 xi, double& ar, double& ai, double2& ca) {
    const double wr = (double)e.x, wi = (double)e.y;
    ar = __builtin_fma(-wi, xj.y, __builtin_fma(wr, xj.x, ar));
    ai = __builtin_fma(wi, xj.x, __builtin_fma(wr, xj.y, ai));
    ca.x = __builtin_fma(wi, xi.y, __builtin_fma(wr, xi.x, ca.x));
    ca.y = __builtin_fma(-wi, xi.x, __builtin_fma(wr, xi.y, ca.y));
}

// Symmetric form of sigma W x: every entry of the upper triangle is
// generated once and used for its row and, conjugated, for its column.
// Rows come in stripes of kSymT = 256 (one block); a work item is stripe I
// against a chunk of up to kSymChunk column stripes J >= I.  Columns are
// taken in pairs (2q, 2q + 1), the two entries of one Philox call.  Lane l
// of wave w (row I*256 + 64w + l) visits pair (l + s) mod 128 of tile J at
// step s, so the 64 lanes of a wave touch 128 different columns at every
// step and each wave adds its column contributions into its own LDS row of
// cacc in a fixed order; the four waves' sums are added in wave order.
// Tiles off the diagonal and inside the matrix need no per-entry test.
// Outputs:
//   rowpart[item][t]        row sums of the item's tiles
//   colpart[tri(J, I)][t]   column sums of tile (I, J), tri(J, I) = J(J+1)/2 + I
// and k_w_combine adds, for row stripe I, the row sums of its items and the
// column sums of the tiles (I', I), I' <= I, in that order.
constexpr int kSymT = 256;
constexpr int kSymPairs = kSymT / 2;
constexpr int kSymChunk = 8;

__device__ __forceinline__ int64_t tri_index(int64_t J, int64_t I) { return J * (J + 1) / 2 + I; }

__global__ __launch_bounds__(kSymT) void k_w_tiles(PhaseOp o, const double2* __restrict__ x,
                                                   const int2* __restrict__ items, int64_t P,
                                                   double2* __restrict__ rowpart, double2* __restrict__ colpart) {
    __shared__ double2 xs[kSymT];
    __shared__ double2 cacc[kSymT / kWave][kSymT];
    const int2 item = items[blockIdx.x];
    const int64_t I = item.x;
    const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
    const int64_t i = I * kSymT + t;
    const bool live = i < o.n;
    const uint32_t iu = static_cast<uint32_t>(i);
    const uint32_t k0 = static_cast<uint32_t>(o.seed), k1 = static_cast<uint32_t>(o.seed >> 32);
    const double2 xi = live ? x[i] : make_double2(0.0, 0.0);
    double ar = 0.0, ai = 0.0;
    const int64_t J0 = I + (int64_t)item.y * kSymChunk, J1 = min(P, J0 + kSymChunk);
    for (int64_t J = J0; J < J1; ++J) {
        __syncthreads();
        const int64_t jt = J * kSymT + t;
        xs[t] = jt < o.n ? x[jt] : make_double2(0.0, 0.0);
#pragma unroll
        for (int v = 0; v < kSymT / kWave; ++v) cacc[v][t] = make_double2(0.0, 0.0);
        __syncthreads();
        const uint32_t qbase = static_cast<uint32_t>(J * kSymPairs);
        if (J != I && (J + 1) * kSymT <= o.n) {
            // J > I, so stripe I is full as well: every entry is strictly
            // above the diagonal and inside the matrix
            for (int st = 0; st < kSymPairs; ++st) {
                const int q = (lane + st) & (kSymPairs - 1);
                const U4 h = philox4x32_10(U4{iu, qbase + q, kWStream, 0u}, k0, k1);
                double2 c0 = cacc[wv][2 * q], c1 = cacc[wv][2 * q + 1];
                w_use(w_off(h.x, h.y), xs[2 * q], xi, ar, ai, c0);
                w_use(w_off(h.z, h.w), xs[2 * q + 1], xi, ar, ai, c1);
                cacc[wv][2 * q] = c0;
                cacc[wv][2 * q + 1] = c1;
                // the next step's lane l reads the pair lane l+1 wrote now
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        } else if (live) {
            // diagonal tile or the last, partial column stripe
            for (int st = 0; st < kSymPairs; ++st) {
                const int q = (lane + st) & (kSymPairs - 1);
                const int64_t j0 = J * kSymT + 2 * q;
                if (j0 + 1 >= i && j0 < o.n) {
                    const U4 h = philox4x32_10(U4{iu, qbase + q, kWStream, 0u}, k0, k1);
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int64_t j = j0 + e;
                        if (j < i || j >= o.n) continue;
                        const uint32_t a = e ? h.z : h.x, b = e ? h.w : h.y;
                        const double2 xj = xs[2 * q + e];
                        if (j == i) {
                            const double d = (double)w_diag(a, b);
                            ar = __builtin_fma(d, xj.x, ar);
                            ai = __builtin_fma(d, xj.y, ai);
                        } else {
                            double2 c = cacc[wv][2 * q + e];
                            w_use(w_off(a, b), xj, xi, ar, ai, c);
                            cacc[wv][2 * q + e] = c;
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        double2 cs = cacc[0][t];
#pragma unroll
        for (int v = 1; v < kSymT / kWave; ++v) {
            cs.x += cacc[v][t].x;
            cs.y += cacc[v][t].y;
        }
        colpart[tri_index(J, I) * kSymT + t] = cs;
    }
    rowpart[(int64_t)blockIdx.x * kSymT + t] = make_double2(ar, ai);
}

// y_i = sum_k U_ik c_k + sigma (row sums of the items of stripe I + column
// sums of tiles (I', I), I' <= I); item_first[I] = first item of stripe I.
__global__ __launch_bounds__(kSymT) void k_w_combine(PhaseOp o, const double2* __restrict__ c,
                                                     const int32_t* __restrict__ item_first, int64_t P,
                                                     const double2* __restrict__ rowpart,
                                                     const double2* __restrict__ colpart, double2* __restrict__ y) {
    const int64_t I = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t i = I * kSymT + t;
    if (i >= o.n) return;
    double ar = 0.0, ai = 0.0;
    for (int32_t it = item_first[I]; it < item_first[I + 1]; ++it) {
        const double2 v = rowpart[(int64_t)it * kSymT + t];
        ar += v.x;
        ai += v.y;
    }
    for (int64_t Ip = 0; Ip <= I; ++Ip) {
        const double2 v = colpart[tri_index(I, Ip) * kSymT + t];
        ar += v.x;
        ai += v.y;
    }
    double yr = o.sigma * ar, yi = o.sigma * ai;
    for (int k = 0; k < o.p; ++k) {
        const double2 u = cmul(o.U[i * o.p + k], c[k]);
        yr += u.x;
        yi += u.y;
    }
    y[i] = make_double2(yr, yi);
    (void)P;
}

// ---------------------------------------------------------------- basis algebra
// h_j = q_j^H w for j < k in two fixed-order stages.  Block (b, c) takes
// rows [b rows, (b + 1) rows) of columns kDotCols c .. kDotCols c + 7 (rows a
// multiple of 256, sized on the host for at least 256 row chunks up to 4096):
// each thread sums its rows (two rows' loads in flight), the 16 sums of a
// wave are added by a transposing butterfly (each exchange halves the
// values a lane holds: 17 shuffles instead of 16 x 6) and the four waves in
// order, giving part[j nb + b]; k_part_sum then adds the nb partials of
// column j (lanes strided, then butterfly).  Q is read once, by as many
// blocks as there are row chunks times column groups.
constexpr int kDotRowsMax = 4096;
constexpr int kDotCols = 8;

int dot_rows(int64_t n) {
    int64_t rows = ((n + 255) / 256 + 255) / 256 * 256;
    return (int)std::min<int64_t>(std::max<int64_t>(rows, 256), kDotRowsMax);
}

// Wave sums of the 16 values acc[0..15]: at the exchange with lane
// distance o = 32, 16, 8, 4 a lane keeps one half of its values (the upper
// one when its bit o is set) and adds its partner's copy of that half; the
// one value left, index lane / 4, is then summed over the four lanes of the
// group.  Returns the wave sum of value lane / 4 (the same in those lanes).
static_assert(2 * kDotCols == 16 && kWave == 64, "the exchange pattern is for 16 values on 64 lanes");
__device__ __forceinline__ double wave_sums16(double (&v)[16]) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int o = 32 >> st, h = 8 >> st;
        const bool hi = (lane & o) != 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k < h) {
                const double send = hi ? v[k] : v[k + h];
                const double keep = hi ? v[k + h] : v[k];
                v[k] = keep + __shfl_xor(send, o, kWave);
            }
        }
    }
    double r = v[0];
    r += __shfl_xor(r, 2, kWave);
    r += __shfl_xor(r, 1, kWave);
    return r;
}

__device__ __forceinline__ void block_sums_to(double (&acc)[2 * kDotCols], int count, double* dst, int64_t stride) {
    __shared__ double red[kBlock / kWave][2 * kDotCols];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const double v = wave_sums16(acc);
    if ((lane & 3) == 0) red[wv][lane >> 2] = v;
    __syncthreads();
    if ((int)threadIdx.x < 2 * count) {
        double v = red[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < kBlock / kWave; ++q) v += red[q][threadIdx.x];
        dst[(int64_t)(threadIdx.x >> 1) * stride + (threadIdx.x & 1)] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_dots_part(const double2* __restrict__ Q, int64_t n,
                                                      const double2* __restrict__ w, int k, int rows, int nb,
                                                      double2* __restrict__ part) {
    const int b = blockIdx.x, j0 = blockIdx.y * kDotCols;
    const int nc = min(kDotCols, k - j0);
    const int64_t i0 = (int64_t)b * rows, i1 = min(n, i0 + rows);
    double acc[2 * kDotCols];
#pragma unroll
    for (int e = 0; e < 2 * kDotCols; ++e) acc[e] = 0.0;
    int64_t i = i0 + threadIdx.x;
    // two rows' loads in flight; each column's sum still runs in row order
    for (; i + kBlock < i1; i += 2 * kBlock) {
        const double2 wa = w[i], wb = w[i + kBlock];
        double2 qa[kDotCols], qb[kDotCols];
#pragma unroll
        for (int c = 0; c < kDotCols; ++c) {
            if (c < nc) {
                qa[c] = Q[(int64_t)(j0 + c) * n + i];
                qb[c] = Q[(int64_t)(j0 + c) * n + i + kBlock];
            }
        }
#pragma unroll
        for (int c = 0; c < kDotCols; ++c) {
            if (c < nc) {                                            // conj(q) w
                acc[2 * c] = __builtin_fma(qa[c].y, wa.y, __builtin_fma(qa[c].x, wa.x, acc[2 * c]));
                acc[2 * c + 1] = __builtin_fma(-qa[c].y, wa.x, __builtin_fma(qa[c].x, wa.y, acc[2 * c + 1]));
                acc[2 * c] = __builtin_fma(qb[c].y, wb.y, __builtin_fma(qb[c].x, wb.x, acc[2 * c]));
                acc[2 * c + 1] = __builtin_fma(-qb[c].y, wb.x, __builtin_fma(qb[c].x, wb.y, acc[2 * c + 1]));
            }
        }
    }
    for (; i < i1; i += kBlock) {
        const double2 wi = w[i];
#pragma unroll
        for (int c = 0; c < kDotCols; ++c) {
            if (c < nc) {
                const double2 q = Q[(int64_t)(j0 + c) * n + i];      // conj(q) w
                acc[2 * c] = __builtin_fma(q.y, wi.y, __builtin_fma(q.x, wi.x, acc[2 * c]));
                acc[2 * c + 1] = __builtin_fma(-q.y, wi.x, __builtin_fma(q.x, wi.y, acc[2 * c + 1]));
            }
        }
    }
    block_sums_to(acc, nc, reinterpret_cast<double*>(part + (int64_t)j0 * nb + b), 2 * (int64_t)nb);
}

// part[k nb + b] = sum over rows of chunk b of conj(U_ik) x_i, k < p
// (U row-major n x p, p <= 8)
__global__ __launch_bounds__(kBlock) void k_utx_part(PhaseOp o, const double2* __restrict__ x, int rows, int nb,
                                                     double2* __restrict__ part) {
    const int b = blockIdx.x;
    const int64_t i0 = (int64_t)b * rows, i1 = min(o.n, i0 + rows);
    double acc[2 * kDotCols];
#pragma unroll
    for (int e = 0; e < 2 * kDotCols; ++e) acc[e] = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const double2 xi = x[i];
#pragma unroll
        for (int c = 0; c < kDotCols; ++c) {
            if (c < o.p) {
                const double2 u = o.U[i * o.p + c];
                acc[2 * c] = __builtin_fma(u.y, xi.y, __builtin_fma(u.x, xi.x, acc[2 * c]));
                acc[2 * c + 1] = __builtin_fma(-u.y, xi.x, __builtin_fma(u.x, xi.y, acc[2 * c + 1]));
            }
        }
    }
    block_sums_to(acc, o.p, reinterpret_cast<double*>(part + b), 2 * (int64_t)nb);
}

// h_j = sum_b part[j nb + b], one wave per column; Re h of the last column
// also into last_re[0] when given
__global__ __launch_bounds__(kWave) void k_part_sum(const double2* __restrict__ part, int nb,
                                                    double2* __restrict__ h, double* __restrict__ last_re) {
    const int j = blockIdx.x;
    double ar = 0.0, ai = 0.0;
    for (int b = threadIdx.x; b < nb; b += kWave) {
        const double2 v = part[(int64_t)j * nb + b];
        ar += v.x;
        ai += v.y;
    }
    ar = wave_sum_f64(ar);
    ai = wave_sum_f64(ai);
    if (threadIdx.x == 0) {
        h[j] = make_double2(ar, ai);
        if (last_re && j == (int)gridDim.x - 1) last_re[0] = ar;
    }
}

// w -= sum_{j<k} q_j h_j
__global__ __launch_bounds__(kBlock) void k_sub(const double2* __restrict__ Q, int64_t n, int k,
                                                const double2* __restrict__ h, double2* __restrict__ w) {
    __shared__ double2 hs[kMaxIter + 1];
    for (int j = threadIdx.x; j < k; j += kBlock) hs[j] = h[j];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    double ar = 0.0, ai = 0.0;
    // eight column loads in flight per thread, the sum still in column order
    constexpr int U = 8;
    int j = 0;
    for (; j + U <= k; j += U) {
        double2 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = Q[(int64_t)(j + u) * n + i];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double2 t = cmul(q[u], hs[j + u]);
            ar += t.x;
            ai += t.y;
        }
    }
    for (; j < k; ++j) {
        const double2 t = cmul(Q[(int64_t)j * n + i], hs[j]);
        ar += t.x;
        ai += t.y;
    }
    const double2 wi = w[i];
    w[i] = make_double2(wi.x - ar, wi.y - ai);
}

__global__ __launch_bounds__(kBlock) void k_norm_part(const double2* __restrict__ w, int64_t n, double* __restrict__ part) {
    double a = 0.0, b = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double2 t = w[i];
        a += t.x * t.x + t.y * t.y;
    }
    block_sum2(a, b);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

// out[0] = sqrt(sum of the partials); also into copy[0] when given
__global__ __launch_bounds__(kBlock) void k_norm_final(const double* __restrict__ part, int count, double* __restrict__ out,
                                                       double* __restrict__ copy) {
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < count; t += kBlock) a += part[t];
    block_sum2(a, b);
    if (threadIdx.x == 0) {
        out[0] = sqrt(a);
        if (copy) copy[0] = sqrt(a);
    }
}

// q = w / nrm (nrm read on the device)
__global__ __launch_bounds__(kBlock) void k_scale(const double2* __restrict__ w, int64_t n, const double* __restrict__ nrm,
                                                  double2* __restrict__ q) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    // a zero vector (breakdown, found by the host at the next check) stays zero
    const double inv = nrm[0] > 0.0 ? 1.0 / nrm[0] : 0.0;
    const double2 t = w[i];
    q[i] = make_double2(t.x * inv, t.y * inv);
}

// start vector: standard complex Gaussian entries from the Philox stream
// (key seed, counter (i lo, i hi, 0x5354524C, 0)), normalised afterwards
__global__ __launch_bounds__(kBlock) void k_start(int64_t n, uint64_t seed, double2* __restrict__ w) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    const U4 o = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), 0x5354524Cu, 0u}, (uint32_t)seed,
                               (uint32_t)(seed >> 32));
    const double u0 = ((double)(o.x >> 9) + 0.5) * 0x1p-23, u1 = ((double)(o.y >> 9) + 0.5) * 0x1p-23;
    const double rad = sqrt(-2.0 * log(u0));
    w[i] = make_double2(rad * cos(2.0 * 3.141592653589793 * u1), rad * sin(2.0 * 3.141592653589793 * u1));
}

// ---------------------------------------------------------------- tridiagonal
// Number of eigenvalues of T (diagonal a, squared off-diagonal bb) below x
// (Sturm sequence of the pivots of T - x I).
__device__ __forceinline__ int sturm_below(const double* a, const double* bb, int m, double x) {
    int cnt = 0;
    double d = a[0] - x;
    if (d == 0.0) d = -1e-300;
    cnt += d < 0.0;
    for (int i = 1; i < m; ++i) {
        d = a[i] - x - bb[i - 1] / d;
        if (d == 0.0) d = -1e-300;
        cnt += d < 0.0;
    }
    return cnt;
}

// Top r eigenpairs of the m x m tridiagonal T (diagonal a, off-diagonal b).
// a, b and b^2 are staged in LDS.  Eigenvalue t (the t-th largest, ascending
// index k = m-1-t) is found by wave t mod 4 by multisection: the 64 lanes
// count the eigenvalues below 64 interior points of the bracket, and the
// first point whose count exceeds k becomes the upper end (a factor of 65
// per round).  Thread t < r then computes the unit vector by inverse
// iteration on T - mu I, mu just off theta (one elimination with partial
// pivoting, three solves); wave 0 orthonormalises the r vectors in order
// (two Gram-Schmidt passes, lane-strided dots added by butterfly) and forms
// the residual bounds |b_last s_{m-1,t}|.  S is m x r column-major; the
// elimination works in LDS for m <= kTriLds, else in `work`.
constexpr int kTriThreads = 256;
constexpr int kTriLds = 224;

__global__ __launch_bounds__(kTriThreads) void k_tridiag_top(const double* __restrict__ a_g,
                                                             const double* __restrict__ b_g, int m, int r,
                                                             double b_last, double* __restrict__ theta,
                                                             double* __restrict__ S, double* __restrict__ resid,
                                                             double* __restrict__ work) {
    __shared__ double a[kMaxIter + 1], b[kMaxIter + 1], bb[kMaxIter + 1];
    __shared__ double wl[LRQO_MAX_R][6 * kTriLds];
    __shared__ double red_lo[kTriThreads / kWave], red_hi[kTriThreads / kWave];
    __shared__ double th_s[LRQO_MAX_R];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    double lo = INFINITY, hi = -INFINITY;
    for (int i = tid; i < m; i += kTriThreads) {
        const double ai = a_g[i], bi = i + 1 < m ? b_g[i] : 0.0, bp = i ? b_g[i - 1] : 0.0;
        a[i] = ai;
        b[i] = bi;
        bb[i] = bi * bi;
        const double rad = fabs(bp) + fabs(bi);           // Gershgorin disc of row i
        lo = fmin(lo, ai - rad);
        hi = fmax(hi, ai + rad);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, kWave));
        hi = fmax(hi, __shfl_xor(hi, off, kWave));
    }
    if (lane == 0) {
        red_lo[wv] = lo;
        red_hi[wv] = hi;
    }
    __syncthreads();
    lo = red_lo[0];
    hi = red_hi[0];
#pragma unroll
    for (int q = 1; q < kTriThreads / kWave; ++q) {
        lo = fmin(lo, red_lo[q]);
        hi = fmax(hi, red_hi[q]);
    }
    const double span = fmax(hi - lo, 1e-300);
    lo -= 1e-12 * span;
    hi += 1e-12 * span;
    for (int t = wv; t < r; t += kTriThreads / kWave) {
        const int k = m - 1 - t;
        double l0 = lo, h0 = hi;
        for (int round = 0; round < 40 && h0 - l0 > 4e-16 * fmax(fabs(l0), fabs(h0)); ++round) {
            const double step = (h0 - l0) / 65.0;
            const bool above = sturm_below(a, bb, m, l0 + step * (double)(lane + 1)) > k;
            const unsigned long long mask = __ballot(above);
            const int first = mask ? __ffsll(mask) - 1 : kWave;
            const double nh = first < kWave ? l0 + step * (double)(first + 1) : h0;
            l0 = first > 0 ? l0 + step * (double)first : l0;
            h0 = nh;
        }
        if (lane == 0) {
            th_s[t] = 0.5 * (l0 + h0);
            theta[t] = th_s[t];
        }
    }
    __syncthreads();
    if (tid < r) {
        const int t = tid;
        const double mu = th_s[t] + 1e-13 * span;
        double* base = m <= kTriLds ? &wl[t][0] : work + (size_t)t * 6 * m;
        const int ld = m <= kTriLds ? kTriLds : m;
        double* rd0 = base;                       // reciprocal pivots
        double* d1 = base + ld;                   // first superdiagonal
        double* d2 = base + 2 * ld;               // second superdiagonal (fill-in)
        double* lm = base + 3 * ld;               // multipliers
        double* pv = base + 4 * ld;               // 1 where rows i, i+1 were swapped
        double* x = base + 5 * ld;
        // eliminate once: rows i, i+1 with partial pivoting
        double cd = a[0] - mu, cu = m > 1 ? b[0] : 0.0;
        for (int i = 0; i + 1 < m; ++i) {
            const double nl = b[i], nd = a[i + 1] - mu, nu = i + 2 < m ? b[i + 1] : 0.0;
            if (fabs(nl) > fabs(cd)) {            // swap rows i and i+1
                const double l = cd / nl;
                rd0[i] = 1.0 / nl;
                d1[i] = nd;
                d2[i] = nu;
                lm[i] = l;
                pv[i] = 1.0;
                cd = cu - l * nd;
                cu = -l * nu;
            } else {
                const double piv = cd != 0.0 ? cd : 1e-300;
                const double l = nl / piv;
                rd0[i] = 1.0 / piv;
                d1[i] = cu;
                d2[i] = 0.0;
                lm[i] = l;
                pv[i] = 0.0;
                cd = nd - l * cu;
                cu = nu;
            }
        }
        rd0[m - 1] = 1.0 / (cd != 0.0 ? cd : 1e-300);
        d1[m - 1] = 0.0;
        d2[m - 1] = 0.0;
        for (int i = 0; i < m; ++i) x[i] = 1.0 + 0.001 * (double)((i * 7919 + t * 104729) % 97);
        if (m == 1) x[0] = 1.0;                   // the 1 x 1 case needs no solve
        for (int iter = 0; iter < (m > 1 ? 3 : 0); ++iter) {
            for (int i = 0; i + 1 < m; ++i) {
                if (pv[i] != 0.0) {
                    const double tmp = x[i];
                    x[i] = x[i + 1];
                    x[i + 1] = tmp;
                }
                x[i + 1] -= lm[i] * x[i];
            }
            double x1 = 0.0, x2 = 0.0, nrm = 0.0;   // x[i+1], x[i+2]
            for (int i = m - 1; i >= 0; --i) {
                const double v = (x[i] - d1[i] * x1 - d2[i] * x2) * rd0[i];
                x[i] = v;
                x2 = x1;
                x1 = v;
                nrm += v * v;
            }
            const double inv = 1.0 / sqrt(nrm);
            for (int i = 0; i < m; ++i) x[i] *= inv;
        }
        for (int i = 0; i < m; ++i) S[(size_t)t * m + i] = x[i];
    }
    __syncthreads();
    if (wv == 0) {
        for (int u = 0; u < r; ++u) {
            double* su = S + (size_t)u * m;
            for (int pass = 0; pass < 2; ++pass)
                for (int v = 0; v < u; ++v) {
                    const double* sv = S + (size_t)v * m;
                    double d = 0.0;
                    for (int i = lane; i < m; i += kWave) d += sv[i] * su[i];
                    d = wave_sum_f64(d);
                    for (int i = lane; i < m; i += kWave) su[i] -= d * sv[i];
                }
            double nrm = 0.0;
            for (int i = lane; i < m; i += kWave) nrm += su[i] * su[i];
            nrm = wave_sum_f64(nrm);
            const double inv = 1.0 / sqrt(nrm);
            for (int i = lane; i < m; i += kWave) {
                su[i] *= inv;
                if (i == m - 1) resid[u] = fabs(b_last * su[i]);
            }
        }
    }
}

// U = Q S (n x r), S m x r column-major
__global__ __launch_bounds__(kBlock) void k_ritz(const double2* __restrict__ Q, int64_t n, int m, int r,
                                                 const double* __restrict__ S, double2* __restrict__ Uo) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    double ar[LRQO_MAX_R], ai[LRQO_MAX_R];
#pragma unroll
    for (int k = 0; k < LRQO_MAX_R; ++k) ar[k] = ai[k] = 0.0;
    for (int j = 0; j < m; ++j) {          // the basis is read once
        const double2 q = Q[(int64_t)j * n + i];
#pragma unroll
        for (int k = 0; k < LRQO_MAX_R; ++k) {
            if (k < r) {
                const double s = S[(size_t)k * m + j];
                ar[k] += q.x * s;
                ai[k] += q.y * s;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < LRQO_MAX_R; ++k)
        if (k < r) Uo[i * r + k] = make_double2(ar[k], ai[k]);
}

// per block: (max |u_ik|^2, lowest index) for each column k
__global__ __launch_bounds__(kBlock) void k_colmax(const double2* __restrict__ Uo, int64_t n, int r,
                                                   double* __restrict__ pmax, int64_t* __restrict__ pidx) {
    __shared__ double sm[kBlock];
    __shared__ int64_t si[kBlock];
    for (int k = 0; k < r; ++k) {
        double best = -1.0;
        int64_t bi = INT64_MAX;
        for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
            const double2 u = Uo[i * r + k];
            const double v = u.x * u.x + u.y * u.y;
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        sm[threadIdx.x] = best;
        si[threadIdx.x] = bi;
        __syncthreads();
        for (unsigned h = kBlock / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                const double o = sm[threadIdx.x + h];
                const int64_t oi = si[threadIdx.x + h];
                if (o > sm[threadIdx.x] || (o == sm[threadIdx.x] && oi < si[threadIdx.x])) {
                    sm[threadIdx.x] = o;
                    si[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            pmax[(size_t)blockIdx.x * r + k] = sm[0];
            pidx[(size_t)blockIdx.x * r + k] = si[0];
        }
        __syncthreads();
    }
}

// phase of each column from the block partials (one block, thread k):
// ph_k = conj(u) / |u| sqrt(max(theta_k, 0)) at the column's largest entry
__global__ void k_phase(const double2* __restrict__ Uo, int r, int parts, const double* __restrict__ pmax,
                        const int64_t* __restrict__ pidx, const double* __restrict__ theta,
                        double2* __restrict__ ph) {
    if ((int)threadIdx.x < r) {
        const int k = threadIdx.x;
        double best = -1.0;
        int64_t bi = INT64_MAX;
        for (int p = 0; p < parts; ++p) {
            const double v = pmax[(size_t)p * r + k];
            const int64_t vi = pidx[(size_t)p * r + k];
            if (v > best || (v == best && vi < bi)) {
                best = v;
                bi = vi;
            }
        }
        const double2 u = Uo[bi * r + k];
        const double mod = sqrt(u.x * u.x + u.y * u.y);
        const double sc = sqrt(fmax(theta[k], 0.0)) / (mod > 0.0 ? mod : 1.0);
        ph[k] = make_double2(u.x * sc, -u.y * sc);
    }
}

// V = U ph (column k times ph_k)
__global__ __launch_bounds__(kBlock) void k_factor(const double2* __restrict__ Uo, int64_t n, int r,
                                                   const double2* __restrict__ ph, double2* __restrict__ V) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < r; ++k) V[i * r + k] = cmul(Uo[i * r + k], ph[k]);
}

enum OpKind { kOpLap = 0, kOpPhase = 1 };

lrqo_status lanczos_factor(int kind, const LapOp& lap, const PhaseOp& ph, int64_t n, int r,
                           const lrqo_eigs_options* opt, double* Vout, lrqo_eigs_result* res) {
    lrqo_eigs_options o{};
    if (opt) o = *opt;
    if (o.max_iter < 0 || o.max_iter > kMaxIter) return fail(LRQO_EINVAL, "max_iter must be in [0, 2000]");
    if (o.check_every < 0) return fail(LRQO_EINVAL, "check_every must be >= 0");
    if (!(o.tol >= 0.0) || o.tol >= 1.0) return fail(LRQO_EINVAL, "tol must be in [0, 1)");
    const int max_iter = (int)std::min<int64_t>(o.max_iter ? o.max_iter : 300, n);
    // a phase-sync product costs n^2/2 entry evaluations, far more than the
    // tridiagonal Ritz step, so that operator is checked after every step
    const int every = o.check_every ? o.check_every : (kind == kOpPhase ? 1 : 10);
    const double tol = o.tol > 0.0 ? o.tol : 1e-10;
    if (max_iter < r) return fail(LRQO_EINVAL, "max_iter (and n) must be at least r");
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const hipStream_t st = current_stream();
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    const int nparts = (int)std::min<int64_t>(blocks, 1024);
    CarveSize cs;
    cs.add<double2>((size_t)n * (max_iter + 1));   // basis
    cs.add<double2>(n);                           // w
    cs.add<double2>(kMaxIter + 1);                // h
    const int drows = dot_rows(n);
    const int nbd = (int)((n + drows - 1) / drows);
    cs.add<double2>((size_t)(kMaxIter + 1) * nbd);  // partial dots
    cs.add<double2>(LRQO_MAX_R);                  // U^H x
    cs.add<double>(nparts);                       // norm partials
    cs.add<double>(4);                            // norm
    cs.add<double>(kMaxIter + 1);                 // alpha
    cs.add<double>(kMaxIter + 1);                 // beta
    cs.add<double>(LRQO_MAX_R);                   // theta
    cs.add<double>(LRQO_MAX_R);                   // resid
    cs.add<double>((size_t)(kMaxIter + 1) * LRQO_MAX_R);       // S
    cs.add<double>((size_t)6 * (kMaxIter + 1) * LRQO_MAX_R);   // tridiagonal work
    cs.add<double2>((size_t)n * r);               // Ritz vectors
    cs.add<double>((size_t)nparts * LRQO_MAX_R);
    cs.add<int64_t>((size_t)nparts * LRQO_MAX_R);
    // symmetric W tiles (phase-sync operator only)
    const int64_t P = (n + kSymT - 1) / kSymT;
    std::vector<int2> items;
    std::vector<int32_t> item_first;
    if (kind == kOpPhase) {
        item_first.reserve(P + 1);
        for (int64_t I = 0; I < P; ++I) {
            item_first.push_back((int32_t)items.size());
            for (int64_t cidx = 0; I + cidx * kSymChunk < P; ++cidx) items.push_back(make_int2((int)I, (int)cidx));
        }
        item_first.push_back((int32_t)items.size());
        cs.add<int2>(items.size());
        cs.add<int32_t>(item_first.size());
        cs.add<double2>(items.size() * (size_t)kSymT);
        cs.add<double2>((size_t)(P * (P + 1) / 2) * kSymT);
    }
    CarveSize hs;
    hs.add<double>(2 * (kMaxIter + 1));
    hs.add<double>(2 * LRQO_MAX_R);
    LRQO_TRY(reserve_arena(ctx, cs.bytes));
    LRQO_TRY(reserve_host(ctx, hs.bytes));
    Carve cv(ctx->arena);
    double2* Q = cv.take<double2>((size_t)n * (max_iter + 1));
    double2* w = cv.take<double2>(n);
    double2* h = cv.take<double2>(kMaxIter + 1);
    double2* dpart = cv.take<double2>((size_t)(kMaxIter + 1) * nbd);
    double2* uc = cv.take<double2>(LRQO_MAX_R);
    double* npart = cv.take<double>(nparts);
    double* nrm = cv.take<double>(4);
    double* alpha = cv.take<double>(kMaxIter + 1);
    double* beta = cv.take<double>(kMaxIter + 1);
    double* theta = cv.take<double>(LRQO_MAX_R);
    double* resid = cv.take<double>(LRQO_MAX_R);
    double* S = cv.take<double>((size_t)(kMaxIter + 1) * LRQO_MAX_R);
    double* work = cv.take<double>((size_t)6 * (kMaxIter + 1) * LRQO_MAX_R);
    double2* Uo = cv.take<double2>((size_t)n * r);
    double* pmax = cv.take<double>((size_t)nparts * LRQO_MAX_R);
    int64_t* pidx = cv.take<int64_t>((size_t)nparts * LRQO_MAX_R);
    int2* d_items = nullptr;
    int32_t* d_first = nullptr;
    double2* rowpart = nullptr;
    double2* colpart = nullptr;
    if (kind == kOpPhase) {
        d_items = cv.take<int2>(items.size());
        d_first = cv.take<int32_t>(item_first.size());
        rowpart = cv.take<double2>(items.size() * (size_t)kSymT);
        colpart = cv.take<double2>((size_t)(P * (P + 1) / 2) * kSymT);
        LRQO_HIP(hipMemcpyAsync(d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, st));
        LRQO_HIP(hipMemcpyAsync(d_first, item_first.data(), sizeof(int32_t) * item_first.size(),
                                hipMemcpyHostToDevice, st));
        LRQO_HIP(hipStreamSynchronize(st));
    }
    Carve hv(ctx->host);
    double* h_ab = hv.take<double>(2 * (kMaxIter + 1));     // alpha then beta
    double* h_tr = hv.take<double>(2 * LRQO_MAX_R);         // theta then resid
    double* h_alpha = h_ab;
    double* h_beta = h_ab + (kMaxIter + 1);

    auto apply = [&](const double2* x, double2* y) -> lrqo_status {
        if (kind == kOpLap) {
            hipLaunchKernelGGL(k_apply_lap, dim3((unsigned)blocks), dim3(kBlock), 0, st, lap, x, y);
        } else {
            if (ph.p > 0) {
                hipLaunchKernelGGL(k_utx_part, dim3(nbd), dim3(kBlock), 0, st, ph, x, drows, nbd, dpart);
                hipLaunchKernelGGL(k_part_sum, dim3(ph.p), dim3(kWave), 0, st, dpart, nbd, uc, nullptr);
            }
            hipLaunchKernelGGL(k_w_tiles, dim3((unsigned)items.size()), dim3(kSymT), 0, st, ph, x, d_items, P,
                               rowpart, colpart);
            hipLaunchKernelGGL(k_w_combine, dim3((unsigned)P), dim3(kSymT), 0, st, ph, uc, d_first, P, rowpart,
                               colpart, y);
        }
        LRQO_HIP(hipGetLastError());
        return LRQO_OK;
    };
    auto normalize_into = [&](double2* dst) -> lrqo_status {
        hipLaunchKernelGGL(k_norm_part, dim3(nparts), dim3(kBlock), 0, st, w, n, npart);
        hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kBlock), 0, st, npart, nparts, nrm, nullptr);
        hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(kBlock), 0, st, w, n, nrm, dst);
        LRQO_HIP(hipGetLastError());
        return LRQO_OK;
    };

    LRQO_HIP(hipEventRecord(ctx->ev_start, st));
    hipLaunchKernelGGL(k_start, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, o.seed, w);
    LRQO_TRY(normalize_into(Q));
    int m = 0;              // Lanczos vectors q_0..q_{m-1} complete, T is m x m
    bool converged = false, breakdown = false;
    // alpha and beta stay on the device; the host reads them at each check,
    // where it also finds a breakdown (the first beta_t not above 1e-13
    // times the largest |alpha_u| + |beta_u|, u <= t) and truncates there
    for (int j = 0; j < max_iter; ++j) {
        double2* qj = Q + (int64_t)j * n;
        LRQO_TRY(apply(qj, w));
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_dots_part, dim3(nbd, (j + kDotCols) / kDotCols), dim3(kBlock), 0, st, Q, n, w,
                               j + 1, drows, nbd, dpart);
            hipLaunchKernelGGL(k_part_sum, dim3(j + 1), dim3(kWave), 0, st, dpart, nbd, h,
                               pass == 0 ? alpha + j : nullptr);
            hipLaunchKernelGGL(k_sub, dim3((unsigned)blocks), dim3(kBlock), 0, st, Q, n, j + 1, h, w);
        }
        hipLaunchKernelGGL(k_norm_part, dim3(nparts), dim3(kBlock), 0, st, w, n, npart);
        hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kBlock), 0, st, npart, nparts, nrm, beta + j);
        LRQO_HIP(hipGetLastError());
        m = j + 1;
        const bool check = m >= r && (m % every == 0 || j + 1 == max_iter || m == n);
        if (check) {
            LRQO_HIP(hipMemcpyAsync(h_alpha, alpha, sizeof(double) * m, hipMemcpyDeviceToHost, st));
            LRQO_HIP(hipMemcpyAsync(h_beta, beta, sizeof(double) * m, hipMemcpyDeviceToHost, st));
            LRQO_HIP(hipStreamSynchronize(st));
            double amax = 0.0;
            for (int t = 0; t < m; ++t) {
                amax = std::max(amax, std::fabs(h_alpha[t]) + std::fabs(h_beta[t]));
                if (!(h_beta[t] > 1e-13 * amax)) {
                    m = t + 1;
                    breakdown = true;
                    break;
                }
            }
            breakdown = breakdown || m == n;
            if (m < r) break;
            hipLaunchKernelGGL(k_tridiag_top, dim3(1), dim3(kTriThreads), 0, st, alpha, beta, m, r,
                               breakdown ? 0.0 : h_beta[m - 1], theta, S, resid, work);
            LRQO_HIP(hipGetLastError());
            LRQO_HIP(hipMemcpyAsync(h_tr, theta, sizeof(double) * r, hipMemcpyDeviceToHost, st));
            LRQO_HIP(hipMemcpyAsync(h_tr + LRQO_MAX_R, resid, sizeof(double) * r, hipMemcpyDeviceToHost, st));
            LRQO_HIP(hipStreamSynchronize(st));
            const double scale = std::max(std::fabs(h_tr[0]), 1e-300);
            converged = true;
            for (int k = 0; k < r; ++k) converged &= h_tr[LRQO_MAX_R + k] <= tol * scale;
            if (converged || breakdown) break;
        }
        hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(kBlock), 0, st, w, n, nrm,
                           Q + (int64_t)(j + 1) * n);
        LRQO_HIP(hipGetLastError());
    }
    if (m < r) return fail(LRQO_EINVAL, "the Krylov space is smaller than r (graph or operator too small)");
    hipLaunchKernelGGL(k_ritz, dim3((unsigned)blocks), dim3(kBlock), 0, st, Q, n, m, r, S, Uo);
    hipLaunchKernelGGL(k_colmax, dim3(nparts), dim3(kBlock), 0, st, Uo, n, r, pmax, pidx);
    hipLaunchKernelGGL(k_phase, dim3(1), dim3(64), 0, st, Uo, r, nparts, pmax, pidx, theta, uc);
    hipLaunchKernelGGL(k_factor, dim3((unsigned)blocks), dim3(kBlock), 0, st, Uo, n, r, uc,
                       reinterpret_cast<double2*>(Vout));
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipEventRecord(ctx->ev_stop, st));
    LRQO_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    LRQO_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
    if (res) {
        std::memset(res, 0, sizeof *res);
        for (int k = 0; k < r; ++k) {
            res->eigenvalues[k] = h_tr[k];
            res->residuals[k] = h_tr[LRQO_MAX_R + k];
        }
        res->iterations = m;
        res->converged = (converged || breakdown) ? 1 : 0;
        res->device_ms = ms;
    }
    return LRQO_OK;
}

}  // namespace
}  // namespace lrqo

extern "C" {

lrqo_status lrqo_laplacian_factor(const lrqo_graph* g, int32_t r, const lrqo_eigs_options* opt, double* V,
                                  lrqo_eigs_result* res) {
    using namespace lrqo;
    clear_error();
    LRQO_TRY(check_graph_args(g));
    if (!V) return fail(LRQO_EINVAL, "null pointer argument");
    if (r < 1 || r > LRQO_MAX_R) return fail(LRQO_EINVAL, "r must be in [1, 8]");
    if (!is_device_pointer(V)) return fail(LRQO_EINVAL, "V is not device memory");
    {
        // the CSR layout is checked on the device before any kernel reads
        // col through row_ptr
        DeviceCtx* ctx = device_ctx();
        if (!ctx) return LRQO_EDEVICE;
        std::lock_guard<std::mutex> lk(ctx->mu);
        LRQO_TRY(reserve_arena(ctx, 256));
        LRQO_TRY(reserve_host(ctx, 256));
        LRQO_TRY(validate_graph(g, 2, nullptr, static_cast<int*>(ctx->arena), static_cast<int*>(ctx->host),
                                current_stream()));
    }
    const LapOp lap{g->row_ptr, g->col, g->w, g->n};
    const PhaseOp ph{};
    return lanczos_factor(kOpLap, lap, ph, g->n, r, opt, V, res);
}

lrqo_status lrqo_phase_sync_factor(const double* U, int64_t n, int32_t p, double sigma, uint64_t w_seed, int32_t r,
                                   const lrqo_eigs_options* opt, double* V, lrqo_eigs_result* res) {
    using namespace lrqo;
    clear_error();
    if (!U || !V) return fail(LRQO_EINVAL, "null pointer argument");
    if (n < 1 || n > 0x7fffffffLL) return fail(LRQO_EINVAL, "n must be in [1, 2^31 - 1]");
    if (p < 0 || p > LRQO_MAX_R) return fail(LRQO_EINVAL, "p must be in [0, 8]");
    if (r < 1 || r > LRQO_MAX_R) return fail(LRQO_EINVAL, "r must be in [1, 8]");
    if (!std::isfinite(sigma)) return fail(LRQO_EINVAL, "sigma must be finite");
    if (!is_device_pointer(U) || !is_device_pointer(V)) return fail(LRQO_EINVAL, "U and V must be device memory");
    const LapOp lap{};
    const PhaseOp ph{reinterpret_cast<const double2*>(U), p, sigma, w_seed, n};
    return lanczos_factor(kOpPhase, lap, ph, n, r, opt, V, res);
}

}  // extern "C"
