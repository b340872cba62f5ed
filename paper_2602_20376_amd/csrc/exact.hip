// Exact maximisation by arrangement-vertex enumeration (Sec. 3, Alg. 2).
//
// Geometry.  Row (i, m), m < B_K, of the augmented real matrix (eq. tildeV)
// is a_{i,m} = [Im(rho_m V_i), Re(rho_m V_i)], rho_m = exp(-i pi (2m+1)/K),
// so that a_{i,m} . [Re c; Im c] = Im(rho_m V_i c): it vanishes when V_i c is
// on the line of decision boundary m (Lemma antipodal).  Rows are numbered
// group-major, j = i B_K + m.  A vertex is the null direction of 2d-1 rows
// with at most two rows per coordinate (Lemma rank_deficiency); level d uses
// the leading d columns (d = r: the main loop of Alg. 2; d < r: its
// recursion), and every candidate is scored with the full factor.
//
// Kernels:
//   k_to_f32        FP32 copy of V for the scorer, and a flag when some
//                   imaginary part is not zero (the row scorers take real
//                   arithmetic, half the FMAs, when none is)
//   k_exact_score   fused form: one thread per index set (grid-stride):
//                   colex unranking (or a random draw), FP64 null vector by
//                   twice-orthogonalised Gram-Schmidt (in the thread for
//                   d <= 4, by sixteen lanes per set for larger d), both signs
//                   scored in FP32 over every row (row tiles in LDS; runs of
//                   32 rows that no set of the wave touches with no per-row
//                   test); coordinates in the set tried with every label the
//                   vertex leaves open; best FP32 score per set -> fbuf
//   k_exact_vertex, k_exact_rows, k_exact_combine
//                   split form, for levels whose rows take several slices:
//                   each set's vertex kept as a record; the row pass per
//                   (set, row slice) into slice sums; the slice sums added in
//                   order, then the label combinations
//   topk_select     best 64 sets of a chunk (select.hip), scores below a
//                   floor read on the device dropped
//   k_exact_merge   the chunk's best into the running shortlist
//   k_exact_rescore_rows  FP64 row sums of each kept set (both signs),
//                   grid (kept sets, row slices)
//   k_exact_rescore FP64 re-evaluation of each kept set from the slice sums
//                   (in slice order), all label combinations over the block
//   k_exact_pick    FP64 arg-max (ties -> lowest set index)
//   k_exact_labels  labels of the winner
#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "lrqo_device.h"
#include "lrqo_runtime.h"
#include "select.h"

namespace lrqo {

namespace {

constexpr int kBlock = 256;
constexpr int kTile = 256;
constexpr int kSub = 32;         // rows per wave-uniform touched test in the row pass
constexpr int kFloorGroup = 2048;  // scores per group of the selection's first pass (select.hip)
constexpr int kMaxR = 8;
constexpr int kThreadMaxD = 4;    // levels whose vertex one thread solves alone
constexpr int kTopT = 64;
constexpr int kRescoreSlices = 64;   // row slices of the FP64 rescore, at most
constexpr double kRankTol = 1e-10;
constexpr int64_t kMaxCombos = 1 << 20;
constexpr uint64_t kChunkSets = 1ull << 26;          // sets scored between shortlist merges
constexpr uint64_t kDefaultMaxSets = 1ull << 34;     // default cap on the index sets of a solve
constexpr uint64_t kHardMaxSets = 1ull << 62;        // limit with the cap lifted (max_sets < 0)

// A vertex as the split scorer reads it: FP32 direction (re, im per
// column), the coordinates of its index set (-1 when it has none), and
// whether the set gave a full-rank vertex.  64 bytes up to d = 4, 128 above.
template <int DP>
struct VertexRecT {
    float c[2 * DP];
    int32_t g[2 * DP - 1];
    int32_t ok;
};
template <int D>
using VertexRec = VertexRecT<(D <= kThreadMaxD ? kThreadMaxD : kMaxR)>;

size_t vertex_rec_bytes(int r) {
    return r <= kThreadMaxD ? sizeof(VertexRecT<kThreadMaxD>) : sizeof(VertexRecT<kMaxR>);
}

struct ExactParams {
    const double* V64;   // n x r complex128, interleaved
    const float* V32;    // n x r complex64, interleaved
    int64_t n;
    int r;
    int K;
    int B;
    int64_t N;                          // n * B rows of the augmented matrix
    const unsigned long long* binom;    // C(x, k) at [k * (N + 1) + x], k = 0 .. 2r - 1
    const double2* rho;                 // [B]
    const double2* roots64;             // [K]
    const float2* roots32;              // [K]
    uint64_t count;                     // index sets of this chunk
    uint64_t rank0;                     // rank (within its level) of the chunk's first set
    float* fbuf;                        // best FP32 score of each set of the chunk
    unsigned long long* stats;          // valid sets, rank deficient, candidates: kStatSlots slots each
    int random;                         // 1: index sets drawn at random (null-vector sampler)
    uint64_t draw_seed;
    int64_t rows_per_slice;             // rows of one slice of the split scorer's grid
    float* part;                        // split form: slice sums
    void* recs;                         // split form: one VertexRec<d> per set
    const int32_t* complex_v;           // nonzero: V has an imaginary part (else real arithmetic)
    const uint32_t* vmax_bits;          // bits of the largest |V| entry (FP32, non-negative)
};

struct LevelTable {
    uint64_t offset[kMaxR + 1];
    uint64_t count[kMaxR + 1];
};

// Shortlist of the enumeration: one entry per FP32 score value (the set
// with the lowest global index), best first; f < 0 marks an empty slot.
struct TopEntry {
    float f;
    int32_t pad;
    uint64_t gidx;      // global set index: level offset + rank within the level
};
static_assert(offsetof(TopEntry, f) == 0, "the selection reads the last entry's score through a float pointer");

struct RescoreEntry {
    double f;
    int32_t sign;     // 0: +v, 1: -v
    int32_t pad;
    int64_t combo;
};

struct ExactDevResult {
    double obj;
    int64_t gidx;
    int32_t level;
    int32_t sign;
    int64_t combo;
    int32_t nonfinite;
    int32_t complex_v;   // some imaginary part of V is not zero
    uint32_t vmax_bits;  // FP32 bits of the largest finite |V| entry (ordered as integers)
};

// ---------------------------------------------------------------- vertex
// Colex unranking: rank = sum_t C(c_t, t+1) with c_0 < c_1 < ... < c_{M-1}
// (binomials C(x, k) for k >= 2 from the table; rank < 2^64).
template <int M>
__device__ __forceinline__ void unrank(uint64_t rank, const unsigned long long* binom, int64_t N,
                                       int64_t (&c)[M]) {
    int64_t hi = N - 1;
#pragma unroll
    for (int t = M - 1; t >= 1; --t) {
        const unsigned long long* col = binom + (size_t)(t + 1) * (N + 1);
        int64_t lo = t, h = hi;
        while (lo < h) {
            const int64_t mid = (lo + h + 1) >> 1;
            if (col[mid] <= rank) lo = mid;
            else h = mid - 1;
        }
        c[t] = lo;
        rank -= col[lo];
        hi = lo - 1;
    }
    c[0] = (int64_t)rank;     // C(x, 1) = x
}

// Null-vector sampler, draw s: M rows of the augmented matrix, row j =
// (2^32 w[2j+1] + w[2j]) mod N with w the words of Philox4x32-10 (key seed,
// counter (s lo, s hi, kNullvecStream, block)), sorted; `distinct` is false
// when a row repeats.
constexpr uint32_t kNullvecStream = 0x4E554C4Cu;

template <int M>
__device__ __forceinline__ void draw_rows(uint64_t seed, uint64_t s, int64_t N, int64_t (&c)[M], bool& distinct) {
    constexpr int NB = (2 * M + 3) / 4;
    uint32_t w[4 * NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const U4 o = philox4x32_10(U4{(uint32_t)s, (uint32_t)(s >> 32), kNullvecStream, (uint32_t)b},
                                   (uint32_t)seed, (uint32_t)(seed >> 32));
        w[4 * b] = o.x;
        w[4 * b + 1] = o.y;
        w[4 * b + 2] = o.z;
        w[4 * b + 3] = o.w;
    }
#pragma unroll
    for (int j = 0; j < M; ++j)
        c[j] = (int64_t)((((uint64_t)w[2 * j + 1] << 32) | (uint64_t)w[2 * j]) % (uint64_t)N);
    for (int t = 1; t < M; ++t) {       // insertion sort, M <= 15
        const int64_t x = c[t];
        int u = t - 1;
        while (u >= 0 && c[u] > x) {
            c[u + 1] = c[u];
            --u;
        }
        c[u + 1] = x;
    }
    distinct = true;
#pragma unroll
    for (int t = 0; t + 1 < M; ++t) distinct &= c[t] < c[t + 1];
}

// The rows of one index set: groups g[t] and boundary ids mm[t]; false for
// a set with a repeated row (random draws) or three rows of one group.
template <int D>
__device__ bool set_rows(const ExactParams& p, uint64_t rank, int64_t (&g)[2 * D - 1], int (&mm)[2 * D - 1]) {
    constexpr int M = 2 * D - 1;
    int64_t c[M];
    bool distinct = true;
    if (p.random) draw_rows<M>(p.draw_seed, rank, p.N, c, distinct);
    else unrank<M>(rank, p.binom, p.N, c);
#pragma unroll
    for (int t = 0; t < M; ++t) {
        g[t] = c[t] / p.B;
        mm[t] = (int)(c[t] - g[t] * p.B);
    }
    bool valid = distinct;
#pragma unroll
    for (int t = 0; t + 2 < M; ++t) valid &= g[t] != g[t + 2];
    return valid;
}

// The vertex of one index set, solved by one thread (d <= 4): groups g[t],
// boundary ids mm[t], unit null vector v in R^{2D}.  Returns false for an
// invalid set or one below the rank tolerance (rank_deficient set
// accordingly).
template <int D>
__device__ bool vertex(const ExactParams& p, uint64_t rank, int64_t (&g)[2 * D - 1],
                       int (&mm)[2 * D - 1], double (&v)[2 * D], bool& valid) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    valid = set_rows<D>(p, rank, g, mm);
    if (!valid) return false;

    double a[M][C2];
    double amax = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const double2 rh = p.rho[mm[t]];
        double nrm = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double vr = p.V64[(g[t] * p.r + j) * 2], vi = p.V64[(g[t] * p.r + j) * 2 + 1];
            const double pr = rh.x * vr - rh.y * vi;   // rho V_ij
            const double pi = rh.x * vi + rh.y * vr;
            a[t][j] = pi;
            a[t][D + j] = pr;
            nrm += pr * pr + pi * pi;
        }
        amax = fmax(amax, sqrt(nrm));
    }
    // orthonormalise the rows (Gram-Schmidt, two passes)
    double rmin = INFINITY;
#pragma unroll
    for (int t = 0; t < M; ++t) {
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int u = 0; u < t; ++u) {
                double d = 0.0;
#pragma unroll
                for (int k = 0; k < C2; ++k) d += a[u][k] * a[t][k];
#pragma unroll
                for (int k = 0; k < C2; ++k) a[t][k] -= d * a[u][k];
            }
        }
        double nrm = 0.0;
#pragma unroll
        for (int k = 0; k < C2; ++k) nrm += a[t][k] * a[t][k];
        nrm = sqrt(nrm);
        rmin = fmin(rmin, nrm);
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
#pragma unroll
        for (int k = 0; k < C2; ++k) a[t][k] *= inv;
    }
    // complement direction: the unit vector e_k with the largest residual
    // after removing the row space, projected and normalised
    int kb = 0;
    double wb = -1.0;
#pragma unroll
    for (int k = 0; k < C2; ++k) {
        double w = 1.0;
#pragma unroll
        for (int t = 0; t < M; ++t) w -= a[t][k] * a[t][k];
        if (w > wb) {
            wb = w;
            kb = k;
        }
    }
#pragma unroll
    for (int j = 0; j < C2; ++j) v[j] = 0.0;
#pragma unroll
    for (int k = 0; k < C2; ++k) {
        if (k == kb) {
#pragma unroll
            for (int j = 0; j < C2; ++j) {
                double x = (j == k) ? 1.0 : 0.0;
#pragma unroll
                for (int t = 0; t < M; ++t) x -= a[t][k] * a[t][j];
                v[j] = x;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < M; ++t) {
        double d = 0.0;
#pragma unroll
        for (int k = 0; k < C2; ++k) d += a[t][k] * v[k];
#pragma unroll
        for (int k = 0; k < C2; ++k) v[k] -= d * a[t][k];
    }
    double nv = 0.0;
#pragma unroll
    for (int k = 0; k < C2; ++k) nv += v[k] * v[k];
    const double inv = 1.0 / sqrt(nv);
#pragma unroll
    for (int k = 0; k < C2; ++k) v[k] *= inv;
    return amax > 0.0 && rmin > kRankTol * amax;
}

// Levels d > 4: the (2d-1) x 2d block of a set no longer fits one thread's
// registers.  Sixteen lanes share a set instead, lane k holding column k of
// its rows (zero for k >= 2d), and every dot product over the 2d columns is a
// butterfly sum over the sixteen lanes, which leaves the same value in each of
// them.  The steps are those of vertex(): row scales, two Gram-Schmidt passes,
// the complement direction e_kb of largest residual, its projection and
// normalisation.
constexpr int kCoopLanes = 16;
static_assert(2 * kMaxR <= kCoopLanes, "a lane per column");

__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int off = kCoopLanes / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

template <int D>
__device__ double solve_columns(const ExactParams& p, const int64_t (&g)[2 * D - 1], const int (&mm)[2 * D - 1],
                                int k, bool& ok) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    const int j = k < D ? k : k - D;          // column of V behind column k
    double a[M];
    double amax = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const double2 rh = p.rho[mm[t]];
        double x = 0.0;
        if (k < C2) {
            const double vr = p.V64[(g[t] * p.r + j) * 2], vi = p.V64[(g[t] * p.r + j) * 2 + 1];
            x = k < D ? rh.x * vi + rh.y * vr      // Im(rho V_ij)
                      : rh.x * vr - rh.y * vi;     // Re(rho V_ij)
        }
        a[t] = x;
        amax = fmax(amax, sqrt(group_sum(x * x)));
    }
    double rmin = INFINITY;
#pragma unroll
    for (int t = 0; t < M; ++t) {
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int u = 0; u < t; ++u) a[t] -= group_sum(a[u] * a[t]) * a[u];
        }
        const double nrm = sqrt(group_sum(a[t] * a[t]));
        rmin = fmin(rmin, nrm);
        a[t] *= nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
    // the unit vector with the largest residual, the lowest k on ties
    double wres = -INFINITY;
    if (k < C2) {
        wres = 1.0;
#pragma unroll
        for (int t = 0; t < M; ++t) wres -= a[t] * a[t];
    }
    int kb = k;
#pragma unroll
    for (int off = kCoopLanes / 2; off > 0; off >>= 1) {
        const double wo = __shfl_xor(wres, off, kWave);
        const int ko = __shfl_xor(kb, off, kWave);
        if (wo > wres || (wo == wres && ko < kb)) {
            wres = wo;
            kb = ko;
        }
    }
    const int base = (int)(threadIdx.x % kWave) & ~(kCoopLanes - 1);
    double vk = k == kb ? 1.0 : 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) vk -= __shfl(a[t], base + kb, kWave) * a[t];
    if (k >= C2) vk = 0.0;
#pragma unroll
    for (int t = 0; t < M; ++t) vk -= group_sum(a[t] * vk) * a[t];
    vk *= 1.0 / sqrt(group_sum(vk * vk));
    ok = amax > 0.0 && rmin > kRankTol * amax;
    return vk;
}

struct CoopLds {
    uint64_t rank[kBlock];
    double v[kBlock][2 * kMaxR];
    int32_t state[kBlock];       // 1: a valid set to solve; then 2 if full rank
};

__device__ __forceinline__ CoopLds& coop_lds() {
    __shared__ CoopLds s;
    return s;
}

// The vertex of each thread's set for every level: alone for d <= 4; for
// d > 4 every thread of the block must call it (it has barriers), sixteen
// lanes per set, each thread getting back its own set's vertex (uniform:
// every thread passes the same rank, solved once).
template <int D>
__device__ bool vertex_blk(const ExactParams& p, uint64_t rank, bool active, bool uniform,
                           int64_t (&g)[2 * D - 1], int (&mm)[2 * D - 1], double (&v)[2 * D], bool& valid) {
    if constexpr (D <= kThreadMaxD) {
        valid = false;
        return active && vertex<D>(p, rank, g, mm, v, valid);
    } else {
        constexpr int M = 2 * D - 1, C2 = 2 * D;
        CoopLds& sh = coop_lds();
        const int tid = threadIdx.x;
        valid = active && set_rows<D>(p, rank, g, mm);
        sh.rank[tid] = rank;
        sh.state[tid] = valid ? 1 : 0;
        __syncthreads();
        const int lane = tid % kCoopLanes;
        const int nsets = uniform ? 1 : kBlock;
        for (int q = tid / kCoopLanes; q < nsets; q += kBlock / kCoopLanes) {
            if (sh.state[q] == 0) continue;          // the same for the sixteen lanes
            int64_t gq[M];
            int mq[M];
            set_rows<D>(p, sh.rank[q], gq, mq);
            bool okq = false;
            const double vk = solve_columns<D>(p, gq, mq, lane, okq);
            if (lane < C2) sh.v[q][lane] = vk;
            if (lane == 0 && okq) sh.state[q] = 2;
        }
        __syncthreads();
        const int src = uniform ? 0 : tid;
        const bool ok = valid && sh.state[src] == 2;
#pragma unroll
        for (int c = 0; c < C2; ++c) v[c] = ok ? sh.v[src][c] : 0.0;
        __syncthreads();                             // before the next call rewrites the block's slots
        return ok;
    }
}

// Options left open at a vertex for the coordinates of the set (both rows
// of a double group share one entry; the second gets count 1): first label
// o[t] and count cnt[t] of consecutive labels mod K.
template <int D>
__device__ void open_labels(const ExactParams& p, const int64_t (&g)[2 * D - 1],
                            const int (&mm)[2 * D - 1], const double (&c)[2 * D],
                            int (&o)[2 * D - 1], int (&cnt)[2 * D - 1]) {
    constexpr int M = 2 * D - 1;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const bool first = (t == 0) || (g[t] != g[t - 1]);
        const bool dbl = first && (t + 1 < M) && (g[t + 1] == g[t]);
        o[t] = 0;
        cnt[t] = 1;
        if (!first) continue;
        if (dbl) {
            cnt[t] = p.K;   // V_i c = 0: every label borders the vertex
            continue;
        }
        double wr = 0.0, wi = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double vr = p.V64[(g[t] * p.r + j) * 2], vi = p.V64[(g[t] * p.r + j) * 2 + 1];
            wr += vr * c[j] - vi * c[D + j];
            wi += vr * c[D + j] + vi * c[j];
        }
        const double2 rh = p.rho[mm[t]];
        const double re = rh.x * wr - rh.y * wi;   // Re(rho_m w_i)
        if (re > 0.0) {
            o[t] = mm[t];                          // on ray pi(2m+1)/K: labels m, m+1
            cnt[t] = 2;
        } else if (p.K & 1) {
            // the opposite ray, at angle pi (2m + 1 + K) / K, points at root
            // m + (K + 1) / 2: the decision rule's label there
            o[t] = (mm[t] + (p.K + 1) / 2) % p.K;
        } else {
            o[t] = (mm[t] + p.K / 2) % p.K;        // opposite ray is boundary m + K/2
            cnt[t] = 2;
        }
    }
}

// ---------------------------------------------------------------- FP32 scoring
template <int R>
__global__ void k_to_f32(const double* __restrict__ V64, float* __restrict__ V32, int64_t count,
                         int* nonfinite, int* complex_v, uint32_t* vmax_bits) {
    __shared__ uint32_t wmax[kBlock / kWave];
    float m = 0.0f;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double x = V64[e];
        if (!isfinite(x)) *nonfinite = 1;
        if ((e & 1) && x != 0.0) *complex_v = 1;   // every writer stores the same value
        const float xf = (float)x;
        V32[e] = xf;
        m = isfinite(xf) ? fmaxf(m, fabsf(xf)) : m;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) wmax[threadIdx.x / kWave] = __float_as_uint(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) b = max(b, wmax[w]);
        if (b) atomicMax(vmax_bits, b);              // non-negative floats order as their bits
    }
}

// r > 4: the factor in kMaxR columns, zeros beyond its r (the kernels for
// those ranks are built for kMaxR columns only; a zero column adds exact
// zeros to every sum and product, so the results are those of r columns).
__global__ void k_pad_columns(const double* __restrict__ V, double* __restrict__ Vp, int64_t n, int r) {
    const int64_t count = n * kMaxR;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / kMaxR;
        const int j = (int)(e - i * kMaxR);
        Vp[2 * e] = j < r ? V[2 * (i * r + j)] : 0.0;
        Vp[2 * e + 1] = j < r ? V[2 * (i * r + j) + 1] : 0.0;
    }
}

// Sums conj(V_i) z_i over rows [r0, r1) for both signs +c and -c of a
// direction (V_i c formed once), skipping the rows of the set (g, sorted,
// -1 for none): rows in LDS tiles, every lane of a wave reading the same row
// (broadcast).  All threads of the block take part in the tile loads.
// REAL: V has no imaginary part; the tiles hold the real parts only and
// the terms with Im V are left out (they are exact zeros, so the sums are
// the same numbers).
// REAL and K = 3: the set's rows are zeroed in V instead of in the labels,
// and each sign accumulates in the basis q = [label != 0]: sum_i V_i q_i and
// sum_i V_i q_i sign(Im w_i), so that s = sum V - 3/2 sum V q +
// i (sqrt(3)/2) sum V q sign(Im w) after the loop; sum V over the untouched
// rows, the same for every direction, is the slice's column sums (one pass
// per block) less the set's rows.
// w is formed from B Im c and -B sqrt(3) Re c (B a power of two sized from
// the largest |V| entry, as in the sampled scorer): |Im w'| + Re w' is
// B (|Im w| - sqrt(3) Re w), the label test for +c, |Im w'| - Re w' the one
// for -c (-c gives -w), each clamped to [0, 1] by the add's output modifier.
__device__ __forceinline__ float exact_q3_scale(uint32_t vmax_bits) {
    const float m = __uint_as_float(vmax_bits);
    if (!(m > 0.0f) || !isfinite(m)) return 1.0f;
    return ldexpf(1.0f, min(126, max(-126, 118 - ilogbf(m))));
}

// Column sums of Re V over rows [r0, r1) of the FP32 copy, added in FP64 in
// a fixed order and rounded once, so every block of a slice holds the same
// numbers.  Called by every thread of the block.
template <int R>
__device__ void slice_col_sums(const ExactParams& p, int64_t r0, int64_t r1, float* colsum) {
    __shared__ double red[kBlock / kWave][R];
    double part[R];
#pragma unroll
    for (int j = 0; j < R; ++j) part[j] = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock)
#pragma unroll
        for (int j = 0; j < R; ++j) part[j] += (double)p.V32[(i * R + j) * 2];
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) part[j] += __shfl_xor(part[j], off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int j = 0; j < R; ++j) red[threadIdx.x / kWave][j] = part[j];
    __syncthreads();
    if (threadIdx.x < R) {
        double t = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) t += red[w][threadIdx.x];
        colsum[threadIdx.x] = (float)t;
    }
    __syncthreads();
}

template <int R, int D, int KS, bool REAL>
__device__ __forceinline__ void score_rows(const ExactParams& p, const float (&c)[2 * D],
                                           const int32_t (&g)[2 * D - 1], int64_t r0, int64_t r1,
                                           float* tile, const float2* roots_s, const float* colsum,
                                           float (&acc)[2][2 * R]) {
    constexpr int M = 2 * D - 1;
    constexpr int RW = REAL ? R : 2 * R;   // floats per staged row
    constexpr bool Q3 = REAL && KS == 3;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) acc[s][j] = 0.0f;
    float cw[Q3 ? 2 * D : 1];              // Q3: -B sqrt(3) Re c, B Im c
    float tq[2][Q3 ? R : 1], ts[2][Q3 ? R : 1], tv[Q3 ? R : 1];
    if constexpr (Q3) {
        const float B = exact_q3_scale(*p.vmax_bits);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            cw[2 * j] = -B * (1.7320508075688772f * c[2 * j]);
            cw[2 * j + 1] = B * c[2 * j + 1];
        }
#pragma unroll
        for (int j = 0; j < R; ++j) tq[0][j] = tq[1][j] = ts[0][j] = ts[1][j] = 0.0f;
    }
    int64_t next = INT64_MAX;                  // r > 4: next touched row at or after r0
#pragma unroll
    for (int t = 0; t < M; ++t)
        if (g[t] >= r0 && g[t] < next) next = g[t];
    uint32_t nx = UINT32_MAX;                  // r <= 4: the same as 32 bits (none: UINT32_MAX)
#pragma unroll
    for (int t = 0; t < M; ++t)
        if (g[t] >= r0) nx = min(nx, (uint32_t)g[t]);
    // One row of the tile; a touched row counts as zeros.
    auto row = [&](int i, bool touched) {
        float vv[RW];
#pragma unroll
        for (int e = 0; e < RW; ++e) vv[e] = tile[i * RW + e];
        if constexpr (Q3) {
            float vz[R];
#pragma unroll
            for (int e = 0; e < R; ++e) vz[e] = touched ? 0.0f : vv[e];
            float wr = 0.0f, wi = 0.0f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                wr = fmaf(vz[j], cw[2 * j], wr);
                wi = fmaf(vz[j], cw[2 * j + 1], wi);
            }
            const float qp = __builtin_amdgcn_fmed3f(fabsf(wi) + wr, 0.0f, 1.0f);   // +c
            const float qm = __builtin_amdgcn_fmed3f(fabsf(wi) - wr, 0.0f, 1.0f);   // -c
            const float sp = copysignf(qp, wi);    // q sign(Im w) for +c
            const float sm = copysignf(qm, wi);    // minus q sign(Im w) for -c
#pragma unroll
            for (int j = 0; j < R; ++j) {
                tq[0][j] = fmaf(vz[j], qp, tq[0][j]);
                ts[0][j] = fmaf(vz[j], sp, ts[0][j]);
                tq[1][j] = fmaf(vz[j], qm, tq[1][j]);
                ts[1][j] = fmaf(-vz[j], sm, ts[1][j]);
            }
        } else {
            // V_i c once: for -c it is exactly -(V_i c)
            float wr = 0.0f, wi = 0.0f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                if constexpr (REAL) {
                    wr = fmaf(vv[j], c[2 * j], wr);
                    wi = fmaf(vv[j], c[2 * j + 1], wi);
                } else {
                    const float vr = vv[2 * j], vi = vv[2 * j + 1];
                    wr = fmaf(vr, c[2 * j], fmaf(-vi, c[2 * j + 1], wr));
                    wi = fmaf(vr, c[2 * j + 1], fmaf(vi, c[2 * j], wi));
                }
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                float zr, zi;
                nearest_root<KS>(s ? -wr : wr, s ? -wi : wi, p.K, roots_s, zr, zi);
                zr = touched ? 0.0f : zr;
                zi = touched ? 0.0f : zi;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    if constexpr (REAL) {
                        acc[s][2 * j] = fmaf(vv[j], zr, acc[s][2 * j]);
                        acc[s][2 * j + 1] = fmaf(vv[j], zi, acc[s][2 * j + 1]);
                    } else {
                        const float vr = vv[2 * j], vi = vv[2 * j + 1];
                        acc[s][2 * j] = fmaf(vr, zr, fmaf(vi, zi, acc[s][2 * j]));
                        acc[s][2 * j + 1] = fmaf(vr, zi, fmaf(-vi, zr, acc[s][2 * j + 1]));
                    }
                }
            }
        }
    };
    // r > 4: one row with the touched test against a cursor over the set's
    // sorted rows, which moves on past a touched row.
    auto row_checked = [&](int i, int64_t rw) {
        const bool touched = rw == next;
        if (touched) {          // rare: advance the cursor
            int64_t nn = INT64_MAX;
#pragma unroll
            for (int t = 0; t < M; ++t)
                if (g[t] > rw && g[t] < nn) nn = g[t];
            next = nn;
        }
        row(i, touched);
    };
    for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, r1 - t0);
        __syncthreads();
        const float* __restrict__ src = p.V32 + t0 * 2 * R;
        for (int e = threadIdx.x; e < cnt * RW; e += kBlock) tile[e] = REAL ? src[2 * e] : src[e];
        __syncthreads();
        if constexpr (R <= kThreadMaxD) {
            // Runs of kSub rows: a run that no set of the wave touches
            // (every lane's cursor lies beyond it; a wave-uniform test, all
            // lanes take part) is scored with no per-row test at all, the
            // others with the set's rows in the run as a bit mask, both
            // unrolled.
            for (int i = 0; i < cnt; i += kSub) {
                const uint32_t a = (uint32_t)(t0 + i);       // rows < 2^31
                if (!__any(nx < a + kSub)) {
                    if (cnt - i >= kSub) {
                        if constexpr (KS != 0) {
#pragma unroll
                            for (int k = 0; k < kSub; ++k) row(i + k, false);
                        } else {
#pragma unroll 4
                            for (int k = 0; k < kSub; ++k) row(i + k, false);
                        }
                    } else {
                        for (int k = 0; k < cnt - i; ++k) row(i + k, false);
                    }
                    continue;
                }
                // the set's rows among rows [a, a + kSub) as one bit each
                // (a row below a, or -1, wraps to a large offset); the
                // cursor moves past the run
                uint32_t mask = 0;
                uint32_t nn = UINT32_MAX;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    const uint32_t gt = (uint32_t)g[t];
                    const uint32_t d = gt - a;
                    mask |= d < (uint32_t)kSub ? 1u << d : 0u;
                    nn = min(nn, d >= (uint32_t)kSub && gt >= a ? gt : UINT32_MAX);
                }
                nx = nn;
                if (cnt - i >= kSub) {
                    if constexpr (KS != 0) {
#pragma unroll
                        for (int k = 0; k < kSub; ++k) row(i + k, (mask >> k) & 1u);
                    } else {
#pragma unroll 4
                        for (int k = 0; k < kSub; ++k) row(i + k, (mask >> k) & 1u);
                    }
                } else {
                    for (int k = 0; k < cnt - i; ++k) row(i + k, (mask >> k) & 1u);
                }
            }
        } else {
            for (int i = 0; i < cnt; ++i) row_checked(i, t0 + i);
        }
    }
    if constexpr (Q3) {
        // sum of V over the untouched rows: the slice's column sums less the
        // set's distinct rows in the slice, in row order
#pragma unroll
        for (int j = 0; j < R; ++j) tv[j] = colsum[j];
#pragma unroll
        for (int t = 0; t < M; ++t) {
            if (g[t] >= r0 && g[t] < r1 && (t == 0 || g[t] != g[t - 1])) {
#pragma unroll
                for (int j = 0; j < R; ++j) tv[j] -= p.V32[((int64_t)g[t] * R + j) * 2];
            }
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < R; ++j) {
                acc[s][2 * j] = fmaf(-1.5f, tq[s][j], tv[j]);
                acc[s][2 * j + 1] = 0.8660254037844386f * ts[s][j];
            }
    }
}

// Best FP32 score over both signs and every open-label combination of the
// set's coordinates, from the sums acc[s] of the untouched rows; also the
// number of combinations tried.  Both signs run in one loop (the mixed-radix
// counter is back at zero after the last combination of +v, where the loop
// turns to -v), so a wave runs the longest lane's total of the two rather
// than the sum of each sign's longest.  The second row of a coordinate with
// two rows adds nothing (its labels are the first row's); it enters as a
// zero row.  KS = 3 takes the roots in closed form (the same FP32 values as
// the table), other K from the table roots_s.
template <int R, int D, int KS>
__device__ float combos_best(const ExactParams& p, const int64_t (&g)[2 * D - 1], const int (&mm)[2 * D - 1],
                             const double (&v)[2 * D], const float (&acc)[2][2 * R],
                             const float2* roots_s, unsigned long long& ncand) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    // the set's rows in registers once (every combination reads them) when
    // they fit; above that they are read from the FP32 copy (cached)
    constexpr bool kHold = M * 2 * R <= 64;
    bool first[M];
#pragma unroll
    for (int t = 0; t < M; ++t) first[t] = g[t] >= 0 && ((t == 0) || (g[t] != g[t - 1]));
    float vt[kHold ? M : 1][kHold ? 2 * R : 1];
    if constexpr (kHold) {
#pragma unroll
        for (int t = 0; t < M; ++t)
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) vt[t][j] = first[t] ? p.V32[g[t] * 2 * R + j] : 0.0f;
    }
    int o[2][M], cn[2][M];
    int64_t tot[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        double cs[C2];
#pragma unroll
        for (int k = 0; k < C2; ++k) cs[k] = s ? -v[k] : v[k];
        open_labels<D>(p, g, mm, cs, o[s], cn[s]);
        tot[s] = 1;
#pragma unroll
        for (int t = 0; t < M; ++t) tot[s] *= cn[s][t];
    }
    ncand += (unsigned long long)(tot[0] + tot[1]);
    // the combinations in mixed radix cn[s][0], cn[s][1], ... (digit t least
    // significant first), stepped by a counter instead of divisions
    int dig[M];
#pragma unroll
    for (int t = 0; t < M; ++t) dig[t] = 0;
    bool neg = false;                 // false: +v, true: -v
    float best = 0.0f;
    for (int64_t it = 0; it < tot[0] + tot[1]; ++it) {
        float sr[2 * R];
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) sr[j] = neg ? acc[1][j] : acc[0][j];
#pragma unroll
        for (int t = 0; t < M; ++t) {
            int k = (neg ? o[1][t] : o[0][t]) + dig[t];
            k = k >= p.K ? k - p.K : k;
            float zx, zy;
            if constexpr (KS == 3) {
                zx = k == 0 ? 1.0f : -0.5f;
                zy = k == 0 ? 0.0f : (k == 1 ? 0.8660254037844386f : -0.8660254037844386f);
            } else {
                const float2 z = roots_s[k];
                zx = z.x;
                zy = z.y;
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                float vr, vi;
                if constexpr (kHold) {
                    vr = vt[t][2 * j];
                    vi = vt[t][2 * j + 1];
                } else {
                    vr = first[t] ? p.V32[g[t] * 2 * R + 2 * j] : 0.0f;
                    vi = first[t] ? p.V32[g[t] * 2 * R + 2 * j + 1] : 0.0f;
                }
                sr[2 * j] = fmaf(vr, zx, fmaf(vi, zy, sr[2 * j]));
                sr[2 * j + 1] = fmaf(vr, zy, fmaf(-vi, zx, sr[2 * j + 1]));
            }
        }
        float f = 0.0f;
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) f = fmaf(sr[j], sr[j], f);
        best = fmaxf(best, f);
        bool carry = true;
#pragma unroll
        for (int t = 0; t < M; ++t) {
            if (carry) {
                carry = ++dig[t] == (neg ? cn[1][t] : cn[0][t]);
                if (carry) dig[t] = 0;
            }
        }
        neg = neg || carry;           // every digit wrapped: +v is done
    }
    return best;
}

// Statistics of the sets (valid, rank deficient, candidates) summed over
// the block, then added into slot (block index mod kStatSlots) of each
// counter, so that same-address atomics stay few; the host adds the slots.
constexpr int kStatSlots = 64;

__device__ __forceinline__ void add_stats(const ExactParams& p, bool active, bool valid, bool ok,
                                          unsigned long long ncand) {
    __shared__ unsigned long long sred[3][kBlock / kWave];
    unsigned long long a0 = (active && valid) ? 1ull : 0ull;
    unsigned long long a1 = (active && valid && !ok) ? 1ull : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a0 += __shfl_xor(a0, off, kWave);
        a1 += __shfl_xor(a1, off, kWave);
        ncand += __shfl_xor(ncand, off, kWave);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sred[0][w] = a0;
        sred[1][w] = a1;
        sred[2][w] = ncand;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
        for (int q = 0; q < kBlock / kWave; ++q) v += sred[threadIdx.x][q];
        if (v) atomicAdd(&p.stats[threadIdx.x * kStatSlots + blockIdx.x % kStatSlots], v);
    }
    __syncthreads();
}

// Fused form (one pass per set, all rows): vertex, both signs scored over
// every row the set does not touch (row tiles in LDS, the touched rows found
// with a cursor over their sorted list), then the label combinations.  Used
// when the sets are too many for the split form's buffers.
// Waves per SIMD the fused scorer asks the compiler for: five at rank 2,
// level 2 (96 VGPRs, a few spilled in the per-set work; the rank-2 campaign
// runs about 4% faster than at four), no bound elsewhere (the larger levels'
// vertex solves need their registers).
template <int R, int D>
constexpr int kScoreMinWaves = (R == 2 && D == 2) ? 5 : 1;

template <int R, int D, int KS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kScoreMinWaves<R, D>)))
void k_exact_score(ExactParams p) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    __shared__ __align__(16) float tile[kTile * 2 * R];
    __shared__ float2 roots_s[KS == 0 ? LRQO_MAX_K : 1];
    __shared__ float2 roots_all[LRQO_MAX_K];      // the label combinations' roots
    const int tid = threadIdx.x;
    if constexpr (KS == 0) {
        for (int k = tid; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
    }
    for (int k = tid; k < p.K; k += kBlock) roots_all[k] = p.roots32[k];   // read after the tile barriers
    const bool cplx = *p.complex_v != 0;   // the same in every thread
    __shared__ float colsum[R];
    if constexpr (KS == 3 && R <= kThreadMaxD) {
        if (!cplx) slice_col_sums<R>(p, 0, p.n, colsum);
    }
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < p.count; base += stride) {
        const uint64_t rank = base + tid;          // within the chunk
        const bool active = rank < p.count;
        int64_t g[M];
        int mm[M];
        double v[C2];
        bool valid = false;
        const bool ok = vertex_blk<D>(p, p.rank0 + rank, active, false, g, mm, v, valid);
        if (!ok) {
#pragma unroll
            for (int t = 0; t < M; ++t) g[t] = -1;
        }
        float c[2 * D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            c[2 * j] = ok ? (float)v[j] : 0.0f;
            c[2 * j + 1] = ok ? (float)v[D + j] : 0.0f;
        }
        int32_t g32[M];
#pragma unroll
        for (int t = 0; t < M; ++t) g32[t] = (int32_t)g[t];
        float acc[2][2 * R];
        if (cplx || R > kThreadMaxD)
            score_rows<R, D, KS, false>(p, c, g32, 0, p.n, tile, roots_s, colsum, acc);
        else
            score_rows<R, D, KS, true>(p, c, g32, 0, p.n, tile, roots_s, colsum, acc);
        unsigned long long ncand = 0;
        const float best = ok ? combos_best<R, D, KS>(p, g, mm, v, acc, roots_all, ncand) : 0.0f;
        if (active) p.fbuf[rank] = best;
        add_stats(p, active, valid, ok, ncand);
    }
}

// Split form, stage 1: the vertex of each set in FP64, kept as its FP32
// direction and its touched rows (-1 where the set has no full-rank vertex).
template <int D>
__global__ __launch_bounds__(kBlock) void k_exact_vertex(ExactParams p, VertexRec<D>* __restrict__ recs) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    using Rec = VertexRec<D>;
    constexpr int DP = (int)(sizeof(Rec::c) / sizeof(float)) / 2;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < p.count; base += stride) {   // block-uniform
        const uint64_t rank = base + threadIdx.x;
        const bool active = rank < p.count;
        int64_t g[M];
        int mm[M];
        double v[C2];
        bool valid = false;
        const bool ok = vertex_blk<D>(p, p.rank0 + rank, active, false, g, mm, v, valid);
        if (!active) continue;
        Rec rec;
#pragma unroll
        for (int j = 0; j < 2 * DP; ++j) rec.c[j] = 0.0f;
#pragma unroll
        for (int t = 0; t < 2 * DP - 1; ++t) rec.g[t] = -1;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            rec.c[2 * j] = ok ? (float)v[j] : 0.0f;
            rec.c[2 * j + 1] = ok ? (float)v[D + j] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < M; ++t) rec.g[t] = ok ? (int32_t)g[t] : -1;
        rec.ok = ok ? 1 : 0;
        recs[rank] = rec;
    }
}

// Split form, stage 2: grid (set blocks, row slices); each thread scores its
// set's two signs over the slice's rows from the stored record (no FP64
// state, so many waves fit on a SIMD) and writes the slice sums to p.part.
template <int R, int D, int KS>
__global__ __launch_bounds__(kBlock) void k_exact_rows(ExactParams p, const VertexRec<D>* __restrict__ recs) {
    constexpr int M = 2 * D - 1;
    __shared__ __align__(16) float tile[kTile * 2 * R];
    __shared__ float2 roots_s[KS == 0 ? LRQO_MAX_K : 1];
    if constexpr (KS == 0) {
        for (int k = threadIdx.x; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
    }
    const int64_t r0 = (int64_t)blockIdx.y * p.rows_per_slice;
    const int64_t r1 = min(p.n, r0 + p.rows_per_slice);
    const bool cplx = *p.complex_v != 0;   // the same in every thread
    __shared__ float colsum[R];
    if constexpr (KS == 3 && R <= kThreadMaxD) {
        if (!cplx) slice_col_sums<R>(p, r0, r1, colsum);
    }
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < p.count; base += stride) {
        const uint64_t rank = base + threadIdx.x;
        const bool active = rank < p.count;
        float c[2 * D];
        int32_t g[M];
        if (active) {
            const VertexRec<D> rec = recs[rank];
#pragma unroll
            for (int j = 0; j < 2 * D; ++j) c[j] = rec.c[j];
#pragma unroll
            for (int t = 0; t < M; ++t) g[t] = rec.g[t];
        } else {
#pragma unroll
            for (int j = 0; j < 2 * D; ++j) c[j] = 0.0f;
#pragma unroll
            for (int t = 0; t < M; ++t) g[t] = -1;
        }
        float acc[2][2 * R];
        if (cplx || R > kThreadMaxD)
            score_rows<R, D, KS, false>(p, c, g, r0, r1, tile, roots_s, colsum, acc);
        else
            score_rows<R, D, KS, true>(p, c, g, r0, r1, tile, roots_s, colsum, acc);
        if (active) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int j = 0; j < 2 * R; ++j)
                    p.part[(((uint64_t)blockIdx.y * 2 + s) * (2 * R) + j) * p.count + rank] = acc[s][j];
        }
    }
}

// Row slices of k_exact_score: per set, the slice sums in slice order, then
// the label combinations and the statistics.
template <int R, int D>
__global__ __launch_bounds__(kBlock) void k_exact_combine(ExactParams p, int slices) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    __shared__ float2 roots_all[LRQO_MAX_K];
    for (int k = threadIdx.x; k < p.K; k += kBlock) roots_all[k] = p.roots32[k];
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < p.count; base += stride) {
        const uint64_t rank = base + threadIdx.x;
        const bool active = rank < p.count;
        int64_t g[M];
        int mm[M];
        double v[C2];
        bool valid = false;
        const bool ok = vertex_blk<D>(p, p.rank0 + rank, active, false, g, mm, v, valid);
        unsigned long long ncand = 0;
        float best = 0.0f;
        if (ok) {
            float acc[2][2 * R];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int j = 0; j < 2 * R; ++j) {
                    float a = 0.0f;
                    for (int q = 0; q < slices; ++q) a += p.part[(((uint64_t)q * 2 + s) * (2 * R) + j) * p.count + rank];
                    acc[s][j] = a;
                }
            best = combos_best<R, D, 0>(p, g, mm, v, acc, roots_all, ncand);
        }
        if (active) p.fbuf[rank] = best;
        add_stats(p, active, valid, ok, ncand);
    }
}

// Merges a chunk's best keys (sorted, one per score value, indices local to
// the chunk, global index base + local) into the running shortlist: sorted by
// score descending then global index ascending, one entry per score value
// (the lower index: earlier chunks hold lower indices), at most kTopT.  One
// thread; the lists are short.
__global__ void k_exact_merge(TopEntry* __restrict__ top, const unsigned long long* __restrict__ keys, int T,
                              uint64_t base) {
    __shared__ TopEntry a[kTopT], out[kTopT];
    if (threadIdx.x != 0) return;
    for (int t = 0; t < kTopT; ++t) a[t] = top[t];
    int i = 0, j = 0, m = 0;
    float last = -1.0f;
    while (m < kTopT) {
        const bool ha = i < kTopT && a[i].f >= 0.0f;
        const bool hb = j < T && keys[j] != 0ull;
        if (!ha && !hb) break;
        TopEntry e;
        if (ha && hb) {
            const float fb = key_value(keys[j]);
            const uint64_t gb = base + key_index(keys[j]);
            const bool take_a = a[i].f > fb || (a[i].f == fb && a[i].gidx < gb);
            e = take_a ? a[i] : TopEntry{fb, 0, gb};
            if (take_a) ++i; else ++j;
        } else if (ha) {
            e = a[i++];
        } else {
            e = TopEntry{key_value(keys[j]), 0, base + key_index(keys[j])};
            ++j;
        }
        if (m > 0 && e.f == last) continue;     // the same score value: keep the earlier set
        out[m++] = e;
        last = e.f;
    }
    for (int t = 0; t < kTopT; ++t) top[t] = t < m ? out[t] : TopEntry{-1.0f, 0, 0};
}

__global__ void k_exact_top_init(TopEntry* __restrict__ top) {
    if (threadIdx.x < kTopT) top[threadIdx.x] = TopEntry{-1.0f, 0, 0};
}

// ---------------------------------------------------------------- FP64 rescore
__device__ __forceinline__ int level_of(const LevelTable& lt, int r, uint64_t gidx,
                                        uint64_t& rank) {
    for (int d = r; d >= 1; --d) {
        if (gidx >= lt.offset[d] && gidx < lt.offset[d] + lt.count[d]) {
            rank = gidx - lt.offset[d];
            return d;
        }
    }
    rank = 0;
    return 0;
}

// Row pass of the FP64 rescore, split over row slices: for both signs of
// the set's vertex, the sum over rows [r0, r1) that the set does not touch
// of conj(V_i) omega^{label(V_i c)} -> out[s * 2R + j] (zeros without a
// full-rank vertex).
template <int R, int D>
__device__ void rescore_rows_one(const ExactParams& p, uint64_t rank, int64_t r0, int64_t r1, double* out) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    __shared__ double red[kBlock / kWave][2 * R];
    int64_t g[M];
    int mm[M];
    double v[C2];
    bool valid;
    const bool ok = vertex_blk<D>(p, rank, true, true, g, mm, v, valid);
    if (!ok) {
        if (threadIdx.x < 4 * R) out[threadIdx.x] = 0.0;
        return;
    }
    for (int s = 0; s < 2; ++s) {
        double cs[C2];
#pragma unroll
        for (int k = 0; k < C2; ++k) cs[k] = s ? -v[k] : v[k];
        double acc[2 * R];
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) acc[j] = 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
            bool touched = false;
#pragma unroll
            for (int t = 0; t < M; ++t) touched |= (i == g[t]);
            if (touched) continue;
            double wr = 0.0, wi = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double vr = p.V64[(i * p.r + j) * 2], vi = p.V64[(i * p.r + j) * 2 + 1];
                wr += vr * cs[j] - vi * cs[D + j];
                wi += vr * cs[D + j] + vi * cs[j];
            }
            const double2 z = p.roots64[label_f64(wr, wi, p.K)];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const double vr = p.V64[(i * R + j) * 2], vi = p.V64[(i * R + j) * 2 + 1];
                acc[2 * j] += vr * z.x + vi * z.y;
                acc[2 * j + 1] += vr * z.y - vi * z.x;
            }
        }
        const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) {
            const double x = wave_sum_f64(acc[j]);
            if (lane == 0) red[wave][j] = x;
        }
        __syncthreads();
        if (threadIdx.x < 2 * R) {
            double x = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) x += red[w][threadIdx.x];
            out[s * 2 * R + threadIdx.x] = x;
        }
        __syncthreads();
    }
}

template <int R, int D>
__device__ void rescore_one(ExactParams p, uint64_t rank, const double* part, int slices, RescoreEntry* out) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    __shared__ double base[2 * R];
    __shared__ double bf[kBlock];
    __shared__ long long bc[kBlock];
    int64_t g[M];
    int mm[M];
    double v[C2];
    bool valid;
    const bool ok = vertex_blk<D>(p, rank, true, true, g, mm, v, valid);
    RescoreEntry best{-1.0, 0, 0, 0};
    if (!ok) {
        if (threadIdx.x == 0) *out = best;
        return;
    }
    for (int s = 0; s < 2; ++s) {
        double cs[C2];
#pragma unroll
        for (int k = 0; k < C2; ++k) cs[k] = s ? -v[k] : v[k];
        // rows the set does not touch: the slice sums in slice order
        if (threadIdx.x < 2 * R) {
            double x = 0.0;
            for (int q = 0; q < slices; ++q) x += part[((size_t)q * 2 + s) * (2 * R) + threadIdx.x];
            base[threadIdx.x] = x;
        }
        __syncthreads();
        int o[M], cn[M];
        open_labels<D>(p, g, mm, cs, o, cn);
        int64_t total = 1;
#pragma unroll
        for (int t = 0; t < M; ++t) total *= cn[t];
        double myf = -1.0;
        long long myc = -1;
        for (int64_t combo = threadIdx.x; combo < total; combo += kBlock) {
            double sr[2 * R];
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) sr[j] = base[j];
            uint32_t rest = (uint32_t)combo;     // total <= 2^20 (checked on the host)
#pragma unroll
            for (int t = 0; t < M; ++t) {
                if (cn[t] == 1 && !((t == 0) || (g[t] != g[t - 1]))) continue;
                const int q = (int)(rest % (uint32_t)cn[t]);
                rest /= (uint32_t)cn[t];
                int k = o[t] + q;
                k = k >= p.K ? k - p.K : k;
                const double2 z = p.roots64[k];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const double vr = p.V64[(g[t] * R + j) * 2], vi = p.V64[(g[t] * R + j) * 2 + 1];
                    sr[2 * j] += vr * z.x + vi * z.y;
                    sr[2 * j + 1] += vr * z.y - vi * z.x;
                }
            }
            double f = 0.0;
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) f += sr[j] * sr[j];
            if (f > myf) {
                myf = f;
                myc = combo;
            }
        }
        bf[threadIdx.x] = myf;
        bc[threadIdx.x] = myc;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int t = 0; t < kBlock; ++t) {
                if (bc[t] < 0) continue;
                if (bf[t] > best.f || (bf[t] == best.f && s == best.sign && bc[t] < best.combo)) {
                    best.f = bf[t];
                    best.sign = s;
                    best.combo = bc[t];
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = best;
}

// Grid (kept sets, row slices): part[(t * slices + q) * 2 * 2R ..] holds
// both signs' sums over slice q of the rows.
template <int R>
__global__ __launch_bounds__(kBlock) void k_exact_rescore_rows(ExactParams p, LevelTable lt,
                                                               const TopEntry* top, int64_t rows,
                                                               double* part) {
    const int t = blockIdx.x, q = blockIdx.y;
    const int64_t r0 = min(p.n, (int64_t)q * rows), r1 = min(p.n, r0 + rows);
    double* out = part + ((size_t)t * gridDim.y + q) * 2 * (2 * R);
    uint64_t rank;
    const int d = top[t].f < 0.0f ? 0 : level_of(lt, R, top[t].gidx, rank);
    switch (d) {
        case 1: rescore_rows_one<R, 1>(p, rank, r0, r1, out); break;
        case 2: if constexpr (R >= 2) rescore_rows_one<R, 2>(p, rank, r0, r1, out); break;
        case 3: if constexpr (R >= 3) rescore_rows_one<R, 3>(p, rank, r0, r1, out); break;
        case 4: if constexpr (R >= 4) rescore_rows_one<R, 4>(p, rank, r0, r1, out); break;
        case 5: if constexpr (R >= 5) rescore_rows_one<R, 5>(p, rank, r0, r1, out); break;
        case 6: if constexpr (R >= 6) rescore_rows_one<R, 6>(p, rank, r0, r1, out); break;
        case 7: if constexpr (R >= 7) rescore_rows_one<R, 7>(p, rank, r0, r1, out); break;
        case 8: if constexpr (R >= 8) rescore_rows_one<R, 8>(p, rank, r0, r1, out); break;
        default:
            if (threadIdx.x < 4 * R) out[threadIdx.x] = 0.0;
    }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_exact_rescore(ExactParams p, LevelTable lt,
                                                          const TopEntry* top, const double* part,
                                                          int slices, RescoreEntry* out) {
    const int t = blockIdx.x;
    const double* pt = part + (size_t)t * slices * 2 * (2 * R);
    uint64_t rank;
    const int d = top[t].f < 0.0f ? 0 : level_of(lt, R, top[t].gidx, rank);
    switch (d) {
        case 1: rescore_one<R, 1>(p, rank, pt, slices, out + t); break;
        case 2: if constexpr (R >= 2) rescore_one<R, 2>(p, rank, pt, slices, out + t); break;
        case 3: if constexpr (R >= 3) rescore_one<R, 3>(p, rank, pt, slices, out + t); break;
        case 4: if constexpr (R >= 4) rescore_one<R, 4>(p, rank, pt, slices, out + t); break;
        case 5: if constexpr (R >= 5) rescore_one<R, 5>(p, rank, pt, slices, out + t); break;
        case 6: if constexpr (R >= 6) rescore_one<R, 6>(p, rank, pt, slices, out + t); break;
        case 7: if constexpr (R >= 7) rescore_one<R, 7>(p, rank, pt, slices, out + t); break;
        case 8: if constexpr (R >= 8) rescore_one<R, 8>(p, rank, pt, slices, out + t); break;
        default:
            if (threadIdx.x == 0) out[t] = RescoreEntry{-1.0, 0, 0, 0};
    }
}

__global__ void k_exact_pick(const RescoreEntry* __restrict__ e, const TopEntry* top,
                             int T, LevelTable lt, int r, ExactDevResult* res) {
    if (threadIdx.x != 0) return;
    int bt = -1;
    uint64_t bidx = ~0ull;
    for (int t = 0; t < T; ++t) {
        if (e[t].f < 0.0 || top[t].f < 0.0f) continue;
        const uint64_t idx = top[t].gidx;
        if (bt < 0 || e[t].f > e[bt].f || (e[t].f == e[bt].f && idx < bidx)) {
            bt = t;
            bidx = idx;
        }
    }
    if (bt < 0) {
        res->obj = -1.0;
        res->level = 0;
        return;
    }
    uint64_t rank;
    res->obj = e[bt].f;
    res->gidx = (int64_t)bidx;
    res->level = level_of(lt, r, bidx, rank);
    res->sign = e[bt].sign;
    res->combo = e[bt].combo;
}

template <int R, int D>
__device__ void labels_one(const ExactParams& p, uint64_t rank, const ExactDevResult& res,
                           int64_t i, uint8_t* z) {
    constexpr int M = 2 * D - 1, C2 = 2 * D;
    int64_t g[M];
    int mm[M];
    double v[C2];
    bool valid;
    vertex_blk<D>(p, rank, true, true, g, mm, v, valid);
    if (i >= p.n) return;
    double cs[C2];
#pragma unroll
    for (int k = 0; k < C2; ++k) cs[k] = res.sign ? -v[k] : v[k];
    int o[M], cn[M];
    open_labels<D>(p, g, mm, cs, o, cn);
    int64_t rest = res.combo;
    int lab = -1;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        if (cn[t] == 1 && !((t == 0) || (g[t] != g[t - 1]))) continue;
        const int q = (int)(rest % cn[t]);
        rest /= cn[t];
        int k = o[t] + q;
        k = k >= p.K ? k - p.K : k;
        if (g[t] == i) lab = k;
    }
    if (lab < 0) {
        double wr = 0.0, wi = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double vr = p.V64[(i * p.r + j) * 2], vi = p.V64[(i * p.r + j) * 2 + 1];
            wr += vr * cs[j] - vi * cs[D + j];
            wi += vr * cs[D + j] + vi * cs[j];
        }
        lab = label_f64(wr, wi, p.K);
    }
    z[i] = (uint8_t)lab;
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_exact_labels(ExactParams p, LevelTable lt,
                                                         const ExactDevResult* __restrict__ res,
                                                         uint8_t* __restrict__ z) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;   // rows past n only join the barriers
    if (res->level == 0) return;
    uint64_t rank;
    const int d = level_of(lt, R, (uint64_t)res->gidx, rank);
    switch (d) {
        case 1: labels_one<R, 1>(p, rank, *res, i, z); break;
        case 2: if constexpr (R >= 2) labels_one<R, 2>(p, rank, *res, i, z); break;
        case 3: if constexpr (R >= 3) labels_one<R, 3>(p, rank, *res, i, z); break;
        case 4: if constexpr (R >= 4) labels_one<R, 4>(p, rank, *res, i, z); break;
        case 5: if constexpr (R >= 5) labels_one<R, 5>(p, rank, *res, i, z); break;
        case 6: if constexpr (R >= 6) labels_one<R, 6>(p, rank, *res, i, z); break;
        case 7: if constexpr (R >= 7) labels_one<R, 7>(p, rank, *res, i, z); break;
        case 8: if constexpr (R >= 8) labels_one<R, 8>(p, rank, *res, i, z); break;
        default: break;
    }
}

// ---------------------------------------------------------------- host
// Bytes of the split form's buffers: one record per set, and the slice sums
// (two signs, 2r components) per set and slice.
uint64_t split_bytes(uint64_t count, int slices, int r) {
    return count * (vertex_rec_bytes(r) + (uint64_t)slices * 2 * (2 * r) * sizeof(float));
}

unsigned __int128 binom128(int64_t x, int k) {
    if (k < 0 || x < k) return 0;
    unsigned __int128 c = 1;
    for (int t = 1; t <= k; ++t) {
        c = c * (unsigned __int128)(x - k + t) / (unsigned __int128)t;
        if (c > ((unsigned __int128)1 << 100)) return (unsigned __int128)1 << 100;
    }
    return c;
}

int boundary_count(int K) { return (K % 2 == 0) ? K / 2 : K; }

// Split form for a level of `count` sets when its buffers fit in
// kSplitBytes: row slices so that the grid fills the chip several times
// over, slices of at least 1024 rows.  Returns the slice count (0: fused).
constexpr uint64_t kSplitBytes = 128ull << 20;

// Form of a level's launch: kFormAuto takes the split form only where it
// slices the rows (one slice would solve each vertex twice for nothing);
// the other two force a form (the split one still needs its buffers).
constexpr int kFormAuto = 0, kFormFused = 1, kFormSplit = 2;

int exact_slices(uint64_t count, int64_t n, int r, int64_t& rows, int form) {
    if (form == kFormFused) return 0;
    const uint64_t blocks = std::min<uint64_t>((count + kBlock - 1) / kBlock, 8192);
    int64_t slices = std::max<int64_t>(1, (int64_t)((2048 + blocks - 1) / blocks));
    slices = std::min<int64_t>(slices, std::max<int64_t>(1, n / 1024));
    rows = (n + slices - 1) / slices;
    rows = ((rows + 63) / 64) * 64;
    slices = (n + rows - 1) / rows;
    if (split_bytes(count, (int)slices, r) > kSplitBytes) return 0;
    if (slices == 1 && form != kFormSplit) return 0;
    return (int)slices;
}

// r > 4 takes the generic quantiser (atan2 and the root table) only: at the
// sizes such enumerations reach (n of a few tens) the row pass is not what
// costs, the vertex solves and the label combinations are.
template <int R, int D>
void launch_level(ExactParams p, int form, hipStream_t st) {
    const uint64_t blocks = std::min<uint64_t>((p.count + kBlock - 1) / kBlock, 8192);
    const int slices = exact_slices(p.count, p.n, R, p.rows_per_slice, form);
    const int ks = R > kThreadMaxD ? 0 : p.K;
    if (slices == 0) {
        switch (ks) {
            case 2: if constexpr (R <= kThreadMaxD) hipLaunchKernelGGL((k_exact_score<R, D, 2>), dim3((unsigned)blocks), dim3(kBlock), 0, st, p); break;
            case 3: if constexpr (R <= kThreadMaxD) hipLaunchKernelGGL((k_exact_score<R, D, 3>), dim3((unsigned)blocks), dim3(kBlock), 0, st, p); break;
            case 4: if constexpr (R <= kThreadMaxD) hipLaunchKernelGGL((k_exact_score<R, D, 4>), dim3((unsigned)blocks), dim3(kBlock), 0, st, p); break;
            default: hipLaunchKernelGGL((k_exact_score<R, D, 0>), dim3((unsigned)blocks), dim3(kBlock), 0, st, p); break;
        }
        return;
    }
    VertexRec<D>* recs = static_cast<VertexRec<D>*>(p.recs);
    hipLaunchKernelGGL((k_exact_vertex<D>), dim3((unsigned)blocks), dim3(kBlock), 0, st, p, recs);
    const dim3 grid((unsigned)blocks, (unsigned)slices);
    switch (ks) {
        case 2: if constexpr (R <= kThreadMaxD) hipLaunchKernelGGL((k_exact_rows<R, D, 2>), grid, dim3(kBlock), 0, st, p, recs); break;
        case 3: if constexpr (R <= kThreadMaxD) hipLaunchKernelGGL((k_exact_rows<R, D, 3>), grid, dim3(kBlock), 0, st, p, recs); break;
        case 4: if constexpr (R <= kThreadMaxD) hipLaunchKernelGGL((k_exact_rows<R, D, 4>), grid, dim3(kBlock), 0, st, p, recs); break;
        default: hipLaunchKernelGGL((k_exact_rows<R, D, 0>), grid, dim3(kBlock), 0, st, p, recs); break;
    }
    hipLaunchKernelGGL((k_exact_combine<R, D>), dim3((unsigned)blocks), dim3(kBlock), 0, st, p, slices);
}

template <int R>
lrqo_status run_exact(ExactParams p, const LevelTable& lt, uint64_t chunk, int form, TopEntry* top,
                      unsigned long long* ka, unsigned long long* kb, float* floor_buf, RescoreEntry* entries,
                      double* rpart, ExactDevResult* dres, uint8_t* z, hipStream_t st) {
    hipLaunchKernelGGL(k_exact_top_init, dim3(1), dim3(kTopT), 0, st, top);
    bool first = true;
    for (int d = R; d >= 1; --d) {
        for (uint64_t c0 = 0; c0 < lt.count[d]; c0 += chunk) {
            ExactParams q = p;
            q.count = std::min<uint64_t>(chunk, lt.count[d] - c0);
            q.rank0 = c0;
            switch (d) {
                case 1: launch_level<R, 1>(q, form, st); break;
                case 2: if constexpr (R >= 2) launch_level<R, 2>(q, form, st); break;
                case 3: if constexpr (R >= 3) launch_level<R, 3>(q, form, st); break;
                case 4: if constexpr (R >= 4) launch_level<R, 4>(q, form, st); break;
                case 5: if constexpr (R >= 5) launch_level<R, 5>(q, form, st); break;
                case 6: if constexpr (R >= 6) launch_level<R, 6>(q, form, st); break;
                case 7: if constexpr (R >= 7) launch_level<R, 7>(q, form, st); break;
                case 8: if constexpr (R >= 8) launch_level<R, 8>(q, form, st); break;
            }
            LRQO_HIP(hipGetLastError());
            const int T = (int)std::min<uint64_t>(kTopT, q.count);
            const unsigned long long* keys = nullptr;
            // a score below the shortlist's last (once it holds kTopT values)
            // cannot enter it: the selection drops those on the device.  The
            // first chunk, with the shortlist still empty, takes its floor
            // from the maxima of its groups of scores instead.
            const float* floor_f = reinterpret_cast<const float*>(top + (kTopT - 1));
            if (first && T == kTopT && q.count >= (uint64_t)kFloorGroup * kTopT) {
                LRQO_TRY(topk_block_floor(p.fbuf, (uint32_t)q.count, T, floor_f, floor_buf, ka, kb, st));
                floor_f = floor_buf;
            }
            first = false;
            LRQO_TRY(topk_select(p.fbuf, (uint32_t)q.count, T, ka, kb, st, &keys, true, floor_f));
            hipLaunchKernelGGL(k_exact_merge, dim3(1), dim3(kTopT), 0, st, top, keys, T, lt.offset[d] + c0);
            LRQO_HIP(hipGetLastError());
        }
    }
    const int64_t rrows = std::max<int64_t>(4096, (p.n + kRescoreSlices - 1) / kRescoreSlices);
    const int rslices = (int)((p.n + rrows - 1) / rrows);
    hipLaunchKernelGGL((k_exact_rescore_rows<R>), dim3(kTopT, rslices), dim3(kBlock), 0, st, p, lt, top, rrows,
                       rpart);
    hipLaunchKernelGGL((k_exact_rescore<R>), dim3(kTopT), dim3(kBlock), 0, st, p, lt, top, rpart, rslices, entries);
    LRQO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_exact_pick, dim3(1), dim3(64), 0, st, entries, top, kTopT, lt, R, dres);
    LRQO_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_exact_labels<R>), dim3((unsigned)((p.n + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, p, lt, dres, z);
    LRQO_HIP(hipGetLastError());
    return LRQO_OK;
}

// Sets per enumeration chunk: each chunk's scores (4 bytes per set) are
// reduced to its best distinct values before the next chunk is scored.
uint64_t exact_chunk() {
    const char* e = std::getenv("LRQO_EXACT_CHUNK");
    if (e && *e) {
        const long long v = std::atoll(e);
        if (v >= 1) return (uint64_t)v;
    }
    return kChunkSets;
}

// LRQO_EXACT_FORM = fused / split forces a form (for tests); unset: auto.
int exact_form() {
    const char* e = std::getenv("LRQO_EXACT_FORM");
    if (e && std::strcmp(e, "fused") == 0) return kFormFused;
    if (e && std::strcmp(e, "split") == 0) return kFormSplit;
    return kFormAuto;
}

// Shared by the exact enumeration (random = false: every valid index set of
// every level, colex order) and the null-vector sampler (random = true:
// S drawn index sets of level r).
lrqo_status vertex_solve(const double* V, int64_t n, int32_t r, int32_t K, int64_t max_sets, bool random,
                         int64_t S, uint64_t seed, uint8_t* z, lrqo_exact_result* res) {
    clear_error();
    if (!V) return fail(LRQO_EINVAL, "V is null");
    if (!z) return fail(LRQO_EINVAL, "z is null");
    if (r < 1 || r > kMaxR) return fail(LRQO_EINVAL, "r must be in [1, 8] for the vertex solvers");
    if (n < r || n > INT32_MAX) return fail(LRQO_EINVAL, "n must be in [r, 2^31 - 1]");
    if (K < 2 || K > LRQO_MAX_K) return fail(LRQO_EINVAL, "K must be in [2, 255]");
    if (random && (S < 1 || S > 0x7FFFFFFFll)) return fail(LRQO_EINVAL, "S must be in [1, 2^31 - 1]");
    const int B = boundary_count(K);
    const int64_t N = n * B;
    // label combinations of one vertex: at most 2^(2r-1-2p) K^p, p double groups
    for (int pdbl = 0; 2 * pdbl <= 2 * r - 1; ++pdbl) {
        long double combos = std::ldexp(1.0L, 2 * r - 1 - 2 * pdbl) * std::pow((long double)K, pdbl);
        if (combos > (long double)kMaxCombos)
            return fail(LRQO_ETOOBIG, "label combinations per vertex exceed 2^20 (K too large for r)");
    }
    const unsigned __int128 cap = max_sets > 0 ? (unsigned __int128)max_sets
                                  : max_sets == 0 ? (unsigned __int128)kDefaultMaxSets
                                                  : (unsigned __int128)kHardMaxSets;
    LevelTable lt{};
    unsigned __int128 total128 = 0;
    if (random) {
        lt.offset[r] = 0;
        lt.count[r] = (uint64_t)S;
        total128 = (unsigned __int128)S;
    } else {
        for (int d = r; d >= 1; --d) {
            const unsigned __int128 c = binom128(N, 2 * d - 1);
            lt.offset[d] = (uint64_t)std::min<unsigned __int128>(total128, kHardMaxSets);
            lt.count[d] = (uint64_t)std::min<unsigned __int128>(c, kHardMaxSets);
            total128 += c;
        }
        if (total128 > cap || total128 > (unsigned __int128)kHardMaxSets)
            return fail(LRQO_ETOOBIG, "number of index sets C(n B_K, 2d-1) summed over levels exceeds the cap "
                                      "(max_sets; 0 means 2^34, a negative value lifts it up to 2^62)");
    }

    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    if (!is_device_pointer(V)) return fail(LRQO_EINVAL, "V is not device memory");
    if (!is_device_pointer(z)) return fail(LRQO_EINVAL, "z is not device memory");

    const uint64_t chunk = random ? (uint64_t)S : exact_chunk();
    const int form = exact_form();
    const int rk = r <= kThreadMaxD ? r : kMaxR;     // columns the kernels see
    const bool pad = rk != r;                        // 4 < r < kMaxR: a zero-padded copy of V
    uint64_t cmax = 0;                   // the largest chunk
    for (int d = r; d >= 1; --d) cmax = std::max<uint64_t>(cmax, std::min<uint64_t>(chunk, lt.count[d]));
    const int Mmax = 2 * r - 1;
    const size_t binom_entries = (random || Mmax < 2) ? 1 : (size_t)(Mmax + 1) * (size_t)(N + 1);
    uint64_t rec_count = 0, part_floats = 0;     // the largest split chunk's needs
    if (form != kFormFused) {
        for (int d = r; d >= 1; --d) {
            if (lt.count[d] == 0) continue;
            const uint64_t cnt = std::min<uint64_t>(chunk, lt.count[d]);
            int64_t rows = 0;
            const int sl = exact_slices(cnt, n, rk, rows, form);
            if (sl == 0) continue;
            rec_count = std::max<uint64_t>(rec_count, cnt);
            part_floats = std::max<uint64_t>(part_floats, cnt * (uint64_t)sl * 2 * (2 * rk));
        }
    }
    CarveSize cs;
    cs.add<ExactDevResult>(1);
    cs.add<unsigned long long>(3 * kStatSlots);
    cs.add<float>((size_t)n * rk * 2);
    cs.add<double>(pad ? (size_t)n * rk * 2 : 0);
    cs.add<unsigned long long>(binom_entries);
    cs.add<double2>(LRQO_MAX_K);
    cs.add<double2>(LRQO_MAX_K);
    cs.add<float2>(LRQO_MAX_K);
    cs.add<float>(cmax);
    cs.add<unsigned long long>(topk_buffer_keys((uint32_t)cmax, kTopT));
    cs.add<unsigned long long>(topk_buffer_keys((uint32_t)cmax, kTopT));
    cs.add<TopEntry>(kTopT);
    cs.add<float>(1);
    cs.add<RescoreEntry>(kTopT);
    cs.add<double>((size_t)kTopT * kRescoreSlices * 2 * (2 * rk));
    cs.add<char>(rec_count * vertex_rec_bytes(rk));
    cs.add<float>(part_floats);
    const size_t host_bytes = 4096 + binom_entries * sizeof(unsigned long long) +
                              LRQO_MAX_K * (2 * sizeof(double2) + sizeof(float2));

    std::lock_guard<std::mutex> lk(ctx->mu);
    LRQO_TRY(reserve_arena(ctx, cs.bytes));
    LRQO_TRY(reserve_host(ctx, host_bytes));
    hipStream_t st = current_stream();
    Carve cv(ctx->arena);
    ExactDevResult* dres = cv.take<ExactDevResult>(1);
    unsigned long long* stats = cv.take<unsigned long long>(3 * kStatSlots);
    float* V32 = cv.take<float>((size_t)n * rk * 2);
    double* Vpad = pad ? cv.take<double>((size_t)n * rk * 2) : nullptr;
    unsigned long long* binom = cv.take<unsigned long long>(binom_entries);
    double2* rho = cv.take<double2>(LRQO_MAX_K);
    double2* roots64 = cv.take<double2>(LRQO_MAX_K);
    float2* roots32 = cv.take<float2>(LRQO_MAX_K);
    float* fbuf = cv.take<float>(cmax);
    unsigned long long* ka = cv.take<unsigned long long>(topk_buffer_keys((uint32_t)cmax, kTopT));
    unsigned long long* kb = cv.take<unsigned long long>(topk_buffer_keys((uint32_t)cmax, kTopT));
    TopEntry* top = cv.take<TopEntry>(kTopT);
    float* floor_buf = cv.take<float>(1);
    RescoreEntry* entries = cv.take<RescoreEntry>(kTopT);
    double* rpart = cv.take<double>((size_t)kTopT * kRescoreSlices * 2 * (2 * rk));
    void* recs = cv.take<char>(rec_count * vertex_rec_bytes(rk));
    float* part = cv.take<float>(part_floats);

    // host tables (pinned staging): result block, binomials, rho, roots
    char* hb = static_cast<char*>(ctx->host);
    ExactDevResult* hres = reinterpret_cast<ExactDevResult*>(hb);
    unsigned long long* hstats = reinterpret_cast<unsigned long long*>(hb + 256);
    unsigned long long* hbin = reinterpret_cast<unsigned long long*>(hb + 4096);
    double2* hrho = reinterpret_cast<double2*>(hbin + binom_entries);
    double2* hr64 = hrho + LRQO_MAX_K;
    float2* hr32 = reinterpret_cast<float2*>(hr64 + LRQO_MAX_K);
    // C(x, k) by Pascal's rule, saturating at 2^64-1 (only values below the
    // set count, < 2^62, are ever compared exactly)
    if (binom_entries == 1) hbin[0] = 0;
    else
        for (int k = 0; k <= Mmax; ++k)
            for (int64_t x = 0; x <= N; ++x) {
                unsigned long long c;
                if (k == 0) c = 1;
                else if (x == 0) c = 0;
                else {
                    const unsigned long long a = hbin[(size_t)k * (N + 1) + x - 1];
                    const unsigned long long b = hbin[(size_t)(k - 1) * (N + 1) + x - 1];
                    c = (a > ~0ull - b) ? ~0ull : a + b;
                }
                hbin[(size_t)k * (N + 1) + x] = c;
            }
    const double pi = 3.14159265358979323846264338327950288;
    for (int m = 0; m < B; ++m) {
        const double a = -pi * (2.0 * m + 1.0) / (double)K;
        hrho[m] = make_double2(std::cos(a), std::sin(a));
    }
    for (int k = 0; k < K; ++k) {
        const double a = 2.0 * pi * (double)k / (double)K;
        hr64[k] = make_double2(std::cos(a), std::sin(a));
        hr32[k] = make_float2((float)hr64[k].x, (float)hr64[k].y);
    }

    LRQO_HIP(hipEventRecord(ctx->ev_start, st));
    LRQO_HIP(hipMemcpyAsync(binom, hbin, binom_entries * sizeof(unsigned long long),
                            hipMemcpyHostToDevice, st));
    LRQO_HIP(hipMemcpyAsync(rho, hrho, sizeof(double2) * B, hipMemcpyHostToDevice, st));
    LRQO_HIP(hipMemcpyAsync(roots64, hr64, sizeof(double2) * K, hipMemcpyHostToDevice, st));
    LRQO_HIP(hipMemcpyAsync(roots32, hr32, sizeof(float2) * K, hipMemcpyHostToDevice, st));
    LRQO_HIP(hipMemsetAsync(dres, 0, sizeof(ExactDevResult), st));
    LRQO_HIP(hipMemsetAsync(stats, 0, 3 * kStatSlots * sizeof(unsigned long long), st));

    ExactParams p{};
    p.V64 = pad ? Vpad : V;
    p.V32 = V32;
    p.n = n;
    p.r = rk;
    p.K = K;
    p.B = B;
    p.N = N;
    p.binom = binom;
    p.rho = rho;
    p.roots64 = roots64;
    p.roots32 = roots32;
    p.fbuf = fbuf;
    p.stats = stats;
    p.random = random ? 1 : 0;
    p.draw_seed = seed;
    p.part = part;
    p.recs = recs;

    const int64_t vcount = n * rk * 2;
    int* nonfinite = &dres->nonfinite;
    int* complex_v = &dres->complex_v;
    p.complex_v = complex_v;
    uint32_t* vmax_bits = &dres->vmax_bits;
    p.vmax_bits = vmax_bits;
    lrqo_status s = LRQO_OK;
    switch (r) {
        case 1:
            hipLaunchKernelGGL((k_to_f32<1>), dim3(256), dim3(256), 0, st, V, V32, vcount, nonfinite, complex_v,
                               vmax_bits);
            s = run_exact<1>(p, lt, chunk, form, top, ka, kb, floor_buf, entries, rpart, dres, z, st);
            break;
        case 2:
            hipLaunchKernelGGL((k_to_f32<2>), dim3(256), dim3(256), 0, st, V, V32, vcount, nonfinite, complex_v,
                               vmax_bits);
            s = run_exact<2>(p, lt, chunk, form, top, ka, kb, floor_buf, entries, rpart, dres, z, st);
            break;
        case 3:
            hipLaunchKernelGGL((k_to_f32<3>), dim3(256), dim3(256), 0, st, V, V32, vcount, nonfinite, complex_v,
                               vmax_bits);
            s = run_exact<3>(p, lt, chunk, form, top, ka, kb, floor_buf, entries, rpart, dres, z, st);
            break;
        case 4:
            hipLaunchKernelGGL((k_to_f32<4>), dim3(256), dim3(256), 0, st, V, V32, vcount, nonfinite, complex_v,
                               vmax_bits);
            s = run_exact<4>(p, lt, chunk, form, top, ka, kb, floor_buf, entries, rpart, dres, z, st);
            break;
        default:
            if (pad) hipLaunchKernelGGL(k_pad_columns, dim3(256), dim3(256), 0, st, V, Vpad, n, r);
            hipLaunchKernelGGL((k_to_f32<kMaxR>), dim3(256), dim3(256), 0, st, p.V64, V32, vcount, nonfinite,
                               complex_v, vmax_bits);
            s = run_exact<kMaxR>(p, lt, chunk, form, top, ka, kb, floor_buf, entries, rpart, dres, z, st);
            break;
    }
    if (s != LRQO_OK) return s;
    LRQO_HIP(hipMemcpyAsync(hres, dres, sizeof(ExactDevResult), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipMemcpyAsync(hstats, stats, 3 * kStatSlots * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipEventRecord(ctx->ev_stop, st));
    LRQO_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    LRQO_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
    if (hres->nonfinite) return fail(LRQO_ENOTFINITE, "V holds a NaN or an infinity");
    if (hres->level == 0)
        return fail(random ? LRQO_EINVAL : LRQO_EDEVICE,
                    random ? "no feasible draw among the S draws" : "no full-rank vertex found (degenerate V)");
    if (res) {
        std::memset(res, 0, sizeof *res);
        res->obj = hres->obj;
        int64_t sum3[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c)
            for (int q = 0; q < kStatSlots; ++q) sum3[c] += (int64_t)hstats[c * kStatSlots + q];
        res->index_sets = sum3[0];
        res->rank_deficient = sum3[1];
        res->candidates = sum3[2];
        res->device_ms = ms;
        // general position (Assumption 1) implies every valid set has full
        // rank; a rank-deficient set shows the input violates it
        res->warning = sum3[1] > 0 ? LRQO_EDEGENERATE : LRQO_OK;
    }
    return LRQO_OK;
}

}  // namespace
}  // namespace lrqo

extern "C" {

lrqo_status lrqo_solve_exact_ex(const double* V, int64_t n, int32_t r, int32_t K,
                                int64_t max_sets, uint8_t* z, lrqo_exact_result* res) {
    return lrqo::vertex_solve(V, n, r, K, max_sets, false, 0, 0, z, res);
}

lrqo_status lrqo_solve_nullvec(const double* V, int64_t n, int32_t r, int32_t K, int64_t S, uint64_t seed,
                               uint8_t* z, lrqo_exact_result* res) {
    return lrqo::vertex_solve(V, n, r, K, 0, true, S, seed, z, res);
}

lrqo_status lrqo_solve_exact(const double* V, int64_t n, int32_t r, int32_t K, uint8_t* z,
                             double* obj) {
    if (!obj) return lrqo::fail(LRQO_EINVAL, "obj is null");
    lrqo_exact_result res;
    const lrqo_status st = lrqo_solve_exact_ex(V, n, r, K, 0, z, &res);
    if (st == LRQO_OK) *obj = res.obj;
    return st;
}

}  // extern "C"
