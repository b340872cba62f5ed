// Objective on the graph and greedy local refinement (appendix "Rank-1 at
// Scale": incremental scoring, eq. incremental; hybrid warm start) for the
// Laplacian Q = L = D - A of a weighted graph in CSR.
//
// Kernels:
//   k_check_ptr     row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
//   k_check_rows    0 <= col < n, no self loop, finite weights, labels < K
//                   (only after k_check_ptr passed: it reads col through row_ptr)
//   k_objective     per vertex: sum over its entries of w |z_i - z_j|^2 and of
//                   w [k_i != k_j] (each edge is seen from both ends), block
//                   partial sums in a fixed order
//   k_sum2          fixed-order sum of the block partials
//   k_gain          per vertex: neighbour label weights c_k in LDS, the best
//                   other label and its gain 2 sum_k c_k (cos(a-k) - cos(b-k))
//   k_move          per candidate: moves when its (gain, -index) beats every
//                   neighbouring candidate; labels go to the other buffer;
//                   moves counted per round (per block, into 64 counters)
// Rounds go out in batches between host checks; a round whose predecessor
// moved nothing returns at once, so a batch that converges early costs a
// launch per remaining round.
// One thread per vertex; the CSR entries of a vertex are read in order, so
// every per-vertex sum has a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "graph_internal.h"
#include "lrqo_device.h"
#include "lrqo_runtime.h"

namespace lrqo {

namespace {

constexpr int kBlock = 256;
#ifndef LRQO_REFINE_BLOCK
#define LRQO_REFINE_BLOCK 512
#endif
constexpr int kRefineBlock = LRQO_REFINE_BLOCK;   // threads per block of the gain and move kernels
constexpr int kMaxKRefine = 16;

enum : int { kBadPtr = 1, kBadCol = 2, kBadWeight = 4, kBadLabel = 8 };

struct GraphDev {
    const int64_t* row_ptr;
    const int32_t* col;
    const double* w;
    int64_t n;
    int64_t nnz;
};

__global__ __launch_bounds__(kBlock) void k_check_ptr(GraphDev g, int* flag) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    bool bad = false;
    if (i < g.n) bad = g.row_ptr[i] > g.row_ptr[i + 1];
    if (i == 0) bad = bad || g.row_ptr[0] != 0 || g.row_ptr[g.n] != g.nnz;
    if (bad) atomicOr(flag, kBadPtr);
}

__global__ __launch_bounds__(kBlock) void k_check_rows(GraphDev g, int K, const uint8_t* z, int* flag) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= g.n) return;
    int bad = (z && z[i] >= K) ? kBadLabel : 0;
    for (int64_t e = g.row_ptr[i]; e < g.row_ptr[i + 1]; ++e) {
        const int32_t j = g.col[e];
        if (j < 0 || j >= g.n || j == i) bad |= kBadCol;
        if (g.w && !isfinite(g.w[e])) bad |= kBadWeight;
    }
    if (bad) atomicOr(flag, bad);
}

// Block sums of two doubles per thread, fixed tree order.
__device__ __forceinline__ void block_sum2(double a, double b, double* out) {
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
    if (threadIdx.x == 0) {
        out[0] = sa[0];
        out[1] = sb[0];
    }
}

// sqd[d] = |1 - omega^d|^2 for the label difference d = (k_i - k_j) mod K.
// The terms of the entries [e, e1) of vertex i (label a) in chunks of U:
// the U column and weight loads, then the U label loads, are issued
// together; the additions keep entry order.  Leaves e at the first entry of
// an incomplete chunk.
template <int U>
__device__ __forceinline__ void objective_chunk(const GraphDev& g, int K, const uint8_t* __restrict__ z,
                                                const double* __restrict__ sqd, int a, int64_t& e, int64_t e1,
                                                double& q, double& cut) {
    for (; e + U <= e1; e += U) {
        int32_t c[U];
        double w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = g.col[e + u];
            w[u] = g.w ? g.w[e + u] : 1.0;
        }
        int b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) b[u] = z[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int d = a - b[u];
            d += d < 0 ? K : 0;
            q += w[u] * sqd[d];
            cut += a != b[u] ? w[u] : 0.0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_objective(GraphDev g, int K, const uint8_t* __restrict__ z,
                                                      const double* __restrict__ sqd,
                                                      double* __restrict__ partial) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    double q = 0.0, cut = 0.0;
    if (i < g.n) {
        const int a = z[i];
        int64_t e = g.row_ptr[i];
        const int64_t e1 = g.row_ptr[i + 1];
        objective_chunk<8>(g, K, z, sqd, a, e, e1, q, cut);
        objective_chunk<4>(g, K, z, sqd, a, e, e1, q, cut);
        for (; e < e1; ++e) {
            const int b = z[g.col[e]];
            const double w = g.w ? g.w[e] : 1.0;
            int d = a - b;
            d += d < 0 ? K : 0;
            q += w * sqd[d];
            cut += a != b ? w : 0.0;
        }
    }
    block_sum2(q, cut, partial + 2 * blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_sum2(const double* __restrict__ partial, int64_t blocks,
                                                 double* __restrict__ out) {
    double a = 0.0, b = 0.0;
    for (int64_t t = threadIdx.x; t < blocks; t += kBlock) {
        a += partial[2 * t];
        b += partial[2 * t + 1];
    }
    block_sum2(a, b, out);
}

constexpr int kMoveLanes = 64;

// Whether the previous round (its kMoveLanes counters; none for the first
// round of a batch) moved nothing: then this round and every later one of
// the batch would leave the labels unchanged, and is skipped.  Lane l reads
// counter l and the wave votes, so every lane of the wave must be active.
static_assert(kMoveLanes == kWave, "one move counter per lane");
__device__ __forceinline__ bool no_moves(const unsigned long long* __restrict__ prev) {
    if (!prev) return false;
    return __ballot(prev[threadIdx.x & (kWave - 1)] != 0ull) == 0ull;
}

// Label weights of the entries [e, e1) in chunks of U: the U column and
// weight loads, then the U label loads, are issued together; the additions
// keep entry order.  Leaves e at the first entry of an incomplete chunk.
template <int U>
__device__ __forceinline__ void gain_chunk(const GraphDev& g, const uint8_t* __restrict__ z, int64_t& e,
                                           int64_t e1, double (*cnt)[kRefineBlock], double& wdeg) {
    for (; e + U <= e1; e += U) {
        int32_t c[U];
        double w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = g.col[e + u];
            w[u] = g.w ? g.w[e + u] : 1.0;
        }
        uint8_t l[U];
#pragma unroll
        for (int u = 0; u < U; ++u) l[u] = z[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cnt[l[u]][threadIdx.x] += w[u];
            wdeg += fabs(w[u]);
        }
    }
}

// Whether a neighbour in [e, e1) beats (gi, i), U neighbours' gains in
// flight at a time; stops at the first chunk that holds one.
template <int U>
__device__ __forceinline__ void move_chunk(const GraphDev& g, const double* __restrict__ gain, int64_t i, double gi,
                                           int64_t& e, int64_t e1, bool& win) {
    for (; win && e + U <= e1; e += U) {
        int32_t j[U];
        double gj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = g.col[e + u];
#pragma unroll
        for (int u = 0; u < U; ++u) gj[u] = gain[j[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (gj[u] > 0.0 && (gj[u] > gi || (gj[u] == gi && j[u] < i))) win = false;
    }
}

// cosd[d] = cos(2 pi d / K).  Gain of moving i from a to b:
// 2 sum_k c_k (cosd[(a-k) mod K] - cosd[(b-k) mod K]).
template <int KM>
__global__ __launch_bounds__(kRefineBlock) void k_gain(GraphDev g, int K, const uint8_t* __restrict__ z,
                                                 const double* __restrict__ cosd,
                                                 double* __restrict__ gain, uint8_t* __restrict__ target,
                                                 const unsigned long long* __restrict__ prev) {
    __shared__ double cnt[KM][kRefineBlock];   // KM >= K rows
    const int64_t i = blockIdx.x * (int64_t)kRefineBlock + threadIdx.x;
    if (no_moves(prev) || i >= g.n) return;   // the vote first, with every lane active
    for (int k = 0; k < K; ++k) cnt[k][threadIdx.x] = 0.0;
    double wdeg = 0.0;
    int64_t e = g.row_ptr[i];
    const int64_t e1 = g.row_ptr[i + 1];
    // eight, then four entries' loads in flight at a time; the sums stay in
    // entry order
    gain_chunk<8>(g, z, e, e1, cnt, wdeg);
    gain_chunk<4>(g, z, e, e1, cnt, wdeg);
    for (; e < e1; ++e) {
        const double w = g.w ? g.w[e] : 1.0;
        cnt[z[g.col[e]]][threadIdx.x] += w;
        wdeg += fabs(w);
    }
    const int a = z[i];
    double best = -INFINITY;
    int bl = a;
    for (int b = 0; b < K; ++b) {
        if (b == a) continue;
        double d = 0.0;
        for (int k = 0; k < K; ++k) {
            const int da = a - k + (a < k ? K : 0), db = b - k + (b < k ? K : 0);
            d += cnt[k][threadIdx.x] * (cosd[da] - cosd[db]);
        }
        d *= 2.0;
        if (d > best) {
            best = d;
            bl = b;
        }
    }
    const bool cand = best > 1e-12 * wdeg;
    gain[i] = cand ? best : 0.0;
    target[i] = (uint8_t)(cand ? bl : a);
}


__global__ __launch_bounds__(kRefineBlock) void k_move(GraphDev g, const uint8_t* __restrict__ z,
                                                 const double* __restrict__ gain,
                                                 const uint8_t* __restrict__ target,
                                                 uint8_t* __restrict__ z_next,
                                                 unsigned long long* __restrict__ moves,
                                                 const unsigned long long* __restrict__ prev) {
    const int64_t i = blockIdx.x * (int64_t)kRefineBlock + threadIdx.x;
    if (no_moves(prev)) return;   // uniform over the grid
    bool win = false;
    if (i < g.n) {
        const double gi = gain[i];
        win = gi > 0.0;
        int64_t e = g.row_ptr[i];
        const int64_t e1 = g.row_ptr[i + 1];
        // eight, then four neighbours' gains in flight at a time
        move_chunk<8>(g, gain, i, gi, e, e1, win);
        move_chunk<4>(g, gain, i, gi, e, e1, win);
        for (; win && e < e1; ++e) {
            const int32_t j = g.col[e];
            const double gj = gain[j];
            if (gj > 0.0 && (gj > gi || (gj == gi && j < i))) win = false;
        }
        z_next[i] = win ? target[i] : z[i];
    }
    // the block's count into one of kMoveLanes counters (block index mod
    // kMoveLanes), so that same-address atomics stay few (at 10^6 vertices
    // 1,954 blocks share them)
    __shared__ unsigned int wm[kRefineBlock / kWave];
    const unsigned long long bal = __ballot(win);
    if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = (unsigned)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < kRefineBlock / kWave; ++w) b += wm[w];
        if (b) atomicAdd(&moves[blockIdx.x % kMoveLanes], b);
    }
}

struct GraphScratch {
    int* flag;
    double* partial;
    double* out2;
    double* table;        // sqd[K] then cosd[K]
    double* gain;
    uint8_t* target;
    uint8_t* zb;
    unsigned long long* moves;
};

constexpr int kMaxCheck = 64;

struct HostScratch {
    double* out;                  // [4]
    int* flag;                    // [16]
    unsigned long long* moves;    // [kMaxCheck][kMoveLanes]
    double* table;                // [2 * LRQO_MAX_K]
};

lrqo_status reserve_graph(DeviceCtx* ctx, int64_t n, bool refine, GraphScratch& s, HostScratch& h) {
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    CarveSize cs;
    cs.add<int>(16);
    cs.add<double>(2 * blocks);
    cs.add<double>(4);
    cs.add<double>(2 * LRQO_MAX_K);
    if (refine) {
        cs.add<double>(n);
        cs.add<uint8_t>(n);
        cs.add<uint8_t>(n);
        cs.add<unsigned long long>(kMaxCheck * kMoveLanes);
    }
    CarveSize hs;
    hs.add<double>(4);
    hs.add<int>(16);
    hs.add<unsigned long long>(kMaxCheck * kMoveLanes);
    hs.add<double>(2 * LRQO_MAX_K);
    LRQO_TRY(reserve_arena(ctx, cs.bytes));
    LRQO_TRY(reserve_host(ctx, hs.bytes));
    Carve cv(ctx->arena);
    s.flag = cv.take<int>(16);
    s.partial = cv.take<double>(2 * blocks);
    s.out2 = cv.take<double>(4);
    s.table = cv.take<double>(2 * LRQO_MAX_K);
    s.gain = refine ? cv.take<double>(n) : nullptr;
    s.target = refine ? cv.take<uint8_t>(n) : nullptr;
    s.zb = refine ? cv.take<uint8_t>(n) : nullptr;
    s.moves = refine ? cv.take<unsigned long long>(kMaxCheck * kMoveLanes) : nullptr;
    Carve hv(ctx->host);
    h.out = hv.take<double>(4);
    h.flag = hv.take<int>(16);
    h.moves = hv.take<unsigned long long>(kMaxCheck * kMoveLanes);
    h.table = hv.take<double>(2 * LRQO_MAX_K);
    return LRQO_OK;
}

lrqo_status upload_tables(int K, const GraphScratch& s, double* h_tab, hipStream_t st) {
    for (int d = 0; d < K; ++d) {
        const double a = 6.283185307179586476925286766559 * (double)d / (double)K;
        const double c = std::cos(a), sn = std::sin(a);
        // |1 - omega^d|^2 = (1 - cos)^2 + sin^2
        h_tab[d] = (1.0 - c) * (1.0 - c) + sn * sn;
        h_tab[LRQO_MAX_K + d] = c;
    }
    if (K == 2 || K == 3 || K == 4) {
        // these values are the integers 0..4 and cos in {1, 0, -1/2, -1}
        for (int d = 0; d < K; ++d) {
            h_tab[d] = std::round(h_tab[d]);
            h_tab[LRQO_MAX_K + d] = std::round(2.0 * h_tab[LRQO_MAX_K + d]) / 2.0;
        }
    }
    LRQO_HIP(hipMemcpyAsync(s.table, h_tab, sizeof(double) * 2 * LRQO_MAX_K, hipMemcpyHostToDevice, st));
    return LRQO_OK;
}

lrqo_status objective(const GraphDev& gd, int K, const uint8_t* z, const GraphScratch& s, double* h_out,
                      hipStream_t st, double* quad, double* cut) {
    const int64_t blocks = (gd.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_objective, dim3((unsigned)blocks), dim3(kBlock), 0, st, gd, K, z, s.table, s.partial);
    LRQO_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum2, dim3(1), dim3(kBlock), 0, st, s.partial, blocks, s.out2);
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipMemcpyAsync(h_out, s.out2, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipStreamSynchronize(st));
    // every edge was seen from both of its ends
    *quad = 0.5 * h_out[0];
    *cut = 0.5 * h_out[1];
    return LRQO_OK;
}

}  // namespace

lrqo_status check_graph_args(const lrqo_graph* g) {
    if (!g) return fail(LRQO_EINVAL, "null graph");
    if (!g->row_ptr) return fail(LRQO_EINVAL, "null row_ptr");
    if (g->nnz > 0 && !g->col) return fail(LRQO_EINVAL, "null col with nnz > 0");
    if (g->n < 1 || g->n > 0x7fffffffLL) return fail(LRQO_EINVAL, "n must be in [1, 2^31 - 1]");
    if (g->nnz < 0) return fail(LRQO_EINVAL, "nnz must be >= 0");
    if (!is_device_pointer(g->row_ptr)) return fail(LRQO_EINVAL, "row_ptr is not device memory");
    if (g->nnz > 0 && !is_device_pointer(g->col)) return fail(LRQO_EINVAL, "col is not device memory");
    if (g->w && !is_device_pointer(g->w)) return fail(LRQO_EINVAL, "w is not device memory");
    return LRQO_OK;
}

lrqo_status validate_graph(const lrqo_graph* g, int K, const uint8_t* z, int* d_flag, int* h_flag,
                           hipStream_t st) {
    const GraphDev gd{g->row_ptr, g->col, g->w, g->n, g->nnz};
    const unsigned blocks = (unsigned)((gd.n + kBlock - 1) / kBlock);
    *h_flag = 0;
    LRQO_HIP(hipMemcpyAsync(d_flag, h_flag, sizeof(int), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_check_ptr, dim3(blocks), dim3(kBlock), 0, st, gd, d_flag);
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipMemcpyAsync(h_flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipStreamSynchronize(st));
    if (*h_flag) return fail(LRQO_EINVAL, "row_ptr is not a CSR row pointer (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz)");
    hipLaunchKernelGGL(k_check_rows, dim3(blocks), dim3(kBlock), 0, st, gd, K, z, d_flag);
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipMemcpyAsync(h_flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipStreamSynchronize(st));
    if (*h_flag & kBadCol) return fail(LRQO_EINVAL, "a column index is out of range or a self loop");
    if (*h_flag & kBadWeight) return fail(LRQO_EINVAL, "a weight is not finite");
    if (*h_flag & kBadLabel) return fail(LRQO_EINVAL, "a label is not below K");
    return LRQO_OK;
}

}  // namespace lrqo

extern "C" {

lrqo_status lrqo_graph_objective(const lrqo_graph* g, int32_t K, const uint8_t* z, double* quad,
                                 double* cut) {
    using namespace lrqo;
    clear_error();
    LRQO_TRY(check_graph_args(g));
    if (!z || !quad || !cut) return fail(LRQO_EINVAL, "null pointer argument");
    if (K < 2 || K > LRQO_MAX_K) return fail(LRQO_EINVAL, "K must be in [2, 255]");
    if (!is_device_pointer(z)) return fail(LRQO_EINVAL, "z is not device memory");
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const hipStream_t st = current_stream();
    GraphScratch s{};
    HostScratch h{};
    LRQO_TRY(reserve_graph(ctx, g->n, false, s, h));
    const GraphDev gd{g->row_ptr, g->col, g->w, g->n, g->nnz};
    LRQO_TRY(validate_graph(g, K, z, s.flag, h.flag, st));
    LRQO_TRY(upload_tables(K, s, h.table, st));
    return objective(gd, K, z, s, h.out, st, quad, cut);
}

lrqo_status lrqo_refine_greedy(const lrqo_graph* g, int32_t K, uint8_t* z, const lrqo_refine_options* opt,
                               lrqo_refine_result* res) {
    using namespace lrqo;
    clear_error();
    LRQO_TRY(check_graph_args(g));
    if (!z) return fail(LRQO_EINVAL, "null pointer argument");
    if (K < 2 || K > kMaxKRefine) return fail(LRQO_EINVAL, "K must be in [2, 16] for the local search");
    lrqo_refine_options o{};
    if (opt) o = *opt;
    if (o.max_rounds < 0) return fail(LRQO_EINVAL, "max_rounds must be >= 0");
    if (o.check_every < 0 || o.check_every > kMaxCheck) return fail(LRQO_EINVAL, "check_every must be in [0, 64]");
    const int64_t max_rounds = o.max_rounds ? o.max_rounds : 1000000;
    const int chunk = o.check_every ? o.check_every : 8;
    if (!is_device_pointer(z)) return fail(LRQO_EINVAL, "z is not device memory");
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const hipStream_t st = current_stream();
    GraphScratch s{};
    HostScratch h{};
    LRQO_TRY(reserve_graph(ctx, g->n, true, s, h));
    const GraphDev gd{g->row_ptr, g->col, g->w, g->n, g->nnz};
    LRQO_TRY(validate_graph(g, K, z, s.flag, h.flag, st));
    LRQO_TRY(upload_tables(K, s, h.table, st));

    lrqo_refine_result r{};
    LRQO_TRY(objective(gd, K, z, s, h.out, st, &r.quad_before, &r.cut_before));

    const unsigned blocks = (unsigned)((gd.n + kRefineBlock - 1) / kRefineBlock);
    const double* cosd = s.table + LRQO_MAX_K;
    uint8_t* zbuf[2] = {z, s.zb};
    int cur = 0;
    int64_t rounds = 0, moves = 0, launched = 0;
    bool converged = false;
    float total_ms = 0.0f;
    while (!converged && rounds < max_rounds) {
        const int todo = (int)std::min<int64_t>(chunk, max_rounds - rounds);
        LRQO_HIP(hipMemsetAsync(s.moves, 0, sizeof(unsigned long long) * todo * kMoveLanes, st));
        LRQO_HIP(hipEventRecord(ctx->ev_start, st));
        for (int t = 0; t < todo; ++t) {
            // the batch runs only after rounds that all moved something
            const unsigned long long* prev = t ? s.moves + (size_t)(t - 1) * kMoveLanes : nullptr;
            if (K <= 4)
                hipLaunchKernelGGL(k_gain<4>, dim3(blocks), dim3(kRefineBlock), 0, st, gd, K, zbuf[cur], cosd, s.gain,
                                   s.target, prev);
            else
                hipLaunchKernelGGL(k_gain<kMaxKRefine>, dim3(blocks), dim3(kRefineBlock), 0, st, gd, K, zbuf[cur], cosd,
                                   s.gain, s.target, prev);
            hipLaunchKernelGGL(k_move, dim3(blocks), dim3(kRefineBlock), 0, st, gd, zbuf[cur], s.gain, s.target,
                               zbuf[cur ^ 1], s.moves + (size_t)t * kMoveLanes, prev);
            cur ^= 1;
        }
        LRQO_HIP(hipGetLastError());
        LRQO_HIP(hipEventRecord(ctx->ev_stop, st));
        launched += todo;
        LRQO_HIP(hipMemcpyAsync(h.moves, s.moves, sizeof(unsigned long long) * todo * kMoveLanes,
                                hipMemcpyDeviceToHost, st));
        LRQO_HIP(hipStreamSynchronize(st));
        float ms = 0.0f;
        LRQO_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
        total_ms += ms;
        // a round without moves leaves the labels as they were, and so do all after it
        for (int t = 0; t < todo; ++t) {
            unsigned long long m = 0;
            for (int l = 0; l < kMoveLanes; ++l) m += h.moves[(size_t)t * kMoveLanes + l];
            if (m == 0) {
                converged = true;
                break;
            }
            ++rounds;
            moves += (int64_t)m;
        }
    }
    // round t reads labels from buffer t mod 2 and writes the other; rounds
    // after the first one without moves were skipped, so the result is in
    // buffer rounds mod 2 (the caller's z is buffer 0)
    if (rounds % 2 == 1) LRQO_HIP(hipMemcpyAsync(z, s.zb, (size_t)gd.n, hipMemcpyDeviceToDevice, st));
    LRQO_TRY(objective(gd, K, z, s, h.out, st, &r.quad_after, &r.cut_after));
    r.moves = moves;
    r.rounds = (int32_t)rounds;
    r.converged = converged ? 1 : 0;
    r.device_ms = total_ms;
    r.launched = (int32_t)launched;
    if (res) *res = r;
    return LRQO_OK;
}

}  // extern "C"
