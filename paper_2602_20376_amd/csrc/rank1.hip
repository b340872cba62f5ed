// Exact rank-1 maximisation by the phase sweep (Sec. 2.5, Alg. 1,
// Thm. rank1): max |z^H q|^2 over z in A_K^n.
//
// Every coordinate changes its label once as the auxiliary angle phi sweeps
// (-pi/K, pi/K]: at phi_i = (2 pi/K)(1/2 + floor(x_i) - x_i), x_i =
// K arg(q_i)/(2 pi).  Starting from k_i = floor(x_i) mod K (the assignment
// at phi = -pi/K), the n+1 cells of the sweep are the prefixes of the
// boundary points in sorted order, and s = sum_i conj(q_i) omega^k_i moves
// by d_i = conj(q_i)(omega^(k_i+1) - omega^k_i) at each of them, so the
// objective of cell l is |s_0 + d_(1) + ... + d_(l)|^2.
//
// Kernels:
//   k_r1_prep     per coordinate: phi (same FP64 expression as Alg. 1),
//                 its exact sortable key and 32-bit image, k_0, d, block
//                 partials of s_0 and of the OR / AND of the keys (digits
//                 that never change skip a pass of the exact-key sort),
//                 finiteness
//   k_r1_reduce0  s_0 and the OR / AND from the block partials
//   radix sort    stable (sort.hip), first by a 32-bit fixed-point image of
//                 phi (four passes; it never reverses the order of two
//                 points), so equal images keep coordinate order
//   k_r1_fixup    runs of equal images whose exact keys differ (rare: points
//                 closer than 2^-32 of the range) are put in (key,
//                 coordinate) order by insertion; a run longer than 16 with
//                 differing keys makes the host sort the exact 64-bit keys
//                 instead (eight passes), so the order is always that of
//                 (key, coordinate)
//   k_r1_tiles    per tile of 2048 sorted positions: gathers d into sorted
//                 order (coalesced write) and sums the tile
//   k_r1_tilepre  s_0 plus the tile sums before each tile (fixed order)
//   k_r1_cells    per tile: running s through its positions, |s|^2 per cell,
//                 best cell of the tile (ties to the earlier cell)
//   k_r1_pick     best cell over the tiles and cell 0, and the (key,
//                 coordinate) pair of its last boundary point
//   k_r1_labels   labels of the best cell, in coordinate order: k_0 advanced
//                 by one where (key, coordinate) is at or below that pair,
//                 which is where the stable sort put the coordinate at or
//                 before the cell; block partials of z^H q
// All sums run in a fixed order (shuffle trees and block scans of fixed
// shape), so a run is reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lrqo_device.h"
#include "lrqo_runtime.h"
#include "sort.h"

namespace lrqo {

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;                  // sorted positions per thread in the cell scan
constexpr int kTile = kBlock * kItems;     // 2048
constexpr double kPi = 3.141592653589793238462643383279502884;

__device__ __forceinline__ unsigned long long order_key(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// A 32-bit image of phi in (-pi/K, pi/K] that never reverses the order of
// two values: (phi K/(2 pi) + 1/2) 2^32, truncated and clamped; every step
// is non-decreasing in phi.
__device__ __forceinline__ uint32_t fixed_key(double phi, int K) {
    double u = fma(phi, (double)K / (2.0 * kPi), 0.5) * 4294967296.0;
    u = u > 0.0 ? u : 0.0;   // also maps a NaN to 0 (reported separately)
    return u >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)u;
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// conj(q) * w
__device__ __forceinline__ double2 cconj_mul(double2 q, double2 w) {
    return make_double2(q.x * w.x + q.y * w.y, q.x * w.y - q.y * w.x);
}

__device__ __forceinline__ double2 shfl_xor_c(double2 v, int m) {
    return make_double2(__shfl_xor(v.x, m, kWave), __shfl_xor(v.y, m, kWave));
}

__device__ __forceinline__ double2 shfl_up_c(double2 v, int off) {
    return make_double2(__shfl_up(v.x, off, kWave), __shfl_up(v.y, off, kWave));
}

// Fixed-order block sum of a complex value per thread: a shuffle tree in
// each wave, then the waves' sums in wave order.  Every thread gets it.
__device__ __forceinline__ double2 block_sum_c(double2 v) {
    __shared__ double2 ws[kBlock / kWave];
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) v = cadd(v, shfl_xor_c(v, m));
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = v;
    __syncthreads();
    double2 r = ws[0];
    for (int w = 1; w < kBlock / kWave; ++w) r = cadd(r, ws[w]);
    __syncthreads();
    return r;
}

// init + the sum of the values of the threads before this one (fixed
// order: a shuffle scan in each wave, the lower waves' totals before it).
__device__ __forceinline__ double2 block_excl_scan_c(double2 v, double2 init) {
    __shared__ double2 ws[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double2 incl = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const double2 y = shfl_up_c(incl, off);
        if (lane >= off) incl = cadd(y, incl);
    }
    if (lane == kWave - 1) ws[w] = incl;
    const double2 below = shfl_up_c(incl, 1);
    __syncthreads();
    double2 r = init;
    for (int u = 0; u < w; ++u) r = cadd(r, ws[u]);
    if (lane > 0) r = cadd(r, below);
    __syncthreads();
    return r;
}

struct R1Dev {
    const double2* q;
    int64_t n;
    int K;
    const double2* roots;            // [K]
    unsigned long long* keys;        // exact order keys of phi
    uint32_t* k32;                   // fixed-point images of phi
    uint8_t* k0;
    double2* d;
    double2* part;                   // block partials
    unsigned long long* orand_part;  // [2 * blocks]: OR, AND of the keys per block
    int* flag;
};

__global__ __launch_bounds__(kBlock) void k_r1_prep(R1Dev p) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    double2 c0 = make_double2(0.0, 0.0);
    unsigned long long key = 0;
    bool live = i < p.n;
    if (live) {
        const double2 q = p.q[i];
        if (!isfinite(q.x) || !isfinite(q.y)) atomicOr(p.flag, 1);
        // the expressions of Alg. 1, rounded step by step as written
        const double theta = atan2(q.y, q.x);
        const double x = __ddiv_rn(__dmul_rn((double)p.K, theta), 2.0 * kPi);
        const double fl = floor(x);
        const double phi = __dmul_rn(__ddiv_rn(2.0 * kPi, (double)p.K), __dsub_rn(__dadd_rn(0.5, fl), x));
        int k = (int)fmod(fl, (double)p.K);
        k += k < 0 ? p.K : 0;
        key = order_key(phi);
        p.keys[i] = key;
        p.k32[i] = fixed_key(phi, p.K);
        p.k0[i] = (uint8_t)k;
        const int k1 = k + 1 == p.K ? 0 : k + 1;
        const double2 a = p.roots[k], b = p.roots[k1];
        p.d[i] = cconj_mul(q, make_double2(b.x - a.x, b.y - a.y));
        c0 = cconj_mul(q, a);
    }
    unsigned long long wor = live ? key : 0ull, wand = live ? key : ~0ull;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        wor |= __shfl_xor(wor, off, kWave);
        wand &= __shfl_xor(wand, off, kWave);
    }
    __shared__ unsigned long long wo[kBlock / kWave], wa[kBlock / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) {
        wo[threadIdx.x / kWave] = wor;
        wa[threadIdx.x / kWave] = wand;
    }
    const double2 s = block_sum_c(c0);   // synchronises the block
    if (threadIdx.x == 0) {
        p.part[blockIdx.x] = s;
        unsigned long long o = 0ull, a = ~0ull;
        for (int w = 0; w < kBlock / kWave; ++w) {
            o |= wo[w];
            a &= wa[w];
        }
        p.orand_part[2 * blockIdx.x] = o;
        p.orand_part[2 * blockIdx.x + 1] = a;
    }
}

// Fixed-order sum of `count` complex partials into out[0] (one block).
__global__ __launch_bounds__(kBlock) void k_r1_sum(const double2* __restrict__ part, int64_t count,
                                                   double2* __restrict__ out) {
    double2 a = make_double2(0.0, 0.0);
    for (int64_t t = threadIdx.x; t < count; t += kBlock) a = cadd(a, part[t]);
    const double2 s = block_sum_c(a);
    if (threadIdx.x == 0) out[0] = s;
}

// s_0 from the prep's block partials, and the OR / AND of its key partials
// (one block).
__global__ __launch_bounds__(kBlock) void k_r1_reduce0(const double2* __restrict__ part,
                                                       const unsigned long long* __restrict__ orand_part,
                                                       int64_t blocks, double2* __restrict__ s0,
                                                       unsigned long long* __restrict__ orand) {
    double2 a = make_double2(0.0, 0.0);
    unsigned long long o = 0ull, m = ~0ull;
    for (int64_t t = threadIdx.x; t < blocks; t += kBlock) {
        a = cadd(a, part[t]);
        o |= orand_part[2 * t];
        m &= orand_part[2 * t + 1];
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        o |= __shfl_xor(o, off, kWave);
        m &= __shfl_xor(m, off, kWave);
    }
    __shared__ unsigned long long wo[kBlock / kWave], wa[kBlock / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) {
        wo[threadIdx.x / kWave] = o;
        wa[threadIdx.x / kWave] = m;
    }
    const double2 s = block_sum_c(a);   // synchronises the block
    if (threadIdx.x == 0) {
        s0[0] = s;
        for (int w = 1; w < kBlock / kWave; ++w) {
            o |= wo[w];
            m &= wa[w];
        }
        orand[0] = o;
        orand[1] = m;
    }
}

// Tile b holds sorted positions b*kTile .. b*kTile + kTile-1; here thread t
// takes positions b*kTile + e*kBlock + t (coalesced), gathers their d into
// d_sorted and sums them.
__global__ __launch_bounds__(kBlock) void k_r1_tiles(const double2* __restrict__ d, const uint32_t* __restrict__ order,
                                                     int64_t n, double2* __restrict__ d_sorted,
                                                     double2* __restrict__ tile_sum) {
    const int64_t b0 = blockIdx.x * (int64_t)kTile + threadIdx.x;
    uint32_t idx[kItems];
#pragma unroll
    for (int e = 0; e < kItems; ++e) {
        const int64_t p = b0 + (int64_t)e * kBlock;
        idx[e] = p < n ? order[p] : 0u;
    }
    double2 v[kItems];
#pragma unroll
    for (int e = 0; e < kItems; ++e) {
        const int64_t p = b0 + (int64_t)e * kBlock;
        v[e] = p < n ? d[idx[e]] : make_double2(0.0, 0.0);
    }
    double2 a = make_double2(0.0, 0.0);
#pragma unroll
    for (int e = 0; e < kItems; ++e) {
        const int64_t p = b0 + (int64_t)e * kBlock;
        if (p < n) d_sorted[p] = v[e];
        a = cadd(a, v[e]);
    }
    const double2 s = block_sum_c(a);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = s;
}

// tile_pre[b] = s_0 + sum of tile_sum[0..b-1] (one block): each thread sums
// a contiguous run of tiles, a block scan offsets the runs, and each thread
// then walks its run.
__global__ __launch_bounds__(kBlock) void k_r1_tilepre(const double2* __restrict__ tile_sum, int64_t tiles,
                                                       const double2* __restrict__ s0,
                                                       double2* __restrict__ tile_pre) {
    const int64_t per = (tiles + kBlock - 1) / kBlock;
    const int64_t lo = min(tiles, (int64_t)threadIdx.x * per), hi = min(tiles, lo + per);
    double2 a = make_double2(0.0, 0.0);
    for (int64_t t = lo; t < hi; ++t) a = cadd(a, tile_sum[t]);
    double2 run = block_excl_scan_c(a, s0[0]);
    for (int64_t t = lo; t < hi; ++t) {
        tile_pre[t] = run;
        run = cadd(run, tile_sum[t]);
    }
}

constexpr int kRunMax = 16;   // longest run of equal images sorted in place

// After the stable sort by image, position p starts a run of equal images
// or sits inside one.  A run start with a run of at most kRunMax puts it in
// (key, coordinate) order by insertion (a run of equal keys is already in
// coordinate order and costs one comparison per member).  An inside
// position whose key differs from its predecessor's, in a run longer than
// kRunMax, sets *overflow; such runs are never touched here.
__global__ __launch_bounds__(kBlock) void k_r1_fixup(const uint32_t* __restrict__ img, uint32_t* __restrict__ order,
                                                     const unsigned long long* __restrict__ keys, int64_t n,
                                                     int* __restrict__ overflow) {
    const int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (p >= n) return;
    const uint32_t q = img[p];
    const bool start = p == 0 || img[p - 1] != q;
    if (start) {
        if (p + 1 >= n || img[p + 1] != q) return;
        int64_t e = p + 1;
        while (e < n && img[e] == q && e - p <= kRunMax) ++e;
        if (e - p > kRunMax) return;     // long run: checked by its members
        for (int64_t a = p + 1; a < e; ++a) {
            const uint32_t v = order[a];
            const unsigned long long kv = keys[v];
            int64_t b = a;
            while (b > p) {
                const uint32_t u = order[b - 1];
                const unsigned long long ku = keys[u];
                if (ku < kv || (ku == kv && u < v)) break;
                order[b] = u;
                --b;
            }
            order[b] = v;
        }
        return;
    }
    // inside a run; order[] of a run of at most kRunMax may be changing
    // under this read, but then the length test below ends it
    if (keys[order[p]] == keys[order[p - 1]]) return;
    int64_t lo = p, hi = p + 1;
    while (lo > 0 && img[lo - 1] == q && hi - lo <= kRunMax) --lo;
    while (hi < n && img[hi] == q && hi - lo <= kRunMax) ++hi;
    if (hi - lo > kRunMax) *overflow = 1;   // every writer stores the same value
}

struct Best {
    double f;
    int64_t cell;
    unsigned long long key;   // key of the cell's last boundary point (cell >= 1)
    uint32_t coord;           // and its coordinate
    int32_t pad;
};

__device__ __forceinline__ bool better(double f, int64_t c, double g, int64_t e) {
    return f > g || (f == g && c < e);
}

__device__ __forceinline__ int64_t shfl_xor_i64(int64_t v, int m) {
    const int lo = __shfl_xor((int)(uint32_t)v, m, kWave);
    const int hi = __shfl_xor((int)(v >> 32), m, kWave);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Best (value, cell) over the block, ties to the lower cell; thread 0 gets it.
__device__ __forceinline__ void block_best(double& f, int64_t& c) {
    __shared__ double wf[kBlock / kWave];
    __shared__ int64_t wc[kBlock / kWave];
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) {
        const double g = __shfl_xor(f, m, kWave);
        const int64_t e = shfl_xor_i64(c, m);
        if (better(g, e, f, c)) {
            f = g;
            c = e;
        }
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        wf[threadIdx.x / kWave] = f;
        wc[threadIdx.x / kWave] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < kBlock / kWave; ++w)
            if (better(wf[w], wc[w], f, c)) {
                f = wf[w];
                c = wc[w];
            }
}

// Thread t of tile b owns sorted positions b*kTile + t*kItems .. + kItems-1.
__global__ __launch_bounds__(kBlock) void k_r1_cells(const double2* __restrict__ d_sorted, int64_t n,
                                                     const double2* __restrict__ tile_pre,
                                                     Best* __restrict__ tile_best) {
    const int64_t p0 = blockIdx.x * (int64_t)kTile + (int64_t)threadIdx.x * kItems;
    double2 dv[kItems];
    double2 a = make_double2(0.0, 0.0);
#pragma unroll
    for (int e = 0; e < kItems; ++e) {
        dv[e] = p0 + e < n ? d_sorted[p0 + e] : make_double2(0.0, 0.0);
        a = cadd(a, dv[e]);
    }
    double2 s = block_excl_scan_c(a, tile_pre[blockIdx.x]);
    double best = -1.0;
    int64_t cell = INT64_MAX;
    for (int e = 0; e < kItems; ++e) {
        if (p0 + e >= n) break;
        s = cadd(s, dv[e]);
        const double f = s.x * s.x + s.y * s.y;
        if (f > best) {          // strict: ties keep the earlier cell
            best = f;
            cell = p0 + e + 1;   // cell l follows the l-th boundary point
        }
    }
    block_best(best, cell);
    if (threadIdx.x == 0) tile_best[blockIdx.x] = Best{best, cell, 0ull, 0u, 0};
}

__global__ __launch_bounds__(kBlock) void k_r1_pick(const Best* __restrict__ tile_best, int64_t tiles,
                                                    const double2* __restrict__ s0,
                                                    const unsigned long long* __restrict__ keys,
                                                    const uint32_t* __restrict__ order, Best* __restrict__ out) {
    double best = -1.0;
    int64_t cell = INT64_MAX;
    if (threadIdx.x == 0) {
        best = s0[0].x * s0[0].x + s0[0].y * s0[0].y;
        cell = 0;
    }
    for (int64_t t = threadIdx.x; t < tiles; t += kBlock)
        if (better(tile_best[t].f, tile_best[t].cell, best, cell)) {
            best = tile_best[t].f;
            cell = tile_best[t].cell;
        }
    block_best(best, cell);
    if (threadIdx.x == 0) {
        Best b{best, cell, 0ull, 0u, 0};
        if (cell >= 1) {
            b.coord = order[cell - 1];
            b.key = keys[b.coord];
        }
        out[0] = b;
    }
}

// Coordinate i moves to k_0 + 1 when its boundary point sits at a sorted
// position below the best cell; the sort is stable, so that is when
// (key_i, i) <= (key, coordinate) of the cell's last point.  Also the block
// partials of z^H q.
__global__ __launch_bounds__(kBlock) void k_r1_labels(const unsigned long long* __restrict__ keys,
                                                      const uint8_t* __restrict__ k0, const double2* __restrict__ q,
                                                      const double2* __restrict__ roots, int64_t n, int K,
                                                      const Best* __restrict__ best, uint8_t* __restrict__ z,
                                                      double2* __restrict__ part) {
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    double2 v = make_double2(0.0, 0.0);
    if (i < n) {
        const Best b = best[0];
        const unsigned long long key = keys[i];
        const bool adv = b.cell >= 1 && (key < b.key || (key == b.key && (uint32_t)i <= b.coord));
        int k = k0[i] + (adv ? 1 : 0);
        k = k == K ? 0 : k;
        z[i] = (uint8_t)k;
        v = cconj_mul(q[i], roots[k]);
    }
    const double2 s = block_sum_c(v);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace
}  // namespace lrqo

extern "C" {

lrqo_status lrqo_solve_rank1(const double* q, int64_t n, int32_t K, uint8_t* z, lrqo_rank1_result* res) {
    using namespace lrqo;
    clear_error();
    if (!q || !z) return fail(LRQO_EINVAL, "null pointer argument");
    if (n < 1 || n > 0x7fffffffLL) return fail(LRQO_EINVAL, "n must be in [1, 2^31 - 1]");
    if (K < 2 || K > LRQO_MAX_K) return fail(LRQO_EINVAL, "K must be in [2, 255]");
    if (!is_device_pointer(q)) return fail(LRQO_EINVAL, "q is not device memory");
    if (!is_device_pointer(z)) return fail(LRQO_EINVAL, "z is not device memory");
    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    const hipStream_t st = current_stream();

    const int64_t blocks = (n + kBlock - 1) / kBlock;
    const int64_t tiles = (n + kTile - 1) / kTile;
    CarveSize cs;
    cs.add<unsigned long long>(n);
    cs.add<uint32_t>(n);
    cs.add<unsigned long long>(n);
    cs.add<uint32_t>(n);
    cs.add<unsigned long long>(n);
    cs.add<uint32_t>(n);
    cs.add<uint32_t>(radix_hist_entries(n));
    cs.add<uint8_t>(n);
    cs.add<double2>(n);
    cs.add<double2>(n);
    cs.add<double2>(blocks);
    cs.add<double2>(tiles);
    cs.add<double2>(tiles);
    cs.add<Best>(tiles);
    cs.add<Best>(1);
    cs.add<double2>(4);
    cs.add<double2>(LRQO_MAX_K);
    cs.add<unsigned long long>(2);
    cs.add<unsigned long long>(2 * blocks);
    cs.add<int>(4);
    CarveSize hs;
    hs.add<double2>(LRQO_MAX_K);
    hs.add<unsigned long long>(2);
    hs.add<int>(4);
    hs.add<double2>(1);
    hs.add<Best>(1);
    LRQO_TRY(reserve_arena(ctx, cs.bytes));
    LRQO_TRY(reserve_host(ctx, hs.bytes));
    Carve cv(ctx->arena);
    unsigned long long* keys = cv.take<unsigned long long>(n);
    uint32_t* k32 = cv.take<uint32_t>(n);
    unsigned long long* keys_a = cv.take<unsigned long long>(n);
    uint32_t* vals_a = cv.take<uint32_t>(n);
    unsigned long long* keys_b = cv.take<unsigned long long>(n);
    uint32_t* vals_b = cv.take<uint32_t>(n);
    uint32_t* hist = cv.take<uint32_t>(radix_hist_entries(n));
    uint8_t* k0 = cv.take<uint8_t>(n);
    double2* d = cv.take<double2>(n);
    double2* d_sorted = cv.take<double2>(n);
    double2* part = cv.take<double2>(blocks);
    double2* tile_sum = cv.take<double2>(tiles);
    double2* tile_pre = cv.take<double2>(tiles);
    Best* tile_best = cv.take<Best>(tiles);
    Best* best = cv.take<Best>(1);
    double2* s0 = cv.take<double2>(4);
    double2* roots = cv.take<double2>(LRQO_MAX_K);
    unsigned long long* orand = cv.take<unsigned long long>(2);
    unsigned long long* orand_part = cv.take<unsigned long long>(2 * blocks);
    int* flag = cv.take<int>(4);
    Carve hv(ctx->host);
    double2* h_roots = hv.take<double2>(LRQO_MAX_K);
    unsigned long long* h_orand = hv.take<unsigned long long>(2);
    int* h_flag = hv.take<int>(4);
    double2* h_s = hv.take<double2>(1);
    Best* h_best = hv.take<Best>(1);

    // roots omega^k = exp(2 pi i k / K), argument (2 pi k)/K
    for (int k = 0; k < K; ++k) {
        const double a = (2.0 * kPi * (double)k) / (double)K;
        h_roots[k] = make_double2(std::cos(a), std::sin(a));
    }
    h_flag[0] = 0;   // non-finite q
    h_flag[1] = 0;   // a long run with differing keys
    LRQO_HIP(hipEventRecord(ctx->ev_start, st));
    LRQO_HIP(hipMemcpyAsync(roots, h_roots, sizeof(double2) * K, hipMemcpyHostToDevice, st));
    LRQO_HIP(hipMemcpyAsync(flag, h_flag, 2 * sizeof(int), hipMemcpyHostToDevice, st));
    R1Dev p{reinterpret_cast<const double2*>(q), n, K, roots, keys, k32, k0, d, part, orand_part, flag};
    hipLaunchKernelGGL(k_r1_prep, dim3((unsigned)blocks), dim3(kBlock), 0, st, p);
    hipLaunchKernelGGL(k_r1_reduce0, dim3(1), dim3(kBlock), 0, st, part, orand_part, blocks, s0, orand);
    LRQO_HIP(hipGetLastError());
    // images first (the 64-bit work buffers hold the 32-bit pairs)
    SortedPairs32 by_img{};
    LRQO_TRY(radix_sort_pairs32(k32, reinterpret_cast<uint32_t*>(keys_a), vals_a, reinterpret_cast<uint32_t*>(keys_b),
                                vals_b, hist, n, 0xFu, st, &by_img));
    uint32_t* order_img = const_cast<uint32_t*>(by_img.vals);   // a work buffer of this call
    hipLaunchKernelGGL(k_r1_fixup, dim3((unsigned)blocks), dim3(kBlock), 0, st, by_img.keys, order_img, keys, n,
                       flag + 1);
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipMemcpyAsync(h_orand, orand, sizeof(unsigned long long) * 2, hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipMemcpyAsync(h_flag, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipStreamSynchronize(st));
    if (h_flag[0]) return fail(LRQO_ENOTFINITE, "q holds a NaN or an infinity");

    int passes = 4;
    const uint32_t* order = order_img;
    if (h_flag[1]) {
        // the exact keys, skipping digits that are the same in all of them
        unsigned mask = 0;
        const unsigned long long varying = h_orand[0] ^ h_orand[1];
        for (int dgt = 0; dgt < 8; ++dgt)
            if ((varying >> (8 * dgt)) & 0xFFull) mask |= 1u << dgt;
        if (!mask) mask = 1u;   // the sort runs one pass at least
        SortedPairs exact{};
        LRQO_TRY(radix_sort_pairs(keys, keys_a, vals_a, keys_b, vals_b, hist, n, mask, st, &exact));
        order = exact.vals;
        passes += __builtin_popcount(mask);
    }

    hipLaunchKernelGGL(k_r1_tiles, dim3((unsigned)tiles), dim3(kBlock), 0, st, d, order, n, d_sorted, tile_sum);
    hipLaunchKernelGGL(k_r1_tilepre, dim3(1), dim3(kBlock), 0, st, tile_sum, tiles, s0, tile_pre);
    hipLaunchKernelGGL(k_r1_cells, dim3((unsigned)tiles), dim3(kBlock), 0, st, d_sorted, n, tile_pre, tile_best);
    hipLaunchKernelGGL(k_r1_pick, dim3(1), dim3(kBlock), 0, st, tile_best, tiles, s0, keys, order, best);
    hipLaunchKernelGGL(k_r1_labels, dim3((unsigned)blocks), dim3(kBlock), 0, st, keys, k0, p.q, roots, n, K, best,
                       z, part);
    hipLaunchKernelGGL(k_r1_sum, dim3(1), dim3(kBlock), 0, st, part, blocks, s0 + 1);
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipEventRecord(ctx->ev_stop, st));
    LRQO_HIP(hipMemcpyAsync(h_s, s0 + 1, sizeof(double2), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipMemcpyAsync(h_best, best, sizeof(Best), hipMemcpyDeviceToHost, st));
    LRQO_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    LRQO_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
    if (res) {
        std::memset(res, 0, sizeof *res);
        res->obj = h_s[0].x * h_s[0].x + h_s[0].y * h_s[0].y;
        res->sweep_obj = h_best[0].f;
        res->best_cell = h_best[0].cell;
        res->device_ms = ms;
        res->sort_passes = passes;
    }
    return LRQO_OK;
}

}  // extern "C"
