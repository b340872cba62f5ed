// Batched sampled maximisation: thousands of small instances of uneven size
// in one persistent, work-queue-driven launch.
//
// Instance t is the problem of Sec. 4.2 on its own factor V_t (n_t x r_t),
// drawn from the direction stream (seed, instance word t), so its result is
// the result of a single solve with instance = t.
//
// Kernels (one sequence, captured once into a hipGraph and replayed):
//   k_bfill          zeroes the work cursor (a kernel, not a memset node)
//   k_batch_score    persistent grid; each block pops (instance, tile) items
//                    from a queue sorted by decreasing cost with an atomic
//                    cursor, stages V_t in LDS, scores its tile of
//                    directions (FP32, CPL per lane) and writes FP32 scores
//   k_batch_select   per instance: best T packed (score, index) keys, FP64
//                    rescore of the T kept directions, arg-max (ties to the
//                    lower index), FP64 labels of the winner into the
//                    library's label buffer, copied to the caller's array
//                    after the replay
// Launch shape (directions per lane, persistent blocks per CU) comes from a
// small autotuner that times the candidates on the device once per batch
// signature and keeps the choice in a JSON cache file.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "lrqo_device.h"
#include "lrqo_runtime.h"

namespace lrqo {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxRows = 256;       // rows of one instance staged in LDS
constexpr int kMaxS = 4096;         // directions per instance
constexpr int kTopT = 64;

struct BatchDevParams {
    const float* V;                 // concatenated factors
    const int64_t* voff;            // [count] float offset of V_t
    const int32_t* n;               // [count]
    const int32_t* r;               // [count]
    const int64_t* zoff;            // [count] label offset of instance t
    const int32_t* items;           // [nitems] packed (instance << 8 | tile)
    int32_t nitems;
    int32_t count;
    int32_t K;
    int32_t S;
    uint64_t seed;
    int32_t real;
    int32_t tile;                   // directions per item
    unsigned int* cursor;
    float* f;                       // [count][S]
    double* obj;                    // [count]
    int64_t* best;                  // [count]
    uint8_t* z;
    const float2* roots32;
    const double2* roots64;
    int32_t T;
};

__global__ void k_bfill(unsigned int* cursor) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *cursor = 0u;
}

// Score one tile of directions of instance t against its LDS-staged rows.
template <int R, int CPL, int KS>
__device__ void score_item(const BatchDevParams& p, int t, int tile, const float* Vs, int n,
                           const float2* roots) {
    float c[CPL][2 * R], c3[CPL][2 * R], acc[CPL][2 * R];
    const int base = tile * p.tile + threadIdx.x;
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int s = base + q * kBlock;
        if (s < p.S) direction_f32<R>(p.seed, (uint64_t)s, (uint32_t)t, c[q]);
        else {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) c[q][j] = 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) {
            acc[q][j] = 0.0f;
            c3[q][j] = re_prescale(KS) * c[q][j];   // K = 3: Re w pre-scaled
        }
        if constexpr (KS == 8 || KS == 16) {        // the direction turned by e^{-i pi/K}
#pragma unroll
            for (int j = 0; j < R; ++j) {
                turn_direction<KS>(c[q][2 * j], c[q][2 * j + 1]);
                c3[q][2 * j] = c[q][2 * j];
                c3[q][2 * j + 1] = c[q][2 * j + 1];
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        float v[2 * R];
#pragma unroll
        for (int e = 0; e < 2 * R; ++e) v[e] = Vs[i * 2 * R + e];
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            float wr = 0.0f, wi = 0.0f;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const float vr = v[2 * j], vi = v[2 * j + 1];
                wr = fmaf(vr, c3[q][2 * j], fmaf(-vi, c3[q][2 * j + 1], wr));
                wi = fmaf(vr, c[q][2 * j + 1], fmaf(vi, c[q][2 * j], wi));
            }
            float zr, zi;
            if constexpr (KS == 3) {
                const bool k0 = fabsf(wi) <= wr;            // |Im w| <= sqrt(3) Re w
                zr = k0 ? 1.0f : -0.5f;
                zi = k0 ? 0.0f : copysignf(0.8660254037844386f, wi);
            } else if constexpr (KS == 8) {
                bisector_k8(wr, wi, zr, zi);        // turned root; ||s||^2 is unchanged
            } else if constexpr (KS == 16) {
                bisector_k16(wr, wi, zr, zi);
            } else {
                nearest_root<KS>(wr, wi, p.K, roots, zr, zi);
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const float vr = v[2 * j], vi = v[2 * j + 1];
                acc[q][2 * j] = fmaf(vr, zr, fmaf(vi, zi, acc[q][2 * j]));
                acc[q][2 * j + 1] = fmaf(vr, zi, fmaf(-vi, zr, acc[q][2 * j + 1]));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int s = base + q * kBlock;
        if (s < p.S) {
            float f = 0.0f;
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) f = fmaf(acc[q][j], acc[q][j], f);
            p.f[(size_t)t * p.S + s] = f;
        }
    }
}

// Persistent scorer.  Every block loops until the shared cursor passes the
// last item, so every wave reaches the exit.  Real factors are staged as
// complex rows with zero imaginary parts.
template <int CPL, int KS>
__global__ __launch_bounds__(kBlock) void k_batch_score(BatchDevParams p) {
    __shared__ __align__(16) float Vs[kMaxRows * 8];
    __shared__ float2 roots_s[LRQO_MAX_K];
    __shared__ int item_s;
    for (int k = threadIdx.x; k < p.K; k += kBlock) roots_s[k] = p.roots32[k];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) item_s = (int)atomicAdd(p.cursor, 1u);
        __syncthreads();
        const int it = item_s;
        if (it >= p.nitems) break;
        const int packed = p.items[it];
        const int t = packed >> 8, tile = packed & 0xFF;
        const int n = p.n[t], r = p.r[t];
        const float* src = p.V + p.voff[t];
        // stage V_t as complex rows (2r floats each)
        for (int e = threadIdx.x; e < n * 2 * r; e += kBlock) {
            float x;
            if (p.real) {
                const int row = e / (2 * r), j2 = e % (2 * r);
                x = (j2 & 1) ? 0.0f : src[row * r + (j2 >> 1)];
            } else {
                x = src[e];
            }
            Vs[e] = x;
        }
        __syncthreads();
        switch (r) {
            case 1: score_item<1, CPL, KS>(p, t, tile, Vs, n, roots_s); break;
            case 2: score_item<2, CPL, KS>(p, t, tile, Vs, n, roots_s); break;
            case 3: score_item<3, CPL, KS>(p, t, tile, Vs, n, roots_s); break;
            case 4: score_item<4, CPL, KS>(p, t, tile, Vs, n, roots_s); break;
            default: break;
        }
    }
}

// Per instance (one block of four waves):
//   select   best T of its S FP32 scores as packed keys.  Threshold pass:
//            every lane takes the largest key of its scores, and tau = the
//            64th largest of the block's 256 lane maxima (64 distinct keys are
//            >= tau, so the best 64 all are); the keys >= tau (about 75 of
//            4,096 for scattered scores) are gathered in LDS and wave 0 keeps
//            the best 64 of them.  If more than kStage keys pass, each wave
//            instead keeps a 64-key list over a quarter of the scores and
//            wave 0 merges the four.
//   rescore  FP64 objective of each kept direction from V_t staged in LDS;
//            wave w takes rows w, w+4, ..., and the four partial sums are
//            added in wave order
//   pick     FP64 arg-max over the kept directions, ties to the lower index
//   labels   FP64 decision rule of the winner for every row
constexpr int kStage = 512;          // keys the threshold pass may keep

template <int KS>
struct SelectShared {
    float Vs[kMaxRows * 8];         // V_t as stored (real: n x r, complex: n x 2r floats)
    unsigned long long top[kBlock / 64][64];
    unsigned long long stage[kStage];
    unsigned long long tau;
    unsigned int cnt;
    double part[kBlock / 64][kTopT][8];
    double2 roots[KS == 0 ? LRQO_MAX_K : 1];   // the generic quantiser's table only (31 KB in all otherwise:
                                               // five blocks per CU)
    double cbest[8];
};

template <int R, int KS>
__device__ void select_rescore(const BatchDevParams& p, int t, SelectShared<KS>& sh) {
    constexpr int NW = kBlock / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int S = p.S, T = p.T, n = p.n[t];
    const float* f = p.f + (size_t)t * S;
    const float* V = sh.Vs;         // staged by the caller before the selection

    // ---- select
    const int per = (S + NW * 64 - 1) / (NW * 64) * 64;
    const int lo = w * per, hi = min(S, lo + per);
    // threshold: the 64th largest of the lane maxima
    unsigned long long lmax = 0;
    for (int s = lo + lane; s < hi; s += 64) lmax = key_max(lmax, pack_key(f[s], (uint32_t)s));
    sh.top[w][lane] = wave_sort_desc(lmax, lane);
    __syncthreads();
    if (w == 0) {
        unsigned long long u = sh.top[0][lane];
        for (int v = 1; v < NW; ++v) u = wave_top_union(u, sh.top[v][lane], lane);
        const unsigned long long tau = __shfl(u, 63, 64);
        if (lane == 0) sh.tau = tau;
    }
    __syncthreads();
    const unsigned long long tau = sh.tau;
    for (int s = lo + lane; s < hi; s += 64) {
        const unsigned long long key = pack_key(f[s], (uint32_t)s);
        if (key >= tau) {
            const unsigned int pos = atomicAdd(&sh.cnt, 1u);
            if (pos < (unsigned)kStage) sh.stage[pos] = key;
        }
    }
    __syncthreads();
    const unsigned int cnt = sh.cnt;
    unsigned long long run = 0;
    if (cnt <= (unsigned)kStage) {
        if (w == 0) {
            for (unsigned int b = 0; b < cnt; b += 64) {
                const unsigned long long key = b + lane < cnt ? sh.stage[b + lane] : 0ull;
                run = wave_top_union(run, wave_sort_desc(key, lane), lane);
            }
            sh.top[0][lane] = run;
        }
    } else {
        for (int b = lo; b < hi; b += 64) {
            const int s = b + lane;
            const unsigned long long key = s < hi ? pack_key(f[s], (uint32_t)s) : 0ull;
            const unsigned long long floor64 = __shfl(run, 63, 64);
            if (__ballot(key > floor64) == 0) continue;  // uniform across the wave
            run = wave_top_union(run, wave_sort_desc(key, lane), lane);
        }
        __syncthreads();        // every wave has read sh.top (threshold pass)
        sh.top[w][lane] = run;
        __syncthreads();
        if (w == 0) {
            for (int v = 1; v < NW; ++v) run = wave_top_union(run, sh.top[v][lane], lane);
            sh.top[0][lane] = run;
        }
    }
    __syncthreads();

    // ---- rescore
    const bool live = lane < T;
    uint32_t idx = 0xFFFFFFFFu;
    if (live) {
        idx = key_index(sh.top[0][lane]);
        float cf[2 * R];
        direction_f32<R>(p.seed, idx, (uint32_t)t, cf);
        double c[2 * R], acc[2 * R];
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) {
            c[j] = (double)cf[j];
            acc[j] = 0.0;
        }
        for (int i = w; i < n; i += NW) {
            double vr[R], vi[R], wr = 0.0, wi = 0.0;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                vr[j] = p.real ? (double)V[i * R + j] : (double)V[(i * R + j) * 2];
                vi[j] = p.real ? 0.0 : (double)V[(i * R + j) * 2 + 1];
                wr += vr[j] * c[2 * j] - vi[j] * c[2 * j + 1];
                wi += vr[j] * c[2 * j + 1] + vi[j] * c[2 * j];
            }
            double zr, zi;
            nearest_root64<KS>(wr, wi, p.K, sh.roots, zr, zi);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                acc[2 * j] += vr[j] * zr + vi[j] * zi;
                acc[2 * j + 1] += vr[j] * zi - vi[j] * zr;
            }
        }
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) sh.part[w][lane][j] = acc[j];
    }
    __syncthreads();

    // ---- pick (wave 0)
    if (w == 0) {
        double fq = -1.0;
        if (live) {
            fq = 0.0;
#pragma unroll
            for (int j = 0; j < 2 * R; ++j) {
                double a = 0.0;
                for (int v = 0; v < NW; ++v) a += sh.part[v][lane][j];
                fq += a * a;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double fo = __shfl_xor(fq, off, 64);
            const uint32_t io = __shfl_xor(idx, off, 64);
            if (fo > fq || (fo == fq && io < idx)) {
                fq = fo;
                idx = io;
            }
        }
        if (lane == 0) {
            p.obj[t] = fq;
            p.best[t] = idx;
            float cf[2 * R];
            direction_f32<R>(p.seed, idx, (uint32_t)t, cf);
            for (int j = 0; j < 2 * R; ++j) sh.cbest[j] = (double)cf[j];
        }
    }
    __syncthreads();

    // ---- labels of the winner
    for (int i = threadIdx.x; i < n; i += kBlock) {
        double wr = 0.0, wi = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const double vr = p.real ? (double)V[i * R + j] : (double)V[(i * R + j) * 2];
            const double vi = p.real ? 0.0 : (double)V[(i * R + j) * 2 + 1];
            wr += vr * sh.cbest[2 * j] - vi * sh.cbest[2 * j + 1];
            wi += vr * sh.cbest[2 * j + 1] + vi * sh.cbest[2 * j];
        }
        p.z[p.zoff[t] + i] = (uint8_t)label_f64(wr, wi, p.K);
    }
}

template <int KS>
__global__ __launch_bounds__(kBlock) void k_batch_select(BatchDevParams p) {
    __shared__ SelectShared<KS> sh;
    const int t = blockIdx.x;
    if constexpr (KS == 0) {
        for (int k = threadIdx.x; k < p.K; k += kBlock) sh.roots[k] = p.roots64[k];
    }
    const int nf = p.n[t] * p.r[t] * (p.real ? 1 : 2);
    const float* src = p.V + p.voff[t];
    for (int e = threadIdx.x; e < nf; e += kBlock) sh.Vs[e] = src[e];
    if (threadIdx.x == 0) sh.cnt = 0u;
    __syncthreads();
    switch (p.r[t]) {
        case 1: select_rescore<1, KS>(p, t, sh); break;
        case 2: select_rescore<2, KS>(p, t, sh); break;
        case 3: select_rescore<3, KS>(p, t, sh); break;
        case 4: select_rescore<4, KS>(p, t, sh); break;
        default: break;
    }
}

void launch_select(const BatchDevParams& p, hipStream_t st) {
    const dim3 g(p.count), b(kBlock);
    switch (k_special(p.K)) {
        case 2: hipLaunchKernelGGL((k_batch_select<2>), g, b, 0, st, p); break;
        case 3: hipLaunchKernelGGL((k_batch_select<3>), g, b, 0, st, p); break;
        case 4: hipLaunchKernelGGL((k_batch_select<4>), g, b, 0, st, p); break;
        case 8: hipLaunchKernelGGL((k_batch_select<8>), g, b, 0, st, p); break;
        case 16: hipLaunchKernelGGL((k_batch_select<16>), g, b, 0, st, p); break;
        default: hipLaunchKernelGGL((k_batch_select<0>), g, b, 0, st, p); break;
    }
}

__global__ void k_batch_check(const float* V, int64_t count, int* flag) {
    bool bad = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(V[e]);
    if (bad) *flag = 1;
}

// ---------------------------------------------------------------- host state
struct LaunchShape {
    int cpl = 4;
    int blocks_per_cu = 4;
};

template <int CPL>
void launch_score_cpl(const BatchDevParams& p, int blocks, hipStream_t st) {
    switch (k_special(p.K)) {
        case 2: hipLaunchKernelGGL((k_batch_score<CPL, 2>), dim3(blocks), dim3(kBlock), 0, st, p); break;
        case 3: hipLaunchKernelGGL((k_batch_score<CPL, 3>), dim3(blocks), dim3(kBlock), 0, st, p); break;
        case 4: hipLaunchKernelGGL((k_batch_score<CPL, 4>), dim3(blocks), dim3(kBlock), 0, st, p); break;
        case 8: hipLaunchKernelGGL((k_batch_score<CPL, 8>), dim3(blocks), dim3(kBlock), 0, st, p); break;
        case 16: hipLaunchKernelGGL((k_batch_score<CPL, 16>), dim3(blocks), dim3(kBlock), 0, st, p); break;
        default: hipLaunchKernelGGL((k_batch_score<CPL, 0>), dim3(blocks), dim3(kBlock), 0, st, p); break;
    }
}

void launch_score(const BatchDevParams& p, int cpl, int blocks, hipStream_t st) {
    if (cpl == 1) launch_score_cpl<1>(p, blocks, st);
    else if (cpl == 2) launch_score_cpl<2>(p, blocks, st);
    else launch_score_cpl<4>(p, blocks, st);
}

struct BatchPlan {
    std::vector<int32_t> items;
    int tile = 0;
};

// Items sorted by decreasing cost n_t r_t, then instance, then tile.
void build_items(int count, const int32_t* n, const int32_t* r, int S, int tile, BatchPlan& bp) {
    const int tiles = (S + tile - 1) / tile;
    std::vector<int> order(count);
    for (int t = 0; t < count; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)n[a] * r[a] > (int64_t)n[b] * r[b];
    });
    bp.items.clear();
    bp.items.reserve((size_t)count * tiles);
    for (int t : order)
        for (int j = 0; j < tiles; ++j) bp.items.push_back((t << 8) | j);
    bp.tile = tile;
}

// ---------------------------------------------------------------- autotuner
std::mutex g_tune_mu;
std::map<std::string, LaunchShape> g_tune;
bool g_tune_loaded = false;

std::string tune_path() {
    const char* e = std::getenv("LRQO_TUNE_CACHE");
    if (e && *e) return e;
    const char* h = std::getenv("HOME");
    return std::string(h && *h ? h : "/tmp") + "/.cache/lrqo_batched_tune.json";
}

// Cache file: one JSON object per line {"key": "...", "cpl": c, "bpc": b}.
void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    FILE* fh = std::fopen(tune_path().c_str(), "r");
    if (!fh) return;
    char line[512];
    while (std::fgets(line, sizeof line, fh)) {
        char key[256];
        int cpl = 0, bpc = 0;
        if (std::sscanf(line, " {\"key\": \"%255[^\"]\", \"cpl\": %d, \"bpc\": %d", key, &cpl, &bpc) == 3 &&
            (cpl == 1 || cpl == 2 || cpl == 4) && bpc >= 1 && bpc <= 16)
            g_tune[key] = LaunchShape{cpl, bpc};
    }
    std::fclose(fh);
}

void make_parent_dirs(const std::string& path) {
    for (size_t pos = path.find('/', 1); pos != std::string::npos; pos = path.find('/', pos + 1))
        (void)::mkdir(path.substr(0, pos).c_str(), 0755);
}

void tune_store(const std::string& key, const LaunchShape& ls) {
    const std::string path = tune_path();
    make_parent_dirs(path);
    FILE* fh = std::fopen(path.c_str(), "a");
    if (!fh) return;
    std::fprintf(fh, "{\"key\": \"%s\", \"cpl\": %d, \"bpc\": %d}\n", key.c_str(), ls.cpl,
                 ls.blocks_per_cu);
    std::fclose(fh);
}

std::string tune_key(int count, const int32_t* n, const int32_t* r, int K, int S, int real) {
    int64_t rows = 0;
    int rmax = 0;
    for (int t = 0; t < count; ++t) {
        rows += n[t];
        rmax = std::max(rmax, (int)r[t]);
    }
    const int64_t nmean = rows / std::max(1, count);
    int nb = 16;
    while (nb < nmean) nb <<= 1;     // n bucket: next power of two of the mean
    char buf[160];
    std::snprintf(buf, sizeof buf, "gfx950/K%d/S%d/r%d/n%d/real%d/count%d", K, S, rmax, nb, real,
                  count >= 1024 ? 1024 : (count >= 64 ? 64 : 1));
    return buf;
}

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::string sig;
};

std::mutex g_batch_mu;
hipStream_t g_batch_stream[64] = {};
GraphCache g_graph[64];

}  // namespace
}  // namespace lrqo

extern "C" {

lrqo_status lrqo_solve_batched(const float* V, int32_t count, const int64_t* v_offset,
                               const int32_t* n, const int32_t* r, int32_t K, int64_t S,
                               uint64_t seed, const lrqo_batch_options* opt, uint8_t* z,
                               double* obj, lrqo_batch_result* res) {
    using namespace lrqo;
    clear_error();
    if (!V || !v_offset || !n || !r || !z || !obj) return fail(LRQO_EINVAL, "null pointer argument");
    if (count < 1 || count > (1 << 22)) return fail(LRQO_EINVAL, "count must be in [1, 2^22]");
    if (K < 2 || K > LRQO_MAX_K) return fail(LRQO_EINVAL, "K must be in [2, 255]");
    if (S < 1 || S > kMaxS) return fail(LRQO_EINVAL, "S must be in [1, 4096] for the batched form");
    lrqo_batch_options o{};
    if (opt) o = *opt;
    if (o.real_v != 0 && o.real_v != 1) return fail(LRQO_EINVAL, "real_v must be 0 or 1");
    if (o.rescore_topk < 0 || o.rescore_topk > kTopT) return fail(LRQO_EINVAL, "rescore_topk must be in [0, 64]");
    if (o.cpl != 0 && o.cpl != 1 && o.cpl != 2 && o.cpl != 4) return fail(LRQO_EINVAL, "cpl must be 0, 1, 2 or 4");
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 16) return fail(LRQO_EINVAL, "blocks_per_cu must be in [0, 16]");
    int64_t rows = 0;
    int64_t vfloats = 0;
    for (int t = 0; t < count; ++t) {
        if (n[t] < 1 || n[t] > kMaxRows) return fail(LRQO_EINVAL, "every n_t must be in [1, 256]");
        if (r[t] < 1 || r[t] > 4) return fail(LRQO_EINVAL, "every r_t must be in [1, 4]");
        if (v_offset[t] < 0) return fail(LRQO_EINVAL, "v_offset must be >= 0");
        rows += n[t];
        vfloats = std::max<int64_t>(vfloats, v_offset[t] + (int64_t)n[t] * r[t] * (o.real_v ? 1 : 2));
    }
    const int T = o.rescore_topk == 0 ? (int)std::min<int64_t>(kTopT, S) : (int)std::min<int64_t>(o.rescore_topk, S);

    DeviceCtx* ctx = device_ctx();
    if (!ctx) return LRQO_EDEVICE;
    if (!is_device_pointer(V)) return fail(LRQO_EINVAL, "V is not device memory");
    if (!is_device_pointer(z)) return fail(LRQO_EINVAL, "z is not device memory");
    int ncu = 256;
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
    }

    std::lock_guard<std::mutex> lk(ctx->mu);
    std::lock_guard<std::mutex> bl(g_batch_mu);
    const int dev = ctx->device;
    if (!g_batch_stream[dev]) LRQO_HIP(hipStreamCreateWithFlags(&g_batch_stream[dev], hipStreamNonBlocking));
    hipStream_t bs = g_batch_stream[dev];

    // the largest possible item list (tile = 256 directions)
    const int max_items = count * ((int)((S + 255) / 256));
    CarveSize cs;
    cs.add<int64_t>(count);            // voff
    cs.add<int32_t>(count);            // n
    cs.add<int32_t>(count);            // r
    cs.add<int64_t>(count);            // zoff
    cs.add<int32_t>(max_items);        // items
    cs.add<unsigned int>(64);          // cursor, flags
    cs.add<float>((size_t)count * S);  // scores
    cs.add<double>(count);             // obj
    cs.add<int64_t>(count);            // best index
    cs.add<float2>(LRQO_MAX_K);
    cs.add<double2>(LRQO_MAX_K);
    cs.add<uint8_t>(rows);             // labels (copied to the caller's z after the graph)
    const size_t host_need = Carve::round(sizeof(int64_t) * count) * 3 + Carve::round(sizeof(int32_t) * count) * 2 +
                             Carve::round(sizeof(int32_t) * max_items) + Carve::round(sizeof(double) * count) +
                             Carve::round(sizeof(int64_t) * count) + 3 * 4096 + 64;
    const void* old_arena = ctx->arena;
    LRQO_TRY(reserve_arena(ctx, cs.bytes));
    LRQO_TRY(reserve_host(ctx, host_need));
    Carve cv(ctx->arena);
    BatchDevParams p{};
    int64_t* d_voff = cv.take<int64_t>(count);
    int32_t* d_n = cv.take<int32_t>(count);
    int32_t* d_r = cv.take<int32_t>(count);
    int64_t* d_zoff = cv.take<int64_t>(count);
    int32_t* d_items = cv.take<int32_t>(max_items);
    unsigned int* d_cursor = cv.take<unsigned int>(64);
    float* d_f = cv.take<float>((size_t)count * S);
    double* d_obj = cv.take<double>(count);
    int64_t* d_best = cv.take<int64_t>(count);
    float2* d_r32 = cv.take<float2>(LRQO_MAX_K);
    double2* d_r64 = cv.take<double2>(LRQO_MAX_K);
    uint8_t* d_z = cv.take<uint8_t>(rows);

    Carve hv(ctx->host);
    int64_t* h_voff = hv.take<int64_t>(count);
    int32_t* h_n = hv.take<int32_t>(count);
    int32_t* h_r = hv.take<int32_t>(count);
    int64_t* h_zoff = hv.take<int64_t>(count);
    int32_t* h_items = hv.take<int32_t>(max_items);
    double* h_obj = hv.take<double>(count);
    int64_t* h_best = hv.take<int64_t>(count);
    double2* h_r64 = hv.take<double2>(LRQO_MAX_K);
    float2* h_r32 = hv.take<float2>(LRQO_MAX_K);
    int* h_flag = hv.take<int>(16);

    int64_t zacc = 0;
    for (int t = 0; t < count; ++t) {
        h_voff[t] = v_offset[t];
        h_n[t] = n[t];
        h_r[t] = r[t];
        h_zoff[t] = zacc;
        zacc += n[t];
    }
    for (int k = 0; k < K; ++k) {
        const double a = 6.283185307179586476925286766559 * (double)k / (double)K;
        h_r64[k] = make_double2(std::cos(a), std::sin(a));
        h_r32[k] = make_float2((float)h_r64[k].x, (float)h_r64[k].y);
    }

    p.V = V;
    p.voff = d_voff;
    p.n = d_n;
    p.r = d_r;
    p.zoff = d_zoff;
    p.items = d_items;
    p.count = count;
    p.K = K;
    p.S = (int32_t)S;
    p.seed = seed;
    p.real = o.real_v;
    p.cursor = d_cursor;
    p.f = d_f;
    p.obj = d_obj;
    p.best = d_best;
    p.z = d_z;
    p.roots32 = d_r32;
    p.roots64 = d_r64;
    p.T = T;

    // the caller's earlier work on its stream comes first
    LRQO_HIP(hipStreamSynchronize(current_stream()));
    LRQO_HIP(hipMemcpyAsync(d_r64, h_r64, sizeof(double2) * K, hipMemcpyHostToDevice, bs));
    LRQO_HIP(hipMemcpyAsync(d_r32, h_r32, sizeof(float2) * K, hipMemcpyHostToDevice, bs));

    // ---- finiteness of every factor
    *h_flag = 0;
    LRQO_HIP(hipMemcpyAsync(d_cursor + 32, h_flag, sizeof(int), hipMemcpyHostToDevice, bs));
    hipLaunchKernelGGL(k_batch_check, dim3(256), dim3(256), 0, bs, V, vfloats,
                       reinterpret_cast<int*>(d_cursor + 32));
    LRQO_HIP(hipGetLastError());
    LRQO_HIP(hipMemcpyAsync(h_flag, d_cursor + 32, sizeof(int), hipMemcpyDeviceToHost, bs));
    LRQO_HIP(hipStreamSynchronize(bs));
    if (*h_flag) return fail(LRQO_ENOTFINITE, "a factor holds a NaN or an infinity");

    // ---- launch shape: explicit, cached, or tuned now
    LaunchShape ls;
    bool tuned_now = false;
    const std::string key = tune_key(count, n, r, K, (int)S, o.real_v);
    {
        std::lock_guard<std::mutex> tl(g_tune_mu);
        tune_load();
        auto itc = g_tune.find(key);
        if (o.cpl && o.blocks_per_cu) {
            ls = LaunchShape{o.cpl, o.blocks_per_cu};
        } else if (itc != g_tune.end()) {
            ls = itc->second;
        } else {
            // time each candidate shape once on this batch (after one warm-up)
            float best_ms = 1e30f;
            const int cpls[3] = {1, 2, 4};
            const int bpcs[3] = {2, 4, 8};
            for (int ci = 0; ci < 3; ++ci) {
                for (int bi = 0; bi < 3; ++bi) {
                    BatchPlan bp;
                    build_items(count, n, r, (int)S, kBlock * cpls[ci], bp);
                    std::memcpy(h_items, bp.items.data(), sizeof(int32_t) * bp.items.size());
                    LRQO_HIP(hipMemcpyAsync(d_voff, h_voff, sizeof(int64_t) * count, hipMemcpyHostToDevice, bs));
                    LRQO_HIP(hipMemcpyAsync(d_n, h_n, sizeof(int32_t) * count, hipMemcpyHostToDevice, bs));
                    LRQO_HIP(hipMemcpyAsync(d_r, h_r, sizeof(int32_t) * count, hipMemcpyHostToDevice, bs));
                    LRQO_HIP(hipMemcpyAsync(d_items, h_items, sizeof(int32_t) * bp.items.size(),
                                            hipMemcpyHostToDevice, bs));
                    BatchDevParams q = p;
                    q.nitems = (int)bp.items.size();
                    q.tile = bp.tile;
                    float ms = 0.0f;
                    for (int rep = 0; rep < 2; ++rep) {
                        hipLaunchKernelGGL(k_bfill, dim3(1), dim3(64), 0, bs, d_cursor);
                        LRQO_HIP(hipEventRecord(ctx->ev_score0, bs));
                        launch_score(q, cpls[ci], ncu * bpcs[bi], bs);
                        LRQO_HIP(hipGetLastError());
                        LRQO_HIP(hipEventRecord(ctx->ev_score1, bs));
                        LRQO_HIP(hipEventSynchronize(ctx->ev_score1));
                        LRQO_HIP(hipEventElapsedTime(&ms, ctx->ev_score0, ctx->ev_score1));
                    }
                    if (ms < best_ms) {
                        best_ms = ms;
                        ls = LaunchShape{cpls[ci], bpcs[bi]};
                    }
                }
            }
            g_tune[key] = ls;
            tune_store(key, ls);
            tuned_now = true;
        }
    }

    BatchPlan bp;
    build_items(count, n, r, (int)S, kBlock * ls.cpl, bp);
    std::memcpy(h_items, bp.items.data(), sizeof(int32_t) * bp.items.size());
    p.nitems = (int)bp.items.size();
    p.tile = bp.tile;
    const int blocks = ncu * ls.blocks_per_cu;

    // ---- the graph: descriptors in, score, select, rescore, results out
    char sigbuf[256];
    std::snprintf(sigbuf, sizeof sigbuf, "%d/%d/%lld/%llu/%d/%d/%d/%d/%p/%p/%p/%lld", count, K,
                  (long long)S, (unsigned long long)seed, o.real_v, T, ls.cpl, blocks, (const void*)V,
                  ctx->arena, ctx->host, (long long)rows);
    GraphCache& gc = g_graph[dev];
    const bool use_graph = !o.no_graph;
    if (use_graph && (gc.sig != sigbuf || ctx->arena != old_arena)) {
        if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
        if (gc.graph) (void)hipGraphDestroy(gc.graph);
        gc.exec = nullptr;
        gc.graph = nullptr;
        gc.sig.clear();
    }
    auto enqueue = [&](hipStream_t s) -> lrqo_status {
        LRQO_HIP(hipMemcpyAsync(d_voff, h_voff, sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
        LRQO_HIP(hipMemcpyAsync(d_n, h_n, sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
        LRQO_HIP(hipMemcpyAsync(d_r, h_r, sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
        LRQO_HIP(hipMemcpyAsync(d_zoff, h_zoff, sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
        LRQO_HIP(hipMemcpyAsync(d_items, h_items, sizeof(int32_t) * p.nitems, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_bfill, dim3(1), dim3(64), 0, s, d_cursor);
        launch_score(p, ls.cpl, blocks, s);
        launch_select(p, s);
        LRQO_HIP(hipMemcpyAsync(h_obj, d_obj, sizeof(double) * count, hipMemcpyDeviceToHost, s));
        LRQO_HIP(hipMemcpyAsync(h_best, d_best, sizeof(int64_t) * count, hipMemcpyDeviceToHost, s));
        return LRQO_OK;
    };
    bool captured_now = false;
    if (use_graph && !gc.exec) {
        LRQO_HIP(hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal));
        const lrqo_status s1 = enqueue(bs);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(bs, &g);
        if (s1 != LRQO_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s1;
        }
        if (e != hipSuccess) return fail(LRQO_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
        LRQO_HIP(hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0));
        gc.graph = g;
        gc.sig = sigbuf;
        captured_now = true;
    }
    LRQO_HIP(hipEventRecord(ctx->ev_start, bs));
    if (use_graph) {
        LRQO_HIP(hipGraphLaunch(gc.exec, bs));
    } else {
        LRQO_TRY(enqueue(bs));
    }
    LRQO_HIP(hipEventRecord(ctx->ev_stop, bs));
    LRQO_HIP(hipMemcpyAsync(z, d_z, (size_t)rows, hipMemcpyDeviceToDevice, bs));
    LRQO_HIP(hipStreamSynchronize(bs));
    float ms = 0.0f;
    LRQO_HIP(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));
    for (int t = 0; t < count; ++t) obj[t] = h_obj[t];
    if (res) {
        std::memset(res, 0, sizeof *res);
        res->device_ms = ms;
        res->cpl = ls.cpl;
        res->blocks_per_cu = ls.blocks_per_cu;
        res->items = p.nitems;
        res->tuned_now = tuned_now ? 1 : 0;
        res->graph_captured_now = captured_now ? 1 : 0;
        res->row_candidates = rows * S;
        if (o.best_index) for (int t = 0; t < count; ++t) o.best_index[t] = h_best[t];
    }
    return LRQO_OK;
}

}  // extern "C"
