/*
 * FP64 CPU oracle for the low-rank K-ary quadratic maximizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the GPU path.
 *
 * What it computes (plain definitions, no blocking or fusion):
 *   - the problem  max_{z in A_K^n} ||V^H z||^2, A_K the K-th roots of unity
 *     (Sec. 1, eq. max_quad and AK_def; the factor form of Sec. 2.2,
 *     eq. quad_max-norm);
 *   - the decision rule z_i = nearest K-th root to arg((V c)_i)
 *     (Sec. 3, eq. decision_rule; rank-1 form k = floor(K theta/2pi + 1/2) of
 *     Sec. 2.5);
 *   - the sampled objective f(c) = ||V^H z(c)||^2 (Sec. 4.2, eq. def_f) and the
 *     best of S directions drawn uniformly from the complex unit sphere as
 *     c = Z/||Z||, Z standard complex Gaussian (Sec. 4.2; proof of
 *     Lemma innerIsBeta).
 *
 * The paper fixes no random-number generator.  The direction stream used by
 * both sides is: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key
 * (seed lo, seed hi) and counter (s lo, s hi, instance, block); the four
 * 32-bit words of block b give uniforms u[4b..4b+3] = ((x >> 9) + 1/2) 2^-23;
 * Box-Muller on pairs (u[2j], u[2j+1]) gives g[2j] = sqrt(-2 ln u[2j])
 * cos(2 pi u[2j+1]) and g[2j+1] = ... sin(...); c_j = (g[2j] + i g[2j+1])/||g||.
 *
 * Everything here is FP64 with libm transcendentals, compiled without
 * fast-math.  V is complex, row-major, interleaved (re, im): V[(i*r + j)*2].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

/* ---------------------------------------------------------------- Philox */

static void philox_round(uint32_t x[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * x[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x[1] ^ k[0];
    const uint32_t y1 = lo1;
    const uint32_t y2 = hi0 ^ x[3] ^ k[1];
    const uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

/* Philox4x32 with 10 rounds: out = F(ctr, key). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(x, k);
    }
    memcpy(out, x, sizeof x);
}

/* Uniform on (0,1) from one 32-bit word: 23 random bits, centred in the cell. */
double oracle_uniform(uint32_t x) {
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Direction c_s in C^r (r <= 8), written as c[2j] = Re c_j, c[2j+1] = Im c_j. */
void oracle_direction(uint64_t seed, uint64_t s, uint32_t instance, int r, double* c) {
    double u[16];
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const int nblocks = (2 * r + 3) / 4;
    for (int b = 0; b < nblocks; ++b) {
        const uint32_t ctr[4] = {(uint32_t)s, (uint32_t)(s >> 32), instance, (uint32_t)b};
        uint32_t out[4];
        oracle_philox4x32_10(ctr, key, out);
        for (int t = 0; t < 4; ++t) u[4 * b + t] = oracle_uniform(out[t]);
    }
    double norm2 = 0.0;
    for (int j = 0; j < r; ++j) {
        const double rad = sqrt(-2.0 * log(u[2 * j]));
        const double ang = TWO_PI * u[2 * j + 1];
        c[2 * j] = rad * cos(ang);
        c[2 * j + 1] = rad * sin(ang);
        norm2 += c[2 * j] * c[2 * j] + c[2 * j + 1] * c[2 * j + 1];
    }
    const double inv = 1.0 / sqrt(norm2);
    for (int j = 0; j < 2 * r; ++j) c[j] *= inv;
}

/* -------------------------------------------------------- decision rule */

/* Label k in [0, K) of the K-th root nearest in phase to w = wr + i wi:
 * k = floor(K arg(w) / 2pi + 1/2) mod K, with w = 0 mapped to k = 0. */
int oracle_label(double wr, double wi, int K) {
    if (wr == 0.0 && wi == 0.0) return 0;
    const double x = (double)K * atan2(wi, wr) / TWO_PI + 0.5;
    long k = (long)floor(x) % K;
    if (k < 0) k += K;
    return (int)k;
}

/* Angular distance (radians) from arg(w) to the nearest decision boundary
 * pi(2m+1)/K; 0 for w = 0. */
double oracle_boundary_distance(double wr, double wi, int K) {
    if (wr == 0.0 && wi == 0.0) return 0.0;
    const double x = (double)K * atan2(wi, wr) / TWO_PI + 0.5;
    const double fr = x - floor(x);
    const double d = fr < 1.0 - fr ? fr : 1.0 - fr;
    return d * TWO_PI / (double)K;
}

/* w = V c for every row, then labels (and optionally per-row boundary
 * distance in radians). */
void oracle_labels(const double* V, int64_t n, int r, int K, const double* c,
                   uint8_t* z, double* dist) {
    for (int64_t i = 0; i < n; ++i) {
        double wr = 0.0, wi = 0.0;
        for (int j = 0; j < r; ++j) {
            const double vr = V[(i * r + j) * 2], vi = V[(i * r + j) * 2 + 1];
            wr += vr * c[2 * j] - vi * c[2 * j + 1];
            wi += vr * c[2 * j + 1] + vi * c[2 * j];
        }
        z[i] = (uint8_t)oracle_label(wr, wi, K);
        if (dist) dist[i] = oracle_boundary_distance(wr, wi, K);
    }
}

/* ||V^H z||^2 with z_i = exp(2 pi i k_i / K). */
double oracle_objective(const double* V, int64_t n, int r, int K, const uint8_t* z) {
    double sr[8] = {0}, si[8] = {0};
    for (int64_t i = 0; i < n; ++i) {
        const double ang = TWO_PI * (double)z[i] / (double)K;
        const double zr = cos(ang), zi = sin(ang);
        for (int j = 0; j < r; ++j) {
            const double vr = V[(i * r + j) * 2], vi = V[(i * r + j) * 2 + 1];
            /* conj(V_ij) * z_i */
            sr[j] += vr * zr + vi * zi;
            si[j] += vr * zi - vi * zr;
        }
    }
    double f = 0.0;
    for (int j = 0; j < r; ++j) f += sr[j] * sr[j] + si[j] * si[j];
    return f;
}

/* f(c) for one direction; optional min over rows of the normalised margin
 * dist_i * |w_i| / sum_j |V_ij||c_j|  (how far, relative to the size of the
 * terms that produced w_i, the row sits from a boundary). */
double oracle_f_of_c(const double* V, int64_t n, int r, int K, const double* c,
                     double* min_margin) {
    double sr[8] = {0}, si[8] = {0};
    double mm = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double wr = 0.0, wi = 0.0, scale = 0.0;
        for (int j = 0; j < r; ++j) {
            const double vr = V[(i * r + j) * 2], vi = V[(i * r + j) * 2 + 1];
            wr += vr * c[2 * j] - vi * c[2 * j + 1];
            wi += vr * c[2 * j + 1] + vi * c[2 * j];
            scale += hypot(vr, vi) * hypot(c[2 * j], c[2 * j + 1]);
        }
        const int k = oracle_label(wr, wi, K);
        if (min_margin && scale > 0.0) {
            const double m = oracle_boundary_distance(wr, wi, K) * hypot(wr, wi) / scale;
            if (m < mm) mm = m;
        }
        const double ang = TWO_PI * (double)k / (double)K;
        const double zr = cos(ang), zi = sin(ang);
        for (int j = 0; j < r; ++j) {
            const double vr = V[(i * r + j) * 2], vi = V[(i * r + j) * 2 + 1];
            sr[j] += vr * zr + vi * zi;
            si[j] += vr * zi - vi * zr;
        }
    }
    if (min_margin) *min_margin = mm;
    double f = 0.0;
    for (int j = 0; j < r; ++j) f += sr[j] * sr[j] + si[j] * si[j];
    return f;
}

/* Best of the directions s = s0 .. s0+count-1 (Sec. 4.2): f for each into
 * f_out[count] (if non-null), optional per-candidate margins, and the
 * arg-max (ties to the smallest s).  OpenMP over candidates.  Returns the
 * number of threads used. */
int oracle_sampled(const double* V, int64_t n, int r, int K, uint64_t seed, uint32_t instance,
                   uint64_t s0, int64_t count, int nthreads, double* f_out, double* margin_out,
                   int64_t* best_s, double* best_f) {
    double* f = f_out ? f_out : (double*)malloc(sizeof(double) * (size_t)count);
    int used = 1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t t = 0; t < count; ++t) {
        double c[16];
        oracle_direction(seed, s0 + (uint64_t)t, instance, r, c);
        f[t] = oracle_f_of_c(V, n, r, K, c, margin_out ? &margin_out[t] : NULL);
#ifdef _OPENMP
        if (t == 0) used = omp_get_num_threads();
#endif
    }
    int64_t arg = 0;
    for (int64_t t = 1; t < count; ++t)
        if (f[t] > f[arg]) arg = t;
    if (best_s) *best_s = (int64_t)s0 + arg;
    if (best_f) *best_f = count > 0 ? f[arg] : 0.0;
    if (!f_out) free(f);
    return used;
}

/* ------------------------------------------------ near-boundary interval
 * f at each of `count` given directions (dirs[t*2r + 2j] = Re c_j,
 * dirs[t*2r + 2j + 1] = Im c_j), with an interval [lo, hi] holding the
 * objective of every labelling that differs from the FP64 decision rule only
 * on ambiguous rows.  A row is ambiguous when a label other than its own
 * borders w_i = V_i c within `reach` times its scale sum_j |V_ij||c_j|:
 *   - |w_i| <= reach * scale: every label;
 *   - otherwise each decision-boundary ray pi(2m+1)/K at angle delta < pi/2
 *     from arg(w_i) whose line lies within |w_i| sin(delta) <= reach * scale
 *     adds its two neighbouring labels.
 * Changing ambiguous row a moves s = V^H z by conj(V_a)(z'_a - z_a), of norm
 * at most D_a = ||V_a|| max |omega^k' - omega^k| over its options, so every
 * such labelling has ||s|| within ||s_0|| +- sum_a D_a:
 *   lo = max(0, ||s_0|| - sum D)^2,  hi = (||s_0|| + sum D)^2.
 * This is a tolerance device for comparing a lower-precision evaluation of
 * the decision rule (whose rounding can move w_i by a bounded amount) with
 * the FP64 one; it adds nothing to the method.  Returns the threads used. */
static double chord(int a, int b, int K) {
    /* |omega^a - omega^b| = 2 |sin(pi (a - b) / K)| */
    return 2.0 * fabs(sin(0.5 * TWO_PI * (double)(a - b) / (double)K));
}

static void score_one_dir(const double* V, int64_t n, int r, int K, const double* c, double reach,
                          double* f, double* lo, double* hi, int64_t* nambig) {
    double sr[8] = {0}, si[8] = {0};
    double spread = 0.0;
    int64_t na = 0;
    const double step = TWO_PI / (double)K;
    for (int64_t i = 0; i < n; ++i) {
        double wr = 0.0, wi = 0.0, scale = 0.0, vn2 = 0.0;
        for (int j = 0; j < r; ++j) {
            const double vr = V[(i * r + j) * 2], vi = V[(i * r + j) * 2 + 1];
            wr += vr * c[2 * j] - vi * c[2 * j + 1];
            wi += vr * c[2 * j + 1] + vi * c[2 * j];
            scale += hypot(vr, vi) * hypot(c[2 * j], c[2 * j + 1]);
            vn2 += vr * vr + vi * vi;
        }
        const int k = oracle_label(wr, wi, K);
        const double aw = hypot(wr, wi);
        const double lim = reach * scale;
        double dmax = 0.0;                 /* largest chord to an open label */
        if (lim > 0.0 && aw <= lim) {
            for (int o = 0; o < K; ++o) dmax = fmax(dmax, chord(o, k, K));
        } else if (lim > 0.0) {
            const double x = (double)K * atan2(wi, wr) / TWO_PI + 0.5;
            const double fr = x - floor(x);
            /* rays below arg(w): between labels k-j-1 and k-j, at fr*step + j*step */
            for (int j = 0;; ++j) {
                const double delta = fr * step + (double)j * step;
                if (delta >= (0.25 * TWO_PI) || aw * sin(delta) > lim) break;
                dmax = fmax(dmax, chord(((k - j - 1) % K + K) % K, k, K));
                dmax = fmax(dmax, chord(((k - j) % K + K) % K, k, K));
            }
            /* rays above: between labels k+j and k+j+1, at (1-fr)*step + j*step */
            for (int j = 0;; ++j) {
                const double delta = (1.0 - fr) * step + (double)j * step;
                if (delta >= (0.25 * TWO_PI) || aw * sin(delta) > lim) break;
                dmax = fmax(dmax, chord((k + j) % K, k, K));
                dmax = fmax(dmax, chord((k + j + 1) % K, k, K));
            }
        }
        if (dmax > 0.0) {
            ++na;
            spread += sqrt(vn2) * dmax;
        }
        const double ang = TWO_PI * (double)k / (double)K;
        const double zr = cos(ang), zi = sin(ang);
        for (int j = 0; j < r; ++j) {
            const double vr = V[(i * r + j) * 2], vi = V[(i * r + j) * 2 + 1];
            sr[j] += vr * zr + vi * zi;
            si[j] += vr * zi - vi * zr;
        }
    }
    double ff = 0.0;
    for (int j = 0; j < r; ++j) ff += sr[j] * sr[j] + si[j] * si[j];
    const double ns = sqrt(ff);
    const double a = ns - spread > 0.0 ? ns - spread : 0.0;
    *f = ff;
    *lo = spread > 0.0 ? a * a : ff;
    *hi = spread > 0.0 ? (ns + spread) * (ns + spread) : ff;
    *nambig = na;
}

int oracle_score_dirs(const double* V, int64_t n, int r, int K, const double* dirs, int64_t count,
                      double reach, int nthreads, double* f_out, double* lo_out, double* hi_out,
                      int64_t* nambig_out) {
    int used = 1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t t = 0; t < count; ++t) {
        score_one_dir(V, n, r, K, dirs + t * 2 * r, reach, &f_out[t], &lo_out[t], &hi_out[t],
                      &nambig_out[t]);
#ifdef _OPENMP
        if (t == 0) used = omp_get_num_threads();
#endif
    }
    return used;
}
