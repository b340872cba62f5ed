// Device-side building blocks shared by the liblrqo kernels: the direction
// stream, the FP64 decision rule and small reductions.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lrqo {

constexpr int kWave = 64;

// ---------------------------------------------------------------- Philox
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): per round
// (hi0,lo0) = M0*x0, (hi1,lo1) = M1*x2, x <- (hi1^x1^k0, lo1, hi0^x3^k1, lo0),
// then the key is bumped by the Weyl constants.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one v_mad_u64_u32 per product (hi and lo together): faster on
        // gfx950 than a v_mul_lo_u32 / v_mul_hi_u32 pair
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
        const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
        const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Uniform on (0,1) with 23 random bits, exactly representable in FP32.
__device__ __forceinline__ float uniform_from_bits(uint32_t x) {
    return (static_cast<float>(x >> 9) + 0.5f) * 0x1p-23f;
}

// Direction c_s of the stream (seed, instance) in C^R, FP32, as
// c[2j] = Re c_j, c[2j+1] = Im c_j.  Box-Muller on uniform pairs, then
// normalisation to the unit sphere.
template <int R>
__device__ __forceinline__ void direction_f32(uint64_t seed, uint64_t s, uint32_t instance,
                                              float (&c)[2 * R]) {
    constexpr int NB = (2 * R + 3) / 4;
    float u[4 * NB];
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const U4 o = philox4x32_10(U4{static_cast<uint32_t>(s), static_cast<uint32_t>(s >> 32),
                                      instance, static_cast<uint32_t>(b)},
                                   k0, k1);
        u[4 * b + 0] = uniform_from_bits(o.x);
        u[4 * b + 1] = uniform_from_bits(o.y);
        u[4 * b + 2] = uniform_from_bits(o.z);
        u[4 * b + 3] = uniform_from_bits(o.w);
    }
    float norm2 = 0.0f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const float rad = sqrtf(-2.0f * logf(u[2 * j]));
        float sn, cs;
        sincospif(2.0f * u[2 * j + 1], &sn, &cs);
        c[2 * j] = rad * cs;
        c[2 * j + 1] = rad * sn;
        norm2 += c[2 * j] * c[2 * j] + c[2 * j + 1] * c[2 * j + 1];
    }
    const float inv = 1.0f / sqrtf(norm2);
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) c[j] *= inv;
}

// Direction s: from the stream, or row s of a caller-supplied list.
template <int R>
__device__ __forceinline__ void direction_any(const float* dirs, uint64_t seed, uint64_t s,
                                              uint32_t instance, float (&c)[2 * R]) {
    if (dirs) {
#pragma unroll
        for (int j = 0; j < 2 * R; ++j) c[j] = dirs[s * (2 * R) + j];
    } else {
        direction_f32<R>(seed, s, instance, c);
    }
}

// ---------------------------------------------------------------- labels
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Decision rule in FP64: the K-th root nearest in phase,
// k = floor(K arg(w)/(2 pi) + 1/2) mod K, with w = 0 -> 0.
// Non-finite input maps to 0 so that table lookups stay in range (the
// library reports such input as an error).
__device__ __forceinline__ int label_f64(double wr, double wi, int K) {
    if (wr == 0.0 && wi == 0.0) return 0;
    const double x = static_cast<double>(K) * atan2(wi, wr) / kTwoPi + 0.5;
    if (!(x > -2.0 * K && x < 2.0 * K)) return 0;
    int k = static_cast<int>(floor(x)) % K;
    return k < 0 ? k + K : k;
}

// Same rule in FP32 for any K.
__device__ __forceinline__ int label_f32_generic(float wr, float wi, int K) {
    const float x = static_cast<float>(K) * (atan2f(wi, wr) * 0.15915494309189535f) + 0.5f;
    if (!(x > -(float)K && x < (float)K)) return 0;
    int k = static_cast<int>(floorf(x));
    k = k >= K ? k - K : k;
    k = k < 0 ? k + K : k;
    return (wr == 0.0f && wi == 0.0f) ? 0 : k;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ---------------------------------------------------------------- wave top-64
// A wave holds a list of 64 packed keys, one per lane, lane l the l-th
// largest.  wave_sort_desc sorts one key per lane (bitonic network over lane
// shuffles); wave_top_union keeps the best 64 of two such lists (a
// half-cleaner against the reversed second list, then a bitonic merge).
__device__ __forceinline__ unsigned long long key_max(unsigned long long a, unsigned long long b) {
    return a > b ? a : b;
}
__device__ __forceinline__ unsigned long long key_min(unsigned long long a, unsigned long long b) {
    return a < b ? a : b;
}

// One key per lane, returned sorted descending by lane.
__device__ __forceinline__ unsigned long long wave_sort_desc(unsigned long long x, int lane) {
    for (int k = 2; k <= 64; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const unsigned long long y = __shfl_xor(x, j, 64);
            // in a descending run the lower lane of a pair keeps the larger key
            const bool keep_max = ((lane & j) == 0) == ((lane & k) == 0);
            x = keep_max ? key_max(x, y) : key_min(x, y);
        }
    }
    return x;
}

// Best 64 of two descending lists (one key per lane), descending.
__device__ __forceinline__ unsigned long long wave_top_union(unsigned long long a,
                                                             unsigned long long b, int lane) {
    unsigned long long x = key_max(a, __shfl(b, 63 - lane, 64));  // bitonic, holds the best 64
    for (int j = 32; j > 0; j >>= 1) {
        const unsigned long long y = __shfl_xor(x, j, 64);
        x = (lane & j) == 0 ? key_max(x, y) : key_min(x, y);
    }
    return x;
}

// Best 64 keys of two descending lists with one key per objective value: the
// 128 keys are merged into a sorted sequence (half-cleaner against the
// reversed second list, both halves sorted), a key whose objective equals the
// one before it is cleared (the larger key, i.e. the lower index, stays), and
// the best 64 survivors are kept.  Clearing to 0 (below every real key) makes
// the result a list padded at its end.
__device__ __forceinline__ unsigned long long wave_top_union_distinct(unsigned long long a,
                                                                      unsigned long long b, int lane) {
    const unsigned long long br = __shfl(b, 63 - lane, 64);
    unsigned long long hi = key_max(a, br), lo = key_min(a, br);
    for (int j = 32; j > 0; j >>= 1) {
        const unsigned long long yh = __shfl_xor(hi, j, 64), yl = __shfl_xor(lo, j, 64);
        const bool up = (lane & j) == 0;
        hi = up ? key_max(hi, yh) : key_min(hi, yh);
        lo = up ? key_max(lo, yl) : key_min(lo, yl);
    }
    // hi holds positions 0..63 of the merged sequence, lo positions 64..127
    const unsigned long long h63 = __shfl(hi, 63, 64);
    const unsigned long long hp = __shfl_up(hi, 1, 64);
    const unsigned long long lp = __shfl_up(lo, 1, 64);
    const unsigned long long hprev = lane == 0 ? 0ull : hp;
    const unsigned long long lprev = lane == 0 ? h63 : lp;
    if (hi != 0 && hprev != 0 && (hi >> 32) == (hprev >> 32)) hi = 0;
    if (lo != 0 && lprev != 0 && (lo >> 32) == (lprev >> 32)) lo = 0;
    return wave_top_union(wave_sort_desc(hi, lane), wave_sort_desc(lo, lane), lane);
}

// Packed arg-max key: objective bits above, complemented index below, so the
// unsigned maximum is the largest objective and, among equal objectives, the
// lowest index.  f >= 0, so its IEEE bits order like the values.
__device__ __forceinline__ unsigned long long pack_key(float f, uint32_t idx) {
    return (static_cast<unsigned long long>(__float_as_uint(f)) << 32) |
           static_cast<unsigned long long>(0xFFFFFFFFu - idx);
}
__device__ __forceinline__ uint32_t key_index(unsigned long long key) {
    return 0xFFFFFFFFu - static_cast<uint32_t>(key & 0xFFFFFFFFull);
}
__device__ __forceinline__ float key_value(unsigned long long key) {
    return __uint_as_float(static_cast<uint32_t>(key >> 32));
}

// ------------------------------------------------------------ nearest root
// KS selects a closed form for K = 2, 3, 4, 8, 16; KS = 0 is any K via atan2
// and an LDS table of roots.  Ties on a boundary (measure zero) may go either
// way; the FP64 rescore decides the returned labels.
template <int KS>
__device__ __forceinline__ void nearest_root(float wr, float wi, int K, const float2* roots,
                                             float& zr, float& zi) {
    if constexpr (KS == 2) {
        const bool k0 = wr >= 0.0f;
        zr = k0 ? 1.0f : -1.0f;
        zi = 0.0f;
    } else if constexpr (KS == 3) {
        // label 0 iff |arg w| < pi/3  <=>  |wi| < sqrt(3) wr; otherwise the
        // sign of wi picks omega (upper half) or omega^2 (lower half)
        const bool k0 = fabsf(wi) <= wr * 1.7320508075688772f;
        zr = k0 ? 1.0f : -0.5f;
        zi = k0 ? 0.0f : copysignf(0.8660254037844386f, wi);
    } else if constexpr (KS == 4) {
        const bool horiz = fabsf(wr) >= fabsf(wi);
        zr = horiz ? copysignf(1.0f, wr) : 0.0f;
        zi = horiz ? 0.0f : copysignf(1.0f, wi);
    } else if constexpr (KS == 8) {
        // fold into the first quadrant; boundaries at 22.5 and 67.5 degrees
        const float ax = fabsf(wr), ay = fabsf(wi);
        const float t = 0.41421356237309505f;        // tan(pi/8)
        const bool h = ay <= t * ax, v = ax <= t * ay;
        const float d = 0.70710678118654752f;
        zr = copysignf(h ? 1.0f : (v ? 0.0f : d), wr);
        zi = copysignf(h ? 0.0f : (v ? 1.0f : d), wi);
    } else if constexpr (KS == 16) {
        // fold into the first octant (swap when ay > ax); roots at 0, 22.5,
        // 45 degrees there, boundaries at 11.25 and 33.75 degrees
        const float ax = fabsf(wr), ay = fabsf(wi);
        const bool sw = ay > ax;
        const float lo = sw ? ax : ay, hi = sw ? ay : ax;
        const bool b1 = lo > 0.19891236737965800f * hi;   // tan(pi/16)
        const bool b2 = lo > 0.66817863791929892f * hi;   // tan(3 pi/16)
        const float cc = b2 ? 0.70710678118654752f : (b1 ? 0.92387953251128676f : 1.0f);
        const float ss = b2 ? 0.70710678118654752f : (b1 ? 0.38268343236508977f : 0.0f);
        zr = copysignf(sw ? ss : cc, wr);
        zi = copysignf(sw ? cc : ss, wi);
    } else {
        const int k = label_f32_generic(wr, wi, K);
        const float2 t = roots[k];
        zr = t.x;
        zi = t.y;
    }
}

// K = 8 in the frame of w' = w e^{-i pi/8} (the caller scores the turned
// direction c e^{-i pi/8}).  The set of w nearest root k, arg w within pi/8
// of k pi/4, becomes the wedge of w' between the lines at (k-1) pi/4 and
// k pi/4: the signs of Re w', Im w' and which of |Re w'|, |Im w'| is larger
// fix it.  The root turned by the same angle, e^{i (k pi/4 - pi/8)}, is the
// wedge's bisector: (cos pi/8, sin pi/8) or (sin pi/8, cos pi/8), with the
// signs of w'.  Sums of V^H times turned roots are the sums of V^H z turned
// by e^{-i pi/8}, a unit factor that leaves ||s||^2 unchanged.
constexpr float kCos8 = 0.92387953251128674f;   // cos(pi/8)
constexpr float kSin8 = 0.38268343236508977f;   // sin(pi/8)

__device__ __forceinline__ void bisector_k8(float a, float b, float& yr, float& yi) {
    const bool big = fabsf(a) >= fabsf(b);
    yr = copysignf(big ? kCos8 : kSin8, a);
    yi = copysignf(big ? kSin8 : kCos8, b);
}

// K = 16 likewise, in the frame of w' = w e^{-i pi/16}: the sectors become
// the wedges between consecutive multiples of pi/8.  In the quadrant of w'
// they are told apart by which part is larger and by whether the smaller
// exceeds tan(pi/8) times the larger; the turned roots are their bisectors,
// at pi/16, 3 pi/16, 5 pi/16 and 7 pi/16 from the real axis.
constexpr float kCos16 = 0.98078528040323043f;    // cos(pi/16)
constexpr float kSin16 = 0.19509032201612826f;    // sin(pi/16)
constexpr float kCos316 = 0.83146961230254524f;   // cos(3 pi/16)
constexpr float kSin316 = 0.55557023301960218f;   // sin(3 pi/16)

__device__ __forceinline__ void bisector_k16(float a, float b, float& yr, float& yi) {
    const float ax = fabsf(a), ay = fabsf(b);
    const bool big = ax >= ay;
    const float lo = big ? ay : ax, hi = big ? ax : ay;
    const bool inner = lo > 0.41421356237309505f * hi;   // tan(pi/8)
    const float p = inner ? kCos316 : kCos16, q = inner ? kSin316 : kSin16;
    yr = copysignf(big ? p : q, a);
    yi = copysignf(big ? q : p, b);
}

// Turn of the direction for the K = 8 and 16 forms: c e^{-i pi/K}.
template <int KS>
__device__ __forceinline__ void turn_direction(float& cr, float& ci) {
    constexpr float co = KS == 8 ? kCos8 : kCos16, si = KS == 8 ? kSin8 : kSin16;
    const float r = cr, i = ci;
    cr = fmaf(r, co, i * si);
    ci = fmaf(i, co, -(r * si));
}

// Factor on c for the real part of w, matching the pre-scaled K = 3 quantiser.
__host__ __device__ constexpr float re_prescale(int KS) {
    return KS == 3 ? 1.7320508075688772f : 1.0f;
}

// The same closed forms in FP64 for the rescore (any K through label_f64
// and an FP64 root table).  Away from decision boundaries they agree with
// label_f64; on a boundary (measure zero) either neighbour may be taken.
template <int KS>
__device__ __forceinline__ void nearest_root64(double wr, double wi, int K, const double2* roots,
                                               double& zr, double& zi) {
    if constexpr (KS == 2) {
        zr = wr >= 0.0 ? 1.0 : -1.0;
        zi = 0.0;
    } else if constexpr (KS == 3) {
        const bool k0 = fabs(wi) <= wr * 1.7320508075688772;
        zr = k0 ? 1.0 : -0.5;
        zi = k0 ? 0.0 : copysign(0.86602540378443865, wi);
    } else if constexpr (KS == 4) {
        const bool horiz = fabs(wr) >= fabs(wi);
        zr = horiz ? copysign(1.0, wr) : 0.0;
        zi = horiz ? 0.0 : copysign(1.0, wi);
    } else if constexpr (KS == 8) {
        const double ax = fabs(wr), ay = fabs(wi);
        const double t = 0.41421356237309505;         // tan(pi/8)
        const bool h = ay <= t * ax, v = ax <= t * ay;
        const double d = 0.70710678118654752;
        zr = copysign(h ? 1.0 : (v ? 0.0 : d), wr);
        zi = copysign(h ? 0.0 : (v ? 1.0 : d), wi);
    } else if constexpr (KS == 16) {
        const double ax = fabs(wr), ay = fabs(wi);
        const bool sw = ay > ax;
        const double lo = sw ? ax : ay, hi = sw ? ay : ax;
        const bool b1 = lo > 0.19891236737965800 * hi;  // tan(pi/16)
        const bool b2 = lo > 0.66817863791929892 * hi;  // tan(3 pi/16)
        const double cc = b2 ? 0.70710678118654752 : (b1 ? 0.92387953251128676 : 1.0);
        const double ss = b2 ? 0.70710678118654752 : (b1 ? 0.38268343236508977 : 0.0);
        zr = copysign(sw ? ss : cc, wr);
        zi = copysign(sw ? cc : ss, wi);
    } else {
        const double2 t = roots[label_f64(wr, wi, K)];
        zr = t.x;
        zi = t.y;
    }
}

// Closed-form specialisation available for this K (0: generic).
__host__ __device__ constexpr int k_special(int K) {
    return (K == 2 || K == 3 || K == 4 || K == 8 || K == 16) ? K : 0;
}

}  // namespace lrqo
