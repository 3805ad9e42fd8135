// Device-side helpers shared by the kernels of libfsg.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsg {

// ---------------------------------------------------------------------------
// 2^a in FP64 for the Gaussian kernel.  a = n + f with n = rint(a) and
// |f| <= 1/2; 2^f = e^(f ln 2) is summed as its Taylor series to degree 11,
// whose remainder is below (ln2/2)^12/12! < 7e-15 relative, and the result is
// scaled by 2^n with ldexp (exact, gradual underflow to 0 below 2^-1074).
// ---------------------------------------------------------------------------
constexpr double kLn2 = 0.693147180559945309417232121458176568;
constexpr double kLog2e = 1.442695040888963407359924681001892137;
constexpr double taylor_coef(int k) {
    double v = 1.0;
    for (int i = 1; i <= k; ++i) v = v * kLn2 / (double)i;
    return v;
}

__device__ __forceinline__ double exp2_fp64(double a) {
    a = __builtin_fmax(a, -2000.0);  // below 2^-1074 anyway; keeps (int)n defined
    double n = __builtin_rint(a);
    double f = a - n;
    double p = taylor_coef(11);
    p = __builtin_fma(p, f, taylor_coef(10));
    p = __builtin_fma(p, f, taylor_coef(9));
    p = __builtin_fma(p, f, taylor_coef(8));
    p = __builtin_fma(p, f, taylor_coef(7));
    p = __builtin_fma(p, f, taylor_coef(6));
    p = __builtin_fma(p, f, taylor_coef(5));
    p = __builtin_fma(p, f, taylor_coef(4));
    p = __builtin_fma(p, f, taylor_coef(3));
    p = __builtin_fma(p, f, taylor_coef(2));
    p = __builtin_fma(p, f, taylor_coef(1));
    p = __builtin_fma(p, f, 1.0);
    return __builtin_ldexp(p, (int)n);
}

// ---------------------------------------------------------------------------
// 2^(a/256) in FP64 with a table (the KDE kernels, where the exponential is
// most of the vector work).  a = 256 e + j + r with m = rint(a), j = m mod 256,
// e = floor(m / 256) and |r| <= 1/2: 2^(a/256) = 2^e 2^(j/256) e^(r ln2/256).
// tab[j] = 2^(j/256) rounded to FP64 (kExp2Table, copied to LDS by the
// caller); e^x - 1 for |x| = |r ln2/256| <= 1.36e-3 is its Taylor series to
// degree 4, whose remainder is below 4e-17 relative; the result is
// tab[j] + tab[j] q scaled by 2^e with ldexp (exact, gradual underflow).
// Arguments below -2000 * 256 give 0, as does -inf.
// ---------------------------------------------------------------------------
constexpr double tab_coef(int k) {
    double v = 1.0;
    for (int i = 1; i <= k; ++i) v = v * (kLn2 / 256.0) / (double)i;
    return v;
}

// The two halves of exp2_256_tab, for callers that issue several table reads
// before the first result is needed: the split gives m = rint(a) (a clamped)
// and r = a - m; the join takes t = tab[m & 255].
__device__ __forceinline__ int32_t exp2_256_split(double a, double* r) {
    a = __builtin_fmax(a, -512000.0);
    const double m = __builtin_rint(a);
    *r = a - m;  // exact: |r| <= 1/2
    return (int32_t)m;
}

__device__ __forceinline__ double exp2_256_join(double t, double r, int32_t mi) {
    double q = __builtin_fma(tab_coef(4), r, tab_coef(3));
    q = __builtin_fma(q, r, tab_coef(2));
    q = __builtin_fma(q, r, tab_coef(1));
    q *= r;
    return __builtin_ldexp(__builtin_fma(t, q, t), mi >> 8);
}

__device__ __forceinline__ double exp2_256_tab(double a, const double* tab) {
    double r;
    const int32_t mi = exp2_256_split(a, &r);
    return exp2_256_join(tab[mi & 255], r, mi);
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 64x64->128 multiplies; the key advances by the Weyl increments between
// rounds.  u(seed, i, l, level) = (word[level % 4] >> 11) * 2^-53 of the block
// with key (seed, 0) and counter (i, l, level / 4, 0).
// ---------------------------------------------------------------------------
struct PhiloxWords {
    uint64_t w[4];
};

__device__ __forceinline__ PhiloxWords philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                      uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t p0hi = __umul64hi(M0, c0), p0lo = M0 * c0;
        const uint64_t p1hi = __umul64hi(M1, c2), p1lo = M1 * c2;
        const uint64_t n0 = p1hi ^ c1 ^ k0;
        const uint64_t n2 = p0hi ^ c3 ^ k1;
        c0 = n0;
        c1 = p1lo;
        c2 = n2;
        c3 = p0lo;
    }
    PhiloxWords o;
    o.w[0] = c0;
    o.w[1] = c1;
    o.w[2] = c2;
    o.w[3] = c3;
    return o;
}

__device__ __forceinline__ double word_to_uniform(uint64_t w) {
    return (double)(w >> 11) * (1.0 / 9007199254740992.0);
}

// Uniform source for one sample: caches the Philox block of the current group
// of four levels.
struct SampleUniforms {
    uint64_t seed, i, l;
    int32_t group;
    PhiloxWords words;
    __device__ void init(uint64_t seed_, uint64_t i_, uint64_t l_) {
        seed = seed_;
        i = i_;
        l = l_;
        group = -1;
    }
    __device__ double at(int32_t level) {
        const int32_t g = level >> 2;
        if (g != group) {
            words = philox4x64_10(i, l, (uint64_t)g, 0, seed, 0);
            group = g;
        }
        const int k = level & 3;  // explicit selects keep the words in registers
        const uint64_t w = (k == 0) ? words.w[0] : (k == 1) ? words.w[1] : (k == 2) ? words.w[2] : words.w[3];
        return word_to_uniform(w);
    }
};

// A value the whole wave agrees on, kept in a scalar register: loop bounds
// and bin indices derived from LDS or vector loads would otherwise be
// treated as per-lane values.
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// The compiler's lane-write intrinsic (v_writelane_b32): lane `lane` of the
// result is `val` (both uniform), the other lanes keep `old`.
__device__ uint32_t writelane_u32(uint32_t val, uint32_t lane, uint32_t old) __asm("llvm.amdgcn.writelane.i32");

// Split of node [a,b): the left half holds floor((b-a)/2) points.
__device__ __forceinline__ int32_t tree_split(int32_t a, int32_t b) { return a + ((b - a) >> 1); }

// Kernel kinds (fsg_kernel): what enters the exponent, times gamma.
constexpr int kKindGaussian = 0;     // ||x - y||_2^2
constexpr int kKindExponential = 1;  // ||x - y||_2
constexpr int kKindLaplacian = 2;    // ||x - y||_1

// The exponent's distance of kernel `kind` between two FP32 points from their
// coordinate differences (exact in FP64), summed in coordinate order:
// squared for the Gaussian kernel, its square root for the exponential one,
// absolute values for the Laplacian one.  vec: 16-byte loads (d % 4 == 0,
// aligned rows), the same summation order.
__device__ __forceinline__ double kernel_distance(int32_t kind, const float* xi, const float* xj, int32_t d,
                                                  bool vec) {
    double D = 0.0;
    if (kind == kKindLaplacian) {
        for (int32_t t = 0; t < d; ++t) D += __builtin_fabs((double)xi[t] - (double)xj[t]);
        return D;
    }
    if (vec) {
        // eight 16-byte pieces of each row are loaded before any is used (the
        // sums still run in feature order)
        const float4* vi = (const float4*)xi;
        const float4* vj = (const float4*)xj;
        const int32_t n4 = d >> 2;
        for (int32_t c = 0; c < n4; c += 8) {
            float4 p[8], q[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                p[u] = (c + u < n4) ? vi[c + u] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                q[u] = (c + u < n4) ? vj[c + u] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (c + u < n4) {
                    double df = (double)p[u].x - (double)q[u].x;
                    D = __builtin_fma(df, df, D);
                    df = (double)p[u].y - (double)q[u].y;
                    D = __builtin_fma(df, df, D);
                    df = (double)p[u].z - (double)q[u].z;
                    D = __builtin_fma(df, df, D);
                    df = (double)p[u].w - (double)q[u].w;
                    D = __builtin_fma(df, df, D);
                }
            }
        }
    } else {
        for (int32_t t = 0; t < d; ++t) {
            const double df = (double)xi[t] - (double)xj[t];
            D = __builtin_fma(df, df, D);
        }
    }
    return (kind == kKindExponential) ? __builtin_sqrt(D) : D;
}

// Precision mode: the largest squared distance a pair may have and still
// carry more than e^-Delta of its row's largest term, given dm >= the row's
// smallest squared distance.  Gaussian (exponent gamma D): dm + Delta/gamma;
// exponential (exponent gamma sqrt(D)): (sqrt(dm) + Delta/gamma)^2.
__host__ __device__ inline double keep_dist2(int32_t kind, double dm, double margin_z, double gamma) {
    if (kind == kKindExponential) {
        const double r = __builtin_sqrt(dm) + margin_z / gamma;
        return r * r;
    }
    return dm + margin_z / gamma;
}

}  // namespace fsg
