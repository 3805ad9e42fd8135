// Point-set preparation of the precision mode: the BF16 hi/lo split operands
// of the data side (index order) and of the query side (pivot order), -|x|^2/2
// in FP32, distance bounds and the query order from pivot points, the largest
// norm; and small fill kernels the orchestration uses.
#include "common.h"
#include "device.h"

namespace fsg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

int split_steps(int d) { return (3 * d + 31) / 32; }

// K steps the filter kernel is built for, per feature-step class (the split
// operands of smaller d are zero-padded up to it).
int filter_steps(int D4) {
    switch (D4) {
        case 1: return 1;
        case 2: return 1;
        case 4: return 2;
        case 8: return 3;
        case 16: return 6;
        case 32: return 12;
        default: return -1;
    }
}

__global__ void fill_i64_kernel(int64_t* p, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st) {
    fill_i64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

__global__ void add_i64_kernel(int64_t* p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p += v;
}

hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t st) {
    add_i64_kernel<<<1, 64, 0, st>>>(p, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Point-set preparation for the filter.
// ---------------------------------------------------------------------------
// Split fragments in the operand layout of v_mfma_f32_16x16x32_bf16: lane l
// holds 8 consecutive K entries 8(l/16).. of row 16b + l%16.  Data rows are
// [hi(x), lo(x), hi(x), 0...], query rows [hi(q), hi(q), lo(q), 0...]; their
// contraction is hi.hi + hi.lo + lo.hi.  xa = -|x|^2/2 in FP32.
__device__ __forceinline__ bf16x8_t split_fragment(const float* __restrict__ X, int64_t row, int32_t d, int32_t kb,
                                                   int32_t lane, bool query) {
    bf16x8_t v;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int32_t k = kb * 32 + (lane >> 4) * 8 + t;
        __bf16 b = (__bf16)0.0f;
        if (row >= 0 && k < 3 * d) {
            const int32_t part = k / d;  // 0, 1, 2
            const float x = X[row * d + (k - part * d)];
            const __bf16 hi = (__bf16)x;
            const __bf16 lo = (__bf16)(x - (float)hi);
            b = (part == (query ? 2 : 1)) ? lo : hi;
        }
        v[t] = b;
    }
    return v;
}

// data-side fragments of the points in index order, and xa
__global__ void prep_split_kernel(const float* __restrict__ X, const double* __restrict__ norm, int64_t n, int32_t d,
                                  int32_t KB, int64_t total, bf16x8_t* __restrict__ Xb, float* __restrict__ xa,
                                  int64_t n_pad) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n_pad) xa[idx] = (idx < n) ? (float)(-0.5 * norm[idx]) : 0.0f;
    if (idx >= total) return;
    const int64_t per_blk = (int64_t)KB * 64;
    const int64_t blk = idx / per_blk;
    const int32_t rem = (int32_t)(idx - blk * per_blk);
    const int32_t kb = rem >> 6, lane = rem & 63;
    const int64_t row = blk * 16 + (lane & 15);
    Xb[idx] = split_fragment(X, row < n ? row : -1, d, kb, lane, false);
}

// query-side fragments in entry order: row e holds point order[e] (zero rows
// past the last entry), so that a tile's operands are contiguous
__global__ void prep_query_split_kernel(const float* __restrict__ X, const int32_t* __restrict__ order, int64_t n,
                                        int32_t d, int32_t KB, int64_t total, bf16x8_t* __restrict__ Qb) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t per_blk = (int64_t)KB * 64;
    const int64_t blk = idx / per_blk;
    const int32_t rem = (int32_t)(idx - blk * per_blk);
    const int32_t kb = rem >> 6, lane = rem & 63;
    const int64_t e = blk * 16 + (lane & 15);
    Qb[idx] = split_fragment(X, e < n ? (int64_t)order[e] : -1, d, kb, lane, true);
}

// data-side fragments and -|x|^2/2 in entry (pivot) order: the operands of
// the pruned keep-mask scan (zero rows past the last entry)
__global__ void prep_split_order_kernel(const float* __restrict__ X, const double* __restrict__ norm,
                                        const int32_t* __restrict__ order, int64_t n, int32_t d, int32_t KB,
                                        int64_t rows, int64_t total, bf16x8_t* __restrict__ Xbp,
                                        float* __restrict__ xap) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < rows) xap[idx] = (idx < n) ? (float)(-0.5 * norm[order[idx]]) : 0.0f;
    if (idx >= total) return;
    const int64_t per_blk = (int64_t)KB * 64;
    const int64_t blk = idx / per_blk;
    const int32_t rem = (int32_t)(idx - blk * per_blk);
    const int32_t kb = rem >> 6, lane = rem & 63;
    const int64_t e = blk * 16 + (lane & 15);
    Xbp[idx] = split_fragment(X, e < n ? (int64_t)order[e] : -1, d, kb, lane, false);
}

// dmin[i] = an upper bound on min_{j != i} |x_i - x_j|^2 over P pivot points
// (indices floor(p n / P)); label[i] = the nearest pivot.  The squared
// distances come from FP32 norms and cross terms, |x|^2 + |p|^2 - 2 x.p (one
// multiply-add per feature), each sum in four partial sums: the cross term's
// error is below (d/4 + 3) 2^-24 sum |x_t p_t| <= (d/4 + 3) 2^-24 (|x|^2 +
// |p|^2) / 2, the norms' likewise, and the three roundings that combine them
// add 3 2^-24 (|x|^2 + |p|^2), so adding (d + 32) 2^-24 (|x|^2 + |p|^2) (at
// least twice their sum) gives an upper bound; the FP32 rounding of that sum
// is covered by a factor 1 + 2^-20 on the result.
template <int DMAX>
__global__ __launch_bounds__(256) void pivot_kernel(const float* __restrict__ X, int64_t n, int32_t d, int32_t P,
                                                    double* __restrict__ dmin, uint32_t* __restrict__ label,
                                                    int32_t* __restrict__ ids) {
    constexpr int CH = 64;  // pivots staged per round
    __shared__ float piv[CH * DMAX];
    __shared__ float pnorm[CH];
    __shared__ int64_t pidx[CH];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    float xi[DMAX];
#pragma unroll
    for (int t = 0; t < DMAX; ++t) xi[t] = (valid && t < d) ? X[i * d + t] : 0.0f;
    auto sum4 = [](const float (&a)[4]) { return (a[0] + a[1]) + (a[2] + a[3]); };
    float xn;
    {
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < DMAX; ++t) acc[t & 3] = __builtin_fmaf(xi[t], xi[t], acc[t & 3]);
        xn = sum4(acc);
    }
    const float slack = 1.0f + (float)(d + 32) * 0x1p-24f;  // (|x|^2 + |p|^2) times this, minus 2 x.p
    float best = __builtin_inff();
    uint32_t arg = 0;
    for (int32_t p0 = 0; p0 < P; p0 += CH) {
        const int32_t pc = min(CH, P - p0);
        __syncthreads();
        if ((int32_t)threadIdx.x < pc) pidx[threadIdx.x] = ((int64_t)(p0 + threadIdx.x) * n) / P;
        __syncthreads();
        for (int32_t k = threadIdx.x; k < pc * DMAX; k += blockDim.x) {
            const int32_t pp = k / DMAX, t = k - pp * DMAX;
            piv[k] = (t < d) ? X[pidx[pp] * d + t] : 0.0f;
        }
        __syncthreads();
        if ((int32_t)threadIdx.x < pc) {
            const float* pj = piv + threadIdx.x * DMAX;
            float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < DMAX; ++t) acc[t & 3] = __builtin_fmaf(pj[t], pj[t], acc[t & 3]);
            pnorm[threadIdx.x] = sum4(acc);
        }
        __syncthreads();
        for (int32_t pp = 0; pp < pc; ++pp) {
            const float* pj = piv + pp * DMAX;
            float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < DMAX; ++t) acc[t & 3] = __builtin_fmaf(xi[t], pj[t], acc[t & 3]);
            const float ub = __builtin_fmaf(-2.0f, sum4(acc), (xn + pnorm[pp]) * slack);
            if (pidx[pp] != i && ub < best) {
                best = ub;
                arg = (uint32_t)(p0 + pp);
            }
        }
    }
    if (!valid) return;
    dmin[i] = (double)best * (1.0 + 0x1p-20);
    label[i] = arg;
    ids[i] = (int32_t)i;
}

// Largest |x|^2 in two stages: block maxima, then one block over them.
constexpr int kMaxNormBlocks = 512;

__global__ __launch_bounds__(256) void max_norm_kernel(const double* __restrict__ norm, int64_t n,
                                                       double* __restrict__ part) {
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmax(m, norm[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void max_norm_final_kernel(const double* __restrict__ part, int32_t np,
                                                             double* __restrict__ out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int32_t i = threadIdx.x; i < np; i += 256) m = fmax(m, part[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = __builtin_sqrt(red[0]);
}

hipError_t launch_prep_split(const float* X, const double* norm, int64_t n, int32_t d, int32_t KB, int64_t n_pad,
                             void* Xb, float* xa, hipStream_t st) {
    const int64_t total = (n_pad / 16) * KB * 64;
    const int64_t threads = total > n_pad ? total : n_pad;
    prep_split_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, st>>>(X, norm, n, d, KB, total, (bf16x8_t*)Xb, xa,
                                                                         n_pad);
    return hipGetLastError();
}

hipError_t launch_prep_query_split(const float* X, const int32_t* order, int64_t n, int32_t d, int32_t KB,
                                   int64_t rows, void* Qb, hipStream_t st) {
    if (rows % 16 != 0 || rows < n) return hipErrorInvalidValue;
    const int64_t total = (rows / 16) * KB * 64;
    if (total == 0) return hipSuccess;
    prep_query_split_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(X, order, n, d, KB, total,
                                                                             (bf16x8_t*)Qb);
    return hipGetLastError();
}

hipError_t launch_prep_split_order(const float* X, const double* norm, const int32_t* order, int64_t n, int32_t d,
                                   int32_t KB, int64_t rows, void* Xbp, float* xap, hipStream_t st) {
    if (rows % 16 != 0 || rows < n) return hipErrorInvalidValue;
    const int64_t total = (rows / 16) * KB * 64;
    const int64_t threads = total > rows ? total : rows;
    if (threads == 0) return hipSuccess;
    prep_split_order_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, st>>>(X, norm, order, n, d, KB, rows, total,
                                                                               (bf16x8_t*)Xbp, xap);
    return hipGetLastError();
}

hipError_t launch_pivots(const float* X, int64_t n, int32_t d, int32_t P, double* dmin, uint32_t* label, int32_t* ids,
                         hipStream_t st) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (d <= 4) pivot_kernel<4><<<blocks, 256, 0, st>>>(X, n, d, P, dmin, label, ids);
    else if (d <= 8) pivot_kernel<8><<<blocks, 256, 0, st>>>(X, n, d, P, dmin, label, ids);
    else if (d <= 16) pivot_kernel<16><<<blocks, 256, 0, st>>>(X, n, d, P, dmin, label, ids);
    else if (d <= 32) pivot_kernel<32><<<blocks, 256, 0, st>>>(X, n, d, P, dmin, label, ids);
    else if (d <= 64) pivot_kernel<64><<<blocks, 256, 0, st>>>(X, n, d, P, dmin, label, ids);
    else if (d <= 128) pivot_kernel<128><<<blocks, 256, 0, st>>>(X, n, d, P, dmin, label, ids);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

int max_norm_parts(int64_t n) {
    const int64_t b = (n + 2047) / 2048;
    return (int)(b < 1 ? 1 : (b > kMaxNormBlocks ? kMaxNormBlocks : b));
}

hipError_t launch_max_norm(const double* norm, int64_t n, double* part, double* out, hipStream_t st) {
    const int np = max_norm_parts(n);
    max_norm_kernel<<<np, 256, 0, st>>>(norm, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    max_norm_final_kernel<<<1, 256, 0, st>>>(part, np, out);
    return hipGetLastError();
}

__global__ void inverse_order_kernel(const int32_t* __restrict__ order, int64_t n, int32_t* __restrict__ inv) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) inv[order[e]] = (int32_t)e;
}

hipError_t launch_inverse_order(const int32_t* order, int64_t n, int32_t* inv, hipStream_t st) {
    if (n == 0) return hipSuccess;
    inverse_order_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(order, n, inv);
    return hipGetLastError();
}

}  // namespace fsg
