// Hot-path step "prep": FP64 matrix-core operand rows, squared norms, the
// integer slices of the precision mode's exact recompute, and the node
// boundaries of one level of the index-order partition tree.
#include "common.h"
#include "device.h"

namespace fsg {

__global__ void prep_fragments_kernel(const float* __restrict__ X, int64_t n, int32_t d, int32_t D4, int64_t total,
                                      double* __restrict__ Xp) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    // position within the row: (kk / 2) * 8 + g * 2 + kk % 2 (D4 >= 2), g (D4 = 1)
    const int64_t per_row = (int64_t)D4 * 4;
    const int64_t row = idx / per_row;
    const int32_t rem = (int32_t)(idx - row * per_row);
    int32_t g, kk;
    if (D4 == 1) {
        g = rem;
        kk = 0;
    } else {
        g = (rem & 7) >> 1;
        kk = ((rem >> 3) << 1) | (rem & 1);
    }
    const int32_t col = kk * 4 + g;
    Xp[idx] = (row < n && col < d) ? (double)X[row * d + col] : 0.0;
}

// Squared norms in FP64, each summed in coordinate order.  A block stages
// the rows it owns through LDS with coalesced loads (a thread per row reading
// its row directly would touch a different cache line per lane and load).
constexpr int kNormStage = 16384;  // floats staged per block (64 KB)

__global__ __launch_bounds__(256) void prep_norms_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                         int64_t n_pad, int32_t rows, double* __restrict__ norm) {
    __shared__ float xs[kNormStage + 256];  // rows padded to d + 1 floats (no bank conflicts)
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    const int64_t r1 = min(r0 + rows, n);
    const int64_t cnt = (r1 > r0) ? (r1 - r0) * d : 0;
    const float* src = X + r0 * d;
    for (int64_t k = threadIdx.x; k < cnt; k += blockDim.x) {
        const int64_t r = k / d, t = k - r * d;
        xs[r * (d + 1) + t] = src[k];
    }
    __syncthreads();
    const int64_t row = r0 + threadIdx.x;
    if ((int32_t)threadIdx.x >= rows || row >= n_pad) return;
    double s = 0.0;
    if (row < n) {
        const float* x = xs + threadIdx.x * (d + 1);
        for (int32_t t = 0; t < d; ++t) {
            const double v = (double)x[t];
            s = __builtin_fma(v, v, s);
        }
    }
    norm[row] = s;
}

hipError_t launch_prep(const float* X, int64_t n, int32_t d, int32_t D4, int64_t n_pad, double* Xp, double* norm,
                       hipStream_t st) {
    const int64_t total = n_pad * D4 * 4;
    prep_fragments_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(X, n, d, D4, total, Xp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // rows per block: 256, fewer where 256 rows of d + 1 floats would not fit the stage
    int32_t rows = kNormStage / (d + 1);
    if (rows > 256) rows = 256;
    if (rows < 1) return hipErrorInvalidValue;
    prep_norms_kernel<<<(unsigned)((n_pad + rows - 1) / rows), 256, 0, st>>>(X, n, d, n_pad, rows, norm);
    return hipGetLastError();
}

// Integer slices (layout in common.h): one wave per point, a lane per
// coordinate.  The scaled coordinate times 2^56 is an integer below 2^55 in
// magnitude (exact in FP64 up to the rounding of coordinates below 2^-56 of
// the scale); its digits come off the low end in 64-bit integers.
__global__ __launch_bounds__(256) void prep_slices_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                                          int64_t n_pad, int8_t* __restrict__ Xs,
                                                          int32_t* __restrict__ xe) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= n_pad) return;
    const float x = (p < n && lane < d) ? X[p * d + lane] : 0.0f;
    float m = __builtin_fabsf(x);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) m = __builtin_fmaxf(m, __shfl_xor(m, off));
    int e = 0;
    if (m > 0.0f) {
        // m = f 2^e with f in [0.5, 1): m 2^-(e+1) < 0.498 unless f >= 0.996
        const float f = __builtin_frexpf(m, &e);
        e += (f >= 0.996f) ? 2 : 1;
    }
    int64_t v = (int64_t)__builtin_rint(__builtin_ldexp((double)x, 56 - e));
    int8_t* row = Xs + p * kSliceRow;
#pragma unroll
    for (int a = kSlices - 1; a >= 0; --a) {
        const int64_t c = ((v + 128) & 255) - 128;
        v = (v - c) >> 8;
        row[64 * a + lane] = (int8_t)c;
    }
    if (lane == 0) xe[p] = e;
}

hipError_t launch_prep_slices(const float* X, int64_t n, int32_t d, int64_t n_pad, int8_t* Xs, int32_t* xe,
                              hipStream_t st) {
    if (d > 64) return hipErrorInvalidValue;
    prep_slices_kernel<<<(unsigned)((n_pad + 3) / 4), 256, 0, st>>>(X, n, d, n_pad, Xs, xe);
    return hipGetLastError();
}

// out[v] = first index of node v at depth `level` (v < 2^level), out[2^level] = n.
// Valid while every node of the level exists, i.e. level <= floor(log2 n).
__global__ void level_bounds_kernel(int64_t n, int32_t level, int32_t* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t count = (int64_t)1 << level;
    if (v > count) return;
    if (v == count) {
        out[v] = (int32_t)n;
        return;
    }
    int64_t lo = 0, size = n;
    for (int32_t t = level - 1; t >= 0; --t) {
        const int64_t half = size >> 1;
        if ((v >> t) & 1) {
            lo += half;
            size -= half;
        } else {
            size = half;
        }
    }
    out[v] = (int32_t)lo;
}

hipError_t launch_level_bounds(int64_t n, int level, int32_t* out, hipStream_t st) {
    const int64_t count = ((int64_t)1 << level) + 1;
    level_bounds_kernel<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(n, level, out);
    return hipGetLastError();
}

}  // namespace fsg
