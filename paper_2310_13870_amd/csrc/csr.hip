// Reweighting and symmetric CSR (hot-path step "reweight + CSR"; Algorithm 2
// after the sampling loop).  Every sample (i, y) emits the directed entries
// (i,y) and (y,i) as keys row*n + col; a radix sort orders them, duplicates
// are dropped (E is a set), and each remaining entry gets
//   w = k/p_hat,  p_hat = p_i + p_j - p_i p_j,  p_i = min(L k/deg_i, 1).
// Both directions of an edge compute the same w (the same operations on the
// same operands), so the matrix is exactly symmetric.
#include "common.h"
#include "device.h"

namespace fsg {

__global__ void csr_emit_kernel(const int32_t* nbr, int64_t n, int32_t L, uint64_t* keys, int32_t* vals) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n * L) return;
    const int64_t i = s / L;
    const int32_t y = nbr[s];
    const uint64_t sentinel = (uint64_t)n * (uint64_t)n;
    if (y >= 0 && y < n && y != i) {
        keys[2 * s] = (uint64_t)i * (uint64_t)n + (uint64_t)y;
        keys[2 * s + 1] = (uint64_t)y * (uint64_t)n + (uint64_t)i;
    } else {
        keys[2 * s] = sentinel;
        keys[2 * s + 1] = sentinel;
    }
    vals[2 * s] = (int32_t)(2 * s);
    vals[2 * s + 1] = (int32_t)(2 * s + 1);
}

hipError_t launch_csr_emit(const int32_t* nbr, int64_t n, int32_t L, uint64_t* keys, int32_t* vals, hipStream_t st) {
    const int64_t ns = n * L;
    csr_emit_kernel<<<(unsigned)((ns + 255) / 256 + 1), 256, 0, st>>>(nbr, n, L, keys, vals);
    return hipGetLastError();
}

__global__ void csr_flags_kernel(const uint64_t* keys, int64_t m, uint64_t sentinel, int64_t* flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    const uint64_t k = keys[p];
    flags[p] = (k != sentinel && (p == 0 || keys[p - 1] != k)) ? 1 : 0;
}

hipError_t launch_csr_flags(const uint64_t* keys, int64_t m, uint64_t sentinel, int64_t* flags, hipStream_t st) {
    csr_flags_kernel<<<(unsigned)((m + 255) / 256 + 1), 256, 0, st>>>(keys, m, sentinel, flags);
    return hipGetLastError();
}

// One thread per sorted position p in [0, m]: unique entries write their
// column and weight; the first entry of each row (or the end) fills the row
// pointers of the rows it closes.
__global__ void csr_fill_kernel(CsrArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > a.m) return;
    const uint64_t sentinel = (uint64_t)a.n * (uint64_t)a.n;
    const uint64_t key = (p < a.m) ? a.keys[p] : sentinel;
    const int64_t cur_row = (key == sentinel) ? a.n : (int64_t)(key / (uint64_t)a.n);
    const uint64_t pkey = (p == 0) ? sentinel : a.keys[p - 1];
    const int64_t prev_row = (p == 0) ? -1 : ((pkey == sentinel) ? a.n : (int64_t)(pkey / (uint64_t)a.n));
    const int64_t here = a.pos[p];  // unique entries before p
    if (cur_row > prev_row) {
        for (int64_t r = prev_row + 1; r <= cur_row; ++r) a.row_ptr[r] = here;
    }
    if (p < a.m && a.flags[p] && here < a.cap) {
        const int64_t i = cur_row;
        const int64_t j = (int64_t)(key - (uint64_t)i * (uint64_t)a.n);
        const float* xi = a.X + i * a.d;
        const float* xj = a.X + j * a.d;
        double D = 0.0;
        if ((a.d & 3) == 0 && (((uintptr_t)a.X) & 15) == 0) {
            // 16-byte loads; the same summation order as the scalar loop
            const float4* vi = (const float4*)xi;
            const float4* vj = (const float4*)xj;
            for (int32_t t4 = 0; t4 < (a.d >> 2); ++t4) {
                const float4 p = vi[t4], q = vj[t4];
                double df = (double)p.x - (double)q.x;
                D = __builtin_fma(df, df, D);
                df = (double)p.y - (double)q.y;
                D = __builtin_fma(df, df, D);
                df = (double)p.z - (double)q.z;
                D = __builtin_fma(df, df, D);
                df = (double)p.w - (double)q.w;
                D = __builtin_fma(df, df, D);
            }
        } else {
            for (int32_t t = 0; t < a.d; ++t) {
                const double df = (double)xi[t] - (double)xj[t];
                D = __builtin_fma(df, df, D);
            }
        }
        const double k = exp2_fp64(-a.s * D);
        const double pi = fmin((double)a.L * k / a.deg[i], 1.0);
        const double pj = fmin((double)a.L * k / a.deg[j], 1.0);
        const double ph = pi + pj - pi * pj;
        a.col[here] = (int32_t)j;
        a.w[here] = (float)(k / ph);
    }
}

hipError_t launch_csr_fill(const CsrArgs& a, hipStream_t st) {
    csr_fill_kernel<<<(unsigned)((a.m + 1 + 255) / 256 + 1), 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace fsg
