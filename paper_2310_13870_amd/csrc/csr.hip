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
        // 16-byte loads where the rows allow, the same summation order
        const double D = kernel_distance(a.kind, xi, xj, a.d, (a.d & 3) == 0 && (((uintptr_t)a.X) & 15) == 0);
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

// ---------------------------------------------------------------------------
// Row-sorted construction (no global sort).  Row i of the entry array holds
// L slots for i's own samples (INT32_MAX where a sample gave no edge) followed
// by one slot per sample (j, i) of another point: the incoming entries are
// counted with atomics, scanned and filled in arbitrary order, then each row
// is sorted and deduplicated by one wave (bitonic sort in registers for rows
// of <= 64 slots, in LDS up to kRowSortMax); a scan of the unique counts gives
// row_ptr, and a last pass writes columns and weights.  Rows longer than
// kRowSortMax are counted in *n_long and left empty; the caller then builds
// the CSR by the global sort.  Row i starts at L i + in_off[i].
// ---------------------------------------------------------------------------
__global__ void csr_zero_kernel(uint32_t* cnt, uint32_t* fillc, int64_t n, int32_t* n_long) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) {
        cnt[i] = 0;
        fillc[i] = 0;
    }
    if (i == 0) *n_long = 0;
}

__global__ void csr_count_kernel(const int32_t* __restrict__ nbr, int64_t n, int32_t L, uint32_t* __restrict__ cnt) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n * L) return;
    const int64_t i = s / L;
    const int32_t y = nbr[s];
    if (y >= 0 && y < n && y != i) atomicAdd(&cnt[y], 1u);
}

__global__ void csr_scatter_kernel(const int32_t* __restrict__ nbr, int64_t n, int32_t L,
                                   const uint32_t* __restrict__ in_off, uint32_t* __restrict__ fillc,
                                   int32_t* __restrict__ ent) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n * L) return;
    const int64_t i = s / L;
    const int32_t y = nbr[s];
    const bool ok = y >= 0 && y < n && y != i;
    ent[(int64_t)in_off[i] + s] = ok ? y : INT32_MAX;  // own slot l of row i: L i + in_off[i] + l
    if (ok) ent[(int64_t)L * y + in_off[y] + L + atomicAdd(&fillc[y], 1u)] = (int32_t)i;
}

constexpr int kRowSortMax = 2048;

__global__ __launch_bounds__(256) void csr_row_sort_kernel(const uint32_t* __restrict__ in_off, int32_t L,
                                                           int32_t* __restrict__ ent, int64_t* __restrict__ uniq,
                                                           int64_t n, int32_t* __restrict__ n_long) {
    __shared__ int32_t buf_all[4][kRowSortMax];
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (int64_t)__builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    if (row >= n) return;  // uniform per wave
    const int64_t b = (int64_t)L * row + in_off[row];
    const int32_t len = (int32_t)(L + in_off[row + 1] - in_off[row]);
    int32_t* seg = ent + b;
    if (len <= 64) {
        int32_t v = lane < len ? seg[lane] : INT32_MAX;
        for (int k = 2; k <= 64; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                const int32_t o = __shfl_xor(v, j);
                const bool up = (lane & k) == 0;
                const bool lower = (lane & j) == 0;
                v = (lower == up) ? min(v, o) : max(v, o);
            }
        }
        const int32_t prev = __shfl_up(v, 1);
        const bool keep = v != INT32_MAX && (lane == 0 || prev != v);
        const uint64_t mask = __ballot(keep);
        if (keep) seg[__popcll(mask & ((1ull << lane) - 1ull))] = v;
        if (lane == 0) uniq[row] = __popcll(mask);
        return;
    }
    if (len > kRowSortMax) {
        if (lane == 0) {
            atomicAdd(n_long, 1);
            uniq[row] = 0;
        }
        return;
    }
    // LDS bitonic sort of the row padded to a power of two; a wave's own LDS
    // accesses complete in order, so no barrier beyond the wave is needed
    int32_t* buf = buf_all[threadIdx.x >> 6];
    int32_t P = 128;
    while (P < len) P <<= 1;
    for (int32_t k = lane; k < P; k += 64) buf[k] = (k < len) ? seg[k] : INT32_MAX;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int32_t k = 2; k <= P; k <<= 1) {
        for (int32_t j = k >> 1; j > 0; j >>= 1) {
            for (int32_t t = lane; t < P / 2; t += 64) {
                const int32_t lo = 2 * t - (t & (j - 1));  // lo has bit j clear
                const int32_t hi = lo + j;
                const int32_t x = buf[lo], y = buf[hi];
                const bool up = (lo & k) == 0;
                if ((x > y) == up) {
                    buf[lo] = y;
                    buf[hi] = x;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    int32_t count = 0;
    for (int32_t base = 0; base < len; base += 64) {
        const int32_t k = base + lane;
        const int32_t v = (k < len) ? buf[k] : INT32_MAX;
        const int32_t pv = (k > 0 && k < len) ? buf[k - 1] : INT32_MIN;
        const bool keep = v != INT32_MAX && (k == 0 || pv != v);
        const uint64_t mask = __ballot(keep);
        if (keep) seg[count + __popcll(mask & ((1ull << lane) - 1ull))] = v;
        count += __popcll(mask);
    }
    if (lane == 0) uniq[row] = count;
}

// Columns and weights of row i from its sorted unique entries; the kernel
// value uses the difference form in FP64 summed in feature order, so both
// directions of an edge get bit-identical weights.
// With a row order, XCD x (workgroups b with b % kXcds == x; the grid is a
// multiple of kXcds) takes the x-th eighth of the order, four rows per
// workgroup, so that each L2 holds the rows of the clusters it works on.
__global__ __launch_bounds__(256) void csr_row_fill_kernel(CsrRowArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t per_xcd = gridDim.x / kXcds;
    const int64_t lb = a.row_order ? (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds : blockIdx.x;
    const int64_t r = lb * 4 + (int64_t)__builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    if (r >= a.n) return;
    const int64_t row = a.row_order ? a.row_order[r] : r;
    const int64_t rp = a.row_ptr[row];
    const int64_t cnt = a.row_ptr[row + 1] - rp;
    const int32_t* seg = a.ent + (int64_t)a.L * row + a.in_off[row];
    const float* xi = a.X + row * a.d;
    const bool vec = (a.d & 3) == 0 && (((uintptr_t)a.X) & 15) == 0;
    for (int64_t k = lane; k < cnt; k += 64) {
        const int64_t j = seg[k];
        const float* xj = a.X + j * a.d;
        const double D = kernel_distance(a.kind, xi, xj, a.d, vec);
        const double kv = exp2_fp64(-a.s * D);
        const double pi = fmin((double)a.L * kv / a.deg[row], 1.0);
        const double pj = fmin((double)a.L * kv / a.deg[j], 1.0);
        const double ph = pi + pj - pi * pj;
        if (rp + k < a.cap) {
            a.col[rp + k] = (int32_t)j;
            a.w[rp + k] = (float)(kv / ph);
        }
    }
}

hipError_t launch_csr_rows(const CsrRowArgs& a, const int32_t* nbr, int32_t L, uint32_t* cnt, uint32_t* fillc,
                           uint32_t* off, uint32_t* off_partials, int64_t* uniq, int64_t* uniq_partials,
                           int32_t* n_long, hipStream_t st) {
    const int64_t n = a.n, ns = n * (int64_t)L;
    hipError_t e;
    csr_zero_kernel<<<(unsigned)((n + 1 + 255) / 256), 256, 0, st>>>(cnt, fillc, n, n_long);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    csr_count_kernel<<<(unsigned)((ns + 255) / 256 + 1), 256, 0, st>>>(nbr, n, L, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_exclusive_scan_u32(cnt, off, n, off + n, off_partials, st)) != hipSuccess) return e;
    csr_scatter_kernel<<<(unsigned)((ns + 255) / 256 + 1), 256, 0, st>>>(nbr, n, L, off, fillc, a.ent);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned row_blocks = (unsigned)((n + 1 + 3) / 4);
    csr_row_sort_kernel<<<row_blocks, 256, 0, st>>>(off, L, a.ent, uniq, n, n_long);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_exclusive_scan_i64(uniq, a.row_ptr, n, a.row_ptr + n, uniq_partials, st)) != hipSuccess) return e;
    const unsigned fill_blocks = a.row_order ? (row_blocks + kXcds - 1) / kXcds * kXcds : row_blocks;
    csr_row_fill_kernel<<<fill_blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace fsg
