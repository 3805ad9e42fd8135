// Scans and a stable LSD radix sort (8-bit digits) for wave64 gfx950.
// Used to group samples by tree node and to order CSR entries.
#include "common.h"

namespace fsg {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int64_t kScanTile = kScanThreads * kScanItems;

int64_t scan_partials(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <typename T>
__global__ __launch_bounds__(256) void scan_reduce_kernel(const T* __restrict__ in, int64_t n, T* __restrict__ partials) {
    __shared__ T red[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// Exclusive scan of the partials in one block of 1024 threads.
template <typename T>
__global__ __launch_bounds__(1024) void scan_partials_kernel(T* partials, int64_t nb, T* total) {
    __shared__ T sums[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    T s = 0;
    for (int64_t k = 0; k < per; ++k)
        if (b0 + k < nb) s += partials[b0 + k];
    sums[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        T v = ((int)threadIdx.x >= off) ? sums[threadIdx.x - off] : (T)0;
        __syncthreads();
        sums[threadIdx.x] += v;
        __syncthreads();
    }
    T run = (threadIdx.x == 0) ? (T)0 : sums[threadIdx.x - 1];
    for (int64_t k = 0; k < per; ++k) {
        if (b0 + k < nb) {
            const T v = partials[b0 + k];
            partials[b0 + k] = run;
            run += v;
        }
    }
    if (threadIdx.x == 1023) *total = sums[1023];
}

template <typename T>
__global__ __launch_bounds__(256) void scan_apply_kernel(const T* in, T* out, int64_t n, const T* __restrict__ partials) {
    __shared__ T sums[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : (T)0;
        s += v[k];
    }
    sums[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        T t = ((int)threadIdx.x >= off) ? sums[threadIdx.x - off] : (T)0;
        __syncthreads();
        sums[threadIdx.x] += t;
        __syncthreads();
    }
    T run = partials[blockIdx.x] + ((threadIdx.x == 0) ? (T)0 : sums[threadIdx.x - 1]);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

template <typename T>
static hipError_t exclusive_scan(const T* in, T* out, int64_t n, T* total, T* partials, hipStream_t st) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipMemsetAsync(total, 0, sizeof(T), st);
        return hipGetLastError();
    }
    scan_reduce_kernel<T><<<(unsigned)nb, kScanThreads, 0, st>>>(in, n, partials);
    scan_partials_kernel<T><<<1, 1024, 0, st>>>(partials, nb, total);
    scan_apply_kernel<T><<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, n, partials);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total, int64_t* partials,
                                     hipStream_t st) {
    return exclusive_scan<int64_t>(in, out, n, total, partials, st);
}

hipError_t launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                                     uint32_t* partials, hipStream_t st) {
    return exclusive_scan<uint32_t>(in, out, n, total, partials, st);
}

// ---------------------------------------------------------------------------
// Radix sort.  A block sorts a tile of 4096 keys; its 4 waves each own 1024
// consecutive keys, handled 64 at a time in order, so ranks are stable.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortTile = 4096;
constexpr int kWaveKeys = kSortTile / 4;

int64_t sort_hist_elems(int64_t n) { return 256 * ((n + kSortTile - 1) / kSortTile) + 1; }

template <typename K>
__global__ __launch_bounds__(256) void radix_hist_kernel(const K* __restrict__ keys, int64_t n, int shift,
                                                       uint32_t* __restrict__ hist, int64_t nb) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int k = threadIdx.x; k < kSortTile; k += kSortThreads) {
        const int64_t idx = base + k;
        if (idx < n) atomicAdd(&cnt[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__device__ __forceinline__ uint64_t peers_of(uint32_t digit, bool active) {
    uint64_t peers = __ballot(active);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (digit >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// The tile is first ordered by digit in LDS (stable), then written out in
// that order: the keys of one digit leave a tile as one contiguous run, so
// the global writes are whole runs instead of 4-byte scatters.
template <typename K>
__global__ __launch_bounds__(256) void radix_scatter_kernel(const K* __restrict__ keys, const int32_t* __restrict__ vals,
                                                          K* __restrict__ keys_out, int32_t* __restrict__ vals_out,
                                                          int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                          int64_t nb) {
    __shared__ uint32_t wcount[4][256];
    __shared__ uint32_t wbase[4][256];   // tile-local position of each wave's next key of a digit
    __shared__ uint32_t dstart[256];     // tile-local start of each digit
    __shared__ uint32_t gstart[256];     // global start of each digit's run of this tile
    __shared__ K lk[kSortTile];
    __shared__ int32_t lv[kSortTile];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = threadIdx.x; k < 4 * 256; k += kSortThreads) (&wcount[0][0])[k] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    const int32_t tile_n = (int32_t)min((int64_t)kSortTile, n - tile0);
    const int64_t wstart = tile0 + (int64_t)wv * kWaveKeys;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // pass 1: per-wave digit counts
    for (int c = 0; c < kWaveKeys; c += 64) {
        const int64_t idx = wstart + c + lane;
        const bool active = idx < n;
        const uint32_t digit = active ? ((uint32_t)(keys[idx] >> shift) & 255u) : 0u;
        const uint64_t peers = peers_of(digit, active);
        if (active && (63 - __clzll(peers)) == lane) wcount[wv][digit] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // tile-local digit starts (exclusive scan over the digits of the tile's
    // counts), then each wave's base within its digit
    {
        const int dg = threadIdx.x;  // 256 threads, one per digit
        const uint32_t tot = wcount[0][dg] + wcount[1][dg] + wcount[2][dg] + wcount[3][dg];
        dstart[dg] = tot;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const uint32_t v = (dg >= off) ? dstart[dg - off] : 0u;
            __syncthreads();
            dstart[dg] += v;
            __syncthreads();
        }
        const uint32_t ex = dstart[dg] - tot;
        __syncthreads();
        dstart[dg] = ex;
        uint32_t run = ex;
        for (int w = 0; w < 4; ++w) {
            wbase[w][dg] = run;
            run += wcount[w][dg];
        }
        gstart[dg] = offs[(int64_t)dg * nb + blockIdx.x];
    }
    __syncthreads();
    // pass 2: stable placement in LDS
    for (int c = 0; c < kWaveKeys; c += 64) {
        const int64_t idx = wstart + c + lane;
        const bool active = idx < n;
        K key = 0;
        int32_t val = 0;
        if (active) {
            key = keys[idx];
            val = vals[idx];
        }
        const uint32_t digit = (uint32_t)(key >> shift) & 255u;
        const uint64_t peers = peers_of(digit, active);
        if (active) {
            const uint32_t pos = wbase[wv][digit] + (uint32_t)__popcll(peers & below);
            lk[pos] = key;
            lv[pos] = val;
        }
        __builtin_amdgcn_wave_barrier();
        if (active && (63 - __clzll(peers)) == lane) wbase[wv][digit] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // runs out in tile order
    for (int32_t p = threadIdx.x; p < tile_n; p += kSortThreads) {
        const K key = lk[p];
        const uint32_t digit = (uint32_t)(key >> shift) & 255u;
        const uint32_t g = gstart[digit] + ((uint32_t)p - dstart[digit]);
        keys_out[g] = key;
        vals_out[g] = lv[p];
    }
}

template <typename K>
static hipError_t radix_sort(K* keys, int32_t* vals, int64_t n, int bits, const SortBufs& b, hipStream_t st) {
    if (n <= 1 || bits <= 0) return hipSuccess;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t hn = 256 * nb;
    K* src_k = keys;
    int32_t* src_v = vals;
    K* dst_k = (K*)b.keys_tmp;
    int32_t* dst_v = b.vals_tmp;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8, ++passes) {
        radix_hist_kernel<K><<<(unsigned)nb, kSortThreads, 0, st>>>(src_k, n, shift, b.hist, nb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_exclusive_scan_u32(b.hist, b.hist, hn, b.hist + hn, b.partials, st);
        if (e != hipSuccess) return e;
        radix_scatter_kernel<K><<<(unsigned)nb, kSortThreads, 0, st>>>(src_k, src_v, dst_k, dst_v, n, shift, b.hist, nb);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        K* tk = src_k; src_k = dst_k; dst_k = tk;
        int32_t* tv = src_v; src_v = dst_v; dst_v = tv;
    }
    if (passes & 1) {
        hipError_t e = hipMemcpyAsync(keys, src_k, n * sizeof(K), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, src_v, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t radix_sort_u32(uint32_t* keys, int32_t* vals, int64_t n, int bits, const SortBufs& b, hipStream_t st) {
    return radix_sort<uint32_t>(keys, vals, n, bits, b, st);
}

hipError_t radix_sort_u64(uint64_t* keys, int32_t* vals, int64_t n, int bits, const SortBufs& b, hipStream_t st) {
    return radix_sort<uint64_t>(keys, vals, n, bits, b, st);
}

}  // namespace fsg
