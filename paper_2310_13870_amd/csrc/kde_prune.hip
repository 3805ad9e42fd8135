// Lossless tile pruning ahead of the keep-mask scan of the precision mode.
//
// The points are grouped into cells by their nearest pivot (the pivot order
// the query tiles already use).  For a cell c with pivot p_c and a radius r_c
// (an upper bound on |x - p_c| over its members) and a query q, the triangle
// inequality gives |q - x| >= |q - p_c| - r_c for every member x.  The keep
// test of the scan can pass for a pair only if its squared distance is at
// most
//     T_q = K_q + 4 E_q + 2^-20 |theta_q|,  K_q = dmin_q (1 + 1e-6) + Delta / gamma
// (the threshold of the test -- for the exponential kernel K_q =
// (sqrt(dmin_q (1 + 1e-6)) + Delta / gamma)^2 --, its error bound E_q counted
// on both sides of the comparison, and the FP32 rounding of theta_q; theta_q
// differs from the test's by the rounding of the FP64 terms, which the
// 2^-20 |theta_q| term covers), so a (query tile, cell)
// pair with |q - p_c| > r_c + sqrt(T_q) for all queries of the tile cannot
// keep any column: the scan skips it, and the kept set -- hence every mass --
// is the same as with the full scan.  This is the first pruning step towards
// the sub-quadratic KDE regime the paper relies on (Section 1 and Theorem 1
// use an approximate KDE; here the pruning is exact).
//
// Steps per call: (1) a plan kernel marks the cells each 64-query tile may
// keep columns of; (2) the cells of each group of tiles are merged into runs
// of 16-column blocks of the data in pivot order, cut into work items; (3)
// the keep-mask kernel scans those items on data operands in pivot order
// (kde_mask.hip); (4) a conversion kernel writes each tile's keep bits back
// in index order, which the exact pass reads.
#include "common.h"
#include "device.h"

namespace fsg {

// the smallest float >= v (v finite, >= 0): one step up when the rounding
// went down (the next float above a non-negative one has the next bit pattern)
__device__ __forceinline__ float float_up(double v) {
    float f = (float)v;
    if ((double)f < v) f = __int_as_float(__float_as_int(f) + 1);
    return f;
}

// ---------------------------------------------------------------------------
// Pivot chain (once per point set): new labels for the pivots such that
// consecutive labels are near each other -- a greedy nearest-neighbour chain
// from pivot 0 over the pivots' squared distances (FP32, truncated to their
// upper 16 bits, which keeps their order).  Cells are laid out in label
// order, so neighbouring cells are close and a 64-query tile that spans two
// cells stays within one cluster.  Only the layout depends on the chain,
// never a result.
// ---------------------------------------------------------------------------
constexpr int kMaxPivots = 256;

__global__ __launch_bounds__(256) void pivot_dist_kernel(const float* __restrict__ X, int64_t n, int32_t d, int32_t P,
                                                         uint16_t* __restrict__ D16) {
    const int32_t a = blockIdx.x, b = threadIdx.x;
    if (b >= P) return;
    const float* pa = X + ((int64_t)a * n / P) * d;
    const float* pb = X + ((int64_t)b * n / P) * d;
    float s = 0.0f;
    for (int32_t t = 0; t < d; ++t) {
        const float u = pa[t] - pb[t];
        s = __builtin_fmaf(u, u, s);
    }
    D16[a * P + b] = (uint16_t)(__float_as_uint(s) >> 16);
}

// one wave: lane l holds candidates l, l + 64, l + 128, l + 192
__global__ __launch_bounds__(64) void pivot_chain_kernel(const uint16_t* __restrict__ D16, int32_t P, int64_t n,
                                                         int32_t* __restrict__ rank, int32_t* __restrict__ cell_pivot) {
    __shared__ __attribute__((aligned(16))) uint16_t dl[kMaxPivots * kMaxPivots];
    const int lane = threadIdx.x;
    {
        // 16 bytes per lane and load, eight loads in flight (D16 is 256-byte
        // aligned workspace)
        const int32_t nv = (P * P) / 8;
        const uint4* src = (const uint4*)D16;
        uint4* dst = (uint4*)dl;
        for (int32_t k0 = 0; k0 < nv; k0 += 64 * 8) {
            uint4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t k = k0 + 64 * u + lane;
                v[u] = (k < nv) ? src[k] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t k = k0 + 64 * u + lane;
                if (k < nv) dst[k] = v[u];
            }
        }
        for (int32_t k = 8 * nv + lane; k < P * P; k += 64) dl[k] = D16[k];
    }
    __syncthreads();
    uint32_t visited = (lane == 0) ? 1u : 0u;
    int32_t cur = 0;
    if (lane == 0) {
        rank[0] = 0;
        cell_pivot[0] = 0;
    }
    for (int32_t s = 1; s < P; ++s) {
        // key = distance bits << 8 | candidate: the smallest is the nearest
        // unvisited pivot (ties to the lower index)
        uint32_t key = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int32_t j = lane + 64 * i;
            if (j < P && !((visited >> i) & 1u)) key = min(key, ((uint32_t)dl[cur * P + j] << 8) | (uint32_t)j);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) key = min(key, (uint32_t)__shfl_xor((int)key, off));
        const int32_t next = (int32_t)(key & 255u);
        if (lane == 0) {
            rank[next] = s;
            cell_pivot[s] = (int32_t)((int64_t)next * n / P);
        }
        if ((next & 63) == lane) visited |= 1u << (next >> 6);
        cur = next;
    }
}

__global__ void relabel_kernel(uint32_t* __restrict__ label, int64_t n, const int32_t* __restrict__ rank) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) label[i] = (uint32_t)rank[label[i]];
}

hipError_t launch_pivot_chain(const float* X, int64_t n, int32_t d, int32_t P, uint16_t* D16, int32_t* rank,
                              int32_t* cell_pivot, uint32_t* label, hipStream_t st) {
    if (P < 1 || P > kMaxPivots) return hipErrorInvalidValue;
    pivot_dist_kernel<<<(unsigned)P, 256, 0, st>>>(X, n, d, P, D16);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    pivot_chain_kernel<<<1, 64, 0, st>>>(D16, P, n, rank, cell_pivot);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    relabel_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(label, n, rank);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cell geometry (once per point set): the pivot's squared norm in FP32 (four
// partial sums, as the plan kernel forms norms) and an upper bound on the
// cell's radius.  dmin[i] is an upper bound on |x_i - p_label(i)|^2 (the
// pivot kernel's distance to the nearest pivot, whose point is
// cell_pivot[c]), so the largest dmin over a cell's members bounds its
// squared radius.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cell_geometry_kernel(const float* __restrict__ X, int32_t d,
                                                            const double* __restrict__ dmin,
                                                            const int32_t* __restrict__ order,
                                                            const int32_t* __restrict__ cell_start,
                                                            const int32_t* __restrict__ cell_pivot,
                                                            float* __restrict__ pnorm, float* __restrict__ prad) {
    __shared__ double red[256];
    const int32_t c = blockIdx.x;
    const int32_t cs = cell_start[c], ce = cell_start[c + 1];
    double m = 0.0;
    for (int32_t e = cs + (int32_t)threadIdx.x; e < ce; e += 256) m = fmax(m, dmin[order[e]]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    prad[c] = float_up(__builtin_sqrt(red[0]) * (1.0 + 0x1p-40));
    const float* pc = X + (int64_t)cell_pivot[c] * d;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int32_t t = 0; t < d; ++t) acc[t & 3] = __builtin_fmaf(pc[t], pc[t], acc[t & 3]);
    pnorm[c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

hipError_t launch_cell_geometry(const float* X, int32_t d, int32_t P, const double* dmin, const int32_t* order,
                                const int32_t* cell_start, const int32_t* cell_pivot, float* pnorm, float* prad,
                                hipStream_t st) {
    if (P < 1) return hipErrorInvalidValue;
    cell_geometry_kernel<<<(unsigned)P, 256, 0, st>>>(X, d, dmin, order, cell_start, cell_pivot, pnorm, prad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// (1) Plan: bit c of surv[t] is set when some query of tile t may keep a
// column of cell c.  One wave per tile, a lane per query entry; the pivot
// coordinates are shared through LDS.  The squared distance to
// the pivot is bounded from below from FP32 norms and cross terms (four
// partial sums each): their errors and the roundings that combine them stay
// below (d + 32) 2^-24 (|q|^2 + |p|^2) (as in the pivot kernel), and the last
// fused multiply-add adds at most 2^-24 of the same magnitude, so subtracting
// (d + 40) 2^-24 (|q|^2 + |p|^2) gives a lower bound D_lb.  A keep is
// possible iff D_lb <= (r_c + sqrt(T_q))^2, the right side rounded up.
// ---------------------------------------------------------------------------
template <int DMAX>
__global__ __launch_bounds__(256) void prune_plan_kernel(PruneArgs a) {
    // pivots staged in LDS 32 at a time (one word of the cell set), zero
    // padded to DMAX features so that the dot products need no guards
    constexpr int CH = 32;
    __shared__ float piv[CH][DMAX];
    __shared__ float pn[CH], pr[CH];
    __shared__ int32_t live[CH];
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + uniform((int32_t)(threadIdx.x >> 6));
    const bool tile_ok = t < a.n_tiles;  // wave-uniform; every wave takes part in the staging
    const int64_t e = t * kTileQ + lane;
    const bool valid = tile_ok && e < a.n;
    const int32_t d = a.d;
    const int32_t p = valid ? a.order[e] : 0;
    float q[DMAX];
#pragma unroll
    for (int k = 0; k < DMAX; ++k) q[k] = (valid && k < d) ? a.X[(int64_t)p * d + k] : 0.0f;
    float qn;
    {
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < DMAX; ++k) acc[k & 3] = __builtin_fmaf(q[k], q[k], acc[k & 3]);
        qn = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
    // square root of the largest squared distance a kept pair can have
    float sT = 0.0f;
    if (valid) {
        const double xmax = *a.xmax;
        const double nq = a.qnorm[p];
        const double dm = a.dmin[p] * (1.0 + 1e-6);
        const double err = a.eps * (__builtin_sqrt(nq) * xmax + 0.5 * xmax * xmax);
        const double Tk = keep_dist2(a.kind, dm, a.margin_z, a.gamma);
        const double th = 0.5 * nq - 0.5 * Tk - err;
        double T = Tk + 4.0 * err + 0x1p-20 * __builtin_fabs(th);
        T *= 1.0 + 0x1p-30;
        sT = float_up(__builtin_sqrt(T) * (1.0 + 0x1p-40));
    }
    const float sl = (float)(d + 40) * 0x1p-24f;
    const int32_t P = a.P;
    for (int32_t c0 = 0; c0 < P; c0 += CH) {
        const int32_t nc = min(CH, P - c0);
        __syncthreads();
        for (int32_t k = threadIdx.x; k < CH * DMAX; k += 256) {
            const int32_t cc = k / DMAX, kk = k - cc * DMAX;
            piv[cc][kk] = (cc < nc && kk < d) ? a.X[(int64_t)a.cell_pivot[c0 + cc] * d + kk] : 0.0f;
        }
        if ((int32_t)threadIdx.x < CH) {
            const int32_t c = c0 + threadIdx.x;
            const bool ok = (int32_t)threadIdx.x < nc;
            pn[threadIdx.x] = ok ? a.pnorm[c] : 0.0f;
            pr[threadIdx.x] = ok ? a.prad[c] : 0.0f;
            live[threadIdx.x] = ok && a.cell_start[c + 1] > a.cell_start[c];
        }
        __syncthreads();
        if (!tile_ok) continue;
        uint32_t word = 0;
        for (int32_t cc = 0; cc < nc; ++cc) {
            if (!live[cc]) continue;  // an empty cell (uniform)
            float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int k = 0; k < DMAX; ++k) acc[k & 3] = __builtin_fmaf(q[k], piv[cc][k], acc[k & 3]);
            const float dot = (acc[0] + acc[1]) + (acc[2] + acc[3]);
            const float s = qn + pn[cc];
            const float dlb = __builtin_fmaf(-sl, s, __builtin_fmaf(-2.0f, dot, s));
            const float lim = pr[cc] + sT;
            const bool need = valid && dlb <= lim * lim * (1.0f + 0x1p-20f);
            if (__ballot(need) != 0) word |= 1u << cc;
        }
        if (lane == 0) a.surv[t * a.words + (c0 >> 5)] = word;
    }
}

// ---------------------------------------------------------------------------
// (2) Work items of the pruned scan, chunk-major: the data blocks (pivot
// order) are cut into chunks of chunk_blocks blocks, and for every (chunk,
// group of TP tiles) the cells the group may keep columns of are merged into
// runs of blocks within the chunk (cells sharing or touching a block merge):
// items {first tile, first block, end block}.  Items of one chunk are
// consecutive, so waves that run together scan the same data -- the groups
// of one cluster share its cells -- and the XCD split below keeps each L2 on
// a few chunks at a time.  Counting and filling take one thread per (chunk,
// group); the count pass also adds the scanned (column, tile) pairs to the
// filter statistics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void group_cells(const PruneArgs& a, int64_t g, uint32_t (&w)[8], int64_t* tl) {
    const int64_t t0 = g * a.TP;
    *tl = min((int64_t)a.TP, a.n_tiles - t0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint32_t v = 0;
        if (k < a.words)
            for (int64_t t = t0; t < t0 + *tl; ++t) v |= a.surv[t * a.words + k];
        w[k] = v;
    }
}

// runs of blocks of group g's cells within block range [lo, hi), in order:
// fn(b0, b1) for each
template <typename F>
__device__ __forceinline__ void group_runs(const PruneArgs& a, const uint32_t (&w)[8], int64_t lo, int64_t hi, F fn) {
    // the first cell that ends after column 16 lo (cells are in pivot order)
    int32_t c = 0, cb = a.P;
    while (c < cb) {
        const int32_t m = (c + cb) >> 1;
        if ((int64_t)a.cell_start[m + 1] <= 16 * lo) c = m + 1; else cb = m;
    }
    int64_t rb0 = -1, rb1 = -1;
    for (; c < a.P && (int64_t)a.cell_start[c] < 16 * hi; ++c) {
        if (!((w[c >> 5] >> (c & 31)) & 1u)) continue;
        const int32_t cs = a.cell_start[c], ce = a.cell_start[c + 1];
        if (ce <= cs) continue;
        const int64_t b0 = max((int64_t)(cs >> 4), lo), b1 = min(((int64_t)ce + 15) >> 4, hi);
        if (b1 <= b0) continue;
        if (rb0 >= 0 && b0 <= rb1) {
            rb1 = max(rb1, b1);
        } else {
            if (rb0 >= 0) fn(rb0, rb1);
            rb0 = b0;
            rb1 = b1;
        }
    }
    if (rb0 >= 0) fn(rb0, rb1);
}

__global__ void prune_count_kernel(PruneArgs a) {
    const int64_t kg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = a.n_chunks * a.n_groups;
    int64_t items = 0, blocks = 0, tl = 0;
    if (kg < total) {
        const int64_t k = kg / a.n_groups, g = kg - k * a.n_groups;
        uint32_t w[8];
        group_cells(a, g, w, &tl);
        const int64_t lo = k * a.chunk_blocks, hi = min(lo + a.chunk_blocks, a.n_blocks_p);
        group_runs(a, w, lo, hi, [&](int64_t b0, int64_t b1) {
            ++items;
            blocks += b1 - b0;
        });
    }
    if (kg <= total) {
        a.counts[kg] = items;
        a.bcounts[kg] = blocks;
    }
    // scanned (column, tile) pairs: one atomic per wave
    unsigned long long sc = (unsigned long long)(blocks * 16 * tl);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sc += (unsigned long long)__shfl_xor((long long)sc, off);
    if ((threadIdx.x & 63) == 0 && sc > 0 && a.scanned) atomicAdd((unsigned long long*)a.scanned, sc);
}

__global__ void prune_fill_kernel(PruneArgs a) {
    const int64_t kg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (kg >= a.n_chunks * a.n_groups) return;
    const int64_t k = kg / a.n_groups, g = kg - k * a.n_groups;
    uint32_t w[8];
    int64_t tl;
    group_cells(a, g, w, &tl);
    int32_t* out = a.items + 3 * a.offsets[kg];
    const int64_t lo = k * a.chunk_blocks, hi = min(lo + a.chunk_blocks, a.n_blocks_p);
    group_runs(a, w, lo, hi, [&](int64_t b0, int64_t b1) {
        out[0] = (int32_t)(g * a.TP);
        out[1] = (int32_t)b0;
        out[2] = (int32_t)b1;
        out += 3;
    });
}

// XCD segments of the item list: segment x holds the items of the (chunk,
// group) pairs whose blocks start in [x B / X, (x + 1) B / X), B the total
// blocks, X = kXcds -- equal scan work per L2, consecutive chunks in each
__global__ void prune_xcd_kernel(PruneArgs a) {
    const int x = threadIdx.x;
    if (x > kXcds) return;
    const int64_t total = a.n_chunks * a.n_groups;
    const int64_t B = a.boffsets[total];
    if (x == 0 || x == kXcds) {
        a.xseg[x] = (x == 0) ? 0 : a.offsets[total];
        return;
    }
    const int64_t target = (B * x) / kXcds;
    int64_t lo = 0, hi = total;  // the first pair whose block offset reaches target
    while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (a.boffsets[m] < target) lo = m + 1; else hi = m;
    }
    a.xseg[x] = a.offsets[lo];
}

hipError_t launch_prune_plan(const PruneArgs& a, hipStream_t st) {
    if (a.words < 1 || a.words > 8 || a.P > 32 * a.words) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((a.n_tiles + 3) / 4);
    if (blocks == 0) return hipSuccess;
    const int d = a.d;
    if (d <= 4) prune_plan_kernel<4><<<blocks, 256, 0, st>>>(a);
    else if (d <= 8) prune_plan_kernel<8><<<blocks, 256, 0, st>>>(a);
    else if (d <= 16) prune_plan_kernel<16><<<blocks, 256, 0, st>>>(a);
    else if (d <= 32) prune_plan_kernel<32><<<blocks, 256, 0, st>>>(a);
    else if (d <= 64) prune_plan_kernel<64><<<blocks, 256, 0, st>>>(a);
    else if (d <= 128) prune_plan_kernel<128><<<blocks, 256, 0, st>>>(a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// counts, bcounts [n_chunks n_groups + 1] -> offsets, boffsets (exclusive
// scans; the last entry is the total), the items, then the XCD segments
hipError_t launch_prune_items(const PruneArgs& a, int64_t* partials, hipStream_t st) {
    const int64_t total = a.n_chunks * a.n_groups;
    prune_count_kernel<<<(unsigned)((total + 1 + 255) / 256), 256, 0, st>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan_i64(a.counts, a.offsets, total + 1, a.total, partials, st);
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan_i64(a.bcounts, a.boffsets, total + 1, a.total + 1, partials, st);
    if (e != hipSuccess) return e;
    prune_fill_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    prune_xcd_kernel<<<1, 64, 0, st>>>(a);
    return hipGetLastError();
}

// an upper bound on the items of a pruned scan: each (chunk, group) pair
// splits its runs at most at the chunk's cell starts, so a group has at most
// one item per surviving cell plus one per chunk
int64_t prune_max_items(int64_t n_groups, int32_t P, int64_t n_chunks) { return n_groups * ((int64_t)P + n_chunks + 1); }

// ---------------------------------------------------------------------------
// (4) Keep bits back to index order.  One workgroup per tile: the bits of the
// tile's scanned blocks (pivot order, position e = point order[e]) are set in
// a bitmap of columns in LDS, a window of 2^20 columns at a time, which is
// then written out whole, so that every block of the tile's index-order row is
// written (blocks without kept columns get 0).  A block's 16 point indices are
// loaded together (four 16-byte loads) before its bits are walked.
// ---------------------------------------------------------------------------
constexpr int kConvThreads = 512;
constexpr int64_t kConvWindow = (int64_t)1 << 20;  // columns per LDS window (128 KB)

__global__ __launch_bounds__(kConvThreads) void mask_to_index_kernel(PruneArgs a, const uint16_t* __restrict__ maskp,
                                                                    int64_t n_blocks_p, uint16_t* __restrict__ mask,
                                                                    int64_t n_blocks) {
    __shared__ uint32_t bits[kConvWindow / 32];
    const int64_t t = blockIdx.x;
    const int64_t g = t / a.TP;
    uint32_t w[8];
    int64_t tl;
    group_cells(a, g, w, &tl);
    const uint16_t* mrow = maskp + t * n_blocks_p;
    const int64_t n_cols = n_blocks * 16;
    for (int64_t w0 = 0; w0 < n_cols; w0 += kConvWindow) {
        const int32_t wwords = (int32_t)((min(kConvWindow, n_cols - w0) + 31) / 32);
        for (int32_t k = threadIdx.x; k < wwords; k += kConvThreads) bits[k] = 0u;
        __syncthreads();
        // the group's scanned blocks are those of its cells: a wave per cell,
        // its lanes over the cell's blocks (a block shared with a neighbour
        // cell may be read twice; the bits it sets are the same)
        for (int32_t c = (int32_t)(threadIdx.x >> 6); c < a.P; c += kConvThreads / 64) {
            if (!((w[c >> 5] >> (c & 31)) & 1u)) continue;
            const int64_t b1 = ((int64_t)a.cell_start[c + 1] + 15) >> 4;
            // four blocks per lane at a time: their masks and point indices
            // are all loaded before the first is used
            for (int64_t bq = (a.cell_start[c] >> 4) + (threadIdx.x & 63); bq < b1; bq += 256) {
                uint32_t m[4];
                int4 o[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t b = bq + 64 * u;
                    m[u] = (b < b1) ? (uint32_t)mrow[b] : 0u;
                    // positions 16 b .. 16 b + 15 exist: the order array is
                    // padded to whole blocks (the padding's bits are never set)
                    const int4* ob = (const int4*)(a.order + 16 * (b < b1 ? b : bq));
#pragma unroll
                    for (int q = 0; q < 4; ++q) o[u][q] = ob[q];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (m[u] == 0u) continue;
                    const int32_t pts[16] = {o[u][0].x, o[u][0].y, o[u][0].z, o[u][0].w, o[u][1].x, o[u][1].y,
                                             o[u][1].z, o[u][1].w, o[u][2].x, o[u][2].y, o[u][2].z, o[u][2].w,
                                             o[u][3].x, o[u][3].y, o[u][3].z, o[u][3].w};
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        if ((m[u] >> k) & 1u) {
                            const int64_t j = (int64_t)pts[k] - w0;
                            if (j >= 0 && j < kConvWindow) atomicOr(&bits[j >> 5], 1u << (j & 31));
                        }
                    }
                }
            }
        }
        __syncthreads();
        // the window's blocks of the tile's row: block k of the window is half
        // k % 2 of word k / 2
        const int64_t kb0 = w0 / 16;
        const int64_t kbn = min(kConvWindow / 16, n_blocks - kb0);
        uint16_t* out = mask + t * n_blocks + kb0;
        int64_t k4 = 0;  // blocks written four at a time (8-byte stores) where aligned
        if (((t * n_blocks + kb0) & 3) == 0) {
            k4 = kbn & ~(int64_t)3;
            uint2* o2 = (uint2*)out;
            for (int64_t k = threadIdx.x; k < k4 / 4; k += kConvThreads)
                o2[k] = make_uint2(bits[2 * k], bits[2 * k + 1]);
        }
        for (int64_t k = k4 + threadIdx.x; k < kbn; k += kConvThreads)
            out[k] = (uint16_t)(bits[k >> 1] >> (16 * (k & 1)));
        __syncthreads();
    }
}

hipError_t launch_mask_to_index(const PruneArgs& a, const uint16_t* maskp, int64_t n_blocks_p, uint16_t* mask,
                                int64_t n_blocks, hipStream_t st) {
    if (a.n_tiles == 0) return hipSuccess;
    mask_to_index_kernel<<<(unsigned)a.n_tiles, kConvThreads, 0, st>>>(a, maskp, n_blocks_p, mask, n_blocks);
    return hipGetLastError();
}

}  // namespace fsg
