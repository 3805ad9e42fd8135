// Segmented Gaussian (and exponential-kernel) KDE over tree bins on the FP64
// matrix cores (hot-path
// step "segmented KDE"; the two KDEs of Algorithm 1 and the degree KDE of
// Algorithm 2, eq. (1) of Section 2.2 over index ranges).
//
// A wave owns one work item: up to 16*RQ query entries of one segment and a
// run of that segment's bins (consecutive index ranges of the data).  It
// streams the data in 16-column blocks.  Per block and query block, D4
// v_mfma_f64_16x16x4f64 give the cross terms x_j . q (data as the A operand,
// so lane l holds data rows l/16 + 4i of query row l%16); the epilogue forms
// the exponent -gamma log2(e) (|q|^2 + |x|^2 - 2 x.q) in FP64, evaluates 2^a
// in FP64, removes the self term, and accumulates per lane.  When a bin
// boundary is crossed the 4 partial sums of each query row are combined with
// two cross-lane steps and written once: no atomics, fixed order, so results
// are bit-reproducible.
#include <type_traits>

#include "common.h"
#include "device.h"
#include "kde_epilogue.h"

namespace fsg {

// MULTI: items of many point sets in one launch; segment sg.job selects the
// arguments of its point set from a.jobs.
// KIND: the Gaussian kernel, or the exponential one (the same cross terms,
// the square root of the distance in the exponent).
template <int D4, int RQ, bool MULTI, int KIND = kKindGaussian>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(D4 <= 16 ? 2 : 1))) void kde_bins_kernel(KdeArgs a) {
    // the table exponential where two waves share a SIMD (d <= 64), whose LDS
    // reads the other wave hides; the polynomial one at one wave per SIMD
    constexpr bool kTab = D4 <= 16;
    constexpr double kScale = kTab ? 256.0 : 1.0;  // exponent terms scaled for exp2_256_tab
    __shared__ int32_t win_all[4][kBinWindow];
    __shared__ double exp_tab[kTab ? 256 : 1];
    if (kTab) load_exp2_table(exp_tab);
    const int lane = threadIdx.x & 63;
    int32_t* win = win_all[threadIdx.x >> 6];
    const int64_t wave = (int64_t)blockIdx.x * 4 + uniform((int32_t)(threadIdx.x >> 6));  // wave-uniform
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    const int32_t n_items = *a.n_items;
    const int grp = lane >> 4;  // data row group inside a 16-column block
    const int r = lane & 15;    // query row inside a query block

    for (int64_t it = wave; it < n_items; it += n_waves) {
        const WorkItem w = a.items[it];
        const SegDesc sg = a.segs[w.seg];
        const KdeArgs& J = MULTI ? a.jobs[sg.job] : a;
        const int32_t* bnd = J.bounds + sg.bound_off;
        const double two_s = 2.0 * kScale * J.s;

        double qf[RQ][D4];
        double hq[RQ];
        int32_t selfv[RQ], smin[RQ], smax[RQ];
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) {
            const int32_t t = 16 * qb + r;
            const bool ok = t < w.ne;
            const int64_t e = w.e0 + (ok ? t : 0);
            int32_t p = J.q_idx ? J.q_idx[e] : (int32_t)e;
            p = min(max(p, 0), (int32_t)(J.n_query - 1));  // never read outside the query set
            int32_t sf = -1;
            if (ok) sf = (J.self_mode == SELF_POINT) ? p : ((J.self_mode == SELF_ARRAY) ? J.self_idx[e] : -1);
            selfv[qb] = sf;
            hq[qb] = (KIND == kKindExponential) ? J.qnorm[p] : -kScale * J.s * J.qnorm[p];
            load_row_part<D4>(qf[qb], J.Qp, p, grp);
            int32_t mn = sf >= 0 ? sf : INT32_MAX, mx = sf;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                mn = min(mn, __shfl_xor(mn, off));
                mx = max(mx, __shfl_xor(mx, off));
            }
            smin[qb] = uniform(mn);
            smax[qb] = uniform(mx);
        }

        // never read outside the data set, whatever the boundaries say
        const int32_t col_end = uniform(min(max(bnd[w.b1], 0), (int32_t)J.n_data));
        const int32_t col_begin = uniform(min(max(bnd[w.b0], 0), col_end));
        // one open bin per lane where there are four query blocks (fewer
        // registers than four parked bins, which lets d <= 32 run two waves
        // per SIMD); the four-bin shift register otherwise
        typename std::conditional<RQ == 4, BinAccumulator1<RQ>, BinAccumulator<RQ>>::type bins;
        __builtin_amdgcn_wave_barrier();
        load_bin_window(win, bnd, w.b0, w.b1, lane);
        bins.init(bnd, win, w.b0, w.b1, col_begin, w.e0, w.ne, J.out_stride, J.out, J.out_rows, lane);

        // the operands of the next block are loaded while the current one is
        // computed
        const int32_t cfirst = col_begin & ~15;
        double xf[D4], xn[4];
        if (cfirst < col_end) {
            load_row_part<D4>(xf, J.Xp, cfirst + perm_row(r), grp);
#pragma unroll
            for (int i = 0; i < 4; ++i) xn[i] = J.xnorm[cfirst + 4 * grp + i];
        }
        for (int32_t c0 = cfirst; c0 < col_end; c0 += 16) {
            double xf_next[D4], xn_next[4];
            // (d > 64: the query fragments fill the register file, no prefetch)
            constexpr bool kPrefetch = D4 <= 16;
            const bool more = c0 + 16 < col_end;
            if (kPrefetch && more) {
                load_row_part<D4>(xf_next, J.Xp, c0 + 16 + perm_row(r), grp);
#pragma unroll
                for (int i = 0; i < 4; ++i) xn_next[i] = J.xnorm[c0 + 16 + 4 * grp + i];
            }
            int32_t jj[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) jj[i] = c0 + 4 * grp + i;
            double4_t c[RQ];
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb) {
                c[qb] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < D4; ++kk) c[qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xf[kk], qf[qb][kk], c[qb], 0, 0, 0);
            }
            double kv[RQ][4];
            exact_values<RQ, kTab, false, KIND>(c, hq, xn, -kScale * J.s, two_s, jj, selfv, smin, smax, c0, c0 + 15,
                                                exp_tab, kv);
            bins.add(kv, jj, c0 + 15);
            if (more) {
                if (kPrefetch) {
#pragma unroll
                    for (int kk = 0; kk < D4; ++kk) xf[kk] = xf_next[kk];
#pragma unroll
                    for (int i = 0; i < 4; ++i) xn[i] = xn_next[i];
                } else {
                    load_row_part<D4>(xf, J.Xp, c0 + 16 + perm_row(r), grp);
#pragma unroll
                    for (int i = 0; i < 4; ++i) xn[i] = J.xnorm[c0 + 16 + 4 * grp + i];
                }
            }
        }
        bins.finish();
    }
}

template <int D4, int RQ>
static hipError_t launch_kde_t(const KdeArgs& a, int64_t max_items, int num_cus, int waves_per_cu, hipStream_t st) {
    int64_t waves = (int64_t)num_cus * waves_per_cu;
    if (max_items < waves) waves = max_items;
    if (waves < 1) waves = 1;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    if (a.kind == kKindExponential) {
        if (a.jobs) return hipErrorInvalidValue;  // multi-set launches are Gaussian only
        kde_bins_kernel<D4, RQ, false, kKindExponential><<<blocks, 256, 0, st>>>(a);
    } else if (a.jobs) {
        kde_bins_kernel<D4, RQ, true><<<blocks, 256, 0, st>>>(a);
    } else {
        kde_bins_kernel<D4, RQ, false><<<blocks, 256, 0, st>>>(a);
    }
    return hipGetLastError();
}

int kde_tile(int D4) { return D4 >= 16 ? 32 : 64; }

int feature_steps(int d) {
    const int d4 = (d + 3) / 4;
    if (d4 <= 1) return 1;
    if (d4 <= 2) return 2;
    if (d4 <= 4) return 4;
    if (d4 <= 8) return 8;
    if (d4 <= 16) return 16;
    if (d4 <= 32) return 32;
    return -1;  // larger d: not built
}

// The query tile (16 RQ entries per item) is kde_tile(D4): 64, and 32 for
// d > 32, where 32 FP64 query rows let two waves share a SIMD (d <= 64) or
// 64 would not fit the register file (d > 64).
hipError_t launch_kde(const KdeArgs& a, int64_t max_items, int num_cus, hipStream_t st, int waves_per_cu) {
    if (a.kind == kKindLaplacian) return launch_kde_l1(a, max_items, num_cus, st);
    switch (a.D4) {
        case 1: return launch_kde_t<1, 4>(a, max_items, num_cus, waves_per_cu, st);
        case 2: return launch_kde_t<2, 4>(a, max_items, num_cus, waves_per_cu, st);
        case 4: return launch_kde_t<4, 4>(a, max_items, num_cus, waves_per_cu, st);
        case 8: return launch_kde_t<8, 4>(a, max_items, num_cus, waves_per_cu, st);
        case 16: return launch_kde_t<16, 2>(a, max_items, num_cus, waves_per_cu, st);
        case 32: return launch_kde_t<32, 2>(a, max_items, num_cus, waves_per_cu, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Work lists.
// ---------------------------------------------------------------------------
__global__ void regular_items_kernel(int64_t n_entries, int32_t nbins, int32_t bpc, int32_t tile, int64_t n_tiles,
                                     int64_t total, WorkItem* items, int32_t* n_items) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) *n_items = (int32_t)total;
    if (t >= total) return;
    // chunk-major: waves that run together share the same data columns
    const int64_t c = t / n_tiles, q = t - c * n_tiles;
    WorkItem w;
    w.seg = 0;
    w.e0 = q * tile;
    const int64_t rem = n_entries - w.e0;
    w.ne = (int32_t)(rem < tile ? rem : tile);
    w.b0 = (int32_t)(c * bpc);
    w.b1 = (int32_t)min((int64_t)nbins, (c + 1) * (int64_t)bpc);
    items[t] = w;
}

hipError_t launch_regular_items(int64_t n_entries, int32_t nbins, int32_t bins_per_chunk, int32_t tile,
                                WorkItem* items, int32_t* n_items, hipStream_t st) {
    const int64_t n_tiles = (n_entries + tile - 1) / tile;
    const int64_t n_chunks = (nbins + bins_per_chunk - 1) / bins_per_chunk;
    const int64_t total = n_tiles * n_chunks;
    regular_items_kernel<<<(unsigned)((total + 255) / 256 + 1), 256, 0, st>>>(n_entries, nbins, bins_per_chunk, tile,
                                                                             n_tiles, total, items, n_items);
    return hipGetLastError();
}

// Work items of many point sets (one segment each, whole tree level): set g
// owns items [jd[g].item_off, jd[g+1].item_off), chunk-major like the
// single-set list.
__global__ void batch_items_kernel(const BatchItemDesc* __restrict__ jd, int32_t n_jobs, int64_t total,
                                   WorkItem* __restrict__ items, int32_t* __restrict__ n_items) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) *n_items = (int32_t)total;
    if (t >= total) return;
    int32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (jd[mid].item_off <= t) lo = mid; else hi = mid;
    }
    const BatchItemDesc d = jd[lo];
    const int64_t local = t - d.item_off;
    const int64_t c = local / d.n_tiles, q = local - c * d.n_tiles;
    WorkItem w;
    w.seg = lo;
    w.e0 = q * d.tile;
    const int64_t rem = d.n_entries - w.e0;
    w.ne = (int32_t)(rem < d.tile ? rem : d.tile);
    w.b0 = (int32_t)(c * d.bpc);
    w.b1 = (int32_t)min((int64_t)d.nbins, (c + 1) * (int64_t)d.bpc);
    items[t] = w;
}

hipError_t launch_batch_items(const BatchItemDesc* jd, int32_t n_jobs, int64_t total, WorkItem* items,
                              int32_t* n_items, hipStream_t st) {
    batch_items_kernel<<<(unsigned)((total + 255) / 256 + 1), 256, 0, st>>>(jd, n_jobs, total, items, n_items);
    return hipGetLastError();
}

__global__ void segment_item_counts_kernel(const int64_t* q_ptr, int64_t n_seg, int32_t n_chunks, int32_t tile,
                                           int64_t* counts) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_seg) return;
    const int64_t cnt = q_ptr[s + 1] - q_ptr[s];
    counts[s] = ((cnt + tile - 1) / tile) * n_chunks;
}

__global__ void segment_items_fill_kernel(const int64_t* q_ptr, const int64_t* offsets, int64_t n_seg,
                                          int32_t nbins, int32_t bpc, int32_t n_chunks, int32_t tile,
                                          const int64_t* total, int64_t max_items, WorkItem* items,
                                          int32_t* n_items) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = *total;
    if (t == 0) *n_items = (int32_t)(tot < max_items ? tot : max_items);
    if (t >= tot || t >= max_items) return;
    // segment of item t: last s with offsets[s] <= t (skipping empty segments)
    int64_t lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (offsets[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int64_t s = lo;
    const int64_t local = t - offsets[s];
    const int64_t cnt = q_ptr[s + 1] - q_ptr[s];
    const int64_t n_tiles = (cnt + tile - 1) / tile;
    const int64_t c = local / n_tiles, q = local - c * n_tiles;
    WorkItem w;
    w.seg = (int32_t)s;
    w.e0 = q_ptr[s] + q * tile;
    const int64_t rem = cnt - q * tile;
    w.ne = (int32_t)(rem < tile ? rem : tile);
    w.b0 = (int32_t)(c * bpc);
    w.b1 = (int32_t)min((int64_t)nbins, (c + 1) * (int64_t)bpc);
    items[t] = w;
}

hipError_t launch_build_items(const int64_t* q_ptr, int64_t n_seg, int32_t nbins, int32_t bins_per_chunk,
                              int32_t tile, int64_t* scratch_counts, WorkItem* items, int32_t* n_items,
                              int64_t max_items, hipStream_t st) {
    // scratch_counts: n_seg + 1 counts, then n_seg + 1 offsets, then 1 total, then scan partials
    const int32_t n_chunks = (nbins + bins_per_chunk - 1) / bins_per_chunk;
    int64_t* counts = scratch_counts;
    int64_t* offsets = counts + (n_seg + 1);
    int64_t* total = offsets + (n_seg + 1);
    int64_t* partials = total + 1;
    segment_item_counts_kernel<<<(unsigned)((n_seg + 255) / 256 + 1), 256, 0, st>>>(q_ptr, n_seg, n_chunks, tile,
                                                                                   counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan_i64(counts, offsets, n_seg, total, partials, st);
    if (e != hipSuccess) return e;
    segment_items_fill_kernel<<<(unsigned)((max_items + 255) / 256 + 1), 256, 0, st>>>(
        q_ptr, offsets, n_seg, nbins, bins_per_chunk, n_chunks, tile, total, max_items, items, n_items);
    return hipGetLastError();
}

__global__ void uniform_segs_kernel(SegDesc* segs, int64_t n_seg, int64_t stride, int32_t nbins) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_seg) return;
    SegDesc g;
    g.bound_off = s * stride;
    g.nbins = nbins;
    g.job = 0;
    segs[s] = g;
}

hipError_t launch_uniform_segs(SegDesc* segs, int64_t n_seg, int64_t stride, int32_t nbins, hipStream_t st) {
    uniform_segs_kernel<<<(unsigned)((n_seg + 255) / 256 + 1), 256, 0, st>>>(segs, n_seg, stride, nbins);
    return hipGetLastError();
}

__global__ void api_segments_kernel(const int32_t* lo, const int32_t* mid, const int32_t* hi, int64_t n_seg,
                                    int32_t* bounds, SegDesc* segs) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_seg) return;
    bounds[3 * s] = lo[s];
    bounds[3 * s + 1] = mid[s];
    bounds[3 * s + 2] = hi[s];
    SegDesc g;
    g.bound_off = 3 * s;
    g.nbins = 2;
    g.job = 0;
    segs[s] = g;
}

hipError_t launch_api_segments(const int32_t* lo, const int32_t* mid, const int32_t* hi, int64_t n_seg,
                               int32_t* bounds, SegDesc* segs, hipStream_t st) {
    api_segments_kernel<<<(unsigned)((n_seg + 255) / 256 + 1), 256, 0, st>>>(lo, mid, hi, n_seg, bounds, segs);
    return hipGetLastError();
}

__global__ void row_sums_kernel(const double* M, int64_t rows, int32_t cols, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const double* m = M + i * cols;
    double s = 0.0;
    for (int32_t b = 0; b < cols; ++b) s += m[b];
    out[i] = s;
}

hipError_t launch_row_sums(const double* M, int64_t rows, int32_t cols, double* out, hipStream_t st) {
    row_sums_kernel<<<(unsigned)((rows + 255) / 256 + 1), 256, 0, st>>>(M, rows, cols, out);
    return hipGetLastError();
}

__global__ void split_pairs_kernel(const double* pairs, int64_t n, double* left, double* right) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    left[e] = pairs[2 * e];
    right[e] = pairs[2 * e + 1];
}

hipError_t launch_split_pairs(const double* pairs, int64_t n, double* left, double* right, hipStream_t st) {
    split_pairs_kernel<<<(unsigned)((n + 255) / 256 + 1), 256, 0, st>>>(pairs, n, left, right);
    return hipGetLastError();
}

}  // namespace fsg
