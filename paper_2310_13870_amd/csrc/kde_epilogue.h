// Binned epilogue shared by the KDE kernels: FP64 kernel values of the pairs
// of one 16-column block (or of 16 gathered columns) are accumulated into
// consecutive index-range bins.  Each lane holds four data columns jj[0..3]
// of one query row (row = lane % 16 of a query block); columns are increasing
// along (lane / 16) + 4 i.  When a bin boundary is crossed the four partial
// sums of a query row are combined with two cross-lane steps; finished bins
// are kept in the lane group (bin mod 4) and written four at a time, so each
// query row receives one contiguous 32-byte segment per four bins.  No
// atomics, fixed order: results are bit-reproducible.
#pragma once
#include "common.h"
#include "device.h"

namespace fsg {

// Boundaries of a work item's bins are copied into a per-wave LDS window so
// that reading the next boundary never waits behind vector-memory prefetches.
constexpr int kBinWindow = 512;

__device__ __forceinline__ void load_bin_window(int32_t* win, const int32_t* bnd, int32_t b0, int32_t b1, int lane) {
    const int32_t cnt = min(b1 - b0 + 1, kBinWindow);
    for (int32_t k = lane; k < cnt; k += 64) win[k] = bnd[b0 + k];
    __builtin_amdgcn_wave_barrier();
}

template <int RQ>
struct BinAccumulator {
    const int32_t* bnd;   // boundaries of the segment's bins
    const int32_t* win;   // LDS copy of bnd[b0 .. b0 + kBinWindow)
    int32_t b0, b1;       // bins [b0, b1) of this work item
    int32_t cur;          // bin being accumulated (b0 - 1: before the first)
    int32_t nxt;          // first column of the next bin
    int64_t stride;
    double* out;
    int64_t orow[RQ];     // output row of this lane's query row in each query block (-1: none)
    int lane;
    double acc[RQ];
    double pend[RQ];

    __device__ void init(const int32_t* bnd_, const int32_t* win_, int32_t b0_, int32_t b1_, int32_t col_begin,
                         int64_t e0_, int32_t ne_, int64_t stride_, double* out_, const int32_t* out_rows_, int lane_) {
        bnd = bnd_;
        win = win_;
        b0 = b0_;
        b1 = b1_;
        cur = b0_ - 1;
        nxt = col_begin;
        stride = stride_;
        out = out_;
        lane = lane_;
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) {
            acc[qb] = 0.0;
            pend[qb] = 0.0;
            // output rows are resolved once, so that flushes issue no loads
            // (a vector load there would wait for every prefetch in flight)
            const int32_t t = 16 * qb + (lane & 15);
            const int64_t e = e0_ + t;
            orow[qb] = (t < ne_) ? (out_rows_ ? (int64_t)out_rows_[e] : e) : -1;
        }
    }

    // write the pending bins [max(b0, base), last] of every valid row
    __device__ void write_pending(int32_t last) {
        const int32_t base = last & ~3;
        const int32_t b = base + (lane >> 4);
        if (b < b0 || b > last) return;
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb)
            if (orow[qb] >= 0) out[orow[qb] * stride + b] = pend[qb];
    }

    __device__ void flush(int32_t bin) {
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) {
            double v = acc[qb];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if ((lane >> 4) == (bin & 3)) pend[qb] = v;
            acc[qb] = 0.0;
        }
        if ((bin & 3) == 3 || bin == b1 - 1) write_pending(bin);
    }

    // Add kernel values kv[qb][i] of columns jj[i]; `last` is the largest
    // column of the block (uniform).  Columns below the first bin or at/after
    // the end of the last bin are dropped.
    __device__ void add(double (&kv)[RQ][4], const int32_t (&jj)[4], int32_t last) {
        while (nxt <= last) {  // a boundary inside this block (uniform)
            if (cur >= b0) {
#pragma unroll
                for (int qb = 0; qb < RQ; ++qb) {
                    double part = 0.0;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (jj[i] < nxt) part += kv[qb][i];
                    acc[qb] += part;
                }
                flush(cur);
            }
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (jj[i] < nxt) kv[qb][i] = 0.0;
            ++cur;
            if (cur < b1) {
                const int32_t k = cur + 1 - b0;
                nxt = (k < kBinWindow) ? win[k] : bnd[cur + 1];
            } else {
                nxt = INT32_MAX;
            }
        }
        if (cur >= b0 && cur < b1) {
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb) acc[qb] += (kv[qb][0] + kv[qb][1]) + (kv[qb][2] + kv[qb][3]);
        }
    }

    // the open bin and any empty bins after the last column
    __device__ void finish() {
        while (cur < b1) {
            if (cur >= b0) flush(cur);
            ++cur;
        }
    }
};

// The FP64 epilogue of one 16x16 block: kernel values from the cross terms c
// (lane layout of v_mfma_f64_16x16x4f64: data rows lane/16 + 4i), the self
// term removed.
template <int RQ>
__device__ __forceinline__ void exact_values(const double4_t (&c)[RQ], const double (&hq)[RQ], const double (&hx)[4],
                                             double two_s, const int32_t (&jj)[4], const int32_t (&selfv)[RQ],
                                             const int32_t (&smin)[RQ], const int32_t (&smax)[RQ], int32_t lo_col,
                                             int32_t hi_col, double (&kv)[RQ][4]) {
#pragma unroll
    for (int qb = 0; qb < RQ; ++qb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) kv[qb][i] = exp2_fp64(__builtin_fma(two_s, c[qb][i], hq[qb] + hx[i]));
        if (smax[qb] >= lo_col && smin[qb] <= hi_col) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (jj[i] == selfv[qb]) kv[qb][i] = 0.0;
        }
    }
}

}  // namespace fsg
