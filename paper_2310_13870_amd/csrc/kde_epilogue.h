// Binned epilogue shared by the KDE kernels: FP64 kernel values of the pairs
// of one 16-column block (or of 16 gathered columns) are accumulated into
// consecutive index-range bins.
//
// Data columns are the A operand of v_mfma_f64_16x16x4f64 with its rows
// permuted, so that lane group g = lane / 16 receives four consecutive
// columns jj[0] < jj[1] < jj[2] < jj[3] (positions 4g .. 4g+3 of the block)
// for query row lane % 16 of every query block.  Within a bin each lane keeps
// its own partial sum; a bin boundary inside a block splits a lane's four
// values with 0/1 weights (exact products, no selects).  The partials of four
// consecutive bins are parked in four slots and combined across the lane
// groups with one permlane32 and one permlane16 swap, which leaves bin 4w + g
// in lane group g: each query row receives one contiguous 32-byte segment per
// four bins.  No atomics, fixed order: results are bit-reproducible.
#pragma once
#include "common.h"
#include "device.h"
#include "exp2_table.h"

namespace fsg {

// Row rho of the A operand holds block position perm_row(rho); the result
// element i of lane group g is then position 4g + i.
__device__ __forceinline__ int perm_row(int rho) { return 4 * (rho & 3) + (rho >> 2); }

// The D4 operands that the lanes of feature row g supply for point p, one
// per feature step, from the point's FP64 row: step pair k of feature row g
// is the 16 bytes at 64 k + 16 g, so the four feature rows of a point read 64
// contiguous bytes per load.
template <int D4>
__device__ __forceinline__ void load_row_part(double (&dst)[D4], const double* base, int64_t p, int g) {
    if constexpr (D4 == 1) {
        dst[0] = base[p * 4 + g];
    } else {
        typedef double double2_t __attribute__((ext_vector_type(2)));
        const double2_t* s2 = (const double2_t*)(base + p * (4 * D4)) + g;
#pragma unroll
        for (int k = 0; k < D4 / 2; ++k) {
            const double2_t v = s2[4 * k];
            dst[2 * k] = v[0];
            dst[2 * k + 1] = v[1];
        }
    }
}

// Boundaries of a work item's bins are copied into a per-wave LDS window so
// that reading the next boundary never waits behind vector-memory prefetches.
constexpr int kBinWindow = 512;

__device__ __forceinline__ void load_bin_window(int32_t* win, const int32_t* bnd, int32_t b0, int32_t b1, int lane) {
    const int32_t cnt = min(b1 - b0 + 1, kBinWindow);
    for (int32_t k = lane; k < cnt; k += 64) win[k] = bnd[b0 + k];
    __builtin_amdgcn_wave_barrier();
}

// a + b after exchanging rows 2-3 of a with rows 0-1 of b: lanes 0-31 get
// a[l] + a[l + 32], lanes 32-63 get b[l - 32] + b[l].
__device__ __forceinline__ double swap32_add(double a, double b) {
    const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)ua, (uint32_t)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
    const double a2 = __longlong_as_double((int64_t)(((uint64_t)hi[0] << 32) | lo[0]));
    const double b2 = __longlong_as_double((int64_t)(((uint64_t)hi[1] << 32) | lo[1]));
    return a2 + b2;
}

// a + b after exchanging the odd rows of a with the even rows of b: row 0 gets
// a[r0] + a[r1], row 1 b[r0] + b[r1], row 2 a[r2] + a[r3], row 3 b[r2] + b[r3].
__device__ __forceinline__ double swap16_add(double a, double b) {
    const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ua, (uint32_t)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
    const double a2 = __longlong_as_double((int64_t)(((uint64_t)hi[0] << 32) | lo[0]));
    const double b2 = __longlong_as_double((int64_t)(((uint64_t)hi[1] << 32) | lo[1]));
    return a2 + b2;
}

// kExp2Table copied into a workgroup's LDS (all threads of the block call it)
__device__ __forceinline__ void load_exp2_table(double* tab) {
    for (int k = threadIdx.x; k < 256; k += blockDim.x) tab[k] = kExp2Table[k];
    __syncthreads();
}

template <int RQ>
struct BinAccumulator {
    const int32_t* bnd;   // boundaries of the segment's bins
    const int32_t* win;   // LDS copy of bnd[b0 .. b0 + kBinWindow)
    int32_t b0, b1;       // bins [b0, b1) of this work item
    int32_t cur;          // bin being accumulated (b0 - 1: before the first)
    int32_t start;        // first column of bin cur
    int32_t nxt;          // first column of bin cur + 1
    int64_t stride;
    double* out;
    int32_t orow[RQ];     // output row of this lane's query row in each query block (-1: none)
    int lane;
    // this lane's partials: slot 3 accumulates bin cur, slots 0-2 hold the
    // bins closed before it in window cur & ~3
    double slot[RQ][4];

    __device__ __forceinline__ void init(const int32_t* bnd_, const int32_t* win_, int32_t b0_, int32_t b1_, int32_t col_begin,
                         int64_t e0_, int32_t ne_, int64_t stride_, double* out_, const int32_t* out_rows_, int lane_) {
        bnd = bnd_;
        win = win_;
        b0 = uniform(b0_);
        b1 = uniform(b1_);
        cur = uniform(b0_ - 1);
        start = INT32_MIN;
        nxt = uniform(col_begin);
        stride = stride_;
        out = out_;
        lane = lane_;
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) {
#pragma unroll
            for (int m = 0; m < 4; ++m) slot[qb][m] = 0.0;
            // output rows are resolved once, so that flushes issue no loads
            // (a vector load there would wait for every prefetch in flight)
            const int32_t t = 16 * qb + (lane & 15);
            const int64_t e = e0_ + t;
            orow[qb] = (t < ne_) ? (out_rows_ ? out_rows_[e] : (int32_t)e) : -1;
        }
    }

    // combine the four slots across the lane groups and write bins w4 .. w4+3
    // that lie in [b0, b1); the slots are cleared
    __device__ __forceinline__ void emit(int32_t w4) {
        const int32_t b = w4 + (lane >> 4);
        const bool ok = b >= b0 && b < b1;
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) {
            const double t02 = swap32_add(slot[qb][0], slot[qb][2]);
            const double t13 = swap32_add(slot[qb][1], slot[qb][3]);
            const double v = swap16_add(t02, t13);
            if (ok && orow[qb] >= 0) out[(int64_t)orow[qb] * stride + b] = v;
#pragma unroll
            for (int m = 0; m < 4; ++m) slot[qb][m] = 0.0;
        }
    }

    // open the next bin in slot 3 (slot j then holds bin w + j once the four
    // bins of window w have been closed, in order)
    __device__ __forceinline__ void shift() {
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) {
            slot[qb][0] = slot[qb][1];
            slot[qb][1] = slot[qb][2];
            slot[qb][2] = slot[qb][3];
            slot[qb][3] = 0.0;
        }
    }

    // bin cur is complete: a finished window, or the last bin's window padded
    // with empty bins, is written out; otherwise the next bin is opened
    __device__ __forceinline__ void close() {
        if ((cur & 3) == 3) {
            emit(cur & ~3);
        } else if (cur == b1 - 1) {
            for (int m = cur & 3; m < 3; ++m) shift();
            emit(cur & ~3);
        } else {
            shift();
        }
    }

    __device__ __forceinline__ void advance() {
        ++cur;
        start = nxt;
        if (cur < b1) {
            const int32_t k = cur + 1 - b0;
            nxt = uniform((k < kBinWindow) ? win[k] : bnd[cur + 1]);
        } else {
            nxt = INT32_MAX;
        }
    }

    // Add kernel values kv[qb][i] of columns jj[i]; `last` is the largest
    // column of the block (uniform).  Columns below the first bin or at/after
    // the end of the last bin are dropped.
    __device__ __forceinline__ void add(const double (&kv)[RQ][4], const int32_t (&jj)[4], int32_t last) {
        if (nxt > last) {  // the whole block lies in bin cur (uniform)
            if (cur >= b0 && cur < b1) {
#pragma unroll
                for (int qb = 0; qb < RQ; ++qb) slot[qb][3] += (kv[qb][0] + kv[qb][1]) + (kv[qb][2] + kv[qb][3]);
            }
            return;
        }
        while (nxt <= last) {  // a boundary inside this block (uniform)
            if (cur >= b0) {
                double wgt[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) wgt[i] = (jj[i] >= start && jj[i] < nxt) ? 1.0 : 0.0;
#pragma unroll
                for (int qb = 0; qb < RQ; ++qb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) slot[qb][3] = __builtin_fma(kv[qb][i], wgt[i], slot[qb][3]);
                close();
            }
            advance();
        }
        if (cur >= b0 && cur < b1) {
            double wgt[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) wgt[i] = (jj[i] >= start) ? 1.0 : 0.0;
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb)
#pragma unroll
                for (int i = 0; i < 4; ++i) slot[qb][3] = __builtin_fma(kv[qb][i], wgt[i], slot[qb][3]);
        }
    }

    // the open bin and the empty bins after the last column
    __device__ __forceinline__ void finish() {
        if (cur < b0) {  // nothing was added: every bin is empty, every slot 0
            cur = b0;
        } else if (cur < b1) {
            // bin cur is open in slot 3: move it to slot cur & 3 (the bins
            // after it in its window are empty) and write the window
            for (int m = cur & 3; m < 3; ++m) shift();
            emit(cur & ~3);
            cur = (cur & ~3) + 4;
        }
        if (cur >= b1) return;
        // the remaining bins are empty and every slot is 0
        if ((cur & 3) != 0) {
            emit(cur & ~3);
            cur = (cur & ~3) + 4;
        }
        for (; cur < b1; cur += 4) emit(cur);
    }
};

// The same accumulation with one open bin per lane, for the gathered columns
// of the precision mode, where a block of 16 kept columns spans several bins
// (their columns are sparse): slot[qb] is this lane's partial of bin cur for
// query block qb (RQ = 4, one per lane group).  Closing a bin combines the
// four query blocks' partials across the lane groups with the same
// permlane32 and permlane16 swaps, which leaves query block g's total in lane
// group g, and shifts it into a 4-bin staging register; every 4 bins each
// lane writes its row's 32 bytes.  Fixed order, no atomics: bit-reproducible.
template <int RQ>
struct BinAccumulator1 {
    static_assert(RQ == 4, "one query block per lane group");
    const int32_t* bnd;  // boundaries of the segment's bins
    const int32_t* win;  // LDS copy of bnd[b0 .. b0 + kBinWindow)
    int32_t b0, b1;      // bins [b0, b1) of this work item
    int32_t cur;         // bin being accumulated (b0 - 1: before the first)
    int32_t start;       // first column of bin cur
    int32_t nxt;         // first column of bin cur + 1
    int64_t stride;
    double* out;
    int32_t orow;        // output row of query row lane % 16 of query block lane / 16 (-1: none)
    double slot[RQ];     // partials of bin cur
    double stage[4];     // stage[3] is the last closed bin, stage[j] the one 3 - j before it

    __device__ __forceinline__ void init(const int32_t* bnd_, const int32_t* win_, int32_t b0_, int32_t b1_,
                                         int32_t col_begin, int64_t e0_, int32_t ne_, int64_t stride_, double* out_,
                                         const int32_t* out_rows_, int lane) {
        bnd = bnd_;
        win = win_;
        b0 = uniform(b0_);
        b1 = uniform(b1_);
        cur = uniform(b0_ - 1);
        start = INT32_MIN;
        nxt = uniform(col_begin);
        stride = stride_;
        out = out_;
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) slot[qb] = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) stage[j] = 0.0;
        const int32_t t = 16 * (lane >> 4) + (lane & 15);
        const int64_t e = e0_ + t;
        orow = (t < ne_) ? (out_rows_ ? out_rows_[e] : (int32_t)e) : -1;
    }

    // write the staged window of 4 bins ending at bin c (c % 4 == 3), those in [b0, b1)
    __device__ __forceinline__ void write_window(int32_t c) {
        if (orow < 0) return;
        double* row = out + (int64_t)orow * stride + (c - 3);
        if (c - 3 >= b0 && c < b1) {
            typedef double double2_t __attribute__((ext_vector_type(2)));
            ((double2_t*)row)[0] = double2_t{stage[0], stage[1]};
            ((double2_t*)row)[1] = double2_t{stage[2], stage[3]};
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c - 3 + j >= b0 && c - 3 + j < b1) row[j] = stage[j];
        }
    }

    __device__ __forceinline__ void push(double v) {
        stage[0] = stage[1];
        stage[1] = stage[2];
        stage[2] = stage[3];
        stage[3] = v;
    }

    // bin cur is complete: combine it and stage it; a full window, or the
    // last bin's window padded with the empty bins after it, is written
    __device__ __forceinline__ void close() {
        const double t02 = swap32_add(slot[0], slot[2]);
        const double t13 = swap32_add(slot[1], slot[3]);
        push(swap16_add(t02, t13));
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) slot[qb] = 0.0;
        if ((cur & 3) == 3) {
            write_window(cur);
        } else if (cur == b1 - 1) {
            for (int32_t c = cur + 1; (c & 3) != 0; ++c) push(0.0);
            write_window(cur | 3);
        }
    }

    __device__ __forceinline__ void advance() {
        ++cur;
        start = nxt;
        if (cur < b1) {
            const int32_t k = cur + 1 - b0;
            nxt = uniform((k < kBinWindow) ? win[k] : bnd[cur + 1]);
        } else {
            nxt = INT32_MAX;
        }
    }

    // Add kernel values kv[qb][i] of columns jj[i]; `last` is the largest
    // column of the block (uniform).  Columns below the first bin or at/after
    // the end of the last bin are dropped.
    __device__ __forceinline__ void add(const double (&kv)[RQ][4], const int32_t (&jj)[4], int32_t last) {
        if (nxt > last) {  // the whole block lies in bin cur (uniform)
            if (cur >= b0 && cur < b1) {
#pragma unroll
                for (int qb = 0; qb < RQ; ++qb) slot[qb] += (kv[qb][0] + kv[qb][1]) + (kv[qb][2] + kv[qb][3]);
            }
            return;
        }
        while (nxt <= last) {  // a boundary inside this block (uniform)
            if (cur >= b0) {
                double wgt[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) wgt[i] = (jj[i] >= start && jj[i] < nxt) ? 1.0 : 0.0;
#pragma unroll
                for (int qb = 0; qb < RQ; ++qb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) slot[qb] = __builtin_fma(kv[qb][i], wgt[i], slot[qb]);
            }
            // bins before b0 are not written (close() writes only in [b0, b1))
            close();
            advance();
        }
        if (cur >= b0 && cur < b1) {
            double wgt[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) wgt[i] = (jj[i] >= start) ? 1.0 : 0.0;
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb)
#pragma unroll
                for (int i = 0; i < 4; ++i) slot[qb] = __builtin_fma(kv[qb][i], wgt[i], slot[qb]);
        }
    }

    // the open bin and the empty bins after it, to the end of the item (once
    // bin b1 - 1 has been closed, by add() or here, every bin is written)
    __device__ __forceinline__ void finish() {
        for (; cur < b1; ++cur) close();
    }
};

// The FP64 epilogue of one query block against 16 columns: kernel values
// from the cross terms c (result element i of lane group g is block position
// 4g + i), the self term removed.  The exponent of each pair is
// fma(two_s, c, fma(|x|^2, neg_s, hq)): the column's norm term enters through
// a fused multiply-add, one rounding of the large partial sum.  With tab (the
// LDS copy of kExp2Table) the exponent terms are scaled by 256 (hq = -256 s
// |q|^2, neg_s = -256 s, two_s = 512 s, s = gamma log2 e), a power of two that
// leaves every rounding as it is, and exp2_256_tab evaluates them; without it
// (tab = nullptr, a compile-time choice of the caller) hq = -s |q|^2, neg_s =
// -s, two_s = 2 s and exp2_fp64 does.  AHEAD (table form only) issues the
// four table reads before the first is used; it pays where the kernel's other
// vector work does not hide the LDS latency (the exact recompute), and the
// values are the same either way.  The self compare runs only when a query of
// the block has its own index in [lo_col, hi_col].
//
// KIND = kKindExponential (the exponential kernel): hq is the raw |q|^2 and
// the exponent is neg_s sqrt(max(|q|^2 + |x|^2 - 2 x.q, 0)) (two_s unused).
template <int KIND>
__device__ __forceinline__ double pair_exponent(double c, double hq, double xn, double neg_s, double two_s) {
    if constexpr (KIND == kKindExponential) {
        const double D = __builtin_fma(-2.0, c, hq + xn);
        return neg_s * __builtin_sqrt(__builtin_fmax(D, 0.0));
    } else {
        return __builtin_fma(two_s, c, __builtin_fma(xn, neg_s, hq));
    }
}

template <bool TAB, bool AHEAD, int KIND = kKindGaussian>
__device__ __forceinline__ void exact_values_block(const double4_t& c, double hq, const double (&xn)[4], double neg_s,
                                                   double two_s, const int32_t (&jj)[4], int32_t selfv, int32_t smin,
                                                   int32_t smax, int32_t lo_col, int32_t hi_col, const double* tab,
                                                   double (&kv)[4]) {
    if constexpr (TAB && AHEAD) {
        // the four table reads are issued before the first is used
        double r[4], t[4];
        int32_t mi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            mi[i] = exp2_256_split(pair_exponent<KIND>(c[i], hq, xn[i], neg_s, two_s), &r[i]);
            t[i] = tab[mi[i] & 255];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) kv[i] = exp2_256_join(t[i], r[i], mi[i]);
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double z = pair_exponent<KIND>(c[i], hq, xn[i], neg_s, two_s);
            kv[i] = TAB ? exp2_256_tab(z, tab) : exp2_fp64(z);
        }
    }
    if (smax >= lo_col && smin <= hi_col && __ballot(selfv >= lo_col && selfv <= hi_col) != 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (jj[i] == selfv) kv[i] = 0.0;
    }
}

// The FP64 epilogue of all query blocks against one 16-column block.
template <int RQ, bool TAB, bool AHEAD = false, int KIND = kKindGaussian>
__device__ __forceinline__ void exact_values(const double4_t (&c)[RQ], const double (&hq)[RQ], const double (&xn)[4],
                                             double neg_s, double two_s, const int32_t (&jj)[4],
                                             const int32_t (&selfv)[RQ], const int32_t (&smin)[RQ],
                                             const int32_t (&smax)[RQ], int32_t lo_col, int32_t hi_col,
                                             const double* tab, double (&kv)[RQ][4]) {
#pragma unroll
    for (int qb = 0; qb < RQ; ++qb)
        exact_values_block<TAB, AHEAD, KIND>(c[qb], hq[qb], xn, neg_s, two_s, jj, selfv[qb], smin[qb], smax[qb], lo_col,
                                             hi_col, tab, kv[qb]);
}

}  // namespace fsg
