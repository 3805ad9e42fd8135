// Segmented KDE of the Laplacian kernel, k = exp(-gamma ||q - x||_1)
// (Section 2.1 names it beside the Gaussian kernel), over tree bins, on the
// FP64 vector units: an L1 distance has no inner-product form for the matrix
// cores.  The same work items as the binned Gaussian KDE (a segment's query
// entries and a run of its bins); here a wave holds up to 64 entries, one per
// lane, and walks the item's columns in index order: every lane is in the
// same bin at the same time, so a bin boundary is a uniform event and each
// lane writes its own sum.  The columns are staged in LDS in FP64 (exact
// copies of the FP32 points), the coordinate differences are exact in FP64
// and summed in coordinate order, the exponential is evaluated in FP64, and
// the self term is skipped.  No atomics, fixed order: bit-reproducible.
#include "common.h"
#include "device.h"

namespace fsg {

template <int DMAX>
__global__ __launch_bounds__(64) void kde_l1_kernel(KdeArgs a) {
    constexpr int CH = (DMAX <= 32) ? 64 : 2048 / DMAX;  // columns per LDS stage (16 KB at most)
    __shared__ double xs[CH][DMAX];
    const int lane = threadIdx.x;
    const int32_t n_items = *a.n_items;
    const int32_t d = a.d;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const WorkItem w = a.items[it];
        const SegDesc sg = a.segs[w.seg];
        const int32_t* bnd = a.bounds + sg.bound_off;
        const bool ok = lane < w.ne;
        const int64_t e = w.e0 + (ok ? lane : 0);
        int32_t p = a.q_idx ? a.q_idx[e] : (int32_t)e;
        p = min(max(p, 0), (int32_t)(a.n_query - 1));  // never read outside the query set
        int32_t selfv = -1;
        if (ok) selfv = (a.self_mode == SELF_POINT) ? p : ((a.self_mode == SELF_ARRAY) ? a.self_idx[e] : -1);
        const int32_t orow = ok ? (a.out_rows ? a.out_rows[e] : (int32_t)e) : -1;
        float q[DMAX];
#pragma unroll
        for (int t = 0; t < DMAX; ++t) q[t] = (t < d) ? a.qpts[(int64_t)p * d + t] : 0.0f;
        // never read outside the data set, whatever the boundaries say
        const int32_t col_end = uniform(min(max(bnd[w.b1], 0), (int32_t)a.n_data));
        const int32_t col_begin = uniform(min(max(bnd[w.b0], 0), col_end));
        int32_t cur = w.b0;  // the open bin (uniform)
        int32_t nxt = uniform((cur + 1 <= w.b1) ? min(max(bnd[cur + 1], col_begin), col_end) : col_end);
        double acc = 0.0;
        auto close_bin = [&]() {
            if (orow >= 0) a.out[(int64_t)orow * a.out_stride + cur] = acc;
            acc = 0.0;
            ++cur;
            nxt = uniform((cur < w.b1) ? min(max(bnd[cur + 1], col_begin), col_end) : INT32_MAX);
        };
        for (int32_t c0 = col_begin; c0 < col_end; c0 += CH) {
            const int32_t nc = min(CH, col_end - c0);
            __syncthreads();
            for (int32_t k = lane; k < CH * DMAX; k += 64) {
                const int32_t cc = k / DMAX, t = k - cc * DMAX;
                xs[cc][t] = (cc < nc && t < d) ? (double)a.xpts[(int64_t)(c0 + cc) * d + t] : 0.0;
            }
            __syncthreads();
            for (int32_t cc = 0; cc < nc; ++cc) {
                const int32_t j = c0 + cc;
                while (j >= nxt && cur < w.b1) close_bin();
                double s1 = 0.0;
#pragma unroll
                for (int t = 0; t < DMAX; ++t) s1 += __builtin_fabs((double)q[t] - xs[cc][t]);
                const double k = exp2_fp64(-a.s * s1);
                if (j != selfv) acc += k;
            }
        }
        // the open bin and the empty bins after the last column
        while (cur < w.b1) close_bin();
    }
}

hipError_t launch_kde_l1(const KdeArgs& a, int64_t max_items, int num_cus, hipStream_t st) {
    int64_t blocks = (int64_t)num_cus * 8;
    if (max_items < blocks) blocks = max_items;
    if (blocks < 1) blocks = 1;
    if (a.jobs) return hipErrorInvalidValue;  // multi-set launches are Gaussian only
    const int d = a.d;
    if (d <= 8) kde_l1_kernel<8><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (d <= 32) kde_l1_kernel<32><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (d <= 64) kde_l1_kernel<64><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (d <= 128) kde_l1_kernel<128><<<(unsigned)blocks, 64, 0, st>>>(a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fsg
