// Filtered segmented KDE on the BF16 matrix cores (precision mode).
//
// Every pair first gets an approximate cross term from BF16 hi/lo split
// operands (hi = bf16(x), lo = bf16(x - hi); one contraction over K = 3d
// gives hi.hi + hi.lo + lo.hi), accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16.  A pair can change a row's masses only if its
// exponent z = gamma |q-x|^2 is within Delta of the row's smallest one (a
// term e^-Delta times the largest term of the row is negligible); with a
// guaranteed bound E on the error of the approximate cross term (it also
// covers the FP32 rounding of the accumulation and of |x|^2/2), the test
//     c~ - theta_q >= |x|^2/2,   theta_q = |q|^2/2 - T_q/(2 gamma) - E,
//     T_q = gamma dmin_q + Delta
// keeps every such pair (dmin_q is an upper bound on the row's smallest
// squared distance).  The accumulator starts at -theta_q (theta_q rounded
// down to FP32), so that the 16 results a lane holds, which share one data
// column, are tested with one max and one compare.  Stage 1 writes, per
// 64-query tile and 16-column block, the mask of columns kept for any query
// of the tile; stage 2 queues the kept columns, gathers every 16 of them into
// one block whose cross terms are recomputed on the FP64 matrix cores, and
// sends them through the same FP64 epilogue and bin accumulation as the plain
// kernel.  Pairs not kept add 0: their total is below (n-1) e^-Delta of the
// row's mass.
#include <type_traits>

#include "common.h"
#include "device.h"
#include "kde_epilogue.h"


namespace fsg {

// exact-pass occupancy: two waves per SIMD (the query fragments are staged
// in LDS in FP32 -- the points' own precision, so the copy is exact -- which
// leaves room for two blocks of four waves per compute unit)
template <int D4>
constexpr int exact_waves() { return 2; }

// ---------------------------------------------------------------------------
// Stage 2: exact recompute of the kept columns.  Work item = (query tile,
// run of bins).  Kept columns enter a per-wave queue in LDS in index order, 16
// mask blocks at a time; every 16 of them form one gathered block for the
// FP64 matrix cores and the binned epilogue.  The operands of the next block
// are loaded while the current one is computed; the FP64 query fragments
// live in LDS.
// ---------------------------------------------------------------------------
template <int D4>
struct Gathered {
    double xf[D4];
    double xn[4];  // |x|^2 of the lane's four columns, +inf for padding (scaled
                   // only when used, so that the loads stay in flight while
                   // the previous block computes)
    int32_t jj[4];
    int32_t first, last;  // smallest and largest column (uniform)
};

// The integer-slice variant (32 < d <= 64, Gaussian kernel): the cross term
// of a pair is 2^(e_q + e_x) sum_{a+b <= kSlices+1} 2^-8(a+b) (q_a . x_b) over
// the slices (layout in common.h), each slice product an exact integer on
// v_mfma_i32_16x16x64_i8 (|q_a . x_b| <= 64 * 2^14 = 2^20; a group of equal
// a+b holds at most 7 of them, so the int32 accumulators cannot overflow and
// two neighbouring groups join exactly in 32 bits).  The joined groups are
// summed in FP64 (three roundings).  Against the exact product, the dropped
// slice pairs (a+b > kSlices+1: at most 6.02 d 2^-58) and the digits past the
// last slice (d 2^-57) add at most 8.1 d 2^(e_q + e_x - 58) <= 4.1 d 2^-53 |q| |x|
// (2^e <= 4.02 max|x_k|), the order of the rounding of a d-term FP64
// accumulation; the FP64 recompute's bin sums then follow unchanged.  Items
// of 32 queries; their slices are staged in LDS.
struct GatheredS {
    int4_t xs[kSlices];  // this lane's 16 bytes of every slice of its column (A row lane % 16)
    double xn[4];        // |x|^2 of the lane's four result columns (padding: jj = INT32_MAX)
    int32_t jj[4];
    int32_t xe[4];       // their row exponents
    int32_t first, last;
};

template <int D4, bool SLICED>
struct GatherSel {
    using type = Gathered<D4>;
};
template <int D4>
struct GatherSel<D4, true> {
    using type = GatheredS;
};

template <int D4, int RQ, bool MULTI, int KIND = kKindGaussian, bool SLICED = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(exact_waves<D4>()))) void
kde_exact_kept_kernel(KdeArgs a, unsigned long long* __restrict__ next_item) {
    static_assert(!SLICED || (D4 == 16 && RQ == 2 && KIND == kKindGaussian && kSlices == 7),
                  "integer slices: 32 < d <= 64, 32-query items, Gaussian kernel");
    // queue length: fewer than 16 entries left over plus the columns of the
    // blocks one fill step takes (at least 17 blocks of 16 fit)
    constexpr int QN = 288;
    __shared__ int32_t queue_all[4][QN];
    // per wave: the FP32 query fragments, or the query slices ([qb][slice][lane] x 16 bytes)
    __shared__ float qf_all[4][SLICED ? RQ * kSlices * 64 * 4 : RQ * D4 * 64];
    __shared__ int32_t win_all[4][kBinWindow];
    __shared__ double exp_tab[256];
    load_exp2_table(exp_tab);
    const int lane = threadIdx.x & 63;
    int32_t* win = win_all[threadIdx.x >> 6];
    int32_t* queue = queue_all[threadIdx.x >> 6];
    float* qf = qf_all[threadIdx.x >> 6];  // [qb][kk][lane]
    const int64_t wave = (int64_t)blockIdx.x * 4 + uniform((int32_t)(threadIdx.x >> 6));  // wave-uniform
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    const int32_t n_items = *a.n_items;
    const int grp = lane >> 4;
    const int r = lane & 15;
    const int pr = perm_row(r);

    // items [0, n_waves) are taken in wave order, later ones from the counter
    int64_t it = wave;
    while (it < n_items) {
        // claim the next item now; the answer is needed only at the end
        unsigned long long claim = 0;
        if (lane == 0) claim = atomicAdd(next_item, 1ull);
        const WorkItem w = a.items[it];
        const SegDesc sg = a.segs[w.seg];
        const KdeArgs& J = MULTI ? a.jobs[sg.job] : a;
        // the set's arrays read per block, loaded once per item (a multi-set
        // table lives in global memory, which the bin stores could alias)
        const double* const Xp = J.Xp;
        const double* const xnorm = J.xnorm;
        const int8_t* const Xs = J.Xs;
        const int32_t* const xe = J.xe;
        const int32_t* bnd = J.bounds + sg.bound_off;
        const double s256 = 256.0 * J.s;  // exponent terms scaled by 256 for exp2_256_tab
        const double two_s = 2.0 * s256;
        double hq[RQ];
        int32_t selfv[RQ], smin[RQ], smax[RQ];
        double two_sq[RQ];  // 2 s 256 2^(e_q - 24): the slice sums' scale on the query side
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int qb = 0; qb < RQ; ++qb) {
            const int32_t t = 16 * qb + r;
            const bool ok = t < w.ne;
            const int64_t e = w.e0 + (ok ? t : 0);
            int32_t p = J.q_idx ? J.q_idx[e] : (int32_t)e;
            p = min(max(p, 0), (int32_t)(J.n_query - 1));
            int32_t sf = -1;
            if (ok) sf = (J.self_mode == SELF_POINT) ? p : ((J.self_mode == SELF_ARRAY) ? J.self_idx[e] : -1);
            selfv[qb] = sf;
            hq[qb] = (KIND == kKindExponential) ? J.qnorm[p] : -s256 * J.qnorm[p];
            if constexpr (SLICED) {
                const int8_t* qrow = J.Qs + (int64_t)p * kSliceRow + 16 * grp;
                int4_t* qs = (int4_t*)qf;
#pragma unroll
                for (int sa = 0; sa < kSlices; ++sa) qs[(qb * kSlices + sa) * 64 + lane] = *(const int4_t*)(qrow + 64 * sa);
                two_sq[qb] = __builtin_ldexp(two_s, J.qe[p] - 24);
            } else {
                double qv[D4];
                load_row_part<D4>(qv, J.Qp, p, grp);
#pragma unroll
                for (int kk = 0; kk < D4; ++kk) qf[(qb * D4 + kk) * 64 + lane] = (float)qv[kk];  // exact
            }
            int32_t mn = sf >= 0 ? sf : INT32_MAX, mx = sf;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                mn = min(mn, __shfl_xor(mn, off));
                mx = max(mx, __shfl_xor(mx, off));
            }
            smin[qb] = uniform(mn);
            smax[qb] = uniform(mx);
        }
        __builtin_amdgcn_wave_barrier();
        const int32_t col_end = uniform(min(max(bnd[w.b1], 0), (int32_t)J.n_data));
        const int32_t col_begin = uniform(min(max(bnd[w.b0], 0), col_end));
        // one open bin per lane with four query blocks, the four-bin shift
        // register with two
        typename std::conditional<RQ == 4, BinAccumulator1<RQ>, BinAccumulator<RQ>>::type bins;
        __builtin_amdgcn_wave_barrier();
        load_bin_window(win, bnd, w.b0, w.b1, lane);
        bins.init(bnd, win, w.b0, w.b1, col_begin, w.e0, w.ne, J.out_stride, J.out, J.out_rows, lane);
        const int64_t blk0 = col_begin >> 4;
        const int64_t blk1 = J.mask_by_item ? min((int64_t)(col_end + 15) >> 4, blk0 + J.n_blocks) : (col_end + 15) >> 4;
        const uint16_t* mrow =
            J.mask_by_item ? J.mask + it * J.n_blocks - blk0 : J.mask + (w.e0 / kTileQ) * J.n_blocks;

        // queue state (uniform): entries [head, tail) are pending
        int32_t head = 0, tail = 0;
        int64_t blk = blk0;  // next block whose mask is to be read
        // masks of a batch of 64 blocks (1024 columns): lane l holds block
        // blk + l; the next batch is loaded while this one is taken
        auto load_masks = [&](int64_t b) -> uint32_t {
            const int64_t mb = b + lane;
            return (mb < blk1) ? (uint32_t)mrow[mb] : 0u;
        };
        uint32_t masks = load_masks(blk);
        uint32_t masks_next = load_masks(blk + 64);

        // append the kept columns of further blocks (in index order) until 16
        // are pending or the range ends.  Lane l's columns go after those of
        // the lanes below it: the exclusive prefix of the per-lane counts is
        // formed bit by bit of the count (a ballot and a masked bit count per
        // bit).  The blocks taken are the longest prefix of the batch whose
        // columns fit the queue -- all 64 unless the masks are dense (at
        // least 17 always fit: fewer than 16 entries are pending).
        auto fill = [&]() {
            while (tail - head < 16 && blk < blk1) {
                if (head > 0) {  // move the fewer than 16 pending entries to the front
                    const int32_t left = tail - head;
                    const int32_t v = queue[head + (lane < left ? lane : 0)];
                    __builtin_amdgcn_wave_barrier();
                    if (lane < left) queue[lane] = v;
                    head = 0;
                    tail = left;
                }
                const int32_t c0 = (int32_t)((blk + lane) << 4);
                const int32_t lo = min(max(col_begin - c0, 0), 16), hi = min(max(col_end - c0, 0), 16);
                uint32_t bits = masks & ((1u << hi) - 1u) & ~((1u << lo) - 1u);
                const int32_t cnt = __popc(bits);
                int32_t excl = 0;
#pragma unroll
                for (int b = 0; b < 5; ++b) {
                    const uint64_t bk = __ballot((cnt >> b) & 1);
                    excl += (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(bk >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bk, 0u))
                            << b;
                }
                const int32_t incl = excl + cnt;
                const int32_t nb = (int32_t)__popcll(__ballot(incl <= QN - tail));  // >= 17
                if (lane < nb) {
                    int32_t pos = tail + excl;
                    while (bits) {
                        queue[pos++] = c0 + (int32_t)__builtin_ctz(bits);
                        bits &= bits - 1u;
                    }
                }
                tail += uniform(__builtin_amdgcn_readlane(incl, nb - 1));
                blk += nb;
                if (nb == 64) {
                    masks = masks_next;
                    masks_next = load_masks(blk + 64);
                } else {  // dense masks: reload from the first block not taken
                    masks = load_masks(blk);
                    masks_next = load_masks(blk + 64);
                }
            }
            __builtin_amdgcn_wave_barrier();
        };

        // gather the operands of the block of queue entries [pos, pos + cnt):
        // A row r holds entry perm_row(r), so that lane group g receives the
        // consecutive entries 4g .. 4g+3
        auto prepare = [&](Gathered<D4>& g, int32_t pos, int32_t cnt) {
            const int32_t gl = queue[pos + ((pr < cnt) ? pr : 0)];
            load_row_part<D4>(g.xf, Xp, gl, grp);
            g.first = uniform(queue[pos]);
            g.last = uniform(queue[pos + cnt - 1]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t idx = 4 * grp + i;
                g.jj[i] = (idx < cnt) ? queue[pos + idx] : INT32_MAX;
                const double v = xnorm[(idx < cnt) ? g.jj[i] : g.first];
                g.xn[i] = (idx < cnt) ? v : __builtin_inf();
            }
        };

        // the same for the slices: A row r holds queue entry r (the i32
        // result element i of lane group g is row 4g + i)
        auto prepare_s = [&](GatheredS& g, int32_t pos, int32_t cnt) {
            const int32_t gl = queue[pos + ((r < cnt) ? r : 0)];
            const int8_t* xrow = Xs + (int64_t)gl * kSliceRow + 16 * grp;
#pragma unroll
            for (int sb = 0; sb < kSlices; ++sb) g.xs[sb] = *(const int4_t*)(xrow + 64 * sb);
            g.first = uniform(queue[pos]);
            g.last = uniform(queue[pos + cnt - 1]);
            // padding positions read the last column; their |x|^2 becomes +inf
            // only where it is used, so that no wait for these loads comes
            // before the next block's products
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t idx = 4 * grp + i;
                const int32_t col = queue[pos + min(idx, cnt - 1)];
                g.jj[i] = (idx < cnt) ? col : INT32_MAX;
                g.xn[i] = xnorm[col];
                g.xe[i] = xe[col];
            }
        };

        // the 28 slice products of query block qb, the query slices read from
        // LDS one at a time: consecutive products go to different accumulators
        auto slice_products = [&](int4_t (&ac)[kSlices], int qb, const GatheredS& g) {
            const int4_t* qs = (const int4_t*)qf + qb * kSlices * 64 + lane;
#pragma unroll
            for (int k = 0; k < kSlices; ++k) ac[k] = int4_t{0, 0, 0, 0};
            int4_t q[kSlices];
#pragma unroll
            for (int sa = 0; sa < kSlices; ++sa) q[sa] = qs[sa * 64];
#pragma unroll
            for (int sa = 0; sa < kSlices; ++sa) {
#pragma unroll
                for (int sb = 0; sa + sb < kSlices; ++sb)
                    ac[sa + sb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(g.xs[sb], q[sa], ac[sa + sb], 0, 0, 0);
            }
        };
        // the kernel values of one query block from its slice sums (no
        // self-pair test; that follows for the whole block)
        auto slice_values = [&](const int4_t (&ac)[kSlices], int qb, const GatheredS& g, const double (&xn)[4],
                                double (&kvq)[4]) {
            double rr[4], t[4];
            int32_t mi[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // groups 2k and 2k+1 joined exactly in 32 bits (|group| < 7 2^20);
                // group 2k+1 has weight 2^-8(2k+3), the last group 2^-64
                int32_t pr[3];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    pr[k] = (int32_t)(((uint32_t)ac[2 * k][i] << 8) + (uint32_t)ac[2 * k + 1][i]);
                double v = __builtin_fma((double)pr[1], 0x1p-16, (double)pr[0]);
                v = __builtin_fma((double)pr[2], 0x1p-32, v);
                v = __builtin_fma((double)ac[6][i], 0x1p-40, v);
                v = __builtin_ldexp(v, g.xe[i]);
                mi[i] = exp2_256_split(pair_exponent<KIND>(v, hq[qb], xn[i], -s256, two_sq[qb]), &rr[i]);
                t[i] = exp_tab[mi[i] & 255];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) kvq[i] = exp2_256_join(t[i], rr[i], mi[i]);
        };

        auto slice_values2 = [&](const int4_t (&ac)[RQ][kSlices], const GatheredS& g, const double (&xn)[4],
                                 double (&kvq)[RQ][4]) {
            double rr[RQ][4], t[RQ][4];
            int32_t mi[RQ][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
                for (int qb = 0; qb < RQ; ++qb) {
                    int32_t pr[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        pr[k] = (int32_t)(((uint32_t)ac[qb][2 * k][i] << 8) + (uint32_t)ac[qb][2 * k + 1][i]);
                    double v = __builtin_fma((double)pr[1], 0x1p-16, (double)pr[0]);
                    v = __builtin_fma((double)pr[2], 0x1p-32, v);
                    v = __builtin_fma((double)ac[qb][6][i], 0x1p-40, v);
                    v = __builtin_ldexp(v, g.xe[i]);
                    mi[qb][i] = exp2_256_split(pair_exponent<KIND>(v, hq[qb], xn[i], -s256, two_sq[qb]), &rr[qb][i]);
                    t[qb][i] = exp_tab[mi[qb][i] & 255];
                }
            }
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb)
#pragma unroll
                for (int i = 0; i < 4; ++i) kvq[qb][i] = exp2_256_join(t[qb][i], rr[qb][i], mi[qb][i]);
        };

        auto compute_s = [&](const GatheredS& g) {
            double kv[RQ][4];
            double xn[4];  // padding columns: |x|^2 = +inf gives exponent -inf and value 0
#pragma unroll
            for (int i = 0; i < 4; ++i) xn[i] = (g.jj[i] == INT32_MAX) ? __builtin_inf() : g.xn[i];
            // both query blocks' products first, then their values together
            // (eight independent chains per lane)
            int4_t acc[RQ][kSlices];
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb) slice_products(acc[qb], qb, g);
            slice_values2(acc, g, xn, kv);
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb) {
                if (smax[qb] >= g.first && smin[qb] <= g.last &&
                    __ballot(selfv[qb] >= g.first && selfv[qb] <= g.last) != 0) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (g.jj[i] == selfv[qb]) kv[qb][i] = 0.0;
                }
            }
            bins.add(kv, g.jj, g.last);
        };

        auto compute = [&](const Gathered<D4>& g) {
            // padding columns: |x|^2 = +inf gives exponent -inf and value 0
            double4_t c[RQ];
#pragma unroll
            for (int qb = 0; qb < RQ; ++qb) {
                double qv[D4];
#pragma unroll
                for (int kk = 0; kk < D4; ++kk) qv[kk] = (double)qf[(qb * D4 + kk) * 64 + lane];
                c[qb] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < D4; ++kk) c[qb] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.xf[kk], qv[kk], c[qb], 0, 0, 0);
            }
            double kv[RQ][4];
            exact_values<RQ, true, true, KIND>(c, hq, g.xn, -s256, two_s, g.jj, selfv, smin, smax, g.first, g.last,
                                               exp_tab, kv);
            bins.add(kv, g.jj, g.last);
        };

        fill();
        if (tail > head) {
            // two operand buffers in turn: the next block gathers while this
            // one computes
            typename GatherSel<D4, SLICED>::type g0, g1;
            auto prep_any = [&](typename GatherSel<D4, SLICED>::type& g, int32_t pos, int32_t cnt) {
                if constexpr (SLICED)
                    prepare_s(g, pos, cnt);
                else
                    prepare(g, pos, cnt);
            };
            auto compute_any = [&](const typename GatherSel<D4, SLICED>::type& g) {
                if constexpr (SLICED)
                    compute_s(g);
                else
                    compute(g);
            };
            int32_t n0 = min(16, tail - head);
            prep_any(g0, head, n0);
            head += n0;
            while (true) {
                fill();
                const int32_t n1 = min(16, tail - head);
                if (n1 > 0) {
                    prep_any(g1, head, n1);
                    head += n1;
                }
                compute_any(g0);
                if (n1 == 0) break;
                fill();
                const int32_t n2 = min(16, tail - head);
                if (n2 > 0) {
                    prep_any(g0, head, n2);
                    head += n2;
                }
                compute_any(g1);
                if (n2 == 0) break;
            }
        }
        bins.finish();
        it = n_waves + (int64_t)(uint32_t)uniform((int32_t)(uint32_t)__shfl(claim, 0));
    }
}

// ---------------------------------------------------------------------------
// Keep masks of a later pass.  A sample's pairs that the root pass dropped --
// pairs more than Delta below the largest term of the sample's point's row --
// stay dropped at every deeper level: their total over the whole row is below
// e^-25 of the degree (n e^-Delta), so a walk that reaches a node through
// them, or whose branch they would change, has probability below that bound
// at each level.  The root pass's masks are per 64-entry tile of the pivot
// order: a sample reads the row of its point's tile, a superset of the
// point's own kept columns.  One wave per work item, a lane per block; the
// union over the item's entries skips repeated tiles (the entries are sorted
// by pivot position within their node).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pass_mask_kernel(KdeArgs a, const int32_t* __restrict__ inv,
                                                        const uint16_t* __restrict__ root_mask, int64_t root_blocks,
                                                        int32_t W, uint16_t* __restrict__ pmask) {
    const int64_t it = (int64_t)blockIdx.x * 4 + uniform((int32_t)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (it >= *a.n_items) return;
    const WorkItem w = a.items[it];
    const SegDesc sg = a.segs[w.seg];
    const int32_t* bnd = a.bounds + sg.bound_off;
    const int32_t col_end = uniform(min(max(bnd[w.b1], 0), (int32_t)a.n_data));
    const int32_t col_begin = uniform(min(max(bnd[w.b0], 0), col_end));
    const int64_t wb = col_begin >> 4;
    const int32_t nblk = (int32_t)(((col_end + 15) >> 4) - wb);
    // lane t: the root tile of entry t; the first entry of each run of equal
    // tiles marks it (entries are sorted by pivot position)
    const int32_t rt_l = (lane < w.ne) ? inv[a.q_idx[w.e0 + lane]] / kTileQ : -1;
    const int32_t rt_prev = __shfl_up(rt_l, 1);
    const uint64_t first = __ballot(lane < w.ne && (lane == 0 || rt_l != rt_prev));
    for (int32_t k0 = 0; k0 < W; k0 += 64) {
        const int32_t k = k0 + lane;
        const bool in = k < nblk && k < W;
        uint32_t acc = 0;
        // eight distinct tiles at a time, their loads in flight together
        uint64_t m = first;
        while (m) {
            int32_t rts[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                rts[u] = -1;
                if (m) {
                    const int32_t src = (int32_t)__builtin_ctzll(m);
                    m &= m - 1ull;
                    rts[u] = __builtin_amdgcn_readlane(rt_l, src);
                }
            }
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = (in && rts[u] >= 0) ? root_mask[(int64_t)rts[u] * root_blocks + wb + k] : 0u;
#pragma unroll
            for (int u = 0; u < 8; ++u) acc |= v[u];
        }
        if (k < W) pmask[it * W + k] = (uint16_t)acc;
    }
}

hipError_t launch_pass_mask(const KdeArgs& a, int64_t max_items, const int32_t* inv, const uint16_t* root_mask,
                            int64_t root_blocks, int32_t W, uint16_t* pmask, hipStream_t st) {
    if (max_items <= 0) return hipSuccess;
    if (W < 1) return hipErrorInvalidValue;
    pass_mask_kernel<<<(unsigned)((max_items + 3) / 4), 256, 0, st>>>(a, inv, root_mask, root_blocks, W, pmask);
    return hipGetLastError();
}

template <int D4>
static hipError_t launch_exact_t(const KdeArgs& a, int64_t max_items, unsigned long long* next_item, int num_cus,
                                 hipStream_t st) {
    if constexpr (D4 == 16) {
        if (a.Xs && a.Qs && a.kind == kKindGaussian) {
            int64_t waves = (int64_t)num_cus * 8;
            if (max_items < waves) waves = max_items;
            if (waves < 1) waves = 1;
            const unsigned blocks = (unsigned)((waves + 3) / 4);
            if (a.jobs)
                kde_exact_kept_kernel<16, 2, true, kKindGaussian, true><<<blocks, 256, 0, st>>>(a, next_item);
            else
                kde_exact_kept_kernel<16, 2, false, kKindGaussian, true><<<blocks, 256, 0, st>>>(a, next_item);
            return hipGetLastError();
        }
    }
    int64_t waves = (int64_t)num_cus * 8;
    if (max_items < waves) waves = max_items;
    if (waves < 1) waves = 1;
    // 32-entry items for d > 64 (exact_tile), whose FP64 query fragments
    // would not fit the LDS at 64
    constexpr int RQ = D4 >= 32 ? 2 : 4;
    if (a.kind == kKindExponential) {
        if (a.jobs) return hipErrorInvalidValue;  // multi-set launches are Gaussian only
        kde_exact_kept_kernel<D4, RQ, false, kKindExponential><<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(a,
                                                                                                          next_item);
    } else if (a.jobs) {
        kde_exact_kept_kernel<D4, RQ, true><<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(a, next_item);
    } else {
        kde_exact_kept_kernel<D4, RQ, false><<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(a, next_item);
    }
    return hipGetLastError();
}

hipError_t launch_exact_kept(const KdeArgs& a, int64_t max_items, unsigned long long* next_item, int num_cus,
                             hipStream_t st) {
    switch (a.D4) {
        case 1: return launch_exact_t<1>(a, max_items, next_item, num_cus, st);
        case 2: return launch_exact_t<2>(a, max_items, next_item, num_cus, st);
        case 4: return launch_exact_t<4>(a, max_items, next_item, num_cus, st);
        case 8: return launch_exact_t<8>(a, max_items, next_item, num_cus, st);
        case 16: return launch_exact_t<16>(a, max_items, next_item, num_cus, st);
        case 32: return launch_exact_t<32>(a, max_items, next_item, num_cus, st);
        default: return hipErrorInvalidValue;
    }
}

int exact_tile(int D4, bool sliced) { return (D4 >= 32 || sliced) ? 32 : 64; }

}  // namespace fsg
