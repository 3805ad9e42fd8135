// Keep masks of the precision mode (stage 1 of the filtered segmented KDE):
// per 64-query tile and 16-column data block, which columns the exact pass
// must recompute.  The cross terms come from BF16 hi/lo split operands on the
// BF16 matrix cores (one contraction over K = 3d gives hi.hi + hi.lo + lo.hi,
// accumulated in FP32); each accumulator starts at minus the query's keep
// threshold, so that a column is kept when the largest of a lane's 16 results
// reaches -|x|^2/2 (the threshold and its error bound are derived beside the
// exact pass, in kde_filter.hip).
//
// Built with the compiler's VGPR form of the matrix ops (see build.py): the
// variants that run one wave per SIMD keep their query fragments in the
// accumulation registers, and the cross terms, which the keep test reads with
// vector ops, in vector registers.
#include "common.h"
#include "device.h"

namespace fsg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Stage 1: keep masks.  For query tile t (64 entries) and data block b (16
// columns) mask[t * n_blocks + b] has bit c set when column 16b + c is kept
// for at least one query of the tile.  Work item = (group of tiles, run of
// blocks); the operands of later blocks load while the current one is
// processed.
// ---------------------------------------------------------------------------
// occupancy targets that fit without spilling (measured on the MI355X: two
// tiles per item at these occupancies beat one tile at three or two waves)
template <int KB>
constexpr int mask_waves() { return KB <= 3 ? 2 : 1; }

int64_t keep_mask_waves(int KB, int num_cus) {
    switch (KB) {
        case 1: return (int64_t)num_cus * 4 * mask_waves<1>();
        case 2: return (int64_t)num_cus * 4 * mask_waves<2>();
        case 3: return (int64_t)num_cus * 4 * mask_waves<3>();
        case 6: return (int64_t)num_cus * 4 * mask_waves<6>();
        default: return (int64_t)num_cus * 4 * mask_waves<12>();
    }
}

// Word 3 of a raw buffer resource on gfx9-family parts: 32-bit data format,
// no swizzle, no index stride.
constexpr int kBufferFlags = 0x00020000;

// Work items: MODE 0 = (tile group, chunk of blocks) of one point set; 1 =
// the same over the point sets of a multi-set launch; 2 = a list of
// {first tile, first block, end block} (the pruned scan over the data in
// pivot order), cut into one segment per XCD: the waves of the workgroups
// an XCD runs (blockIdx % kXcds) take its segment, so that each L2 holds the
// data chunks of its own segment only.
template <int KB, int TP, int WAVES, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) void kde_keep_mask_kernel(MaskArgs m0) {
    constexpr bool MULTI = MODE == 1;
    // Queries are the A operand and data the B operand, so lane l receives
    // query rows 4(l/16) + i of a query block and data column l % 16: a column
    // is kept for a tile when any of the 4 lane groups sees a compare succeed
    // in one of the tile's four query blocks.  A work item covers TP
    // consecutive tiles, so that every data operand loaded feeds 4 TP matrix
    // ops per K step.
    constexpr int QB = 4 * TP;
    const int lane = threadIdx.x & 63;
    int64_t wave = (int64_t)blockIdx.x * 4 + uniform((int32_t)(threadIdx.x >> 6));  // wave-uniform
    int64_t n_waves = (int64_t)gridDim.x * 4;
    int64_t it0 = 0, n_items;
    if constexpr (MODE == 2) {  // the grid is a multiple of kXcds workgroups
        const int32_t x = (int32_t)(blockIdx.x % kXcds);
        wave = (int64_t)(blockIdx.x / kXcds) * 4 + uniform((int32_t)(threadIdx.x >> 6));
        n_waves = (int64_t)(gridDim.x / kXcds) * 4;
        it0 = m0.xseg[x];
        n_items = m0.xseg[x + 1];
    } else {
        n_items = MULTI ? m0.n_items_total : mask_items(m0);
    }
    const int grp = lane >> 4;
    const int r = lane & 15;
    int64_t kept = 0;
    for (int64_t it = it0 + wave; it < n_items; it += n_waves) {
        int64_t local = it;
        int32_t job = 0;
        if (MULTI) {  // the point set owning item it (uniform binary search)
            int32_t lo = 0, hi = m0.n_jobs;
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (m0.job_item_off[mid] <= it) lo = mid; else hi = mid;
            }
            job = lo;
            local = it - m0.job_item_off[job];
        }
        const MaskArgs& m = MULTI ? m0.jobs[job] : m0;
        int64_t tile0;
        int32_t bb, be;  // the item's blocks [bb, be)
        if constexpr (MODE == 2) {
            const int32_t* li = m.list + 3 * it;
            tile0 = li[0];
            bb = li[1];
            be = li[2];
        } else {
            // block indices fit in 32 bits (n < 2^31 columns), so that the
            // loop control stays on the scalar unit
            const int64_t n_groups = (m.n_tiles + TP - 1) / TP;
            const int64_t chunk = local / n_groups;
            tile0 = (local - chunk * n_groups) * TP;
            bb = (int32_t)(chunk * m.blocks_per_chunk);
            be = (int32_t)min(m.n_blocks, (int64_t)bb + m.blocks_per_chunk);
        }
        const int64_t e0 = tile0 * kTileQ;
        const int32_t ne = (int32_t)min((int64_t)(TP * kTileQ), m.n_entries - e0);
        bf16x8_t qb16[QB][KB];
        // minus the keep-thresholds of result rows 4(l/16)+i of each query
        // block (consecutive entries; -inf past the last): the accumulators
        // start there
        float4_t ntheta[QB];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            // operand rows: entries e0 + 16 qb .. (fragments in entry order)
            const bf16x8_t* bsrc = (const bf16x8_t*)m.Qb + ((e0 >> 4) + qb) * KB * 64 + lane;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                qb16[qb][kb] = bsrc[kb * 64];
                // one wave per SIMD: the query fragments, read only by the
                // matrix ops, go to the accumulation registers
                if constexpr (WAVES == 1) asm volatile("" : "+a"(qb16[qb][kb]));
            }
            ntheta[qb] = *(const float4_t*)(m.ntheta + e0 + 16 * qb + 4 * grp);
        }
        __builtin_amdgcn_wave_barrier();
        const int32_t n_data = (int32_t)m.n_data;
        const int32_t n_live = (int32_t)min((int64_t)TP, m.n_tiles - tile0);  // tiles of this item that exist
        uint16_t* mrow = m.mask + tile0 * m.n_blocks;
        const int64_t mstride = m.n_blocks;
        // the operands of block b: split data rows and -|x|^2/2 of this lane's
        // column, as buffer loads from the chunk's first block with the
        // block's offset in a scalar register (the lane offsets stay constant,
        // so the loop does no vector address arithmetic); a chunk spans at
        // most a few MB, well inside the 32-bit offsets
        const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)((const char*)m.Xb + (int64_t)bb * (KB * 1024)), (short)0, 0x7fffffff, kBufferFlags);
        const __amdgpu_buffer_rsrc_t ars =
            __builtin_amdgcn_make_buffer_rsrc((void*)(m.xa + (int64_t)bb * 16), (short)0, 0x7fffffff, kBufferFlags);
        auto load = [&](bf16x8_t (&x)[KB], float& xa, int32_t blk) {
            const int32_t rel = blk - bb;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(xrs, kb * 1024 + lane * 16, rel * (KB * 1024), 0);
                x[kb] = __builtin_bit_cast(bf16x8_t, v);
            }
            xa = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ars, r * 4, rel * 64, 0));
        };
        // lane (b mod 64) keeps the masks of block b until 64 blocks are ready
        uint32_t pending[TP];
#pragma unroll
        for (int h = 0; h < TP; ++h) pending[h] = 0;
        // cross terms of one block: independent accumulators, K step outer,
        // so that no matrix op waits for the previous one's result
        auto mma = [&](float4_t (&cc)[QB], const bf16x8_t (&x)[KB]) {
#pragma unroll
            for (int qb = 0; qb < QB; ++qb)
                cc[qb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qb16[qb][0], x[0], ntheta[qb], 0, 0, 0);
#pragma unroll
            for (int kb = 1; kb < KB; ++kb)
#pragma unroll
                for (int qb = 0; qb < QB; ++qb)
                    cc[qb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qb16[qb][kb], x[kb], cc[qb], 0, 0, 0);
        };
        // keep bits of one block from its cross terms
        auto finish = [&](const float4_t (&cc)[QB], float xa, int32_t blk) {
            const uint32_t tail = (16 * (blk + 1) > n_data) ? (1u << (n_data - 16 * blk)) - 1u : 0xFFFFu;
#pragma unroll
            for (int h = 0; h < TP; ++h) {
                // the lane's 16 results all belong to its one data column:
                // a column is kept when the largest of them reaches |x|^2/2
                // (the NaN-propagating maximum needs no canonicalising of its
                // operands; the operands are finite or -inf)
                float dm = cc[4 * h][0];
#pragma unroll
                for (int qb = 4 * h; qb < 4 * h + 4; ++qb)
#pragma unroll
                    for (int i = (qb == 4 * h) ? 1 : 0; i < 4; ++i) dm = __builtin_elementwise_maximum(dm, cc[qb][i]);
                const uint64_t any = __ballot(dm >= -xa);
                const uint32_t keep = (uint32_t)((any | (any >> 16) | (any >> 32) | (any >> 48)) & tail);
                kept += __popc(keep);
                // lane blk % 64 takes the (uniform) keep bits
                pending[h] = writelane_u32(keep, (uint32_t)(blk & 63), pending[h]);
            }
            if ((blk & 63) == 63 || blk + 1 == be) {
                const int32_t b = (blk & ~63) + lane;
                if (b >= bb && b <= blk) {
#pragma unroll
                    for (int h = 0; h < TP; ++h)
                        if (h < n_live) mrow[h * mstride + b] = (uint16_t)pending[h];
                }
            }
        };
        // Software pipeline over the blocks.  Past the end the last block is
        // loaded and multiplied again (in bounds, results unused), so that
        // every step issues the same instructions.
        auto clampb = [&](int32_t b) { return b < be ? b : be - 1; };
        bf16x8_t x0[KB], x1[KB], x2[KB], x3[KB];
        float a0, a1, a2, a3;
        float4_t c0[QB], c1[QB];
        float f0, f1;  // -|x|^2/2 of the blocks whose keep bits are taken next
        int32_t blk = bb;
        if constexpr (WAVES == 2) {
            // Two waves per SIMD: one accumulator set, whose keep bits are
            // taken right after its matrix ops (the other wave's matrix ops
            // fill the wait), which leaves the registers for four operand
            // buffers: the loads run four blocks ahead.
            load(x0, a0, bb);
            load(x1, a1, clampb(bb + 1));
            load(x2, a2, clampb(bb + 2));
            load(x3, a3, clampb(bb + 3));
            auto step = [&](bf16x8_t (&xb)[KB], float& ab) {
                mma(c0, xb);
                f0 = ab;
                load(xb, ab, clampb(blk + 4));
                finish(c0, f0, blk);
            };
            for (;;) {
                step(x0, a0);
                if (++blk >= be) break;
                step(x1, a1);
                if (++blk >= be) break;
                step(x2, a2);
                if (++blk >= be) break;
                step(x3, a3);
                if (++blk >= be) break;
            }
        } else {
            // One wave per SIMD: the matrix ops of block b + 1 are issued
            // before the keep bits of block b are taken (two accumulator
            // sets), and the operands of block b + 3 load meanwhile (three
            // buffers in turn: a load has two blocks' worth of matrix work to
            // arrive; four buffers were slower).
            // one step: load block blk + 3 into the free buffer xl, multiply
            // block blk + 1 (buffer xm) into cm, take the keep bits of block blk (cf)
            auto step = [&](bf16x8_t (&xl)[KB], float& al, const bf16x8_t (&xm)[KB], float am, float4_t (&cm)[QB],
                            float& fm, const float4_t (&cf)[QB], float ff) {
                load(xl, al, clampb(blk + 3));
                mma(cm, xm);
                fm = am;
                finish(cf, ff, blk);
            };
            load(x0, a0, bb);
            load(x1, a1, clampb(bb + 1));
            load(x2, a2, clampb(bb + 2));
            mma(c0, x0);
            f0 = a0;
            for (;;) {
                step(x0, a0, x1, a1, c1, f1, c0, f0);
                if (++blk >= be) break;
                step(x1, a1, x2, a2, c0, f0, c1, f1);
                if (++blk >= be) break;
                step(x2, a2, x0, a0, c1, f1, c0, f0);
                if (++blk >= be) break;
                step(x0, a0, x1, a1, c0, f0, c1, f1);
                if (++blk >= be) break;
                step(x1, a1, x2, a2, c1, f1, c0, f0);
                if (++blk >= be) break;
                step(x2, a2, x0, a0, c0, f0, c1, f1);
                if (++blk >= be) break;
            }
        }
    }
    if (m0.kept != nullptr && lane == 0 && kept > 0) atomicAdd((unsigned long long*)m0.kept, (unsigned long long)kept);
}

// Minus the keep-threshold of every entry:
//     theta_q = |q|^2/2 - T_q/2 - E,  T_q = dmin_q (1 + 1e-6) + Delta/gamma
// (Gaussian kernel; for the exponential kernel T_q = (sqrt(dmin_q (1 + 1e-6))
// + Delta/gamma)^2, whose square root is the largest distance a kept pair
// can have),
//     E = eps (|q| xmax + xmax^2/2),
// in FP64, then rounded down to FP32 (the test c~ - theta_q >= |x|^2/2 only
// keeps more); entries past the last get -inf (never kept).
__global__ void mask_theta_kernel(MaskArgs m, float* __restrict__ out, int64_t n_out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n_out) return;
    if (e >= m.n_entries) {
        out[e] = -__builtin_inff();
        return;
    }
    int32_t p = m.q_idx ? m.q_idx[e] : (int32_t)e;
    p = min(max(p, 0), (int32_t)(m.n_query - 1));
    const double xmax = *m.xmax;
    const double nq = m.qnorm[p];
    const double err = m.eps * (__builtin_sqrt(nq) * xmax + 0.5 * xmax * xmax);
    // Gaussian: T = dmin (1 + 1e-6) + Delta/gamma; exponential: the squared
    // distance whose square root is Delta/gamma beyond sqrt(dmin (1 + 1e-6))
    const double th = (m.kind == kKindExponential)
                          ? 0.5 * nq - 0.5 * keep_dist2(m.kind, m.dmin[p] * (1.0 + 1e-6), m.margin_z, m.gamma) - err
                          : 0.5 * nq - 0.5 * m.dmin[p] * (1.0 + 1e-6) - m.margin_z / (2.0 * m.gamma) - err;
    float thf = (float)th;
    if ((double)thf > th) {  // step one FP32 ulp down
        int32_t bits = __float_as_int(thf);
        bits = (thf > 0.0f) ? bits - 1 : ((thf < 0.0f) ? bits + 1 : (int32_t)0x80000001);
        thf = __int_as_float(bits);
    }
    out[e] = -thf;
}

hipError_t launch_mask_theta(const MaskArgs& m, float* out, int64_t n_out, hipStream_t st) {
    if (n_out < m.n_entries || n_out % kThetaPad != 0) return hipErrorInvalidValue;
    if (n_out == 0) return hipSuccess;
    mask_theta_kernel<<<(unsigned)((n_out + 255) / 256), 256, 0, st>>>(m, out, n_out);
    return hipGetLastError();
}

template <int KB>
static hipError_t launch_mask_t(const MaskArgs& m, int num_cus, hipStream_t st) {
    constexpr int TP = mask_tiles_per_item(KB), WAVES = mask_waves<KB>();
    static_assert(kThetaPad % (TP * kTileQ) == 0, "threshold padding must hold whole tile groups");
    const int64_t n_items = m.jobs ? m.n_items_total : mask_items(m);
    int64_t waves = (int64_t)num_cus * 4 * WAVES;
    if (n_items < waves) waves = n_items;
    if (waves < 1) waves = 1;
    if (m.list) {
        // the item count is on the device: every wave slot of the chip, in a
        // whole number of workgroups per XCD
        const int64_t per_xcd = ((int64_t)num_cus * WAVES + kXcds - 1) / kXcds;
        kde_keep_mask_kernel<KB, TP, WAVES, 2><<<(unsigned)(per_xcd * kXcds), 256, 0, st>>>(m);
    } else if (m.jobs) {
        kde_keep_mask_kernel<KB, TP, WAVES, 1><<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(m);
    } else {
        kde_keep_mask_kernel<KB, TP, WAVES, 0><<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(m);
    }
    return hipGetLastError();
}

hipError_t launch_keep_mask(const MaskArgs& m, int num_cus, hipStream_t st) {
    switch (m.KB) {
        case 1: return launch_mask_t<1>(m, num_cus, st);
        case 2: return launch_mask_t<2>(m, num_cus, st);
        case 3: return launch_mask_t<3>(m, num_cus, st);
        case 6: return launch_mask_t<6>(m, num_cus, st);
        case 12: return launch_mask_t<12>(m, num_cus, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fsg
