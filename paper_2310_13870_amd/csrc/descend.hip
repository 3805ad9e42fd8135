// Randomised tree descent (hot-path step "descent"; Algorithm 1's branch on r,
// Section 4.1).  Two stages:
//  * after a binned KDE pass, each entry's 2^D bin masses form the leaves of a
//    perfect binary sum tree (built in LDS); every sample of the entry walks D
//    levels down it, one Philox uniform per level;
//  * the leaf stage resolves nodes of at most 64 points directly: a wave takes
//    up to 64 samples that sit in the same node, evaluates the kernel of each
//    sample's point against every point of the node (FP64, as the binned
//    passes do: |q|^2 + |x|^2 - 2 q.x and the table exponential), keeps the
//    row in registers, and each lane walks its own sample to a leaf.
#include <type_traits>

#include "common.h"
#include "device.h"
#include "kde_epilogue.h"

namespace fsg {

// The descent rule of Algorithm 1 at one node: left iff u*(mL+mR) < mL, never
// into a child of zero mass.  Returns true for left.  With want_margin (a
// uniform flag: the caller keeps margins) *mg becomes min(*mg, |u - mL/t|);
// without it the division is skipped.
__device__ __forceinline__ bool choose_left(double u, double mL, double mR, bool want_margin, float* mg) {
    const double t = mL + mR;
    bool left = (u * t < mL);
    if (left && mL == 0.0) left = false;
    if (!left && mR == 0.0) left = true;
    if (want_margin) *mg = fminf(*mg, (float)__builtin_fabs(u - mL / t));
    return left;
}

// Root pass: one block of 256 threads per point.  LDS holds the sum tree
// (2^D doubles) and the Philox blocks of up to 64 of the point's samples.
constexpr int kDescThreads = 256;
constexpr int kDescChunk = 64;

// Philox level groups a root descent draws from (the levels it resolves)
__host__ __device__ inline int32_t desc_groups(const DescArgs& a) {
    const int32_t last_level = a.start_level + a.D - 1;
    return (last_level >> 2) - (a.start_level >> 2) + 1;
}

// MULTI: the entries of several point sets' root passes (a0.jobs), one
// block per entry as for one set.
template <bool MULTI>
__global__ __launch_bounds__(kDescThreads) void descend_root_kernel(DescArgs a0, int32_t n_groups0) {
    // LDS: the internal nodes of the sum tree, tree[k] for k in [1, 2^D)
    // (children 2k, 2k+1; the bins are the leaves 2^D + b and stay in global
    // memory), then the Philox blocks of up to 64 samples.
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    for (int64_t ge = blockIdx.x; ge < a0.n_entries; ge += gridDim.x) {
        int64_t e = ge;
        int32_t job = 0;
        if (MULTI) {  // the point set owning entry ge (uniform binary search)
            int32_t lo = 0, hi = a0.n_jobs;
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (a0.job_entry_off[mid] <= ge) lo = mid; else hi = mid;
            }
            job = lo;
            e = ge - a0.job_entry_off[job];
        }
        const DescArgs& a = MULTI ? a0.jobs[job] : a0;
        const int32_t n_groups = MULTI ? desc_groups(a) : n_groups0;
        const int32_t nb = 1 << a.D;
        double* tree = smem;
        uint64_t* words = (uint64_t*)(smem + nb);  // [kDescChunk][n_groups][4]
        const int32_t g0 = a.start_level >> 2;
        // bins summed per thread in registers before the LDS levels
        const int32_t per = (nb >= 8 * kDescThreads) ? 8 : ((nb >= 2 * kDescThreads) ? nb / kDescThreads : 1);
        const double* M = a.M + e * nb;
        int32_t top;  // the LDS levels built below start at nodes [top, 2 top)
        if (per >= 2) {
            // thread t owns bins [per t, per t + per): its local subtree
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = (k < per) ? M[tid * per + k] : 0.0;
            int32_t cnt = per, lvl_nodes = nb;  // nodes on the current level
            while (cnt > 1) {
                cnt >>= 1;
                lvl_nodes >>= 1;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < cnt) v[k] = v[2 * k] + v[2 * k + 1];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < cnt) tree[lvl_nodes + tid * cnt + k] = v[k];
            }
            top = lvl_nodes;  // = nb / per = number of threads that own bins
        } else {
            // fewer bins than 2 per thread: the first internal level from global
            for (int32_t k = tid; k < nb / 2; k += kDescThreads) tree[nb / 2 + k] = M[2 * k] + M[2 * k + 1];
            top = nb / 2;
        }
        __syncthreads();
        for (int32_t cnt = top >> 1; cnt >= 1; cnt >>= 1) {
            for (int32_t k = tid; k < cnt; k += kDescThreads) tree[cnt + k] = tree[2 * (cnt + k)] + tree[2 * (cnt + k) + 1];
            __syncthreads();
        }
        const double root = (nb >= 2) ? tree[1] : M[0];
        if (a.deg != nullptr && tid == 0) a.deg[e] = root;
        for (int32_t c0 = 0; c0 < a.L; c0 += kDescChunk) {
            const int32_t cn = min(kDescChunk, a.L - c0);
            // Philox blocks of every (sample, level group) of this chunk, spread over the block
            for (int32_t c = tid; c < cn * n_groups; c += kDescThreads) {
                const int32_t k = c / n_groups, g = g0 + (c - k * n_groups);
                const PhiloxWords w = philox4x64_10((uint64_t)e, (uint64_t)(c0 + k), (uint64_t)g, 0, a.seed, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) words[c * 4 + q] = w.w[q];
            }
            __syncthreads();
            if (tid < cn) {
                const int32_t l = c0 + tid;
                const int64_t smp = e * a.L + l;
                const uint64_t* wk = words + (int64_t)tid * n_groups * 4;
                if (!(root > 0.0)) {
                    a.node[smp] = -1;  // isolated point: no neighbour
                } else {
                    float mg = (a.margin != nullptr) ? a.margin[smp] : 0.0f;
                    int32_t m = 0;
                    for (int32_t t = 0; t < a.D; ++t) {
                        const int32_t level = a.start_level + t;
                        const double u = word_to_uniform(wk[((level >> 2) - g0) * 4 + (level & 3)]);
                        const int32_t c = (1 << (t + 1)) + 2 * m;
                        double mL, mR;
                        if (t + 1 < a.D) {
                            mL = tree[c];
                            mR = tree[c + 1];
                        } else {
                            mL = M[2 * m];  // the children are bins
                            mR = M[2 * m + 1];
                        }
                        const bool left = choose_left(u, mL, mR, a.margin != nullptr, &mg);
                        m = 2 * m + (left ? 0 : 1);
                    }
                    a.node[smp] = m;
                    if (a.margin != nullptr) a.margin[smp] = mg;
                }
            }
            __syncthreads();
        }
    }
}

// Root pass with 2^D <= 1024 bins: one wave per point (four per block, each
// with its own LDS), so that four times as many points are in flight and no
// block-wide barrier is needed.  Lane t sums its 2^D / 64 consecutive bins in
// registers; every internal node is the sum of its two children, as in
// descend_root_kernel, so the trees (and the walks) are the same bit for bit.
// MULTI: entries of several sets (a0.jobs), each wave's LDS region sized by
// a0.lds_bytes (the largest set's).
constexpr int kWaveRootMaxD = 10;

template <bool MULTI>
__global__ __launch_bounds__(256) void descend_root_wave_kernel(DescArgs a0, int32_t n_groups0) {
    extern __shared__ double smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    for (int64_t ge = (int64_t)blockIdx.x * 4 + wv; ge < a0.n_entries; ge += n_waves) {
        int64_t e = ge;
        int32_t job = 0;
        if (MULTI) {  // the point set owning entry ge (uniform binary search)
            int32_t lo = 0, hi = a0.n_jobs;
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (a0.job_entry_off[mid] <= ge) lo = mid; else hi = mid;
            }
            job = lo;
            e = ge - a0.job_entry_off[job];
        }
        // a copy: the stores below could alias a job table in global memory
        const DescArgs a = MULTI ? a0.jobs[job] : a0;
        const int32_t n_groups = MULTI ? desc_groups(a) : n_groups0;
        const int32_t nb = 1 << a.D;
        const int32_t chunk = a.L < kDescChunk ? a.L : kDescChunk;
        // per wave: tree[k], k in [1, nb), then the Philox blocks of its chunk
        const size_t region = MULTI ? a0.lds_bytes / sizeof(double) : (size_t)nb + (size_t)4 * chunk * n_groups;
        double* tree = smem + (size_t)wv * region;
        uint64_t* words = (uint64_t*)(tree + nb);
        const int32_t g0 = a.start_level >> 2;
        const int32_t per = nb >= 64 ? nb / 64 : 1;  // bins per lane (<= 16)
        const double* M = a.M + e * nb;
        int32_t top;  // the LDS levels built below start at nodes [top, 2 top)
        if (nb >= 2) {
            double v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = (k < per && lane * per + k < nb) ? M[lane * per + k] : 0.0;
            int32_t cnt = per, lvl_nodes = nb;
            while (cnt > 1) {
                cnt >>= 1;
                lvl_nodes >>= 1;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k < cnt) v[k] = v[2 * k] + v[2 * k + 1];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k < cnt) tree[lvl_nodes + lane * cnt + k] = v[k];
            }
            if (per == 1) {
                // one bin per lane: the first internal level from pairs of lanes
                const double o = __shfl_xor(v[0], 1);
                if ((lane & 1) == 0 && lane < nb) tree[nb / 2 + lane / 2] = v[0] + o;
                top = nb / 2;
            } else {
                top = lvl_nodes;  // 64
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int32_t c = top >> 1; c >= 1; c >>= 1) {
                if (lane < c) tree[c + lane] = tree[2 * (c + lane)] + tree[2 * (c + lane) + 1];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
        const double root = (nb >= 2) ? tree[1] : M[0];
        if (a.deg != nullptr && lane == 0) a.deg[e] = root;
        for (int32_t c0 = 0; c0 < a.L; c0 += kDescChunk) {
            const int32_t cn = min(kDescChunk, a.L - c0);
            for (int32_t c = lane; c < cn * n_groups; c += 64) {
                const int32_t k = c / n_groups, g = g0 + (c - k * n_groups);
                const PhiloxWords w = philox4x64_10((uint64_t)e, (uint64_t)(c0 + k), (uint64_t)g, 0, a.seed, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) words[c * 4 + q] = w.w[q];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane < cn) {
                const int32_t l = c0 + lane;
                const int64_t smp = e * a.L + l;
                const uint64_t* wk = words + (int64_t)lane * n_groups * 4;
                if (!(root > 0.0)) {
                    a.node[smp] = -1;  // isolated point: no neighbour
                } else {
                    float mg = (a.margin != nullptr) ? a.margin[smp] : 0.0f;
                    int32_t m = 0;
                    for (int32_t t = 0; t < a.D; ++t) {
                        const int32_t level = a.start_level + t;
                        const double u = word_to_uniform(wk[((level >> 2) - g0) * 4 + (level & 3)]);
                        const int32_t c = (1 << (t + 1)) + 2 * m;
                        double mL, mR;
                        if (t + 1 < a.D) {
                            mL = tree[c];
                            mR = tree[c + 1];
                        } else {
                            mL = M[2 * m];  // the children are bins
                            mR = M[2 * m + 1];
                        }
                        const bool left = choose_left(u, mL, mR, a.margin != nullptr, &mg);
                        m = 2 * m + (left ? 0 : 1);
                    }
                    a.node[smp] = m;
                    if (a.margin != nullptr) a.margin[smp] = mg;
                }
            }
            // the next point (or chunk) rewrites the tree and the words
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Later passes: one thread per entry (a single sample); the 2^D bin masses are
// held in registers and each level's child masses are summed directly.
template <int D>
__global__ __launch_bounds__(256) void descend_entries_kernel(DescArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n_entries) return;
    const int32_t smp = a.entry_sample[e];
    const int32_t v = a.node[smp];
    if (v < 0) return;
    constexpr int NB = 1 << D;
    double bins[NB];
    const double* M = a.M + e * NB;
#pragma unroll
    for (int b = 0; b < NB; ++b) bins[b] = M[b];
    const int32_t i = smp / a.L, l = smp - i * a.L;
    SampleUniforms uni;
    uni.init(a.seed, (uint64_t)i, (uint64_t)l);
    float mg = (a.margin != nullptr) ? a.margin[smp] : 0.0f;
    int32_t m = 0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const int w = NB >> (t + 1);  // bins per child
        const int lo = 2 * m * w;
        double mL = 0.0, mR = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            mL += (b >= lo && b < lo + w) ? bins[b] : 0.0;
            mR += (b >= lo + w && b < lo + 2 * w) ? bins[b] : 0.0;
        }
        const bool left = choose_left(uni.at(a.start_level + t), mL, mR, a.margin != nullptr, &mg);
        m = 2 * m + (left ? 0 : 1);
    }
    a.node[smp] = (v << D) + m;
    if (a.margin != nullptr) a.margin[smp] = mg;
}

// Philox blocks of at most min(L, kDescChunk) samples at a time: at L = 17
// and D = 11 this keeps a block at 19 KB (8 blocks per CU)
size_t desc_root_lds(const DescArgs& a, int32_t* n_groups) {
    *n_groups = desc_groups(a);
    const int32_t chunk = a.L < kDescChunk ? a.L : kDescChunk;
    return sizeof(double) * ((size_t)1 << a.D) + sizeof(uint64_t) * 4 * chunk * (*n_groups);
}

hipError_t launch_descend_bins(const DescArgs& a, hipStream_t st) {
    if (a.n_entries < 1) return hipSuccess;
    if (a.jobs != nullptr) {  // root passes of several sets (tables built by the caller)
        if (a.lds_bytes == 0) return hipErrorInvalidValue;
        // a.D: the largest D of the sets
        if (a.D <= kWaveRootMaxD && 4 * a.lds_bytes <= 65536) {
            int64_t blocks = (a.n_entries + 3) / 4;
            if (blocks > (1 << 18)) blocks = 1 << 18;
            descend_root_wave_kernel<true><<<(unsigned)blocks, 256, 4 * a.lds_bytes, st>>>(a, 0);
            return hipGetLastError();
        }
        int64_t blocks = a.n_entries;
        if (blocks > (1 << 20)) blocks = 1 << 20;
        descend_root_kernel<true><<<(unsigned)blocks, kDescThreads, a.lds_bytes, st>>>(a, 0);
        return hipGetLastError();
    }
    if (a.entry_sample == nullptr) {
        if (a.D < 1 || a.D > 11) return hipErrorInvalidValue;  // the tree build assumes 2 <= 2^D <= 8 * 256
        int32_t n_groups = 0;
        const size_t lds = desc_root_lds(a, &n_groups);
        if (a.D <= kWaveRootMaxD && 4 * lds <= 65536) {
            // one wave per point (LDS: four trees and their Philox blocks)
            int64_t blocks = (a.n_entries + 3) / 4;
            if (blocks > (1 << 18)) blocks = 1 << 18;
            descend_root_wave_kernel<false><<<(unsigned)blocks, 256, 4 * lds, st>>>(a, n_groups);
            return hipGetLastError();
        }
        int64_t blocks = a.n_entries;
        if (blocks > (1 << 20)) blocks = 1 << 20;
        descend_root_kernel<false><<<(unsigned)blocks, kDescThreads, lds, st>>>(a, n_groups);
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)((a.n_entries + 255) / 256);
    switch (a.D) {
        case 1: descend_entries_kernel<1><<<blocks, 256, 0, st>>>(a); break;
        case 2: descend_entries_kernel<2><<<blocks, 256, 0, st>>>(a); break;
        case 3: descend_entries_kernel<3><<<blocks, 256, 0, st>>>(a); break;
        case 4: descend_entries_kernel<4><<<blocks, 256, 0, st>>>(a); break;
        case 5: descend_entries_kernel<5><<<blocks, 256, 0, st>>>(a); break;
        case 6: descend_entries_kernel<6><<<blocks, 256, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Leaf stage.  items[2k] = node, items[2k+1] = first position of the item's
// samples in sorted_samples; an item holds up to 64 samples of one node.
// ---------------------------------------------------------------------------

// Leaf stage: each lane keeps its sample's (<= 64) kernel values
// in registers; the child masses of every level are summed with static
// predicates, so the descent has no dependent memory chains.
// The scaled exponent (for exp2_256_tab) of one leaf pair from its sum over
// the features (a cross term, or an L1 distance for the Laplacian kernel).
template <int KIND>
__device__ __forceinline__ double leaf_exponent(double sum, double hq, double xn, double s256, double two_s,
                                                double qn) {
    if constexpr (KIND == kKindLaplacian) return -s256 * sum;
    if constexpr (KIND == kKindExponential)
        return -s256 * __builtin_sqrt(__builtin_fmax(__builtin_fma(-2.0, sum, qn + xn), 0.0));
    return __builtin_fma(two_s, sum, hq - s256 * xn);
}

// Sparse leaf path (precision mode, exact KDE, with the root pass's keep
// masks): a sample's pairs that the root pass dropped total below e^-25 of
// its degree, so they change its walk with probability below that bound
// (the same reading as the later passes).  The item evaluates only the node's
// points kept at the root for some of its samples (the union of their tiles'
// mask bits), at most kLeafSparse of them, with the cross terms in the same
// order as the full path (features 0 .. d-1, one fused multiply-add each), so
// a kept point's value is the full path's.  Returns false, having written
// nothing, when the union holds more points (or none), or when some sample
// would see a zero total (the walk reached the node through pairs its own
// tile dropped): the caller then runs the full path for the item.
constexpr int kLeafSparse = 16;

// The cross terms, values and walk of the sparse path for NG groups of four
// kept points (nk <= 4 NG; the padding columns are zero and their values are
// set to 0): whole groups are updated at once, so the sums stay in place.
template <int NG, int DMAX, int KIND>
__device__ __forceinline__ bool leaf_sparse_tail(const LeafArgs& a, const float (&q)[DMAX], const float* xsp,
                                                 const double* xnsp, const int32_t (&jk)[kLeafSparse], int32_t nk,
                                                 int32_t lo, int32_t cnt, bool active, int32_t smp, int32_t i,
                                                 int32_t l, int32_t self, double qn, double hq, double s256,
                                                 double two_s, const double* exp_tab) {
    constexpr int K = 4 * NG;
    double kv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) kv[k] = 0.0;
#pragma unroll
    for (int t = 0; t < DMAX; ++t) {
        if (t < a.d) {  // uniform
            const double qt = (double)q[t];
            const float4* row = (const float4*)(xsp + t * kLeafSparse);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const float4 v = row[g];
                kv[4 * g + 0] = __builtin_fma(qt, (double)v.x, kv[4 * g + 0]);
                kv[4 * g + 1] = __builtin_fma(qt, (double)v.y, kv[4 * g + 1]);
                kv[4 * g + 2] = __builtin_fma(qt, (double)v.z, kv[4 * g + 2]);
                kv[4 * g + 3] = __builtin_fma(qt, (double)v.w, kv[4 * g + 3]);
            }
        }
    }
    // values, 0 for the sample's own point and the padding
    double total = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double v = exp2_256_tab(leaf_exponent<KIND>(kv[k], hq, xnsp[k], s256, two_s, qn), exp_tab);
        kv[k] = (k < nk && jk[k] != self) ? v : 0.0;
        total += kv[k];
    }
    if (__ballot(active && !(total > 0.0)) != 0) {
        __syncthreads();  // the full path restages the LDS
        return false;
    }
    // the walk over the node's levels, as in the full path
    if (active) {
        SampleUniforms uni;
        uni.init(a.seed, (uint64_t)i, (uint64_t)l);
        float mg = (a.margin != nullptr) ? a.margin[smp] : 0.0f;
        int32_t na = 0, nbd = cnt, level = a.level;
        while (nbd - na > 1) {
            const int32_t mid = tree_split(na, nbd);
            double mL = 0.0, mR = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool in_node = (jk[k] >= na) && (jk[k] < nbd);
                const bool left = jk[k] < mid;
                mL += (in_node && left) ? kv[k] : 0.0;
                mR += (in_node && !left) ? kv[k] : 0.0;
            }
            const double u = uni.at(level);
            const bool go_left = choose_left(u, mL, mR, a.margin != nullptr, &mg);
            if (go_left) nbd = mid; else na = mid;
            ++level;
        }
        a.nbr[smp] = lo + na;
        if (a.margin != nullptr) a.margin[smp] = mg;
    }
    return true;
}

template <int DMAX, int KIND>
__device__ __forceinline__ bool leaf_sparse(const LeafArgs& a, int32_t lo, int32_t cnt, bool active, int32_t smp,
                                            int32_t i, int32_t l, int32_t self, double qn, double hq, double s256,
                                            double two_s, const double* exp_tab, float* xsp, double* xnsp,
                                            int32_t* idxp) {
    const int lane = threadIdx.x;
    // (1) the keep bits of the node's points, bit j for point lo + j: this
    // sample's tile row, the blocks of the node concatenated, then ORed over
    // the item's samples
    const int64_t b0 = lo >> 4;
    const int32_t sh = lo & 15;
    const int32_t nblk = (sh + cnt + 15) >> 4;  // at most 5 (cnt <= 64)
    uint64_t w0 = 0, w1 = 0;
    if (active) {
        const uint16_t* row = a.root_mask + (int64_t)(a.inv[i] / kTileQ) * a.root_blocks + b0;
        uint64_t m[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) m[b] = (b < nblk) ? row[b] : 0u;
        w0 = m[0] | (m[1] << 16) | (m[2] << 32) | (m[3] << 48);
        w1 = m[4];
    }
    uint64_t kb = (sh == 0) ? w0 : ((w0 >> sh) | (w1 << (64 - sh)));
    if (cnt < 64) kb &= (1ull << cnt) - 1ull;
    uint32_t klo = (uint32_t)kb, khi = (uint32_t)(kb >> 32);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        klo |= (uint32_t)__shfl_xor((int)klo, off);
        khi |= (uint32_t)__shfl_xor((int)khi, off);
    }
    const uint64_t keep = ((uint64_t)(uint32_t)uniform((int32_t)khi) << 32) | (uint32_t)uniform((int32_t)klo);
    const int32_t nk = __popcll(keep);
    if (nk == 0 || nk > kLeafSparse) return false;
    // (2) the kept points in index order, their rows feature-major in LDS
    // (16 per feature, zeros past nk) and their squared norms
    if ((keep >> lane) & 1ull) idxp[__popcll(keep & ((1ull << lane) - 1ull))] = lane;
    __syncthreads();
    int32_t jk[kLeafSparse];
#pragma unroll
    for (int k = 0; k < kLeafSparse; ++k) jk[k] = (k < nk) ? uniform(idxp[k]) : 0;
    {
        // every load issued before the first store (DMAX / 4 per lane)
        // (lane l stages point l % 16 at features l / 16 + 4 r)
        constexpr int kPer = (DMAX * kLeafSparse + 63) / 64;
        const int32_t myk = lane & (kLeafSparse - 1);
        const float* src = a.X + (int64_t)(lo + ((myk < nk) ? idxp[myk] : 0)) * a.d;
        float v[kPer];
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int32_t t = (lane >> 4) + 4 * r;
            v[r] = (t < a.d && myk < nk) ? src[t] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < kPer; ++r) xsp[lane + 64 * r] = v[r];
    }
    if (lane < kLeafSparse) xnsp[lane] = (lane < nk) ? a.norm[lo + idxp[lane]] : 0.0;
    // the sample's row in registers (vector loads where rows are 16-byte aligned)
    const float* xi = a.X + (int64_t)i * a.d;
    float q[DMAX];
    if ((a.d & 3) == 0 && ((uintptr_t)a.X & 15) == 0) {
#pragma unroll
        for (int t = 0; t < DMAX; t += 4) {
            float4 w = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (t < a.d) w = *(const float4*)(xi + t);
            q[t] = w.x;
            q[t + 1] = w.y;
            q[t + 2] = w.z;
            q[t + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int t = 0; t < DMAX; ++t) q[t] = (t < a.d) ? xi[t] : 0.0f;
    }
    __syncthreads();
    switch ((nk + 3) >> 2) {
        case 1: return leaf_sparse_tail<1, DMAX, KIND>(a, q, xsp, xnsp, jk, nk, lo, cnt, active, smp, i, l, self, qn,
                                                       hq, s256, two_s, exp_tab);
        case 2: return leaf_sparse_tail<2, DMAX, KIND>(a, q, xsp, xnsp, jk, nk, lo, cnt, active, smp, i, l, self, qn,
                                                       hq, s256, two_s, exp_tab);
        case 3: return leaf_sparse_tail<3, DMAX, KIND>(a, q, xsp, xnsp, jk, nk, lo, cnt, active, smp, i, l, self, qn,
                                                       hq, s256, two_s, exp_tab);
        default: return leaf_sparse_tail<4, DMAX, KIND>(a, q, xsp, xnsp, jk, nk, lo, cnt, active, smp, i, l, self,
                                                        qn, hq, s256, two_s, exp_tab);
    }
}

// KIND: the Gaussian kernel (cross terms, the norm expansion), the exponential
// one (the same, then the square root) or the Laplacian one (the L1 distance
// from coordinate differences, summed in coordinate order).
template <int DMAX, bool MULTI, int KIND = kKindGaussian>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void leaf_reg_kernel(LeafArgs a0) {
    // d <= 32: the query row in registers, node points in LDS row by row, four
    // points at a time.  d > 32: features outer, the 64 points' cross terms in
    // registers, node points staged transposed (feature-major) in FP32 (the
    // input precision; products are formed in FP64, where they are exact).
    // z = -256 s (|q|^2 + |x|^2) + 512 s q.x, as in the binned passes, and
    // 2^(z/256) from the table.
    constexpr bool kWide = DMAX > 32;
    typedef typename std::conditional<kWide, float, double>::type stage_t;
    __shared__ __attribute__((aligned(16))) stage_t xs[kWide ? DMAX * kLeafMax : (kLeafMax + 3) * DMAX];
    __shared__ double xns[kLeafMax];  // |x|^2 of the node's points, 0 past the last
    __shared__ double exp_tab[256];
    __shared__ int32_t idxp[kLeafSparse];  // the sparse path's kept points
    load_exp2_table(exp_tab);
    const int lane = threadIdx.x;
    const int64_t n_items = (int64_t)*a0.n_items;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        int32_t v = a0.items[2 * it];
        const int32_t p0 = a0.items[2 * it + 1];
        int32_t job = 0;
        if (MULTI) {  // the job owning global node v (binary search, uniform)
            int32_t lo_j = 0, hi_j = a0.n_jobs;
            while (hi_j - lo_j > 1) {
                const int32_t mid_j = (lo_j + hi_j) >> 1;
                if (a0.job_node_off[mid_j] <= v) lo_j = mid_j; else hi_j = mid_j;
            }
            job = lo_j;
            v -= a0.job_node_off[job];
        }
        const LeafArgs& a = MULTI ? a0.jobs[job] : a0;
        const double s256 = 256.0 * a.s, two_s = 2.0 * s256;
        // the grouping of a multi-set launch is the launch's own (global
        // positions, job-local sample ids)
        const int32_t* nstart = MULTI ? a0.node_start + a0.job_node_off[job] : a.node_start;
        const int32_t* sorted = MULTI ? a0.sorted_samples : a.sorted_samples;
        const int32_t p1 = nstart[v + 1];
        const int32_t lo = a.bounds[v];
        const int32_t hi = min(a.bounds[v + 1], lo + kLeafMax);  // the planner keeps nodes within kLeafMax
        const int32_t cnt = hi - lo;
        const int32_t pos = p0 + lane;
        const bool active = pos < p1;
        const int32_t smp = active ? sorted[pos] : sorted[p0];
        const int32_t i = smp / a.L, l = smp - i * a.L;
        const float* xi = a.X + (int64_t)i * a.d;
        const int32_t self = i - lo;  // the sample's own point, if it lies in the node
        const double qn = a.norm[i];
        const double hq = -s256 * qn;
        if constexpr (!MULTI && KIND != kKindLaplacian) {
            if (a.root_mask != nullptr && leaf_sparse<DMAX, KIND>(a, lo, cnt, active, smp, i, l, self, qn, hq, s256,
                                                                  two_s, exp_tab, (float*)xs, xns, idxp)) {
                __syncthreads();  // xs is reused by the next item
                continue;
            }
        }
        xns[lane] = (lane < cnt) ? a.norm[lo + lane] : 0.0;
        double kv[kLeafMax];
        if constexpr (kWide) {
            // xs[t * 64 + j] = X[lo + j][t]; points past the node are 0
            for (int32_t k = lane; k < a.d * kLeafMax; k += 64) {
                const int32_t t = k / kLeafMax, j = k - t * kLeafMax;
                xs[k] = (j < cnt) ? a.X[(int64_t)(lo + j) * a.d + t] : 0.0f;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kLeafMax; ++j) kv[j] = 0.0;  // the cross terms first
            for (int32_t t = 0; t < a.d; ++t) {
                const double qt = (double)xi[t];
                const stage_t* xt = xs + t * kLeafMax;
#pragma unroll
                for (int j = 0; j < kLeafMax; ++j) {
                    if constexpr (KIND == kKindLaplacian)
                        kv[j] += __builtin_fabs(qt - (double)xt[j]);
                    else
                        kv[j] = __builtin_fma(qt, (double)xt[j], kv[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < kLeafMax; ++j) {
                // (a uniform branch per point: evaluated unconditionally, the 64
                // exponentials get interleaved and spill)
                const double k = (j < cnt) ? exp2_256_tab(leaf_exponent<KIND>(kv[j], hq, xns[j], s256, two_s, qn),
                                                          exp_tab)
                                           : 0.0;
                kv[j] = (j != self) ? k : 0.0;
            }
        } else {
            {
                // rows of the node's points, zero-padded to DMAX features
                const float* src = a.X + (int64_t)lo * a.d;
                for (int32_t k = lane; k < cnt * DMAX; k += 64) {
                    const int32_t r = k / DMAX, t = k - r * DMAX;
                    xs[k] = (t < a.d) ? (stage_t)src[(int64_t)r * a.d + t] : (stage_t)0;
                }
            }
            __syncthreads();
            stage_t q[DMAX];
#pragma unroll
            for (int t = 0; t < DMAX; ++t) q[t] = (t < a.d) ? (stage_t)xi[t] : (stage_t)0;
#pragma unroll
            for (int j0 = 0; j0 < kLeafMax; j0 += 4) {
                if (j0 < cnt) {
                    double c[4] = {0.0, 0.0, 0.0, 0.0};
                    const stage_t* xj = xs + j0 * DMAX;
#pragma unroll
                    for (int t = 0; t < DMAX; ++t) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if constexpr (KIND == kKindLaplacian)
                                c[u] += __builtin_fabs((double)q[t] - (double)xj[u * DMAX + t]);
                            else
                                c[u] = __builtin_fma((double)q[t], (double)xj[u * DMAX + t], c[u]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int j = j0 + u;
                        const double k = exp2_256_tab(leaf_exponent<KIND>(c[u], hq, xns[j], s256, two_s, qn), exp_tab);
                        kv[j] = (j < cnt && j != self) ? k : 0.0;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) kv[j0 + u] = 0.0;
                }
            }
        }
        __syncthreads();  // xs is reused by the next item
        if (active) {
            double total = 0.0;
#pragma unroll
            for (int j = 0; j < kLeafMax; ++j) total += kv[j];
            if (!(total > 0.0)) {
                // only reachable at the root (a sample never enters a node of
                // zero mass): an isolated point has no neighbour
                a.nbr[smp] = -1;
            } else {
                SampleUniforms uni;
                uni.init(a.seed, (uint64_t)i, (uint64_t)l);
                        float mg = (a.margin != nullptr) ? a.margin[smp] : 0.0f;
                int32_t na = 0, nbd = cnt, level = a.level;
                while (nbd - na > 1) {
                    const int32_t mid = tree_split(na, nbd);
                    double mL = 0.0, mR = 0.0;
#pragma unroll
                    for (int j = 0; j < kLeafMax; ++j) {
                        const bool in_node = (j >= na) && (j < nbd);
                        const bool left = j < mid;
                        mL += (in_node && left) ? kv[j] : 0.0;
                        mR += (in_node && !left) ? kv[j] : 0.0;
                    }
                    const double u = uni.at(level);
                    const bool go_left = choose_left(u, mL, mR, a.margin != nullptr, &mg);
                    if (go_left) nbd = mid; else na = mid;
                    ++level;
                }
                a.nbr[smp] = lo + na;
                if (a.margin != nullptr) a.margin[smp] = mg;
            }
        }
    }
}

template <int DMAX>
static void launch_leaf_t(const LeafArgs& a, int64_t blocks, hipStream_t st) {
    if (a.jobs)
        leaf_reg_kernel<DMAX, true><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (a.kind == kKindExponential)
        leaf_reg_kernel<DMAX, false, kKindExponential><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (a.kind == kKindLaplacian)
        leaf_reg_kernel<DMAX, false, kKindLaplacian><<<(unsigned)blocks, 64, 0, st>>>(a);
    else
        leaf_reg_kernel<DMAX, false><<<(unsigned)blocks, 64, 0, st>>>(a);
}

// a.d is the largest d of the launch (every job of a multi-job launch is in
// the same class of d)
hipError_t launch_leaf(const LeafArgs& a, int64_t max_items, int num_cus, hipStream_t st) {
    int64_t blocks = max_items;
    const int64_t cap = (int64_t)num_cus * 32;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    if (a.d <= 2) launch_leaf_t<2>(a, blocks, st);
    else if (a.d <= 4) launch_leaf_t<4>(a, blocks, st);
    else if (a.d <= 8) launch_leaf_t<8>(a, blocks, st);
    else if (a.d <= 16) launch_leaf_t<16>(a, blocks, st);
    else if (a.d <= 32) launch_leaf_t<32>(a, blocks, st);
    else if (a.d <= 64) launch_leaf_t<64>(a, blocks, st);
    else if (a.d <= 128) launch_leaf_t<128>(a, blocks, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

int leaf_class(int32_t d) {
    int c = 2;
    while (c < d) c *= 2;
    return c < 2 ? 2 : c;
}

// ---------------------------------------------------------------------------
// Sample bookkeeping.
// ---------------------------------------------------------------------------
__global__ void init_samples_kernel(int64_t n_samples, int32_t* node, float* margin) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_samples) return;
    node[s] = 0;
    if (margin != nullptr) margin[s] = __builtin_inff();
}

hipError_t launch_init_samples(int64_t n_samples, int32_t* node, float* margin, hipStream_t st) {
    init_samples_kernel<<<(unsigned)((n_samples + 255) / 256 + 1), 256, 0, st>>>(n_samples, node, margin);
    return hipGetLastError();
}

__global__ void node_keys_kernel(const int32_t* node, int64_t n_samples, uint32_t inactive_key, uint32_t* keys,
                                 int32_t* vals) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_samples) return;
    const int32_t v = node[s];
    keys[s] = v < 0 ? inactive_key : (uint32_t)v;
    vals[s] = (int32_t)s;
}

hipError_t launch_node_keys(const int32_t* node, int64_t n_samples, uint32_t inactive_key, uint32_t* keys,
                            int32_t* vals, hipStream_t st) {
    node_keys_kernel<<<(unsigned)((n_samples + 255) / 256 + 1), 256, 0, st>>>(node, n_samples, inactive_key, keys,
                                                                             vals);
    return hipGetLastError();
}

__global__ void node_keys_sub_kernel(const int32_t* node, int64_t n_samples, int32_t L, const int32_t* inv,
                                     int32_t sub_shift, int32_t sub_bits, uint32_t inactive_node, uint32_t* keys,
                                     int32_t* vals) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_samples) return;
    const int32_t v = node[s];
    const uint32_t sub = (uint32_t)inv[s / L] >> sub_shift;
    keys[s] = v < 0 ? (inactive_node << sub_bits) : (((uint32_t)v << sub_bits) | sub);
    vals[s] = (int32_t)s;
}

hipError_t launch_node_keys_sub(const int32_t* node, int64_t n_samples, int32_t L, const int32_t* inv,
                                int32_t sub_shift, int32_t sub_bits, uint32_t inactive_node, uint32_t* keys,
                                int32_t* vals, hipStream_t st) {
    if (L < 1 || sub_bits < 0 || sub_bits > 31) return hipErrorInvalidValue;
    node_keys_sub_kernel<<<(unsigned)((n_samples + 255) / 256 + 1), 256, 0, st>>>(node, n_samples, L, inv, sub_shift,
                                                                                 sub_bits, inactive_node, keys, vals);
    return hipGetLastError();
}

// start[v] = first position whose key >> shift is >= v (v in [0, n_nodes]).
__global__ void node_starts_kernel(const uint32_t* keys, int64_t n, int64_t n_nodes, int32_t shift, int32_t* start) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n_nodes) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(keys[mid] >> shift) < v) lo = mid + 1; else hi = mid;
    }
    start[v] = (int32_t)lo;
}

hipError_t launch_node_starts(const uint32_t* sorted_keys, int64_t n_samples, int64_t n_nodes, int32_t* start,
                              hipStream_t st, int32_t key_shift) {
    node_starts_kernel<<<(unsigned)((n_nodes + 1 + 255) / 256 + 1), 256, 0, st>>>(sorted_keys, n_samples, n_nodes,
                                                                                 key_shift, start);
    return hipGetLastError();
}

__global__ void entry_points_kernel(const int32_t* sorted_samples, int64_t n, int32_t L, int32_t* q_idx) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    q_idx[e] = sorted_samples[e] / L;
}

hipError_t launch_entry_points(const int32_t* sorted_samples, int64_t n, int32_t L, int32_t* q_idx,
                               hipStream_t st) {
    entry_points_kernel<<<(unsigned)((n + 255) / 256 + 1), 256, 0, st>>>(sorted_samples, n, L, q_idx);
    return hipGetLastError();
}

__global__ void node_qptr_kernel(const int32_t* start, int64_t n_nodes, int64_t* q_ptr) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n_nodes) return;
    q_ptr[v] = start[v];
}

hipError_t launch_node_qptr(const int32_t* node_start, int64_t n_nodes, int64_t* q_ptr, hipStream_t st) {
    node_qptr_kernel<<<(unsigned)((n_nodes + 1 + 255) / 256 + 1), 256, 0, st>>>(node_start, n_nodes, q_ptr);
    return hipGetLastError();
}

// Leaf items: node v contributes ceil(cnt_v / 64) items.
__global__ void leaf_item_counts_kernel(const int32_t* start, int64_t n_nodes, int64_t* counts) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_nodes) return;
    counts[v] = (start[v + 1] - start[v] + 63) / 64;
}

__global__ void leaf_item_fill_kernel(const int32_t* start, const int64_t* offsets, int64_t n_nodes,
                                      const int64_t* total, int32_t* items, int32_t* n_items) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0) *n_items = (int32_t)*total;
    if (v >= n_nodes) return;
    const int64_t o = offsets[v];
    const int32_t s0 = start[v], s1 = start[v + 1];
    int64_t k = 0;
    for (int32_t p = s0; p < s1; p += 64, ++k) {
        items[2 * (o + k)] = (int32_t)v;
        items[2 * (o + k) + 1] = p;
    }
}

hipError_t launch_leaf_items(const int32_t* node_start, int64_t n_nodes, int64_t* scratch, int32_t* items,
                             int32_t* n_items, hipStream_t st) {
    int64_t* counts = scratch;
    int64_t* offsets = counts + (n_nodes + 1);
    int64_t* total = offsets + (n_nodes + 1);
    int64_t* partials = total + 1;
    leaf_item_counts_kernel<<<(unsigned)((n_nodes + 255) / 256 + 1), 256, 0, st>>>(node_start, n_nodes, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan_i64(counts, offsets, n_nodes, total, partials, st);
    if (e != hipSuccess) return e;
    leaf_item_fill_kernel<<<(unsigned)((n_nodes + 255) / 256 + 1), 256, 0, st>>>(node_start, offsets, n_nodes, total,
                                                                               items, n_items);
    return hipGetLastError();
}

__global__ void multi_node_keys_kernel(const LeafKeyJob* __restrict__ jobs, const int64_t* __restrict__ sample_off,
                                       const int32_t* __restrict__ node_off, int32_t n_jobs, int64_t total,
                                       uint32_t inactive_key, uint32_t* __restrict__ keys, int32_t* __restrict__ vals) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    int32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (sample_off[mid] <= g) lo = mid; else hi = mid;
    }
    const int64_t s = g - sample_off[lo];
    const int32_t v = jobs[lo].node[s];
    if (v < 0) jobs[lo].nbr[s] = -1;  // no neighbour (an isolated point)
    keys[g] = v < 0 ? inactive_key : (uint32_t)(node_off[lo] + v);
    vals[g] = (int32_t)s;
}

hipError_t launch_multi_node_keys(const LeafKeyJob* jobs, const int64_t* sample_off, const int32_t* node_off,
                                  int32_t n_jobs, int64_t total, uint32_t inactive_key, uint32_t* keys, int32_t* vals,
                                  hipStream_t st) {
    if (total == 0) return hipSuccess;
    multi_node_keys_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(jobs, sample_off, node_off, n_jobs, total,
                                                                          inactive_key, keys, vals);
    return hipGetLastError();
}

__global__ void finish_inactive_kernel(const int32_t* node, int64_t n_samples, int32_t* nbr) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_samples) return;
    if (node[s] < 0) nbr[s] = -1;
}

hipError_t launch_finish_inactive(const int32_t* node, int64_t n_samples, int32_t* nbr, hipStream_t st) {
    finish_inactive_kernel<<<(unsigned)((n_samples + 255) / 256 + 1), 256, 0, st>>>(node, n_samples, nbr);
    return hipGetLastError();
}

}  // namespace fsg
