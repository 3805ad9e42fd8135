// Randomised tree descent (hot-path step "descent"; Algorithm 1's branch on r,
// Section 4.1).  Two stages:
//  * after a binned KDE pass, each entry's 2^D bin masses form the leaves of a
//    perfect binary sum tree (built in LDS); every sample of the entry walks D
//    levels down it, one Philox uniform per level;
//  * the leaf stage resolves nodes of at most 64 points directly: a wave takes
//    up to 64 samples that sit in the same node, evaluates the kernel of each
//    sample's point against every point of the node (difference form, FP64),
//    keeps the row in LDS, and each lane walks its own sample to a leaf.
#include "common.h"
#include "device.h"

namespace fsg {

// One wave per entry; dynamic LDS holds the sum tree (2^(D+1) doubles).
__global__ __launch_bounds__(64) void descend_bins_kernel(DescArgs a) {
    extern __shared__ double tree[];
    const int lane = threadIdx.x;
    const int32_t nb = 1 << a.D;
    for (int64_t e = blockIdx.x; e < a.n_entries; e += gridDim.x) {
        const double* M = a.M + e * nb;
        for (int32_t b = lane; b < nb; b += 64) tree[nb + b] = M[b];
        __syncthreads();
        for (int32_t t = a.D - 1; t >= 0; --t) {
            const int32_t cnt = 1 << t;
            for (int32_t k = lane; k < cnt; k += 64) tree[cnt + k] = tree[2 * (cnt + k)] + tree[2 * (cnt + k) + 1];
            __syncthreads();
        }
        const double root = tree[1];
        int32_t first_sample, n_samp;
        if (a.entry_sample == nullptr) {
            first_sample = (int32_t)(e * a.L);
            n_samp = a.L;
            if (a.deg != nullptr && lane == 0) a.deg[e] = root;
        } else {
            first_sample = -1;
            n_samp = 1;
        }
        for (int32_t k = lane; k < n_samp; k += 64) {
            const int32_t smp = (a.entry_sample == nullptr) ? first_sample + k : a.entry_sample[e];
            const int32_t i = smp / a.L, l = smp - i * a.L;
            int32_t v = a.node[smp];
            if (v < 0) continue;
            if (!(root > 0.0)) {
                a.node[smp] = -1;  // isolated point: no neighbour
                continue;
            }
            float mg = (a.margin != nullptr) ? a.margin[smp] : 0.0f;
            SampleUniforms uni;
            uni.init(a.seed, (uint64_t)i, (uint64_t)l);
            int32_t m = 0;
            for (int32_t t = 0; t < a.D; ++t) {
                const double u = uni.at(a.start_level + t);
                const int32_t c = (1 << (t + 1)) + 2 * m;
                double margin;
                const bool left = choose_left(u, tree[c], tree[c + 1], &margin);
                mg = fminf(mg, (float)margin);
                m = 2 * m + (left ? 0 : 1);
            }
            a.node[smp] = (v << a.D) + m;
            if (a.margin != nullptr) a.margin[smp] = mg;
        }
        __syncthreads();
    }
}

hipError_t launch_descend_bins(const DescArgs& a, hipStream_t st) {
    int64_t blocks = a.n_entries;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) return hipSuccess;
    const size_t lds = sizeof(double) * ((size_t)2 << a.D);
    descend_bins_kernel<<<(unsigned)blocks, 64, lds, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Leaf stage.  items[2k] = node, items[2k+1] = first position of the item's
// samples in sorted_samples; an item holds up to 64 samples of one node.
// ---------------------------------------------------------------------------
template <int DMAX>
__global__ __launch_bounds__(64) void leaf_kernel(LeafArgs a) {
    __shared__ double row[kLeafMax * 64];  // row[j * 64 + lane]: kernel of sample `lane` to node point j
    const int lane = threadIdx.x;
    const int32_t n_items = *a.n_items;
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int32_t v = a.items[2 * it], p0 = a.items[2 * it + 1];
        const int32_t p1 = a.node_start[v + 1];
        const int32_t lo = a.bounds[v];
        const int32_t hi = min(a.bounds[v + 1], lo + kLeafMax);  // the planner keeps nodes within kLeafMax
        const int32_t pos = p0 + lane;
        const bool active = pos < p1 && lane < 64;
        const int32_t smp = active ? a.sorted_samples[pos] : a.sorted_samples[p0];
        const int32_t i = smp / a.L, l = smp - i * a.L;
        const float* xi = a.X + (int64_t)i * a.d;
        double q[DMAX > 0 ? DMAX : 1];
        if (DMAX > 0) {
#pragma unroll
            for (int t = 0; t < DMAX; ++t) q[t] = (t < a.d) ? (double)xi[t] : 0.0;
        }
        for (int32_t j = lo; j < hi; ++j) {
            const float* xj = a.X + (int64_t)j * a.d;
            double D = 0.0;
            if (DMAX > 0) {
#pragma unroll
                for (int t = 0; t < DMAX; ++t) {
                    if (t < a.d) {
                        const double df = q[t] - (double)xj[t];
                        D = __builtin_fma(df, df, D);
                    }
                }
            } else {
                for (int32_t t = 0; t < a.d; ++t) {
                    const double df = (double)xi[t] - (double)xj[t];
                    D = __builtin_fma(df, df, D);
                }
            }
            row[(j - lo) * 64 + lane] = (j == i) ? 0.0 : exp2_fp64(-a.s * D);
        }
        __syncthreads();
        if (active) {
            double total = 0.0;
            for (int32_t j = lo; j < hi; ++j) total += row[(j - lo) * 64 + lane];
            if (!(total > 0.0)) {
                // only reachable at the root (a sample never enters a node of
                // zero mass): an isolated point has no neighbour
                a.nbr[smp] = -1;
            } else {
                SampleUniforms uni;
                uni.init(a.seed, (uint64_t)i, (uint64_t)l);
                float mg = (a.margin != nullptr) ? a.margin[smp] : 0.0f;
                int32_t na = lo, nbd = hi, level = a.level;
                while (nbd - na > 1) {
                    const int32_t mid = tree_split(na, nbd);
                    double mL = 0.0, mR = 0.0;
                    for (int32_t j = na; j < mid; ++j) mL += row[(j - lo) * 64 + lane];
                    for (int32_t j = mid; j < nbd; ++j) mR += row[(j - lo) * 64 + lane];
                    double margin;
                    const bool left = choose_left(uni.at(level), mL, mR, &margin);
                    mg = fminf(mg, (float)margin);
                    if (left) nbd = mid; else na = mid;
                    ++level;
                }
                a.nbr[smp] = na;
                if (a.margin != nullptr) a.margin[smp] = mg;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_leaf(const LeafArgs& a, int64_t max_items, int num_cus, hipStream_t st) {
    int64_t blocks = max_items;
    const int64_t cap = (int64_t)num_cus * 16;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    if (a.d <= 4) leaf_kernel<4><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (a.d <= 8) leaf_kernel<8><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (a.d <= 16) leaf_kernel<16><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (a.d <= 32) leaf_kernel<32><<<(unsigned)blocks, 64, 0, st>>>(a);
    else if (a.d <= 64) leaf_kernel<64><<<(unsigned)blocks, 64, 0, st>>>(a);
    else leaf_kernel<0><<<(unsigned)blocks, 64, 0, st>>>(a);
    return hipGetLastError();
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

// start[v] = first position whose key is >= v (v in [0, n_nodes]).
__global__ void node_starts_kernel(const uint32_t* keys, int64_t n, int64_t n_nodes, int32_t* start) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n_nodes) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < v) lo = mid + 1; else hi = mid;
    }
    start[v] = (int32_t)lo;
}

hipError_t launch_node_starts(const uint32_t* sorted_keys, int64_t n_samples, int64_t n_nodes, int32_t* start,
                              hipStream_t st) {
    node_starts_kernel<<<(unsigned)((n_nodes + 1 + 255) / 256 + 1), 256, 0, st>>>(sorted_keys, n_samples, n_nodes,
                                                                                 start);
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
