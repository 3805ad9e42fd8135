// Internal declarations shared by the HIP sources of libfsg.so (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>
#include <map>
#include <set>

#include "fsg.h"

namespace fsg {

// ---------------------------------------------------------------------------
// Geometry of the FP64 matrix-core operand layout.
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// receives C[l/16 + 4i][l%16] in element i.  Each point is one FP64 row of
// 4*D4 values (D4 = number of 4-wide feature steps, features zero-padded to
// 4*D4, rows zero-padded to a multiple of 16); feature 4*kk + g of point p is
//   Xp[p * 4 * D4 + (kk / 2) * 8 + g * 2 + kk % 2]   (D4 >= 2),
//   Xp[p * 4 + g]                                     (D4 = 1),
// so the four lanes that supply feature rows 0-3 of a point read 64
// contiguous bytes per 16-byte load, and a gathered point is 32*D4
// contiguous bytes.
// ---------------------------------------------------------------------------
constexpr int kLeafMax = 64;     // largest node the leaf stage resolves
// smallest point set the tile pruning runs on by default: below it the
// plan and the conversion back to index order cost more than the scan saves
constexpr int64_t kPruneMinPoints = (int64_t)1 << 18;
constexpr int kTileQ = 64;       // query entries per wave in the KDE kernel

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef int32_t int4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Integer slices of the points (precision mode, 32 < d <= 64): point p's row
// scaled by 2^-e_p (e_p chosen so that every |x_k| 2^-e_p < 0.498) and
// rounded to a multiple of 2^-56 is written as kSlices signed base-256 digits
// per coordinate,
//   x_k 2^-e_p = sum_{a=1..kSlices} c_{a,k} 2^-8a + r_k,  c in [-128, 127], |r_k| <= 2^-57,
// (balanced digits, taken from the least significant up; every FP32
// coordinate at least 2^-30 times its row's largest is exact).  Slice a of point
// p is 64 bytes at Xs[p * kSliceRow + 64 a] (coordinates zero-padded to 64),
// e_p is xe[p].  v_mfma_i32_16x16x64_i8: lane l supplies 16 bytes of row l%16
// of A and of column l%16 of B (the same 16 of the 64 K positions, at byte
// 16 (l/16) of the slice) and receives C[4 (l/16) + i][l%16] in element i.
// ---------------------------------------------------------------------------
constexpr int kSlices = 7;
constexpr int kSliceRow = 64 * kSlices;

// One unit of KDE work for one wave: up to 16*RQ query entries of one
// segment against the bins [b0, b1) of that segment.
struct WorkItem {
    int32_t seg;
    int32_t ne;      // number of valid entries (<= tile)
    int64_t e0;      // first entry
    int32_t b0, b1;  // bin range (indices into the segment's boundary list)
};

// Work items of one point set in a multi-set launch.
struct BatchItemDesc {
    int64_t item_off;   // first item of the set (entry n_jobs: the total)
    int64_t n_entries;  // query entries (the set's points)
    int32_t nbins;
    int32_t bpc;        // bins per item
    int32_t tile;       // query entries per item
    int32_t n_tiles;
};

struct SegDesc {
    int64_t bound_off;  // offset of the segment's boundary list in the bounds array
    int32_t nbins;      // bins in the segment (boundaries: nbins + 1)
    int32_t job;        // point set of the segment in a multi-set launch (index into KdeArgs::jobs)
};

enum SelfMode : int32_t { SELF_NONE = 0, SELF_POINT = 1, SELF_ARRAY = 2 };

struct KdeArgs {
    const double* Qp;        // query operand rows
    const double* qnorm;     // ||q||^2, FP64
    const double* Xp;        // data operand rows
    const double* xnorm;     // ||x||^2, FP64 (padded rows hold 0)
    int32_t D4;              // feature steps
    int64_t n_query;         // points in the query set (indices are clamped into range)
    int64_t n_data;          // points in the data set (column ranges are clamped into range)
    const int32_t* q_idx;    // entry -> query point (NULL: entry index itself)
    const int32_t* self_idx; // entry -> excluded data index (SELF_ARRAY)
    int32_t self_mode;
    const int32_t* bounds;   // boundary lists
    const SegDesc* segs;
    const WorkItem* items;
    const int32_t* n_items;  // device-side count
    double s;                // gamma * log2(e)
    int32_t kind;            // fsg_kernel of the exponent
    const float* qpts;       // FP32 query points, row-major (the Laplacian kernel's L1 distances)
    const float* xpts;       // FP32 data points
    int32_t d;
    double* out;             // out[row * out_stride + bin]
    int64_t out_stride;
    const int32_t* out_rows; // entry -> output row (NULL: the entry index)
    const KdeArgs* jobs;     // multi-set launch: per point set arguments (NULL: this one)
    const uint16_t* mask;    // precision mode: keep masks of this point set [tiles][n_blocks]
    int64_t n_blocks;        // precision mode: 16-column blocks per mask row
    // precision mode, later passes: one mask row per work item, holding the
    // blocks from the item's first column on (row `item`, entry b - first block)
    int32_t mask_by_item;
    // precision mode, 32 < d <= 64, Gaussian kernel: integer slices of the
    // query and data points (NULL: the cross terms are recomputed in FP64)
    const int8_t* Qs;
    const int32_t* qe;
    const int8_t* Xs;
    const int32_t* xe;
};

// Filtered KDE (precision mode): BF16 split operands decide which pairs are
// recomputed exactly; the rest add 0 (provably below e^-Delta of the row).
struct MaskArgs {
    const void* Xb;            // data-side split fragments [n_pad/16][KB][64] x 8 bf16
    const void* Qb;            // query-side split fragments of the entries, in entry order
                               // (rows up to a multiple of kThetaPad, zero past the last)
    const float* xa;           // -|x|^2/2 of the data points [n_pad]
    int32_t KB;                // 32-wide K steps of the split operands
    const int32_t* q_idx;      // entry -> query point (NULL: the entry itself)
    int64_t n_entries;
    int64_t n_query;
    int64_t n_data;
    const double* qnorm;       // ||q||^2
    const double* dmin;        // query point -> upper bound on its smallest squared distance
    const double* xmax;        // device scalar: max |x| over the data set
    double margin_z;           // Delta
    double eps;                // relative error bound of the split cross term
    double gamma;
    int32_t kind;              // fsg_kernel: Gaussian or exponential
    int64_t n_tiles;           // 64-entry query tiles
    int64_t n_blocks;          // 16-column data blocks
    int64_t blocks_per_chunk;
    int64_t n_chunks;
    uint16_t* mask;            // [n_tiles][n_blocks]: bit c = column c of the block kept for the tile
    const float* ntheta;       // per entry: minus its keep-threshold (FP32, rounded so that the test
                               // only keeps more); -inf up to a multiple of kThetaPad entries
    int64_t* kept;             // optional: number of (column, tile) pairs kept
    // multi-set launch: items of point set j are [job_item_off[j], job_item_off[j+1]),
    // each set's arguments in jobs[j] (NULL: this one; kept is this launch's)
    const MaskArgs* jobs;
    const int64_t* job_item_off;
    int32_t n_jobs;
    int64_t n_items_total;
    // pruned scan: work items {first tile, first block, end block} of the
    // data in pivot order (Xb, xa, mask then refer to that order); XCD x takes
    // items [xseg[x], xseg[x+1])
    const int32_t* list;
    const int64_t* xseg;
};

// Tile pruning ahead of the keep-mask scan (kde_prune.hip).
struct PruneArgs {
    const float* X;            // FP32 points, row-major n x d
    int64_t n;
    int32_t d;
    int32_t P;                 // pivots (= cells)
    const int32_t* cell_pivot; // [P]: the point that is the pivot of cell c
    const int32_t* order;      // entry (pivot order) -> point
    const double* qnorm;       // FP64 |x|^2 per point
    const double* dmin;        // per point: upper bound on its smallest squared distance
    const double* xmax;        // device scalar: max |x|
    double margin_z;           // Delta
    double eps;                // relative error bound of the split cross term
    double gamma;
    int32_t kind;              // fsg_kernel: Gaussian or exponential
    const float* pnorm;        // FP32 |p_c|^2 per cell
    const float* prad;         // upper bound on each cell's radius
    const int32_t* cell_start; // [P + 1]: cell c holds entries [cell_start[c], cell_start[c+1])
    int64_t n_tiles;           // 64-entry query tiles
    int32_t words;             // 32-bit words of a tile's cell set, (P + 31) / 32 <= 8
    uint32_t* surv;            // [n_tiles][words]: cells a tile may keep columns of
    int32_t TP;                // tiles per keep-mask work item
    int64_t n_groups;          // groups of TP tiles
    int64_t n_blocks_p;        // 16-column blocks of the data in pivot order
    int32_t chunk_blocks;      // blocks per chunk (an item stays within one)
    int64_t n_chunks;
    int64_t* counts;           // [n_chunks n_groups + 1] items per (chunk, group)
    int64_t* offsets;          // exclusive scan of counts
    int64_t* bcounts;          // [n_chunks n_groups + 1] blocks per (chunk, group)
    int64_t* boffsets;         // exclusive scan of bcounts
    int64_t* total;            // device: [0] the number of items, [1] of blocks
    int32_t* items;            // [3 x items]
    int64_t* xseg;             // [kXcds + 1] item segments of the XCDs
    int64_t* scanned;          // optional: adds the scanned (column, tile) pairs
};
// XCDs of the MI355X: workgroup b runs on XCD b % kXcds (round-robin
// dispatch); the pruned scan gives each XCD its own segment of the items
constexpr int kXcds = 8;

constexpr int kThetaPad = 128;  // padding of MaskArgs::ntheta: a whole number of tile groups
// 64-entry query tiles per keep-mask work item: two tiles use each loaded
// data operand twice as often as one (the kernel is bound by operand traffic
// more than by occupancy); for d > 32 their operands need one wave per SIMD
__host__ __device__ constexpr int mask_tiles_per_item(int KB) { return KB <= 6 ? 2 : 1; }

// work items of one point set's keep-mask pass: (group of tiles, chunk of blocks)
__host__ __device__ inline int64_t mask_items(const MaskArgs& m) {
    const int tp = mask_tiles_per_item(m.KB);
    return (m.n_tiles + tp - 1) / tp * m.n_chunks;
}

// ---------------------------------------------------------------------------
// Internal handles.
// ---------------------------------------------------------------------------
struct Arena;

}  // namespace fsg

namespace fsg {
struct BatchTables;  // device tables of a batched root pass (api.hip)
struct LeafTables;   // device tables of a batched leaf stage (api.hip)
struct DescTables;   // device tables of a batched root descent (api.hip)
}
struct fsg_server;

struct fsg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t budget = 0;
    int num_cus = 256;
    std::string arch;  // gcnArchName of the device
    std::string last_error;
    // workspace: named device buffers that grow on demand (never shrink)
    std::map<std::string, std::pair<void*, size_t>> bufs;
    size_t held = 0;
    // pinned host scratch for small device->host reads
    int64_t* host_scratch = nullptr;
    // stage timing (opt-in): recorded event pairs per stage
    bool profiling = false;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> marks;
    std::vector<hipEvent_t> free_events;
    // cap on the tree levels one binned pass resolves (0: automatic)
    int max_levels_per_pass = 0;
    // precision mode: skip (query tile, cell) pairs that cannot keep a column
    int32_t pruning = -1;        // tile pruning: -1 by size (n >= kPruneMinPoints), 0 off, 1 on
    int32_t slices = -1;         // integer-slice recompute: 0 off, otherwise where it applies
    // kernel of later calls (fsg_ctx_set_kernel)
    fsg_kernel kernel = FSG_GAUSSIAN;
    // precision mode: the dropped share of every degree allowed (0: e^-25)
    double kde_error = 0.0;
    // precision-mode statistics (device counters)
    int64_t* filter_counts = nullptr;  // [kept, scanned]
    // live point sets; detached (their ctx cleared) when the context is destroyed
    std::set<fsg_points*> points;
    // device blocks of destroyed point sets, kept for reuse by later point
    // sets on the same stream (size -> block); sizes of every pooled block
    std::multimap<size_t, void*> pool_free;
    std::map<void*, size_t> pool_size;
    size_t pool_cached = 0;
    // batched root passes: launch shapes tuned per (feature steps, precision)
    // as (waves per CU, data columns per work item), and the device tables of
    // the job groups seen so far
    bool autotune = true;
    std::map<std::pair<int, int>, std::pair<int, int>> tuned;
    std::vector<fsg::BatchTables*> batch_cache;
    std::vector<fsg::LeafTables*> leaf_cache;
    std::vector<fsg::DescTables*> desc_cache;
    // live batch jobs; their buffers are freed and they are detached when the
    // context is destroyed
    std::set<fsg_job*> jobs;
    // live servers: their sets and requests are released when the context is
    // destroyed (the handles stay valid for fsg_server_destroy)
    std::set<fsg_server*> servers;
    // HIP graphs recorded on this context and not yet destroyed.  While any
    // exists, device and pinned host blocks the context would free (a grown
    // workspace buffer, released pool blocks, dropped batch tables) may still
    // be named by a graph node: they are parked here and freed when the last
    // graph is destroyed.
    std::set<fsg_graph*> graphs;
    std::vector<void*> retired;
    std::vector<void*> retired_host;
    // device address of the no-allocation entry point's static scratch on
    // this context's device (nullptr if it could not be located)
    void* noalloc_scratch = nullptr;
};


struct fsg_points {
    fsg_ctx* ctx = nullptr;
    const float* X = nullptr;  // borrowed, FP32 row-major n x d
    int64_t n = 0;
    int32_t d = 0;
    int32_t D4 = 0;            // padded feature steps
    int64_t n_pad = 0;         // rows padded to a multiple of 16
    fsg_precision prec = FSG_PLAIN_FP64;
    double* Xp = nullptr;      // FP64 operand rows [n_pad][4*D4] (layout above)
    double* norm = nullptr;    // FP64 ||x||^2 [n_pad]
    // precision mode (FSG_BF16_SPLIT)
    int32_t KB = 0;            // 32-wide K steps of the split operands
    void* Xb = nullptr;        // data-side split fragments (with xa: written on first use by a full scan)
    bool xb_ready = false;
    void* Qb = nullptr;        // query-side split fragments in pivot order (rows: n rounded up to kThetaPad)
    float* xa = nullptr;       // -|x|^2/2 in FP32 [n_pad]
    double* dmin = nullptr;    // upper bound on each point's smallest squared distance
    int32_t* order = nullptr;  // points ordered by nearest pivot
    double* xmax = nullptr;    // device scalar: max |x|
    // precision mode, pruned scan: data-side split fragments and -|x|^2/2 in
    // pivot order (rows as Qb), the cells of the pivots (entries
    // [cell_start[c], cell_start[c+1]) are nearest to pivot c), each pivot's
    // FP32 squared norm and an upper bound on each cell's radius
    void* Xbp = nullptr;
    float* xap = nullptr;
    int32_t* cell_start = nullptr;
    int32_t* cell_pivot = nullptr;
    int32_t* inv = nullptr;    // point -> its position in the pivot order
    int8_t* Xs = nullptr;      // integer slices [n_pad][kSliceRow] (32 < d <= 64)
    int32_t* xe = nullptr;     // their row exponents [n_pad]
    float* pnorm = nullptr;
    float* prad = nullptr;
    int32_t P = 0;
    // tree level boundaries, computed on demand: level -> int32 [2^level + 1]
    std::map<int, int32_t*> levels;
    size_t bytes = 0;
};

namespace fsg {

// Point-set memory: stream-ordered reuse of the blocks of destroyed point sets
// (no hipMalloc / hipFree, hence no device synchronisation, in the steady state).
hipError_t pool_alloc(fsg_ctx* ctx, size_t bytes, void** out);
void pool_release(fsg_ctx* ctx, void* p);
void pool_clear(fsg_ctx* ctx);

// Error helpers: every API function funnels HIP failures through these.
fsg_status set_error(fsg_ctx* ctx, fsg_status s, const std::string& msg);
#define FSG_HIP(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return ::fsg::set_error((ctx), e_ == hipErrorOutOfMemory ? FSG_E_NOMEM : FSG_E_DEVICE, \
                                    std::string(#call) + ": " + hipGetErrorString(e_));          \
    } while (0)
#define FSG_CHECK_LAUNCH(ctx) FSG_HIP(ctx, hipGetLastError())

// Stage timing: begin/end record events on the context stream when enabled.
struct StageTimer {
    fsg_ctx* ctx;
    std::string name;
    hipEvent_t start = nullptr;
    StageTimer(fsg_ctx* c, const char* n);
    ~StageTimer();
};

// Workspace buffer of at least `bytes`, keyed by name (reused across calls).
fsg_status ws_get(fsg_ctx* ctx, const char* name, size_t bytes, void** out);
// Segmented KDE (fsg_kde_segmented and its no-allocation variant): argument
// checks, buffer sizes (elements) and the launches on given buffers.
struct KdeSegSizes {
    int32_t tile = 0;
    int64_t max_items = 0;  // WorkItem
    int64_t bounds = 0;     // int32
    int64_t counts = 0;     // int64
    int64_t pairs = 0;      // double
};
struct KdeSegBufs {
    int32_t* bounds = nullptr;
    SegDesc* segs = nullptr;  // [n_seg]
    WorkItem* items = nullptr;
    int32_t* n_items = nullptr;  // [1]
    int64_t* counts = nullptr;
    double* pairs = nullptr;
};
fsg_status kde_segmented_check(fsg_ctx* ctx, const fsg_points* Q, const fsg_points* X, double gamma, int64_t n_seg,
                               int64_t n_entries, const int64_t* q_ptr, const int32_t* q_idx, const int32_t* lo,
                               const int32_t* mid, const int32_t* hi, const double* out_left,
                               const double* out_right, bool* empty);
KdeSegSizes kde_segmented_sizes(const fsg_points* X, int64_t n_seg, int64_t n_entries);
fsg_status kde_segmented_enqueue(fsg_ctx* ctx, const fsg_points* Q, const fsg_points* X, double gamma,
                                 int64_t n_seg, int64_t n_entries, const int64_t* q_ptr, const int32_t* q_idx,
                                 const int32_t* lo, const int32_t* mid, const int32_t* hi, const int32_t* self_idx,
                                 double* out_left, double* out_right, const KdeSegBufs& b);
// The static scratch of the no-allocation entry point: its device address on
// `device` (looked up once per device, with that device current), or nullptr.
void* noalloc_scratch_setup(int device);

// Free a device block (hipMalloc) or pinned host block (hipHostMalloc) of the
// context, or park it while a recorded graph may name it.
void dev_free(fsg_ctx* ctx, void* p);
void host_free(fsg_ctx* ctx, void* p);

// Feature-step count used for a dimension d (a size the KDE kernel is built for).
int feature_steps(int d);

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip sources).
// ---------------------------------------------------------------------------
hipError_t launch_prep_slices(const float* X, int64_t n, int32_t d, int64_t n_pad, int8_t* Xs, int32_t* xe,
                              hipStream_t st);
hipError_t launch_prep(const float* X, int64_t n, int32_t d, int32_t D4, int64_t n_pad, double* Xp, double* norm,
                       hipStream_t st);
hipError_t launch_level_bounds(int64_t n, int level, int32_t* out, hipStream_t st);

// KDE over a work list; grid = waves / 4 blocks of 256 threads.
hipError_t launch_kde(const KdeArgs& a, int64_t max_items, int num_cus, hipStream_t st, int waves_per_cu = 8);
// the Laplacian kernel's binned KDE on the vector units (kde_l1.hip)
hipError_t launch_kde_l1(const KdeArgs& a, int64_t max_items, int num_cus, hipStream_t st);
int kde_tile(int D4);  // query entries per work item of the plain kernel
// query entries per work item of the exact recompute (precision mode; sliced:
// the integer-slice variant runs)
int exact_tile(int D4, bool sliced);
hipError_t launch_batch_items(const BatchItemDesc* jd, int32_t n_jobs, int64_t total, WorkItem* items,
                              int32_t* n_items, hipStream_t st);
hipError_t launch_keep_mask(const MaskArgs& m, int num_cus, hipStream_t st);
// waves of one keep-mask launch (before clamping to the item count)
int64_t keep_mask_waves(int KB, int num_cus);
// MaskArgs::ntheta of every entry of m (n_out = n_entries rounded up to kThetaPad)
hipError_t launch_mask_theta(const MaskArgs& m, float* out, int64_t n_out, hipStream_t st);
// next_item: a counter that must read 0 when the kernel starts (work items
// beyond the first wave of the grid are claimed from it)
hipError_t launch_exact_kept(const KdeArgs& a, int64_t max_items, unsigned long long* next_item, int num_cus,
                             hipStream_t st);
int split_steps(int d);
hipError_t launch_prep_split(const float* X, const double* norm, int64_t n, int32_t d, int32_t KB, int64_t n_pad,
                             void* Xb, float* xa, hipStream_t st);
// query-side split fragments of points order[0..n) in that order, rows
// (a multiple of 16, at least n) rows with zeros past n
hipError_t launch_prep_query_split(const float* X, const int32_t* order, int64_t n, int32_t d, int32_t KB,
                                   int64_t rows, void* Qb, hipStream_t st);
hipError_t launch_pivots(const float* X, int64_t n, int32_t d, int32_t P, double* dmin, uint32_t* label, int32_t* ids,
                         hipStream_t st);
hipError_t launch_prep_split_order(const float* X, const double* norm, const int32_t* order, int64_t n, int32_t d,
                                   int32_t KB, int64_t rows, void* Xbp, float* xap, hipStream_t st);
hipError_t launch_pivot_chain(const float* X, int64_t n, int32_t d, int32_t P, uint16_t* D16, int32_t* rank,
                              int32_t* cell_pivot, uint32_t* label, hipStream_t st);
hipError_t launch_cell_geometry(const float* X, int32_t d, int32_t P, const double* dmin, const int32_t* order,
                                const int32_t* cell_start, const int32_t* cell_pivot, float* pnorm, float* prad,
                                hipStream_t st);
// inv[order[e]] = e
hipError_t launch_inverse_order(const int32_t* order, int64_t n, int32_t* inv, hipStream_t st);
// keep masks of a later pass's work items (a.items, a.n_items; entries a.q_idx):
// row it, entry k = the union over the item's entries of the root pass's mask
// bits of block first + k (first = the item's first column / 16) in the row
// of the entry's root tile (inv[point] / kTileQ); W entries per row
hipError_t launch_pass_mask(const KdeArgs& a, int64_t max_items, const int32_t* inv, const uint16_t* root_mask,
                            int64_t root_blocks, int32_t W, uint16_t* pmask, hipStream_t st);
hipError_t launch_prune_plan(const PruneArgs& a, hipStream_t st);
hipError_t launch_prune_items(const PruneArgs& a, int64_t* partials, hipStream_t st);
int64_t prune_max_items(int64_t n_groups, int32_t P, int64_t n_chunks);
hipError_t launch_mask_to_index(const PruneArgs& a, const uint16_t* maskp, int64_t n_blocks_p, uint16_t* mask,
                                int64_t n_blocks, hipStream_t st);
int max_norm_parts(int64_t n);  // partial maxima launch_max_norm needs in `part`
hipError_t launch_max_norm(const double* norm, int64_t n, double* part, double* out, hipStream_t st);
int filter_steps(int D4);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t st);
// Work list for segments given by q_ptr (device, int64 [n_seg+1]); every
// segment has `nbins` bins split into chunks of `bins_per_chunk`.
hipError_t launch_build_items(const int64_t* q_ptr, int64_t n_seg, int32_t nbins, int32_t bins_per_chunk,
                              int32_t tile, int64_t* scratch_counts, WorkItem* items, int32_t* n_items,
                              int64_t max_items, hipStream_t st);
hipError_t launch_regular_items(int64_t n_entries, int32_t nbins, int32_t bins_per_chunk, int32_t tile,
                                WorkItem* items, int32_t* n_items, hipStream_t st);
hipError_t launch_uniform_segs(SegDesc* segs, int64_t n_seg, int64_t stride, int32_t nbins, hipStream_t st);
hipError_t launch_row_sums(const double* M, int64_t rows, int32_t cols, double* out, hipStream_t st);
hipError_t launch_api_segments(const int32_t* lo, const int32_t* mid, const int32_t* hi, int64_t n_seg,
                               int32_t* bounds, SegDesc* segs, hipStream_t st);
hipError_t launch_split_pairs(const double* pairs, int64_t n, double* left, double* right, hipStream_t st);

// Descent over the bins of one binned pass.
struct DescArgs {
    const double* M;           // masses [entries][2^D]
    int64_t n_entries;
    int32_t D;                 // levels resolved by this pass (multi-set launch: the largest)
    int32_t start_level;       // level of the nodes the entries sit at
    int32_t L;
    uint64_t seed;
    const int32_t* entry_sample;  // pass >= 1: entry -> sample id; NULL for the root pass
    int32_t* node;             // sample -> node index at the current level (in/out)
    float* margin;             // sample -> running min margin (in/out), may be NULL
    double* deg;               // root pass: point -> degree, may be NULL
    // root passes of several point sets in one launch (jobs != NULL): entries
    // [job_entry_off[k], job_entry_off[k+1]) are job k's, with the arguments
    // jobs[k]; n_entries is the total and lds_bytes the largest job's LDS
    const DescArgs* jobs;
    const int64_t* job_entry_off;
    int32_t n_jobs;
    size_t lds_bytes;
};
hipError_t launch_descend_bins(const DescArgs& a, hipStream_t st);
// LDS bytes and Philox level groups of a root descent
size_t desc_root_lds(const DescArgs& a, int32_t* n_groups);

struct LeafArgs {
    const float* X;            // FP32 points
    const double* norm;        // FP64 ||x||^2
    int64_t n;
    int32_t d;
    const int32_t* bounds;     // boundaries of the nodes at `level`
    int32_t level;
    double s;                  // gamma * log2(e)
    int32_t kind;              // fsg_kernel of the exponent
    int32_t L;
    uint64_t seed;
    const int32_t* sorted_samples;  // samples ordered by node
    const int32_t* node_start;      // node -> first position in sorted_samples ([n_nodes+1])
    const int32_t* items;           // (node, first position) pairs, 64 samples per item
    const int32_t* n_items;
    int32_t* nbr;
    float* margin;
    // precision mode, exact KDE: the root pass's keep masks (index order, a
    // row of root_blocks 16-column blocks per 64-entry tile of the pivot
    // order) and the points' pivot positions; NULL: every point is evaluated
    const uint16_t* root_mask;
    int64_t root_blocks;
    const int32_t* inv;
    // several point sets in one launch (jobs != NULL): their samples were
    // grouped by one sort over global node ids (job k's nodes are
    // [job_node_off[k], job_node_off[k+1])); items and n_items are the
    // combined work list (global node, global position), node_start the
    // combined node starts (global positions) and sorted_samples the combined
    // list of job-local sample ids; jobs[k] holds job k's other arguments
    const LeafArgs* jobs;
    const int32_t* job_node_off;
    int32_t n_jobs;
};
// The grouping keys of several jobs' samples in one launch: sample s of job k
// (global position sample_off[k] + s) gets key node_off[k] + node, or
// inactive_key when it has no node (its neighbour is then set to -1), and the
// value s.
struct LeafKeyJob {
    const int32_t* node;
    int32_t* nbr;
};
hipError_t launch_multi_node_keys(const LeafKeyJob* jobs, const int64_t* sample_off, const int32_t* node_off,
                                  int32_t n_jobs, int64_t total, uint32_t inactive_key, uint32_t* keys, int32_t* vals,
                                  hipStream_t st);
// max_items: the item bound of one set, or the slots of all jobs
hipError_t launch_leaf(const LeafArgs& a, int64_t max_items, int num_cus, hipStream_t st);
int leaf_class(int32_t d);  // the class of d a leaf launch is built for (2, 4, ..., 128)

// Samples: sort ids by node; inactive samples (node < 0) go last.
hipError_t launch_init_samples(int64_t n_samples, int32_t* node, float* margin, hipStream_t st);
hipError_t launch_node_keys(const int32_t* node, int64_t n_samples, uint32_t inactive_key, uint32_t* keys,
                            int32_t* vals, hipStream_t st);
// start[v] = first position whose key >> key_shift is >= v
hipError_t launch_node_starts(const uint32_t* sorted_keys, int64_t n_samples, int64_t n_nodes, int32_t* start,
                              hipStream_t st, int32_t key_shift = 0);
// keys node << sub_bits | (inv[s / L] >> sub_shift) (inactive: inactive_node <<
// sub_bits): the samples of a node ordered by where their points lie in the
// pivot order
hipError_t launch_node_keys_sub(const int32_t* node, int64_t n_samples, int32_t L, const int32_t* inv,
                                int32_t sub_shift, int32_t sub_bits, uint32_t inactive_node, uint32_t* keys,
                                int32_t* vals, hipStream_t st);
hipError_t launch_entry_points(const int32_t* sorted_samples, int64_t n, int32_t L, int32_t* q_idx,
                               hipStream_t st);
hipError_t launch_leaf_items(const int32_t* node_start, int64_t n_nodes, int64_t* scratch, int32_t* items,
                             int32_t* n_items, hipStream_t st);
hipError_t launch_finish_inactive(const int32_t* node, int64_t n_samples, int32_t* nbr, hipStream_t st);
hipError_t launch_node_qptr(const int32_t* node_start, int64_t n_nodes, int64_t* q_ptr, hipStream_t st);

// Stable LSD radix sort of 32- or 64-bit keys with int32 values over the low
// `bits` key bits.  tmp buffers must hold n elements each.
struct SortBufs {
    void* keys_tmp;     // n keys
    int32_t* vals_tmp;  // n values
    uint32_t* hist;     // sort_hist_elems(n)
    uint32_t* partials; // scan_partials(sort_hist_elems(n)) + 1
};
int64_t sort_hist_elems(int64_t n);
hipError_t radix_sort_u32(uint32_t* keys, int32_t* vals, int64_t n, int bits, const SortBufs& b, hipStream_t st);
hipError_t radix_sort_u64(uint64_t* keys, int32_t* vals, int64_t n, int bits, const SortBufs& b, hipStream_t st);

// Exclusive scan (three phases, tiles of 4096); out may alias in; *total
// receives the sum; partials needs scan_partials(n) elements.
int64_t scan_partials(int64_t n);
hipError_t launch_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total, int64_t* partials,
                                     hipStream_t st);
hipError_t launch_exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                                     uint32_t* partials, hipStream_t st);

// CSR.
hipError_t launch_csr_emit(const int32_t* nbr, int64_t n, int32_t L, uint64_t* keys, int32_t* vals, hipStream_t st);
hipError_t launch_csr_flags(const uint64_t* keys, int64_t m, uint64_t sentinel, int64_t* flags, hipStream_t st);
struct CsrArgs {
    const uint64_t* keys;    // sorted directed entries row*n + col (sentinel n*n)
    const int64_t* pos;      // exclusive scan of the unique flags, pos[m] = nnz
    const int64_t* flags;
    int64_t m;
    int64_t n;
    int32_t d;
    const float* X;
    const double* deg;
    double s;                // gamma * log2(e)
    int32_t kind;            // fsg_kernel of the weights
    int32_t L;
    int64_t* row_ptr;
    int32_t* col;
    float* w;
    int64_t cap;
};

struct CsrRowArgs {
    int32_t* ent;            // entries grouped by row, sorted and unique at the start of each row
    const uint32_t* in_off;  // exclusive scan of the incoming counts [n + 1]; row i starts at L i + in_off[i]
    int64_t n;
    int32_t d;
    const float* X;
    const double* deg;
    double s;                // gamma * log2(e)
    int32_t kind;            // fsg_kernel of the weights
    int32_t L;
    int64_t* row_ptr;        // [n + 1]: exclusive scan of the unique counts (written by the caller)
    int32_t* col;
    float* w;
    int64_t cap;
    // rows filled in this order (NULL: index order); the pivot order keeps a
    // cluster's rows, whose neighbours are mostly in the same cluster, together
    const int32_t* row_order;
};
bool job_finished(const fsg_job* j);
void server_detach(fsg_server* s);  // release everything a server holds on its context
void build_bytes_estimate(const fsg_ctx* ctx, int64_t n, int32_t d, int32_t L, fsg_precision prec,
                          uint64_t* resident, uint64_t* transient);
fsg_status csr_rows_async(fsg_ctx* ctx, const fsg_points* X, double gamma, int32_t L, const int32_t* nbr_dev,
                          const double* deg_dev, int64_t* row_ptr_dev, int32_t* col_dev, float* w_dev, int64_t cap,
                          int32_t* n_long_dev);
hipError_t launch_csr_rows(const CsrRowArgs& a, const int32_t* nbr, int32_t L, uint32_t* cnt, uint32_t* fillc,
                           uint32_t* off, uint32_t* off_partials, int64_t* uniq, int64_t* uniq_partials,
                           int32_t* n_long, hipStream_t st);
hipError_t launch_csr_fill(const CsrArgs& a, hipStream_t st);

}  // namespace fsg
