// C ABI of libfsg.so: argument checks, workspace, pass planning and the
// orchestration of the kernels on the context's stream.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include <algorithm>
#include <cmath>
#include "common.h"


namespace fsg {

fsg_status set_error(fsg_ctx* ctx, fsg_status s, const std::string& msg) {
    if (ctx) ctx->last_error = msg;
    return s;
}

static hipEvent_t take_event(fsg_ctx* ctx) {
    if (!ctx->free_events.empty()) {
        hipEvent_t e = ctx->free_events.back();
        ctx->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

StageTimer::StageTimer(fsg_ctx* c, const char* n) : ctx(c), name(n) {
    if (!ctx->profiling) return;
    start = take_event(ctx);
    if (start) (void)hipEventRecord(start, ctx->stream);
}

StageTimer::~StageTimer() {
    if (!ctx->profiling || !start) return;
    hipEvent_t stop = take_event(ctx);
    if (!stop) return;
    (void)hipEventRecord(stop, ctx->stream);
    ctx->marks.push_back({name, {start, stop}});
}

void dev_free(fsg_ctx* ctx, void* p) {
    if (!p) return;
    if (ctx && !ctx->graphs.empty()) ctx->retired.push_back(p);
    else (void)hipFree(p);
}

void host_free(fsg_ctx* ctx, void* p) {
    if (!p) return;
    if (ctx && !ctx->graphs.empty()) ctx->retired_host.push_back(p);
    else (void)hipHostFree(p);
}

// free what was parked while graphs existed (none exists any more)
static void free_retired(fsg_ctx* ctx) {
    if (ctx->retired.empty() && ctx->retired_host.empty()) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : ctx->retired) (void)hipFree(p);
    for (void* p : ctx->retired_host) (void)hipHostFree(p);
    ctx->retired.clear();
    ctx->retired_host.clear();
}

fsg_status ws_get(fsg_ctx* ctx, const char* name, size_t bytes, void** out) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = ctx->bufs.find(name);
    if (it != ctx->bufs.end() && it->second.second >= bytes) {
        *out = it->second.first;
        return FSG_OK;
    }
    size_t old = 0;
    if (it != ctx->bufs.end()) {
        old = it->second.second;
        // the stream may still use the old buffer, and a recorded graph may
        // name it (then it is parked until the last graph is destroyed)
        FSG_HIP(ctx, hipStreamSynchronize(ctx->stream));
        dev_free(ctx, it->second.first);
        ctx->held -= old;
        ctx->bufs.erase(it);
    }
    if (ctx->held + bytes > ctx->budget)
        return set_error(ctx, FSG_E_BUDGET,
                         std::string("workspace budget exceeded by buffer ") + name + " (" + std::to_string(bytes) +
                             " bytes, " + std::to_string(ctx->held) + " held, budget " +
                             std::to_string(ctx->budget) + ")");
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, FSG_E_NOMEM, std::string("hipMalloc of workspace ") + name + " failed");
    }
    ctx->bufs[name] = {p, bytes};
    ctx->held += bytes;
    *out = p;
    return FSG_OK;
}

template <typename T>
static fsg_status ws(fsg_ctx* ctx, const char* name, size_t count, T** out) {
    void* p = nullptr;
    fsg_status s = ws_get(ctx, name, count * sizeof(T), &p);
    *out = (T*)p;
    return s;
}

static bool gamma_ok(double g) { return std::isfinite(g) && g > 0.0; }


// Largest total of cached point-set blocks; beyond it released blocks are freed.
constexpr size_t kPoolCacheCap = (size_t)16 << 30;

hipError_t pool_alloc(fsg_ctx* ctx, size_t bytes, void** out) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = ctx->pool_free.lower_bound(bytes);
    if (it != ctx->pool_free.end() && it->first <= 2 * bytes) {
        *out = it->second;
        ctx->pool_cached -= it->first;
        ctx->pool_free.erase(it);
        return hipSuccess;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess && !ctx->pool_free.empty()) {
        // drop the cache and try once more
        (void)hipGetLastError();
        (void)hipStreamSynchronize(ctx->stream);
        for (auto& kv : ctx->pool_free) {
            ctx->pool_size.erase(kv.second);
            dev_free(ctx, kv.second);
        }
        ctx->pool_free.clear();
        ctx->pool_cached = 0;
        e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) return e;
    ctx->pool_size[p] = bytes;
    *out = p;
    return hipSuccess;
}

void pool_release(fsg_ctx* ctx, void* p) {
    if (!p) return;
    auto it = ctx->pool_size.find(p);
    if (it == ctx->pool_size.end()) {
        dev_free(ctx, p);
        return;
    }
    if (ctx->pool_cached + it->second > kPoolCacheCap) {
        (void)hipStreamSynchronize(ctx->stream);
        dev_free(ctx, p);
        ctx->pool_size.erase(it);
        return;
    }
    ctx->pool_free.emplace(it->second, p);
    ctx->pool_cached += it->second;
}

void pool_clear(fsg_ctx* ctx) {
    for (auto& kv : ctx->pool_free) (void)hipFree(kv.second);
    ctx->pool_free.clear();
    ctx->pool_size.clear();
    ctx->pool_cached = 0;
}

// a point-set array: pooled while the point set is attached to its context
template <typename T>
static hipError_t pts_alloc(fsg_points* p, size_t count, T** out) {
    void* v = nullptr;
    hipError_t e = p->ctx ? pool_alloc(p->ctx, count * sizeof(T), &v) : hipMalloc(&v, count * sizeof(T));
    *out = (T*)v;
    return e;
}

static void pts_free(fsg_points* p, void* v) {
    if (!v) return;
    if (p->ctx) {
        pool_release(p->ctx, v);
    } else {
        (void)hipFree(v);
    }
}

static const int32_t* level_bounds(fsg_points* pts, int level, fsg_status* st) {
    auto it = pts->levels.find(level);
    if (it != pts->levels.end()) {
        *st = FSG_OK;
        return it->second;
    }
    int32_t* p = nullptr;
    const size_t count = ((size_t)1 << level) + 1;
    hipError_t e = pts_alloc(pts, count, &p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *st = set_error(pts->ctx, FSG_E_NOMEM, "hipMalloc of tree level boundaries failed");
        return nullptr;
    }
    e = launch_level_bounds(pts->n, level, p, pts->ctx->stream);
    if (e != hipSuccess) {
        pts_free(pts, p);
        *st = set_error(pts->ctx, FSG_E_DEVICE, std::string("level bounds: ") + hipGetErrorString(e));
        return nullptr;
    }
    pts->levels[level] = p;
    pts->bytes += count * sizeof(int32_t);
    *st = FSG_OK;
    return p;
}

static int floor_log2(int64_t v) {
    int r = -1;
    while (v > 0) {
        v >>= 1;
        ++r;
    }
    return r;
}

static int bit_length(uint64_t v) {
    int r = 0;
    while (v) {
        v >>= 1;
        ++r;
    }
    return r;
}

// The levels of the tree are resolved in passes.  A binned pass starting at
// level `start` computes, for every entry, the masses of the 2^D nodes D
// levels below the entry's node; the leaf stage finishes nodes of at most
// kLeafMax points.
struct Plan {
    int leaf_level = 0;
    std::vector<std::pair<int, int>> passes;  // (start level, D)
};

// Deepest root pass of the precision mode from 2^19 points on: the exact
// pass closes every bin of every tile and splits its gathered blocks at bin
// boundaries, so with few kept columns per bin a shallower root (one more
// later pass over the kept columns) is cheaper -- measured on a 50-cluster
// mixture at n = 1e6, D = 10 takes 3% less time than 11; at n = 1e5, 11 is 6%
// faster than 10.
constexpr int kPrecisionRootMaxD = 10;
constexpr int64_t kPrecisionShallowRoot = (int64_t)1 << 19;

static Plan make_plan(int64_t n, int32_t L, uint64_t budget, int cap, fsg_precision prec) {
    Plan p;
    int lv = 0;
    while ((n + ((int64_t)1 << lv) - 1) >> lv > kLeafMax) ++lv;
    p.leaf_level = lv;
    int start = 0;
    const uint64_t per_pass = budget / 2;
    while (start < lv) {
        const uint64_t rows = (start == 0) ? (uint64_t)n : (uint64_t)n * (uint64_t)L;
        int maxD = floor_log2((int64_t)(per_pass / (rows * 8)));
        // the root descent keeps its sum tree in LDS (2^(D+1) doubles); later
        // passes keep 2^D bins per sample in registers
        int hard = (start == 0) ? 11 : 6;
        if (start == 0 && prec == FSG_BF16_SPLIT && n >= kPrecisionShallowRoot) hard = kPrecisionRootMaxD;
        if (maxD > hard) maxD = hard;
        if (cap > 0 && maxD > cap) maxD = cap;
        if (maxD < 1) maxD = 1;
        int D = lv - start;
        if (D > maxD) D = maxD;
        p.passes.push_back({start, D});
        start += D;
    }
    return p;
}

static int tree_depth(int64_t n) {
    int dpt = 0;
    while (((int64_t)1 << dpt) < n) ++dpt;
    return dpt;
}

static KdeArgs kde_args(const fsg_points* Q, const fsg_points* X, double gamma, int32_t kind = FSG_GAUSSIAN) {
    KdeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.kind = kind;
    a.qpts = Q->X;
    a.xpts = X->X;
    a.d = X->d;
    a.Qp = Q->Xp;
    a.qnorm = Q->norm;
    a.Xp = X->Xp;
    a.xnorm = X->norm;
    a.D4 = X->D4;
    a.n_query = Q->n;
    a.n_data = X->n;
    a.s = gamma * 1.442695040888963407359924681001892137;
    if (kind == FSG_GAUSSIAN && Q->Xs && X->Xs) {
        a.Qs = Q->Xs;
        a.qe = Q->xe;
        a.Xs = X->Xs;
        a.xe = X->xe;
    }
    return a;
}

// Precision-mode margin: pairs whose exponent exceeds the row's smallest by
// more than ln(n) + kMarginExtra are dropped; their total is below
// e^-kMarginExtra (1.4e-11) of the row's degree.
constexpr double kMarginExtra = 25.0;

// Bins per work item of a root pass: about 32 items per wave of the grid.
// In the precision mode the item boundaries decide how kept columns are
// grouped, hence the rounding order of the bin sums, so every root pass of a
// point set uses this one rule.
static int32_t root_bins_per_item(const fsg_ctx* ctx, int64_t tiles, int32_t nbins) {
    const int64_t waves = (int64_t)ctx->num_cus * 8;
    int64_t chunks = (32 * waves + tiles - 1) / tiles;
    if (chunks > nbins) chunks = nbins;
    if (chunks < 1) chunks = 1;
    int64_t bpc = (nbins + chunks - 1) / chunks;
    // whole 128-byte lines (16 doubles) of each output row per item, so that
    // no line is written back in part by two items
    if (nbins >= 16) bpc = std::min<int64_t>(nbins, (bpc + 15) / 16 * 16);
    return (int32_t)bpc;
}

// 16-column blocks per keep-mask chunk.  Work items (chunk, group of tiles)
// go round-robin to the waves, so the slowest wave does rounds x chunk
// blocks plus a start-up per item (loading its query operands, worth about
// kItemStart blocks): the chunk is chosen to make that smallest, which mostly
// means a chunk count that just fills whole rounds.  A chunk's operands
// (16 x 64 x KB bytes per block) are capped at 3 MB: every item reloads its
// query operands, so longer chunks cut that traffic (at n = 1e6, 1.5 MB chunks
// were 4% slower), while at 6 MB the chunks the waves share no longer stay in
// an XCD's 4 MB L2 (2% slower).
static int64_t mask_chunk_blocks(int64_t n_blocks, int64_t n_groups, int64_t n_waves, int KB) {
    constexpr int64_t kItemStart = 16, kChunkBytes = 3072 * 1024;
    const int64_t max_bpc = std::max<int64_t>(32, std::min<int64_t>(1024, kChunkBytes / (16 * 64 * KB)));
    int64_t best_bpc = n_blocks, best = INT64_MAX;
    for (int64_t c = (n_blocks + max_bpc - 1) / max_bpc; c <= (n_blocks + 31) / 32; ++c) {
        const int64_t bpc = (n_blocks + c - 1) / c;
        const int64_t chunks = (n_blocks + bpc - 1) / bpc;
        const int64_t rounds = (chunks * n_groups + n_waves - 1) / n_waves;
        const int64_t load = rounds * (bpc + kItemStart);
        if (load < best || (load == best && bpc > best_bpc)) {
            best = load;
            best_bpc = bpc;
        }
    }
    return best_bpc;
}

// Keep-mask arguments of a root pass over point set X (precision mode):
// entries are the points in pivot order, so that each 64-query tile holds
// points close together and keeps few columns.
// kde_error = 0: drop only pairs more than Delta = ln n + 25 below their
// row's largest term (the exact mode); kde_error = eps > 0: Delta = ln(n-1) +
// ln(1/eps), so that the dropped total is below eps of every degree.
static double margin_for(int64_t n, double kde_error) {
    if (kde_error > 0.0 && n >= 2) return std::log((double)(n - 1)) - std::log(kde_error);
    return std::log((double)n) + kMarginExtra;
}

// The index-order split fragments and -|x|^2/2 of a point set, which only a
// scan over every tile reads (the pruned scan reads the pivot-order copies):
// written on the first such scan.  Under stream capture the launch is
// recorded each time, so that an eager call never reads them unwritten.
static fsg_status ensure_index_split(fsg_ctx* ctx, fsg_points* X) {
    if (X->xb_ready) return FSG_OK;
    FSG_HIP(ctx, launch_prep_split(X->X, X->norm, X->n, X->d, X->KB, X->n_pad, X->Xb, X->xa, ctx->stream));
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    FSG_HIP(ctx, hipStreamIsCapturing(ctx->stream, &cs));
    if (cs == hipStreamCaptureStatusNone) X->xb_ready = true;
    return FSG_OK;
}

static MaskArgs root_mask_args(const fsg_points* X, double gamma, int num_cus, int32_t kind = FSG_GAUSSIAN,
                               double kde_error = 0.0) {
    MaskArgs m;
    std::memset(&m, 0, sizeof(m));
    m.kind = kind;
    const int64_t n = X->n;
    m.Xb = X->Xb;
    m.Qb = X->Qb;
    m.xa = X->xa;
    m.KB = X->KB;
    m.q_idx = X->order;
    m.n_entries = n;
    m.n_query = n;
    m.n_data = n;
    m.qnorm = X->norm;
    m.dmin = X->dmin;
    m.xmax = X->xmax;
    m.margin_z = margin_for(n, kde_error);
    m.eps = 1.0 / 1024.0;
    m.gamma = gamma;
    m.n_tiles = (n + kTileQ - 1) / kTileQ;
    m.n_blocks = X->n_pad / 16;
    const int tp = mask_tiles_per_item(m.KB);
    m.blocks_per_chunk = mask_chunk_blocks(m.n_blocks, (m.n_tiles + tp - 1) / tp, keep_mask_waves(m.KB, num_cus), m.KB);
    m.n_chunks = (m.n_blocks + m.blocks_per_chunk - 1) / m.blocks_per_chunk;
    return m;
}

fsg_status kde_segmented_check(fsg_ctx* ctx, const fsg_points* Q, const fsg_points* X, double gamma, int64_t n_seg,
                               int64_t n_entries, const int64_t* q_ptr, const int32_t* q_idx, const int32_t* lo,
                               const int32_t* mid, const int32_t* hi, const double* out_left,
                               const double* out_right, bool* empty) {
    *empty = false;
    if (!ctx) return FSG_E_INVALID;
    if (!Q || !X) return set_error(ctx, FSG_E_INVALID, "NULL points");
    if (Q->ctx != ctx || X->ctx != ctx) return set_error(ctx, FSG_E_INVALID, "points belong to another context");
    if (Q->d != X->d) return set_error(ctx, FSG_E_INVALID, "Q and X differ in d");
    if (!gamma_ok(gamma)) return set_error(ctx, FSG_E_INVALID, "gamma must be finite and > 0");
    if (n_seg < 0 || n_entries < 0) return set_error(ctx, FSG_E_INVALID, "negative count");
    if (n_seg > 2147483647LL || n_entries > 2147483647LL)
        return set_error(ctx, FSG_E_UNSUPPORTED, "more than 2^31-1 segments or entries");
    if (n_seg == 0 || n_entries == 0) {
        *empty = true;
        return FSG_OK;
    }
    if (!q_ptr || !q_idx || !lo || !mid || !hi || !out_left || !out_right)
        return set_error(ctx, FSG_E_INVALID, "NULL array");
    return FSG_OK;
}

KdeSegSizes kde_segmented_sizes(const fsg_points* X, int64_t n_seg, int64_t n_entries) {
    KdeSegSizes z;
    z.tile = kde_tile(X->D4);
    z.max_items = n_entries / z.tile + n_seg + 1;
    z.bounds = 3 * n_seg;
    // segment item counts and offsets (n_seg + 1 each), their total, scan partials
    z.counts = 2 * (n_seg + 1) + 1 + scan_partials(n_seg);
    z.pairs = 2 * n_entries;
    return z;
}

fsg_status kde_segmented_enqueue(fsg_ctx* ctx, const fsg_points* Q, const fsg_points* X, double gamma,
                                 int64_t n_seg, int64_t n_entries, const int64_t* q_ptr, const int32_t* q_idx,
                                 const int32_t* lo, const int32_t* mid, const int32_t* hi, const int32_t* self_idx,
                                 double* out_left, double* out_right, const KdeSegBufs& b) {
    const KdeSegSizes z = kde_segmented_sizes(X, n_seg, n_entries);
    FSG_HIP(ctx, launch_api_segments(lo, mid, hi, n_seg, b.bounds, b.segs, ctx->stream));
    FSG_HIP(ctx, launch_build_items(q_ptr, n_seg, 2, 2, z.tile, b.counts, b.items, b.n_items, z.max_items,
                                    ctx->stream));
    KdeArgs a = kde_args(Q, X, gamma, ctx->kernel);
    a.q_idx = q_idx;
    a.self_idx = self_idx;
    a.self_mode = self_idx ? SELF_ARRAY : SELF_NONE;
    a.bounds = b.bounds;
    a.segs = b.segs;
    a.items = b.items;
    a.n_items = b.n_items;
    a.out = b.pairs;
    a.out_stride = 2;
    FSG_HIP(ctx, launch_kde(a, z.max_items, ctx->num_cus, ctx->stream));
    FSG_HIP(ctx, launch_split_pairs(b.pairs, n_entries, out_left, out_right, ctx->stream));
    return FSG_OK;
}

// entries of a keep-threshold array for n entries
static int64_t theta_entries(int64_t n) { return (n + kThetaPad - 1) / kThetaPad * kThetaPad; }

// The keep masks of a root pass (m: the full scan's arguments, mask in index
// order) from the pruned scan: cells the tiles may keep columns of, work items
// over the data in pivot order, the scan, and the conversion of its keep bits
// to index order.  The kept set equals the full scan's.
static fsg_status pruned_keep_mask(fsg_ctx* ctx, const fsg_points* X, const MaskArgs& m0) {
    fsg_status st;
    const int64_t n = X->n;
    const int TP = mask_tiles_per_item(m0.KB);
    PruneArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.X = X->X;
    pa.n = n;
    pa.d = X->d;
    pa.P = X->P;
    pa.order = X->order;
    pa.qnorm = X->norm;
    pa.dmin = X->dmin;
    pa.xmax = X->xmax;
    pa.margin_z = m0.margin_z;
    pa.eps = m0.eps;
    pa.gamma = m0.gamma;
    pa.kind = m0.kind;
    pa.cell_pivot = X->cell_pivot;
    pa.pnorm = X->pnorm;
    pa.prad = X->prad;
    pa.cell_start = X->cell_start;
    pa.n_tiles = m0.n_tiles;
    pa.words = (X->P + 31) / 32;
    pa.TP = TP;
    pa.n_groups = (m0.n_tiles + TP - 1) / TP;
    // chunks of about 1.5 MB of data operands, so that the chunks an XCD
    // scans at one time stay in its 4 MB L2
    const int64_t n_blocks_p = theta_entries(n) / 16;
    pa.n_blocks_p = n_blocks_p;
    pa.chunk_blocks = (int32_t)std::max<int64_t>(32, std::min<int64_t>(1024, (1536 * 1024) / (1024 * m0.KB)));
    pa.n_chunks = (n_blocks_p + pa.chunk_blocks - 1) / pa.chunk_blocks;
    const int64_t pairs = pa.n_chunks * pa.n_groups;
    const int64_t max_items = prune_max_items(pa.n_groups, pa.P, pa.n_chunks);
    int64_t* partials;
    uint16_t* maskp;
    if ((st = ws(ctx, "prune_surv", (size_t)(pa.n_tiles * pa.words), &pa.surv)) != FSG_OK) return st;
    if ((st = ws(ctx, "prune_counts", (size_t)pairs + 1, &pa.counts)) != FSG_OK) return st;
    if ((st = ws(ctx, "prune_offsets", (size_t)pairs + 1, &pa.offsets)) != FSG_OK) return st;
    if ((st = ws(ctx, "prune_bcounts", (size_t)pairs + 1, &pa.bcounts)) != FSG_OK) return st;
    if ((st = ws(ctx, "prune_boffsets", (size_t)pairs + 1, &pa.boffsets)) != FSG_OK) return st;
    if ((st = ws(ctx, "prune_total", 2 + kXcds + 1, &pa.total)) != FSG_OK) return st;
    pa.xseg = pa.total + 2;
    if ((st = ws(ctx, "prune_partials", (size_t)scan_partials(pairs + 1), &partials)) != FSG_OK) return st;
    if ((st = ws(ctx, "prune_items", (size_t)(3 * max_items), &pa.items)) != FSG_OK) return st;
    if ((st = ws(ctx, "keep_mask_pivot", (size_t)(m0.n_tiles * n_blocks_p), &maskp)) != FSG_OK) return st;
    pa.scanned = m0.kept ? m0.kept + 1 : nullptr;
    {
        StageTimer t(ctx, "prune");
        FSG_HIP(ctx, launch_prune_plan(pa, ctx->stream));
        FSG_HIP(ctx, launch_prune_items(pa, partials, ctx->stream));
    }
    MaskArgs m = m0;
    m.Xb = X->Xbp;
    m.xa = X->xap;
    m.mask = maskp;
    m.n_blocks = n_blocks_p;
    m.list = pa.items;
    m.xseg = pa.xseg;
    {
        StageTimer t(ctx, "kde_mask");
        FSG_HIP(ctx, launch_keep_mask(m, ctx->num_cus, ctx->stream));
    }
    StageTimer t(ctx, "mask_convert");
    FSG_HIP(ctx, launch_mask_to_index(pa, maskp, n_blocks_p, m0.mask, m0.n_blocks, ctx->stream));
    return FSG_OK;
}

// Binned KDE of all n points against the nodes of tree level D (one segment).
// In the precision mode the root pass's keep masks (index order, a row per
// 64-entry tile of the pivot order) are returned through root_mask and
// root_blocks when asked for: the later passes of the same build use them.
static fsg_status root_bins(fsg_ctx* ctx, fsg_points* X, double gamma, int D, double* M,
                            const uint16_t** root_mask = nullptr, int64_t* root_blocks = nullptr) {
    fsg_status st;
    if (X->prec == FSG_BF16_SPLIT && ctx->kernel == FSG_LAPLACIAN)
        return set_error(ctx, FSG_E_UNSUPPORTED, "the Laplacian kernel runs in the plain path only");
    const int32_t* bnd = level_bounds(X, D, &st);
    if (!bnd) return st;
    const int64_t n = X->n;
    const int32_t nbins = 1 << D;
    const bool sliced = ctx->slices != 0 && X->Xs && ctx->kernel == FSG_GAUSSIAN;
    const int32_t tile = (X->prec == FSG_BF16_SPLIT) ? exact_tile(X->D4, sliced) : kde_tile(X->D4);
    const int64_t tiles = (n + tile - 1) / tile;
    const int32_t bpc = root_bins_per_item(ctx, tiles, nbins);
    const int64_t n_items = tiles * ((nbins + bpc - 1) / bpc);
    WorkItem* items;
    SegDesc* segs;
    int32_t* n_items_dev;
    if ((st = ws(ctx, "root_items", (size_t)n_items, &items)) != FSG_OK) return st;
    if ((st = ws(ctx, "root_segs", 1, &segs)) != FSG_OK) return st;
    if ((st = ws(ctx, "root_nitems", 1, &n_items_dev)) != FSG_OK) return st;
    FSG_HIP(ctx, launch_uniform_segs(segs, 1, 0, nbins, ctx->stream));
    FSG_HIP(ctx, launch_regular_items(n, nbins, bpc, tile, items, n_items_dev, ctx->stream));
    KdeArgs a = kde_args(X, X, gamma, ctx->kernel);
    if (!sliced) {
        a.Qs = a.Xs = nullptr;
        a.qe = a.xe = nullptr;
    }
    a.q_idx = nullptr;
    a.self_mode = SELF_POINT;
    a.bounds = bnd;
    a.segs = segs;
    a.items = items;
    a.n_items = n_items_dev;
    a.out = M;
    a.out_stride = nbins;
    if (X->prec == FSG_BF16_SPLIT) {
        // entries in pivot order, so that each wave's 64 queries are close
        // together and keep few columns; rows are written by point
        a.q_idx = X->order;
        a.out_rows = X->order;
        MaskArgs m = root_mask_args(X, gamma, ctx->num_cus, ctx->kernel, ctx->kde_error);
        float* ntheta;
        if ((st = ws(ctx, "mask_theta", (size_t)theta_entries(n), &ntheta)) != FSG_OK) return st;
        FSG_HIP(ctx, launch_mask_theta(m, ntheta, theta_entries(n), ctx->stream));
        m.ntheta = ntheta;
        if ((st = ws(ctx, "keep_mask", (size_t)(m.n_tiles * m.n_blocks), &m.mask)) != FSG_OK) return st;
        if (ctx->filter_counts == nullptr) {
            if (hipMalloc(&ctx->filter_counts, 2 * sizeof(int64_t)) != hipSuccess) {
                (void)hipGetLastError();
                return set_error(ctx, FSG_E_NOMEM, "hipMalloc of filter statistics failed");
            }
            FSG_HIP(ctx, launch_fill_i64(ctx->filter_counts, 2, 0, ctx->stream));
        }
        m.kept = ctx->filter_counts;
        const bool prune = ctx->pruning > 0 || (ctx->pruning < 0 && n >= kPruneMinPoints);
        if (prune && X->Xbp) {
            if ((st = pruned_keep_mask(ctx, X, m)) != FSG_OK) return st;
        } else {
            if ((st = ensure_index_split(ctx, X)) != FSG_OK) return st;
            // pairs examined: every data column once per 64-query tile
            FSG_HIP(ctx, launch_add_i64(ctx->filter_counts + 1, tiles * n, ctx->stream));
            StageTimer t(ctx, "kde_mask");
            FSG_HIP(ctx, launch_keep_mask(m, ctx->num_cus, ctx->stream));
        }
        int64_t* next_item;
        if ((st = ws(ctx, "exact_next_item", 1, &next_item)) != FSG_OK) return st;
        FSG_HIP(ctx, launch_fill_i64(next_item, 1, 0, ctx->stream));
        StageTimer t(ctx, "kde_root");
        a.mask = m.mask;
        a.n_blocks = m.n_blocks;
        FSG_HIP(ctx, launch_exact_kept(a, n_items, (unsigned long long*)next_item, ctx->num_cus, ctx->stream));
        if (root_mask) *root_mask = m.mask;
        if (root_blocks) *root_blocks = m.n_blocks;
        return FSG_OK;
    }
    {
        StageTimer t(ctx, "kde_root");
        FSG_HIP(ctx, launch_kde(a, n_items, ctx->num_cus, ctx->stream));
    }
    return FSG_OK;
}

static SortBufs sort_bufs(fsg_ctx* ctx, int64_t n, size_t key_bytes, fsg_status* st) {
    SortBufs b{};
    void* p;
    if ((*st = ws_get(ctx, "sort_keys_tmp", n * key_bytes, &p)) != FSG_OK) return b;
    b.keys_tmp = p;
    if ((*st = ws(ctx, "sort_vals_tmp", (size_t)n, &b.vals_tmp)) != FSG_OK) return b;
    const int64_t h = sort_hist_elems(n);
    if ((*st = ws(ctx, "sort_hist", (size_t)h, &b.hist)) != FSG_OK) return b;
    if ((*st = ws(ctx, "sort_partials", (size_t)scan_partials(h) + 1, &b.partials)) != FSG_OK) return b;
    return b;
}

// Orders the samples by their node at `level` (2^level nodes); inactive
// samples last.  Returns sorted sample ids and node starts, in the given
// buffers ([ns], [2^level + 1]) or else in the workspace.
// With sub (the pivot positions of the points, n of them, L samples per
// point) the samples of each node are further ordered by where their points
// lie in the pivot order, to the precision the 24-bit key leaves.
static fsg_status group_by_node(fsg_ctx* ctx, const int32_t* node, int64_t ns, int level, int32_t** sorted,
                                int32_t** starts, int32_t* vals_out = nullptr, int32_t* starts_out = nullptr,
                                const int32_t* sub = nullptr, int64_t n = 0, int32_t L = 1) {
    fsg_status st;
    uint32_t* keys;
    int32_t* vals = vals_out;
    int32_t* start = starts_out;
    const int64_t n_nodes = (int64_t)1 << level;
    if ((st = ws(ctx, "grp_keys", (size_t)ns, &keys)) != FSG_OK) return st;
    if (!vals && (st = ws(ctx, "grp_vals", (size_t)ns, &vals)) != FSG_OK) return st;
    if (!start && (st = ws(ctx, "grp_starts", (size_t)n_nodes + 1, &start)) != FSG_OK) return st;
    SortBufs b = sort_bufs(ctx, ns, sizeof(uint32_t), &st);
    if (st != FSG_OK) return st;
    const int node_bits = bit_length((uint64_t)n_nodes);
    const int pos_bits = bit_length((uint64_t)std::max<int64_t>(n - 1, 1));
    const int sub_bits = sub ? std::min(pos_bits, std::max(0, 24 - node_bits)) : 0;
    StageTimer t(ctx, "group");
    if (sub_bits > 0)
        FSG_HIP(ctx, launch_node_keys_sub(node, ns, L, sub, pos_bits - sub_bits, sub_bits, (uint32_t)n_nodes, keys,
                                          vals, ctx->stream));
    else
        FSG_HIP(ctx, launch_node_keys(node, ns, (uint32_t)n_nodes, keys, vals, ctx->stream));
    FSG_HIP(ctx, radix_sort_u32(keys, vals, ns, node_bits + sub_bits, b, ctx->stream));
    FSG_HIP(ctx, launch_node_starts(keys, ns, n_nodes, start, ctx->stream, sub_bits));
    *sorted = vals;
    *starts = start;
    return FSG_OK;
}

// Precision-mode arrays of a point set: split BF16 operands, distance bounds
// from pivots and the pivot order of the points.
static fsg_status prep_precision_mode(fsg_ctx* ctx, fsg_points* p) {
    const int KB = filter_steps(p->D4);
    p->KB = KB;
    const size_t split_bytes = (size_t)(p->n_pad / 16) * KB * 64 * 16;
    const int64_t n = p->n;
    const int64_t q_rows = (n + kThetaPad - 1) / kThetaPad * kThetaPad;
    const size_t q_split_bytes = (size_t)(q_rows / 16) * KB * 64 * 16;
    uint32_t* label = nullptr;
    auto fail = [&](const char* what) {
        (void)hipGetLastError();
        return set_error(ctx, FSG_E_NOMEM, std::string("hipMalloc of ") + what + " failed");
    };
    char* xb = nullptr;
    char* qb = nullptr;
    if (pts_alloc(p, split_bytes, &xb) != hipSuccess) return fail("split operands");
    p->Xb = xb;
    if (pts_alloc(p, q_split_bytes, &qb) != hipSuccess) return fail("split operands");
    p->Qb = qb;
    if (pts_alloc(p, (size_t)n, &p->dmin) != hipSuccess) return fail("distance bounds");
    // the pivot order padded to whole 16-point blocks (read a block at a time)
    if (pts_alloc(p, (size_t)((n + 15) & ~(int64_t)15), &p->order) != hipSuccess) return fail("pivot order");
    if (pts_alloc(p, 1, &p->xmax) != hipSuccess) return fail("norm bound");
    if (pts_alloc(p, (size_t)p->n_pad, &p->xa) != hipSuccess) return fail("norm terms");
    const int32_t P = (int32_t)(n < 256 ? n : 256);
    p->P = P;
    char* xbp = nullptr;
    if (pts_alloc(p, q_split_bytes, &xbp) != hipSuccess) return fail("split operands");
    p->Xbp = xbp;
    if (pts_alloc(p, (size_t)q_rows, &p->xap) != hipSuccess) return fail("norm terms");
    if (pts_alloc(p, (size_t)P + 1, &p->cell_start) != hipSuccess) return fail("cell table");
    if (pts_alloc(p, (size_t)P, &p->cell_pivot) != hipSuccess) return fail("cell table");
    if (pts_alloc(p, (size_t)P, &p->pnorm) != hipSuccess) return fail("cell table");
    if (pts_alloc(p, (size_t)P, &p->prad) != hipSuccess) return fail("cell table");
    if (pts_alloc(p, (size_t)n, &p->inv) != hipSuccess) return fail("pivot positions");
    p->bytes += split_bytes + 2 * q_split_bytes + n * (sizeof(double) + sizeof(int32_t)) + sizeof(double) +
                p->n_pad * sizeof(float) + q_rows * sizeof(float) + (4 * (size_t)P + 1) * 4 + n * sizeof(int32_t);
    // the exact recompute's integer slices (32 < d <= 64)
    const bool sliced = p->D4 == 16;
    if (sliced) {
        if (pts_alloc(p, (size_t)p->n_pad * kSliceRow, &p->Xs) != hipSuccess) return fail("integer slices");
        if (pts_alloc(p, (size_t)p->n_pad, &p->xe) != hipSuccess) return fail("integer slices");
        p->bytes += (size_t)p->n_pad * (kSliceRow + sizeof(int32_t));
    }
    fsg_status st;
    if ((st = ws(ctx, "pivot_labels", (size_t)n, &label)) != FSG_OK) return st;
    SortBufs b = sort_bufs(ctx, n, sizeof(uint32_t), &st);
    if (st != FSG_OK) return st;
    double* part;
    if ((st = ws(ctx, "max_norm_parts", (size_t)max_norm_parts(n), &part)) != FSG_OK) return st;
    uint16_t* d16;
    int32_t* rank;
    if ((st = ws(ctx, "pivot_dist16", (size_t)P * P, &d16)) != FSG_OK) return st;
    if ((st = ws(ctx, "pivot_rank", (size_t)P, &rank)) != FSG_OK) return st;
    StageTimer t(ctx, "prep");
    if (sliced) FSG_HIP(ctx, launch_prep_slices(p->X, n, p->d, p->n_pad, p->Xs, p->xe, ctx->stream));
    FSG_HIP(ctx, launch_pivots(p->X, n, p->d, P, p->dmin, label, p->order, ctx->stream));
    // cells labelled along a nearest-neighbour chain of the pivots, so that
    // neighbouring cells of the pivot order are close together
    FSG_HIP(ctx, launch_pivot_chain(p->X, n, p->d, P, d16, rank, p->cell_pivot, label, ctx->stream));
    FSG_HIP(ctx, radix_sort_u32(label, p->order, n, 8, b, ctx->stream));
    FSG_HIP(ctx, launch_inverse_order(p->order, n, p->inv, ctx->stream));
    FSG_HIP(ctx, launch_prep_query_split(p->X, p->order, n, p->d, KB, q_rows, p->Qb, ctx->stream));
    FSG_HIP(ctx, launch_max_norm(p->norm, n, part, p->xmax, ctx->stream));
    // the pruned scan: cells of the pivot order, data operands in that order
    FSG_HIP(ctx, launch_node_starts(label, n, P, p->cell_start, ctx->stream));
    FSG_HIP(ctx, launch_prep_split_order(p->X, p->norm, p->order, n, p->d, KB, q_rows, p->Xbp, p->xap, ctx->stream));
    FSG_HIP(ctx, launch_cell_geometry(p->X, p->d, P, p->dmin, p->order, p->cell_start, p->cell_pivot, p->pnorm,
                                      p->prad, ctx->stream));
    return FSG_OK;
}

// ---------------------------------------------------------------------------
// One build's sampling state, advanced stage by stage: the root pass (binned
// KDE over all points, then the descent over its bins), later binned passes,
// and the leaf stage.  fsg_sample_edges runs the stages back to back; a batch
// job runs one stage per fsg_batch_step (the root passes of many jobs share
// launches).
// ---------------------------------------------------------------------------
struct Sampler {
    fsg_points* X = nullptr;
    double gamma = 0.0;
    int32_t kind = FSG_GAUSSIAN;  // fsg_kernel
    int32_t L = 0;
    uint64_t seed = 0;
    Plan plan;
    int64_t ns = 0;
    int32_t* node = nullptr;   // [ns] current node of every sample
    double* deg = nullptr;     // [n] degrees (NULL: not wanted)
    int32_t* nbr = nullptr;    // [ns] result
    float* margin = nullptr;   // [ns] optional decision margins
    // precision mode, exact KDE: the root pass's keep masks, which the later
    // passes narrow their columns to (NULL: later passes scan every column)
    const uint16_t* root_mask = nullptr;
    int64_t root_blocks = 0;
};

static fsg_status sampler_plan(fsg_ctx* ctx, Sampler& S) {
    S.ns = S.X->n * (int64_t)S.L;
    if (S.ns > 2147483647LL) return set_error(ctx, FSG_E_UNSUPPORTED, "n*L must be < 2^31");
    S.plan = make_plan(S.X->n, S.L, ctx->budget, ctx->max_levels_per_pass, S.X->prec);
    return FSG_OK;
}

static DescArgs desc_args(const Sampler& S, size_t p) {
    DescArgs da;
    std::memset(&da, 0, sizeof(da));
    da.D = S.plan.passes[p].second;
    da.start_level = S.plan.passes[p].first;
    da.L = S.L;
    da.seed = S.seed;
    da.node = S.node;
    da.margin = S.margin;
    return da;
}

// descent over the root pass's bins M [n][2^D]
static fsg_status stage_root_descend(fsg_ctx* ctx, const Sampler& S, const double* M) {
    DescArgs da = desc_args(S, 0);
    da.M = M;
    da.n_entries = S.X->n;
    da.entry_sample = nullptr;
    da.deg = S.deg;
    StageTimer t(ctx, "descend");
    FSG_HIP(ctx, launch_descend_bins(da, ctx->stream));
    return FSG_OK;
}

// later binned pass p >= 1: samples grouped by node, binned KDE of every
// sample's point over its node, descent
static fsg_status stage_pass(fsg_ctx* ctx, const Sampler& S, size_t p) {
    fsg_points* X = S.X;
    const int start = S.plan.passes[p].first, D = S.plan.passes[p].second;
    const int32_t nbins = 1 << D;
    const int64_t ns = S.ns;
    fsg_status st;
    const int64_t n_nodes = (int64_t)1 << start;
    // precision mode with the root pass's masks: every item reads only the
    // columns its samples' points kept at the root (W blocks per item at
    // most: a node holds at most ceil(n / 2^start) points)
    // later passes recompute in FP64 (64-query items): their items hold few
    // kept columns each, where the integer slices' 32-query items cost more
    const int32_t tile_m = exact_tile(X->D4, false);
    const int64_t max_items_m = ns / tile_m + n_nodes + 1;
    const int64_t node_max = (X->n + n_nodes - 1) / n_nodes;
    const int32_t W = (int32_t)((node_max + 15) / 16 + 2);
    const bool masked = S.root_mask != nullptr && X->inv != nullptr &&
                        (uint64_t)max_items_m * W * sizeof(uint16_t) <= ctx->budget / 8;
    int32_t *sorted, *starts;
    if ((st = group_by_node(ctx, S.node, ns, start, &sorted, &starts, nullptr, nullptr, masked ? X->inv : nullptr,
                            X->n, S.L)) != FSG_OK)
        return st;
    const int32_t* bnd = level_bounds(X, start + D, &st);
    if (!bnd) return st;
    int64_t* q_ptr;
    int32_t* q_idx;
    SegDesc* segs;
    WorkItem* items;
    int32_t* n_items;
    int64_t* scratch;
    double* M;
    const int32_t tile = masked ? tile_m : kde_tile(X->D4);
    const int64_t max_items = ns / tile + n_nodes + 1;
    if ((st = ws(ctx, "pass_qptr", (size_t)n_nodes + 1, &q_ptr)) != FSG_OK) return st;
    if ((st = ws(ctx, "pass_qidx", (size_t)ns, &q_idx)) != FSG_OK) return st;
    if ((st = ws(ctx, "pass_segs", (size_t)n_nodes, &segs)) != FSG_OK) return st;
    if ((st = ws(ctx, "pass_items", (size_t)max_items, &items)) != FSG_OK) return st;
    if ((st = ws(ctx, "pass_nitems", 1, &n_items)) != FSG_OK) return st;
    if ((st = ws(ctx, "pass_scratch", (size_t)(2 * (n_nodes + 1) + 1 + scan_partials(n_nodes)), &scratch)) != FSG_OK)
        return st;
    if ((st = ws(ctx, "pass_masses", (size_t)ns << D, &M)) != FSG_OK) return st;
    FSG_HIP(ctx, launch_node_qptr(starts, n_nodes, q_ptr, ctx->stream));
    FSG_HIP(ctx, launch_entry_points(sorted, ns, S.L, q_idx, ctx->stream));
    FSG_HIP(ctx, launch_uniform_segs(segs, n_nodes, nbins, nbins, ctx->stream));
    FSG_HIP(ctx, launch_build_items(q_ptr, n_nodes, nbins, nbins, tile, scratch, items, n_items, max_items,
                                    ctx->stream));
    KdeArgs a = kde_args(X, X, S.gamma, S.kind);
    a.Qs = a.Xs = nullptr;
    a.qe = a.xe = nullptr;
    a.q_idx = q_idx;
    a.self_idx = q_idx;
    a.self_mode = SELF_ARRAY;
    a.bounds = bnd;
    a.segs = segs;
    a.items = items;
    a.n_items = n_items;
    a.out = M;
    a.out_stride = nbins;
    if (masked) {
        uint16_t* pmask;
        int64_t* next_item;
        if ((st = ws(ctx, "pass_mask", (size_t)(max_items * W), &pmask)) != FSG_OK) return st;
        if ((st = ws(ctx, "exact_next_item", 1, &next_item)) != FSG_OK) return st;
        {
            StageTimer t(ctx, "pass_mask");
            FSG_HIP(ctx, launch_pass_mask(a, max_items, X->inv, S.root_mask, S.root_blocks, W, pmask, ctx->stream));
        }
        FSG_HIP(ctx, launch_fill_i64(next_item, 1, 0, ctx->stream));
        a.mask = pmask;
        a.n_blocks = W;
        a.mask_by_item = 1;
        StageTimer t(ctx, "kde_pass");
        FSG_HIP(ctx, launch_exact_kept(a, max_items, (unsigned long long*)next_item, ctx->num_cus, ctx->stream));
    } else {
        StageTimer t(ctx, "kde_pass");
        FSG_HIP(ctx, launch_kde(a, max_items, ctx->num_cus, ctx->stream));
    }
    DescArgs da = desc_args(S, p);
    da.M = M;
    da.n_entries = ns;
    da.entry_sample = sorted;
    da.deg = nullptr;
    StageTimer t(ctx, "descend");
    FSG_HIP(ctx, launch_descend_bins(da, ctx->stream));
    return FSG_OK;
}

// leaf stage: nodes of at most kLeafMax points resolved with exact kernel
// values; the degrees come from here too when there was no binned pass
// leaf-stage arguments of sampler S (node boundaries bnd at its leaf level,
// samples grouped by node, work items)
static LeafArgs leaf_args(const Sampler& S, const int32_t* bnd, const int32_t* sorted, const int32_t* starts,
                          const int32_t* items, const int32_t* n_items) {
    LeafArgs la;
    std::memset(&la, 0, sizeof(la));
    const fsg_points* X = S.X;
    la.X = X->X;
    la.norm = X->norm;
    la.n = X->n;
    la.d = X->d;
    la.bounds = bnd;
    la.level = S.plan.leaf_level;
    la.s = S.gamma * 1.442695040888963407359924681001892137;
    la.kind = S.kind;
    la.L = S.L;
    la.seed = S.seed;
    la.sorted_samples = sorted;
    la.node_start = starts;
    la.items = items;
    la.n_items = n_items;
    la.nbr = S.nbr;
    la.margin = S.margin;
    if (S.root_mask != nullptr && X->inv != nullptr) {
        la.root_mask = S.root_mask;
        la.root_blocks = S.root_blocks;
        la.inv = X->inv;
    }
    return la;
}

// work items of a leaf stage over 2^level nodes: at most this many
static int64_t leaf_max_items(int64_t ns, int level) { return ns / 64 + ((int64_t)1 << level) + 1; }

static fsg_status stage_leaf(fsg_ctx* ctx, const Sampler& S) {
    fsg_points* X = S.X;
    const int64_t ns = S.ns;
    fsg_status st;
    int32_t *sorted, *starts;
    // with the root pass's masks, a node's samples are ordered by pivot
    // position, so that an item's samples share few root tiles
    const bool masked = S.root_mask != nullptr && X->inv != nullptr;
    if ((st = group_by_node(ctx, S.node, ns, S.plan.leaf_level, &sorted, &starts, nullptr, nullptr,
                            masked ? X->inv : nullptr, X->n, S.L)) != FSG_OK)
        return st;
    const int64_t n_nodes = (int64_t)1 << S.plan.leaf_level;
    const int32_t* bnd = level_bounds(X, S.plan.leaf_level, &st);
    if (!bnd) return st;
    int32_t* items;
    int32_t* n_items;
    int64_t* scratch;
    const int64_t max_items = leaf_max_items(ns, S.plan.leaf_level);
    if ((st = ws(ctx, "leaf_items", (size_t)(2 * max_items), &items)) != FSG_OK) return st;
    if ((st = ws(ctx, "leaf_nitems", 1, &n_items)) != FSG_OK) return st;
    if ((st = ws(ctx, "leaf_scratch", (size_t)(2 * (n_nodes + 1) + 1 + scan_partials(n_nodes)), &scratch)) != FSG_OK)
        return st;
    {
        StageTimer t(ctx, "leaf");
        FSG_HIP(ctx, launch_leaf_items(starts, n_nodes, scratch, items, n_items, ctx->stream));
        const LeafArgs la = leaf_args(S, bnd, sorted, starts, items, n_items);
        FSG_HIP(ctx, launch_leaf(la, max_items, ctx->num_cus, ctx->stream));
        FSG_HIP(ctx, launch_finish_inactive(S.node, ns, S.nbr, ctx->stream));
    }
    return FSG_OK;
}

// Row-sorted CSR (Algorithm 2's reweighting) enqueued without
// synchronisation: row_ptr[n] receives 2|E| on the device and *n_long_dev the
// number of rows longer than the row sort handles (their rows are left empty:
// the caller then rebuilds with fsg_build_csr, which falls back to a global
// sort).  cap >= 2 n L always suffices.
fsg_status csr_rows_async(fsg_ctx* ctx, const fsg_points* X, double gamma, int32_t L, const int32_t* nbr_dev,
                          const double* deg_dev, int64_t* row_ptr_dev, int32_t* col_dev, float* w_dev, int64_t cap,
                          int32_t* n_long_dev) {
    const int64_t n = X->n;
    const int64_t m = 2 * n * (int64_t)L;
    if (m > 2147483647LL) return set_error(ctx, FSG_E_UNSUPPORTED, "2*n*L must be < 2^31");
    fsg_status st;
    int32_t* ent;
    uint32_t *cnt, *fillc, *off, *off_part;
    int64_t *uniq, *uniq_part;
    if ((st = ws(ctx, "csr_ent", (size_t)m + 1, &ent)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_cnt", (size_t)n + 1, &cnt)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_fillc", (size_t)n + 1, &fillc)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_off", (size_t)n + 1, &off)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_off_part", (size_t)scan_partials(n) + 1, &off_part)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_uniq", (size_t)n + 1, &uniq)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_uniq_part", (size_t)scan_partials(n) + 1, &uniq_part)) != FSG_OK) return st;
    CsrRowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ent = ent;
    a.in_off = off;
    a.n = n;
    a.d = X->d;
    a.X = X->X;
    a.deg = deg_dev;
    a.s = gamma * 1.442695040888963407359924681001892137;
    a.kind = ctx->kernel;
    a.L = L;
    a.row_ptr = row_ptr_dev;
    a.col = col_dev;
    a.w = w_dev;
    a.cap = cap;
    a.row_order = X->order;  // the pivot order in the precision mode
    StageTimer t(ctx, "csr");
    FSG_HIP(ctx, launch_csr_rows(a, nbr_dev, L, cnt, fillc, off, off_part, uniq, uniq_part, n_long_dev, ctx->stream));
    return FSG_OK;
}

// ---------------------------------------------------------------------------
// Batching: jobs, and the root pass of many jobs in one launch.
// ---------------------------------------------------------------------------
static fsg_status ensure_filter_counts(fsg_ctx* ctx) {
    if (ctx->filter_counts != nullptr) return FSG_OK;
    if (hipMalloc(&ctx->filter_counts, 2 * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, FSG_E_NOMEM, "hipMalloc of filter statistics failed");
    }
    FSG_HIP(ctx, launch_fill_i64(ctx->filter_counts, 2, 0, ctx->stream));
    return FSG_OK;
}

// Device tables of one group of jobs (same feature-step class and precision)
// for one launch shape; built once per (jobs, shape) and reused, so that
// repeated batches (and graph replays) upload nothing.
struct BatchTables {
    std::vector<fsg_job*> jobs;
    int waves_per_cu = 8;
    int cols = 2048;
    int32_t slices = -1;        // the context's integer-slice setting the tables were built with
    void* dev = nullptr;        // one block: KdeArgs[G] SegDesc[G] BatchItemDesc[G+1] MaskArgs[G] int64[G+1] counter
    void* host = nullptr;       // pinned staging of the same layout
    size_t bytes = 0;
    WorkItem* items = nullptr;  // [total_items]
    int32_t* n_items = nullptr;
    int64_t total_items = 0;
    int64_t mask_items = 0;
    int64_t scanned = 0;        // (column, tile) pairs the filter examines
    KdeArgs a0;                 // launch arguments (job tables bound)
    MaskArgs m0;
    unsigned long long* counter = nullptr;
};

static void free_tables(fsg_ctx* ctx, BatchTables* T) {
    dev_free(ctx, T->dev);
    dev_free(ctx, T->items);
    host_free(ctx, T->host);
    delete T;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// device tables of a batched leaf stage: the jobs' leaf arguments and their
// work-slot offsets
// device tables of a batched leaf stage: per job its leaf arguments and its
// grouping-key entry, the jobs' sample and node offsets, and the buffers of
// the combined grouping (one sort of every job's samples by global node id)
struct LeafTables {
    std::vector<fsg_job*> jobs;
    void* dev = nullptr;   // LeafArgs[G], LeafKeyJob[G], int64[G+1] sample offsets, int32[G+1] node offsets
    void* host = nullptr;  // pinned staging of the same layout
    LeafArgs a0;           // launch arguments (tables bound; the grouping buffers are set per launch)
    const LeafKeyJob* key_jobs = nullptr;
    const int64_t* sample_off = nullptr;
    const int32_t* node_off = nullptr;
    int64_t samples = 0;   // all jobs' samples
    int64_t nodes = 0;     // all jobs' leaf-level nodes
    int64_t max_items = 0; // work items at most
};

static void free_leaf_tables(fsg_ctx* ctx, LeafTables* T) {
    dev_free(ctx, T->dev);
    host_free(ctx, T->host);
    delete T;
}

// device tables of a batched root descent: every job's descent arguments and
// entry offsets (job buffers only, so they are built once per job list)
struct DescTables {
    std::vector<fsg_job*> jobs;
    void* dev = nullptr;   // DescArgs[G], int64[G+1]
    void* host = nullptr;
    DescArgs a0;
};

static void free_desc_tables(fsg_ctx* ctx, DescTables* T) {
    dev_free(ctx, T->dev);
    host_free(ctx, T->host);
    delete T;
}


}  // namespace fsg

struct fsg_job {
    fsg_ctx* ctx = nullptr;
    fsg::Sampler S;
    int stage = 0;
    int n_stages = 0;
    int root_D = 0;
    double* M = nullptr;       // root-pass bins [n][2^root_D]
    uint16_t* mask = nullptr;  // precision mode: keep masks of the root pass
    float* ntheta = nullptr;   // precision mode: keep-thresholds of the root pass
    std::vector<void*> owned;  // device blocks from the context's pool
};

struct fsg_graph {
    fsg_ctx* ctx = nullptr;  // cleared if the context is destroyed first
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace fsg {

static void* job_alloc(fsg_job* j, size_t bytes, fsg_status* st) {
    void* p = nullptr;
    if (pool_alloc(j->ctx, bytes, &p) != hipSuccess) {
        (void)hipGetLastError();
        *st = set_error(j->ctx, FSG_E_NOMEM, "hipMalloc of job buffers failed");
        return nullptr;
    }
    j->owned.push_back(p);
    return p;
}

static void batch_cache_drop(fsg_ctx* ctx, const fsg_job* j) {
    auto& c = ctx->batch_cache;
    for (size_t i = 0; i < c.size();) {
        if (std::find(c[i]->jobs.begin(), c[i]->jobs.end(), j) != c[i]->jobs.end()) {
            (void)hipStreamSynchronize(ctx->stream);
            free_tables(ctx, c[i]);
            c.erase(c.begin() + i);
        } else {
            ++i;
        }
    }
    auto& lc = ctx->leaf_cache;
    for (size_t i = 0; i < lc.size();) {
        if (std::find(lc[i]->jobs.begin(), lc[i]->jobs.end(), j) != lc[i]->jobs.end()) {
            (void)hipStreamSynchronize(ctx->stream);
            free_leaf_tables(ctx, lc[i]);
            lc.erase(lc.begin() + i);
        } else {
            ++i;
        }
    }
    auto& dc = ctx->desc_cache;
    for (size_t i = 0; i < dc.size();) {
        if (std::find(dc[i]->jobs.begin(), dc[i]->jobs.end(), j) != dc[i]->jobs.end()) {
            (void)hipStreamSynchronize(ctx->stream);
            free_desc_tables(ctx, dc[i]);
            dc.erase(dc.begin() + i);
        } else {
            ++i;
        }
    }
}

// the arguments of job j's root pass as a plain single-set launch would use them
static fsg_status job_root_args(fsg_ctx* ctx, fsg_job* j, KdeArgs* a, MaskArgs* m) {
    fsg_points* X = j->S.X;
    fsg_status st;
    const int32_t* bnd = level_bounds(X, j->root_D, &st);
    if (!bnd) return st;
    const int64_t n = X->n;
    *a = kde_args(X, X, j->S.gamma);
    a->self_mode = SELF_POINT;
    a->bounds = bnd;
    a->out = j->M;
    a->out_stride = (int64_t)1 << j->root_D;
    std::memset(m, 0, sizeof(*m));
    if (X->prec == FSG_BF16_SPLIT) {
        a->q_idx = X->order;
        a->out_rows = X->order;
        a->mask = j->mask;
        a->n_blocks = X->n_pad / 16;
        if ((st = ensure_index_split(ctx, X)) != FSG_OK) return st;
        *m = root_mask_args(X, j->S.gamma, ctx->num_cus);
        m->ntheta = j->ntheta;
        m->mask = j->mask;
    }
    return FSG_OK;
}

static fsg_status batch_tables(fsg_ctx* ctx, const std::vector<fsg_job*>& g, int waves_per_cu, int cols,
                               BatchTables** out) {
    for (BatchTables* T : ctx->batch_cache)
        if (T->jobs == g && T->waves_per_cu == waves_per_cu && T->cols == cols && T->slices == ctx->slices) {
            *out = T;
            return FSG_OK;
        }
    const int32_t G = (int32_t)g.size();
    const bool bf16 = g[0]->S.X->prec == FSG_BF16_SPLIT;
    const size_t o_args = 0;
    const size_t o_segs = align256(o_args + G * sizeof(KdeArgs));
    const size_t o_desc = align256(o_segs + G * sizeof(SegDesc));
    const size_t o_margs = align256(o_desc + (G + 1) * sizeof(BatchItemDesc));
    const size_t o_moff = align256(o_margs + G * sizeof(MaskArgs));
    const size_t o_cnt = align256(o_moff + (G + 1) * sizeof(int64_t));
    const size_t bytes = align256(o_cnt + sizeof(unsigned long long));
    BatchTables* T = new BatchTables();
    T->jobs = g;
    T->waves_per_cu = waves_per_cu;
    T->cols = cols;
    T->slices = ctx->slices;
    T->bytes = bytes;
    auto fail = [&](fsg_status s) {
        free_tables(ctx, T);
        return s;
    };
    if (hipMalloc(&T->dev, bytes) != hipSuccess || hipHostMalloc(&T->host, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(ctx, FSG_E_NOMEM, "allocation of batch tables failed"));
    }
    char* h = (char*)T->host;
    char* d = (char*)T->dev;
    std::memset(h, 0, bytes);
    KdeArgs* hargs = (KdeArgs*)(h + o_args);
    SegDesc* hsegs = (SegDesc*)(h + o_segs);
    BatchItemDesc* hdesc = (BatchItemDesc*)(h + o_desc);
    MaskArgs* hmargs = (MaskArgs*)(h + o_margs);
    int64_t* hmoff = (int64_t*)(h + o_moff);
    int64_t total = 0, mtotal = 0;
    fsg_status st;
    // one exact-recompute variant per launch: the integer slices only where
    // every set of the launch has them
    bool all_sliced = bf16 && ctx->slices != 0;
    for (int32_t i = 0; i < G; ++i) all_sliced = all_sliced && g[i]->S.X->Xs != nullptr;
    for (int32_t i = 0; i < G; ++i) {
        fsg_job* j = g[i];
        if ((st = job_root_args(ctx, j, &hargs[i], &hmargs[i])) != FSG_OK) return fail(st);
        if (!all_sliced) {
            hargs[i].Qs = hargs[i].Xs = nullptr;
            hargs[i].qe = hargs[i].xe = nullptr;
        }
        const int64_t n = j->S.X->n;
        const int32_t nbins = 1 << j->root_D;
        const int32_t tile = bf16 ? exact_tile(j->S.X->D4, all_sliced) : kde_tile(j->S.X->D4);
        const int64_t n_tiles = (n + tile - 1) / tile;
        int64_t bpc;
        if (bf16) {
            // item shape as in the single-set pass (see root_bins_per_item);
            // `cols` sets the keep-mask kernel's data columns per work item
            bpc = root_bins_per_item(ctx, n_tiles, nbins);
            MaskArgs& m = hmargs[i];
            if (cols > 0) {  // 0: the set's own balanced chunk
                m.blocks_per_chunk = cols / 16;
                m.n_chunks = (m.n_blocks + m.blocks_per_chunk - 1) / m.blocks_per_chunk;
            }
        } else {
            bpc = (int64_t)std::llround((double)cols * nbins / (double)n);
            if (bpc < 1) bpc = 1;
            if (bpc > nbins) bpc = nbins;
        }
        const int64_t n_chunks = (nbins + bpc - 1) / bpc;
        hsegs[i].bound_off = 0;
        hsegs[i].nbins = nbins;
        hsegs[i].job = i;
        hdesc[i].item_off = total;
        hdesc[i].n_entries = n;
        hdesc[i].nbins = nbins;
        hdesc[i].bpc = (int32_t)bpc;
        hdesc[i].tile = tile;
        hdesc[i].n_tiles = (int32_t)n_tiles;
        total += n_tiles * n_chunks;
        hmoff[i] = mtotal;
        if (bf16) {
            mtotal += mask_items(hmargs[i]);
            T->scanned += hmargs[i].n_tiles * n;
        }
    }
    hdesc[G].item_off = total;
    hmoff[G] = mtotal;
    T->total_items = total;
    T->mask_items = mtotal;
    if (total > 2147483647LL) return fail(set_error(ctx, FSG_E_UNSUPPORTED, "more than 2^31-1 work items in a batch"));
    if (hipMalloc(&T->items, total * sizeof(WorkItem) + 256) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(ctx, FSG_E_NOMEM, "allocation of batch work items failed"));
    }
    T->n_items = (int32_t*)((char*)T->items + total * sizeof(WorkItem));
    T->counter = (unsigned long long*)(d + o_cnt);
    hipError_t e = hipMemcpyAsync(T->dev, T->host, bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_batch_items((const BatchItemDesc*)(d + o_desc), G, total, T->items, T->n_items, ctx->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(ctx, FSG_E_DEVICE, std::string("batch tables: ") + hipGetErrorString(e)));
    }
    T->a0 = hargs[0];
    T->a0.jobs = (const KdeArgs*)(d + o_args);
    T->a0.segs = (const SegDesc*)(d + o_segs);
    T->a0.items = T->items;
    T->a0.n_items = T->n_items;
    T->m0 = hmargs[0];
    T->m0.jobs = (const MaskArgs*)(d + o_margs);
    T->m0.job_item_off = (const int64_t*)(d + o_moff);
    T->m0.n_jobs = G;
    T->m0.n_items_total = mtotal;
    ctx->batch_cache.push_back(T);
    *out = T;
    return FSG_OK;
}

// the KDE launches of a batched root pass
static fsg_status batch_root_launch(fsg_ctx* ctx, BatchTables* T, bool stats) {
    if (T->jobs[0]->S.X->prec == FSG_BF16_SPLIT) {
        MaskArgs m = T->m0;
        m.kept = nullptr;
        if (stats) {
            fsg_status st;
            if ((st = ensure_filter_counts(ctx)) != FSG_OK) return st;
            m.kept = ctx->filter_counts;
            FSG_HIP(ctx, launch_add_i64(ctx->filter_counts + 1, T->scanned, ctx->stream));
        }
        {
            StageTimer t(ctx, "kde_mask");
            FSG_HIP(ctx, launch_keep_mask(m, ctx->num_cus, ctx->stream));
        }
        FSG_HIP(ctx, launch_fill_i64((int64_t*)T->counter, 1, 0, ctx->stream));
        StageTimer t(ctx, "kde_root");
        FSG_HIP(ctx, launch_exact_kept(T->a0, T->total_items, T->counter, ctx->num_cus, ctx->stream));
        return FSG_OK;
    }
    StageTimer t(ctx, "kde_root");
    FSG_HIP(ctx, launch_kde(T->a0, T->total_items, ctx->num_cus, ctx->stream, T->waves_per_cu));
    return FSG_OK;
}

static bool stream_capturing(fsg_ctx* ctx) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs != hipStreamCaptureStatusNone;
}

// Root passes of a group of jobs in one launch (per KDE stage), with the
// launch shape tuned on the group's first use when autotuning is on.
static fsg_status batch_root(fsg_ctx* ctx, const std::vector<fsg_job*>& g) {
    const fsg_points* X0 = g[0]->S.X;
    const std::pair<int, int> key(X0->D4, (int)X0->prec);
    auto it = ctx->tuned.find(key);
    const bool bf16 = X0->prec == FSG_BF16_SPLIT;
    int waves = 8, cols = bf16 ? 0 : 2048;
    fsg_status st;
    if (it != ctx->tuned.end()) {
        waves = it->second.first;
        cols = it->second.second;
    } else if (ctx->autotune && !stream_capturing(ctx)) {
        hipEvent_t e0, e1;
        FSG_HIP(ctx, hipEventCreate(&e0));
        FSG_HIP(ctx, hipEventCreate(&e1));
        float best = 3.0e38f;
        // plain: grid size and data columns per item; precision mode: data
        // columns per keep-mask item (the filter kernels fix their occupancy,
        // and the exact pass keeps the single-set item shape)
        const int wave_opts[3] = {4, 8, 12};
        const int col_opts[3] = {1024, 2048, 4096};
        const int mask_col_opts[3] = {0, 4096, 8192};
        for (int wi = 0; wi < 3; ++wi) {
            if (bf16 && wave_opts[wi] != 8) continue;
            for (int ci = 0; ci < 3; ++ci) {
                const int cand = bf16 ? mask_col_opts[ci] : col_opts[ci];
                BatchTables* T;
                if ((st = batch_tables(ctx, g, wave_opts[wi], cand, &T)) != FSG_OK) return st;
                FSG_HIP(ctx, hipEventRecord(e0, ctx->stream));
                if ((st = batch_root_launch(ctx, T, false)) != FSG_OK) return st;
                FSG_HIP(ctx, hipEventRecord(e1, ctx->stream));
                FSG_HIP(ctx, hipEventSynchronize(e1));
                float ms = 0.0f;
                FSG_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    waves = wave_opts[wi];
                    cols = cand;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        // keep only the tables of the chosen shape
        auto& c = ctx->batch_cache;
        for (size_t i = 0; i < c.size();) {
            if (c[i]->jobs == g && !(c[i]->waves_per_cu == waves && c[i]->cols == cols)) {
                free_tables(ctx, c[i]);
                c.erase(c.begin() + i);
            } else {
                ++i;
            }
        }
        ctx->tuned[key] = {waves, cols};
    }
    BatchTables* T;
    if ((st = batch_tables(ctx, g, waves, cols, &T)) != FSG_OK) return st;
    return batch_root_launch(ctx, T, true);
}

// the device tables of a group's leaf stage (built on its first use, cached)
static fsg_status leaf_tables(fsg_ctx* ctx, const std::vector<fsg_job*>& g, LeafTables** out) {
    for (LeafTables* T : ctx->leaf_cache)
        if (T->jobs == g) {
            *out = T;
            return FSG_OK;
        }
    const int32_t G = (int32_t)g.size();
    const size_t o_keyjobs = align256(G * sizeof(LeafArgs));
    const size_t o_soff = align256(o_keyjobs + G * sizeof(LeafKeyJob));
    const size_t o_noff = align256(o_soff + (G + 1) * sizeof(int64_t));
    const size_t bytes = align256(o_noff + (G + 1) * sizeof(int32_t));
    LeafTables* T = new LeafTables();
    T->jobs = g;
    auto fail = [&](fsg_status s) {
        free_leaf_tables(ctx, T);
        return s;
    };
    int64_t S = 0, N = 0;
    for (const fsg_job* j : g) {
        S += j->S.ns;
        N += (int64_t)1 << j->S.plan.leaf_level;
    }
    if (S + 1 > 2147483647LL || N + 1 > 2147483647LL)
        return fail(set_error(ctx, FSG_E_UNSUPPORTED, "a batched leaf stage holds more than 2^31 samples or nodes"));
    T->samples = S;
    T->nodes = N;
    T->max_items = S / 64 + N + 1;
    if (hipMalloc(&T->dev, bytes) != hipSuccess || hipHostMalloc(&T->host, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(ctx, FSG_E_NOMEM, "allocation of leaf tables failed"));
    }
    char* h = (char*)T->host;
    std::memset(h, 0, bytes);
    LeafArgs* hargs = (LeafArgs*)h;
    LeafKeyJob* hkey = (LeafKeyJob*)(h + o_keyjobs);
    int64_t* hsoff = (int64_t*)(h + o_soff);
    int32_t* hnoff = (int32_t*)(h + o_noff);
    int64_t soff = 0;
    int32_t noff = 0;
    fsg_status st;
    for (int32_t i = 0; i < G; ++i) {
        const fsg_job* j = g[i];
        const int32_t* bnd = level_bounds(j->S.X, j->S.plan.leaf_level, &st);
        if (!bnd) return fail(st);
        // (the combined grouping arrays are the launch's, in a0)
        hargs[i] = leaf_args(j->S, bnd, nullptr, nullptr, nullptr, nullptr);
        hkey[i].node = j->S.node;
        hkey[i].nbr = j->S.nbr;
        hsoff[i] = soff;
        hnoff[i] = noff;
        soff += j->S.ns;
        noff += (int32_t)(1 << j->S.plan.leaf_level);
    }
    hsoff[G] = soff;
    hnoff[G] = noff;
    const hipError_t e = hipMemcpyAsync(T->dev, T->host, bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(set_error(ctx, FSG_E_DEVICE, std::string("leaf tables: ") + hipGetErrorString(e)));
    }
    T->a0 = hargs[0];
    T->a0.jobs = (const LeafArgs*)T->dev;
    T->a0.job_node_off = (const int32_t*)((char*)T->dev + o_noff);
    T->a0.n_jobs = G;
    T->key_jobs = (const LeafKeyJob*)((char*)T->dev + o_keyjobs);
    T->sample_off = (const int64_t*)((char*)T->dev + o_soff);
    T->node_off = (const int32_t*)((char*)T->dev + o_noff);
    ctx->leaf_cache.push_back(T);
    *out = T;
    return FSG_OK;
}

// Leaf stages of a group of jobs (one class of d) in a few launches: one
// sort groups every job's samples by global node id (job-major, stable, so
// each node's samples keep the order the single-set sort gives them), one
// pass lists the work items of all nodes, and one kernel walks them.  Per item
// the work is that of the single-set leaf stage, so the results are the same
// bit for bit.
static fsg_status batch_leaf(fsg_ctx* ctx, const std::vector<fsg_job*>& g) {
    fsg_status st;
    LeafTables* T;
    if ((st = leaf_tables(ctx, g, &T)) != FSG_OK) return st;
    SortBufs b = sort_bufs(ctx, T->samples, sizeof(uint32_t), &st);
    if (st != FSG_OK) return st;
    int64_t* scratch;
    uint32_t* keys;
    int32_t *vals, *starts, *items;
    if ((st = ws(ctx, "leaf_scratch", (size_t)(2 * (T->nodes + 1) + 1 + scan_partials(T->nodes)), &scratch)) !=
        FSG_OK)
        return st;
    if ((st = ws(ctx, "grp_keys", (size_t)T->samples, &keys)) != FSG_OK) return st;
    if ((st = ws(ctx, "grp_vals", (size_t)T->samples, &vals)) != FSG_OK) return st;
    if ((st = ws(ctx, "grp_starts", (size_t)T->nodes + 1, &starts)) != FSG_OK) return st;
    if ((st = ws(ctx, "leaf_items", (size_t)(2 * T->max_items + 1), &items)) != FSG_OK) return st;
    {
        StageTimer t(ctx, "group");
        FSG_HIP(ctx, launch_multi_node_keys(T->key_jobs, T->sample_off, T->node_off, (int32_t)g.size(), T->samples,
                                            (uint32_t)T->nodes, keys, vals, ctx->stream));
        FSG_HIP(ctx, radix_sort_u32(keys, vals, T->samples, bit_length((uint64_t)T->nodes), b, ctx->stream));
        FSG_HIP(ctx, launch_node_starts(keys, T->samples, T->nodes, starts, ctx->stream));
    }
    StageTimer t(ctx, "leaf");
    FSG_HIP(ctx, launch_leaf_items(starts, T->nodes, scratch, items, items + 2 * T->max_items, ctx->stream));
    LeafArgs a0 = T->a0;
    a0.sorted_samples = vals;
    a0.node_start = starts;
    a0.items = items;
    a0.n_items = items + 2 * T->max_items;
    FSG_HIP(ctx, launch_leaf(a0, T->max_items, ctx->num_cus, ctx->stream));
    return FSG_OK;
}

// The descents over the root bins of several jobs in one launch (a block per
// point, as for one job: the same results).
static fsg_status batch_root_descend(fsg_ctx* ctx, const std::vector<fsg_job*>& g) {
    if (g.size() == 1) return stage_root_descend(ctx, g[0]->S, g[0]->M);
    DescTables* T = nullptr;
    for (DescTables* c : ctx->desc_cache)
        if (c->jobs == g) T = c;
    if (!T) {
        const int32_t G = (int32_t)g.size();
        const size_t o_off = align256(G * sizeof(DescArgs));
        const size_t bytes = align256(o_off + (G + 1) * sizeof(int64_t));
        T = new DescTables();
        T->jobs = g;
        if (hipMalloc(&T->dev, bytes) != hipSuccess ||
            hipHostMalloc(&T->host, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            free_desc_tables(ctx, T);
            return set_error(ctx, FSG_E_NOMEM, "allocation of descent tables failed");
        }
        char* h = (char*)T->host;
        std::memset(h, 0, bytes);
        DescArgs* hargs = (DescArgs*)h;
        int64_t* hoff = (int64_t*)(h + o_off);
        int64_t total = 0;
        size_t lds = 0;
        int32_t max_D = 0;
        for (int32_t i = 0; i < G; ++i) {
            const fsg_job* j = g[i];
            DescArgs da = desc_args(j->S, 0);
            max_D = std::max(max_D, da.D);
            da.M = j->M;
            da.n_entries = j->S.X->n;
            da.entry_sample = nullptr;
            da.deg = j->S.deg;
            int32_t ng = 0;
            lds = std::max(lds, desc_root_lds(da, &ng));
            hargs[i] = da;
            hoff[i] = total;
            total += da.n_entries;
        }
        hoff[G] = total;
        const hipError_t e = hipMemcpyAsync(T->dev, T->host, bytes, hipMemcpyHostToDevice, ctx->stream);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_desc_tables(ctx, T);
            return set_error(ctx, FSG_E_DEVICE, std::string("descent tables: ") + hipGetErrorString(e));
        }
        T->a0 = hargs[0];
        T->a0.n_entries = total;
        T->a0.jobs = (const DescArgs*)T->dev;
        T->a0.job_entry_off = (const int64_t*)((char*)T->dev + o_off);
        T->a0.n_jobs = G;
        T->a0.lds_bytes = lds;
        T->a0.D = max_D;  // a multi-set launch reads each set's D from its table; this picks the kernel
        ctx->desc_cache.push_back(T);
    }
    StageTimer t(ctx, "descend");
    FSG_HIP(ctx, launch_descend_bins(T->a0, ctx->stream));
    return FSG_OK;
}

}  // namespace fsg

using namespace fsg;

extern "C" {

const char* fsg_status_string(fsg_status s) {
    switch (s) {
        case FSG_OK: return "FSG_OK";
        case FSG_E_INVALID: return "FSG_E_INVALID";
        case FSG_E_NOMEM: return "FSG_E_NOMEM";
        case FSG_E_DEVICE: return "FSG_E_DEVICE";
        case FSG_E_UNSUPPORTED: return "FSG_E_UNSUPPORTED";
        case FSG_E_BUDGET: return "FSG_E_BUDGET";
    }
    return "FSG_UNKNOWN";
}

fsg_status fsg_ctx_create(int device, void* hip_stream, uint64_t ws_budget_bytes, fsg_ctx** out) {
    if (!out) return FSG_E_INVALID;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        (void)hipGetLastError();
        return FSG_E_DEVICE;
    }
    if (device < 0 || device >= count) return FSG_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return FSG_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FSG_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FSG_E_UNSUPPORTED;
    fsg_ctx* c = new (std::nothrow) fsg_ctx();
    if (!c) return FSG_E_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->budget = ws_budget_bytes ? ws_budget_bytes : ((uint64_t)32 << 30);
    c->num_cus = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    c->noalloc_scratch = noalloc_scratch_setup(device);  // with `device` current
    if (hipHostMalloc((void**)&c->host_scratch, 64, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return FSG_E_NOMEM;
    }
    *out = c;
    return FSG_OK;
}

void fsg_ctx_destroy(fsg_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    // live graphs are detached (they can no longer be launched); what they
    // may name is freed below
    for (fsg_graph* g : ctx->graphs) g->ctx = nullptr;
    ctx->graphs.clear();
    // live point sets stay valid: their pooled blocks become theirs to free
    for (fsg_points* p : ctx->points) {
        for (void* v : {(void*)p->Xp, (void*)p->norm, (void*)p->Xb, (void*)p->Qb, (void*)p->dmin, (void*)p->order,
                        (void*)p->xmax, (void*)p->xa, (void*)p->Xbp, (void*)p->xap, (void*)p->cell_start,
                        (void*)p->cell_pivot, (void*)p->pnorm, (void*)p->prad, (void*)p->inv, (void*)p->Xs,
                        (void*)p->xe})
            if (v) ctx->pool_size.erase(v);
        for (auto& kv : p->levels) ctx->pool_size.erase(kv.second);
        p->ctx = nullptr;
    }
    {
        const std::set<fsg_server*> servers = ctx->servers;
        for (fsg_server* srv : servers) server_detach(srv);
    }
    for (BatchTables* T : ctx->batch_cache) free_tables(ctx, T);
    ctx->batch_cache.clear();
    for (LeafTables* T : ctx->leaf_cache) free_leaf_tables(ctx, T);
    ctx->leaf_cache.clear();
    for (DescTables* T : ctx->desc_cache) free_desc_tables(ctx, T);
    ctx->desc_cache.clear();
    // live jobs are detached; their buffers are freed here
    for (fsg_job* j : ctx->jobs) {
        for (void* v : j->owned) {
            ctx->pool_size.erase(v);
            (void)hipFree(v);
        }
        j->owned.clear();
        j->ctx = nullptr;
    }
    pool_clear(ctx);
    free_retired(ctx);
    for (auto& kv : ctx->bufs) (void)hipFree(kv.second.first);
    for (auto& m : ctx->marks) {
        (void)hipEventDestroy(m.second.first);
        (void)hipEventDestroy(m.second.second);
    }
    for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    if (ctx->filter_counts) (void)hipFree(ctx->filter_counts);
    if (ctx->host_scratch) (void)hipHostFree(ctx->host_scratch);
    delete ctx;
}

const char* fsg_last_error(const fsg_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

fsg_status fsg_ctx_sync(fsg_ctx* ctx) {
    if (!ctx) return FSG_E_INVALID;
    FSG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    FSG_HIP(ctx, hipGetLastError());
    return FSG_OK;
}

uint64_t fsg_ctx_workspace_bytes(const fsg_ctx* ctx) { return ctx ? ctx->held : 0; }

fsg_status fsg_ctx_set_kde_error(fsg_ctx* ctx, double eps) {
    if (!ctx) return FSG_E_INVALID;
    if (!(eps >= 0.0 && eps < 1.0)) return set_error(ctx, FSG_E_INVALID, "eps must be in [0, 1)");
    ctx->kde_error = eps;
    return FSG_OK;
}

fsg_status fsg_ctx_set_kernel(fsg_ctx* ctx, fsg_kernel kind) {
    if (!ctx) return FSG_E_INVALID;
    if (kind != FSG_GAUSSIAN && kind != FSG_EXPONENTIAL && kind != FSG_LAPLACIAN)
        return set_error(ctx, FSG_E_INVALID, "unknown kernel kind");
    ctx->kernel = kind;
    return FSG_OK;
}

fsg_status fsg_ctx_set_pruning(fsg_ctx* ctx, int32_t enabled) {
    if (!ctx) return FSG_E_INVALID;
    ctx->pruning = enabled < 0 ? -1 : (enabled > 0 ? 1 : 0);
    return FSG_OK;
}

fsg_status fsg_ctx_set_exact_slices(fsg_ctx* ctx, int32_t enabled) {
    if (!ctx) return FSG_E_INVALID;
    ctx->slices = enabled < 0 ? -1 : (enabled > 0 ? 1 : 0);
    return FSG_OK;
}

fsg_status fsg_ctx_set_levels_per_pass(fsg_ctx* ctx, int32_t max_levels) {
    if (!ctx) return FSG_E_INVALID;
    if (max_levels < 0) return set_error(ctx, FSG_E_INVALID, "max_levels must be >= 0");
    ctx->max_levels_per_pass = max_levels;
    return FSG_OK;
}

fsg_status fsg_ctx_set_profiling(fsg_ctx* ctx, int enabled) {
    if (!ctx) return FSG_E_INVALID;
    ctx->profiling = enabled != 0;
    return FSG_OK;
}

fsg_status fsg_ctx_reset_profiling(fsg_ctx* ctx) {
    if (!ctx) return FSG_E_INVALID;
    FSG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (auto& m : ctx->marks) {
        ctx->free_events.push_back(m.second.first);
        ctx->free_events.push_back(m.second.second);
    }
    ctx->marks.clear();
    if (ctx->filter_counts != nullptr) FSG_HIP(ctx, launch_fill_i64(ctx->filter_counts, 2, 0, ctx->stream));
    return FSG_OK;
}

fsg_status fsg_ctx_filter_stats(fsg_ctx* ctx, int64_t* kept, int64_t* scanned) {
    if (!ctx || !kept || !scanned) return FSG_E_INVALID;
    *kept = 0;
    *scanned = 0;
    if (ctx->filter_counts == nullptr) return FSG_OK;
    FSG_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, ctx->filter_counts, 2 * sizeof(int64_t), hipMemcpyDeviceToHost,
                                ctx->stream));
    FSG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *kept = ctx->host_scratch[0];
    *scanned = ctx->host_scratch[1];
    return FSG_OK;
}

fsg_status fsg_ctx_stage_time(fsg_ctx* ctx, const char* stage, double* ms, int64_t* launches) {
    if (!ctx || !stage || !ms || !launches) return FSG_E_INVALID;
    FSG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    double total = 0.0;
    int64_t count = 0;
    for (auto& m : ctx->marks) {
        if (m.first != stage) continue;
        float t = 0.0f;
        FSG_HIP(ctx, hipEventElapsedTime(&t, m.second.first, m.second.second));
        total += t;
        ++count;
    }
    *ms = total;
    *launches = count;
    return FSG_OK;
}

fsg_status fsg_points_create(fsg_ctx* ctx, const float* X_dev, int64_t n, int32_t d, fsg_precision prec,
                             fsg_points** out) {
    if (!ctx || !out) return FSG_E_INVALID;
    *out = nullptr;
    if (!X_dev) return set_error(ctx, FSG_E_INVALID, "X_dev is NULL");
    if (n < 1 || n > 2147483647LL) return set_error(ctx, FSG_E_INVALID, "n must be in [1, 2^31-1]");
    if (d < 1 || d > 1024) return set_error(ctx, FSG_E_INVALID, "d must be in [1, 1024]");
    if (prec != FSG_PLAIN_FP64 && prec != FSG_BF16_SPLIT) return set_error(ctx, FSG_E_INVALID, "unknown precision");
    const int D4 = feature_steps(d);
    if (D4 < 0) return set_error(ctx, FSG_E_UNSUPPORTED, "d > 128 is not built in this version");
    if (prec == FSG_BF16_SPLIT && filter_steps(D4) < 0)
        return set_error(ctx, FSG_E_UNSUPPORTED, "the precision mode is built for d <= 128");
    fsg_points* p = new (std::nothrow) fsg_points();
    if (!p) return set_error(ctx, FSG_E_NOMEM, "host allocation failed");
    p->ctx = ctx;
    p->X = X_dev;
    p->n = n;
    p->d = d;
    p->D4 = D4;
    p->n_pad = (n + 15) & ~(int64_t)15;
    p->prec = prec;
    const size_t frag = (size_t)p->n_pad * D4 * 4 * sizeof(double);
    const size_t nrm = (size_t)p->n_pad * sizeof(double);
    if (pts_alloc(p, frag / sizeof(double), &p->Xp) != hipSuccess ||
        pts_alloc(p, nrm / sizeof(double), &p->norm) != hipSuccess) {
        (void)hipGetLastError();
        pts_free(p, p->Xp);
        delete p;
        return set_error(ctx, FSG_E_NOMEM, "hipMalloc of point arrays failed");
    }
    p->bytes = frag + nrm;
    hipError_t e;
    {
        StageTimer t(ctx, "prep");
        e = launch_prep(X_dev, n, d, D4, p->n_pad, p->Xp, p->norm, ctx->stream);
    if (e != hipSuccess) {
        pts_free(p, p->Xp);
        pts_free(p, p->norm);
        delete p;
        return set_error(ctx, FSG_E_DEVICE, std::string("prep: ") + hipGetErrorString(e));
    }
    }
    if (prec == FSG_BF16_SPLIT) {
        fsg_status st = prep_precision_mode(ctx, p);
        if (st != FSG_OK) {
            fsg_points_destroy(p);
            return st;
        }
    }
    ctx->points.insert(p);
    *out = p;
    return FSG_OK;
}

void fsg_points_destroy(fsg_points* p) {
    if (!p) return;
    if (p->ctx) {
        // the arrays go back to the context's pool: work already enqueued on
        // its stream finishes before any later use of them on that stream
        p->ctx->points.erase(p);
    } else {
        (void)hipDeviceSynchronize();
    }
    pts_free(p, p->Xp);
    pts_free(p, p->norm);
    pts_free(p, p->Xb);
    pts_free(p, p->Qb);
    pts_free(p, p->dmin);
    pts_free(p, p->order);
    pts_free(p, p->xmax);
    pts_free(p, p->xa);
    pts_free(p, p->Xbp);
    pts_free(p, p->xap);
    pts_free(p, p->cell_start);
    pts_free(p, p->cell_pivot);
    pts_free(p, p->pnorm);
    pts_free(p, p->prad);
    pts_free(p, p->inv);
    pts_free(p, p->Xs);
    pts_free(p, p->xe);
    for (auto& kv : p->levels) pts_free(p, kv.second);
    delete p;
}

uint64_t fsg_points_bytes(const fsg_points* p) { return p ? p->bytes : 0; }

fsg_status fsg_degrees(fsg_ctx* ctx, const fsg_points* Xc, double gamma, double* deg_dev) {
    if (!ctx) return FSG_E_INVALID;
    if (!Xc || !deg_dev) return set_error(ctx, FSG_E_INVALID, "NULL argument");
    if (Xc->ctx != ctx) return set_error(ctx, FSG_E_INVALID, "points belong to another context");
    if (!gamma_ok(gamma)) return set_error(ctx, FSG_E_INVALID, "gamma must be finite and > 0");
    fsg_points* X = const_cast<fsg_points*>(Xc);
    const int64_t n = X->n;
    int D = floor_log2(n);
    if (D > 3) D = 3;
    double* M;
    fsg_status st;
    if ((st = ws(ctx, "deg_bins", (size_t)n << D, &M)) != FSG_OK) return st;
    if ((st = root_bins(ctx, X, gamma, D, M)) != FSG_OK) return st;
    FSG_HIP(ctx, launch_row_sums(M, n, 1 << D, deg_dev, ctx->stream));
    return FSG_OK;
}

fsg_status fsg_kde_segmented(fsg_ctx* ctx, const fsg_points* Q, const fsg_points* X, double gamma, int64_t n_seg,
                             int64_t n_entries, const int64_t* q_ptr, const int32_t* q_idx, const int32_t* lo,
                             const int32_t* mid, const int32_t* hi, const int32_t* self_idx, double* out_left,
                             double* out_right) {
    bool empty = false;
    fsg_status st = kde_segmented_check(ctx, Q, X, gamma, n_seg, n_entries, q_ptr, q_idx, lo, mid, hi, out_left,
                                        out_right, &empty);
    if (st != FSG_OK || empty) return st;
    const KdeSegSizes z = kde_segmented_sizes(X, n_seg, n_entries);
    KdeSegBufs b;
    if ((st = ws(ctx, "seg_bounds", (size_t)z.bounds, &b.bounds)) != FSG_OK) return st;
    if ((st = ws(ctx, "seg_descs", (size_t)n_seg, &b.segs)) != FSG_OK) return st;
    if ((st = ws(ctx, "seg_items", (size_t)z.max_items, &b.items)) != FSG_OK) return st;
    if ((st = ws(ctx, "seg_nitems", 1, &b.n_items)) != FSG_OK) return st;
    if ((st = ws(ctx, "seg_scratch", (size_t)z.counts, &b.counts)) != FSG_OK) return st;
    if ((st = ws(ctx, "seg_pairs", (size_t)z.pairs, &b.pairs)) != FSG_OK) return st;
    return kde_segmented_enqueue(ctx, Q, X, gamma, n_seg, n_entries, q_ptr, q_idx, lo, mid, hi, self_idx, out_left,
                                 out_right, b);
}

fsg_status fsg_sample_edges(fsg_ctx* ctx, const fsg_points* Xc, double gamma, int32_t L, uint64_t seed,
                            int32_t* nbr_dev, double* deg_dev, float* margin_dev) {
    if (!ctx) return FSG_E_INVALID;
    if (!Xc || !nbr_dev) return set_error(ctx, FSG_E_INVALID, "NULL argument");
    if (Xc->ctx != ctx) return set_error(ctx, FSG_E_INVALID, "points belong to another context");
    if (!gamma_ok(gamma)) return set_error(ctx, FSG_E_INVALID, "gamma must be finite and > 0");
    if (L < 1) return set_error(ctx, FSG_E_INVALID, "L must be >= 1");
    if (ctx->kernel == FSG_LAPLACIAN && Xc->prec == FSG_BF16_SPLIT)
        return set_error(ctx, FSG_E_UNSUPPORTED, "the Laplacian kernel runs in the plain path only");
    Sampler S;
    S.X = const_cast<fsg_points*>(Xc);
    S.gamma = gamma;
    S.kind = ctx->kernel;
    S.L = L;
    S.seed = seed;
    S.deg = deg_dev;
    S.nbr = nbr_dev;
    S.margin = margin_dev;
    fsg_status st;
    if ((st = sampler_plan(ctx, S)) != FSG_OK) return st;
    if ((st = ws(ctx, "smp_node", (size_t)S.ns, &S.node)) != FSG_OK) return st;
    FSG_HIP(ctx, launch_init_samples(S.ns, S.node, margin_dev, ctx->stream));
    if (!S.plan.passes.empty()) {
        const int D = S.plan.passes[0].second;
        double* M;
        if ((st = ws(ctx, "pass_masses", (size_t)S.X->n << D, &M)) != FSG_OK) return st;
        // the later passes and the leaf stage read only the columns the root
        // pass kept (exact mode: the dropped pairs total below e^-25 of each
        // degree; with an eps bound, below eps of it)
        const bool reuse = S.X->prec == FSG_BF16_SPLIT;
        if ((st = root_bins(ctx, S.X, gamma, D, M, reuse ? &S.root_mask : nullptr, &S.root_blocks)) != FSG_OK)
            return st;
        if ((st = stage_root_descend(ctx, S, M)) != FSG_OK) return st;
    }
    for (size_t p = 1; p < S.plan.passes.size(); ++p)
        if ((st = stage_pass(ctx, S, p)) != FSG_OK) return st;
    if ((st = stage_leaf(ctx, S)) != FSG_OK) return st;
    if (S.plan.passes.empty() && deg_dev) return fsg_degrees(ctx, S.X, gamma, deg_dev);
    return FSG_OK;
}

fsg_status fsg_build_csr(fsg_ctx* ctx, const fsg_points* X, double gamma, int32_t L, const int32_t* nbr_dev,
                         const double* deg_dev, int64_t* row_ptr_dev, int32_t* col_dev, float* w_dev, int64_t cap,
                         int64_t* nnz) {
    if (!ctx) return FSG_E_INVALID;
    if (!X || !nbr_dev || !deg_dev || !row_ptr_dev || !nnz) return set_error(ctx, FSG_E_INVALID, "NULL argument");
    if (X->ctx != ctx) return set_error(ctx, FSG_E_INVALID, "points belong to another context");
    if (!gamma_ok(gamma)) return set_error(ctx, FSG_E_INVALID, "gamma must be finite and > 0");
    if (L < 1) return set_error(ctx, FSG_E_INVALID, "L must be >= 1");
    if (cap < 0 || (cap > 0 && (!col_dev || !w_dev))) return set_error(ctx, FSG_E_INVALID, "bad cap or outputs");
    const int64_t n = X->n;
    const int64_t m = 2 * n * (int64_t)L;
    if (m > 2147483647LL) return set_error(ctx, FSG_E_UNSUPPORTED, "2*n*L must be < 2^31");
    fsg_status st;
    // row-sorted construction
    {
        int32_t* n_long;
        if ((st = ws(ctx, "csr_nlong", 1, &n_long)) != FSG_OK) return st;
        if ((st = csr_rows_async(ctx, X, gamma, L, nbr_dev, deg_dev, row_ptr_dev, col_dev, w_dev, cap, n_long)) !=
            FSG_OK)
            return st;
        FSG_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, row_ptr_dev + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                                    ctx->stream));
        FSG_HIP(ctx, hipMemcpyAsync(ctx->host_scratch + 1, n_long, sizeof(int32_t), hipMemcpyDeviceToHost,
                                    ctx->stream));
        FSG_HIP(ctx, hipStreamSynchronize(ctx->stream));
        const int32_t longs = (int32_t)(ctx->host_scratch[1] & 0xFFFFFFFF);
        if (longs == 0) {
            *nnz = ctx->host_scratch[0];
            if (*nnz > cap) return set_error(ctx, FSG_E_INVALID, "cap is smaller than 2|E|");
            return FSG_OK;
        }
    }
    // some row has more than 2048 entries: global sort of all entries
    uint64_t* keys;
    int32_t* vals;
    int64_t* flags;
    int64_t* pos;
    int64_t* partials;
    if ((st = ws(ctx, "csr_keys", (size_t)m, &keys)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_vals", (size_t)m, &vals)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_flags", (size_t)m, &flags)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_pos", (size_t)m + 1, &pos)) != FSG_OK) return st;
    if ((st = ws(ctx, "csr_partials", (size_t)scan_partials(m) + 1, &partials)) != FSG_OK) return st;
    SortBufs b = sort_bufs(ctx, m, sizeof(uint64_t), &st);
    if (st != FSG_OK) return st;
    const uint64_t sentinel = (uint64_t)n * (uint64_t)n;
    {
    StageTimer t(ctx, "csr");
    FSG_HIP(ctx, launch_csr_emit(nbr_dev, n, L, keys, vals, ctx->stream));
    FSG_HIP(ctx, radix_sort_u64(keys, vals, m, bit_length(sentinel), b, ctx->stream));
    FSG_HIP(ctx, launch_csr_flags(keys, m, sentinel, flags, ctx->stream));
    FSG_HIP(ctx, launch_exclusive_scan_i64(flags, pos, m, pos + m, partials, ctx->stream));
    CsrArgs a;
    std::memset(&a, 0, sizeof(a));
    a.keys = keys;
    a.pos = pos;
    a.flags = flags;
    a.m = m;
    a.n = n;
    a.d = X->d;
    a.X = X->X;
    a.deg = deg_dev;
    a.s = gamma * 1.442695040888963407359924681001892137;
    a.kind = ctx->kernel;
    a.L = L;
    a.row_ptr = row_ptr_dev;
    a.col = col_dev;
    a.w = w_dev;
    a.cap = cap;
    FSG_HIP(ctx, launch_csr_fill(a, ctx->stream));
    }
    FSG_HIP(ctx, hipMemcpyAsync(ctx->host_scratch, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    FSG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *nnz = ctx->host_scratch[0];
    if (*nnz > cap) return set_error(ctx, FSG_E_INVALID, "cap is smaller than 2|E|");
    return FSG_OK;
}


}  // extern "C"

namespace fsg {

bool job_finished(const fsg_job* j) { return j && j->stage >= j->n_stages; }

// Bytes a build of n points in R^d needs: the point set's arrays, the
// result kept with it (sampled neighbours, degrees, CSR) and a server copy
// of the input (*resident), and the job's buffers while it runs (*transient).
void build_bytes_estimate(const fsg_ctx* ctx, int64_t n, int32_t d, int32_t L, fsg_precision prec,
                          uint64_t* resident, uint64_t* transient) {
    const int D4 = feature_steps(d);
    const uint64_t n_pad = (uint64_t)((n + 15) & ~(int64_t)15);
    const uint64_t ns = (uint64_t)n * (uint64_t)L;
    uint64_t pts = n_pad * 4 * (uint64_t)D4 * 8 + n_pad * 8 + 2 * n_pad * 4;  // rows, norms, level bounds
    if (prec == FSG_BF16_SPLIT) {
        const uint64_t KB = (uint64_t)filter_steps(D4);
        const uint64_t q_rows = ((uint64_t)n + kThetaPad - 1) / kThetaPad * kThetaPad;
        pts += (n_pad / 16 + q_rows / 16) * KB * 64 * 16 + (uint64_t)n * 12 + n_pad * 4 + 256;
    }
    const uint64_t result = ((uint64_t)n + 1) * 8 + 2 * ns * 8 + ns * 4 + (uint64_t)n * 8 + 256;
    *resident = pts + result + (uint64_t)n * (uint64_t)d * 4;
    const Plan plan = make_plan(n, L, ctx->budget, ctx->max_levels_per_pass, prec);
    uint64_t job = ns * 8 + (uint64_t)n * 8;
    // the leaf stage's grouped samples, node starts and work items
    job += ns * 4 + (((uint64_t)1 << plan.leaf_level) + 1) * 4 +
           (2 * (uint64_t)leaf_max_items((int64_t)ns, plan.leaf_level) + 1) * 4;
    if (!plan.passes.empty()) {
        const int D = plan.passes[0].second;
        job += ((uint64_t)n << D) * 8;
        if (prec == FSG_BF16_SPLIT)  // keep masks and thresholds
            job += (uint64_t)((n + kTileQ - 1) / kTileQ) * (n_pad / 16) * 2 +
                   ((uint64_t)n + kThetaPad - 1) / kThetaPad * kThetaPad * 4;
    }
    *transient = job;
}

}  // namespace fsg

extern "C" {

fsg_status fsg_job_create(fsg_ctx* ctx, const fsg_points* Xc, double gamma, int32_t L, uint64_t seed,
                          fsg_job** out) {
    if (ctx && ctx->kernel != FSG_GAUSSIAN)
        return set_error(ctx, FSG_E_UNSUPPORTED, "batch jobs use the Gaussian kernel only");
    if (!ctx || !out) return FSG_E_INVALID;
    *out = nullptr;
    if (!Xc) return set_error(ctx, FSG_E_INVALID, "NULL points");
    if (Xc->ctx != ctx) return set_error(ctx, FSG_E_INVALID, "points belong to another context");
    if (!gamma_ok(gamma)) return set_error(ctx, FSG_E_INVALID, "gamma must be finite and > 0");
    if (L < 1) return set_error(ctx, FSG_E_INVALID, "L must be >= 1");
    fsg_job* j = new (std::nothrow) fsg_job();
    if (!j) return set_error(ctx, FSG_E_NOMEM, "host allocation failed");
    j->ctx = ctx;
    j->S.X = const_cast<fsg_points*>(Xc);
    j->S.gamma = gamma;
    j->S.L = L;
    j->S.seed = seed;
    fsg_status st;
    auto fail = [&](fsg_status s) {
        for (void* p : j->owned) pool_release(ctx, p);
        delete j;
        return s;
    };
    if ((st = sampler_plan(ctx, j->S)) != FSG_OK) return fail(st);
    const int64_t n = Xc->n, ns = j->S.ns;
    j->n_stages = (int)j->S.plan.passes.size() + 1;
    if (!(j->S.node = (int32_t*)job_alloc(j, ns * sizeof(int32_t), &st))) return fail(st);
    if (!(j->S.nbr = (int32_t*)job_alloc(j, ns * sizeof(int32_t), &st))) return fail(st);
    if (!(j->S.deg = (double*)job_alloc(j, n * sizeof(double), &st))) return fail(st);
    if (!j->S.plan.passes.empty()) {
        j->root_D = j->S.plan.passes[0].second;
        if (!(j->M = (double*)job_alloc(j, (size_t)(n << j->root_D) * sizeof(double), &st))) return fail(st);
        if (Xc->prec == FSG_BF16_SPLIT) {
            const size_t tiles = (size_t)((n + kTileQ - 1) / kTileQ);
            if (!(j->mask = (uint16_t*)job_alloc(j, tiles * (size_t)(Xc->n_pad / 16) * sizeof(uint16_t), &st)))
                return fail(st);
            if (!(j->ntheta = (float*)job_alloc(j, (size_t)theta_entries(n) * sizeof(float), &st))) return fail(st);
            const hipError_t e = launch_mask_theta(root_mask_args(Xc, j->S.gamma, ctx->num_cus), j->ntheta, theta_entries(n), ctx->stream);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(set_error(ctx, FSG_E_DEVICE, std::string("keep-thresholds: ") + hipGetErrorString(e)));
            }
        }
    }
    ctx->jobs.insert(j);
    *out = j;
    return FSG_OK;
}

fsg_status fsg_batch_step(fsg_ctx* ctx, fsg_job* const* jobs, int32_t n_jobs, int32_t* n_done) {
    if (!ctx || !n_done) return FSG_E_INVALID;
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return set_error(ctx, FSG_E_INVALID, "bad job list");
    for (int32_t i = 0; i < n_jobs; ++i) {
        if (!jobs[i] || jobs[i]->ctx != ctx) return set_error(ctx, FSG_E_INVALID, "job is NULL or of another context");
        for (int32_t k = 0; k < i; ++k)
            if (jobs[k] == jobs[i]) return set_error(ctx, FSG_E_INVALID, "a job appears twice");
    }
    fsg_status st;
    // root passes: grouped by feature-step class and precision, in list order
    std::map<std::pair<int, int>, std::vector<fsg_job*>> groups;
    for (int32_t i = 0; i < n_jobs; ++i) {
        fsg_job* j = jobs[i];
        if (j->stage != 0) continue;
        FSG_HIP(ctx, launch_init_samples(j->S.ns, j->S.node, nullptr, ctx->stream));
        if (!j->S.plan.passes.empty()) groups[{j->S.X->D4, (int)j->S.X->prec}].push_back(j);
    }
    for (auto& kv : groups)
        if ((st = batch_root(ctx, kv.second)) != FSG_OK) return st;
    // root descents of every job in its root stage: one launch
    {
        std::vector<fsg_job*> desc;
        for (int32_t i = 0; i < n_jobs; ++i)
            if (jobs[i]->stage == 0 && !jobs[i]->S.plan.passes.empty()) desc.push_back(jobs[i]);
        if (!desc.empty() && (st = batch_root_descend(ctx, desc)) != FSG_OK) return st;
    }
    // leaf stages: grouped by class of d, one launch per group
    std::map<int, std::vector<fsg_job*>> leaf_groups;
    for (int32_t i = 0; i < n_jobs; ++i) {
        fsg_job* j = jobs[i];
        if (j->stage >= j->n_stages) continue;
        const int P = (int)j->S.plan.passes.size();
        if (j->stage == 0 && P > 0) {
            // (descended above)
        } else if (j->stage < P) {
            if ((st = stage_pass(ctx, j->S, (size_t)j->stage)) != FSG_OK) return st;
        } else {
            leaf_groups[leaf_class(j->S.X->d)].push_back(j);
            continue;
        }
        ++j->stage;
    }
    for (auto& kv : leaf_groups) {
        if ((st = batch_leaf(ctx, kv.second)) != FSG_OK) return st;
        for (fsg_job* j : kv.second) {
            if (j->S.plan.passes.empty() && (st = fsg_degrees(ctx, j->S.X, j->S.gamma, j->S.deg)) != FSG_OK)
                return st;
            ++j->stage;
        }
    }
    int32_t done = 0;
    for (int32_t i = 0; i < n_jobs; ++i) done += (jobs[i]->stage >= jobs[i]->n_stages) ? 1 : 0;
    *n_done = done;
    return FSG_OK;
}

fsg_status fsg_job_reset(fsg_job* j) {
    if (!j || !j->ctx) return FSG_E_INVALID;
    j->stage = 0;
    return FSG_OK;
}

fsg_status fsg_job_result(fsg_job* j, int32_t* nbr_dev, double* deg_dev) {
    if (!j || !j->ctx) return FSG_E_INVALID;
    fsg_ctx* ctx = j->ctx;
    if (j->stage < j->n_stages) return set_error(ctx, FSG_E_INVALID, "the job has not finished");
    if (nbr_dev)
        FSG_HIP(ctx, hipMemcpyAsync(nbr_dev, j->S.nbr, j->S.ns * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
    if (deg_dev)
        FSG_HIP(ctx, hipMemcpyAsync(deg_dev, j->S.deg, j->S.X->n * sizeof(double), hipMemcpyDeviceToDevice,
                                    ctx->stream));
    return FSG_OK;
}

fsg_status fsg_job_outputs(fsg_job* j, const int32_t** nbr_dev, const double** deg_dev) {
    if (!j || !j->ctx) return FSG_E_INVALID;
    if (nbr_dev) *nbr_dev = j->S.nbr;
    if (deg_dev) *deg_dev = j->S.deg;
    return FSG_OK;
}

void fsg_job_destroy(fsg_job* j) {
    if (!j) return;
    if (j->ctx) {
        batch_cache_drop(j->ctx, j);
        for (void* p : j->owned) pool_release(j->ctx, p);
        j->ctx->jobs.erase(j);
    }
    delete j;
}

fsg_status fsg_ctx_set_autotune(fsg_ctx* ctx, int32_t enabled) {
    if (!ctx) return FSG_E_INVALID;
    ctx->autotune = enabled != 0;
    return FSG_OK;
}

fsg_status fsg_ctx_tuned_shape(fsg_ctx* ctx, int32_t D4, fsg_precision prec, int32_t* waves_per_cu,
                               int32_t* cols_per_item) {
    if (!ctx || !waves_per_cu || !cols_per_item) return FSG_E_INVALID;
    auto it = ctx->tuned.find({(int)D4, (int)prec});
    if (it == ctx->tuned.end()) return set_error(ctx, FSG_E_INVALID, "no tuned shape for this class");
    *waves_per_cu = it->second.first;
    *cols_per_item = it->second.second;
    return FSG_OK;
}

fsg_status fsg_ctx_save_tuning(fsg_ctx* ctx, const char* path) {
    if (!ctx) return FSG_E_INVALID;
    if (!path) return set_error(ctx, FSG_E_INVALID, "NULL path");
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(ctx, FSG_E_INVALID, std::string("cannot write ") + path);
    std::fprintf(f, "fsg-tuning 1 %s %d\n", ctx->arch.c_str(), ctx->num_cus);
    for (const auto& kv : ctx->tuned)
        std::fprintf(f, "%d %d %d %d\n", kv.first.first, kv.first.second, kv.second.first, kv.second.second);
    const bool ok = std::fclose(f) == 0;
    return ok ? FSG_OK : set_error(ctx, FSG_E_INVALID, std::string("cannot write ") + path);
}

fsg_status fsg_ctx_load_tuning(fsg_ctx* ctx, const char* path, int32_t* n_loaded) {
    if (!ctx) return FSG_E_INVALID;
    if (n_loaded) *n_loaded = 0;
    if (!path) return set_error(ctx, FSG_E_INVALID, "NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) return set_error(ctx, FSG_E_INVALID, std::string("cannot read ") + path);
    char tag[32] = {0}, arch[128] = {0};
    int version = 0, cus = 0;
    if (std::fscanf(f, "%31s %d %127s %d", tag, &version, arch, &cus) != 4 || std::strcmp(tag, "fsg-tuning") != 0 ||
        version != 1) {
        std::fclose(f);
        return set_error(ctx, FSG_E_INVALID, std::string("not a tuning file: ") + path);
    }
    int32_t loaded = 0;
    if (ctx->arch == arch && ctx->num_cus == cus) {
        int D4, prec, waves, cols;
        while (std::fscanf(f, "%d %d %d %d", &D4, &prec, &waves, &cols) == 4) {
            const bool sane = (D4 == 1 || D4 == 2 || D4 == 4 || D4 == 8 || D4 == 16 || D4 == 32) &&
                              (prec == FSG_PLAIN_FP64 || prec == FSG_BF16_SPLIT) && waves >= 1 && waves <= 64 &&
                              cols >= 0 && cols <= (1 << 24);
            if (!sane) {
                std::fclose(f);
                return set_error(ctx, FSG_E_INVALID, std::string("bad entry in tuning file ") + path);
            }
            ctx->tuned[{D4, prec}] = {waves, cols};
            ++loaded;
        }
    }
    std::fclose(f);
    if (n_loaded) *n_loaded = loaded;
    return FSG_OK;
}

fsg_status fsg_graph_begin(fsg_ctx* ctx) {
    if (!ctx) return FSG_E_INVALID;
    if (ctx->stream == nullptr) return set_error(ctx, FSG_E_UNSUPPORTED, "recording needs a non-default stream");
    FSG_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
    return FSG_OK;
}

fsg_status fsg_graph_end(fsg_ctx* ctx, fsg_graph** out) {
    if (!ctx || !out) return FSG_E_INVALID;
    *out = nullptr;
    fsg_graph* g = new (std::nothrow) fsg_graph();
    if (!g) return set_error(ctx, FSG_E_NOMEM, "host allocation failed");
    hipError_t e = hipStreamEndCapture(ctx->stream, &g->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return set_error(ctx, FSG_E_DEVICE, std::string("graph: ") + hipGetErrorString(e));
    }
    g->ctx = ctx;
    ctx->graphs.insert(g);
    *out = g;
    return FSG_OK;
}

fsg_status fsg_graph_launch(fsg_ctx* ctx, fsg_graph* g) {
    if (!ctx || !g) return FSG_E_INVALID;
    if (g->ctx != ctx) return set_error(ctx, FSG_E_INVALID, "the graph was not recorded on this context");
    FSG_HIP(ctx, hipGraphLaunch(g->exec, ctx->stream));
    return FSG_OK;
}

void fsg_graph_destroy(fsg_graph* g) {
    if (!g) return;
    fsg_ctx* ctx = g->ctx;
    if (ctx) (void)hipStreamSynchronize(ctx->stream);  // a replay may still run
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (ctx) {
        ctx->graphs.erase(g);
        if (ctx->graphs.empty()) free_retired(ctx);
    }
    delete g;
}

}  // extern "C"
