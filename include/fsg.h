/*
 * fsg.h -- C ABI of libfsg.so: the data-parallel hot path of
 * FastSimilarityGraph (Macgregor & Sun, "A Fast Similarity Graph Construction
 * via Kernel Density Estimation", NeurIPS 2023) on AMD Instinct MI355X (gfx950).
 *
 * The library builds a sparse approximation of the fully connected Gaussian
 * similarity graph of n points (Section 2.1) without forming the n x n kernel
 * matrix: every point draws L neighbours j with probability k(x_i,x_j)/deg(x_i)
 * by a randomised descent of an index-order binary partition tree whose branch
 * probabilities are kernel density estimates over the tree nodes (Algorithm 1,
 * Section 4.1, Lemma 1), and the sampled edges are reweighted into a
 * symmetric CSR graph (Algorithm 2).  The KDE is exact (brute force): the
 * cross term x.y runs on the FP64 matrix cores, the squared distance is formed
 * by the norm expansion in FP64, and exp is evaluated in FP64.
 *
 * Conventions shared by every call:
 *  - Points are FP32, row-major n x d, in device memory owned by the caller.
 *  - Kernel k(x,y) = exp(-gamma ||x-y||^2); gamma > 0 (gamma = 1/sigma^2 in the
 *    paper's notation, 1/(2 sigma^2) in the usual statistics convention).
 *  - No self loops: the term j == i is left out of every degree and node mass.
 *  - Tree: node [a,b) splits at mid = a + floor((b-a)/2) (Section 4.1: the first
 *    half holds floor(|X|/2) points); the root is [0,n) at level 0.
 *  - Uniforms: Philox4x64-10 (Salmon et al., SC 2011) with key (seed, 0) and
 *    counter (i, l, floor(level/4), 0); the uniform of sample l of point i at
 *    level `level` is (word[level mod 4] >> 11) * 2^-53.  A sample at node
 *    [a,b) with masses mL, mR of its halves goes left iff u*(mL+mR) < mL
 *    (Algorithm 1's test r <= g_X1/(g_X1+g_X2)), and never enters a child of
 *    zero mass.
 *  - Ownership: every *_dev pointer is device memory owned by the caller; a
 *    points handle borrows X_dev (which must outlive it) and owns the arrays
 *    derived from it; a context owns its workspace.
 *  - Ordering: every call is enqueued on the context's stream, in call order.
 *    Outputs are valid once that stream is synchronised.  Only fsg_build_csr
 *    (which returns nnz to the host) synchronises the stream itself.
 *  - Errors: calls return a status and never throw.  Argument checks are done
 *    on the host before anything is enqueued (FSG_E_INVALID); HIP failures are
 *    returned as FSG_E_DEVICE (asynchronous faults surface at a later call or at
 *    fsg_ctx_sync).  On any error the outputs are unspecified.  fsg_last_error
 *    gives a message for the last failing call on a context.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef FSG_H
#define FSG_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSG_OK = 0,
    FSG_E_INVALID = -1,     /* bad argument (checked on the host) */
    FSG_E_NOMEM = -2,       /* device allocation failed */
    FSG_E_DEVICE = -3,      /* a HIP call failed */
    FSG_E_UNSUPPORTED = -4, /* valid request outside what this build supports */
    FSG_E_BUDGET = -5       /* the request needs more workspace than the budget allows */
} fsg_status;

typedef enum {
    /* plain path: FP32 points, every pair's cross term on the FP64 matrix
     * cores, FP64 distance, exp and masses (no pair is skipped).  It is not an
     * FP32 path: FP32 distances from the norm expansion would move kernel
     * values, and so node masses, by up to ~1e-5 relative at n = 1e5, d = 32
     * and ~3e-5 at n = 1e6, d = 64 -- more than the 1e-6 decision band of the
     * descent, and at the larger size more than a 1e-5 degree tolerance. */
    FSG_PLAIN_FP64 = 0,
    /* precision mode: BF16 hi/lo split operands (hi = bf16(x), lo = bf16(x-hi))
     * on the BF16 matrix cores with FP32 accumulation give every pair an
     * approximate exponent with a guaranteed error bound; only pairs that can
     * carry more than e^-Delta of their row's largest term (Delta = ln n + 25)
     * are recomputed in FP64 as in FSG_PLAIN_FP64, the others add 0.  Every degree
     * and node mass then differs from the exact one by less than
     * (n-1) e^-Delta < e^-25 = 1.4e-11 of the degree.
     * Applies to the pass over all points (fsg_degrees, the first pass of
     * fsg_sample_edges); d <= 128. */
    FSG_BF16_SPLIT = 1
} fsg_precision;

/* The kernels of Section 2.1 (its last sentence names the Laplacian and the
 * exponential kernel beside the Gaussian one), all with scale gamma > 0. */
typedef enum {
    FSG_GAUSSIAN = 0,    /* k = exp(-gamma ||x - y||_2^2) */
    FSG_EXPONENTIAL = 1, /* k = exp(-gamma ||x - y||_2)   */
    FSG_LAPLACIAN = 2    /* k = exp(-gamma ||x - y||_1)   */
} fsg_kernel;

typedef struct fsg_ctx fsg_ctx;
typedef struct fsg_points fsg_points;

/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  ws_budget_bytes caps the workspace the context may
 * allocate (0 = a default of 32 GiB). */
fsg_status fsg_ctx_create(int device, void* hip_stream, uint64_t ws_budget_bytes, fsg_ctx** out);
void fsg_ctx_destroy(fsg_ctx* ctx);
/* Static string naming a status code. */
const char* fsg_status_string(fsg_status s);
/* Message for the last failing call on ctx ("" if none); valid until the next call. */
const char* fsg_last_error(const fsg_ctx* ctx);
/* Synchronise the context's stream and report any device error. */
fsg_status fsg_ctx_sync(fsg_ctx* ctx);
/* Device workspace currently held by the context, in bytes. */
uint64_t fsg_ctx_workspace_bytes(const fsg_ctx* ctx);

/* Stage timing.  When enabled, the context records a pair of HIP events on
 * its stream around every stage it launches; fsg_ctx_stage_time synchronises
 * the stream and returns the summed elapsed time (ms) and the number of
 * launches of one stage since the last reset.  Stages: "prep", "prune" (the
 * precision mode's tile pruning plan), "kde_mask" (its BF16 keep-mask scan),
 * "mask_convert" (keep bits back to index order), "kde_root"
 * (the binned KDE over all points), "pass_mask" (the keep masks of a later
 * pass in the precision mode, narrowed from the root pass's), "kde_pass"
 * (binned KDE of later passes), "descend" (descent over bins), "group"
 * (sample sort by node), "leaf" (leaf stage), "csr" (reweighting and CSR).
 * Unknown names report 0. */
fsg_status fsg_ctx_set_profiling(fsg_ctx* ctx, int enabled);
fsg_status fsg_ctx_stage_time(fsg_ctx* ctx, const char* stage, double* ms, int64_t* launches);
fsg_status fsg_ctx_reset_profiling(fsg_ctx* ctx);
/* Precision-mode statistics since the last reset: *kept = (data column,
 * 64-query tile) pairs that the BF16 filter keeps for exact recomputation,
 * *scanned = (data column, 64-query tile) pairs it examined.  Synchronises the
 * stream. */
fsg_status fsg_ctx_filter_stats(fsg_ctx* ctx, int64_t* kept, int64_t* scanned);

/* Kernel of every later call on the context (default FSG_GAUSSIAN): degrees,
 * segmented KDE, sampling and the CSR weights all use it, with the same
 * gamma argument.  The exponential kernel runs like the Gaussian one (cross
 * terms on the FP64 matrix cores, the distance from the norm expansion, then
 * its square root), in both precisions: the precision mode's keep test then
 * accepts squared distances up to (sqrt(dmin) + Delta/gamma)^2.  The
 * Laplacian kernel has no inner-product form: its L1 distances are summed on
 * the FP64 vector units, in the plain path only (FSG_E_UNSUPPORTED for
 * FSG_BF16_SPLIT point sets).  Batch jobs and servers use the Gaussian kernel
 * only (FSG_E_UNSUPPORTED otherwise).  Near-duplicate pairs of the
 * exponential kernel carry the norm expansion's absolute error into the
 * square root: |x - y|_2 is then known to about 1e-7 (relative error of k
 * about gamma 1e-7), a bound the other distances do not need.
 * FSG_E_INVALID for an unknown kind. */
fsg_status fsg_ctx_set_kernel(fsg_ctx* ctx, fsg_kernel kind);

/* Error budget of the precision mode's KDE over all points (the root pass of
 * fsg_sample_edges and fsg_degrees; batch jobs and servers always use 0).
 * eps = 0 (default): pairs more than Delta = ln n + 25 below their row's
 * largest exponent term are dropped, so that every degree loses less than
 * e^-25 of itself and a sampled neighbour differs from the exact method's
 * with probability below ceil(log2 n) e^-25.  0 < eps < 1: the paper's
 * approximate-KDE regime (Theorem 1 asks for (1 +- eps)-accurate KDEs with
 * eps <= 1/(6 log2 n)): Delta = ln(n-1) + ln(1/eps), so every degree is
 * within [1 - eps, 1] of the exact one and fewer pairs are recomputed.  In
 * both cases every level of fsg_sample_edges evaluates only pairs the root
 * pass kept (a superset of each point's own), so each level's branch
 * probabilities differ from the exact ones by at most the dropped mass over
 * the degree: the sampled neighbour's distribution is within total variation
 * ceil(log2 n) e^-25 (eps = 0) or ceil(log2 n) eps (at most 1/6 for the
 * paper's eps) of the exact k/deg.  FSG_E_INVALID outside [0, 1). */
fsg_status fsg_ctx_set_kde_error(fsg_ctx* ctx, double eps);

/* Tile pruning of the precision mode: before the BF16 keep-mask
 * scan of a pass over all points, each 64-query tile is checked against the
 * cells of the 256 pivots (points grouped by nearest pivot, each with an upper
 * bound on its radius); by the triangle inequality a (tile, cell) pair whose
 * every query is farther than radius + sqrt(T_q) from the cell's pivot --
 * T_q the largest squared distance the keep test can accept for query q --
 * cannot keep a column and is not scanned.  The kept set, and so every
 * result, is the same with and without it; on well-separated clusters the
 * scan shrinks to the tiles' own clusters (Section 1 and Theorem 1 rely on a
 * KDE that is fast on such data).  enabled > 0: on; 0: off, every pair is
 * scanned; < 0 (default): on for point sets of at least 2^18 points, where
 * the scan it saves outweighs the plan and the conversion of the keep bits
 * back to index order. */
fsg_status fsg_ctx_set_pruning(fsg_ctx* ctx, int32_t enabled);

/* Integer slices in the precision mode's exact recompute (32 < d <= 64,
 * Gaussian kernel, root pass): each point's coordinates, scaled by a power
 * of two per point, are cut into seven signed base-256 digits, the cross term
 * of a kept pair is the sum of the 28 most significant digit-slice products
 * (exact in int32 on the int8 matrix cores) joined in FP64, with error at
 * most 4.1 d 2^-53 |q| |x| -- the order of a d-term FP64 accumulation -- and
 * the exponent and bin sums follow in FP64 as before.  enabled != 0 (default
 * < 0): used where it applies; 0: the cross terms are recomputed on the FP64
 * matrix cores.  The kept set does not depend on it; masses differ within
 * the two recomputes' error bounds. */
fsg_status fsg_ctx_set_exact_slices(fsg_ctx* ctx, int32_t enabled);

/* Cap the number of tree levels one binned KDE pass resolves (0 restores the
 * automatic choice, which is bounded by the workspace budget).  Results do not
 * depend on it; smaller caps trade more passes for less workspace. */
fsg_status fsg_ctx_set_levels_per_pass(fsg_ctx* ctx, int32_t max_levels);

/* Make a point set resident: X_dev is FP32 row-major n x d (borrowed).  Derives
 * the FP64 matrix-core operand layout and the squared norms (hot-path step
 * "prep"); with FSG_BF16_SPLIT also the split BF16 operands, an upper bound on
 * each point's smallest squared distance (from 256 pivot points) and an order
 * of the points by nearest pivot (used to form coherent query tiles).
 * 1 <= n <= 2^31-1, 1 <= d <= 128 (both precisions). */
fsg_status fsg_points_create(fsg_ctx* ctx, const float* X_dev, int64_t n, int32_t d, fsg_precision prec,
                             fsg_points** out);
void fsg_points_destroy(fsg_points* pts);
/* Device bytes owned by the handle (for HBM admission). */
uint64_t fsg_points_bytes(const fsg_points* pts);

/* Degrees: deg_dev[i] = sum_{j != i} exp(-gamma ||x_i - x_j||^2), FP64 [n].
 * This is the KDE g_[1,n](x_i) of Algorithm 2 (eq. (1) of Section 2.2) without
 * the self term. */
fsg_status fsg_degrees(fsg_ctx* ctx, const fsg_points* X, double gamma, double* deg_dev);

/* Segmented KDE (eq. (1) of Section 2.2 over index ranges; the two KDEs of
 * Algorithm 1).  Segment s pairs the query entries e in [q_ptr[s], q_ptr[s+1])
 * -- query point Q[q_idx[e]] -- with the data range X[lo[s]:hi[s]) split at
 * mid[s]:
 *   out_left[e]  = sum_{j in [lo[s], mid[s]), j != self_idx[e]} k(Q[q_idx[e]], X[j])
 *   out_right[e] = sum_{j in [mid[s], hi[s]), j != self_idx[e]} k(Q[q_idx[e]], X[j])
 * All arrays are device memory: q_ptr int64 [n_seg+1] non-decreasing from 0;
 * q_idx, self_idx int32 [q_ptr[n_seg]] (self_idx may be NULL: nothing
 * excluded; a negative entry excludes nothing); lo, mid, hi int32 [n_seg] with
 * 0 <= lo <= mid <= hi <= n(X); outputs FP64 [q_ptr[n_seg]].  Q and X must
 * have the same d.  n_entries = q_ptr[n_seg] must be passed by the caller (the
 * library does not read device memory on the host); segments may be empty,
 * overlap, and have any size.  Out-of-range device indices are the caller's
 * responsibility (they are not checked on the host). */
fsg_status fsg_kde_segmented(fsg_ctx* ctx, const fsg_points* Q, const fsg_points* X, double gamma,
                             int64_t n_seg, int64_t n_entries, const int64_t* q_ptr, const int32_t* q_idx,
                             const int32_t* lo, const int32_t* mid, const int32_t* hi,
                             const int32_t* self_idx, double* out_left, double* out_right);

/* Size of the static device scratch of fsg_kde_segmented_noalloc (per GPU). */
#define FSG_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation, arguments, results and errors as fsg_kde_segmented, but it
 * calls no allocating routine.  Its work lists and pair sums live in a static
 * device array of FSG_NOALLOC_SCRATCH_BYTES (64 MiB) on each GPU, held until
 * the process ends, instead of the context's workspace.  A call needs about
 * 16 bytes per query entry plus 70 per segment (each of six regions rounded
 * up to 256 bytes); larger calls return FSG_E_UNSUPPORTED with the byte count
 * in fsg_last_error, and enqueue nothing.  Every call on one GPU shares that
 * GPU's array and leaves its contents behind (nothing in it needs to start at
 * zero): calls that overlap on one GPU -- on two streams or two contexts of
 * the same device -- race, and the caller must order them.  FSG_E_DEVICE if
 * the array's address could not be looked up when the context was created.
 * Point sets Q and X must already exist (fsg_points_create allocates). */
fsg_status fsg_kde_segmented_noalloc(fsg_ctx* ctx, const fsg_points* Q, const fsg_points* X, double gamma,
                                     int64_t n_seg, int64_t n_entries, const int64_t* q_ptr, const int32_t* q_idx,
                                     const int32_t* lo, const int32_t* mid, const int32_t* hi,
                                     const int32_t* self_idx, double* out_left, double* out_right);

/* Algorithm 1 run L times from the root for every point (Algorithm 2's
 * sampling loop).  nbr_dev int32 [n*L]: nbr[i*L+l] = the neighbour sampled by
 * sample l of point i, or -1 when deg_i == 0.  deg_dev FP64 [n] (may be NULL)
 * receives the degrees.  margin_dev FP32 [n*L] (may be NULL) receives, per
 * sample, min over its levels of |u - mL/(mL+mR)| as computed on the device. */
fsg_status fsg_sample_edges(fsg_ctx* ctx, const fsg_points* X, double gamma, int32_t L, uint64_t seed,
                            int32_t* nbr_dev, double* deg_dev, float* margin_dev);

/* Algorithm 2 after the sampling loop: the set E of undirected edges
 * {i, nbr[i*L+l]} (entries -1 skipped), each weighted w = k/p_hat with
 *   p_i = min(L k/deg_i, 1), p_j = min(L k/deg_j, 1), p_hat = p_i + p_j - p_i p_j,
 * written as a symmetric CSR: each edge appears in both of its rows, columns
 * ascending.  nbr_dev int32 [n*L] (entries in [-1, n), never i itself),
 * deg_dev FP64 [n] (from fsg_degrees or fsg_sample_edges), row_ptr_dev int64
 * [n+1], col_dev int32 [cap], w_dev FP32 [cap].  *nnz (host) receives 2|E|;
 * FSG_E_INVALID if cap < 2|E| would be needed (cap >= 2 n L always suffices).
 * Synchronises the stream. */
fsg_status fsg_build_csr(fsg_ctx* ctx, const fsg_points* X, double gamma, int32_t L, const int32_t* nbr_dev,
                         const double* deg_dev, int64_t* row_ptr_dev, int32_t* col_dev, float* w_dev,
                         int64_t cap, int64_t* nnz);

/* ------------------------------------------------------------------------
 * Batching: many independent graph builds (Algorithm 2's sampling loop, as in
 * fsg_sample_edges, per point set) advanced together.  A job runs its stages
 * in order: the root pass (binned KDE over all its points, then the descent),
 * later binned passes, the leaf stage.  fsg_batch_step advances every
 * unfinished job in `jobs` by one stage; the root passes of all jobs that
 * share a feature-step class and precision run as ONE launch of the KDE
 * kernels (every (point set, query tile, bin run) work item of those jobs in
 * one persistent grid).  Results equal fsg_sample_edges on the same inputs,
 * bit for bit.
 * ------------------------------------------------------------------------ */
typedef struct fsg_job fsg_job;

/* A build of X with kernel scale gamma, L samples per point and Philox seed
 * `seed`.  X must outlive the job.  The job owns device buffers for its
 * samples, degrees and root-pass masses (from the context's pool; about
 * n*2^D*8 bytes with 2^D ~ n/48 for the root bins).  FSG_E_INVALID on bad
 * arguments, FSG_E_NOMEM if the buffers cannot be allocated. */
fsg_status fsg_job_create(fsg_ctx* ctx, const fsg_points* X, double gamma, int32_t L, uint64_t seed, fsg_job** out);

/* Advance every unfinished job by one stage (jobs must belong to ctx; a job
 * may appear once).  *n_done (host) receives the number of jobs in `jobs`
 * that have finished.  Enqueues work only: no synchronisation, so a sequence
 * of calls can be captured with fsg_graph_begin/fsg_graph_end. */
fsg_status fsg_batch_step(fsg_ctx* ctx, fsg_job* const* jobs, int32_t n_jobs, int32_t* n_done);

/* Rewind a job to its first stage (its buffers are kept). */
fsg_status fsg_job_reset(fsg_job* job);

/* Enqueue copies of a finished job's result: nbr_dev int32 [n*L] as in
 * fsg_sample_edges, deg_dev FP64 [n] (either may be NULL).  FSG_E_INVALID if
 * the job has not finished. */
fsg_status fsg_job_result(fsg_job* job, int32_t* nbr_dev, double* deg_dev);

/* Device pointers of a job's own result arrays (valid until destroy). */
fsg_status fsg_job_outputs(fsg_job* job, const int32_t** nbr_dev, const double** deg_dev);

/* Release a job (its buffers return to the context's pool). */
void fsg_job_destroy(fsg_job* job);

/* Launch shapes of batched root passes are autotuned when enabled (default
 * on): the first batch of a new shape class times a few candidates with HIP
 * events and keeps the fastest for the context — in the plain path the grid
 * size and the data columns per work item, in the precision mode the data
 * columns per keep-mask work item.  Results do not depend on the shape (the
 * precision mode's exact pass keeps the single-set item shape, which decides
 * its rounding order).  Tuning is skipped while the stream is being captured. */
fsg_status fsg_ctx_set_autotune(fsg_ctx* ctx, int32_t enabled);

/* The shape tuned for a class (feature steps D4 in {1,2,4,8,16,32},
 * precision): waves per compute unit and data columns per work item (per
 * keep-mask work item in the precision mode, where 0 means each set's own
 * chunk, the one its single-set pass uses).  FSG_E_INVALID if that class has
 * not been tuned. */
fsg_status fsg_ctx_tuned_shape(fsg_ctx* ctx, int32_t D4, fsg_precision prec, int32_t* waves_per_cu,
                               int32_t* cols_per_item);

/* The tuned shapes outlive the context in a small text file: save writes
 * every tuned class with the device's architecture name and compute-unit
 * count; load reads a file written on the same kind of device (other files
 * load nothing) and *n_loaded (may be NULL) receives the classes taken over,
 * which are then not tuned again.  FSG_E_INVALID if the file cannot be
 * written, or read or parsed. */
fsg_status fsg_ctx_save_tuning(fsg_ctx* ctx, const char* path);
fsg_status fsg_ctx_load_tuning(fsg_ctx* ctx, const char* path, int32_t* n_loaded);

/* ------------------------------------------------------------------------
 * HIP graphs of the context's stream: everything enqueued between
 * fsg_graph_begin and fsg_graph_end (which must not synchronise; e.g.
 * fsg_batch_step, fsg_sample_edges) is recorded into a graph that
 * fsg_graph_launch replays on the stream.  The recorded calls must have run
 * once before (so that no workspace grows while recording).  While a graph
 * exists, device blocks it may name stay allocated: a later call that grows a
 * workspace buffer parks the old one instead of freeing it, and parked blocks
 * are freed when the context's last graph is destroyed.  The point sets and
 * jobs a graph uses must outlive its launches; a graph is launched only on the
 * context it was recorded on (FSG_E_INVALID otherwise); if the context is
 * destroyed first, the graph is valid for fsg_graph_destroy only.
 * ------------------------------------------------------------------------ */
typedef struct fsg_graph fsg_graph;
fsg_status fsg_graph_begin(fsg_ctx* ctx);
fsg_status fsg_graph_end(fsg_ctx* ctx, fsg_graph** out);
fsg_status fsg_graph_launch(fsg_ctx* ctx, fsg_graph* g);
void fsg_graph_destroy(fsg_graph* g);

/* ------------------------------------------------------------------------
 * Serving: a request loop over one context.  Graph-build requests (Algorithm
 * 2 for a new point set) and KDE requests (eq. (1) for query points against a
 * resident set) are queued, admitted in arrival order while the HBM budget
 * and the active-build limit allow (ready sets that no queued or running
 * request needs are evicted, least recently used first), and advanced by
 * fsg_server_poll: every admitted build moves one stage per poll, and the
 * root passes of builds admitted together run in one launch (continuous
 * batching).  A finished build's point set, sampled neighbours, degrees and
 * symmetric CSR stay resident until evicted.  Results equal the single-call
 * path (fsg_sample_edges + fsg_build_csr, fsg_kde_segmented) bit for bit,
 * whatever else is in flight.  Not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct fsg_server fsg_server;

/* hbm_budget_bytes bounds the server's resident sets plus admitted builds
 * (the context's workspace is counted separately); max_active bounds the
 * builds in flight (>= 1). */
fsg_status fsg_server_create(fsg_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_active, fsg_server** out);
void fsg_server_destroy(fsg_server* srv);

/* Build request for a new set `set_id` (caller's unique id >= 0): X_dev is
 * FP32 n x d on the device and must stay valid until the request completes
 * (the server copies it at admission).  *req_id receives the request id.
 * FSG_E_INVALID for a reused set_id or bad arguments; FSG_E_BUDGET if the set
 * alone could never fit the budget. */
fsg_status fsg_server_submit_build(fsg_server* srv, int64_t set_id, const float* X_dev, int64_t n, int32_t d,
                                   double gamma, int32_t L, uint64_t seed, fsg_precision prec, int64_t* req_id);

/* KDE request: out_dev[i] = sum_j exp(-gamma |q_i - x_j|^2) over all points
 * x_j of set `set_id`, for the m query rows of Q_dev (FP32 m x d, valid until
 * completion; out_dev FP64 [m]).  Waits while the set is still being built;
 * completes with FSG_E_INVALID if the set is unknown or has been evicted. */
fsg_status fsg_server_submit_kde(fsg_server* srv, int64_t set_id, const float* Q_dev, int64_t m, double gamma,
                                 double* out_dev, int64_t* req_id);

/* One turn of the loop: collect requests whose device work has finished;
 * then, if the work the previous turn enqueued has finished, admit queued
 * requests, advance every active build by one stage and launch admitted KDE
 * requests (iteration-level scheduling: requests arriving while the device
 * is busy are admitted together, and their root passes share launches).  Up
 * to `cap` finished request ids and their statuses are written to done_ids /
 * done_status (*n_done of them); the rest are reported by later polls.  Does
 * not wait for the device. */
fsg_status fsg_server_poll(fsg_server* srv, int64_t* done_ids, int32_t* done_status, int32_t cap, int32_t* n_done);

/* Device arrays of a resident, finished set (owned by the server, valid until
 * the set is evicted or the server destroyed): row_ptr int64 [n+1], col int32
 * [nnz], w FP32 [nnz], nbr int32 [n*L], deg FP64 [n].  Any output may be NULL. */
fsg_status fsg_server_graph(fsg_server* srv, int64_t set_id, const int64_t** row_ptr, const int32_t** col,
                            const float** w, int64_t* nnz, const int32_t** nbr, const double** deg);

/* Counters: bytes held by resident sets and admitted builds, builds in flight,
 * queued requests, evicted sets so far. */
fsg_status fsg_server_stats(fsg_server* srv, uint64_t* resident_bytes, int32_t* active, int32_t* queued,
                            int64_t* evictions);

#ifdef __cplusplus
}
#endif
#endif
