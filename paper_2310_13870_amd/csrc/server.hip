// Request loop (serving) over one context: graph builds (Algorithm 2 for a new
// point set) and KDE queries (eq. (1) against a resident set) admitted against
// an HBM budget, with continuous batching of the builds' sampling stages.
//
// Every request's device work is enqueued on the context's stream; a request
// is complete when the event recorded after its last operation has passed.
// Builds run as batch jobs: each poll advances every admitted build by one
// stage, and the root passes of builds admitted in the same poll share the
// KDE launches.  Results equal the single-call path bit for bit.
#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "common.h"

namespace fsg {
namespace {

enum class Kind { kBuild, kKde };

struct SetRec {
    int64_t id = -1;
    int64_t n = 0;
    int32_t d = 0;
    double gamma = 0.0;
    int32_t L = 0;
    uint64_t seed = 0;
    fsg_precision prec = FSG_PLAIN_FP64;
    float* X = nullptr;        // the server's copy of the points
    fsg_points* pts = nullptr;
    fsg_job* job = nullptr;    // while the build runs
    int64_t* row_ptr = nullptr;
    int32_t* col = nullptr;
    float* w = nullptr;
    int32_t* nbr = nullptr;
    double* deg = nullptr;
    int32_t* n_long = nullptr;  // rows over the row-sort limit (device counter)
    int32_t slot = -1;         // pinned host slot receiving {nnz, n_long} at completion
    int64_t nnz = -1;
    bool ready = false;
    uint64_t resident = 0;     // bytes held while the set is resident
    uint64_t transient = 0;    // bytes held while the build runs
    uint64_t last_use = 0;
    int users = 0;             // queued or running KDE requests on this set
    std::vector<void*> blocks; // pooled device blocks owned by the set
};

struct Req {
    int64_t id = -1;
    Kind kind = Kind::kBuild;
    int64_t set_id = -1;
    bool admitted = false;
    // build
    const float* X_src = nullptr;
    // KDE
    const float* Q = nullptr;
    int64_t m = 0;
    double gamma = 0.0;
    double* out = nullptr;
    fsg_points* qpts = nullptr;
    std::vector<void*> blocks;
    hipEvent_t ev = nullptr;
    int32_t status = FSG_OK;
};

__global__ void kde_request_setup_kernel(int64_t m, int32_t n, int64_t* q_ptr, int32_t* q_idx, int32_t* seg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) q_idx[i] = (int32_t)i;
    if (i == 0) {
        q_ptr[0] = 0;
        q_ptr[1] = m;
        seg[0] = 0;  // lo
        seg[1] = n;  // mid: the whole set in the first half
        seg[2] = n;  // hi
    }
}

}  // namespace
}  // namespace fsg

using namespace fsg;

struct fsg_server {
    fsg_ctx* ctx = nullptr;
    uint64_t budget = 0;
    int32_t max_active = 1;
    int64_t next_req = 0;
    uint64_t used = 0;
    uint64_t tick = 0;
    int64_t evictions = 0;
    std::map<int64_t, SetRec*> sets;
    std::deque<Req*> queue;
    std::vector<Req*> running;    // admitted, device work not yet seen complete
    std::vector<SetRec*> building;
    std::deque<Req*> finished;    // complete, not yet reported
    std::vector<hipEvent_t> events;
    hipEvent_t step_ev = nullptr; // recorded after the work a poll enqueued
    int64_t* host = nullptr;      // pinned slots: {nnz, n_long} of finished builds
    std::vector<int32_t> free_slots;
};

// pinned {nnz, n_long} slots: one per build in flight
constexpr int32_t kServerSlots = 4096;

namespace {

void* blk(fsg_ctx* ctx, std::vector<void*>& owner, size_t bytes) {
    void* p = nullptr;
    if (pool_alloc(ctx, bytes, &p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    owner.push_back(p);
    return p;
}

void release(fsg_ctx* ctx, std::vector<void*>& owner) {
    for (void* p : owner) pool_release(ctx, p);
    owner.clear();
}

hipEvent_t take_ev(fsg_server* s) {
    if (!s->events.empty()) {
        hipEvent_t e = s->events.back();
        s->events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void drop_set(fsg_server* s, SetRec* r) {
    if (r->slot >= 0) s->free_slots.push_back(r->slot);
    if (r->job) fsg_job_destroy(r->job);
    if (r->pts) fsg_points_destroy(r->pts);
    release(s->ctx, r->blocks);
    s->used -= r->resident + (r->ready ? 0 : r->transient);
    s->sets.erase(r->id);
    delete r;
}

// evict ready, unused sets (least recently used first) until `need` more
// bytes fit; false if they cannot
bool make_room(fsg_server* s, uint64_t need) {
    while (s->used + need > s->budget) {
        SetRec* victim = nullptr;
        for (auto& kv : s->sets) {
            SetRec* r = kv.second;
            if (r->ready && r->users == 0 && (!victim || r->last_use < victim->last_use)) victim = r;
        }
        if (!victim) return false;
        drop_set(s, victim);
        ++s->evictions;
    }
    return true;
}

fsg_status admit_build(fsg_server* s, Req* q) {
    fsg_ctx* ctx = s->ctx;
    SetRec* r = s->sets[q->set_id];
    fsg_status st;
    r->X = (float*)blk(ctx, r->blocks, (size_t)r->n * r->d * sizeof(float));
    if (!r->X) return set_error(ctx, FSG_E_NOMEM, "server: allocation of a point set failed");
    FSG_HIP(ctx, hipMemcpyAsync(r->X, q->X_src, (size_t)r->n * r->d * sizeof(float), hipMemcpyDeviceToDevice,
                                ctx->stream));
    if ((st = fsg_points_create(ctx, r->X, r->n, r->d, r->prec, &r->pts)) != FSG_OK) return st;
    if ((st = fsg_job_create(ctx, r->pts, r->gamma, r->L, r->seed, &r->job)) != FSG_OK) return st;
    const int64_t ns = r->n * (int64_t)r->L;
    r->row_ptr = (int64_t*)blk(ctx, r->blocks, (size_t)(r->n + 1) * sizeof(int64_t));
    r->col = (int32_t*)blk(ctx, r->blocks, (size_t)(2 * ns) * sizeof(int32_t));
    r->w = (float*)blk(ctx, r->blocks, (size_t)(2 * ns) * sizeof(float));
    r->nbr = (int32_t*)blk(ctx, r->blocks, (size_t)ns * sizeof(int32_t));
    r->deg = (double*)blk(ctx, r->blocks, (size_t)r->n * sizeof(double));
    r->n_long = (int32_t*)blk(ctx, r->blocks, sizeof(int32_t));
    if (!r->row_ptr || !r->col || !r->w || !r->nbr || !r->deg || !r->n_long)
        return set_error(ctx, FSG_E_NOMEM, "server: allocation of a result failed");
    if (s->free_slots.empty()) return set_error(ctx, FSG_E_BUDGET, "server: too many builds in flight");
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->building.push_back(r);
    return FSG_OK;
}

fsg_status admit_kde(fsg_server* s, Req* q, SetRec* r) {
    fsg_ctx* ctx = s->ctx;
    fsg_status st;
    if ((st = fsg_points_create(ctx, q->Q, q->m, r->d, FSG_PLAIN_FP64, &q->qpts)) != FSG_OK) return st;
    int64_t* q_ptr = (int64_t*)blk(ctx, q->blocks, 2 * sizeof(int64_t));
    int32_t* q_idx = (int32_t*)blk(ctx, q->blocks, (size_t)q->m * sizeof(int32_t));
    int32_t* seg = (int32_t*)blk(ctx, q->blocks, 3 * sizeof(int32_t));
    double* right = (double*)blk(ctx, q->blocks, (size_t)q->m * sizeof(double));
    if (!q_ptr || !q_idx || !seg || !right) return set_error(ctx, FSG_E_NOMEM, "server: allocation failed");
    kde_request_setup_kernel<<<(unsigned)((q->m + 255) / 256 + 1), 256, 0, ctx->stream>>>(q->m, (int32_t)r->n, q_ptr,
                                                                                          q_idx, seg);
    FSG_HIP(ctx, hipGetLastError());
    if ((st = fsg_kde_segmented(ctx, q->qpts, r->pts, q->gamma, 1, q->m, q_ptr, q_idx, seg, seg + 1, seg + 2, nullptr,
                                q->out, right)) != FSG_OK)
        return st;
    return FSG_OK;
}

void finish(fsg_server* s, Req* q, int32_t status) {
    q->status = status;
    s->finished.push_back(q);
}

// hand up to `cap` finished requests to the caller
fsg_status report(fsg_server* s, int64_t* done_ids, int32_t* done_status, int32_t cap, int32_t* n_done) {
    int32_t nd = 0;
    while (nd < cap && !s->finished.empty()) {
        Req* q = s->finished.front();
        s->finished.pop_front();
        done_ids[nd] = q->id;
        done_status[nd] = q->status;
        ++nd;
        delete q;
    }
    *n_done = nd;
    return FSG_OK;
}

}  // namespace

namespace fsg {

// Release every set, request, event and pinned slot of a server (its context
// is about to be destroyed, or the server is); the handle stays valid.
void server_detach(fsg_server* s) {
    if (!s->ctx) return;
    (void)hipStreamSynchronize(s->ctx->stream);
    std::vector<SetRec*> all;
    for (auto& kv : s->sets) all.push_back(kv.second);
    for (SetRec* r : all) drop_set(s, r);
    auto drop_req = [&](Req* q) {
        if (q->qpts) fsg_points_destroy(q->qpts);
        release(s->ctx, q->blocks);
        if (q->ev) (void)hipEventDestroy(q->ev);
        delete q;
    };
    for (Req* q : s->queue) drop_req(q);
    for (Req* q : s->running) drop_req(q);
    for (Req* q : s->finished) drop_req(q);
    s->queue.clear();
    s->running.clear();
    s->finished.clear();
    s->building.clear();
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    s->events.clear();
    if (s->step_ev) (void)hipEventDestroy(s->step_ev);
    s->step_ev = nullptr;
    if (s->host) (void)hipHostFree(s->host);
    s->host = nullptr;
    s->ctx->servers.erase(s);
    s->ctx = nullptr;
}

}  // namespace fsg

extern "C" {

fsg_status fsg_server_create(fsg_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_active, fsg_server** out) {
    if (!ctx || !out) return FSG_E_INVALID;
    *out = nullptr;
    if (max_active < 1) return set_error(ctx, FSG_E_INVALID, "max_active must be >= 1");
    if (hbm_budget_bytes == 0) return set_error(ctx, FSG_E_INVALID, "the budget must be > 0");
    if (max_active > kServerSlots) return set_error(ctx, FSG_E_INVALID, "max_active is too large");
    fsg_server* s = new (std::nothrow) fsg_server();
    if (!s) return set_error(ctx, FSG_E_NOMEM, "host allocation failed");
    if (hipHostMalloc((void**)&s->host, (size_t)kServerSlots * 2 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return set_error(ctx, FSG_E_NOMEM, "pinned host allocation failed");
    }
    for (int32_t k = kServerSlots - 1; k >= 0; --k) s->free_slots.push_back(k);
    s->ctx = ctx;
    ctx->servers.insert(s);
    s->budget = hbm_budget_bytes;
    s->max_active = max_active;
    *out = s;
    return FSG_OK;
}

void fsg_server_destroy(fsg_server* s) {
    if (!s) return;
    if (s->ctx) server_detach(s);
    delete s;
}

fsg_status fsg_server_submit_build(fsg_server* s, int64_t set_id, const float* X_dev, int64_t n, int32_t d,
                                   double gamma, int32_t L, uint64_t seed, fsg_precision prec, int64_t* req_id) {
    if (s && !s->ctx) return FSG_E_INVALID;  // its context was destroyed
    if (!s || !req_id) return FSG_E_INVALID;
    fsg_ctx* ctx = s->ctx;
    if (ctx->kernel != FSG_GAUSSIAN) return set_error(ctx, FSG_E_UNSUPPORTED, "servers use the Gaussian kernel only");
    if (set_id < 0 || s->sets.count(set_id)) return set_error(ctx, FSG_E_INVALID, "set_id is negative or in use");
    if (!X_dev || n < 1 || n > 2147483647LL || d < 1) return set_error(ctx, FSG_E_INVALID, "bad point set");
    if (!(gamma > 0.0) || !(gamma < 1e308) || L < 1) return set_error(ctx, FSG_E_INVALID, "bad gamma or L");
    if (feature_steps(d) < 0 || (prec == FSG_BF16_SPLIT && filter_steps(feature_steps(d)) < 0))
        return set_error(ctx, FSG_E_UNSUPPORTED, "d is not built for this precision");
    SetRec* r = new (std::nothrow) SetRec();
    if (!r) return set_error(ctx, FSG_E_NOMEM, "host allocation failed");
    r->id = set_id;
    r->n = n;
    r->d = d;
    r->gamma = gamma;
    r->L = L;
    r->seed = seed;
    r->prec = prec;
    build_bytes_estimate(ctx, n, d, L, prec, &r->resident, &r->transient);
    if (r->resident + r->transient > s->budget) {
        delete r;
        return set_error(ctx, FSG_E_BUDGET, "the build needs more than the whole budget");
    }
    Req* q = new (std::nothrow) Req();
    if (!q) {
        delete r;
        return set_error(ctx, FSG_E_NOMEM, "host allocation failed");
    }
    q->id = s->next_req++;
    q->kind = Kind::kBuild;
    q->set_id = set_id;
    q->X_src = X_dev;
    s->sets[set_id] = r;
    s->queue.push_back(q);
    *req_id = q->id;
    return FSG_OK;
}

fsg_status fsg_server_submit_kde(fsg_server* s, int64_t set_id, const float* Q_dev, int64_t m, double gamma,
                                 double* out_dev, int64_t* req_id) {
    if (s && !s->ctx) return FSG_E_INVALID;  // its context was destroyed
    if (!s || !req_id) return FSG_E_INVALID;
    fsg_ctx* ctx = s->ctx;
    if (!Q_dev || !out_dev || m < 1 || m > 2147483647LL) return set_error(ctx, FSG_E_INVALID, "bad query set");
    if (!(gamma > 0.0) || !(gamma < 1e308)) return set_error(ctx, FSG_E_INVALID, "bad gamma");
    Req* q = new (std::nothrow) Req();
    if (!q) return set_error(ctx, FSG_E_NOMEM, "host allocation failed");
    q->id = s->next_req++;
    q->kind = Kind::kKde;
    q->set_id = set_id;
    q->Q = Q_dev;
    q->m = m;
    q->gamma = gamma;
    q->out = out_dev;
    auto it = s->sets.find(set_id);
    if (it != s->sets.end()) ++it->second->users;
    s->queue.push_back(q);
    *req_id = q->id;
    return FSG_OK;
}

fsg_status fsg_server_poll(fsg_server* s, int64_t* done_ids, int32_t* done_status, int32_t cap, int32_t* n_done) {
    if (s && !s->ctx) return FSG_E_INVALID;  // its context was destroyed
    if (!s || !n_done || cap < 0 || (cap > 0 && (!done_ids || !done_status))) return FSG_E_INVALID;
    fsg_ctx* ctx = s->ctx;
    fsg_status st;
    ++s->tick;
    // 1. requests whose device work has finished
    for (size_t k = 0; k < s->running.size();) {
        Req* q = s->running[k];
        if (q->ev == nullptr) {  // a build still running its stages
            ++k;
            continue;
        }
        const hipError_t e = hipEventQuery(q->ev);
        if (e == hipErrorNotReady) {
            ++k;
            continue;
        }
        int32_t status = (e == hipSuccess) ? FSG_OK : FSG_E_DEVICE;
        if (e != hipSuccess) (void)hipGetLastError();
        s->events.push_back(q->ev);
        q->ev = nullptr;
        auto it = s->sets.find(q->set_id);
        SetRec* r = (it != s->sets.end()) ? it->second : nullptr;
        if (q->kind == Kind::kBuild && r) {
            // copied to the pinned slot before the completion event
            int64_t nnz = s->host[2 * r->slot];
            const int32_t longs = (int32_t)(s->host[2 * r->slot + 1] & 0xFFFFFFFF);
            s->free_slots.push_back(r->slot);
            r->slot = -1;
            if (status == FSG_OK && longs > 0)  // a row over the row-sort limit: rebuild by the global sort
                status = fsg_build_csr(ctx, r->pts, r->gamma, r->L, r->nbr, r->deg, r->row_ptr, r->col, r->w,
                                       2 * r->n * (int64_t)r->L, &nnz);
            r->nnz = nnz;
            r->ready = status == FSG_OK;
            r->last_use = s->tick;
        } else if (q->kind == Kind::kKde) {
            if (q->qpts) fsg_points_destroy(q->qpts);
            q->qpts = nullptr;
            release(ctx, q->blocks);
            if (r) {
                --r->users;
                r->last_use = s->tick;
            }
        }
        s->running.erase(s->running.begin() + k);
        finish(s, q, status);
    }
    // new work starts once the previous poll's work has finished, so that the
    // requests arriving meanwhile are admitted (and their root passes
    // batched) together
    if (s->step_ev != nullptr) {
        const hipError_t e = hipEventQuery(s->step_ev);
        if (e == hipErrorNotReady) return report(s, done_ids, done_status, cap, n_done);
        if (e != hipSuccess) (void)hipGetLastError();
    }
    // 2. admission in arrival order; a KDE request whose set is still being
    // built waits without holding up the requests behind it
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Req* q = *it;
        if (q->kind == Kind::kBuild) {
            if ((int32_t)s->building.size() >= s->max_active) break;
            SetRec* r = s->sets[q->set_id];
            const uint64_t need = r->resident + r->transient;
            if (!make_room(s, need)) break;
            s->used += need;
            if ((st = admit_build(s, q)) != FSG_OK) {
                // the set's memory is released; the request fails
                s->building.erase(std::remove(s->building.begin(), s->building.end(), r), s->building.end());
                drop_set(s, r);
                it = s->queue.erase(it);
                finish(s, q, st);
                continue;
            }
            q->admitted = true;
            s->running.push_back(q);
            it = s->queue.erase(it);
            continue;
        }
        auto si = s->sets.find(q->set_id);
        if (si == s->sets.end()) {  // never built, or evicted
            it = s->queue.erase(it);
            finish(s, q, FSG_E_INVALID);
            continue;
        }
        SetRec* r = si->second;
        if (!r->ready) {
            ++it;
            continue;
        }
        if ((st = admit_kde(s, q, r)) != FSG_OK) {
            if (q->qpts) fsg_points_destroy(q->qpts);
            q->qpts = nullptr;
            release(ctx, q->blocks);
            --r->users;
            it = s->queue.erase(it);
            finish(s, q, st);
            continue;
        }
        q->ev = take_ev(s);
        if (!q->ev) return set_error(ctx, FSG_E_DEVICE, "server: event creation failed");
        FSG_HIP(ctx, hipEventRecord(q->ev, ctx->stream));
        q->admitted = true;
        s->running.push_back(q);
        it = s->queue.erase(it);
    }
    // 3. one stage of every active build
    if (!s->building.empty()) {
        std::vector<fsg_job*> jobs;
        for (SetRec* r : s->building) jobs.push_back(r->job);
        int32_t done = 0;
        if ((st = fsg_batch_step(ctx, jobs.data(), (int32_t)jobs.size(), &done)) != FSG_OK) return st;
        for (size_t k = 0; k < s->building.size();) {
            SetRec* r = s->building[k];
            if (!job_finished(r->job)) {
                ++k;
                continue;
            }
            if ((st = fsg_job_result(r->job, r->nbr, r->deg)) != FSG_OK) return st;
            if ((st = csr_rows_async(ctx, r->pts, r->gamma, r->L, r->nbr, r->deg, r->row_ptr, r->col, r->w,
                                     2 * r->n * (int64_t)r->L, r->n_long)) != FSG_OK)
                return st;
            FSG_HIP(ctx, hipMemcpyAsync(s->host + 2 * r->slot, r->row_ptr + r->n, sizeof(int64_t),
                                        hipMemcpyDeviceToHost, ctx->stream));
            FSG_HIP(ctx, hipMemcpyAsync(s->host + 2 * r->slot + 1, r->n_long, sizeof(int32_t), hipMemcpyDeviceToHost,
                                        ctx->stream));
            // the job's buffers return to the pool (stream-ordered reuse)
            fsg_job_destroy(r->job);
            r->job = nullptr;
            s->used -= r->transient;
            Req* q = nullptr;
            for (Req* x : s->running)
                if (x->kind == Kind::kBuild && x->set_id == r->id) q = x;
            if (q) {
                q->ev = take_ev(s);
                if (!q->ev) return set_error(ctx, FSG_E_DEVICE, "server: event creation failed");
                FSG_HIP(ctx, hipEventRecord(q->ev, ctx->stream));
            }
            s->building.erase(s->building.begin() + k);
        }
    }
    if (s->step_ev == nullptr) {
        s->step_ev = take_ev(s);
        if (!s->step_ev) return set_error(ctx, FSG_E_DEVICE, "server: event creation failed");
    }
    FSG_HIP(ctx, hipEventRecord(s->step_ev, ctx->stream));
    return report(s, done_ids, done_status, cap, n_done);
}

fsg_status fsg_server_graph(fsg_server* s, int64_t set_id, const int64_t** row_ptr, const int32_t** col,
                            const float** w, int64_t* nnz, const int32_t** nbr, const double** deg) {
    if (s && !s->ctx) return FSG_E_INVALID;  // its context was destroyed
    if (!s) return FSG_E_INVALID;
    auto it = s->sets.find(set_id);
    if (it == s->sets.end() || !it->second->ready)
        return set_error(s->ctx, FSG_E_INVALID, "the set is not resident or not finished");
    SetRec* r = it->second;
    r->last_use = s->tick;
    if (row_ptr) *row_ptr = r->row_ptr;
    if (col) *col = r->col;
    if (w) *w = r->w;
    if (nnz) *nnz = r->nnz;
    if (nbr) *nbr = r->nbr;
    if (deg) *deg = r->deg;
    return FSG_OK;
}

fsg_status fsg_server_stats(fsg_server* s, uint64_t* resident_bytes, int32_t* active, int32_t* queued,
                            int64_t* evictions) {
    if (s && !s->ctx) return FSG_E_INVALID;  // its context was destroyed
    if (!s) return FSG_E_INVALID;
    if (resident_bytes) *resident_bytes = s->used;
    if (active) *active = (int32_t)s->building.size();
    if (queued) *queued = (int32_t)s->queue.size();
    if (evictions) *evictions = s->evictions;
    return FSG_OK;
}

}  // extern "C"
