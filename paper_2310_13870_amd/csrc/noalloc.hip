// The no-allocation variant of the segmented KDE, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its work lists and partial sums live in
// a static device array of fixed size instead of the context's workspace.
#include <mutex>

#include "common.h"

namespace fsg {

// The scratch of fsg_kde_segmented_noalloc: one copy per GPU, held until the
// process ends.  In host code this name is only a stand-in for the symbol;
// kernels get the device address looked up by noalloc_scratch_setup.
static __device__ __align__(256) unsigned char scratch[FSG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};
}  // namespace

void* noalloc_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        // the caller (fsg_ctx_create) has made `device` current
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;  // retried by the next context on this device
        }
        g_ptr[device] = p;
        g_done[device] = true;
    }
    return g_ptr[device];
}

static size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace fsg

using namespace fsg;

extern "C" {

fsg_status fsg_kde_segmented_noalloc(fsg_ctx* ctx, const fsg_points* Q, const fsg_points* X, double gamma,
                                     int64_t n_seg, int64_t n_entries, const int64_t* q_ptr, const int32_t* q_idx,
                                     const int32_t* lo, const int32_t* mid, const int32_t* hi,
                                     const int32_t* self_idx, double* out_left, double* out_right) {
    bool empty = false;
    fsg_status st = kde_segmented_check(ctx, Q, X, gamma, n_seg, n_entries, q_ptr, q_idx, lo, mid, hi, out_left,
                                        out_right, &empty);
    if (st != FSG_OK || empty) return st;
    if (ctx->noalloc_scratch == nullptr)
        return set_error(ctx, FSG_E_DEVICE, "the static scratch of this device could not be located");
    const KdeSegSizes z = kde_segmented_sizes(X, n_seg, n_entries);
    // carve the buffers out of the scratch, each on a 256-byte boundary
    const size_t o_bounds = 0;
    const size_t o_segs = up256(o_bounds + (size_t)z.bounds * sizeof(int32_t));
    const size_t o_items = up256(o_segs + (size_t)n_seg * sizeof(SegDesc));
    const size_t o_nitems = up256(o_items + (size_t)z.max_items * sizeof(WorkItem));
    const size_t o_counts = up256(o_nitems + sizeof(int32_t));
    const size_t o_pairs = up256(o_counts + (size_t)z.counts * sizeof(int64_t));
    const size_t need = up256(o_pairs + (size_t)z.pairs * sizeof(double));
    if (need > (size_t)FSG_NOALLOC_SCRATCH_BYTES)
        return set_error(ctx, FSG_E_UNSUPPORTED,
                         "fsg_kde_segmented_noalloc needs " + std::to_string(need) +
                             " bytes of scratch for these sizes; the static scratch holds " +
                             std::to_string((size_t)FSG_NOALLOC_SCRATCH_BYTES) + " bytes");
    char* base = (char*)ctx->noalloc_scratch;
    KdeSegBufs b;
    b.bounds = (int32_t*)(base + o_bounds);
    b.segs = (SegDesc*)(base + o_segs);
    b.items = (WorkItem*)(base + o_items);
    b.n_items = (int32_t*)(base + o_nitems);
    b.counts = (int64_t*)(base + o_counts);
    b.pairs = (double*)(base + o_pairs);
    return kde_segmented_enqueue(ctx, Q, X, gamma, n_seg, n_entries, q_ptr, q_idx, lo, mid, hi, self_idx, out_left,
                                 out_right, b);
}

}  // extern "C"
