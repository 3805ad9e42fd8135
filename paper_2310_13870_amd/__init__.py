"""Python binding of libfsg.so (FastSimilarityGraph hot path on MI355X).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.
The names follow the C ABI in include/fsg.h.  There is no fallback: if the
library is missing, importing the binding raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsg.so")

FSG_OK, FSG_E_INVALID, FSG_E_NOMEM, FSG_E_DEVICE, FSG_E_UNSUPPORTED, FSG_E_BUDGET = 0, -1, -2, -3, -4, -5
FSG_PLAIN_FP64, FSG_BF16_SPLIT = 0, 1
PRECISIONS = {"plain_fp64": FSG_PLAIN_FP64, "bf16_split": FSG_BF16_SPLIT}
FSG_GAUSSIAN, FSG_EXPONENTIAL, FSG_LAPLACIAN = 0, 1, 2
KERNELS = {"gaussian": FSG_GAUSSIAN, "exponential": FSG_EXPONENTIAL, "laplacian": FSG_LAPLACIAN}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libfsg.so is not built ({LIB_PATH}); run paper_2310_13870_amd/build.py")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i64, _i32, _u64, _dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_lib_fns = dict(
    fsg_ctx_create=_sig("fsg_ctx_create", ctypes.c_int, ctypes.c_int, _vp, _u64, ctypes.POINTER(_vp)),
    fsg_ctx_destroy=_sig("fsg_ctx_destroy", None, _vp),
    fsg_status_string=_sig("fsg_status_string", ctypes.c_char_p, ctypes.c_int),
    fsg_last_error=_sig("fsg_last_error", ctypes.c_char_p, _vp),
    fsg_ctx_sync=_sig("fsg_ctx_sync", ctypes.c_int, _vp),
    fsg_ctx_workspace_bytes=_sig("fsg_ctx_workspace_bytes", _u64, _vp),
    fsg_ctx_set_levels_per_pass=_sig("fsg_ctx_set_levels_per_pass", ctypes.c_int, _vp, _i32),
    fsg_ctx_set_pruning=_sig("fsg_ctx_set_pruning", ctypes.c_int, _vp, _i32),
    fsg_ctx_set_exact_slices=_sig("fsg_ctx_set_exact_slices", ctypes.c_int, _vp, _i32),
    fsg_ctx_set_kernel=_sig("fsg_ctx_set_kernel", ctypes.c_int, _vp, ctypes.c_int),
    fsg_ctx_set_kde_error=_sig("fsg_ctx_set_kde_error", ctypes.c_int, _vp, _dbl),
    fsg_ctx_set_profiling=_sig("fsg_ctx_set_profiling", ctypes.c_int, _vp, ctypes.c_int),
    fsg_ctx_stage_time=_sig("fsg_ctx_stage_time", ctypes.c_int, _vp, ctypes.c_char_p, ctypes.POINTER(_dbl),
                            ctypes.POINTER(_i64)),
    fsg_ctx_reset_profiling=_sig("fsg_ctx_reset_profiling", ctypes.c_int, _vp),
    fsg_ctx_filter_stats=_sig("fsg_ctx_filter_stats", ctypes.c_int, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)),
    fsg_points_create=_sig("fsg_points_create", ctypes.c_int, _vp, _vp, _i64, _i32, ctypes.c_int,
                           ctypes.POINTER(_vp)),
    fsg_points_destroy=_sig("fsg_points_destroy", None, _vp),
    fsg_points_bytes=_sig("fsg_points_bytes", _u64, _vp),
    fsg_degrees=_sig("fsg_degrees", ctypes.c_int, _vp, _vp, _dbl, _vp),
    fsg_kde_segmented=_sig("fsg_kde_segmented", ctypes.c_int, _vp, _vp, _vp, _dbl, _i64, _i64, _vp, _vp, _vp,
                           _vp, _vp, _vp, _vp, _vp),
    fsg_kde_segmented_noalloc=_sig("fsg_kde_segmented_noalloc", ctypes.c_int, _vp, _vp, _vp, _dbl, _i64, _i64, _vp,
                                   _vp, _vp, _vp, _vp, _vp, _vp, _vp),
    fsg_sample_edges=_sig("fsg_sample_edges", ctypes.c_int, _vp, _vp, _dbl, _i32, _u64, _vp, _vp, _vp),
    fsg_build_csr=_sig("fsg_build_csr", ctypes.c_int, _vp, _vp, _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _i64,
                       ctypes.POINTER(_i64)),
    fsg_job_create=_sig("fsg_job_create", ctypes.c_int, _vp, _vp, _dbl, _i32, _u64, ctypes.POINTER(_vp)),
    fsg_batch_step=_sig("fsg_batch_step", ctypes.c_int, _vp, ctypes.POINTER(_vp), _i32, ctypes.POINTER(_i32)),
    fsg_job_reset=_sig("fsg_job_reset", ctypes.c_int, _vp),
    fsg_job_result=_sig("fsg_job_result", ctypes.c_int, _vp, _vp, _vp),
    fsg_job_outputs=_sig("fsg_job_outputs", ctypes.c_int, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)),
    fsg_job_destroy=_sig("fsg_job_destroy", None, _vp),
    fsg_ctx_set_autotune=_sig("fsg_ctx_set_autotune", ctypes.c_int, _vp, _i32),
    fsg_ctx_save_tuning=_sig("fsg_ctx_save_tuning", ctypes.c_int, _vp, ctypes.c_char_p),
    fsg_ctx_load_tuning=_sig("fsg_ctx_load_tuning", ctypes.c_int, _vp, ctypes.c_char_p, ctypes.POINTER(_i32)),
    fsg_ctx_tuned_shape=_sig("fsg_ctx_tuned_shape", ctypes.c_int, _vp, _i32, ctypes.c_int, ctypes.POINTER(_i32),
                             ctypes.POINTER(_i32)),
    fsg_graph_begin=_sig("fsg_graph_begin", ctypes.c_int, _vp),
    fsg_graph_end=_sig("fsg_graph_end", ctypes.c_int, _vp, ctypes.POINTER(_vp)),
    fsg_graph_launch=_sig("fsg_graph_launch", ctypes.c_int, _vp, _vp),
    fsg_graph_destroy=_sig("fsg_graph_destroy", None, _vp),
    fsg_server_create=_sig("fsg_server_create", ctypes.c_int, _vp, _u64, _i32, ctypes.POINTER(_vp)),
    fsg_server_destroy=_sig("fsg_server_destroy", None, _vp),
    fsg_server_submit_build=_sig("fsg_server_submit_build", ctypes.c_int, _vp, _i64, _vp, _i64, _i32, _dbl, _i32,
                                 _u64, ctypes.c_int, ctypes.POINTER(_i64)),
    fsg_server_submit_kde=_sig("fsg_server_submit_kde", ctypes.c_int, _vp, _i64, _vp, _i64, _dbl, _vp,
                               ctypes.POINTER(_i64)),
    fsg_server_poll=_sig("fsg_server_poll", ctypes.c_int, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32), _i32,
                         ctypes.POINTER(_i32)),
    fsg_server_graph=_sig("fsg_server_graph", ctypes.c_int, _vp, _i64, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                          ctypes.POINTER(_vp), ctypes.POINTER(_i64), ctypes.POINTER(_vp), ctypes.POINTER(_vp)),
    fsg_server_stats=_sig("fsg_server_stats", ctypes.c_int, _vp, ctypes.POINTER(_u64), ctypes.POINTER(_i32),
                          ctypes.POINTER(_i32), ctypes.POINTER(_i64)),
)
EXPORTED = sorted(_lib_fns)


class FsgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


def status_string(status: int) -> str:
    return _lib.fsg_status_string(status).decode()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_tensor(t, dtype, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """fsg_ctx: one device and one HIP stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None, ws_budget_bytes: int = 0):
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = _vp()
        st = _lib.fsg_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ws_budget_bytes, ctypes.byref(h))
        if st != FSG_OK:
            raise FsgError(st, "fsg_ctx_create failed")
        self._h = h

    def check(self, st):
        if st != FSG_OK:
            raise FsgError(st, _lib.fsg_last_error(self._h).decode())

    def sync(self):
        self.check(_lib.fsg_ctx_sync(self._h))

    def set_levels_per_pass(self, max_levels: int):
        """Cap the tree levels one binned pass resolves (0 = automatic)."""
        self.check(_lib.fsg_ctx_set_levels_per_pass(self._h, max_levels))

    def set_kernel(self, kind):
        """Kernel of later calls: "gaussian" (default), "exponential" or "laplacian"."""
        if isinstance(kind, str):
            kind = KERNELS[kind]
        self.check(_lib.fsg_ctx_set_kernel(self._h, kind))

    def set_kde_error(self, eps: float):
        """Precision mode: the share of every degree the root KDE may drop (0: e^-25, the exact mode)."""
        self.check(_lib.fsg_ctx_set_kde_error(self._h, float(eps)))

    def set_pruning(self, enabled):
        """Precision mode: skip (query tile, cell) pairs that cannot keep a column.
        True: on; False: off; None (default): on for sets of at least 2^18 points."""
        self.check(_lib.fsg_ctx_set_pruning(self._h, -1 if enabled is None else (1 if enabled else 0)))

    def set_exact_slices(self, enabled):
        """Precision mode, 32 < d <= 64, Gaussian kernel: recompute kept pairs' cross terms from
        int8 slice products (True or None, the default) or on the FP64 matrix cores (False)."""
        self.check(_lib.fsg_ctx_set_exact_slices(self._h, -1 if enabled is None else (1 if enabled else 0)))

    def set_profiling(self, enabled: bool):
        self.check(_lib.fsg_ctx_set_profiling(self._h, 1 if enabled else 0))

    def reset_profiling(self):
        self.check(_lib.fsg_ctx_reset_profiling(self._h))

    def stage_time(self, stage: str):
        """(summed ms, launches) of one stage since the last reset."""
        ms, cnt = _dbl(0.0), _i64(0)
        self.check(_lib.fsg_ctx_stage_time(self._h, stage.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def filter_stats(self):
        """(kept, scanned) (data column, 64-query tile) pairs of the precision-mode
        filter since the last reset."""
        kept, scanned = _i64(0), _i64(0)
        self.check(_lib.fsg_ctx_filter_stats(self._h, ctypes.byref(kept), ctypes.byref(scanned)))
        return kept.value, scanned.value

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.fsg_ctx_workspace_bytes(self._h))

    def set_autotune(self, enabled: bool):
        self.check(_lib.fsg_ctx_set_autotune(self._h, 1 if enabled else 0))

    def tuned_shape(self, D4: int, precision=FSG_PLAIN_FP64):
        """(waves per CU, data columns per work item) tuned for a class, or None."""
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        w, c = _i32(0), _i32(0)
        st = _lib.fsg_ctx_tuned_shape(self._h, D4, precision, ctypes.byref(w), ctypes.byref(c))
        return (w.value, c.value) if st == FSG_OK else None

    def save_tuning(self, path: str):
        self.check(_lib.fsg_ctx_save_tuning(self._h, os.fsencode(path)))

    def load_tuning(self, path: str) -> int:
        """Tuned shapes from a file written on the same kind of device; returns how many were taken over."""
        n = _i32(0)
        self.check(_lib.fsg_ctx_load_tuning(self._h, os.fsencode(path), ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.fsg_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Points:
    """fsg_points: a resident point set.  Keeps a reference to X (borrowed by the library)."""

    def __init__(self, ctx: Context, X: torch.Tensor, precision=FSG_PLAIN_FP64):
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        _dev_tensor(X, torch.float32, "X")
        if X.dim() != 2:
            raise ValueError("X must be n x d")
        self.ctx, self.X = ctx, X
        self.n, self.d = X.shape
        h = _vp()
        ctx.check(_lib.fsg_points_create(ctx._h, _ptr(X), self.n, self.d, precision, ctypes.byref(h)))
        self._h = h

    @property
    def bytes(self) -> int:
        return int(_lib.fsg_points_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.fsg_points_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def degrees(ctx: Context, pts: Points, gamma: float, out: torch.Tensor = None) -> torch.Tensor:
    if out is None:
        out = torch.empty(pts.n, dtype=torch.float64, device=pts.X.device)
    _dev_tensor(out, torch.float64, "out")
    ctx.check(_lib.fsg_degrees(ctx._h, pts._h, gamma, _ptr(out)))
    return out


def kde_segmented(ctx: Context, Q: Points, X: Points, gamma: float, q_ptr, q_idx, lo, mid, hi, self_idx=None):
    _dev_tensor(q_ptr, torch.int64, "q_ptr")
    for name, t in (("q_idx", q_idx), ("lo", lo), ("mid", mid), ("hi", hi)):
        _dev_tensor(t, torch.int32, name)
    if self_idx is not None:
        _dev_tensor(self_idx, torch.int32, "self_idx")
    n_seg = lo.shape[0]
    n_ent = q_idx.shape[0]
    left = torch.empty(n_ent, dtype=torch.float64, device=Q.X.device)
    right = torch.empty(n_ent, dtype=torch.float64, device=Q.X.device)
    ctx.check(_lib.fsg_kde_segmented(ctx._h, Q._h, X._h, gamma, n_seg, n_ent, _ptr(q_ptr), _ptr(q_idx), _ptr(lo),
                                     _ptr(mid), _ptr(hi), _ptr(self_idx), _ptr(left), _ptr(right)))
    return left, right


NOALLOC_SCRATCH_BYTES = 64 << 20  # FSG_NOALLOC_SCRATCH_BYTES


def kde_segmented_noalloc(ctx: Context, Q: Points, X: Points, gamma: float, q_ptr, q_idx, lo, mid, hi,
                          out_left: torch.Tensor, out_right: torch.Tensor, self_idx=None):
    """fsg_kde_segmented_noalloc: the segmented KDE into caller-given outputs,
    with the library's static scratch instead of workspace allocations."""
    _dev_tensor(q_ptr, torch.int64, "q_ptr")
    for name, t in (("q_idx", q_idx), ("lo", lo), ("mid", mid), ("hi", hi)):
        _dev_tensor(t, torch.int32, name)
    if self_idx is not None:
        _dev_tensor(self_idx, torch.int32, "self_idx")
    _dev_tensor(out_left, torch.float64, "out_left")
    _dev_tensor(out_right, torch.float64, "out_right")
    n_seg = lo.shape[0]
    n_ent = q_idx.shape[0]
    if out_left.numel() < n_ent or out_right.numel() < n_ent:
        raise ValueError("outputs hold fewer entries than q_idx")
    ctx.check(_lib.fsg_kde_segmented_noalloc(ctx._h, Q._h, X._h, gamma, n_seg, n_ent, _ptr(q_ptr), _ptr(q_idx),
                                             _ptr(lo), _ptr(mid), _ptr(hi), _ptr(self_idx), _ptr(out_left),
                                             _ptr(out_right)))
    return out_left, out_right


def sample_edges(ctx: Context, pts: Points, gamma: float, L: int, seed: int, want_deg: bool = True,
                 want_margin: bool = False, nbr: torch.Tensor = None):
    dev = pts.X.device
    if nbr is None:
        nbr = torch.empty((pts.n, L), dtype=torch.int32, device=dev)
    deg = torch.empty(pts.n, dtype=torch.float64, device=dev) if want_deg else None
    margin = torch.empty((pts.n, L), dtype=torch.float32, device=dev) if want_margin else None
    ctx.check(_lib.fsg_sample_edges(ctx._h, pts._h, gamma, L, seed, _ptr(nbr), _ptr(deg), _ptr(margin)))
    return nbr, deg, margin


def build_csr(ctx: Context, pts: Points, gamma: float, L: int, nbr: torch.Tensor, deg: torch.Tensor, cap: int = None,
              row_ptr=None, col=None, w=None):
    dev = pts.X.device
    if cap is None:
        cap = 2 * pts.n * L
    if row_ptr is None:
        row_ptr = torch.empty(pts.n + 1, dtype=torch.int64, device=dev)
    if col is None:
        col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    if w is None:
        w = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    _dev_tensor(nbr, torch.int32, "nbr")
    _dev_tensor(deg, torch.float64, "deg")
    nnz = _i64(0)
    ctx.check(_lib.fsg_build_csr(ctx._h, pts._h, gamma, L, _ptr(nbr), _ptr(deg), _ptr(row_ptr), _ptr(col), _ptr(w),
                                 cap, ctypes.byref(nnz)))
    return row_ptr, col[: nnz.value], w[: nnz.value]


def build_graph(ctx: Context, X: torch.Tensor, gamma: float, L: int, seed: int, precision=FSG_PLAIN_FP64):
    """Algorithm 2 end to end: prep, sampling, degrees, reweighting and CSR."""
    pts = Points(ctx, X, precision)
    nbr, deg, _ = sample_edges(ctx, pts, gamma, L, seed)
    row_ptr, col, w = build_csr(ctx, pts, gamma, L, nbr, deg)
    return row_ptr, col, w, nbr, deg


class Job:
    """fsg_job: one graph build advanced by batch_step together with others."""

    def __init__(self, ctx: Context, pts: Points, gamma: float, L: int, seed: int):
        self.ctx, self.pts, self.gamma, self.L, self.seed = ctx, pts, gamma, L, seed
        h = _vp()
        ctx.check(_lib.fsg_job_create(ctx._h, pts._h, gamma, L, seed, ctypes.byref(h)))
        self._h = h

    def reset(self):
        self.ctx.check(_lib.fsg_job_reset(self._h))

    def result(self, nbr: torch.Tensor = None, deg: torch.Tensor = None):
        dev = self.pts.X.device
        if nbr is None:
            nbr = torch.empty((self.pts.n, self.L), dtype=torch.int32, device=dev)
        if deg is None:
            deg = torch.empty(self.pts.n, dtype=torch.float64, device=dev)
        self.ctx.check(_lib.fsg_job_result(self._h, _ptr(nbr), _ptr(deg)))
        return nbr, deg

    def close(self):
        if getattr(self, "_h", None):
            _lib.fsg_job_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step(ctx: Context, jobs) -> int:
    """Advance every unfinished job by one stage; returns how many have finished."""
    arr = (_vp * max(len(jobs), 1))(*[j._h for j in jobs])
    done = _i32(0)
    ctx.check(_lib.fsg_batch_step(ctx._h, arr, len(jobs), ctypes.byref(done)))
    return done.value


def batch_run(ctx: Context, jobs) -> int:
    """batch_step until every job has finished; returns the number of steps."""
    steps = 0
    while True:
        steps += 1
        if batch_step(ctx, jobs) == len(jobs):
            return steps


class Graph:
    """fsg_graph: the work enqueued between begin() and end() on the context's
    stream, replayed by launch()."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self._h = None

    def begin(self):
        self.ctx.check(_lib.fsg_graph_begin(self.ctx._h))

    def end(self):
        h = _vp()
        self.ctx.check(_lib.fsg_graph_end(self.ctx._h, ctypes.byref(h)))
        self._h = h

    def launch(self):
        self.ctx.check(_lib.fsg_graph_launch(self.ctx._h, self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.fsg_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip_rt = None


def _view(ptr: int, count: int, dtype, device) -> torch.Tensor:
    """A copy of `count` elements at a library-owned device address (copied
    out, so that the result does not alias memory the library may reuse)."""
    global _hip_rt
    out = torch.empty(count, dtype=dtype, device=device)
    if count == 0:
        return out
    if _hip_rt is None:
        _hip_rt = ctypes.CDLL("libamdhip64.so")
        _hip_rt.hipMemcpy.restype = ctypes.c_int
        _hip_rt.hipMemcpy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int]
    err = _hip_rt.hipMemcpy(out.data_ptr(), ptr, count * out.element_size(), 3)  # device to device
    if err != 0:
        raise RuntimeError(f"hipMemcpy failed ({err})")
    return out


class Server:
    """fsg_server: request loop with HBM-budget admission, resident sets and
    continuous batching of graph builds and KDE queries."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_active: int = 16):
        self.ctx = ctx
        h = _vp()
        ctx.check(_lib.fsg_server_create(ctx._h, hbm_budget_bytes, max_active, ctypes.byref(h)))
        self._h = h
        self._keep = {}  # request id -> tensors that must stay valid until completion

    def submit_build(self, set_id: int, X: torch.Tensor, gamma: float, L: int, seed: int, precision=FSG_PLAIN_FP64) -> int:
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        _dev_tensor(X, torch.float32, "X")
        rid = _i64(0)
        self.ctx.check(_lib.fsg_server_submit_build(self._h, set_id, _ptr(X), X.shape[0], X.shape[1], gamma, L, seed,
                                                    precision, ctypes.byref(rid)))
        self._keep[rid.value] = (X,)
        return rid.value

    def submit_kde(self, set_id: int, Q: torch.Tensor, gamma: float, out: torch.Tensor = None):
        _dev_tensor(Q, torch.float32, "Q")
        if out is None:
            out = torch.empty(Q.shape[0], dtype=torch.float64, device=Q.device)
        rid = _i64(0)
        self.ctx.check(_lib.fsg_server_submit_kde(self._h, set_id, _ptr(Q), Q.shape[0], gamma, _ptr(out),
                                                  ctypes.byref(rid)))
        self._keep[rid.value] = (Q, out)
        return rid.value, out

    def poll(self, cap: int = 256):
        """[(request id, status)] of requests completed since the last poll."""
        ids = (_i64 * cap)()
        sts = (_i32 * cap)()
        nd = _i32(0)
        self.ctx.check(_lib.fsg_server_poll(self._h, ids, sts, cap, ctypes.byref(nd)))
        out = [(ids[k], sts[k]) for k in range(nd.value)]
        for rid, _ in out:
            self._keep.pop(rid, None)
        return out

    def graph(self, set_id: int, n: int, L: int):
        """Copies of a finished set's (row_ptr, col, w, nbr, deg)."""
        rp, c, w, nb, dg = _vp(), _vp(), _vp(), _vp(), _vp()
        nnz = _i64(0)
        self.ctx.check(_lib.fsg_server_graph(self._h, set_id, ctypes.byref(rp), ctypes.byref(c), ctypes.byref(w),
                                             ctypes.byref(nnz), ctypes.byref(nb), ctypes.byref(dg)))
        dev = torch.device("cuda", self.ctx.device)
        torch.cuda.current_stream().synchronize()
        return (_view(rp.value, n + 1, torch.int64, dev), _view(c.value, nnz.value, torch.int32, dev),
                _view(w.value, nnz.value, torch.float32, dev), _view(nb.value, n * L, torch.int32, dev),
                _view(dg.value, n, torch.float64, dev))

    def stats(self):
        b, a, q, e = _u64(0), _i32(0), _i32(0), _i64(0)
        self.ctx.check(_lib.fsg_server_stats(self._h, ctypes.byref(b), ctypes.byref(a), ctypes.byref(q),
                                             ctypes.byref(e)))
        return {"bytes": b.value, "active": a.value, "queued": q.value, "evictions": e.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.fsg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
