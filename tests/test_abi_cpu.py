"""CPU-side checks of the C ABI: the library loads, exports every function the
public header declares, and validates arguments on the host without a GPU."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsg.h")
LIB = os.path.join(ROOT, "paper_2310_13870_amd", "libfsg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ("fsg_degrees", "fsg_kde_segmented", "fsg_sample_edges", "fsg_build_csr",
                     "fsg_points_create", "fsg_ctx_create"):
        assert required in names


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_every_declared_function():
    import paper_2310_13870_amd as fsg
    assert set(declared_functions()) <= set(fsg.EXPORTED)


def test_status_strings_and_host_validation():
    lib = ctypes.CDLL(LIB)
    lib.fsg_status_string.restype = ctypes.c_char_p
    assert lib.fsg_status_string(0) == b"FSG_OK"
    assert lib.fsg_status_string(-1) == b"FSG_E_INVALID"
    assert lib.fsg_status_string(-5) == b"FSG_E_BUDGET"
    # NULL out-pointer is rejected before any device call
    lib.fsg_ctx_create.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    assert lib.fsg_ctx_create(0, None, 0, None) == -1
    # a NULL context is rejected by every call
    lib.fsg_ctx_sync.argtypes = [ctypes.c_void_p]
    assert lib.fsg_ctx_sync(None) == -1
    lib.fsg_degrees.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    assert lib.fsg_degrees(None, None, 1.0, None) == -1
    lib.fsg_last_error.restype = ctypes.c_char_p
    lib.fsg_last_error.argtypes = [ctypes.c_void_p]
    assert lib.fsg_last_error(None) == b""
    # the context settings, too
    for name in ("fsg_ctx_set_pruning", "fsg_ctx_set_exact_slices", "fsg_ctx_set_levels_per_pass"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        assert f(None, 1) == -1, name


def test_batch_and_graph_calls_validate_on_the_host():
    """The batching, autotuning and graph calls reject NULL handles without
    touching a device; destroying NULL is a no-op."""
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    lib.fsg_job_create.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.c_uint64, vp]
    assert lib.fsg_job_create(None, None, 1.0, 4, 1, None) == -1
    lib.fsg_batch_step.argtypes = [vp, vp, ctypes.c_int32, vp]
    assert lib.fsg_batch_step(None, None, 0, None) == -1
    for name in ("fsg_job_reset", "fsg_graph_begin"):
        f = getattr(lib, name)
        f.argtypes = [vp]
        assert f(None) == -1
    lib.fsg_job_result.argtypes = [vp, vp, vp]
    assert lib.fsg_job_result(None, None, None) == -1
    lib.fsg_graph_end.argtypes = [vp, vp]
    assert lib.fsg_graph_end(None, None) == -1
    lib.fsg_graph_launch.argtypes = [vp, vp]
    assert lib.fsg_graph_launch(None, None) == -1
    lib.fsg_ctx_set_autotune.argtypes = [vp, ctypes.c_int32]
    assert lib.fsg_ctx_set_autotune(None, 1) == -1
    for name in ("fsg_job_destroy", "fsg_graph_destroy"):
        f = getattr(lib, name)
        f.argtypes = [vp]
        f.restype = None
        f(None)


def test_no_gpu_reports_device_error():
    """Without a GPU, creating a context fails with FSG_E_DEVICE (never a crash)."""
    import torch
    if torch.cuda.is_available():
        return
    lib = ctypes.CDLL(LIB)
    h = ctypes.c_void_p()
    lib.fsg_ctx_create.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]
    assert lib.fsg_ctx_create(0, None, 0, ctypes.byref(h)) == -3


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workload_generators_are_deterministic():
    import workloads
    a = workloads.mixture(1000, 5, 3, 17, (-2, 2), (0.5, 1.0))
    b = workloads.mixture(1000, 5, 3, 17, (-2, 2), (0.5, 1.0))
    assert a.dtype == np.float32 and a.shape == (1000, 5)
    assert np.array_equal(a, b)
    w = workloads.mixture32()
    assert (w.n, w.d, w.L, w.sigma) == (100_000, 32, 17, 2.0) and w.gamma == 1 / 8
    assert workloads.depth_of(100_000) == 17 and workloads.depth_of(1000) == 10
    s = workloads.subsample(100, 10, 3)
    assert len(np.unique(s)) == 10 and s.min() >= 0 and s.max() < 100
