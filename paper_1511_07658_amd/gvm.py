"""ctypes binding of libgvm.so with the names of the C-ABI (include/gvm.h).

Argument marshalling only: every step of the path runs in the native
library.  Functions return the C status codes unchanged (0 = GVM_OK,
negative = error); ``gvm_last_error()`` gives the text.  Buffers may be
numpy arrays (C-contiguous), raw addresses (int) or None.

The library is loaded on first use; if ``libgvm.so`` has not been built the
import of a function fails loudly (there is no fallback of any kind).
"""

from __future__ import annotations

import ctypes
import json
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgvm.so")

# status codes
GVM_OK = 0
GVM_EINVAL = -1
GVM_ENOMEM = -2
GVM_EAGAIN = -3
GVM_ETIMEDOUT = -4
GVM_EDEAD = -5
GVM_ESTATE = -6
GVM_EDEVICE = -7
GVM_ESYS = -8
GVM_ECANCELED = -9

# kernel ids
GVM_K_VECADD = 1
GVM_K_BLACKSCHOLES = 2
GVM_K_SGEMM = 3
GVM_K_VECMUL = 4
GVM_K_EP = 5

GVM_MODE_BATCH = 0
GVM_MODE_SERVING = 1

GVM_POLICY_AUTO = 0
GVM_POLICY_PS1 = 1
GVM_POLICY_PS2 = 2
GVM_POLICY_GROUPED = 3

GVM_BACKEND_HIP = 0
GVM_BACKEND_LOOPBACK = 1

GVM_F_IN_RESIDENT = 1
GVM_F_OUT_RESIDENT = 2
GVM_F_NONBLOCK = 4

GVM_NAME_MAX = 48


class gvm_config(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32),
        ("nranks", ctypes.c_uint32),
        ("shm_bytes_per_rank", ctypes.c_uint64),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("staging_bytes", ctypes.c_uint64),
        ("mode", ctypes.c_uint32),
        ("policy", ctypes.c_uint32),
        ("batch_window_us", ctypes.c_uint32),
        ("max_inflight", ctypes.c_uint32),
        ("nstreams", ctypes.c_uint32),
        ("use_graphs", ctypes.c_uint32),
        ("backend", ctypes.c_uint32),
        ("copy_threads", ctypes.c_uint32),
        ("bs_rate", ctypes.c_float),
        ("bs_volatility", ctypes.c_float),
        ("batch_timing", ctypes.c_uint32),
        ("latency_cus", ctypes.c_uint32),
        ("small_request_bytes", ctypes.c_uint32),
        ("early_copy_in", ctypes.c_uint32),
        ("name", ctypes.c_char * GVM_NAME_MAX),
    ]


_lib = None


def lib():
    """The loaded libgvm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1511_07658_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        u32, u64, i32, i64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        L.gvm_config_default.argtypes = [ctypes.POINTER(gvm_config)]
        L.gvm_config_default.restype = None
        L.gvm_init.argtypes = [ctypes.POINTER(gvm_config)]
        L.gvm_init.restype = i32
        L.gvm_cu_partition_masks.argtypes = [u32, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]
        L.gvm_cu_partition_masks.restype = i32
        L.gvm_attach.argtypes = [i32]
        L.gvm_attach.restype = i32
        L.gvm_attach_ns.argtypes = [ctypes.c_char_p, i32]
        L.gvm_attach_ns.restype = i32
        L.gvm_submit.argtypes = [i32, i32, vp, vp, u64]
        L.gvm_submit.restype = i64
        L.gvm_submit_ex.argtypes = [i32, i32, vp, vp, u64, u32]
        L.gvm_submit_ex.restype = i64
        L.gvm_wait.argtypes = [i32, i64, i64]
        L.gvm_wait.restype = i32
        L.gvm_wait_timed.argtypes = [i32, i64, i64, ctypes.POINTER(ctypes.c_uint64)]
        L.gvm_wait_timed.restype = i32
        L.gvm_wait_any.argtypes = [i32, i64, ctypes.POINTER(i64)]
        L.gvm_wait_any.restype = i32
        L.gvm_wait_any_timed.argtypes = [i32, i64, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_uint64)]
        L.gvm_wait_any_timed.restype = i32
        L.gvm_detach.argtypes = [i32]
        L.gvm_detach.restype = i32
        L.gvm_shutdown.argtypes = []
        L.gvm_shutdown.restype = i32
        L.gvm_rank_buffer.argtypes = [i32, u64]
        L.gvm_rank_buffer.restype = vp
        L.gvm_stats_json.argtypes = [ctypes.c_char_p, u64]
        L.gvm_stats_json.restype = i32
        L.gvm_stats_reset.argtypes = []
        L.gvm_stats_reset.restype = i32
        L.gvm_trace_dump.argtypes = [ctypes.c_char_p]
        L.gvm_trace_dump.restype = i32
        L.gvm_last_error.argtypes = []
        L.gvm_last_error.restype = ctypes.c_char_p
        L.gvm_plain_run.argtypes = [i32, vp, vp, u64, ctypes.c_float, ctypes.c_float, ctypes.POINTER(ctypes.c_double)]
        L.gvm_plain_run.restype = i32
        L.gvm_plain_run_noalloc.argtypes = [i32, vp, vp, u64, ctypes.c_float, ctypes.c_float, vp]
        L.gvm_plain_run_noalloc.restype = i32
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("buffer must be C-contiguous")
        return x.ctypes.data
    raise TypeError(f"unsupported buffer type {type(x)}")


def gvm_config_default(**overrides) -> gvm_config:
    cfg = gvm_config()
    lib().gvm_config_default(ctypes.byref(cfg))
    for k, v in overrides.items():
        if k == "name":
            v = v.encode() if isinstance(v, str) else v
        setattr(cfg, k, v)
    return cfg


def gvm_cu_partition_masks(latency_cus: int):
    """(latency mask, bulk mask) as two lists of 8 uint32 words, or raises."""
    lat = (ctypes.c_uint32 * 8)()
    bulk = (ctypes.c_uint32 * 8)()
    check(lib().gvm_cu_partition_masks(latency_cus, lat, bulk), "gvm_cu_partition_masks")
    return list(lat), list(bulk)


def gvm_init(cfg: gvm_config) -> int:
    return lib().gvm_init(ctypes.byref(cfg))


def gvm_attach(rank: int) -> int:
    return lib().gvm_attach(rank)


def gvm_attach_ns(name, rank: int) -> int:
    return lib().gvm_attach_ns(name.encode() if isinstance(name, str) else name, rank)


def gvm_submit(rank, kernel_id, in_buf, out_buf, n) -> int:
    return lib().gvm_submit(rank, kernel_id, _ptr(in_buf), _ptr(out_buf), n)


def gvm_submit_ex(rank, kernel_id, in_buf, out_buf, n, flags) -> int:
    return lib().gvm_submit_ex(rank, kernel_id, _ptr(in_buf), _ptr(out_buf), n, flags)


def gvm_wait(rank, ticket=-1, timeout_ns=-1) -> int:
    return lib().gvm_wait(rank, ticket, timeout_ns)


def gvm_wait_timed(rank, ticket, timeout_ns=-1):
    """Returns (status, [t_submit, t_admit, t_launch, t_device, t_done]) in ns."""
    ts = (ctypes.c_uint64 * 5)()
    rc = lib().gvm_wait_timed(rank, ticket, timeout_ns, ts)
    return rc, list(ts)


def gvm_wait_any(rank, timeout_ns=-1):
    t = ctypes.c_int64(-1)
    rc = lib().gvm_wait_any(rank, timeout_ns, ctypes.byref(t))
    return rc, t.value


def gvm_wait_any_timed(rank, timeout_ns=-1):
    """Returns (status, ticket, [t_submit, t_admit, t_launch, t_device, t_done])."""
    t = ctypes.c_int64(-1)
    ts = (ctypes.c_uint64 * 5)()
    rc = lib().gvm_wait_any_timed(rank, timeout_ns, ctypes.byref(t), ts)
    return rc, t.value, list(ts)


def gvm_detach(rank) -> int:
    return lib().gvm_detach(rank)


def gvm_shutdown() -> int:
    return lib().gvm_shutdown()


def gvm_rank_buffer(rank, nbytes, dtype=np.float32):
    """numpy view of the first ``nbytes`` of the rank's shared-memory space
    (zero-copy submission), or None."""
    p = lib().gvm_rank_buffer(rank, nbytes)
    if not p:
        return None
    count = nbytes // np.dtype(dtype).itemsize
    buf = (ctypes.c_char * nbytes).from_address(p)
    return np.frombuffer(buf, dtype=dtype, count=count)


def gvm_stats_json():
    cap = 1 << 16
    buf = ctypes.create_string_buffer(cap)
    rc = lib().gvm_stats_json(buf, cap)
    if rc < 0:
        return None
    return json.loads(buf.value.decode())


def gvm_stats_reset() -> int:
    return lib().gvm_stats_reset()


def gvm_last_error() -> str:
    s = lib().gvm_last_error()
    return s.decode() if s else ""


def gvm_plain_run(kernel_id, in_buf, out_buf, n, bs_rate=0.02, bs_volatility=0.30):
    t = (ctypes.c_double * 6)()
    rc = lib().gvm_plain_run(kernel_id, _ptr(in_buf), _ptr(out_buf), n, bs_rate, bs_volatility, t)
    return rc, list(t)


def gvm_plain_run_noalloc(kernel_id, d_in, d_out, n, bs_rate=0.02, bs_volatility=0.30, stream=None):
    """d_in, d_out: device addresses (int); stream: a hipStream_t as int, or None."""
    return lib().gvm_plain_run_noalloc(kernel_id, d_in, d_out, n, bs_rate, bs_volatility, stream)


def gvm_trace_dump(path) -> int:
    return lib().gvm_trace_dump(path.encode() if isinstance(path, str) else path)


class GvmError(RuntimeError):
    pass


def check(rc, what="gvm call"):
    """Raise GvmError with the library's error text if ``rc`` is negative."""
    if rc < 0:
        raise GvmError(f"{what} failed with status {rc}: {gvm_last_error()}")
    return rc


def in_elems(kernel_id, n):
    """32-bit elements of a request's input (EP: the two 64-bit key words)."""
    return {GVM_K_VECADD: 2 * n, GVM_K_VECMUL: 2 * n, GVM_K_BLACKSCHOLES: 3 * n, GVM_K_SGEMM: 2 * n * n,
            GVM_K_EP: 4}[kernel_id]


def out_elems(kernel_id, n):
    """32-bit elements of a request's output (EP: twelve 64-bit words)."""
    return {GVM_K_VECADD: n, GVM_K_VECMUL: n, GVM_K_BLACKSCHOLES: 2 * n, GVM_K_SGEMM: n * n,
            GVM_K_EP: 24}[kernel_id]


def header_symbols(header_path=None):
    """Names of the functions include/gvm.h declares (for the export check)."""
    import re

    if header_path is None:
        header_path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gvm.h")
    with open(header_path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gvm_[a-z_]+)\s*\(", text)))
