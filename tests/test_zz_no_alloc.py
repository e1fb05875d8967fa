"""The allocation-free entry point (gvm_plain_run_noalloc) against the plain
path it varies (gvm_plain_run), through the C-ABI.

The caller's device buffers come from the HIP runtime the library itself
uses (libamdhip64, loaded with it), through ctypes.  For every kernel id,
two calls in a row, the second with a smaller request, each compared byte
for byte with gvm_plain_run on the same input: the two run the same kernel
code objects, so the bytes must be identical (the EP-like tally keeps its
per-unit partial records in the static scratch, whose contents the first
call leaves behind).  An EP request larger than the scratch is refused
before anything is enqueued.
"""

import ctypes

import numpy as np
import pytest

from paper_1511_07658_amd import gvm as G
from paper_1511_07658_amd import spmd
from paper_1511_07658_amd import workloads as wl

pytestmark = pytest.mark.gpu

R32 = float(np.float32(wl.BS_RATE))
V32 = float(np.float32(wl.BS_VOLATILITY))
H2D, D2H = 1, 2


def hip():
    G.lib()  # loads the HIP runtime the library links
    h = ctypes.CDLL("libamdhip64.so.7")
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipFree.argtypes = [ctypes.c_void_p]
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    h.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    h.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    h.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    for f in ("hipMalloc", "hipFree", "hipMemcpy", "hipSetDevice", "hipDeviceSynchronize", "hipStreamCreate",
              "hipStreamSynchronize", "hipStreamDestroy"):
        getattr(h, f).restype = ctypes.c_int
    assert h.hipSetDevice(0) == 0
    return h


def run_noalloc(h, k, x, n, stream):
    nout = G.out_elems(k, n)
    d_in, d_out = ctypes.c_void_p(), ctypes.c_void_p()
    assert h.hipMalloc(ctypes.byref(d_in), x.nbytes) == 0
    assert h.hipMalloc(ctypes.byref(d_out), nout * 4) == 0
    try:
        assert h.hipMemcpy(d_in, x.ctypes.data, x.nbytes, H2D) == 0
        rc = G.gvm_plain_run_noalloc(k, d_in.value, d_out.value, n, R32, V32, stream)
        assert rc == 0, G.gvm_last_error()
        assert (h.hipStreamSynchronize(stream) if stream else h.hipDeviceSynchronize()) == 0
        out = np.empty(nout, np.float32)
        assert h.hipMemcpy(out.ctypes.data, d_out, nout * 4, D2H) == 0
        return out
    finally:
        h.hipFree(d_in)
        h.hipFree(d_out)


CASES = [
    (G.GVM_K_EP, 0, [3 * (1 << 15) + 5, (1 << 15) + 1]),
    (G.GVM_K_VECADD, 0, [(1 << 20) + 3, 4097]),
    (G.GVM_K_VECMUL, 0, [70001, 129]),
    (G.GVM_K_BLACKSCHOLES, 2, [300001, 1000]),
    (G.GVM_K_SGEMM, 1, [517, 96]),
]


@pytest.mark.parametrize("kernel_id,cfg,sizes", CASES)
def test_noalloc_equals_plain_run_twice(kernel_id, cfg, sizes):
    h = hip()
    stream = ctypes.c_void_p()
    assert h.hipStreamCreate(ctypes.byref(stream)) == 0
    try:
        for call, n in enumerate(sizes):
            print(f"noalloc kernel {kernel_id} n {n} call {call}", flush=True)
            x = spmd.make_input(kernel_id, cfg, call, n)
            want = np.empty(G.out_elems(kernel_id, n), np.float32)
            rc, _ = G.gvm_plain_run(kernel_id, x, want, n, R32, V32)
            assert rc == 0, G.gvm_last_error()
            got = run_noalloc(h, kernel_id, x, n, stream.value if call else None)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (kernel_id, n)
    finally:
        h.hipStreamDestroy(stream)


def test_noalloc_refuses_ep_beyond_scratch():
    h = hip()
    key = np.zeros(4, np.float32)
    d = ctypes.c_void_p()
    assert h.hipMalloc(ctypes.byref(d), 256) == 0
    try:
        assert h.hipMemcpy(d, key.ctypes.data, key.nbytes, H2D) == 0
        too_many = (1 << 20) // 96 * (1 << 15) + 1
        assert G.gvm_plain_run_noalloc(G.GVM_K_EP, d.value, d.value + 128, too_many, R32, V32, None) == G.GVM_ENOMEM
        assert "scratch" in G.gvm_last_error()
        assert G.gvm_plain_run_noalloc(G.GVM_K_VECADD, None, d.value, 16, R32, V32, None) == G.GVM_EINVAL
    finally:
        h.hipFree(d)
