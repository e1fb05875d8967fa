"""ctypes access to the plain C restatement of the oracle, oracle/c/oracle.c
(test infrastructure only; see package header).  The shared library
oracle/liboracle.so is built by the repository's build step (gcc, no
fast-math, no contraction); ``compile_to`` builds a private copy for tests.

Every function here is a thin marshalling wrapper; the definitions, with
their citations, are in oracle.c."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "c", "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

_libs = {}


def compile_to(path):
    """Build oracle.c into `path` with the repository's flags."""
    subprocess.run(["gcc", *CFLAGS, SOURCE, "-o", path, "-lm"], check=True)
    return path


def load(path=LIB):
    if path not in _libs:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run the build step (__graft_entry__.build())")
        L = ctypes.CDLL(path)
        f32p, f64p, u64, d = (ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double), ctypes.c_uint64,
                              ctypes.c_double)
        L.ref_vecadd_f32.argtypes = [f32p, f32p, f32p, u64]
        L.ref_vecmul_f32.argtypes = [f32p, f32p, f32p, u64, ctypes.c_int]
        L.ref_bs_f64.argtypes = [f32p, f32p, f32p, d, d, f64p, f64p, u64]
        L.ref_sgemm_f64.argtypes = [f32p, f32p, f64p, u64]
        L.ref_sgemm_rows_f64.argtypes = [f32p, f32p, f64p, u64, u64, u64]
        for name in ("ref_vecadd_f32", "ref_vecmul_f32", "ref_bs_f64", "ref_sgemm_f64", "ref_sgemm_rows_f64"):
            getattr(L, name).restype = None
        for k in (1, 8, 9):
            getattr(L, f"model_eq{k}").argtypes = [d] * 6
        for k in (2, 3, 4, 5, 6, 7):
            getattr(L, f"model_eq{k}").argtypes = [d] * 4
        for k in (10, 11):
            getattr(L, f"model_eq{k}").argtypes = [d] * 5
        for k in range(1, 12):
            getattr(L, f"model_eq{k}").restype = d
        L.des_simulate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d, d]
        L.des_simulate.restype = d
        _libs[path] = L
    return _libs[path]


def _f32(x):
    x = np.ascontiguousarray(x)
    if x.dtype != np.float32:
        raise TypeError(f"expected float32, got {x.dtype}")
    return x


def _p(x, t):
    return x.ctypes.data_as(ctypes.POINTER(t))


def vecadd_f32(a, b, lib=None):
    a, b = _f32(a), _f32(b)
    c = np.empty_like(a)
    (lib or load()).ref_vecadd_f32(_p(a, ctypes.c_float), _p(b, ctypes.c_float), _p(c, ctypes.c_float), a.size)
    return c


def vecmul_f32(a, b, iters=1, lib=None):
    a, b = _f32(a), _f32(b)
    c = np.empty_like(a)
    (lib or load()).ref_vecmul_f32(_p(a, ctypes.c_float), _p(b, ctypes.c_float), _p(c, ctypes.c_float), a.size,
                                   int(iters))
    return c


def black_scholes_f64(S, K, T, r, sigma, lib=None):
    S, K, T = _f32(S), _f32(K), _f32(T)
    call = np.empty(S.size, np.float64)
    put = np.empty(S.size, np.float64)
    (lib or load()).ref_bs_f64(_p(S, ctypes.c_float), _p(K, ctypes.c_float), _p(T, ctypes.c_float), float(r),
                               float(sigma), _p(call, ctypes.c_double), _p(put, ctypes.c_double), S.size)
    return call, put


def sgemm_f64(A, B, lib=None):
    A, B = _f32(A), _f32(B)
    n = A.shape[0]
    C = np.empty((n, n), np.float64)
    (lib or load()).ref_sgemm_f64(_p(A, ctypes.c_float), _p(B, ctypes.c_float), _p(C, ctypes.c_double), n)
    return C


def sgemm_rows_f64(A, B, row0, rows, lib=None):
    """Rows [row0, row0 + rows) of A B (float64), as a rows x n array."""
    A, B = _f32(A), _f32(B)
    n = A.shape[0]
    rows = max(0, min(rows, n - row0))
    C = np.empty((rows, n), np.float64)
    (lib or load()).ref_sgemm_rows_f64(_p(A, ctypes.c_float), _p(B, ctypes.c_float), _p(C, ctypes.c_double), n,
                                       row0, rows)
    return C


def eq(k, *args, lib=None):
    return getattr(lib or load(), f"model_eq{k}")(*[float(a) for a in args])


def des_simulate(style, n, t_in, t_comp, t_out, rules="paper", lib=None):
    s = {"PS1": 1, "PS2": 2}[style]
    r = {"paper": 0, "multiqueue": 1}[rules]
    return (lib or load()).des_simulate(s, r, int(n), float(t_in), float(t_comp), float(t_out))
