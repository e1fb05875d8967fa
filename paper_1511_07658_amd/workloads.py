"""Seeded synthetic inputs shared by the tests, the smoke run and the bench.

This module holds no arithmetic of the method: it only draws random inputs of
the shapes, sizes and distributions of the workloads, so that the oracle and
the GPU path can be fed identical bytes.  Every stream of random numbers is
``numpy.random.Generator(PCG64(SeedSequence([1511, config, rank, request])))``.

Workloads (stand-ins for the benchmark profiles of Table 3; the paper's own
datasets and benchmark programs are not used):

* vector add: ``a, b ~ U[-1, 1]`` binary32;
* Black-Scholes: spot ``S ~ U[5, 30]``, strike ``K ~ U[1, 100]``, expiry
  ``T ~ U[0.25, 10]`` years, binary32, with rate 0.02 and volatility 0.30;
* matrix multiply: square ``A, B ~ N(0, 1)`` binary32, row-major;
  ``sgemm_int_inputs`` draws small integers instead, for which every partial
  sum is exactly representable in binary32.
"""

from __future__ import annotations

import math

import numpy as np

SEED_ROOT = 1511

BS_RATE = 0.02
BS_VOLATILITY = 0.30

# Request layouts of the C-ABI (in / out element counts for a request size n).
KERNEL_VECADD = 1
KERNEL_BLACKSCHOLES = 2
KERNEL_SGEMM = 3
KERNEL_EP = 5


def generator(config: int, rank: int, request: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, config, rank, request])))


def vecadd_inputs(config: int, rank: int, n: int, request: int = 0):
    g = generator(config, rank, request)
    a = g.uniform(-1.0, 1.0, n).astype(np.float32)
    b = g.uniform(-1.0, 1.0, n).astype(np.float32)
    return a, b


def bs_inputs(config: int, rank: int, n: int, request: int = 0):
    g = generator(config, rank, request)
    S = g.uniform(5.0, 30.0, n).astype(np.float32)
    K = g.uniform(1.0, 100.0, n).astype(np.float32)
    T = g.uniform(0.25, 10.0, n).astype(np.float32)
    return S, K, T


def sgemm_inputs(config: int, rank: int, n: int, request: int = 0):
    g = generator(config, rank, request)
    A = g.standard_normal((n, n), dtype=np.float32)
    B = g.standard_normal((n, n), dtype=np.float32)
    return A, B


def sgemm_int_inputs(config: int, rank: int, n: int, request: int = 0, lo: int = -8, hi: int = 8):
    g = generator(config, rank, request)
    A = g.integers(lo, hi + 1, (n, n)).astype(np.float32)
    B = g.integers(lo, hi + 1, (n, n)).astype(np.float32)
    return A, B


def ep_key(config: int, rank: int, request: int = 0) -> np.ndarray:
    """The 128-bit generator key (k0, k1) of one EP-like request."""
    return generator(config, rank, request).integers(0, 2**64, size=2, dtype=np.uint64)


def ep_request(key) -> np.ndarray:
    """The packed input of an EP-like request: the two key words, viewed as
    the four 32-bit elements the C-ABI transports."""
    return np.ascontiguousarray(np.asarray(key, dtype=np.uint64)).view(np.float32)


def ep_result(out) -> dict:
    """Decode an EP-like output (24 32-bit elements): sx, sy and q[0..9]."""
    w = np.ascontiguousarray(out).view(np.uint64)
    return {"sx": float(w[:1].view(np.float64)[0]), "sy": float(w[1:2].view(np.float64)[0]),
            "q": w[2:12].astype(np.int64)}


def edge_floats():
    """Binary32 operands at the edges of the format: signed zeros, the
    smallest normal and subnormals, values one ulp and half an ulp from 1,
    the largest finite value, 2**24 and its neighbour, and a few ordinary
    numbers."""
    vals = [0.0, -0.0, 1.0, -1.0, 1.5, 2.0 ** -126, 2.0 ** -149, -(2.0 ** -149), 3 * 2.0 ** -149,
            1.0 + 2.0 ** -23, 1.0 - 2.0 ** -24, 3.4028234663852886e38, 2.0 ** 24, 2.0 ** 24 + 2.0,
            0.1, 1e-30, 5e-39]
    return [float(np.float32(v)) for v in vals]


def edge_pairs():
    """Every ordered pair of edge_floats (plus their negations), then the
    infinities and NaN against each other and against 1 and the largest
    finite value, and rounding ties: operand arrays (a, b) in binary32."""
    e = edge_floats()
    e = e + [-x for x in e if x != 0.0]
    a = [x for x in e for _ in e]
    b = [y for _ in e for y in e]
    special = [math.inf, -math.inf, math.nan, 1.0, 3.4028234663852886e38, -3.4028234663852886e38]
    a += [x for x in special for _ in special]
    b += [y for _ in special for y in special]
    # ties: halfway between two binary32 values, both parities of the lower one
    for m in range(1, 64):
        x = 1.0 + m * 2.0 ** -23
        a += [x, -x, x * 2.0 ** -120]
        b += [2.0 ** -24, -(2.0 ** -24), 2.0 ** -144]
    return np.array(a, dtype=np.float32), np.array(b, dtype=np.float32)


def pack_request(kernel_id: int, *arrays) -> np.ndarray:
    """Concatenate the input arrays of one request into the packed binary32
    layout the C-ABI expects (``[a|b]``, ``[S|K|T]`` or ``[A|B]``)."""
    return np.ascontiguousarray(np.concatenate([np.ravel(x) for x in arrays]).astype(np.float32, copy=False))


def in_elems(kernel_id: int, n: int) -> int:
    if kernel_id == KERNEL_VECADD:
        return 2 * n
    if kernel_id == KERNEL_BLACKSCHOLES:
        return 3 * n
    if kernel_id == KERNEL_SGEMM:
        return 2 * n * n
    if kernel_id == KERNEL_EP:
        return 4
    raise ValueError(f"unknown kernel id {kernel_id}")


def out_elems(kernel_id: int, n: int) -> int:
    if kernel_id == KERNEL_VECADD:
        return n
    if kernel_id == KERNEL_BLACKSCHOLES:
        return 2 * n
    if kernel_id == KERNEL_SGEMM:
        return n * n
    if kernel_id == KERNEL_EP:
        return 24
    raise ValueError(f"unknown kernel id {kernel_id}")


# ---- uneven sizes and arrival traces of the mixed and serving workloads ----

def uneven_vecadd_sizes(config: int, count: int, lo_log2: float = 16.0, hi_log2: float = 24.0):
    """Vector lengths ``floor(2**U[lo, hi])``."""
    g = generator(config, 10_000)
    return [int(math.floor(2.0 ** g.uniform(lo_log2, hi_log2))) for _ in range(count)]


def uneven_sgemm_sizes(config: int, count: int, lo: int = 256, hi: int = 2048, step: int = 64):
    """Square sizes uniform over the multiples of ``step`` in ``[lo, hi]``."""
    g = generator(config, 10_001)
    choices = list(range(lo, hi + 1, step))
    return [int(choices[i]) for i in g.integers(0, len(choices), count)]


def poisson_trace(config: int, nranks: int, total_rate: float, duration_s: float,
                  vec_log2=(16.0, 24.0), bs_log2=(16.0, 22.0), gemm=(256, 2048, 64)):
    """Open-loop arrivals: each rank draws exponential inter-arrival times at
    ``total_rate / nranks`` requests per second; every request picks one of
    the three kernels uniformly and a size from that kernel's range.
    Returns, per rank, a list of ``(t_arrival_s, kernel_id, n)``."""
    per_rank = total_rate / nranks
    traces = []
    for r in range(nranks):
        g = generator(config, 20_000 + r)
        t = 0.0
        reqs = []
        while True:
            t += g.exponential(1.0 / per_rank)
            if t >= duration_s:
                break
            k = int(g.integers(1, 4))
            if k == KERNEL_VECADD:
                n = int(math.floor(2.0 ** g.uniform(*vec_log2)))
            elif k == KERNEL_BLACKSCHOLES:
                n = int(math.floor(2.0 ** g.uniform(*bs_log2)))
            else:
                lo, hi, step = gemm
                n = int(lo + step * g.integers(0, (hi - lo) // step + 1))
            reqs.append((t, k, n))
        traces.append(reqs)
    return traces
