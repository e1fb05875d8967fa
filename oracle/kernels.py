"""Reference per-rank kernels (test infrastructure only; see package header).

The paper's benchmark profiles (Table 3, Section 6) name the per-rank GPU
tasks that SPMD processes hand to the virtualization manager: vector
addition (I/O-intensive), vector multiplication (I/O-intensive, used for the
model validation of Section 6), single-precision matrix multiplication
("intermediate" class) and Black-Scholes European option pricing
(I/O-intensive; the paper cites Black and Scholes 1973 and prints no
formula).  Each function below is the plain definition of one of them.

Precision
---------
* vector add / multiply: the definition fixes IEEE-754 binary32 with
  round-to-nearest-even (the paper says "Float"), so the oracle computes in
  binary32 and the GPU must match bit for bit.
* matrix multiply and Black-Scholes: computed in float64 from the binary32
  inputs; the GPU's binary32 result is compared under a tolerance.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc as _erfc64

__all__ = [
    "vecadd_f32",
    "vecmul_f32",
    "norm_cdf_f64",
    "black_scholes_f64",
    "sgemm_f64",
    "sgemm_bruteforce",
]


def _as_f32(x) -> np.ndarray:
    a = np.asarray(x)
    if a.dtype != np.float32:
        raise TypeError(f"expected float32 input, got {a.dtype}")
    return a


def vecadd_f32(a, b) -> np.ndarray:
    """Vector addition of Table 3: ``c[i] = fl32(a[i] + b[i])``.

    One correctly rounded binary32 addition per element (round to nearest,
    ties to even), denormals kept.  numpy's float32 add on x86-64 is SSE
    scalar/vector IEEE addition, so it *is* the definition.
    """
    a = _as_f32(a)
    b = _as_f32(b)
    if a.shape != b.shape:
        raise ValueError("a and b must have the same shape")
    with np.errstate(over="ignore", invalid="ignore"):
        return np.add(a, b, dtype=np.float32)


def vecmul_f32(a, b, iters: int = 1) -> np.ndarray:
    """Vector multiplication of Table 3 (16M floats, 15 iterations).

    Reading: each iteration multiplies the running vector element-wise by
    ``b`` in binary32, ``x <- fl32(x * b)`` starting from ``x = a``; one
    iteration is ``fl32(a[i] * b[i])``.
    """
    a = _as_f32(a)
    b = _as_f32(b)
    if a.shape != b.shape:
        raise ValueError("a and b must have the same shape")
    if iters < 1:
        raise ValueError("iters must be >= 1")
    x = a.copy()
    with np.errstate(over="ignore", under="ignore", invalid="ignore"):
        for _ in range(iters):
            x = np.multiply(x, b, dtype=np.float32)
    return x


def norm_cdf_f64(x) -> np.ndarray:
    """Standard normal cumulative distribution ``N(x) = erfc(-x/sqrt(2)) / 2``
    in float64 (the complementary error function form keeps full relative
    accuracy in the lower tail)."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * _erfc64(-x / math.sqrt(2.0))


def black_scholes_f64(S, K, T, r: float, sigma: float):
    """European call and put prices without dividends (Black and Scholes 1973,
    the pricing model behind the BlackScholes benchmark of Table 3).

        d1   = (ln(S/K) + (r + sigma^2/2) T) / (sigma sqrt(T))
        d2   = d1 - sigma sqrt(T)
        call = S N(d1) - K exp(-r T) N(d2)
        put  = K exp(-r T) N(-d2) - S N(-d1)

    ``S``, ``K``, ``T`` are binary32 arrays (spot, strike, years to expiry);
    ``r`` (risk-free rate) and ``sigma`` (volatility) are scalars shared by
    every option of a request.  All arithmetic is float64.  Where
    ``sigma sqrt(T) == 0`` the price is its limit, the discounted intrinsic
    value.  Returns ``(call, put)`` as float64 arrays.
    """
    S = np.asarray(_as_f32(S), dtype=np.float64)
    K = np.asarray(_as_f32(K), dtype=np.float64)
    T = np.asarray(_as_f32(T), dtype=np.float64)
    if not (S.shape == K.shape == T.shape):
        raise ValueError("S, K, T must have the same shape")
    r = float(r)
    sigma = float(sigma)
    vol = sigma * np.sqrt(T)
    disc_k = K * np.exp(-r * T)
    with np.errstate(divide="ignore", invalid="ignore"):
        d1 = (np.log(S / K) + (r + 0.5 * sigma * sigma) * T) / vol
        d2 = d1 - vol
        call = S * norm_cdf_f64(d1) - disc_k * norm_cdf_f64(d2)
        put = disc_k * norm_cdf_f64(-d2) - S * norm_cdf_f64(-d1)
    degenerate = vol == 0.0
    if np.any(degenerate):
        call = np.where(degenerate, np.maximum(S - disc_k, 0.0), call)
        put = np.where(degenerate, np.maximum(disc_k - S, 0.0), put)
    return call, put


def sgemm_f64(A, B) -> np.ndarray:
    """Single-precision matrix multiplication of Table 3, reference value.

    ``C = A B`` for row-major binary32 ``A`` (m x k) and ``B`` (k x n), no
    scaling factors and no transposes; accumulated in float64 (a library
    float64 matmul serves as the contraction step).
    """
    A = _as_f32(A)
    B = _as_f32(B)
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("A must be m x k and B k x n")
    return A.astype(np.float64) @ B.astype(np.float64)


def sgemm_bruteforce(A, B):
    """``C[i][j] = sum_k A[i][k] B[k][j]`` as three nested Python loops over
    Python floats (float64).  For tiny inputs only."""
    A = _as_f32(A)
    B = _as_f32(B)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    C = [[0.0] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            s = 0.0
            for p in range(k):
                s += float(A[i, p]) * float(B[p, j])
            C[i][j] = s
    return np.array(C, dtype=np.float64)
