"""Reference for the second workload family: a small compute-intensive
"EP-like" kernel (test infrastructure only; see package header).

The paper's compute-intensive benchmark is the NPB "embarrassingly parallel"
kernel EP at sizes M = 24 and M = 30 (Table 3; Section 6 uses EP(M24), grid
size 1, for the compute-intensive model validation and EP(M30), grid size
4, for the turnaround experiment).  Its character: every work item draws
pairs of uniform deviates, turns the accepted ones into Gaussian pairs and
reduces them to two sums and ten annulus counts; almost no input or output
bytes, all arithmetic.

Reading (listed with the others in the design notes): the NPB generator, its
seed and its published verification values are not reproduced.  The
uniform deviates come from the counter-based generator Philox4x64-10 of
Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as easy as 1, 2,
3", SC 2011), so that any GPU thread can start at any point of the stream;
the GPU implements the same generator from the same definition, and the
oracle is pinned to numpy's Philox bit generator.

Definition of one request (key k = (k0, k1), n pairs):

* block b = 0, 1, ... : (w0, w1, w2, w3) = Philox4x64-10(counter (b, 0, 0, 0), key k);
  pair 2b takes (w0, w1), pair 2b + 1 takes (w2, w3); pairs j < n are used;
* u(w) = (w >> 11) * 2^-53 in [0, 1);  x = 2 u(w_even) - 1, y = 2 u(w_odd) - 1
  (exact in binary64);
* t = x*x + y*y, each operation rounded to binary64 (no fused multiply-add);
  the pair is accepted when 0 < t <= 1 (Marsaglia's polar method);
* f = sqrt(-2 ln t / t);  X = x f,  Y = y f (a pair of independent standard
  normal deviates);
* outputs: sx = sum X, sy = sum Y over the accepted pairs, and q[l] = the
  number of accepted pairs with l <= max(|X|, |Y|) < l + 1, l = 0..9.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "PHILOX_M",
    "PHILOX_W",
    "philox4x64_10_scalar",
    "philox4x64_10",
    "ep_words",
    "ep_uniform_pairs",
    "ep_polar",
    "ep_reference",
    "EP_ANNULI",
]

# Multipliers and Weyl key increments of Philox4x64 (Salmon et al., 2011).
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
EP_ANNULI = 10
_MASK64 = (1 << 64) - 1


def philox4x64_10_scalar(counter, key):
    """Philox4x64 with 10 rounds on Python integers: each round multiplies
    words 0 and 2 by the two multipliers (full 128-bit products), and the
    next counter is (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
    lo(M0 c0)); the key is bumped by the Weyl increments between rounds."""
    c0, c1, c2, c3 = (int(v) & _MASK64 for v in counter)
    k0, k1 = (int(v) & _MASK64 for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W[0]) & _MASK64
            k1 = (k1 + PHILOX_W[1]) & _MASK64
        p0 = PHILOX_M[0] * c0
        p1 = PHILOX_M[1] * c2
        hi0, lo0 = p0 >> 64, p0 & _MASK64
        hi1, lo1 = p1 >> 64, p1 & _MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _mulhilo64(a: int, b: np.ndarray):
    """(hi, lo) 64-bit halves of the 128-bit products a * b, b uint64 array,
    from 32-bit partial products (schoolbook)."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = np.uint64(a & 0xFFFFFFFF), np.uint64(a >> 32)
    b_lo, b_hi = b & m32, b >> s32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)          # < 3 * 2^32, no overflow
    lo = (ll & m32) | ((mid & m32) << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox4x64_10(counters: np.ndarray, key) -> np.ndarray:
    """Vectorised Philox4x64-10: counters (m, 4) uint64 -> (m, 4) uint64."""
    c = np.asarray(counters, dtype=np.uint64)
    c0, c1, c2, c3 = c[:, 0].copy(), c[:, 1].copy(), c[:, 2].copy(), c[:, 3].copy()
    k0, k1 = int(key[0]) & _MASK64, int(key[1]) & _MASK64
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd:
                k0 = (k0 + PHILOX_W[0]) & _MASK64
                k1 = (k1 + PHILOX_W[1]) & _MASK64
            hi0, lo0 = _mulhilo64(PHILOX_M[0], c0)
            hi1, lo1 = _mulhilo64(PHILOX_M[1], c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return np.stack([c0, c1, c2, c3], axis=1)


def ep_words(key, n: int) -> np.ndarray:
    """The 2n generator words of the n pairs: pair j -> words (2j, 2j + 1)."""
    if n < 0:
        raise ValueError("n must be >= 0")
    blocks = (n + 1) // 2
    ctr = np.zeros((blocks, 4), np.uint64)
    ctr[:, 0] = np.arange(blocks, dtype=np.uint64)
    return philox4x64_10(ctr, key).reshape(-1)[: 2 * n]


def ep_uniform_pairs(key, n: int):
    """x, y in [-1, 1) of the n pairs (binary64, exact)."""
    w = ep_words(key, n)
    u = (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    x = 2.0 * u[0::2] - 1.0
    y = 2.0 * u[1::2] - 1.0
    return x, y


def ep_polar(x: np.ndarray, y: np.ndarray):
    """Marsaglia's polar method: accepted mask and the Gaussian pairs (X, Y)
    of the accepted (x, y)."""
    t = x * x + y * y      # numpy: two rounded products and a rounded sum
    acc = (t > 0.0) & (t <= 1.0)
    ta = t[acc]
    f = np.sqrt(-2.0 * np.log(ta) / ta)
    return acc, x[acc] * f, y[acc] * f


def ep_reference(key, n: int) -> dict:
    """Outputs of one request: sx, sy (exactly rounded sums, math.fsum), the
    ten annulus counts q, the accepted count, and sum |X|, sum |Y| (for the
    tolerance of the sums)."""
    x, y = ep_uniform_pairs(key, n)
    acc, X, Y = ep_polar(x, y)
    m = np.maximum(np.abs(X), np.abs(Y))
    q = np.zeros(EP_ANNULI, np.int64)
    lvl = np.floor(m).astype(np.int64)
    inside = lvl < EP_ANNULI
    np.add.at(q, lvl[inside], 1)
    return {
        "sx": math.fsum(X.tolist()),
        "sy": math.fsum(Y.tolist()),
        "q": q,
        "accepted": int(acc.sum()),
        "abs_x": float(np.abs(X).sum()),
        "abs_y": float(np.abs(Y).sum()),
    }
