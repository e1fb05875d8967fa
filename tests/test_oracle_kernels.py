"""Pins of the per-rank reference kernels (oracle.kernels) to things other
than themselves: exact rational arithmetic, textbook values, closed forms,
a risk-neutral quadrature and brute-force loops."""

import json
import math
import os
import struct
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

from oracle import kernels as ok
from paper_1511_07658_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- vector add

def _round_to_binary32(x: Fraction) -> float:
    """Round an exact rational to the nearest binary32 value (ties to even),
    written out from the IEEE-754 definition: no float arithmetic involved."""
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    ax = -x if x < 0 else x
    e = ax.numerator.bit_length() - ax.denominator.bit_length()
    # adjust so that 2**e <= ax < 2**(e+1)
    while Fraction(2) ** e > ax:
        e -= 1
    while Fraction(2) ** (e + 1) <= ax:
        e += 1
    e = max(e, -126)                      # subnormal range shares the ulp of 2**-126
    ulp = Fraction(2) ** (e - 23)
    q = ax / ulp
    fl = q.numerator // q.denominator
    rem = q - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    val = fl * ulp
    if val >= Fraction(2) ** 128:
        return sign * math.inf
    return sign * float(val)


def _bits(x) -> int:
    return struct.unpack("<I", struct.pack("<f", x))[0]


def _edge_floats():
    return wl.edge_floats()


def test_vecadd_matches_exact_rounding_random():
    g = np.random.default_rng(7)
    a = g.uniform(-1, 1, 3000).astype(np.float32)
    b = g.uniform(-1, 1, 3000).astype(np.float32)
    b[:500] = (a[:500] * -0.999).astype(np.float32)          # heavy cancellation
    b[500:1000] = (b[500:1000] * 2.0 ** -30).astype(np.float32)  # large exponent gaps
    c = ok.vecadd_f32(a, b)
    for x, y, z in zip(a, b, c):
        want = _round_to_binary32(Fraction(float(x)) + Fraction(float(y)))
        assert _bits(float(z)) == _bits(want), (x, y, z, want)


def test_vecadd_edge_values_and_ties():
    e = _edge_floats()
    a = np.array([x for x in e for _ in e], dtype=np.float32)
    b = np.array([y for _ in e for y in e], dtype=np.float32)
    c = ok.vecadd_f32(a, b)
    for x, y, z in zip(a, b, c):
        want = _round_to_binary32(Fraction(float(x)) + Fraction(float(y)))
        if want == 0.0:
            # exact zero sum: +0 unless both operands are -0 (IEEE sign rule)
            want_bits = _bits(-0.0) if (_bits(float(x)) == _bits(-0.0) and _bits(float(y)) == _bits(-0.0)) else 0
            assert _bits(float(z)) == want_bits
        else:
            assert _bits(float(z)) == _bits(want), (x, y, z, want)
    # a tie that must round to even: 1 + 2**-24 lies halfway between 1 and 1+2**-23
    t = ok.vecadd_f32(np.array([1.0], np.float32), np.array([2.0 ** -24], np.float32))
    assert t[0] == np.float32(1.0)
    t = ok.vecadd_f32(np.array([1.0 + 2.0 ** -23], np.float32), np.array([2.0 ** -24], np.float32))
    assert t[0] == np.float32(1.0 + 2.0 ** -22)


def test_vecadd_and_vecmul_on_the_edge_pair_grid():
    # the operand grid the GPU parity test feeds the kernels: every finite
    # pair against exact rational rounding (zeros by the IEEE sign rule),
    # specials by the IEEE rules for inf and NaN
    a, b = wl.edge_pairs()
    for op, f in ((ok.vecadd_f32, lambda x, y: x + y), (ok.vecmul_f32, lambda x, y: x * y)):
        c = op(a, b)
        for x, y, z in zip(a.tolist(), b.tolist(), c.tolist()):
            if math.isnan(x) or math.isnan(y):
                assert math.isnan(z)
                continue
            if math.isinf(x) or math.isinf(y):
                with np.errstate(invalid="ignore", over="ignore"):
                    want = float(f(np.float64(x), np.float64(y)))
                assert (math.isnan(z) and math.isnan(want)) or z == want, (x, y, z)
                continue
            exact = f(Fraction(x), Fraction(y))
            want = _round_to_binary32(exact)
            if want == 0.0:
                if op is ok.vecadd_f32:
                    neg = _bits(x) == _bits(-0.0) and _bits(y) == _bits(-0.0)
                else:
                    neg = (math.copysign(1.0, x) * math.copysign(1.0, y)) < 0
                assert _bits(z) == (_bits(-0.0) if neg else 0), (x, y, z)
            else:
                assert _bits(z) == _bits(want), (x, y, z, want)


def test_vecadd_special_values():
    a = np.array([np.inf, -np.inf, np.inf, np.nan, 3.0e38], dtype=np.float32)
    b = np.array([1.0, 1.0, -np.inf, 1.0, 3.0e38], dtype=np.float32)
    c = ok.vecadd_f32(a, b)
    assert c[0] == np.inf and c[1] == -np.inf
    assert np.isnan(c[2]) and np.isnan(c[3])
    assert c[4] == np.inf


def test_vecadd_rejects_bad_inputs():
    with pytest.raises(TypeError):
        ok.vecadd_f32(np.zeros(4), np.zeros(4, np.float32))
    with pytest.raises(ValueError):
        ok.vecadd_f32(np.zeros(4, np.float32), np.zeros(5, np.float32))
    assert ok.vecadd_f32(np.zeros(0, np.float32), np.zeros(0, np.float32)).shape == (0,)


def test_vecmul_matches_exact_rounding():
    g = np.random.default_rng(8)
    a = g.uniform(-2, 2, 500).astype(np.float32)
    b = g.uniform(-2, 2, 500).astype(np.float32)
    c1 = ok.vecmul_f32(a, b)
    for x, y, z in zip(a, b, c1):
        assert _bits(float(z)) == _bits(_round_to_binary32(Fraction(float(x)) * Fraction(float(y))))
    c3 = ok.vecmul_f32(a[:50], b[:50], iters=3)
    for x, y, z in zip(a[:50], b[:50], c3):
        w = Fraction(float(x))
        for _ in range(3):
            w = Fraction(_round_to_binary32(w * Fraction(float(y))))
        assert _bits(float(z)) == _bits(float(w))


# ---------------------------------------------------------------- Black-Scholes

def test_norm_cdf_table_values():
    with open(os.path.join(GOLDEN, "normal_cdf_table.json")) as f:
        tab = json.load(f)
    for x, p in tab["cases"]:
        assert abs(float(ok.norm_cdf_f64(x)) - p) <= tab["tol"]
        assert abs(float(ok.norm_cdf_f64(-x)) - (1.0 - p)) <= tab["tol"]


def test_black_scholes_textbook_example():
    with open(os.path.join(GOLDEN, "black_scholes_textbook.json")) as f:
        gold = json.load(f)
    for c in gold["cases"]:
        S = np.array([c["S"]], np.float32)
        K = np.array([c["K"]], np.float32)
        T = np.array([c["T"]], np.float32)
        call, put = ok.black_scholes_f64(S, K, T, c["r"], c["sigma"])
        assert abs(call[0] - c["call"]) <= c["price_tol"]
        assert abs(put[0] - c["put"]) <= c["price_tol"]
        # the intermediate d1, d2 of the same example, from the stated definition
        vol = c["sigma"] * math.sqrt(c["T"])
        d1 = (math.log(c["S"] / c["K"]) + (c["r"] + c["sigma"] ** 2 / 2) * c["T"]) / vol
        assert abs(d1 - c["d1"]) <= c["d_tol"] and abs(d1 - vol - c["d2"]) <= c["d_tol"]


def _bs_quadrature(S, K, T, r, sigma):
    """Discounted risk-neutral expectation of the call and put payoffs,
    integrated numerically over the log-normal terminal price (no closed
    form involved)."""
    mu = math.log(S) + (r - 0.5 * sigma * sigma) * T
    sd = sigma * math.sqrt(T)
    disc = math.exp(-r * T)

    def dens(z):  # standard normal density
        return math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)

    zk = (math.log(K) - mu) / sd
    call = integrate.quad(lambda z: (math.exp(mu + sd * z) - K) * dens(z), zk, zk + 40, epsabs=1e-12, epsrel=1e-12, limit=200)[0]
    put = integrate.quad(lambda z: (K - math.exp(mu + sd * z)) * dens(z), zk - 40, zk, epsabs=1e-12, epsrel=1e-12, limit=200)[0]
    return disc * call, disc * put


def test_black_scholes_matches_risk_neutral_quadrature():
    S, K, T = wl.bs_inputs(99, 0, 24)
    r, sigma = float(np.float32(wl.BS_RATE)), float(np.float32(wl.BS_VOLATILITY))
    call, put = ok.black_scholes_f64(S, K, T, r, sigma)
    for i in range(len(S)):
        qc, qp = _bs_quadrature(float(S[i]), float(K[i]), float(T[i]), r, sigma)
        assert abs(call[i] - qc) <= 1e-8 * max(1.0, qc), (i, call[i], qc)
        assert abs(put[i] - qp) <= 1e-8 * max(1.0, qp), (i, put[i], qp)


def test_black_scholes_parity_bounds_and_atm_forward():
    S, K, T = wl.bs_inputs(98, 3, 20000)
    r, sigma = 0.02, 0.30
    call, put = ok.black_scholes_f64(S, K, T, r, sigma)
    S64, K64, T64 = (x.astype(np.float64) for x in (S, K, T))
    dk = K64 * np.exp(-r * T64)
    np.testing.assert_allclose(call - put, S64 - dk, rtol=0, atol=1e-12 * (S64 + K64).max())
    assert np.all(call >= np.maximum(S64 - dk, 0) - 1e-12) and np.all(call <= S64 + 1e-12)
    assert np.all(put >= np.maximum(dk - S64, 0) - 1e-12) and np.all(put <= dk + 1e-12)
    # at-the-money forward, S = K exp(-rT): C = P = S erf(sigma sqrt(T) / (2 sqrt 2))
    Ta = np.array([0.25, 1.0, 4.0, 10.0], np.float32)
    Ka = np.array([50.0, 50.0, 50.0, 50.0], np.float32)
    Sa64 = 50.0 * np.exp(-r * Ta.astype(np.float64))
    Sa = Sa64.astype(np.float32)
    c, p = ok.black_scholes_f64(Sa, Ka, Ta, r, sigma)
    for i in range(4):
        s = float(Sa[i])
        # exact ATMF formula evaluated at the binary32 spot, corrected to first order for its rounding
        want = s * math.erf(sigma * math.sqrt(float(Ta[i])) / (2 * math.sqrt(2)))
        shift = s - float(Sa64[i])
        assert abs(c[i] - want) <= abs(shift) + 1e-9
        assert abs(p[i] - want) <= abs(shift) + 1e-9


def test_black_scholes_degenerate_volatility_is_intrinsic():
    S = np.array([30.0, 10.0, 20.0], np.float32)
    K = np.array([20.0, 40.0, 20.0], np.float32)
    T = np.array([1.0, 2.0, 0.0], np.float32)
    call, put = ok.black_scholes_f64(S, K, T, 0.05, 0.0)
    dk = K.astype(np.float64) * np.exp(-0.05 * T.astype(np.float64))
    np.testing.assert_allclose(call, np.maximum(S - dk, 0), atol=1e-12)
    np.testing.assert_allclose(put, np.maximum(dk - S, 0), atol=1e-12)
    # tiny but non-zero volatility converges to the same limit
    c2, p2 = ok.black_scholes_f64(S[:2], K[:2], T[:2], 0.05, 1e-9)
    np.testing.assert_allclose(c2, np.maximum(S[:2] - dk[:2], 0), atol=1e-9)
    np.testing.assert_allclose(p2, np.maximum(dk[:2] - S[:2], 0), atol=1e-9)


def test_black_scholes_monotone_in_spot_and_strike():
    S = np.linspace(5, 30, 101).astype(np.float32)
    K = np.full(101, 20.0, np.float32)
    T = np.full(101, 1.0, np.float32)
    call, put = ok.black_scholes_f64(S, K, T, 0.02, 0.3)
    assert np.all(np.diff(call) > 0) and np.all(np.diff(put) < 0)


# ---------------------------------------------------------------- SGEMM

def test_sgemm_matches_bruteforce_loops_nonsquare():
    g = np.random.default_rng(3)
    for (m, k, n) in [(1, 1, 1), (3, 5, 7), (8, 2, 3), (17, 9, 4)]:
        A = g.standard_normal((m, k)).astype(np.float32)
        B = g.standard_normal((k, n)).astype(np.float32)
        np.testing.assert_allclose(ok.sgemm_f64(A, B), ok.sgemm_bruteforce(A, B), rtol=1e-13, atol=1e-13)


def test_sgemm_bruteforce_exact_on_integers():
    A, B = wl.sgemm_int_inputs(97, 0, 6)
    want = [[sum(Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(6)) for j in range(6)] for i in range(6)]
    got = ok.sgemm_bruteforce(A, B)
    assert all(got[i, j] == want[i][j] for i in range(6) for j in range(6))
    np.testing.assert_array_equal(ok.sgemm_f64(A, B), got)


def test_sgemm_identity_permutation_and_transpose():
    g = np.random.default_rng(4)
    n = 64
    A = g.standard_normal((n, n)).astype(np.float32)
    I = np.eye(n, dtype=np.float32)
    np.testing.assert_array_equal(ok.sgemm_f64(A, I), A.astype(np.float64))
    np.testing.assert_array_equal(ok.sgemm_f64(I, A), A.astype(np.float64))
    perm = g.permutation(n)
    P = I[perm]                      # row i of P is the unit vector e_perm[i]
    np.testing.assert_array_equal(ok.sgemm_f64(P, A), A[perm].astype(np.float64))
    B = g.standard_normal((n, n)).astype(np.float32)
    np.testing.assert_allclose(ok.sgemm_f64(A, B).T, ok.sgemm_f64(B.T.copy(), A.T.copy()), rtol=1e-12, atol=1e-12)
    # a transposed operand is caught: A B differs from A^T B for a non-symmetric A
    assert np.abs(ok.sgemm_f64(A, B) - ok.sgemm_f64(A.T.copy(), B)).max() > 1.0


def test_sgemm_rejects_bad_shapes():
    with pytest.raises(ValueError):
        ok.sgemm_f64(np.zeros((2, 3), np.float32), np.zeros((2, 3), np.float32))
    with pytest.raises(TypeError):
        ok.sgemm_f64(np.zeros((2, 2)), np.zeros((2, 2), np.float32))
