"""Pins of the plain C oracle (oracle/c/oracle.c, loaded through
oracle.c_oracle) to the same things the Python oracle is pinned to, none of
them the oracle itself: exact rational rounding of binary32 sums and
products, the textbook Black-Scholes example and a risk-neutral quadrature,
put-call parity and bounds, exact integer matrix products, identity and
permutation matrices, and the execution model's discrete-event schedule
against the closed forms, their N = 1 reductions and their limits.  Last,
the two restatements agree with each other on seeded inputs.

The library is compiled privately here with the build step's flags."""

import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import c_oracle as co
from oracle import kernels as ok
from oracle import model as m
from paper_1511_07658_amd import workloads as wl

from test_oracle_kernels import _bits, _bs_quadrature, _round_to_binary32
from test_oracle_model import _draw

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    path = str(tmp_path_factory.mktemp("oracle") / "liboracle.so")
    return co.load(co.compile_to(path))


def test_vecadd_vecmul_edge_pair_grid_exact(lib):
    a, b = wl.edge_pairs()
    for op, f, is_add in ((co.vecadd_f32, lambda x, y: x + y, True), (co.vecmul_f32, lambda x, y: x * y, False)):
        c = op(a, b, lib=lib)
        for x, y, z in zip(a.tolist(), b.tolist(), c.tolist()):
            if math.isnan(x) or math.isnan(y):
                assert math.isnan(z)
                continue
            if math.isinf(x) or math.isinf(y):
                with np.errstate(invalid="ignore", over="ignore"):
                    want = float(f(np.float64(x), np.float64(y)))
                assert (math.isnan(z) and math.isnan(want)) or z == want, (x, y, z)
                continue
            want = _round_to_binary32(f(Fraction(x), Fraction(y)))
            if want == 0.0:
                if is_add:
                    neg = _bits(x) == _bits(-0.0) and _bits(y) == _bits(-0.0)
                else:
                    neg = (math.copysign(1.0, x) * math.copysign(1.0, y)) < 0
                assert _bits(z) == (_bits(-0.0) if neg else 0), (x, y, z)
            else:
                assert _bits(z) == _bits(want), (x, y, z, want)


def test_vecadd_random_and_ties_exact(lib):
    g = np.random.default_rng(17)
    a = g.uniform(-1, 1, 2000).astype(np.float32)
    b = g.uniform(-1, 1, 2000).astype(np.float32)
    b[:300] = (a[:300] * -0.999).astype(np.float32)
    c = co.vecadd_f32(a, b, lib=lib)
    for x, y, z in zip(a, b, c):
        assert _bits(float(z)) == _bits(_round_to_binary32(Fraction(float(x)) + Fraction(float(y))))
    t = co.vecadd_f32(np.array([1.0, 1.0 + 2.0 ** -23], np.float32), np.array([2.0 ** -24] * 2, np.float32), lib=lib)
    assert t[0] == np.float32(1.0) and t[1] == np.float32(1.0 + 2.0 ** -22)


def test_vecmul_iterated_exact(lib):
    g = np.random.default_rng(18)
    a = g.uniform(-2, 2, 60).astype(np.float32)
    b = g.uniform(-2, 2, 60).astype(np.float32)
    c = co.vecmul_f32(a, b, iters=3, lib=lib)
    for x, y, z in zip(a, b, c):
        w = Fraction(float(x))
        for _ in range(3):
            w = Fraction(_round_to_binary32(w * Fraction(float(y))))
        assert _bits(float(z)) == _bits(float(w))


def test_black_scholes_textbook_and_quadrature(lib):
    with open(os.path.join(GOLDEN, "black_scholes_textbook.json")) as f:
        gold = json.load(f)
    for c in gold["cases"]:
        call, put = co.black_scholes_f64(np.array([c["S"]], np.float32), np.array([c["K"]], np.float32),
                                         np.array([c["T"]], np.float32), c["r"], c["sigma"], lib=lib)
        assert abs(call[0] - c["call"]) <= c["price_tol"] and abs(put[0] - c["put"]) <= c["price_tol"]
    S, K, T = wl.bs_inputs(99, 0, 16)
    r, sigma = float(np.float32(wl.BS_RATE)), float(np.float32(wl.BS_VOLATILITY))
    call, put = co.black_scholes_f64(S, K, T, r, sigma, lib=lib)
    for i in range(len(S)):
        qc, qp = _bs_quadrature(float(S[i]), float(K[i]), float(T[i]), r, sigma)
        assert abs(call[i] - qc) <= 1e-8 * max(1.0, qc)
        assert abs(put[i] - qp) <= 1e-8 * max(1.0, qp)


def test_black_scholes_parity_bounds_and_degenerate(lib):
    S, K, T = wl.bs_inputs(98, 3, 5000)
    r, sigma = 0.02, 0.30
    call, put = co.black_scholes_f64(S, K, T, r, sigma, lib=lib)
    S64, K64, T64 = (x.astype(np.float64) for x in (S, K, T))
    dk = K64 * np.exp(-r * T64)
    np.testing.assert_allclose(call - put, S64 - dk, rtol=0, atol=1e-12 * (S64 + K64).max())
    assert np.all(call >= np.maximum(S64 - dk, 0) - 1e-12) and np.all(call <= S64 + 1e-12)
    assert np.all(put >= np.maximum(dk - S64, 0) - 1e-12) and np.all(put <= dk + 1e-12)
    Sd = np.array([30.0, 10.0, 20.0], np.float32)
    Kd = np.array([20.0, 40.0, 20.0], np.float32)
    Td = np.array([1.0, 2.0, 0.0], np.float32)
    c0, p0 = co.black_scholes_f64(Sd, Kd, Td, 0.05, 0.0, lib=lib)
    dkd = Kd.astype(np.float64) * np.exp(-0.05 * Td.astype(np.float64))
    np.testing.assert_allclose(c0, np.maximum(Sd - dkd, 0), atol=1e-12)
    np.testing.assert_allclose(p0, np.maximum(dkd - Sd, 0), atol=1e-12)


def test_sgemm_integer_exact_identity_permutation(lib):
    A, B = wl.sgemm_int_inputs(97, 0, 9)
    want = [[sum(Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(9)) for j in range(9)]
            for i in range(9)]
    got = co.sgemm_f64(A, B, lib=lib)
    assert all(got[i, j] == want[i][j] for i in range(9) for j in range(9))
    g = np.random.default_rng(4)
    n = 48
    X = g.standard_normal((n, n)).astype(np.float32)
    I = np.eye(n, dtype=np.float32)
    np.testing.assert_array_equal(co.sgemm_f64(X, I, lib=lib), X.astype(np.float64))
    perm = g.permutation(n)
    np.testing.assert_array_equal(co.sgemm_f64(I[perm].copy(), X, lib=lib), X[perm].astype(np.float64))
    Y = g.standard_normal((n, n)).astype(np.float32)
    assert np.abs(co.sgemm_f64(X, Y, lib=lib) - co.sgemm_f64(X.T.copy(), Y, lib=lib)).max() > 1.0
    # a row slice is those rows of the whole product, bit for bit
    np.testing.assert_array_equal(co.sgemm_rows_f64(X, Y, 5, 7, lib=lib), co.sgemm_f64(X, Y, lib=lib)[5:12])


@pytest.mark.parametrize("cls", ["CI", "IOI", "INT"])
def test_des_reproduces_closed_forms(lib, cls):
    rng = random.Random(hash(cls) & 0xFFFF ^ 0x55)
    for _ in range(1500):
        n = rng.randint(1, 16)
        ti, tc, to = _draw(rng, cls)
        s1 = co.des_simulate("PS1", n, ti, tc, to, lib=lib)
        s2 = co.des_simulate("PS2", n, ti, tc, to, lib=lib)
        assert s1 == pytest.approx(co.eq(2, n, ti, tc, to, lib=lib), rel=1e-12, abs=1e-12)
        assert s1 == pytest.approx(co.eq(4, n, ti, tc, to, lib=lib), rel=1e-12, abs=1e-12)
        if cls == "CI":
            assert s2 == pytest.approx(co.eq(3, n, ti, tc, to, lib=lib), rel=1e-12, abs=1e-12)
        if cls == "IOI":
            assert s2 == pytest.approx(co.eq(7, n, ti, tc, to, lib=lib), rel=1e-12, abs=1e-12)
            k = 5 if to < ti else 6
            assert s2 == pytest.approx(co.eq(k, n, ti, tc, to, lib=lib), rel=1e-12, abs=1e-12)
        for style in ("PS1", "PS2"):
            assert co.des_simulate(style, n, ti, tc, to, "multiqueue", lib=lib) <= \
                co.des_simulate(style, n, ti, tc, to, lib=lib) + 1e-12


def test_des_worked_schedules(lib):
    assert co.des_simulate("PS2", 3, 2.0, 1.0, 1.0, lib=lib) == 8.0
    assert co.des_simulate("PS1", 2, 1.0, 3.0, 1.0, lib=lib) == 7.0
    assert lib.des_simulate(1, 0, 0, 1.0, 1.0, 1.0) == -1.0      # no streams
    assert lib.des_simulate(3, 0, 2, 1.0, 1.0, 1.0) == -1.0      # no such style


def test_model_reductions_and_limits(lib):
    for (ti, tc, to) in [(1, 2, 3), (3, 1, 2), (0.5, 0.5, 0.5)]:
        one = ti + tc + to
        for k in (2, 3, 4, 7):
            assert co.eq(k, 1, ti, tc, to, lib=lib) == pytest.approx(one)
        assert co.eq(1, 1, 7.0, 11.0, ti, tc, to, lib=lib) == pytest.approx(7.0 + one)
        assert co.eq(8, 1, 0, 0, ti, tc, to, lib=lib) == pytest.approx(1.0)
        assert co.eq(9, 1, 0, 0, ti, tc, to, lib=lib) == pytest.approx(1.0)
    rng = random.Random(21)
    for _ in range(200):
        ti, tc, to = _draw(rng, rng.choice(["CI", "IOI"]))
        t_init, t_ctx = rng.uniform(0, 50), rng.uniform(0, 5)
        assert co.eq(8, 10 ** 9, t_init, t_ctx, ti, tc, to, lib=lib) == pytest.approx(
            co.eq(10, t_init, t_ctx, ti, tc, to, lib=lib), rel=1e-6)
        assert co.eq(9, 10 ** 9, t_init, t_ctx, ti, tc, to, lib=lib) == pytest.approx(
            co.eq(11, t_init, t_ctx, ti, tc, to, lib=lib), rel=1e-6)
        n = rng.randint(1, 64)
        assert co.eq(4, n, ti, tc, to, lib=lib) - co.eq(7, n, ti, tc, to, lib=lib) == pytest.approx(
            (n - 1) * min(ti, to), rel=1e-9, abs=1e-9)


def test_c_and_python_oracles_agree(lib):
    a, b = wl.vecadd_inputs(5, 1, 10007)
    assert np.array_equal(co.vecadd_f32(a, b, lib=lib).view(np.uint32), ok.vecadd_f32(a, b).view(np.uint32))
    S, K, T = wl.bs_inputs(5, 1, 3001)
    cc, cp = co.black_scholes_f64(S, K, T, 0.02, 0.3, lib=lib)
    pc, pp = ok.black_scholes_f64(S, K, T, 0.02, 0.3)
    np.testing.assert_allclose(cc, pc, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(cp, pp, rtol=1e-13, atol=1e-13)
    A, B = wl.sgemm_inputs(5, 1, 67)
    np.testing.assert_allclose(co.sgemm_f64(A, B, lib=lib), ok.sgemm_f64(A, B), rtol=1e-12, atol=1e-12)
    rng = random.Random(3)
    for _ in range(200):
        n = rng.randint(1, 20)
        ti, tc, to = rng.uniform(0, 5), rng.uniform(0.01, 5), rng.uniform(0, 5)
        assert co.eq(1, n, 3, 0.5, ti, tc, to, lib=lib) == pytest.approx(m.eq1_total_no_vt(n, 3, 0.5, ti, tc, to))
        assert co.eq(7, n, ti, tc, to, lib=lib) == pytest.approx(m.eq7_total_ioi_ps2(n, ti, tc, to))
