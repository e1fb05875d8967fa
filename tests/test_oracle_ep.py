"""Pins of the EP-like oracle (oracle/ep.py) to things other than itself:
numpy's Philox bit generator, the algebra of the polar method, and the
distribution its outputs must follow."""

import math

import numpy as np
import pytest
from scipy.special import erf
from scipy.stats import chi2

from oracle import ep

KEYS = [(0, 0), (1, 2), (0xDEADBEEF12345678, 0x0123456789ABCDEF), (2**64 - 1, 2**63 + 5)]


def _numpy_block(key, counter):
    """Philox4x64-10 of `counter` from numpy: its generator increments the
    256-bit counter (word 0 least significant) before each block."""
    words = [int(c) for c in counter]
    v = sum(w << (64 * i) for i, w in enumerate(words))
    v = (v - 1) % (1 << 256)
    start = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=start)
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("key", KEYS)
def test_philox_matches_numpy(key):
    counters = [(0, 0, 0, 0), (1, 0, 0, 0), (12345, 0, 0, 0), (2**64 - 1, 0, 0, 0), (7, 3, 0, 0),
                (0, 0, 0, 1), (2**64 - 1, 2**64 - 1, 5, 9)]
    for c in counters:
        assert list(ep.philox4x64_10_scalar(c, key)) == _numpy_block(key, c), (key, c)


def test_vectorised_philox_matches_scalar():
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2**64, size=(64, 4), dtype=np.uint64)
    ctr[0] = 0
    ctr[1] = 2**64 - 1
    for key in KEYS:
        v = ep.philox4x64_10(ctr, key)
        for i in range(ctr.shape[0]):
            assert [int(x) for x in v[i]] == list(ep.philox4x64_10_scalar(ctr[i], key))


def test_words_follow_block_layout():
    key = KEYS[2]
    w = ep.ep_words(key, 5)  # 3 blocks, last one half used
    assert w.shape == (10,)
    for b in range(3):
        blk = ep.philox4x64_10_scalar((b, 0, 0, 0), key)
        for i in range(4):
            if 4 * b + i < 10:
                assert int(w[4 * b + i]) == blk[i]
    assert ep.ep_words(key, 0).shape == (0,)


def test_uniform_pairs_exact_and_in_range():
    key = KEYS[1]
    x, y = ep.ep_uniform_pairs(key, 4097)
    w = ep.ep_words(key, 4097)
    assert x.shape == y.shape == (4097,)
    assert np.all(x >= -1.0) and np.all(x < 1.0) and np.all(y >= -1.0) and np.all(y < 1.0)
    # exact: x = 2 * (w >> 11) / 2^53 - 1 as a rational, compared with Python integers
    for j in range(0, 4097, 97):
        m = int(w[2 * j]) >> 11
        assert x[j] == (2 * m - 2**53) / 2**53


def test_polar_algebra():
    key = KEYS[3]
    x, y = ep.ep_uniform_pairs(key, 20000)
    acc, X, Y = ep.ep_polar(x, y)
    t = (x * x + y * y)[acc]
    # X^2 + Y^2 = -2 ln t, and (X, Y) points the way (x, y) does
    np.testing.assert_allclose(X * X + Y * Y, -2.0 * np.log(t), rtol=1e-13, atol=1e-15)
    assert np.all(np.sign(X) == np.sign(x[acc])) and np.all(np.sign(Y) == np.sign(y[acc]))
    np.testing.assert_allclose(X * y[acc], Y * x[acc], rtol=1e-12, atol=1e-15)
    # acceptance is exactly the unit disk (minus the origin)
    assert np.array_equal(acc, ((x * x + y * y) <= 1.0) & ((x * x + y * y) > 0.0))


def _distribution_pins(polar, key=(5, 6), n=1 << 20):
    """Statistics that any correct polar method satisfies: acceptance pi/4,
    zero mean, unit variance, and annulus counts of two independent
    standard normals: P(max(|X|,|Y|) < l) = erf(l / sqrt 2)^2."""
    x, y = ep.ep_uniform_pairs(key, n)
    acc, X, Y = polar(x, y)
    a = int(acc.sum())
    p = math.pi / 4
    ok = abs(a - n * p) < 6 * math.sqrt(n * p * (1 - p))
    for v in (X, Y):
        ok &= abs(v.mean()) < 6 / math.sqrt(a)
        ok &= abs(v.var() - 1.0) < 6 * math.sqrt(2.0 / a)
    m = np.maximum(np.abs(X), np.abs(Y))
    edges = np.arange(0, ep.EP_ANNULI + 1, dtype=np.float64)
    obs = np.histogram(m, bins=np.append(edges[:6], np.inf))[0]
    cdf = erf(np.append(edges[:6], np.inf) / math.sqrt(2.0)) ** 2
    exp = a * np.diff(cdf)
    stat = float(((obs - exp) ** 2 / np.maximum(exp, 1e-300)).sum())
    ok &= stat < chi2.ppf(1 - 1e-6, df=len(obs) - 1)
    return bool(ok)


def test_distribution_of_the_pairs():
    assert _distribution_pins(ep.ep_polar)


def test_pins_catch_planted_mistakes():
    def no_two(x, y):
        t = x * x + y * y
        acc = (t > 0) & (t <= 1)
        f = np.sqrt(-np.log(t[acc]) / t[acc])
        return acc, x[acc] * f, y[acc] * f

    def no_divide(x, y):
        t = x * x + y * y
        acc = (t > 0) & (t <= 1)
        f = np.sqrt(-2.0 * np.log(t[acc]))
        return acc, x[acc] * f, y[acc] * f

    def swapped(x, y):
        acc, X, Y = ep.ep_polar(x, y)
        return acc, X, np.abs(Y)  # a sign lost

    for bad in (no_two, no_divide, swapped):
        assert not _distribution_pins(bad), bad.__name__


def test_reference_outputs_consistent():
    key = KEYS[2]
    r = ep.ep_reference(key, 1 << 16)
    x, y = ep.ep_uniform_pairs(key, 1 << 16)
    acc, X, Y = ep.ep_polar(x, y)
    assert r["accepted"] == int(acc.sum())
    assert int(r["q"].sum()) == int((np.maximum(np.abs(X), np.abs(Y)) < ep.EP_ANNULI).sum())
    assert r["sx"] == math.fsum(X.tolist()) and r["sy"] == math.fsum(Y.tolist())
    # brute force on a few pairs with Python floats
    small = ep.ep_reference(key, 9)
    xs, ys = ep.ep_uniform_pairs(key, 9)
    sx = []
    for xv, yv in zip(xs.tolist(), ys.tolist()):
        t = xv * xv + yv * yv
        if 0.0 < t <= 1.0:
            sx.append(xv * math.sqrt(-2.0 * math.log(t) / t))
    assert small["accepted"] == len(sx)
    assert small["sx"] == pytest.approx(math.fsum(sx), rel=1e-14, abs=1e-15)
