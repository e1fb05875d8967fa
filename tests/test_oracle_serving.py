"""Pins of the serving-run checks (oracle.serving): hand-made logs whose
verdict is known, and the nearest-rank percentile against its definition on
small samples and against numpy's inverted-CDF percentile."""

import random

import numpy as np
import pytest

from oracle import serving as sv


def test_budget_check_accepts_and_reports_peak():
    ev = [(0.0, "admit", 1, 40), (0.1, "admit", 2, 60), (0.2, "complete", 1, 40),
          (0.2, "admit", 3, 40), (0.5, "complete", 2, 60), (0.6, "complete", 3, 40)]
    assert sv.check_budget(ev, 100) == 100


def test_budget_check_rejects_overcommit():
    ev = [(0.0, "admit", 1, 40), (0.1, "admit", 2, 61), (0.3, "complete", 1, 40), (0.4, "complete", 2, 61)]
    with pytest.raises(AssertionError):
        sv.check_budget(ev, 100)


def test_lifecycle_checks():
    ev = [(0.0, "admit", 1, 1), (0.1, "complete", 1, 1), (0.1, "admit", 2, 1), (0.2, "complete", 2, 1)]
    sv.check_lifecycle([1, 2], ev)
    with pytest.raises(AssertionError):
        sv.check_lifecycle([1, 2, 3], ev)
    with pytest.raises(AssertionError):
        sv.check_lifecycle([1, 2], ev + [(0.3, "complete", 2, 1)])
    with pytest.raises(AssertionError):
        sv.check_lifecycle([1], [(0.5, "admit", 1, 1), (0.4, "complete", 1, 1)])


def test_fifo_check():
    sv.check_fifo([3, 1, 2], [3, 1, 2])
    with pytest.raises(AssertionError):
        sv.check_fifo([3, 1, 2], [1, 3, 2])


def test_percentile_definition():
    xs = [15, 20, 35, 40, 50]
    assert sv.percentile_nearest_rank(xs, 5) == 15
    assert sv.percentile_nearest_rank(xs, 30) == 20
    assert sv.percentile_nearest_rank(xs, 40) == 20
    assert sv.percentile_nearest_rank(xs, 50) == 35
    assert sv.percentile_nearest_rank(xs, 100) == 50
    rng = random.Random(2)
    for _ in range(200):
        s = [rng.random() for _ in range(rng.randint(1, 300))]
        for p in (50, 90, 99):
            assert sv.percentile_nearest_rank(s, p) == np.percentile(s, p, method="inverted_cdf")
    with pytest.raises(ValueError):
        sv.percentile_nearest_rank([], 50)
