"""Pins of the execution model (oracle.model, oracle.des): the closed forms of
Section 4 against the discrete-event schedule of the stream rules, their
stated special cases, limits and orderings."""

import random

import pytest

from oracle import des
from oracle import model as m


def _draw(rng, cls):
    tc = rng.uniform(0.05, 10.0)
    if cls == "CI":
        return rng.uniform(0, tc), tc, rng.uniform(0, tc)
    if cls == "IOI":
        return rng.uniform(tc * 1.001, tc * 20), tc, rng.uniform(tc * 1.001, tc * 20)
    lo, hi = rng.uniform(0, tc), rng.uniform(tc * 1.001, tc * 20)
    return (lo, tc, hi) if rng.random() < 0.5 else (hi, tc, lo)


@pytest.mark.parametrize("cls", ["CI", "IOI", "INT"])
def test_des_reproduces_closed_forms(cls):
    rng = random.Random(hash(cls) & 0xFFFF)
    for _ in range(3000):
        n = rng.randint(1, 16)
        ti, tc, to = _draw(rng, cls)
        assert m.classify(ti, tc, to) == cls
        s1 = des.simulate("PS1", n, ti, tc, to)
        s2 = des.simulate("PS2", n, ti, tc, to)
        assert s1 == pytest.approx(m.eq2_total_ci_ps1(n, ti, tc, to), rel=1e-12, abs=1e-12)
        assert s1 == pytest.approx(m.eq4_total_ioi_ps1(n, ti, tc, to), rel=1e-12, abs=1e-12)
        if cls == "CI":
            assert s2 == pytest.approx(m.eq3_total_ci_ps2(n, ti, tc, to), rel=1e-12, abs=1e-12)
        if cls == "IOI":
            assert s2 == pytest.approx(m.eq7_total_ioi_ps2(n, ti, tc, to), rel=1e-12, abs=1e-12)
            eq56 = m.eq5_total_ioi_ps2_out_lt_in if to < ti else m.eq6_total_ioi_ps2_out_ge_in
            assert s2 == pytest.approx(eq56(n, ti, tc, to), rel=1e-12, abs=1e-12)
        assert s2 == pytest.approx(m.modelled_total("PS2", n, ti, tc, to), rel=1e-12, abs=1e-12)


def test_des_worked_schedule_ps2_ioi():
    # 3 streams, send 2, kernel 1, retrieve 1 (IO-I, t_out < t_in): sends back to
    # back at 0-2, 2-4, 4-6; kernels at 2-3, 4-5, 6-7; retrieves at 3-4, 5-6, 7-8.
    times = des.schedule(des.enqueue_order("PS2", 3, 2.0, 1.0, 1.0))
    assert times == [(0, 2), (2, 3), (3, 4), (2, 4), (4, 5), (5, 6), (4, 6), (6, 7), (7, 8)]
    assert m.eq5_total_ioi_ps2_out_lt_in(3, 2.0, 1.0, 1.0) == 8.0


def test_des_worked_schedule_ps1_ci():
    # 2 streams, send 1, kernel 3, retrieve 1 under PS-1: sends 0-1, 1-2; kernels
    # overlap 1-4, 2-5; the first retrieve waits for the last kernel: 5-6, 6-7.
    times = des.schedule(des.enqueue_order("PS1", 2, 1.0, 3.0, 1.0))
    assert times == [(0, 1), (1, 2), (1, 4), (2, 5), (5, 6), (6, 7)]
    assert m.eq2_total_ci_ps1(2, 1.0, 3.0, 1.0) == 7.0


def test_multiqueue_rules_never_slower():
    rng = random.Random(5)
    for _ in range(500):
        n = rng.randint(1, 12)
        ti, tc, to = _draw(rng, rng.choice(["CI", "IOI", "INT"]))
        for style in ("PS1", "PS2"):
            assert des.simulate(style, n, ti, tc, to, "multiqueue") <= des.simulate(style, n, ti, tc, to) + 1e-12
        # without false dependencies both styles approach max(N t_in, N t_out) + ...
        assert des.simulate("PS2", n, ti, tc, to, "multiqueue") >= n * max(ti, to)


def test_single_process_reduces_to_one_cycle():
    for (ti, tc, to) in [(1, 2, 3), (3, 1, 2), (0.5, 0.5, 0.5)]:
        one = ti + tc + to
        for f in (m.eq2_total_ci_ps1, m.eq3_total_ci_ps2, m.eq4_total_ioi_ps1, m.eq7_total_ioi_ps2):
            assert f(1, ti, tc, to) == pytest.approx(one)
        assert m.eq1_total_no_vt(1, 7.0, 11.0, ti, tc, to) == pytest.approx(7.0 + one)
        assert m.eq8_speedup_ci(1, 0, 0, ti, tc, to) == pytest.approx(1.0)
        assert m.eq9_speedup_ioi(1, 0, 0, ti, tc, to) == pytest.approx(1.0)


def test_eq1_grows_by_one_full_cycle_per_process():
    for n in range(1, 10):
        d = m.eq1_total_no_vt(n + 1, 5, 0.3, 1, 2, 3) - m.eq1_total_no_vt(n, 5, 0.3, 1, 2, 3)
        assert d == pytest.approx(5 + 0.3 + 1 + 2 + 3)


def test_speedup_limits_match_eq10_eq11():
    rng = random.Random(11)
    for _ in range(200):
        ti, tc, to = _draw(rng, rng.choice(["CI", "IOI"]))
        t_init, t_ctx = rng.uniform(0, 50), rng.uniform(0, 5)
        big = 10 ** 9
        assert m.eq8_speedup_ci(big, t_init, t_ctx, ti, tc, to) == pytest.approx(
            m.eq10_speedup_max_ci(t_init, t_ctx, ti, tc, to), rel=1e-6)
        assert m.eq9_speedup_ioi(big, t_init, t_ctx, ti, tc, to) == pytest.approx(
            m.eq11_speedup_max_ioi(t_init, t_ctx, ti, tc, to), rel=1e-6)


def test_ps2_never_worse_than_ps1_for_ioi():
    rng = random.Random(13)
    for _ in range(1000):
        n = rng.randint(1, 64)
        ti, tc, to = _draw(rng, "IOI")
        diff = m.eq4_total_ioi_ps1(n, ti, tc, to) - m.eq7_total_ioi_ps2(n, ti, tc, to)
        assert diff == pytest.approx((n - 1) * min(ti, to), rel=1e-9, abs=1e-9)
        assert m.paper_ps_choice(ti, tc, to) == "PS2" == m.best_ps_choice(n, ti, tc, to) or n == 1


def test_ci_claim_holds_only_when_transfers_are_shorter_than_compute():
    # Eq2 - Eq3 = (N-1)(t_in + t_out - t_comp)
    n, ti, tc, to = 2, 0.8, 1.0, 0.8
    assert m.classify(ti, tc, to) == "CI"
    assert m.eq2_total_ci_ps1(n, ti, tc, to) == pytest.approx(4.2)
    assert m.eq3_total_ci_ps2(n, ti, tc, to) == pytest.approx(3.6)
    assert m.paper_ps_choice(ti, tc, to) == "PS1"
    assert m.best_ps_choice(n, ti, tc, to) == "PS2"
    assert m.best_ps_choice(n, 0.2, 1.0, 0.3) == "PS1"


def test_classification_boundaries():
    assert m.classify(1.0, 1.0, 1.0) == "CI"
    assert m.classify(1.0001, 1.0, 1.0001) == "IOI"
    assert m.classify(2.0, 1.0, 0.5) == "INT"
    assert m.classify(0.5, 1.0, 2.0) == "INT"


def test_model_rejects_bad_parameters():
    with pytest.raises(ValueError):
        m.eq2_total_ci_ps1(0, 1, 1, 1)
    with pytest.raises(ValueError):
        m.eq3_total_ci_ps2(2, -1, 1, 1)
    with pytest.raises(ValueError):
        m.eq1_total_no_vt(2.5, 0, 0, 1, 1, 1)
    with pytest.raises(ValueError):
        des.enqueue_order("PS3", 2, 1, 1, 1)
