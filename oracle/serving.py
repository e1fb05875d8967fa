"""Checks of a serving run (test infrastructure only; see package header).

The paper's manager serves one barrier-synchronised batch at a time
(Section 5).  The serving mode of this project keeps the manager's resources
of Section 5 (one context, per-process device memory objects whose total must
fit the GPU memory) but admits requests continuously.  What must hold of such
a run is stated here as plain checks over its event log, and the latency
statistics are defined here once:

* memory: the device bytes held by admitted, not yet completed requests never
  exceed the budget (Section 5: the per-process memory spaces are sized so
  that their total does not exceed the GPU memory);
* completeness: every submitted ticket is admitted exactly once and completed
  exactly once, and never completes before it is admitted;
* order: admission is first-come first-served per kernel queue, i.e. tickets
  are admitted in submission order.

Percentiles use the nearest-rank definition: the p-th percentile of ``m``
sorted samples is the sample of rank ``ceil(p/100 * m)`` (1-based).
"""

from __future__ import annotations

import math

__all__ = ["check_budget", "check_lifecycle", "check_fifo", "percentile_nearest_rank"]


def check_budget(events, budget_bytes):
    """``events``: iterable of ``(t, kind, ticket, nbytes)`` with ``kind`` in
    {"admit", "complete"}.  Returns the peak resident bytes; raises
    AssertionError if it ever exceeds ``budget_bytes``.  Events at the same
    instant release before they admit."""
    order = {"complete": 0, "admit": 1}
    held = {}
    resident = 0
    peak = 0
    for t, kind, ticket, nbytes in sorted(events, key=lambda e: (e[0], order[e[1]])):
        if kind == "admit":
            held[ticket] = nbytes
            resident += nbytes
        elif kind == "complete":
            resident -= held.pop(ticket)
        else:
            raise ValueError(f"unknown event kind {kind!r}")
        if resident > budget_bytes:
            raise AssertionError(f"resident {resident} B > budget {budget_bytes} B at t={t}")
        peak = max(peak, resident)
    return peak


def check_lifecycle(submitted, events):
    """Every ticket in ``submitted`` is admitted once and completed once,
    completion not before admission; no unknown tickets."""
    admit = {}
    done = {}
    for t, kind, ticket, _ in events:
        table = admit if kind == "admit" else done
        if ticket in table:
            raise AssertionError(f"ticket {ticket} {kind} twice")
        table[ticket] = t
    want = set(submitted)
    if set(admit) != want:
        raise AssertionError("admitted tickets differ from submitted tickets")
    if set(done) != want:
        raise AssertionError("completed tickets differ from submitted tickets")
    for k in want:
        if done[k] < admit[k]:
            raise AssertionError(f"ticket {k} completed before it was admitted")


def check_fifo(submission_order, admission_order):
    """Tickets are admitted in the order they were submitted."""
    if list(submission_order) != list(admission_order):
        raise AssertionError("admission order differs from submission order")


def percentile_nearest_rank(samples, p):
    """Nearest-rank percentile, ``0 < p <= 100``."""
    xs = sorted(samples)
    if not xs:
        raise ValueError("no samples")
    if not (0 < p <= 100):
        raise ValueError("p must be in (0, 100]")
    rank = max(1, math.ceil(p / 100.0 * len(xs)))
    return xs[rank - 1]
