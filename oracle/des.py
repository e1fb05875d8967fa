"""Discrete-event schedule of the stream rules of Section 4.2.1
(test infrastructure only; see package header).

This is the brute-force side of the execution model: instead of a closed
form, it replays the enqueue order of a programming style operation by
operation under the paper's hardware rules and reports when the last
operation ends.  On the cases the closed forms cover it must reproduce
Eq. 2, Eq. 3, Eq. 4 and Eq. 7 exactly.

Operations
----------
Each of the ``N`` streams carries three operations, "send" (host to device,
T_data_in), "comp" (the kernel, T_comp) and "rtrv" (device to host,
T_data_out), with the data dependencies send -> comp -> rtrv of one stream
(Section 4.2.1: no dependencies across streams of an SPMD program).

Enqueue orders (the two programming styles of Section 4.2.1)
------------------------------------------------------------
* PS-1: all sends, then all kernels, then all retrieves (three loops).
* PS-2: per stream, send, kernel, retrieve (one loop).

Rules ("paper" rule set, the Fermi model of Section 4.2.1 / 4.2.3)
------------------------------------------------------------------
1. Stream order: an operation starts after the previous operation of its
   stream has ended.
2. A single-direction transfer takes the whole link, so the sends are served
   one at a time, and so are the retrieves, each in enqueue order; a send
   and a retrieve may overlap (concurrency type (c)).
3. The GPU holds every kernel at once: kernels never wait for each other
   except through rules 4 and 5 (assumption of Section 4.2.3).
4. A retrieve that checks for the end of a kernel waits until every kernel
   enqueued before it in the single hardware work queue has ended.
5. That check blocks every kernel enqueued after the retrieve until the
   check is satisfied (the condition of rule 4 holds).

Reading: the text says a retrieve may start "when all prior kernel launches
have started executing" yet derives Eq. 2 from a retrieve that begins after
the last kernel; rule 4 takes the reading that reproduces the printed
equations.

The "multiqueue" rule set drops rules 4 and 5 (independent hardware queues
with no false dependencies between streams) and keeps 1 to 3.

Because every constraint of an operation refers to operations enqueued
before it, one pass in enqueue order computes every start time exactly.
"""

from __future__ import annotations

from dataclasses import dataclass

__all__ = ["Op", "enqueue_order", "schedule", "makespan", "simulate"]

SEND, COMP, RTRV = "send", "comp", "rtrv"


@dataclass(frozen=True)
class Op:
    stream: int
    kind: str  # "send" | "comp" | "rtrv"
    duration: float


def enqueue_order(style, n, t_in, t_comp, t_out):
    """Operations of ``n`` streams in the enqueue order of ``style``
    ("PS1" or "PS2", the two listings of Section 4.2.1)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    if style == "PS1":
        return (
            [Op(i, SEND, t_in) for i in range(n)]
            + [Op(i, COMP, t_comp) for i in range(n)]
            + [Op(i, RTRV, t_out) for i in range(n)]
        )
    if style == "PS2":
        ops = []
        for i in range(n):
            ops += [Op(i, SEND, t_in), Op(i, COMP, t_comp), Op(i, RTRV, t_out)]
        return ops
    raise ValueError("style must be 'PS1' or 'PS2'")


def schedule(ops, rules="paper"):
    """Start and end time of every operation of ``ops`` (in enqueue order)."""
    if rules not in ("paper", "multiqueue"):
        raise ValueError("rules must be 'paper' or 'multiqueue'")
    false_deps = rules == "paper"
    stream_end = {}          # rule 1: end of the last op of each stream
    send_free = 0.0          # rule 2: link host->device free from
    rtrv_free = 0.0          # rule 2: link device->host free from
    kernel_ends = []         # ends of kernels enqueued so far (rule 4)
    kernel_gate = 0.0        # rule 5: earliest start of later kernels
    times = []
    for op in ops:
        start = stream_end.get(op.stream, 0.0)
        if op.kind == SEND:
            start = max(start, send_free)
        elif op.kind == COMP:
            if false_deps:
                start = max(start, kernel_gate)
        elif op.kind == RTRV:
            start = max(start, rtrv_free)
            if false_deps and kernel_ends:
                check = max(kernel_ends)
                start = max(start, check)
                kernel_gate = max(kernel_gate, check)
        else:
            raise ValueError(f"unknown op kind {op.kind!r}")
        end = start + op.duration
        if op.kind == SEND:
            send_free = end
        elif op.kind == RTRV:
            rtrv_free = end
        else:
            kernel_ends.append(end)
        stream_end[op.stream] = end
        times.append((start, end))
    return times


def makespan(times):
    return max((e for _, e in times), default=0.0)


def simulate(style, n, t_in, t_comp, t_out, rules="paper"):
    """Total time for ``n`` virtualised processes under ``style``."""
    return makespan(schedule(enqueue_order(style, n, t_in, t_comp, t_out), rules))
