"""The LDS schedule of the SGEMM k-loop, restated as a sequence of tile
writes, fragment reads and barriers, checked for races on the CPU.

Within one barrier interval the waves of a workgroup run unsynchronised, so
a buffer that any wave writes in an interval must not be read (for a value
that is used) by any wave in the same interval, and a used read of tile t
from a buffer must find tile t there, written in an earlier interval.  Both
loops of `csrc/sgemm.hip` are restated here step by step (the two-buffer
loop, and the PIPE loop that reads the next k-tile's fragments during the
current MFMAs), for interior tiles (FAST: every step writes and reads,
the extra ones at the end unused) and edge tiles (conditional), over two
work units back to back as the persistent loop runs them.  The restated
PIPE loop without the barrier after its prologue's fragment read fails the
check, which is the race the mixed-size GPU test caught.
"""

import pytest

JUNK = None  # a tile past the last one: written or read, never used


def two_buffer_loop(ktiles, fast):
    """Events of one unit of the two-buffer loop: ("W", buf, tile),
    ("R", buf, tile) and ("B",)."""
    ev = [("W", 0, 0), ("B",)]
    for kt in range(ktiles):
        buf = kt & 1
        ev.append(("R", buf, kt))
        if fast or kt + 1 < ktiles:   # the next tile goes to the other buffer half-way
            ev.append(("W", buf ^ 1, kt + 1 if kt + 1 < ktiles else JUNK))
        ev.append(("B",))
    return ev


def pipe_loop(ktiles, fast, prologue_barrier=True):
    """Events of one unit of the PIPE loop."""
    ev = [("W", 0, 0)]
    if fast or ktiles > 1:
        ev.append(("W", 1, 1 if ktiles > 1 else JUNK))
    ev.append(("B",))
    ev.append(("R", 0, 0))
    if prologue_barrier:
        ev.append(("B",))
    for kt in range(ktiles):
        buf = kt & 1
        if fast or kt + 1 < ktiles:   # fragments of tile kt + 1
            ev.append(("R", buf ^ 1, kt + 1 if kt + 1 < ktiles else JUNK))
        if fast or kt + 2 < ktiles:   # tile kt + 2 into this step's buffer
            ev.append(("W", buf, kt + 2 if kt + 2 < ktiles else JUNK))
        ev.append(("B",))
    return ev


def races(events):
    """Problems of an event list: a used read in the same interval as a
    write of its buffer, or a used read that does not find its tile."""
    problems = []
    writes_in = {}     # interval -> buffers written in it
    interval = 0
    for e in events:
        if e[0] == "B":
            interval += 1
        elif e[0] == "W":
            writes_in.setdefault(interval, set()).add(e[1])
    held = {}          # buffer -> (tile, interval of the write)
    interval = 0
    for i, e in enumerate(events):
        if e[0] == "B":
            interval += 1
        elif e[0] == "W":
            held[e[1]] = (e[2], interval)
        elif e[0] == "R" and e[2] is not JUNK:
            tile, when = held.get(e[1], (None, None))
            if tile != e[2] or when is None or when >= interval:
                problems.append(("stale", i, e, tile, when, interval))
            if e[1] in writes_in.get(interval, set()):
                problems.append(("write in the read's interval", i, e, interval))
    return problems


@pytest.mark.parametrize("loop", [two_buffer_loop, pipe_loop])
@pytest.mark.parametrize("ktiles", [1, 2, 3, 4, 5, 8, 24])
def test_k_loops_have_no_lds_race(loop, ktiles):
    for fast in (False, True):
        if fast and ktiles % 2:   # the branch-free loop needs whole loop trips
            continue
        # two units back to back: the persistent loop's next prologue
        # follows the previous unit's last barrier
        ev = loop(ktiles, fast) + loop(ktiles, fast)
        assert races(ev) == [], (loop.__name__, ktiles, fast)


def test_pipe_loop_without_the_prologue_barrier_races():
    # tile 0's fragments are read after the prologue's barrier, and step 0
    # writes tile 2 into the same buffer in the same interval
    found = races(pipe_loop(8, True, prologue_barrier=False))
    assert any(p[0] == "write in the read's interval" and p[2] == ("R", 0, 0) for p in found), found


def test_the_check_catches_a_missing_step_barrier():
    # a pin for the checker itself: dropping one step barrier from the
    # two-buffer loop puts a write and a read of one buffer together
    ev = two_buffer_loop(6, True)
    step_barriers = [i for i, e in enumerate(ev) if e == ("B",)][1:]
    del ev[step_barriers[2]]
    assert races(ev)
