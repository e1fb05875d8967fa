"""Open-loop load generator for the GVM serving mode.

N rank processes replay seeded Poisson traces (``workloads.poisson_trace``):
each request arrives at its scheduled time whatever the state of the rank's
earlier requests, picks vector add, Black-Scholes or SGEMM uniformly, and
has a size drawn from that kernel's range.  Latency is measured from the
scheduled arrival to the moment the rank holds the result (so queueing in
the rank, in the manager and on the device all count).  The manager runs in
serving mode: continuous admission under an HBM budget with resident
per-rank buffers.

The same trace is replayed against the plain method (no virtualization):
``--plain-procs`` processes, each with its own device context, serve the
ranks' requests in arrival order with ``gvm_plain_run`` (allocate, copy in,
kernel, copy out, free per request).  One GPU allows only 16 processes on the
device at once, so the 64 ranks' traces are merged onto those processes.

    python -m paper_1511_07658_amd.loadgen --ranks 64 --rate 2000 --duration 10 --warmup 1

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

from . import gvm as G
from . import spmd
from . import workloads as wl

CONFIG = 5
MAX_VEC = 1 << 24
MAX_BS = 4 << 20
MAX_GEMM = 2048


def _now():
    return time.clock_gettime_ns(time.CLOCK_MONOTONIC)


class _Inputs:
    """Seeded pools of the largest request of each kernel; a request of size
    n uses their first n elements (same bytes in the GVM and plain runs)."""

    def __init__(self, rank):
        g = wl.generator(CONFIG, rank, 0)
        self.a = g.uniform(-1, 1, MAX_VEC).astype(np.float32)
        self.b = g.uniform(-1, 1, MAX_VEC).astype(np.float32)
        self.S = g.uniform(5, 30, MAX_BS).astype(np.float32)
        self.K = g.uniform(1, 100, MAX_BS).astype(np.float32)
        self.T = g.uniform(0.25, 10, MAX_BS).astype(np.float32)
        self.A = g.standard_normal(MAX_GEMM * MAX_GEMM, dtype=np.float32)
        self.B = g.standard_normal(MAX_GEMM * MAX_GEMM, dtype=np.float32)
        self.buf = np.empty(max(2 * MAX_VEC, 3 * MAX_BS, 2 * MAX_GEMM * MAX_GEMM), np.float32)

    def packed(self, k, n, b=None):
        """The packed input of a request (k, n), written into `b` (default:
        a private buffer) and returned as a view."""
        b = self.buf if b is None else b
        if k == G.GVM_K_VECADD:
            b[:n] = self.a[:n]
            b[n:2 * n] = self.b[:n]
            return b[:2 * n]
        if k == G.GVM_K_BLACKSCHOLES:
            b[:n] = self.S[:n]
            b[n:2 * n] = self.K[:n]
            b[2 * n:3 * n] = self.T[:n]
            return b[:3 * n]
        nn = n * n
        b[:nn] = self.A[:nn]
        b[nn:2 * nn] = self.B[:nn]
        return b[:2 * nn]


def _work(k, n):
    if k == G.GVM_K_SGEMM:
        return 2.0 * n ** 3, 12.0 * n * n
    if k == G.GVM_K_BLACKSCHOLES:
        return 0.0, 20.0 * n
    return float(n), 12.0 * n


def sampled(rank, index, k, n, every):
    """Whether request `index` of `rank` keeps a copy of its result for a
    later check: every `every`-th request of the rank (offset by the rank),
    when its result is at most 8 MiB."""
    return every > 0 and (index + rank) % every == 0 and out_bytes(k, n) <= (8 << 20)


def out_bytes(k, n):
    return G.out_elems(k, n) * 4


SMALL_BYTES = 8 << 20


def request_bytes(k, n):
    """Input and output bytes of a request (the manager's size classes)."""
    return (G.in_elems(k, n) + G.out_elems(k, n)) * 4


def gvm_rank(ns, rank, trace, start_box, warmup_s, barrier, zero_copy=True, slot_bytes=0, nslots=2, sample_every=0):
    """One open-loop rank against the manager; returns {"records": per-request
    (arrival offset s, kernel, n, latency s, status, stages), "samples":
    [(request index, kernel, n, result)] for the requests `sampled` picks}.

    With `zero_copy` the rank builds each input directly in its shared-memory
    space (`nslots` request slots of `slot_bytes` from gvm_rank_buffer) and
    takes the result there, so the API copies nothing on the rank side."""
    inp = _Inputs(rank)
    G.check(G.gvm_attach_ns(ns, rank), "attach")
    space = None
    free_slots = []
    if zero_copy:
        space = G.gvm_rank_buffer(rank, slot_bytes * nslots)
        if space is None:
            raise RuntimeError(f"rank {rank}: no zero-copy space: {G.gvm_last_error()}")
        per = slot_bytes // 4
        free_slots = [space[i * per:(i + 1) * per] for i in range(nslots)]
    barrier.wait()
    barrier.wait()  # the parent has written the common start time
    t0 = start_box.value
    pending = {}
    out = []
    samples = []
    i = 0
    while i < len(trace) or pending:
        now = _now()
        if i < len(trace) and now >= t0 + int(trace[i][0] * 1e9) and (free_slots or not zero_copy):
            ta, k, n = trace[i]
            if zero_copy:
                slot = free_slots.pop()
                ni, no = G.in_elems(k, n), G.out_elems(k, n)
                x = inp.packed(k, n, slot)
                o = slot[ni:ni + no]
            else:
                slot = None
                x = inp.packed(k, n)
                o = np.empty(G.out_elems(k, n), np.float32)
            t = G.gvm_submit(rank, k, x, o, n)
            if t < 0:
                out.append((ta, k, n, -1.0, int(t), None))
                if slot is not None:
                    free_slots.append(slot)
            else:
                pending[t] = (ta, k, n, slot, i, o)
            i += 1
            continue
        if not pending:
            time.sleep(max(0.0, (t0 + int(trace[i][0] * 1e9) - now) * 1e-9))
            continue
        # wait for a result; with a free slot only until the next arrival.
        # With every slot busy a due arrival waits in the rank (its latency
        # counts) and the rank blocks until a result frees a slot.
        if i < len(trace) and (free_slots or not zero_copy):
            wait_ns = t0 + int(trace[i][0] * 1e9) - now
        else:
            wait_ns = 60_000_000_000
        rc, t, ts = G.gvm_wait_any_timed(rank, max(wait_ns, 0))
        if rc == G.GVM_ETIMEDOUT:
            continue
        if t in pending:
            ta, k, n, slot, idx, o = pending.pop(t)
            if rc == 0 and sampled(rank, idx, k, n, sample_every):
                samples.append((idx, k, n, np.array(o, copy=True)))
            arrive = t0 + int(ta * 1e9)
            # arrival->submit (rank queue), submit->admit, admit->launch (copy-in),
            # launch->device done, device done->posted (copy-out)
            stages = (ts[0] - arrive, ts[1] - ts[0], ts[2] - ts[1], ts[3] - ts[2], ts[4] - ts[3]) if ts[4] else None
            out.append((ta, k, n, (_now() - t0) * 1e-9 - ta, rc, stages))
            if slot is not None:
                free_slots.append(slot)
        elif rc < 0:
            raise RuntimeError(f"rank {rank}: wait failed {rc}: {G.gvm_last_error()}")
    G.gvm_detach(rank)
    return {"records": out, "samples": samples}


def plain_proc(traces, start_box, barrier, rate_r, rate_v):
    """One plain process serving the merged traces of several ranks in
    arrival order (own context, no virtualization)."""
    reqs = sorted((ta, k, n, r) for r, tr in traces for (ta, k, n) in tr)
    pools = {r: _Inputs(r) for r, _ in traces}
    warm = np.zeros(8, np.float32)
    G.gvm_plain_run(G.GVM_K_VECADD, warm, warm[:4], 4)   # context created before the start
    barrier.wait()
    barrier.wait()
    t0 = start_box.value
    out = []
    for ta, k, n, r in reqs:
        now = _now()
        tgt = t0 + int(ta * 1e9)
        if now < tgt:
            time.sleep((tgt - now) * 1e-9)
        o = np.empty(G.out_elems(k, n), np.float32)
        rc, _ = G.gvm_plain_run(k, pools[r].packed(k, n), o, n, rate_r, rate_v)
        out.append((ta, k, n, (_now() - t0) * 1e-9 - ta, rc, None))
    return out


def summarize(records, warmup_s, duration_s):
    recs = [x for x in records if x[0] >= warmup_s]
    ok = [x for x in recs if x[4] == 0]
    lat = sorted(x[3] for x in ok)

    def pct(v, p):
        if not v:
            return None
        idx = max(1, int(np.ceil(p / 100.0 * len(v))))
        return round(v[idx - 1] * 1e3, 3)

    window = duration_s - warmup_s
    flop = sum(_work(x[1], x[2])[0] for x in ok)
    byts = sum(_work(x[1], x[2])[1] for x in ok)
    st = [x[5] for x in ok if x[5] is not None]
    stage_ms = None
    if st:
        names = ["rank_queue", "submit_to_admit", "admit_to_launch", "launch_to_device_done", "device_done_to_posted"]
        stage_ms = {nm: round(float(np.mean([s[i] for s in st])) * 1e-6, 3) for i, nm in enumerate(names)}
    per_kernel = {}
    for name, kid in (("vecadd", 1), ("blackscholes", 2), ("sgemm", 3)):
        lk = sorted(x[3] for x in ok if x[1] == kid)
        per_kernel[name] = {"count": len(lk), "p50_ms": pct(lk, 50), "p99_ms": pct(lk, 99)}
    # by size class: input and output together at most 8 MiB, or more
    per_size = {}
    for name, keep in (("small_le_8MiB", lambda b: b <= SMALL_BYTES), ("large", lambda b: b > SMALL_BYTES)):
        ls = sorted(x[3] for x in ok if keep(request_bytes(x[1], x[2])))
        per_size[name] = {"count": len(ls), "p50_ms": pct(ls, 50), "p99_ms": pct(ls, 99)}
    return {"requests": len(recs), "ok": len(ok), "failed": len(recs) - len(ok),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "max_ms": pct(lat, 100),
            "throughput_req_s": round(len(ok) / window, 2),
            "gemm_GFLOPs": round(flop / window / 1e9, 2), "algorithmic_GBs": round(byts / window / 1e9, 2),
            "per_kernel": per_kernel, "per_size": per_size, "mean_stage_ms": stage_ms}


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--ranks", type=int, default=64)
    ap.add_argument("--rate", type=float, default=2000.0, help="total requests per second")
    ap.add_argument("--duration", type=float, default=11.0, help="trace length (s), warm-up included")
    ap.add_argument("--warmup", type=float, default=1.0)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--plain-procs", type=int, default=16)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-threads", type=int, default=16, help="manager threads for shm <-> pinned staging copies")
    ap.add_argument("--copy-api", action="store_true",
                    help="ranks pass private buffers (the API copies them) instead of building in shared memory")
    ap.add_argument("--small-mib", type=int, default=8,
                    help="requests of at most this many MiB (input + output) form the manager's small class; "
                         "0: one class, first-come first-served throughout")
    ap.add_argument("--sample-every", type=int, default=0,
                    help="keep every k-th result of each rank (up to 8 MiB each) for a check after the run")
    ap.add_argument("--loopback", action="store_true", help=argparse.SUPPRESS)  # host-protocol dry run, no GPU
    return ap.parse_args(argv)


def run(a):
    """Replay the trace against the plain method (unless a.no_plain) and the
    GVM; returns (the result record, the sampled results per rank)."""
    if a.loopback:
        a.no_plain = True
    traces = wl.poisson_trace(CONFIG, a.ranks, a.rate, a.duration)
    spmd.prestart()
    ctx = spmd.context()
    r32, v32 = float(np.float32(wl.BS_RATE)), float(np.float32(wl.BS_VOLATILITY))
    result = {"config": {"small_class_MiB": a.small_mib, "ranks": a.ranks, "rank_buffers": "copied by the API" if a.copy_api else "zero-copy in shm", "rate_req_s": a.rate, "duration_s": a.duration, "warmup_s": a.warmup,
                         "budget_GiB": a.budget_gib, "copy_threads": a.copy_threads, "kernels": "vecadd n<=2^24, Black-Scholes n<=4M, SGEMM n<=2048",
                         "requests_in_trace": sum(len(t) for t in traces)}}

    # plain first: this process must not touch the GPU before forking them
    if not a.no_plain:
        P = min(a.plain_procs, 16)
        groups = [[(r, traces[r]) for r in range(a.ranks) if r % P == p] for p in range(P)]
        start = ctx.Value("q", 0)
        bar = ctx.Barrier(P + 1)
        res = {}

        def run_plain():
            res["r"] = spmd.run_processes(plain_proc, [(g, start, bar, r32, v32) for g in groups],
                                          timeout_s=a.duration * 20 + 300)

        th = threading.Thread(target=run_plain)
        th.start()
        bar.wait()
        start.value = _now() + 200_000_000
        bar.wait()
        th.join()
        recs = [x for part in res["r"] for x in part]
        result["plain"] = {"processes": P, **summarize(recs, a.warmup, a.duration)}
        print(f"[loadgen] plain done: {result['plain']['p50_ms']} / {result['plain']['p99_ms']} ms", file=sys.stderr,
              flush=True)

    ns = f"gvm.serve.{os.getpid()}"
    slot = (2 * MAX_VEC + MAX_VEC) * 4                    # the largest request: vector add of 2^24, in + out
    space = slot * 2 + (1 << 20)                          # two requests in flight per rank
    cfg = G.gvm_config_default(nranks=a.ranks, shm_bytes_per_rank=space, staging_bytes=(3 * MAX_VEC) * 4 + (1 << 20),
                               hbm_budget_bytes=int(a.budget_gib * (1 << 30)), mode=G.GVM_MODE_SERVING,
                               policy=G.GVM_POLICY_AUTO, max_inflight=0, copy_threads=a.copy_threads, name=ns,
                               small_request_bytes=a.small_mib << 20,
                               backend=G.GVM_BACKEND_LOOPBACK if a.loopback else G.GVM_BACKEND_HIP)
    start = ctx.Value("q", 0)
    bar = ctx.Barrier(a.ranks + 1)
    G.check(G.gvm_init(cfg), "gvm_init")
    try:
        res = {}

        def run_gvm():
            res["r"] = spmd.run_processes(
                gvm_rank, [(ns, r, traces[r], start, a.warmup, bar, not a.copy_api, slot, 2, a.sample_every)
                           for r in range(a.ranks)],
                timeout_s=a.duration * 20 + 300)

        th = threading.Thread(target=run_gvm)
        th.start()
        bar.wait()
        G.gvm_stats_reset()
        cpu0 = os.times()
        start.value = _now() + 200_000_000
        bar.wait()
        th.join()
        cpu1 = os.times()
        stats = G.gvm_stats_json()
    finally:
        G.gvm_shutdown()
    recs = [x for part in res["r"] for x in part["records"]]
    samples = {r: part["samples"] for r, part in enumerate(res["r"])}
    result["gvm"] = {**summarize(recs, a.warmup, a.duration), "peak_device_bytes": stats["peak_device_bytes"],
                     "admit_wait_us": stats["admit_wait_us"],
                     "device_ms": {k: v["device_ms"] for k, v in stats["kernels"].items()},
                     "launches": {k: v["launches"] for k, v in stats["kernels"].items()},
                     "ring_us": stats["ring_us"], "busy_iteration_us": stats["busy_iteration_us"],
                     # CPU time of the manager's process (service thread, copy workers), whole run
                     "host": {**stats["host"],
                              "manager_process_cpu_s": round(cpu1.user + cpu1.system - cpu0.user - cpu0.system, 3)}}
    if "plain" in result and result["plain"]["p99_ms"] and result["gvm"]["p99_ms"]:
        result["p99_plain_over_gvm"] = round(result["plain"]["p99_ms"] / result["gvm"]["p99_ms"], 3)
        result["throughput_gvm_over_plain"] = round(result["gvm"]["throughput_req_s"] /
                                                    max(result["plain"]["throughput_req_s"], 1e-9), 3)
    result["gvm"]["sampled_results"] = sum(len(v) for v in samples.values())
    return result, samples


def main(argv=None):
    result, _ = run(parse_args(argv))
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
