"""Benchmark of the GVM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mixed32|sgemm8|vecadd4|vecadd16|bs16|ep8]

Default workload: 32 SPMD rank processes with uneven sizes, served by one GVM
manager on device 0 -- 16 FP32 vector adds with n = floor(2^U[16,24]) and 16
FP32 SGEMMs with n drawn from {256, ..., 2048} step 64, seeded by rank.  One
step is every row of the method's hot path: each rank submits its request
through the shared-memory rings (its input already built in its
shared-memory space), the manager gathers the batch at its request barrier,
copies every input to HBM, runs one grouped launch per kernel class, copies
every result back, and every rank receives its completion with the result in
its shared memory.  ``value`` is the SGEMM GFLOP/s of those whole steps,
copies included (the vector adds' GB/s go beside it).

Beside it:
* ``device_phase`` / ``roofline``: the same requests with inputs and results
  left resident in HBM (GVM_F_IN_RESIDENT | GVM_F_OUT_RESIDENT), so a step is
  the manager round trip plus the kernels; the dominant kernel's roofline
  fraction comes from device events around its launches, timed after about
  60 ms of untimed resident steps (the engine clock's climb to its plateau
  under load);
* ``plain*``: the plain per-process method (own context, pageable copies,
  allocate / free per request; Eq. 1 path) in three variants; above 16 ranks
  the ranks are dealt round robin onto 16 processes, each running its ranks'
  requests one after another;
* ``serving``: a short run of the serving configuration (64 open-loop ranks,
  Poisson arrivals at 2000 requests/s) with its p50 / p99 latency;
* ``cpu_baseline``: the plain C oracle run SPMD on the host cores (one
  process per rank, at most 16) over a bounded sample; ``cpu_baseline_python``
  the Python oracle (a float64 library matmul) on one process.

Prints ONE JSON line.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import platform
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1511_07658_amd import gvm as G  # noqa: E402
from paper_1511_07658_amd import spmd  # noqa: E402
from paper_1511_07658_amd import workloads as wl  # noqa: E402

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0
MAX_GPU_PROCESSES = 16

# EP-like kernel.  Its roofline counts the method's binary64 operations per
# generated pair (the definition in include/gvm.h, each of log, sqrt and
# divide as one operation): scaling both words to [0, 1) (2), x = 2u - 1 and
# y = 2v - 1 (4), t = x^2 + y^2 (3); for an accepted pair (probability pi/4):
# ln t, -2 ln t / t, the square root, X and Y, the two sums and max(|X|, |Y|)
# (9).  Against the chip's binary64 vector peak; the counter-based generator's
# 64-bit integer products, which dominate the kernel, are not in the count.
EP_FP64_OPS_PER_PAIR = 9.0 + math.pi / 4.0 * 9.0
# VALU issue utilisation of the compiled kernel (a diagnostic of the code,
# not a roofline): the unit loop of csrc/ep_kernels.hip issues 602 wave64
# VALU instructions per Philox block (2 pairs per lane, both accepted), one
# per 4 cycles per SIMD: 4 * 602 / 128 SIMD cycles per pair.
EP_SIMD_CYCLES_PER_PAIR = 4.0 * 602 / 128
EP_ISSUE_GPAIRS = 256 * 4 * 2.4e9 / EP_SIMD_CYCLES_PER_PAIR / 1e9

# HBM bytes per launch of the dominant kernel from rocprofv3 --pmc FETCH_SIZE /
# WRITE_SIZE (KiB per dispatch), each scaled by what the counter reads for a
# plain 1 GiB copy (fetch x2.000, write x1.000); valid only for the kernel
# sources they were taken on (sha256 over `sources` in csrc/, in order;
# profiles/mixed32_uneven.md, profiles/sgemm_grouped_8x1024.md,
# profiles/blackscholes_grouped_16x4M.md, profiles/vecadd_grouped_16x16M.md).
SGEMM_SOURCES = ("sgemm.hip", "group_device.hpp", "kernels.hpp", "gemm_tiles.inc", "gemm_balance.hpp")
STREAM_SOURCES = ("stream_kernels.hip", "group_device.hpp", "kernels.hpp")
MEASURED_TRAFFIC = {
    "mixed32": {"sources": SGEMM_SOURCES, "kernels_sha256": "3d2c051e13bf44668076478faae892d99794840189aad7e4a9d42bb5e104c64e",
                "fetch_kib": 459439.1, "fetch_factor": 2.000, "write_kib": 85152.0, "write_factor": 1.000},
    "sgemm8": {"sources": SGEMM_SOURCES, "kernels_sha256": "3d2c051e13bf44668076478faae892d99794840189aad7e4a9d42bb5e104c64e",
               "fetch_kib": 32838.3, "fetch_factor": 2.000, "write_kib": 32768.0, "write_factor": 1.000},
    "bs16": {"sources": STREAM_SOURCES, "kernels_sha256": "8fe15074feb50f84a1329d139469e3f76e1f9b34fe8eeb59000d99b7b62abbab",
             "fetch_kib": 393326.6, "fetch_factor": 2.000, "write_kib": 524300.7, "write_factor": 1.000},
    "vecadd16": {"sources": STREAM_SOURCES, "kernels_sha256": "8fe15074feb50f84a1329d139469e3f76e1f9b34fe8eeb59000d99b7b62abbab",
                 "fetch_kib": 1048597.1, "fetch_factor": 2.000, "write_kib": 1048576.0, "write_factor": 1.000},
}


def sources_sha256(sources):
    import hashlib

    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_1511_07658_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload):
    """Traffic in bytes per launch, or None if the kernel source changed since
    the counters were taken."""
    m = MEASURED_TRAFFIC.get(workload)
    if not m or sources_sha256(m["sources"]) != m["kernels_sha256"]:
        return None
    return round((m["fetch_kib"] * m["fetch_factor"] + m["write_kib"] * m["write_factor"]) * 1024)


WORKLOADS = {
    "mixed32": "32 ranks via GVM with uneven sizes: 16 FP32 vector adds n=floor(2^U[16,24]) and 16 FP32 SGEMMs "
               "n in {256..2048 step 64}, tuned tiles, one grouped launch per kernel class per step; "
               "inputs from the ranks' shared memory, copies to and from HBM in every step",
    "sgemm8": "8 ranks via GVM, FP32 SGEMM 1024x1024 each, grouped MFMA launch; copies in every step",
    "vecadd4": "4 ranks via GVM, FP32 vector add n=2^20 each; copies in every step",
    "vecadd16": "16 ranks via GVM, FP32 vector add n=2^24 each (3.2 GB per step, beyond the memory-side cache), "
                "one grouped launch; copies in every step",
    "bs16": "16 ranks via GVM, FP32 Black-Scholes 4M options each, one fused launch; copies in every step",
    "ep8": "8 ranks via GVM, EP-like Gaussian-pair tally of 2^24 pairs each (the size of the paper's EP(M24)), "
           "one grouped launch plus a per-request reduction",
}


def rank_specs(workload):
    """Per-rank (kernel id, n, config index of the seeded inputs)."""
    if workload == "sgemm8":
        return [(G.GVM_K_SGEMM, 1024, 1)] * 8
    if workload == "vecadd4":
        return [(G.GVM_K_VECADD, 1 << 20, 0)] * 4
    if workload == "vecadd16":
        return [(G.GVM_K_VECADD, 1 << 24, 0)] * 16
    if workload == "bs16":
        return [(G.GVM_K_BLACKSCHOLES, 4 << 20, 2)] * 16
    if workload == "ep8":
        return [(G.GVM_K_EP, 1 << 24, 4)] * 8
    if workload == "mixed32":
        return ([(G.GVM_K_VECADD, n, 3) for n in wl.uneven_vecadd_sizes(3, 16)] +
                [(G.GVM_K_SGEMM, n, 3) for n in wl.uneven_sgemm_sizes(3, 16)])
    raise ValueError(workload)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def work_of(kernel_id, n):
    """Algorithmic FLOP and HBM bytes of one request."""
    if kernel_id == G.GVM_K_SGEMM:
        return 2.0 * n ** 3, 12.0 * n * n
    if kernel_id == G.GVM_K_BLACKSCHOLES:
        return 0.0, 20.0 * n
    if kernel_id == G.GVM_K_EP:
        return 0.0, 112.0   # the work is its n pairs (ALU), not bytes
    return float(n), 12.0 * n


def resident_warmup_steps(specs, target_ms=60.0):
    """Resident warm-up steps that keep the device busy for about `target_ms`
    before the timed resident steps.  Under a sustained load the engine clock
    climbs for about 20 ms from where a mostly idle device left it (2.1-2.3
    GHz, after the copy-bound leg) to its plateau (2.37-2.46 GHz); timing
    before the plateau measures the clock ramp, not the kernel.  The step
    time is estimated from the algorithmic work at sustained rates (FP32
    MFMA 110 TFLOP/s, HBM 5 TB/s, 120 G EP pairs/s) plus 50 us per step."""
    us = 50.0
    for k, n, _ in specs:
        flop, nbytes = work_of(k, n)
        if k == G.GVM_K_SGEMM:
            us += flop / 110e6
        elif k == G.GVM_K_EP:
            us += n / 120e3
        else:
            us += nbytes / 5e6
    return max(3, min(5000, int(math.ceil(target_ms * 1e3 / us))))


def pct(v, p):
    if not len(v):
        return None
    v = sorted(v)
    return v[max(1, int(math.ceil(p / 100.0 * len(v)))) - 1]


# ----------------------------------------------------------------- rank side

def bench_rank(ns, rank, kernel_id, n, cfg_idx, warmup, steps, res_warmup, res_steps, barrier):
    """One SPMD rank process.  Its input is built once in its shared-memory
    space; then warm-up and timed steps with every copy (the manager moves
    the input to HBM and the result back into shared memory), then steps on
    the inputs left resident in HBM.  Returns CLOCK_MONOTONIC stamps."""
    x = spmd.make_input(kernel_id, cfg_idx, rank, n)
    nout = G.out_elems(kernel_id, n)
    G.check(G.gvm_attach_ns(ns, rank), "attach")
    view = G.gvm_rank_buffer(rank, (x.size + nout) * 4)
    if view is None:
        raise RuntimeError(f"rank {rank}: no zero-copy space: {G.gvm_last_error()}")
    xin, oview = view[:x.size], view[x.size:x.size + nout]
    xin[:] = x
    lib = G.lib()
    submit_ex, wait_timed = lib.gvm_submit_ex, lib.gvm_wait_timed
    ts = (ctypes.c_uint64 * 5)()
    clock, mono = time.clock_gettime_ns, time.CLOCK_MONOTONIC
    barrier.wait()                       # 1: attached, inputs in place
    for _ in range(max(warmup, 1)):
        t = G.check(G.gvm_submit(rank, kernel_id, xin, oview, n), "warm-up")
        G.check(G.gvm_wait(rank, t, 120_000_000_000), "warm-up wait")
    first = spmd.digest(oview)
    barrier.wait()                       # 2: warm-up done
    barrier.wait()                       # 3: statistics reset, go

    def timed(nsteps, flags, inp, outp):
        parts = [0, 0, 0, 0, 0, 0]
        stamps = []                      # per step: submit, admit, posted, seen (ns)
        t0 = clock(mono)
        seen = t0
        for _ in range(nsteps):
            t = submit_ex(rank, kernel_id, inp, outp, n, flags)
            if t < 0:
                G.check(t, "step")
            st = wait_timed(rank, t, 120_000_000_000, ts)
            if st != 0:
                G.check(st, "step wait")
            now = clock(mono)
            # submit->admit, admit->launch, launch->device done, device->posted, posted->seen, seen->next submit
            parts[0] += ts[1] - ts[0]
            parts[1] += ts[2] - ts[1]
            parts[2] += ts[3] - ts[2]
            parts[3] += ts[4] - ts[3]
            parts[4] += now - ts[4]
            parts[5] += ts[0] - seen
            stamps.append((ts[0], ts[1], ts[4], now))
            seen = now
        return {"t0": t0, "t1": clock(mono), "parts_ns": [p / max(nsteps, 1) for p in parts], "stamps": stamps}

    e2e = timed(steps, 0, xin.ctypes.data, oview.ctypes.data)
    same = spmd.digest(oview) == first
    barrier.wait()                       # 4: timed steps done
    barrier.wait()                       # 5: statistics read
    flags = G.GVM_F_IN_RESIDENT | G.GVM_F_OUT_RESIDENT
    for _ in range(res_warmup):
        t = G.check(G.gvm_submit_ex(rank, kernel_id, None, None, n, flags), "resident warm-up")
        G.check(G.gvm_wait(rank, t, 120_000_000_000), "resident warm-up wait")
    barrier.wait()                       # 6: resident warm-up done
    barrier.wait()                       # 7: statistics reset, go
    res = timed(res_steps, flags, None, None)
    barrier.wait()                       # 8: resident steps done
    G.gvm_detach(rank)
    return {"e2e": e2e, "resident": res, "same_bytes": same, "digest": first}


def step_detail(runs):
    """Across ranks, per timed step: spread of the submit times, spread of
    the completion posts, and the gap from the previous step's last post to
    this step's first submit (means, us), plus how often each rank submitted
    last (the one the request barrier waits for)."""
    st = np.array([r["stamps"] for r in runs], dtype=np.float64)   # ranks x steps x 4
    if st.ndim != 3 or st.shape[1] < 2:
        return None
    sub, post = st[:, :, 0], st[:, :, 2]
    last = np.bincount(np.argmax(sub, axis=0), minlength=st.shape[0])
    return {"submit_spread": round(float(np.mean(sub.max(0) - sub.min(0))) * 1e-3, 2),
            "post_spread": round(float(np.mean(post.max(0) - post.min(0))) * 1e-3, 2),
            "last_post_to_first_submit": round(float(np.mean(sub.min(0)[1:] - post.max(0)[:-1])) * 1e-3, 2),
            "last_post_to_last_submit": round(float(np.mean(sub.max(0)[1:] - post.max(0)[:-1])) * 1e-3, 2),
            "last_submitter_counts": last.tolist()}


def leg_summary(runs, steps):
    """Whole-job time of a leg (first start to last end over the ranks), the
    request latency percentiles (submit to seen, us) and the mean stage
    breakdown."""
    elapsed = (max(r["t1"] for r in runs) - min(r["t0"] for r in runs)) * 1e-9
    lat = [(s[3] - s[0]) * 1e-3 for r in runs for s in r["stamps"]]
    return elapsed, {
        "ms_per_step": round(elapsed / max(steps, 1) * 1e3, 4),
        "latency_us": {"p50": round(pct(lat, 50), 2), "p99": round(pct(lat, 99), 2), "count": len(lat)},
        "step_breakdown_us": dict(zip(
            ["barrier_and_drain", "admit_to_launch", "launch_to_device_done", "device_done_to_posted",
             "posted_to_seen", "rank_loop"],
            [round(float(x) * 1e-3, 2) for x in np.mean([r["parts_ns"] for r in runs], axis=0)])),
        "step_detail_us": step_detail(runs),
    }


PLAIN_WARM_N = {G.GVM_K_VECADD: 4096, G.GVM_K_VECMUL: 4096, G.GVM_K_BLACKSCHOLES: 4096, G.GVM_K_SGEMM: 64,
                G.GVM_K_EP: 4096}


def plain_proc(jobs, barrier, warm=False, baton=None):
    """One process of the plain method (no virtualization): its own device
    context, pageable copies, the same kernel code objects (Section 4.1).
    `jobs` = [(rank, kernel id, n, config index)], run one after another.

    Variants of the baseline:
    * cold (default): the context is created inside the timed region, by the
      process's first request, as in the paper's turnaround (T_init included);
    * ``warm``: a small request of the first job's kernel runs before the
      start barrier, so context creation and code-object loading fall outside;
    * ``baton`` (a shared turn counter and its condition): the GPU phases run
      one after another in rank order, the sequential execution that Eq. 1
      models, instead of letting the device's scheduler interleave them."""
    inputs = {r: spmd.make_input(k, c, r, n) for r, k, n, c in jobs}
    G.lib()
    args = (float(np.float32(wl.BS_RATE)), float(np.float32(wl.BS_VOLATILITY)))
    if warm:
        r0, k0, _, c0 = jobs[0]
        m = PLAIN_WARM_N[k0]
        wx = spmd.make_input(k0, c0, r0, m)
        wo = np.empty(G.out_elems(k0, m), np.float32)
        rc, _ = G.gvm_plain_run(k0, wx, wo, m, *args)
        if rc != 0:
            return {"rc": rc, "t0": 0, "t1": 0, "stages": [], "digests": {}}
    barrier.wait()
    t0 = time.clock_gettime_ns(time.CLOCK_MONOTONIC)
    stages, digests, worst = [], {}, 0
    for r, k, n, c in jobs:
        out = np.empty(G.out_elems(k, n), np.float32)
        if baton is not None:
            turn, cond = baton
            with cond:
                cond.wait_for(lambda: turn.value == r)
        rc, st = G.gvm_plain_run(k, inputs[r], out, n, *args)
        if baton is not None:
            with cond:
                turn.value += 1
                cond.notify_all()
        worst = worst or rc
        stages.append(st)
        digests[r] = spmd.digest(out)
    t1 = time.clock_gettime_ns(time.CLOCK_MONOTONIC)
    return {"rc": worst, "t0": t0, "t1": t1, "stages": stages, "digests": digests}


# ----------------------------------------------------------------- main

def cpu_baseline(specs, main_kernel, budget_s=10.0):
    """The oracle as it stands, on this host's cores, over a bounded sample of
    the same workload: the workload's requests of its main kernel, cycled,
    for about `budget_s` seconds."""
    from oracle import ep as oe
    from oracle import kernels as ok

    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    reqs = [(r, n, c) for r, (k, n, c) in enumerate(specs) if k == main_kernel]
    if main_kernel == G.GVM_K_EP:
        sample = min(reqs[0][1], 1 << 20)   # a bounded slice of each rank's pair stream
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            r, _, c = reqs[done % len(reqs)]
            oe.ep_reference(wl.ep_key(c, r), sample)
            done += 1
        el = time.perf_counter() - t0
        return {"value": round(done * sample / el / 1e9, 6), "unit": "Gpairs/s", "cores": 1, "kind": "oracle",
                "sample": f"{done} slices of {sample} pairs through oracle.ep.ep_reference in {el:.1f} s "
                          f"(the first {sample} pairs of the ranks' keys, cycled)"}
    cache = {}
    done = flop = byts = 0.0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        r, n, c = reqs[int(done) % len(reqs)]
        if (r, n) not in cache and len(cache) < 8:
            if main_kernel == G.GVM_K_SGEMM:
                cache[(r, n)] = wl.sgemm_inputs(c, r, n)
            elif main_kernel == G.GVM_K_BLACKSCHOLES:
                cache[(r, n)] = wl.bs_inputs(c, r, n)
            else:
                cache[(r, n)] = wl.vecadd_inputs(c, r, n)
        args = cache.get((r, n))
        if args is None:   # beyond the input cache: reuse the first request's inputs at its own size
            r, n, c = reqs[0]
            args = cache[(r, n)]
        if main_kernel == G.GVM_K_SGEMM:
            ok.sgemm_f64(*args)
        elif main_kernel == G.GVM_K_BLACKSCHOLES:
            ok.black_scholes_f64(*args, wl.BS_RATE, wl.BS_VOLATILITY)
        else:
            ok.vecadd_f32(*args)
        f, b = work_of(main_kernel, n)
        flop += f
        byts += b
        done += 1
    el = time.perf_counter() - t0
    if main_kernel == G.GVM_K_SGEMM:
        value, unit = flop / el / 1e9, "GFLOP/s"
    else:
        value, unit = byts / el / 1e9, "GB/s"
    kname = {1: "vecadd_f32", 2: "black_scholes_f64", 3: "sgemm_f64"}[main_kernel]
    return {"value": round(value, 3), "unit": unit, "cores": threads, "kind": "oracle",
            "sample": f"{int(done)} requests through oracle.kernels.{kname} in {el:.1f} s (the workload's "
                      f"{len(reqs)} requests of this kernel, sizes {sorted({n for _, n, _ in reqs})}, cycled)"}


def c_oracle_rank(kernel_id, cfg_idx, rank, n, budget_s):
    """One SPMD process of the C oracle's CPU baseline: the plain C oracle
    (oracle/liboracle.so) on this rank's request, repeated (SGEMM: eight rows
    of C at a time, cycling over the rows) for about `budget_s` seconds.
    Returns the algorithmic work done and the time taken."""
    from oracle import c_oracle as co

    lib = co.load()
    t0 = time.perf_counter()
    flop = byts = 0.0
    if kernel_id == G.GVM_K_SGEMM:
        A, B = wl.sgemm_inputs(cfg_idx, rank, n)
        row = 0
        while time.perf_counter() - t0 < budget_s:
            rows = min(8, n - row)
            co.sgemm_rows_f64(A, B, row, rows, lib=lib)
            flop += 2.0 * rows * n * n
            row = (row + rows) % n
    elif kernel_id == G.GVM_K_BLACKSCHOLES:
        S, K, T = wl.bs_inputs(cfg_idx, rank, n)
        while time.perf_counter() - t0 < budget_s:
            co.black_scholes_f64(S, K, T, wl.BS_RATE, wl.BS_VOLATILITY, lib=lib)
            byts += 20.0 * n
    else:
        a, b = wl.vecadd_inputs(cfg_idx, rank, n)
        while time.perf_counter() - t0 < budget_s:
            co.vecadd_f32(a, b, lib=lib)
            byts += 12.0 * n
    return {"flop": flop, "bytes": byts, "elapsed": time.perf_counter() - t0}


def cpu_baseline_c(ctx, specs, main_kernel, budget_s=10.0):
    """The plain C oracle run SPMD on the host's cores, as the paper runs its
    SPMD programs: one process per rank of the main kernel (at most 16, the
    host share of the box), each repeating its own request (SGEMM: a slice of
    rows of C) for about `budget_s` seconds."""
    reqs = [(r, n, c) for r, (k, n, c) in enumerate(specs) if k == main_kernel]
    procs = min(len(reqs), MAX_GPU_PROCESSES, os.cpu_count() or 1)
    res = spmd.run_processes(c_oracle_rank, [(main_kernel, c, r, n, budget_s) for r, n, c in reqs[:procs]],
                             timeout_s=budget_s * 4 + 120)
    el = max(x["elapsed"] for x in res)
    if main_kernel == G.GVM_K_SGEMM:
        value, unit, what = sum(x["flop"] for x in res) / el / 1e9, "GFLOP/s", "rows of C through ref_sgemm_rows_f64"
    else:
        value, unit = sum(x["bytes"] for x in res) / el / 1e9, "GB/s"
        what = "whole requests through " + ("ref_bs_f64" if main_kernel == G.GVM_K_BLACKSCHOLES else "ref_vecadd_f32")
    return {"value": round(value, 3), "unit": unit, "cores": procs, "kind": "oracle",
            "sample": f"plain C oracle (oracle/liboracle.so, gcc -O2), SPMD: {procs} processes, one per rank of the "
                      f"workload's {len(reqs)} requests of this kernel, each repeating its own request ({what}) for "
                      f"{budget_s:.0f} s; sizes {sorted(n for _, n, _ in reqs[:procs])}"}


def run_plain(ctx, specs, warm=False, seq=False, flop_total=0.0, bytes_total=0.0, unit="GFLOP/s"):
    nranks = len(specs)
    nproc = min(nranks, MAX_GPU_PROCESSES)
    groups = [[(r, k, n, c) for r, (k, n, c) in enumerate(specs) if r % nproc == p] for p in range(nproc)]
    bar = ctx.Barrier(nproc)
    baton = (ctx.Value("i", 0), ctx.Condition()) if seq else None
    res = spmd.run_processes(plain_proc, [(g, bar, warm, baton) for g in groups], timeout_s=600)
    bad = [r for r in res if r["rc"] != 0]
    if bad:
        raise SystemExit(f"plain baseline failed: {bad}")
    turn = (max(r["t1"] for r in res) - min(r["t0"] for r in res)) * 1e-9
    stages = np.array([s for r in res for s in r["stages"]])
    digests = {}
    for r in res:
        digests.update(r["digests"])
    work = flop_total if unit == "GFLOP/s" else bytes_total
    return {"processes": nproc, "ranks_per_process": [len(g) for g in groups][:1] + ([] if nranks % nproc == 0 else
                                                                                     [len(g) for g in groups][-1:]),
            "turnaround_s": round(turn, 6), "value": round(work / turn / 1e9, 3), "unit": unit,
            "mean_stage_s": dict(zip(["init", "alloc", "copy_in", "kernel", "copy_out", "free"],
                                     [round(float(v), 6) for v in stages.mean(axis=0)])),
            "digests": [digests[r] for r in range(nranks)]}


def serving_leg(seconds, copy_threads):
    """A short run of the serving configuration through the load generator."""
    from paper_1511_07658_amd import loadgen

    warm = 0.5
    a = loadgen.parse_args(["--ranks", "64", "--rate", "2000", "--duration", str(seconds + warm), "--warmup", str(warm),
                            "--no-plain", "--copy-threads", str(copy_threads)])
    res, _ = loadgen.run(a)
    g = res["gvm"]
    return {"ranks": 64, "rate_req_s": 2000, "measured_s": seconds, "requests": g["requests"], "ok": g["ok"],
            "failed": g["failed"], "p50_ms": g["p50_ms"], "p99_ms": g["p99_ms"], "max_ms": g["max_ms"],
            "throughput_req_s": g["throughput_req_s"], "gemm_GFLOPs": g["gemm_GFLOPs"],
            "algorithmic_GBs": g["algorithmic_GBs"], "per_kernel": g["per_kernel"], "per_size": g["per_size"],
            "mean_stage_ms": g["mean_stage_ms"],
            "budget_GiB": 64, "command": "python -m paper_1511_07658_amd.loadgen --ranks 64 --rate 2000 "
                                         f"--duration {seconds + warm} --warmup {warm} --no-plain"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixed32", choices=sorted(WORKLOADS))
    ap.add_argument("--resident-steps", type=int, default=30, help="steps of the device-phase (resident) leg")
    ap.add_argument("--resident-warmup", type=int, default=-1,
                    help="untimed resident steps before them (default: about 60 ms of device work, so that the "
                         "engine clock has reached its plateau under load)")
    ap.add_argument("--serving-seconds", type=float, default=3.0,
                    help="measured seconds of the serving leg (64 ranks, 2000 req/s); 0 skips it")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--graphs", type=int, default=0, help="replay repeated batches as HIP graphs")
    ap.add_argument("--copy-threads", type=int, default=8, help="manager threads for shared memory <-> pinned copies")
    ap.add_argument("--early-copy-in", type=int, default=1, choices=(0, 1),
                    help="start a rank's next input while the running batch finishes (gvm_config.early_copy_in)")
    ap.add_argument("--trace", default=None,
                    help="write the per-request trace of the copy-inclusive steps there (Chrome trace JSON)")
    ap.add_argument("--rank-threads", action="store_true",
                    help="run the ranks as threads of this process (for profilers that cannot follow forks)")
    ap.add_argument("--loopback", action="store_true", help=argparse.SUPPRESS)  # host-protocol dry run, no GPU
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only: the GVM serves every rank from a single device "
              f"context; --gpus {a.gpus} is not supported (one manager per GPU would shard ranks "
              f"with no exchange step).", file=sys.stderr)
        return 2
    specs = rank_specs(a.workload)
    nranks = len(specs)
    kinds = sorted({k for k, _, _ in specs})
    main_kernel = G.GVM_K_SGEMM if G.GVM_K_SGEMM in kinds else kinds[0]
    flop_total = sum(work_of(k, n)[0] for k, n, _ in specs if k == main_kernel)
    bytes_total = sum(work_of(k, n)[1] for k, n, _ in specs if k == main_kernel)
    pairs_total = sum(n for k, n, _ in specs if k == G.GVM_K_EP)
    unit = {G.GVM_K_SGEMM: "GFLOP/s", G.GVM_K_EP: "Gpairs/s"}.get(main_kernel, "GB/s")
    work_total = {G.GVM_K_SGEMM: flop_total, G.GVM_K_EP: pairs_total}.get(main_kernel, bytes_total)

    if a.rank_threads:
        a.no_plain = True
    else:
        spmd.prestart()  # rank processes fork from a GPU-free server
    ctx = None if a.rank_threads else spmd.context()
    mixed = len(kinds) > 1

    # 1. plain per-process baselines (before this process touches the GPU):
    # cold with the device's own scheduling (the paper's turnaround), warm
    # (contexts created before the start), and cold with the GPU phases run
    # one rank after another (Eq. 1)
    plain = plain_warm = plain_seq = None
    if not a.no_plain and not a.loopback:
        log(f"plain baseline: {nranks} ranks on {min(nranks, MAX_GPU_PROCESSES)} processes (cold, warm, sequential)")
        kw = dict(flop_total=flop_total, bytes_total=bytes_total if main_kernel != G.GVM_K_EP else pairs_total,
                  unit="GFLOP/s" if main_kernel == G.GVM_K_SGEMM else unit)
        plain = run_plain(ctx, specs, **kw)
        plain_warm = run_plain(ctx, specs, warm=True, **kw)
        plain_seq = run_plain(ctx, specs, seq=True, **kw)

    # 2. the GVM manager in this process, ranks in forked processes
    ns = f"gvm.bench.{os.getpid()}"
    space = max((G.in_elems(k, n) + G.out_elems(k, n)) * 4 for k, n, _ in specs) + (1 << 20)
    copy_threads = a.copy_threads
    cfg = G.gvm_config_default(nranks=nranks, shm_bytes_per_rank=space,
                               hbm_budget_bytes=max(2 << 30, 2 * nranks * space),
                               mode=G.GVM_MODE_BATCH, policy=G.GVM_POLICY_AUTO, batch_window_us=5_000_000,
                               use_graphs=1 if a.graphs else 0, copy_threads=copy_threads, name=ns,
                               early_copy_in=a.early_copy_in,
                               backend=G.GVM_BACKEND_LOOPBACK if a.loopback else G.GVM_BACKEND_HIP)
    log(f"GVM: {nranks} ranks, {a.workload}")
    G.check(G.gvm_init(cfg), "gvm_init")
    try:
        bar = threading.Barrier(nranks + 1) if a.rank_threads else ctx.Barrier(nranks + 1)
        results = {}
        res_warmup = a.resident_warmup if a.resident_warmup >= 0 else resident_warmup_steps(specs)
        args = [(ns, r, k, n, c, a.warmup, a.steps, res_warmup, a.resident_steps, bar)
                for r, (k, n, c) in enumerate(specs)]

        def runner():
            if a.rank_threads:
                out = [None] * nranks

                def one(r):
                    out[r] = bench_rank(*args[r])

                ths = [threading.Thread(target=one, args=(r,)) for r in range(nranks)]
                for t in ths:
                    t.start()
                for t in ths:
                    t.join()
                results["r"] = out
            else:
                results["r"] = spmd.run_processes(bench_rank, args, timeout_s=900)

        th = threading.Thread(target=runner)
        th.start()
        bar.wait()                      # 1: attached
        bar.wait()                      # 2: warm-up done
        G.gvm_stats_reset()
        bar.wait()                      # 3: go (timed steps with copies)
        bar.wait()                      # 4: timed steps done
        e2e_stats = G.gvm_stats_json()
        if a.trace:
            G.check(G.gvm_trace_dump(a.trace), "trace dump")
        bar.wait()                      # 5: resident warm-up
        bar.wait()                      # 6: resident warm-up done
        G.gvm_stats_reset()
        bar.wait()                      # 7: go (resident steps)
        bar.wait()                      # 8: resident steps done
        stats = G.gvm_stats_json()
        th.join()
        rr = results["r"]
    finally:
        G.gvm_shutdown()
    elapsed, e2e = leg_summary([r["e2e"] for r in rr], a.steps)
    res_elapsed, dev = leg_summary([r["resident"] for r in rr], a.resident_steps)
    value = a.steps * work_total / elapsed / 1e9
    dev_value = a.resident_steps * work_total / res_elapsed / 1e9

    # roofline of the dominant kernel, from the resident leg's launch events
    knames = {0: "mixed_graph", 1: "vecadd", 2: "blackscholes", 3: "sgemm", 4: "vecmul", 5: "ep"}
    kname = "mixed_graph" if (mixed and a.graphs and "mixed_graph" in stats["kernels"]) else knames[main_kernel]
    ks = stats["kernels"][kname]
    launches = max(ks["launches"], 1)
    avg_launch_s = max(ks["device_ms"] / launches * 1e-3, 1e-12)
    dev_s = max(ks["device_ms"] * 1e-3, 1e-12)
    per_step_launches = launches / max(a.resident_steps, 1)
    if main_kernel == G.GVM_K_SGEMM:
        achieved = (ks["work_flop"] if kname != "mixed_graph" else a.resident_steps * flop_total) / dev_s / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": measured_traffic(a.workload)}
    elif main_kernel == G.GVM_K_EP:
        pairs_s = ks["requests"] / max(sum(1 for k, _, _ in specs if k == G.GVM_K_EP), 1) * pairs_total / dev_s
        achieved = pairs_s * EP_FP64_OPS_PER_PAIR / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4), "traffic": None,
                "ops_per_pair": round(EP_FP64_OPS_PER_PAIR, 3), "Gpairs_per_s": round(pairs_s / 1e9, 2),
                "valu_issue_utilisation": round(pairs_s / 1e9 / EP_ISSUE_GPAIRS, 4)}
    else:
        achieved = (ks["work_bytes"] if kname != "mixed_graph" else a.resident_steps * bytes_total) / dev_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": measured_traffic(a.workload)}
    roof["kernel"] = f"{kname}: {ks['requests']} requests in {ks['launches']} grouped launches"
    roof["avg_launch_us"] = round(avg_launch_s * 1e6, 3)
    roof["launches"] = ks["launches"]
    roof["launches_per_step"] = round(per_step_launches, 3)
    roof["algorithmic_bytes"] = round(ks["work_bytes"] / launches)
    roof["algorithmic_flop"] = round(ks["work_flop"] / launches)
    # the kernel's work per resident step over the whole step, in the unit of
    # `achieved` (manager round trip and any concurrent launch included)
    step_s = res_elapsed / max(a.resident_steps, 1)
    if main_kernel == G.GVM_K_SGEMM:
        roof["step_achieved"] = round(flop_total / step_s / 1e12, 3)
    elif main_kernel == G.GVM_K_EP:
        roof["step_achieved"] = round(pairs_total * EP_FP64_OPS_PER_PAIR / step_s / 1e12, 3)
    else:
        roof["step_achieved"] = round(bytes_total / step_s / 1e9, 3)
    if per_step_launches > 1.0:
        roof["note"] = "launches of one step overlap; step_achieved is the kernel's work per resident step"

    extra = {}
    if mixed:
        vbytes = sum(work_of(k, n)[1] for k, n, _ in specs if k == G.GVM_K_VECADD)
        extra["vecadd_GBps"] = round(a.steps * vbytes / elapsed / 1e9, 3)
        extra["sizes"] = [[k, n] for k, n, _ in specs]
        extra["work_per_step"] = {"sgemm_GFLOP": round(flop_total / 1e9, 4), "vecadd_MB": round(vbytes / 1e6, 3)}
    # bytes crossing PCIe per step: every input in, every result out
    pcie_bytes = sum((G.in_elems(k, n) + G.out_elems(k, n)) * 4 for k, n, _ in specs)

    cpu = cpu_py = None
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        if main_kernel != G.GVM_K_EP and not a.rank_threads:
            cpu = cpu_baseline_c(ctx, specs, main_kernel, a.cpu_seconds)
            cpu_py = cpu_baseline(specs, main_kernel, a.cpu_seconds / 2)
        else:
            cpu = cpu_baseline(specs, main_kernel, a.cpu_seconds)

    serving = None
    if a.serving_seconds > 0 and not a.loopback and not a.rank_threads:
        log(f"serving leg: 64 ranks, 2000 req/s, {a.serving_seconds} s")
        serving = serving_leg(a.serving_seconds, 16)

    ms_step = elapsed / a.steps * 1e3
    line = {
        "metric": "aggregate GB/s & GFLOP/s, N ranks on 1 GPU, GVM vs plain; p50/p99 req latency",
        "value": round(value, 3),
        "unit": unit,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded by rank)",
        "config": {"workload": WORKLOADS[a.workload], "name": a.workload,
                   "ranks": nranks, "mode": "batch", "policy": "auto", "graphs": bool(a.graphs),
                   "copy_threads": copy_threads, "early_copy_in": bool(a.early_copy_in),
                   "timed": "every step: shared memory -> HBM copies, kernels, HBM -> shared memory copies, "
                            "completions", "rank_kind": "threads" if a.rank_threads else "processes"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_baseline_python": cpu_py,
        "latency_us": e2e["latency_us"],
        "step_breakdown_us": e2e["step_breakdown_us"],
        "step_detail_us": e2e["step_detail_us"],
        "pcie_GBps": round(a.steps * pcie_bytes / elapsed / 1e9, 3),
        "device_phase": {"value": round(dev_value, 3), "unit": unit, "steps": a.resident_steps, "warmup_steps": res_warmup, **dev},
        "manager_us": {"ring": stats.get("ring_us"), "batch_admit_lag": stats.get("batch_admit_lag_us"),
                       "busy_iteration": stats.get("busy_iteration_us")},
        "plain": None if plain is None else {k: v for k, v in plain.items() if k != "digests"},
        "plain_warm": None if plain_warm is None else {k: v for k, v in plain_warm.items() if k != "digests"},
        "plain_sequential": None if plain_seq is None else {k: v for k, v in plain_seq.items() if k != "digests"},
        "gvm_vs_plain_turnaround": None if plain is None else round(plain["turnaround_s"] * 1e3 / ms_step, 3),
        "gvm_vs_plain_warm_turnaround": None if plain_warm is None else round(
            plain_warm["turnaround_s"] * 1e3 / ms_step, 3),
        "gvm_vs_plain_sequential_turnaround": None if plain_seq is None else round(
            plain_seq["turnaround_s"] * 1e3 / ms_step, 3),
        "serving": serving,
        **extra,
        "results_unchanged_by_virtualization": all(r["same_bytes"] for r in rr) and all(
            p is None or [r["digest"] for r in rr] == p["digests"] for p in (plain, plain_warm, plain_seq)),
        "host": {"nproc": os.cpu_count(), "machine": platform.machine(),
                 "GPU_MAX_HW_QUEUES": os.environ.get("GPU_MAX_HW_QUEUES")},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
