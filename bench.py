"""Benchmark of the GVM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sgemm8|vecadd4|vecadd16|bs16|ep8|mixed32]

Default workload (the configuration the headline metric is quoted on): 8 SPMD
rank processes, each an FP32 square GEMM C = A B with 1024 x 1024 A, B ~ N(0,1)
seeded by rank, served by one GVM manager on device 0.  One step = every rank
submits its request through the shared-memory rings, the manager gathers the
batch at its request barrier, runs one grouped persistent MFMA launch over all
eight GEMMs, and every rank receives its completion.  The inputs are resident
in HBM when the timed region starts (submitted once before it, then re-used
with GVM_F_IN_RESIDENT | GVM_F_OUT_RESIDENT), so ``value`` is whole-job device
throughput plus the manager round trip; the PCIe-inclusive rate and the plain
per-process baseline (Eq. 1 path) are reported beside it.

Prints ONE JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1511_07658_amd import gvm as G  # noqa: E402
from paper_1511_07658_amd import spmd  # noqa: E402
from paper_1511_07658_amd import workloads as wl  # noqa: E402

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBPS = 8000.0
# EP-like kernel: VALU issue bound.  A SIMD issues one wave64 VALU
# instruction per 4 cycles (16 lanes); the compiled unit loop of
# csrc/ep_kernels.hip issues 602 VALU instructions per Philox block, i.e.
# per 2 pairs of each of the 64 lanes (both pairs accepted; the rejected path
# is a subset): 4 * 602 / 128 = 18.8 SIMD cycles per pair, and 256 CUs x 4
# SIMDs x 2.4 GHz / 18.8 = 130.6 Gpairs/s.
EP_SIMD_CYCLES_PER_PAIR = 4.0 * 602 / 128
PEAK_EP_GPAIRS = 256 * 4 * 2.4e9 / EP_SIMD_CYCLES_PER_PAIR / 1e9

# HBM bytes per launch of the dominant kernel from rocprofv3 --pmc FETCH_SIZE /
# WRITE_SIZE (KiB per dispatch), each scaled by what the counter reads for a
# plain 1 GiB copy (fetch x2.000, write x1.000); valid only for the kernel
# sources they were taken on (sha256 over `sources` in csrc/, in order;
# profiles/sgemm_grouped_8x1024.md, profiles/blackscholes_grouped_16x4M.md,
# profiles/vecadd_grouped_16x16M.md).
SGEMM_SOURCES = ("sgemm.hip", "group_device.hpp", "kernels.hpp", "gemm_tiles.inc")
STREAM_SOURCES = ("stream_kernels.hip", "group_device.hpp", "kernels.hpp")
MEASURED_TRAFFIC = {
    "sgemm8": {"sources": SGEMM_SOURCES, "kernels_sha256": "452827a72b9d2496626dc6a41bb430ee412892a55e6c23e19a35f4b924dc6957",
               "fetch_kib": 32854.9, "fetch_factor": 2.000, "write_kib": 32768.0, "write_factor": 1.000},
    "bs16": {"sources": STREAM_SOURCES, "kernels_sha256": "b6e37850a81652cdfbfcb6ef5733e38694e16acd5b1e2a7223c8bda01e96637c",
             "fetch_kib": 393326.6, "fetch_factor": 2.000, "write_kib": 524311.7, "write_factor": 1.000},
    "vecadd16": {"sources": STREAM_SOURCES, "kernels_sha256": "b6e37850a81652cdfbfcb6ef5733e38694e16acd5b1e2a7223c8bda01e96637c",
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
    "sgemm8": "8 ranks via GVM, FP32 SGEMM 1024x1024 each, grouped MFMA launch, inputs resident in HBM",
    "vecadd4": "4 ranks via GVM, FP32 vector add n=2^20 each, inputs resident in HBM",
    "vecadd16": "16 ranks via GVM, FP32 vector add n=2^24 each (3.2 GB per step, beyond the memory-side cache), "
                "one grouped launch, inputs resident in HBM",
    "bs16": "16 ranks via GVM, FP32 Black-Scholes 4M options each, one fused launch, inputs resident in HBM",
    "mixed32": "32 ranks via GVM with uneven sizes: 16 vector adds n=floor(2^U[16,24]) and 16 SGEMMs "
               "n in {256..2048 step 64}, tuned tiles, one grouped launch per kernel per step, inputs resident in HBM",
    "ep8": "8 ranks via GVM, EP-like Gaussian-pair tally of 2^24 pairs each (the size of the paper's EP(M24)), "
           "one grouped launch plus a per-request reduction, keys and results resident in HBM",
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


# ----------------------------------------------------------------- rank side

def bench_rank(ns, rank, kernel_id, n, cfg_idx, warmup, steps, e2e_steps, barrier):
    """One SPMD rank process: attach, upload once, then timed resident steps,
    then a few PCIe-inclusive steps.  Returns CLOCK_MONOTONIC stamps."""
    x = spmd.make_input(kernel_id, cfg_idx, rank, n)
    out = np.empty(G.out_elems(kernel_id, n), np.float32)
    G.check(G.gvm_attach_ns(ns, rank), "attach")
    t = G.check(G.gvm_submit(rank, kernel_id, x, out, n), "upload")
    G.check(G.gvm_wait(rank, t, 120_000_000_000), "upload wait")
    first = spmd.digest(out)
    flags = G.GVM_F_IN_RESIDENT | G.GVM_F_OUT_RESIDENT
    barrier.wait()                       # 1: uploads done
    for _ in range(warmup):
        t = G.check(G.gvm_submit_ex(rank, kernel_id, None, None, n, flags), "warmup")
        G.check(G.gvm_wait(rank, t, 120_000_000_000), "warmup wait")
    barrier.wait()                       # 2: warm-up done
    barrier.wait()                       # 3: statistics reset, go
    import ctypes

    clock = time.clock_gettime_ns
    mono = time.CLOCK_MONOTONIC
    lib = G.lib()
    submit_ex, wait_timed = lib.gvm_submit_ex, lib.gvm_wait_timed
    ts = (ctypes.c_uint64 * 5)()
    parts = [0, 0, 0, 0, 0, 0]
    stamps = []                          # per step: submit, admit, posted, seen (ns)
    t0 = clock(mono)
    seen = t0
    for _ in range(steps):
        t = submit_ex(rank, kernel_id, None, None, n, flags)
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
    t1 = clock(mono)
    barrier.wait()                       # 4: timed steps done
    # PCIe-inclusive steps: the input sits in the rank's shared memory
    # (zero-copy region), the manager moves it to HBM and the result back
    view = G.gvm_rank_buffer(rank, (x.size + out.size) * 4)
    if view is None:
        raise RuntimeError(f"rank {rank}: no zero-copy space: {G.gvm_last_error()}")
    xin, oview = view[:x.size], view[x.size:x.size + out.size]
    xin[:] = x
    barrier.wait()                       # 5: statistics read, go
    e0 = time.clock_gettime_ns(time.CLOCK_MONOTONIC)
    for _ in range(e2e_steps):
        t = G.check(G.gvm_submit(rank, kernel_id, xin, oview, n), "e2e step")
        G.check(G.gvm_wait(rank, t, 120_000_000_000), "e2e wait")
    e1 = time.clock_gettime_ns(time.CLOCK_MONOTONIC)
    same = spmd.digest(oview if e2e_steps else out) == first
    G.gvm_detach(rank)
    return {"t0": t0, "t1": t1, "e0": e0, "e1": e1, "same_bytes": same, "digest": first,
            "parts_ns": [x / max(steps, 1) for x in parts], "stamps": stamps}


def step_detail(rr):
    """Across ranks, per timed step: spread of the submit times, spread of
    the completion posts, and the gap from the previous step's last post to
    this step's first submit (means, us), plus how often each rank submitted
    last (the one the request barrier waits for)."""
    st = np.array([r["stamps"] for r in rr], dtype=np.float64)   # ranks x steps x 4
    if st.ndim != 3 or st.shape[1] < 2:
        return None
    sub, post = st[:, :, 0], st[:, :, 2]
    last = np.bincount(np.argmax(sub, axis=0), minlength=st.shape[0])
    return {"submit_spread": round(float(np.mean(sub.max(0) - sub.min(0))) * 1e-3, 2),
            "post_spread": round(float(np.mean(post.max(0) - post.min(0))) * 1e-3, 2),
            "last_post_to_first_submit": round(float(np.mean(sub.min(0)[1:] - post.max(0)[:-1])) * 1e-3, 2),
            "last_post_to_last_submit": round(float(np.mean(sub.max(0)[1:] - post.max(0)[:-1])) * 1e-3, 2),
            "last_submitter_counts": last.tolist()}


PLAIN_WARM_N = {G.GVM_K_VECADD: 4096, G.GVM_K_VECMUL: 4096, G.GVM_K_BLACKSCHOLES: 4096, G.GVM_K_SGEMM: 64,
                G.GVM_K_EP: 4096}


def plain_rank(kernel_id, n, cfg_idx, rank, barrier, warm=False, baton=None):
    """One process of the plain method (no virtualization): its own device
    context, pageable copies, the same kernel code object (Section 4.1).

    Variants of the baseline:
    * cold (default): the context is created inside the timed region, as in
      the paper's turnaround (T_init included);
    * ``warm``: a small request of the same kernel runs before the start
      barrier, so context creation and code-object loading fall outside it;
    * ``baton`` (a shared turn counter and its condition): the processes run
      their GPU phases one after another in rank order, the sequential
      execution that Eq. 1 models, instead of letting the device's
      scheduler interleave them."""
    x = spmd.make_input(kernel_id, cfg_idx, rank, n)
    out = np.empty(G.out_elems(kernel_id, n), np.float32)
    G.lib()
    args = (float(np.float32(wl.BS_RATE)), float(np.float32(wl.BS_VOLATILITY)))
    if warm:
        m = PLAIN_WARM_N[kernel_id]
        wx = spmd.make_input(kernel_id, cfg_idx, rank, m)
        wo = np.empty(G.out_elems(kernel_id, m), np.float32)
        rc, _ = G.gvm_plain_run(kernel_id, wx, wo, m, *args)
        if rc != 0:
            return {"rc": rc, "t0": 0, "t1": 0, "stages": [0.0] * 6, "digest": ""}
    barrier.wait()
    t0 = time.clock_gettime_ns(time.CLOCK_MONOTONIC)
    if baton is not None:
        turn, cond = baton
        with cond:
            cond.wait_for(lambda: turn.value == rank)
    rc, stages = G.gvm_plain_run(kernel_id, x, out, n, *args)
    if baton is not None:
        with cond:
            turn.value += 1
            cond.notify_all()
    t1 = time.clock_gettime_ns(time.CLOCK_MONOTONIC)
    return {"rc": rc, "t0": t0, "t1": t1, "stages": stages, "digest": spmd.digest(out)}


# ----------------------------------------------------------------- main

def cpu_baseline(kernel_id, nranks, n, cfg_idx, budget_s=10.0):
    """The oracle as it stands, on this host's cores, over a bounded sample of
    the same workload (whole passes over the ranks' requests, ~budget_s)."""
    from oracle import ep as oe
    from oracle import kernels as ok

    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    if kernel_id == G.GVM_K_EP:
        sample = min(n, 1 << 20)   # a bounded slice of each rank's pair stream
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            oe.ep_reference(wl.ep_key(cfg_idx, done % nranks), sample)
            done += 1
        el = time.perf_counter() - t0
        return {"value": round(done * sample / el / 1e9, 6), "unit": "Gpairs/s", "cores": 1, "kind": "oracle",
                "sample": f"{done} slices of {sample} pairs through oracle.ep.ep_reference in {el:.1f} s "
                          f"(the first {sample} pairs of the ranks' keys, cycled)"}
    inputs = []
    for r in range(min(nranks, 4)):
        if kernel_id == G.GVM_K_SGEMM:
            inputs.append(wl.sgemm_inputs(cfg_idx, r, n))
        elif kernel_id == G.GVM_K_BLACKSCHOLES:
            inputs.append(wl.bs_inputs(cfg_idx, r, n))
        else:
            inputs.append(wl.vecadd_inputs(cfg_idx, r, n))
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        args = inputs[done % len(inputs)]
        if kernel_id == G.GVM_K_SGEMM:
            ok.sgemm_f64(*args)
        elif kernel_id == G.GVM_K_BLACKSCHOLES:
            ok.black_scholes_f64(*args, wl.BS_RATE, wl.BS_VOLATILITY)
        else:
            ok.vecadd_f32(*args)
        done += 1
    el = time.perf_counter() - t0
    flop, byts = work_of(kernel_id, n)
    if kernel_id == G.GVM_K_SGEMM:
        value, unit = done * flop / el / 1e9, "GFLOP/s"
    else:
        value, unit = done * byts / el / 1e9, "GB/s"
    kname = {1: "vecadd_f32", 2: "black_scholes_f64", 3: "sgemm_f64"}[kernel_id]
    return {"value": round(value, 3), "unit": unit, "cores": threads, "kind": "oracle",
            "sample": f"{done} requests of n={n} through oracle.kernels.{kname} in {el:.1f} s "
                      f"(the workload's {nranks} requests, cycled)"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sgemm8", choices=sorted(WORKLOADS))
    ap.add_argument("--e2e-steps", type=int, default=10)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--graphs", type=int, default=None, help="replay repeated batches as HIP graphs (switched off in this build)")
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
    if a.graphs is None:
        a.graphs = 0  # graph replay is switched off in the library
    nranks = len(specs)
    kinds = sorted({k for k, _, _ in specs})
    main_kernel = G.GVM_K_SGEMM if G.GVM_K_SGEMM in kinds else kinds[0]
    flop_total = sum(work_of(k, n)[0] for k, n, _ in specs)
    bytes_total = sum(work_of(k, n)[1] for k, n, _ in specs)
    import threading

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

    def run_plain(warm=False, seq=False):
        bar = ctx.Barrier(nranks)
        baton = (ctx.Value("i", 0), ctx.Condition()) if seq else None
        res = spmd.run_processes(plain_rank, [(k, n, c, r, bar, warm, baton) for r, (k, n, c) in enumerate(specs)],
                                 timeout_s=300)
        bad = [r for r in res if r["rc"] != 0]
        if bad:
            raise SystemExit(f"plain baseline failed: {bad}")
        turn = (max(r["t1"] for r in res) - min(r["t0"] for r in res)) * 1e-9
        stages = np.array([r["stages"] for r in res])
        return {"turnaround_s": round(turn, 6),
                "value": round((flop_total if main_kernel == G.GVM_K_SGEMM else
                                sum(n for _, n, _ in specs) if main_kernel == G.GVM_K_EP else bytes_total)
                               / turn / 1e9, 3),
                "mean_stage_s": dict(zip(["init", "alloc", "copy_in", "kernel", "copy_out", "free"],
                                         [round(float(v), 6) for v in stages.mean(axis=0)])),
                "digests": [r["digest"] for r in res]}

    if not a.no_plain and not a.loopback and nranks <= 16:
        log(f"plain baseline: {nranks} processes, each its own context (cold, warm, sequential)")
        plain = run_plain()
        plain_warm = run_plain(warm=True)
        plain_seq = run_plain(seq=True)

    # 2. the GVM manager in this process, ranks in forked processes
    ns = f"gvm.bench.{os.getpid()}"
    space = max((G.in_elems(k, n) + G.out_elems(k, n)) * 4 for k, n, _ in specs) + (1 << 20)
    cfg = G.gvm_config_default(nranks=nranks, shm_bytes_per_rank=space,
                               hbm_budget_bytes=max(2 << 30, 2 * nranks * space),
                               mode=G.GVM_MODE_BATCH, policy=G.GVM_POLICY_AUTO, batch_window_us=5_000_000,
                               use_graphs=1 if a.graphs else 0, copy_threads=8, name=ns,
                               backend=G.GVM_BACKEND_LOOPBACK if a.loopback else G.GVM_BACKEND_HIP)
    log(f"GVM: {nranks} ranks, {a.workload}")
    G.check(G.gvm_init(cfg), "gvm_init")
    try:
        bar = threading.Barrier(nranks + 1) if a.rank_threads else ctx.Barrier(nranks + 1)
        results = {}
        args = [(ns, r, k, n, c, a.warmup, a.steps, a.e2e_steps, bar) for r, (k, n, c) in enumerate(specs)]

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
                results["r"] = spmd.run_processes(bench_rank, args, timeout_s=600)

        th = threading.Thread(target=runner)
        th.start()
        bar.wait()                      # 1: uploads done
        bar.wait()                      # 2: warm-up done
        G.gvm_stats_reset()
        bar.wait()                      # 3: go
        bar.wait()                      # 4: timed steps done
        stats = G.gvm_stats_json()
        bar.wait()                      # 5: PCIe-inclusive steps start
        th.join()
        rr = results["r"]
    finally:
        G.gvm_shutdown()
    elapsed = (max(r["t1"] for r in rr) - min(r["t0"] for r in rr)) * 1e-9
    e2e = (max(r["e1"] for r in rr) - min(r["e0"] for r in rr)) * 1e-9
    knames = {0: "mixed_graph", 1: "vecadd", 2: "blackscholes", 3: "sgemm", 4: "vecmul", 5: "ep"}
    kname = "mixed_graph" if (mixed and a.graphs and "mixed_graph" in stats["kernels"]) else knames[main_kernel]
    ks = stats["kernels"][kname]
    launches = max(ks["launches"], 1)
    avg_launch_s = max(ks["device_ms"] / launches * 1e-3, 1e-12)
    # the launch of the dominant kernel covers every request of its kind in a step
    main_specs = [(k, n) for k, n, _ in specs if k == main_kernel]
    main_flop = sum(work_of(k, n)[0] for k, n in main_specs)
    main_bytes = sum(work_of(k, n)[1] for k, n in main_specs)
    dev_s = max(ks["device_ms"] * 1e-3, 1e-12)
    if main_kernel == G.GVM_K_SGEMM:
        value = a.steps * main_flop / elapsed / 1e9
        unit = "GFLOP/s"
        # algorithmic FLOP of every timed launch / their summed device time
        achieved = (ks["work_flop"] if kname != "mixed_graph" else a.steps * main_flop) / dev_s / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": measured_traffic(a.workload)}
        e2e_value = a.e2e_steps * main_flop / e2e / 1e9
    elif main_kernel == G.GVM_K_EP:
        pairs = sum(n for k, n in main_specs)
        value = a.steps * pairs / elapsed / 1e9
        unit = "Gpairs/s"
        achieved = ks["requests"] / len(main_specs) * pairs / dev_s / 1e9
        roof = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(PEAK_EP_GPAIRS, 1), "unit": "Gpairs/s",
                "frac": round(achieved / PEAK_EP_GPAIRS, 4), "traffic": None}
        e2e_value = a.e2e_steps * pairs / e2e / 1e9
    else:
        value = a.steps * main_bytes / elapsed / 1e9
        unit = "GB/s"
        achieved = (ks["work_bytes"] if kname != "mixed_graph" else a.steps * main_bytes) / dev_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": measured_traffic(a.workload)}
        e2e_value = a.e2e_steps * main_bytes / e2e / 1e9
    roof["kernel"] = f"{kname}: {ks['requests']} requests in {ks['launches']} grouped launches"
    roof["avg_launch_us"] = round(avg_launch_s * 1e6, 3)
    roof["launches"] = ks["launches"]
    roof["algorithmic_bytes"] = round(ks["work_bytes"] / launches)
    extra = {}
    if mixed:
        extra["vecadd_GBps"] = round(a.steps * sum(work_of(k, n)[1] for k, n, _ in specs if k == G.GVM_K_VECADD)
                                     / elapsed / 1e9, 3)
        extra["sizes"] = [[k, n] for k, n, _ in specs]

    cpu = None
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        k0, n0, c0 = next(sp for sp in specs if sp[0] == main_kernel)
        cpu = cpu_baseline(k0, len(main_specs), n0, c0, a.cpu_seconds)

    line = {
        "metric": "aggregate GB/s & GFLOP/s, N ranks on 1 GPU, GVM vs plain; p50/p99 req latency",
        "value": round(value, 3),
        "unit": unit,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded by rank)",
        "config": {"workload": WORKLOADS[a.workload], "name": a.workload,
                   "ranks": nranks, "mode": "batch", "policy": "auto (grouped when resident)",
                   "graphs": bool(a.graphs),
                   "rank_kind": "threads" if a.rank_threads else "processes"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "latency_us": {"p50": ks["latency_us"]["p50"], "p99": ks["latency_us"]["p99"], "count": ks["latency_us"]["count"]},
        "step_breakdown_us": dict(zip(
            ["barrier_and_drain", "admit_to_launch", "launch_to_device_done", "device_done_to_posted",
             "posted_to_seen", "rank_loop"],
            [round(float(x) * 1e-3, 2) for x in np.mean([r["parts_ns"] for r in rr], axis=0)])),
        "step_detail_us": step_detail(rr),
        "manager_us": {"ring": stats.get("ring_us"), "batch_admit_lag": stats.get("batch_admit_lag_us"),
                       "busy_iteration": stats.get("busy_iteration_us")},
        "e2e_pcie": {"value": round(e2e_value, 3), "unit": unit, "steps": a.e2e_steps,
                     "ms_per_step": round(e2e / max(a.e2e_steps, 1) * 1e3, 3)},
        "plain": None if plain is None else {k: v for k, v in plain.items() if k != "digests"},
        "plain_warm": None if plain_warm is None else {k: v for k, v in plain_warm.items() if k != "digests"},
        "plain_sequential": None if plain_seq is None else {k: v for k, v in plain_seq.items() if k != "digests"},
        "gvm_vs_plain_turnaround": None if plain is None else round(plain["turnaround_s"] / (e2e / max(a.e2e_steps, 1)), 3),
        "gvm_vs_plain_warm_turnaround": None if plain_warm is None else round(
            plain_warm["turnaround_s"] / (e2e / max(a.e2e_steps, 1)), 3),
        "gvm_vs_plain_sequential_turnaround": None if plain_seq is None else round(
            plain_seq["turnaround_s"] / (e2e / max(a.e2e_steps, 1)), 3),
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
