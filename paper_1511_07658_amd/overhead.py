"""Virtualization overhead of the GVM for one rank (the overhead
micro-benchmark of Section 6).

One SPMD rank process submits vector-add requests c = a + b of a given data
size (a, b and c together) one after another.  For each request:

* turnaround: from the rank calling ``gvm_submit`` (inputs in its own
  memory) to ``gvm_wait`` returning with c in its own memory, on the rank's
  clock;
* GPU time: the time the request spends on the device inside the manager,
  its copy-in, kernel and copy-out device times (HIP events, ``batch_timing``;
  a request's copies move in 8 MiB pieces and the piece times are summed).

overhead = (turnaround - GPU time) / turnaround.  Two submission modes:
``copy`` (the rank's arrays are copied into its shared-memory data space by
``gvm_submit`` and back by ``gvm_wait``) and ``zero-copy`` (the rank builds
its inputs directly in its data space, ``gvm_rank_buffer``, and reads c
there).  Prints one JSON object per (size, mode) and a summary line.

    python -m paper_1511_07658_amd.overhead [--sizes-mb 4,16,64,100,200,400] [--reps 10]
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import threading
import time

import numpy as np

from . import gvm as G
from . import spmd
from . import workloads as wl


def _rank(ns: str, n: int, warmup: int, reps: int, zero_copy: bool, barrier):
    """Rank program: `warmup` untimed then `reps` timed vector adds of length
    n (the manager's statistics are reset at the barrier in between);
    per-request turnaround (ns) of the timed ones."""
    G.check(G.gvm_attach_ns(ns, 0), "attach")
    a, b = wl.vecadd_inputs(61, 0, n, 0)
    if zero_copy:
        view = G.gvm_rank_buffer(0, 3 * n * 4)
        view[:n] = a
        view[n:2 * n] = b
        inb, outb = view[:2 * n], view[2 * n:3 * n]
    else:
        inb = np.concatenate([a, b])
        outb = np.empty(n, np.float32)
    for _ in range(warmup):
        t = G.check(G.gvm_submit(0, G.GVM_K_VECADD, inb, outb, n), "warm-up submit")
        G.check(G.gvm_wait(0, t, 60_000_000_000), "warm-up wait")
    barrier.wait()   # warm-up done
    barrier.wait()   # statistics reset
    times, stages = [], []
    for _ in range(reps):
        t0 = time.perf_counter_ns()
        t = G.check(G.gvm_submit(0, G.GVM_K_VECADD, inb, outb, n), "submit")
        st, ts = G.gvm_wait_timed(0, t, 60_000_000_000)
        G.check(st, "wait")
        times.append(time.perf_counter_ns() - t0)
        # manager timestamps: submit -> admitted -> launched (input staged) ->
        # device done -> answered (result back in shared memory)
        stages.append([ts[1] - ts[0], ts[2] - ts[1], ts[3] - ts[2], ts[4] - ts[3]])
    ok = bool(np.array_equal(outb, a + b))
    G.check(G.gvm_detach(0), "detach")
    return {"turnaround_ns": times, "stages_ns": stages, "exact": ok}


def run(sizes_mb, reps: int, warmup: int = 2, loopback: bool = False):
    ns = f"gvm.overhead.{os.getpid()}"
    n_max = max(int(mb * (1 << 20)) // 12 for mb in sizes_mb)
    n_max -= n_max % 4
    cfg = G.gvm_config_default(nranks=1, shm_bytes_per_rank=3 * n_max * 4 + (1 << 20),
                               staging_bytes=3 * n_max * 4 + (1 << 20), hbm_budget_bytes=4 << 30,
                               mode=G.GVM_MODE_SERVING, policy=G.GVM_POLICY_PS2, batch_timing=1, name=ns,
                               backend=G.GVM_BACKEND_LOOPBACK if loopback else G.GVM_BACKEND_HIP)
    G.check(G.gvm_init(cfg), "gvm_init")
    rows = []
    try:
        for mb in sizes_mb:
            n = int(mb * (1 << 20)) // 12
            n -= n % 4
            for mode in ("copy", "zero-copy"):
                zc = mode == "zero-copy"
                bar = spmd.context().Barrier(2)
                box = {}
                th = threading.Thread(target=lambda: box.update(r=spmd.run_processes(_rank, [(ns, n, warmup, reps, zc, bar)])[0]))
                th.start()
                bar.wait()
                G.gvm_stats_reset()
                bar.wait()
                th.join()
                res = box["r"]
                st = G.gvm_stats_json()
                tt = [x / 1e3 for x in res["turnaround_ns"]]
                tm = st["timing"]
                ks = st["kernels"]["vecadd"]
                turn = statistics.median(tt)
                # means over the timed requests
                h2d = tm["h2d"]["ms"] * 1e3 / max(tm["h2d"]["count"], 1)
                kern = ks["device_ms"] * 1e3 / max(ks["launches"], 1)
                d2h = tm["d2h"]["ms"] * 1e3 / max(tm["d2h"]["count"], 1)
                gpu = h2d + kern + d2h
                row = {
                    "size_mb": mb, "n": n, "mode": mode, "reps": reps, "exact": res["exact"],
                    "turnaround_us": round(turn, 1), "gpu_us": round(gpu, 1),
                    "h2d_us": round(h2d, 1), "kernel_us": round(kern, 1), "d2h_us": round(d2h, 1),
                    "overhead_us": round(turn - gpu, 1),
                    "overhead_frac": round((turn - gpu) / turn, 4),
                    # medians of the manager's stage times (us)
                    "stages_us": {name: round(statistics.median(x[i] for x in res["stages_ns"]) / 1e3, 1)
                                  for i, name in enumerate(("submit_to_admit", "admit_to_launch",
                                                            "launch_to_device_done", "device_done_to_answer"))},
                }
                rows.append(row)
                print(json.dumps(row), flush=True)
    finally:
        G.gvm_shutdown()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes-mb", default="4,16,64,100,200,400")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--loopback", action="store_true", help=argparse.SUPPRESS)  # host-protocol dry run, no GPU
    a = ap.parse_args(argv)
    spmd.prestart()
    sizes = [float(x) for x in a.sizes_mb.split(",") if x]
    rows = run(sizes, a.reps, a.warmup, a.loopback)
    print(json.dumps({"summary": [(r["size_mb"], r["mode"], r["overhead_frac"]) for r in rows]}), flush=True)
    return 0 if all(r["exact"] for r in rows) else 1


if __name__ == "__main__":
    sys.exit(main())
