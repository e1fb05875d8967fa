"""Enqueue policies of Section 4.2.1 on the MI355X: PS-1, PS-2 and the grouped
persistent launch, for I/O-intensive and compute-intensive request shapes.

For every case (kernel, size), N rank threads submit one request each per
batch, ``--reps`` batches per policy, in batch mode with ``batch_timing``
(a batch is enqueued as a whole; its device phase, first copy-in to last
copy-out, is timed with device events).  Two data paths:

* ``copy``: inputs come from the ranks' shared memory and results go back
  there (copy-in, kernel, copy-out per request);
* ``resident``: inputs stay in HBM from a previous request and results are
  left there (``GVM_F_IN_RESIDENT | GVM_F_OUT_RESIDENT``): kernel work only.

Besides the measured device phase, each row carries the single-rank profile
(T_in, T_comp, T_out, copies timed with device events), from which the class
of Section 4.2.3 and the policy the paper's rule picks follow: compute-
intensive (PS-1) when T_comp is at least T_in and at least T_out, I/O-
intensive (PS-2) when both transfers take longer than T_comp.

    python -m paper_1511_07658_amd.policy_study [--ranks 8] [--reps 5] [--json out.json]
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import threading

from . import gvm as G
from . import spmd

POLICIES = (("PS1", G.GVM_POLICY_PS1), ("PS2", G.GVM_POLICY_PS2), ("GROUPED", G.GVM_POLICY_GROUPED))

# (name, kernel id, n): small and large requests of each kernel
CASES = (
    ("vecadd", G.GVM_K_VECADD, 1 << 16),
    ("vecadd", G.GVM_K_VECADD, 1 << 22),
    ("blackscholes", G.GVM_K_BLACKSCHOLES, 1 << 18),
    ("blackscholes", G.GVM_K_BLACKSCHOLES, 1 << 22),
    ("sgemm", G.GVM_K_SGEMM, 256),
    ("sgemm", G.GVM_K_SGEMM, 1024),
)


def _batches(ns, kernel_id, n, nranks, reps, resident):
    """`reps` batches of one request from each of `nranks` rank threads."""
    errs = []
    bar = threading.Barrier(nranks + 1)

    def rank(r):
        try:
            G.check(G.gvm_attach_ns(ns, r), "attach")
            ni, no = G.in_elems(kernel_id, n), G.out_elems(kernel_id, n)
            view = G.gvm_rank_buffer(r, (ni + no) * 4)
            view[:ni] = spmd.make_input(kernel_id, 73, r, n)
            inb, outb = view[:ni], view[ni:ni + no]
            if resident:  # place the input on the device once
                t = G.check(G.gvm_submit(r, kernel_id, inb, outb, n), "upload")
                G.check(G.gvm_wait(r, t, 60_000_000_000), "upload")
            bar.wait()
            bar.wait()  # statistics reset
            flags = (G.GVM_F_IN_RESIDENT | G.GVM_F_OUT_RESIDENT) if resident else 0
            for _ in range(reps):
                t = G.check(G.gvm_submit_ex(r, kernel_id, inb, outb, n, flags), "submit")
                G.check(G.gvm_wait(r, t, 60_000_000_000), "wait")
                bar.wait()
            G.check(G.gvm_detach(r), "detach")
        except Exception as e:  # collected
            errs.append(repr(e))
            bar.abort()

    ths = [threading.Thread(target=rank, args=(r,)) for r in range(nranks)]
    [t.start() for t in ths]
    try:
        bar.wait()
        G.gvm_stats_reset()
        bar.wait()
        for _ in range(reps):
            bar.wait()
    except threading.BrokenBarrierError:
        pass
    [t.join() for t in ths]
    if errs:
        raise RuntimeError(errs)
    return G.gvm_stats_json()


def run(nranks: int, reps: int, loopback: bool = False):
    rows = []
    for name, kid, n in CASES:
        prof = None
        for pname, pol in POLICIES:
            ns = f"gvm.policy.{os.getpid()}.{name}.{n}.{pname}"
            ni, no = G.in_elems(kid, n), G.out_elems(kid, n)
            cfg = G.gvm_config_default(nranks=nranks, shm_bytes_per_rank=(ni + no) * 4 + (1 << 20),
                                       hbm_budget_bytes=8 << 30, policy=pol, batch_timing=1,
                                       batch_window_us=10_000_000, name=ns,
                                       backend=G.GVM_BACKEND_LOOPBACK if loopback else G.GVM_BACKEND_HIP)
            G.check(G.gvm_init(cfg), "gvm_init")
            try:
                # one untimed batch over every rank: first copies into fresh
                # device slots and staging run several times slower
                _batches(ns, kid, n, nranks, 1, False)
                if prof is None:  # single-rank profile with copies
                    st = _batches(ns, kid, n, 1, reps, False)
                    tm = st["timing"]
                    ks = st["kernels"][name]
                    prof = (tm["h2d"]["ms"] / tm["h2d"]["count"] * 1e-3, ks["device_ms"] / ks["launches"] * 1e-3,
                            tm["d2h"]["ms"] / tm["d2h"]["count"] * 1e-3)
                for resident in (False, True):
                    st = _batches(ns, kid, n, nranks, reps, resident)
                    spans = st["timing"]["batch_device_us"]
                    ks = st["kernels"][name]
                    row = {
                        "kernel": name, "n": n, "ranks": nranks, "policy": pname,
                        "data": "resident" if resident else "copy",
                        "device_phase_us": round(statistics.median(spans), 1),
                        "launches_per_batch": round(ks["launches"] / max(len(spans), 1), 2),
                        "t_in_us": round(prof[0] * 1e6, 1), "t_comp_us": round(prof[1] * 1e6, 1),
                        "t_out_us": round(prof[2] * 1e6, 1),
                    }
                    rows.append(row)
                    print(json.dumps(row), flush=True)
            finally:
                G.gvm_shutdown()
    # fastest policy per (case, data path)
    best = {}
    for r in rows:
        key = (r["kernel"], r["n"], r["data"])
        if key not in best or r["device_phase_us"] < best[key]["device_phase_us"]:
            best[key] = r
    summary = [{"kernel": k[0], "n": k[1], "data": k[2], "fastest": b["policy"]} for k, b in best.items()]
    return rows, summary


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--ranks", type=int, default=8)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--json", default=None)
    ap.add_argument("--loopback", action="store_true", help=argparse.SUPPRESS)  # host-protocol dry run, no GPU
    a = ap.parse_args(argv)
    rows, summary = run(a.ranks, a.reps, a.loopback)
    for s in summary:
        print(json.dumps(s), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump({"rows": rows, "summary": summary}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
