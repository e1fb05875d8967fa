"""Spatial partitioning of the MI355X for serving QoS (gvm_config.latency_cus).

Serving mode, inputs resident in HBM (kernel work only), two kinds of ranks:

* bulk ranks submit large SGEMMs (n = 2048, about 150 us each on the whole
  device) back to back, keeping the device busy;
* latency ranks submit small requests (vector add 2^18, Black-Scholes 2^16,
  SGEMM 256: a few us of device work each) at seeded Poisson arrival times.

Each configuration runs the same seeded arrivals for ``--seconds``:

* ``alone``: latency ranks only, no partition (their latency with an idle
  device);
* ``shared``: both kinds, no partition: a small request's kernel waits for
  CUs that the bulk SGEMM's workgroups hold;
* ``streams``: both kinds, each class on a stream of its own but without
  CU masks (``GVM_PARTITION_MASKS=0``): what separate queues alone give;
* ``cus=32`` and ``cus=64``: both kinds, the latency class restricted to 32
  or 64 CUs and the bulk class to the rest.

A request's latency is the manager's time from its submit to its answer
(``gvm_wait_timed``), so the Python loop of the rank does not count.  Bulk
throughput is the SGEMM work completed in the window.

    python -m paper_1511_07658_amd.qos_study [--seconds 3] [--json out.json]
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

SMALL = ((G.GVM_K_VECADD, 1 << 18, "vecadd"), (G.GVM_K_BLACKSCHOLES, 1 << 16, "blackscholes"),
         (G.GVM_K_SGEMM, 256, "sgemm256"))
BULK_N = 2048
RESIDENT = G.GVM_F_IN_RESIDENT | G.GVM_F_OUT_RESIDENT


def _pct(v, p):
    if not v:
        return None
    v = sorted(v)
    return round(v[max(0, int(np.ceil(p / 100.0 * len(v))) - 1)], 1)


def run_case(latency_cus: int, bulk_ranks: int, lat_ranks: int, rate: float, seconds: float, loopback=False):
    nranks = bulk_ranks + lat_ranks
    ns = f"gvm.qos.{os.getpid()}.{latency_cus}.{bulk_ranks}"
    big = (G.in_elems(G.GVM_K_SGEMM, BULK_N) + G.out_elems(G.GVM_K_SGEMM, BULK_N)) * 4
    cfg = G.gvm_config_default(nranks=nranks, mode=G.GVM_MODE_SERVING, latency_cus=latency_cus,
                               shm_bytes_per_rank=big + (1 << 20), hbm_budget_bytes=16 << 30, name=ns,
                               backend=G.GVM_BACKEND_LOOPBACK if loopback else G.GVM_BACKEND_HIP)
    G.check(G.gvm_init(cfg), "gvm_init")
    bar = threading.Barrier(nranks + 1)
    stop = threading.Event()
    window = {}
    lat_us = {name: [] for _, _, name in SMALL}
    bulk_done = []
    errs = []

    def upload(r, k, n):
        ni, no = G.in_elems(k, n), G.out_elems(k, n)
        view = G.gvm_rank_buffer(r, (ni + no) * 4)
        view[:ni] = spmd.make_input(k, 77, r, n)
        t = G.check(G.gvm_submit(r, k, view[:ni], view[ni:ni + no], n), "upload")
        G.check(G.gvm_wait(r, t, 120_000_000_000), "upload")
        return view[:ni], view[ni:ni + no]

    def bulk(r):
        try:
            G.check(G.gvm_attach_ns(ns, r), "attach")
            inb, outb = upload(r, G.GVM_K_SGEMM, BULK_N)
            bar.wait()
            bar.wait()
            while not stop.is_set():
                t = G.check(G.gvm_submit_ex(r, G.GVM_K_SGEMM, inb, outb, BULK_N, RESIDENT), "submit")
                G.check(G.gvm_wait(r, t, 60_000_000_000), "wait")
                bulk_done.append(time.monotonic())
            G.check(G.gvm_detach(r), "detach")
        except Exception as e:  # collected
            errs.append(repr(e))
            bar.abort()

    def latency(r, idx):
        try:
            G.check(G.gvm_attach_ns(ns, r), "attach")
            k, n, name = SMALL[idx % len(SMALL)]
            inb, outb = upload(r, k, n)
            gaps = np.random.Generator(np.random.PCG64([1511, 77, idx])).exponential(1.0 / rate, int(rate * seconds * 2) + 10)
            bar.wait()
            bar.wait()
            t0 = window["t0"]
            due = t0
            for g in gaps:
                due += g
                if due >= window["t1"]:
                    break
                wait = due - time.monotonic()
                if wait > 0:
                    time.sleep(wait)
                t = G.check(G.gvm_submit_ex(r, k, inb, outb, n, RESIDENT), "submit")
                st, ts = G.gvm_wait_timed(r, t, 60_000_000_000)
                G.check(st, "wait")
                lat_us[name].append((ts[4] - ts[0]) * 1e-3)
            G.check(G.gvm_detach(r), "detach")
        except Exception as e:  # collected
            errs.append(repr(e))
            bar.abort()

    ths = [threading.Thread(target=bulk, args=(r,)) for r in range(bulk_ranks)]
    ths += [threading.Thread(target=latency, args=(bulk_ranks + i, i)) for i in range(lat_ranks)]
    [t.start() for t in ths]
    try:
        bar.wait()  # uploads done
        G.gvm_stats_reset()
        window["t0"] = time.monotonic() + 0.2   # bulk ranks start first; latency arrivals from t0
        window["t1"] = window["t0"] + seconds
        bar.wait()
        time.sleep(max(0.0, window["t1"] - time.monotonic()))
    except threading.BrokenBarrierError:
        pass
    stop.set()
    [t.join() for t in ths]
    st = G.gvm_stats_json()
    G.check(G.gvm_shutdown(), "shutdown")
    if errs:
        raise RuntimeError(errs)
    in_window = [x for x in bulk_done if window["t0"] <= x < window["t1"]]
    every = [v for vs in lat_us.values() for v in vs]
    return {
        "latency_cus": latency_cus, "bulk_ranks": bulk_ranks, "latency_ranks": lat_ranks,
        "latency_class_us": {"count": len(every), "p50": _pct(every, 50), "p99": _pct(every, 99),
                             "max": round(max(every), 1) if every else None},
        "per_kernel_us": {k: {"count": len(v), "p50": _pct(v, 50), "p99": _pct(v, 99)} for k, v in lat_us.items()},
        "bulk_sgemm_TFLOPs": round(len(in_window) * 2.0 * BULK_N ** 3 / seconds / 1e12, 2),
        "partition_launches": st["device"].get("partition_launches"),
        "partition_masked": st["device"].get("partition_masked"),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=3.0)
    ap.add_argument("--bulk-ranks", type=int, default=4)
    ap.add_argument("--latency-ranks", type=int, default=8)
    ap.add_argument("--rate", type=float, default=250.0, help="arrivals per second per latency rank")
    ap.add_argument("--json", default=None)
    ap.add_argument("--loopback", action="store_true", help=argparse.SUPPRESS)  # host-protocol dry run, no GPU
    a = ap.parse_args(argv)
    cases = [("alone", 0, 0, True), ("shared", 0, a.bulk_ranks, True), ("streams", 64, a.bulk_ranks, False),
             ("cus=32", 32, a.bulk_ranks, True), ("cus=64", 64, a.bulk_ranks, True)]
    rows = []
    for name, cus, bulk, masked in cases:
        os.environ["GVM_PARTITION_MASKS"] = "1" if masked else "0"
        try:
            row = {"case": name, **run_case(cus, bulk, a.latency_ranks, a.rate, a.seconds, a.loopback)}
        finally:
            os.environ.pop("GVM_PARTITION_MASKS", None)
        rows.append(row)
        print(json.dumps(row), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
