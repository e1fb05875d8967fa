"""SGEMM tile autotuner.

For every matrix size n of the search (default: the multiples of 64 in
[256, 2048] plus the small sizes), runs a grouped launch of ``--group``
identical-size requests (resident in HBM) through the GVM manager for every
compiled tile configuration, times the launches with the manager's HIP
events, and keeps the fastest configuration.  Each size starts with about
60 ms of untimed launches (the engine clock climbs for about 20 ms under
load), then passes over the configurations in index order and in reverse.  The result is written as the
compiled-in table ``csrc/gemm_tiles.inc`` (rows of {largest n, config}),
so the tile choice stays a pure function of n: a rank's SGEMM result does
not depend on what it is grouped with.

    python -m paper_1511_07658_amd.tune [--sizes 256,512,...] [--group 8] [--reps 10] [--rounds 2] [--write] [--json out.json]
    python -m paper_1511_07658_amd.tune --from-json a.json,b.json    # table from saved sweeps (mean time)

Timing needs the GPU; rebuild the library after writing the table.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import threading

import numpy as np

from . import gvm as G
from . import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "gemm_tiles.inc")
NUM_CONFIGS = 30
# "T": B staged k-contiguous (transposed) in LDS; "R": B row-major in LDS;
# "2", "3": k-tiles fetched two or three ahead instead of one; "P": the next
# k-tile's fragments read from LDS during the current MFMAs; "W4": registers
# held to four waves per SIMD
CONFIG_NAMES = ["64x64x16T", "128x64x16T", "128x128x16T", "128x128x32T", "256x128x16T", "128x256x16T",
                "256x128x32T", "64x128x16T", "128x128x16R", "256x128x16R", "128x256x16R", "256x128x32R",
                "128x128x32R", "64x128x16R", "256x128x16R2", "128x128x16R2", "256x128x32R2", "64x128x16R2",
                "128x128x32R2", "256x128x16R3", "256x128x32R3", "128x128x16R3", "256x128x16R2P", "128x128x32R2P",
                "128x128x16R2P", "64x128x16R2P", "256x128x16RP", "128x256x32R2",
                "256x256x16R2", "64x128x16R2W4"]


def warmup_launches(n, group, target_ms=60.0):
    """Launches of the first configuration, untimed, before a size is timed:
    about `target_ms` of device work at 110 TFLOP/s.  From an idle device
    (the ranks' uploads) the engine clock climbs for about 20 ms under load;
    configurations timed during the climb would be timed on a lower clock
    than the ones after them."""
    us = group * 2.0 * n ** 3 / 110e6 + 20.0
    return max(2, min(2000, int(-(-target_ms * 1e3 // us))))


def _time_size(ns, n, group, reps, configs, rounds=2):
    """Mean device time (us) of one grouped launch of `group` n x n GEMMs,
    per tile configuration: after a warm-up, `rounds` passes over the
    configurations, in index order and then in reverse, so that a slow drift
    of the clock weighs on every configuration alike."""
    bar = threading.Barrier(group + 1)
    stop = threading.Event()
    plan = {"launches": reps}
    errors = []

    def rank(r):
        try:
            A, B = wl.sgemm_inputs(90, r, n)
            x = wl.pack_request(3, A, B)
            out = np.empty(n * n, np.float32)
            G.check(G.gvm_attach_ns(ns, r), "attach")
            t = G.check(G.gvm_submit(r, 3, x, out, n), "upload")
            G.check(G.gvm_wait(r, t, 60_000_000_000), "upload")
            flags = G.GVM_F_IN_RESIDENT | G.GVM_F_OUT_RESIDENT
            bar.wait()  # uploads done
            while True:
                bar.wait()
                if stop.is_set():
                    break
                for _ in range(plan["launches"]):
                    t = G.check(G.gvm_submit_ex(r, 3, None, None, n, flags), "step")
                    G.check(G.gvm_wait(r, t, 60_000_000_000), "step")
                bar.wait()
            G.gvm_detach(r)
        except Exception as e:  # reported by the caller
            errors.append(repr(e))
            bar.abort()

    ths = [threading.Thread(target=rank, args=(r,)) for r in range(group)]
    for t in ths:
        t.start()
    total = {c: 0.0 for c in configs}
    count = {c: 0 for c in configs}
    try:
        bar.wait()  # uploads done
        os.environ["GVM_SGEMM_CONFIG"] = str(configs[0])
        plan["launches"] = warmup_launches(n, group)
        bar.wait()          # go (warm-up, untimed)
        bar.wait()          # done
        plan["launches"] = reps
        for k in range(rounds):
            for c in (configs if k % 2 == 0 else configs[::-1]):
                os.environ["GVM_SGEMM_CONFIG"] = str(c)
                G.gvm_stats_reset()
                bar.wait()          # go
                bar.wait()          # done
                st = G.gvm_stats_json()["kernels"]["sgemm"]
                total[c] += st["device_ms"]
                count[c] += st["launches"]
        stop.set()
        bar.wait()
    finally:
        os.environ.pop("GVM_SGEMM_CONFIG", None)
        for t in ths:
            t.join()
    if errors:
        raise RuntimeError(errors[0])
    return {c: total[c] / max(count[c], 1) * 1e3 for c in configs}


def tune(sizes, group=8, reps=10, configs=None, rounds=2):
    configs = list(range(NUM_CONFIGS)) if configs is None else configs
    ns = f"gvm.tune.{os.getpid()}"
    nmax = max(sizes)
    cfg = G.gvm_config_default(nranks=group, shm_bytes_per_rank=12 * nmax * nmax + (1 << 20),
                               hbm_budget_bytes=max(1 << 30, group * (12 * nmax * nmax + (1 << 20))),
                               batch_window_us=10_000_000, policy=G.GVM_POLICY_GROUPED, name=ns)
    G.check(G.gvm_init(cfg), "gvm_init")
    results = {}
    try:
        for n in sizes:
            # sizes change the resident input, so every size re-attaches
            t = _time_size(ns, n, group, reps, configs, rounds)
            best = min(t, key=lambda c: (round(t[c], 1), c))
            results[n] = {"best": best, "us": {CONFIG_NAMES[c]: round(v, 2) for c, v in t.items()},
                          "tflops": round(group * 2.0 * n ** 3 / (t[best] * 1e-6) / 1e12, 2)}
            print(json.dumps({"n": n, **results[n]}), flush=True)
    finally:
        G.gvm_shutdown()
    return results


def merge_sweeps(sweeps):
    """One result per size from several saved sweeps: the mean time of each
    configuration over the sweeps that timed it, fastest mean first (ties to
    0.1 us go to the lower configuration index)."""
    out = {}
    for n in sorted({int(k) for s in sweeps for k in s}):
        runs = [s[str(n)]["us"] for s in sweeps if str(n) in s]
        names = [c for c in CONFIG_NAMES if any(c in r for r in runs)]
        mean = {c: sum(r[c] for r in runs if c in r) / sum(1 for r in runs if c in r) for c in names}
        best = min(names, key=lambda c: (round(mean[c], 1), CONFIG_NAMES.index(c)))
        out[n] = {"best": CONFIG_NAMES.index(best), "us": {c: round(v, 2) for c, v in mean.items()}}
    return out


def write_table(results, path=TABLE):
    """The compiled-in table (every configuration gives a request the same
    bits, so the fastest one is taken)."""
    rows = []
    for n in sorted(results):
        c = results[n]["best"]
        if rows and rows[-1][1] == c:
            rows[-1][0] = n
        else:
            rows.append([n, c])
    rows[-1][0] = 1 << 30
    with open(path, "w") as f:
        f.write("// SGEMM tile table: rows of {largest n, tile configuration index},\n")
        f.write("// written by `python -m paper_1511_07658_amd.tune --write` on an MI355X\n")
        f.write("// (grouped launches of identical-size requests, fastest mean device time).\n")
        f.write("constexpr uint64_t kTileTable[][2] = {\n")
        for n, c in rows:
            f.write(f"    {{{n}u, {c}}},  // {CONFIG_NAMES[c]}\n")
        f.write("};\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default=None, help="comma-separated sizes (default 64,128,192 and 256..2048 step 64)")
    ap.add_argument("--group", type=int, default=8)
    ap.add_argument("--reps", type=int, default=10, help="launches per configuration per round")
    ap.add_argument("--rounds", type=int, default=2,
                    help="passes over the configurations after the warm-up (index order, then reverse)")
    ap.add_argument("--configs", default=None)
    ap.add_argument("--write", action="store_true")
    ap.add_argument("--json", default=None)
    ap.add_argument("--from-json", default=None,
                    help="write the table from saved sweeps (comma-separated --json outputs of runs on the GPU; "
                         "the mean time of each configuration decides) without timing")
    a = ap.parse_args(argv)
    if a.from_json:
        sweeps = []
        for path in a.from_json.split(","):
            with open(path) as f:
                sweeps.append(json.load(f))
        write_table(merge_sweeps(sweeps))
        print(f"wrote {TABLE} from {a.from_json}; rebuild the library", file=sys.stderr)
        return 0
    sizes = [int(s) for s in a.sizes.split(",")] if a.sizes else [64, 128, 192] + list(range(256, 2049, 64))
    configs = [int(c) for c in a.configs.split(",")] if a.configs else None
    res = tune(sizes, a.group, a.reps, configs, a.rounds)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)
    if a.write:
        write_table(res)
        print(f"wrote {TABLE}; rebuild the library", file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
