"""The execution model of Section 4.2.3 against the GVM on an MI355X (the
paper's model-validation experiment of Section 6).

For each kernel and programming style, the per-rank transfer and compute
times are profiled with one rank (medians over 24 requests after 4 of
warm-up, each copy and launch timed with device events on the same copy
FIFOs and kernel streams the batches use), then N = 1..64 ranks (1..8 for
VecMul) run one request each as one batch, and the device phase of the batch (first copy-in to last
copy-out, device events) is compared with the closed forms (Eq. 2/4 for
PS-1, Eq. 3/7 for PS-2) and with the discrete-event schedule under the
paper's single-queue rules and under independent queues.  Every kernel here
but EP is I/O-intensive on this machine (PCIe ~57 GB/s against ~110 TFLOP/s
FP32); EP moves 112 bytes per request and is compute-intensive.

The table goes to stdout (and to $GVM_VALIDATION_OUT as JSON when set).  The
assertions are loose sanity bounds: the point is the reported deviations.
"""

import json
import os
import statistics
import threading

import numpy as np
import pytest

from oracle import des
from oracle import model
from paper_1511_07658_amd import gvm as G
from paper_1511_07658_amd import spmd

pytestmark = pytest.mark.gpu

# vecadd 4M, VecMul of Table 3 (16M floats; its 15 iterations are the
# repeated batches), SGEMM 1024, and the compute-intensive case: EP-like with
# one work unit (2^15 pairs), i.e. one workgroup per request, the "kernel
# size one" of the paper's EP(M24) validation
# N runs to 64 ranks (one request each per batch) except for VecMul, whose
# 256 MB per rank stops at 8
NS_WIDE = [1, 2, 4, 8, 16, 32, 64]
CASES = [("vecadd", G.GVM_K_VECADD, 1 << 22, 5, NS_WIDE), ("vecmul", G.GVM_K_VECMUL, 1 << 24, 15, [1, 2, 4, 8]),
         ("sgemm", G.GVM_K_SGEMM, 1024, 5, NS_WIDE), ("ep", G.GVM_K_EP, 1 << 15, 5, NS_WIDE)]
PROFILE_WARM, PROFILE_REPS = 4, 24


def _run(ns, kernel_id, n, nranks, reps):
    """`nranks` rank threads, `reps` batches of one request per rank (inputs
    built in shared memory); returns the manager statistics."""
    errs = []
    bar = threading.Barrier(nranks)

    def rank(r):
        try:
            assert G.gvm_attach_ns(ns, r) == 0
            ni, no = G.in_elems(kernel_id, n), G.out_elems(kernel_id, n)
            view = G.gvm_rank_buffer(r, (ni + no) * 4)
            view[:ni] = spmd.make_input(kernel_id, 71, r, n)
            for _ in range(reps):
                bar.wait()
                t = G.gvm_submit(r, kernel_id, view[:ni], view[ni:ni + no], n)
                assert t > 0 and G.gvm_wait(r, t, 60_000_000_000) == 0
            assert G.gvm_detach(r) == 0
        except Exception as e:  # collected
            errs.append(repr(e))
            bar.abort()

    ths = [threading.Thread(target=rank, args=(r,)) for r in range(nranks)]
    [t.start() for t in ths]
    [t.join() for t in ths]
    assert not errs, errs
    return G.gvm_stats_json()


def test_execution_model_on_mi355x(ns_name):
    rows = []
    for name, kid, n, reps, ns_list in CASES:
        space = (G.in_elems(kid, n) + G.out_elems(kid, n)) * 4 + (1 << 20)
        for policy, pname in ((G.GVM_POLICY_PS1, "PS1"), (G.GVM_POLICY_PS2, "PS2")):
            ns = f"{ns_name}.{name}.{pname}"
            cfg = G.gvm_config_default(nranks=ns_list[-1], shm_bytes_per_rank=space, hbm_budget_bytes=8 << 30,
                                       policy=policy, batch_timing=1, batch_window_us=10_000_000, name=ns)
            G.check(G.gvm_init(cfg), "gvm_init")
            try:
                # one untimed batch over every rank first: the first copy into a
                # fresh device slot runs several times slower than later ones
                _run(ns, kid, n, ns_list[-1], 1)
                # profile one rank: T_in, T_out, T_comp as medians of the timed
                # copies and launches after a warm-up
                G.gvm_stats_reset()
                st = _run(ns, kid, n, 1, PROFILE_WARM + PROFILE_REPS)
                tm = st["timing"]
                assert len(tm["h2d_us"]) == len(tm["d2h_us"]) == PROFILE_WARM + PROFILE_REPS, tm
                t_in = statistics.median(tm["h2d_us"][PROFILE_WARM:]) * 1e-6
                t_out = statistics.median(tm["d2h_us"][PROFILE_WARM:]) * 1e-6
                t_comp = statistics.median(tm["launch_us"][PROFILE_WARM:]) * 1e-6
                for N in ns_list:
                    G.gvm_stats_reset()
                    st = _run(ns, kid, n, N, reps)
                    spans = st["timing"]["batch_device_us"]
                    assert len(spans) == reps, (N, spans)
                    meas = statistics.median(spans) * 1e-6
                    closed = model.modelled_total(pname, N, t_in, t_comp, t_out)
                    des_paper = des.simulate(pname, N, t_in, t_comp, t_out, "paper")
                    des_multi = des.simulate(pname, N, t_in, t_comp, t_out, "multiqueue")
                    rows.append({
                        "kernel": name, "n": n, "style": pname, "N": N,
                        "class": model.classify(t_in, t_comp, t_out),
                        "t_in_us": round(t_in * 1e6, 2), "t_comp_us": round(t_comp * 1e6, 2),
                        "t_out_us": round(t_out * 1e6, 2), "measured_us": round(meas * 1e6, 2),
                        "closed_form_us": round(closed * 1e6, 2), "des_paper_us": round(des_paper * 1e6, 2),
                        "des_multiqueue_us": round(des_multi * 1e6, 2),
                        "dev_closed": round(abs(meas - closed) / meas, 4),
                        "dev_des_multiqueue": round(abs(meas - des_multi) / meas, 4),
                    })
            finally:
                G.gvm_shutdown()
    hdr = ["kernel", "style", "N", "class", "t_in_us", "t_comp_us", "t_out_us", "measured_us", "closed_form_us",
           "des_multiqueue_us", "dev_closed", "dev_des_multiqueue"]
    print("\n" + " | ".join(hdr))
    for r in rows:
        print(" | ".join(str(r[h]) for h in hdr))
    out = os.environ.get("GVM_VALIDATION_OUT")
    if out:
        with open(out, "w") as f:
            json.dump(rows, f, indent=1)
    # sanity: one rank's device phase is its copy-in + kernel + copy-out
    for r in rows:
        if r["N"] == 1:
            one = r["t_in_us"] + r["t_comp_us"] + r["t_out_us"]
            assert 0.5 * one <= r["measured_us"] <= 2.0 * one + 50, r
        assert r["measured_us"] > 0
