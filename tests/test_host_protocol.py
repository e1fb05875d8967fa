"""Host logic of the manager on the loopback backend (no GPU, no kernel
arithmetic): C-ABI exports, shared-memory rings and allocator, request
barrier, admission under a device-memory budget, rank and manager failure.

The loopback backend copies each request's first out_bytes of input to its
output, which lets these tests check routing: every rank must get back its
own bytes."""

import ctypes
import glob
import os
import signal
import subprocess
import threading
import time

import numpy as np
import pytest

from oracle import serving as sv
from paper_1511_07658_amd import gvm as G
from paper_1511_07658_amd import spmd


def loop_cfg(name, **kw):
    base = dict(nranks=4, shm_bytes_per_rank=4 << 20, hbm_budget_bytes=64 << 20,
                backend=G.GVM_BACKEND_LOOPBACK, batch_window_us=1000, name=name)
    base.update(kw)
    return G.gvm_config_default(**base)


class Manager:
    def __init__(self, name, **kw):
        self.cfg = loop_cfg(name, **kw)

    def __enter__(self):
        G.check(G.gvm_init(self.cfg), "gvm_init")
        return self

    def __exit__(self, *a):
        G.gvm_shutdown()


def expect_loopback(kernel_id, inp, n):
    return inp[: G.out_elems(kernel_id, n)] if inp.size >= G.out_elems(kernel_id, n) else \
        np.concatenate([inp, np.zeros(G.out_elems(kernel_id, n) - inp.size, np.float32)])


def test_library_exports_every_header_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", G.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    declared = G.header_symbols()
    assert declared, "no declarations found in include/gvm.h"
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    G.lib()  # loads and binds every symbol


def test_config_struct_matches_c_layout():
    cfg = G.gvm_config_default()
    assert cfg.size == ctypes.sizeof(G.gvm_config)
    assert cfg.nranks == 8 and abs(cfg.bs_rate - 0.02) < 1e-7 and abs(cfg.bs_volatility - 0.30) < 1e-7


def test_bad_config_rejected(ns_name):
    assert G.gvm_init(loop_cfg(ns_name, nranks=0)) == G.GVM_EINVAL
    assert G.gvm_init(loop_cfg(ns_name, hbm_budget_bytes=1000)) == G.GVM_EINVAL
    cfg = loop_cfg(ns_name)
    cfg.size = 7
    assert G.gvm_init(cfg) == G.GVM_EINVAL


def test_threads_get_their_own_data_back(ns_name):
    with Manager(ns_name, nranks=4):
        errs = []

        def rank(r):
            assert G.gvm_attach_ns(ns_name, r) == 0
            for i, (k, n) in enumerate([(1, 1), (1, 4097), (2, 333), (3, 17), (4, 5), (5, 7), (5, 1 << 20)]):
                inp = (np.arange(G.in_elems(k, n), dtype=np.float32) + 1000 * r + 10 * i)
                out = np.full(G.out_elems(k, n), -1, np.float32)
                t = G.gvm_submit(r, k, inp, out, n)
                if t < 0 or G.gvm_wait(r, t, 5_000_000_000) != 0:
                    errs.append((r, i, G.gvm_last_error()))
                elif not np.array_equal(out, expect_loopback(k, inp, n)):
                    errs.append((r, i, "wrong bytes"))
            assert G.gvm_detach(r) == 0

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(4)]
        [t.start() for t in ths]
        [t.join() for t in ths]
        assert not errs, errs


def test_ring_wraparound_and_many_outstanding(ns_name):
    # more requests in flight than ring entries, sizes that wrap the allocator
    with Manager(ns_name, nranks=1, mode=G.GVM_MODE_SERVING, shm_bytes_per_rank=1 << 20):
        assert G.gvm_attach_ns(ns_name, 0) == 0
        tickets, outs, ins = [], [], []
        for i in range(300):
            n = 1000 + (i * 7919) % 20000
            inp = np.full(2 * n, float(i), np.float32)
            out = np.zeros(n, np.float32)
            t = G.gvm_submit(0, G.GVM_K_VECADD, inp, out, n)
            assert t == i + 1, (t, G.gvm_last_error())
            tickets.append(t); outs.append(out); ins.append(inp)
        assert G.gvm_wait(0, -1, 10_000_000_000) == 0
        for i, out in enumerate(outs):
            assert np.all(out == float(i))
        assert G.gvm_detach(0) == 0


def test_nonblocking_submit_reports_eagain(ns_name):
    # batch mode with two ranks: rank 0's requests wait for the barrier
    with Manager(ns_name, nranks=2, batch_window_us=2_000_000):
        assert G.gvm_attach_ns(ns_name, 0) == 0
        assert G.gvm_attach_ns(ns_name, 1) == 0
        inp = np.ones(8, np.float32)
        outs = [np.zeros(4, np.float32) for _ in range(70)]
        got = []
        for o in outs:
            t = G.gvm_submit_ex(0, G.GVM_K_VECADD, inp, o, 4, G.GVM_F_NONBLOCK)
            got.append(t)
            if t == G.GVM_EAGAIN:
                break
        assert got[-1] == G.GVM_EAGAIN and len(got) == 64  # ring capacity - 1 outstanding
        assert G.gvm_wait(0, -1, 10_000_000_000) == 0       # the window expires, all run
        G.gvm_detach(0)
        G.gvm_detach(1)


def test_batch_barrier_holds_until_all_ranks_submit(ns_name):
    with Manager(ns_name, nranks=2, batch_window_us=5_000_000):
        assert G.gvm_attach_ns(ns_name, 0) == 0
        assert G.gvm_attach_ns(ns_name, 1) == 0
        inp = np.ones(8, np.float32)
        o0, o1 = np.zeros(4, np.float32), np.zeros(4, np.float32)
        t0 = G.gvm_submit(0, 1, inp, o0, 4)
        assert G.gvm_wait(0, t0, 200_000_000) == G.GVM_ETIMEDOUT  # barrier not reached
        t1 = G.gvm_submit(1, 1, inp, o1, 4)
        st0, ts0 = G.gvm_wait_timed(0, t0, 5_000_000_000)
        st1, ts1 = G.gvm_wait_timed(1, t1, 5_000_000_000)
        assert st0 == 0 and st1 == 0
        assert abs(int(ts0[1]) - int(ts1[1])) < 50_000_000  # admitted together
        assert ts0[0] <= ts0[1] <= ts0[2] <= ts0[3] <= ts0[4]
        G.gvm_detach(0)
        G.gvm_detach(1)


@pytest.mark.parametrize("early", [1, 0])
def test_batch_early_copy_in_moves_inputs_before_the_barrier(ns_name, early):
    """Batch mode, two SPMD ranks of very different sizes: the small rank is
    answered first and resubmits while the large rank's result is still
    being copied out.  With early copy-in its next request is admitted (its
    input starts moving) before the large rank has submitted, yet its
    kernel is launched only after that submit (the request barrier); without
    it, admission waits for the barrier.  Every result carries its own
    bytes."""
    sizes = [1024, 4 << 20]
    steps = 12
    with Manager(ns_name, nranks=2, batch_window_us=5_000_000, early_copy_in=early, copy_threads=1,
                 shm_bytes_per_rank=(3 * max(sizes)) * 4 + (1 << 20), hbm_budget_bytes=512 << 20):
        stamps = [[None] * steps for _ in range(2)]
        errs = []
        go = threading.Barrier(2)

        def rank(r):
            assert G.gvm_attach_ns(ns_name, r) == 0
            n = sizes[r]
            go.wait()
            for step in range(steps):
                inp = np.arange(2 * n, dtype=np.float32) + 3 * step + r
                out = np.zeros(n, np.float32)
                t = G.gvm_submit(r, G.GVM_K_VECADD, inp, out, n)
                st, ts = G.gvm_wait_timed(r, t, 20_000_000_000)
                if t < 0 or st != 0:
                    errs.append((r, step, st, G.gvm_last_error()))
                elif not np.array_equal(out, inp[:n]):
                    errs.append((r, step, "wrong bytes"))
                stamps[r][step] = [int(x) for x in ts]
            assert G.gvm_detach(r) == 0

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(2)]
        [t.start() for t in ths]
        [t.join() for t in ths]
        assert not errs, errs
    ahead = 0
    for step in range(steps):
        small, large = stamps[0][step], stamps[1][step]
        assert small[2] >= large[0] and large[2] >= small[0], step  # kernels after the barrier
        ahead += small[1] < large[0]                              # admitted before the barrier
    if early:
        assert ahead > 0
    else:
        assert ahead == 0


def test_batch_per_rank_chains_launch_in_chunks(ns_name):
    """Batch mode with large copies (AUTO picks per-rank chains): the ready
    requests of a batch are handed to the device at most four per service
    iteration, so twelve ranks take at least three launch calls per step,
    and every result still carries its own bytes."""
    nranks, steps, n = 12, 5, 600_000          # 7.2 MB in, 2.4 MB out: pieces, not local
    with Manager(ns_name, nranks=nranks, batch_window_us=5_000_000, copy_threads=2,
                 shm_bytes_per_rank=(3 * n) * 4 + (1 << 20), hbm_budget_bytes=1 << 30):
        errs = []
        go = threading.Barrier(nranks)

        def rank(r):
            assert G.gvm_attach_ns(ns_name, r) == 0
            go.wait()
            for step in range(steps):
                inp = np.arange(2 * n, dtype=np.float32) + 5 * step + r
                out = np.zeros(n, np.float32)
                t = G.gvm_submit(r, G.GVM_K_VECADD, inp, out, n)
                if t < 0 or G.gvm_wait(r, t, 20_000_000_000) != 0:
                    errs.append((r, step, G.gvm_last_error()))
                elif not np.array_equal(out, inp[:n]):
                    errs.append((r, step, "wrong bytes"))
            assert G.gvm_detach(r) == 0

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(nranks)]
        [t.start() for t in ths]
        [t.join() for t in ths]
        assert not errs, errs
        st = G.gvm_stats_json()
        assert st["requests_done"] == nranks * steps
        assert st["batches"] >= 3 * steps, st["batches"]


@pytest.mark.parametrize("mode", [G.GVM_MODE_SERVING, G.GVM_MODE_BATCH])
@pytest.mark.parametrize("timing", [0, 1])
def test_large_requests_move_in_pieces(ns_name, timing, mode):
    # serving mode: inputs of 5 and 9 pieces (8 MiB each, the last one
    # short), outputs of 3 and 5; batch mode: 2 and 3 pieces of 32 MiB, and
    # 1 and 2; with batch_timing the copies are whole instead
    sizes = [5_000_003, 9_000_001]
    with Manager(ns_name, nranks=2, mode=mode, batch_timing=timing,
                 shm_bytes_per_rank=(3 * max(sizes) + 8) * 4 + (1 << 20), hbm_budget_bytes=1 << 30):
        errs = []

        def rank(r):
            assert G.gvm_attach_ns(ns_name, r) == 0
            n = sizes[r]
            inp = np.arange(2 * n, dtype=np.float32) * (r + 1)
            out = np.zeros(n, np.float32)
            for rep in range(2):
                t = G.gvm_submit(r, G.GVM_K_VECADD, inp, out, n)
                if t < 0 or G.gvm_wait(r, t, 20_000_000_000) != 0:
                    errs.append((r, G.gvm_last_error()))
                elif not np.array_equal(out, inp[:n]):
                    errs.append((r, rep, "wrong bytes"))
                out[:] = 0
            assert G.gvm_detach(r) == 0

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(2)]
        [t.start() for t in ths]
        [t.join() for t in ths]
        assert not errs, errs


def test_batch_timing_enqueues_whole_batches(ns_name):
    # PS-2 with copies starts each rank's chain as its input lands; with
    # batch_timing a batch goes to the device as one launch (one span)
    reps, nranks = 3, 4
    with Manager(ns_name, nranks=nranks, policy=G.GVM_POLICY_PS2, batch_timing=1, batch_window_us=10_000_000):
        G.gvm_stats_reset()
        bar = threading.Barrier(nranks)
        errs = []

        def rank(r):
            assert G.gvm_attach_ns(ns_name, r) == 0
            bar.wait()
            for i in range(reps):
                inp = np.full(2 * 4096, float(r * 10 + i), np.float32)
                out = np.zeros(4096, np.float32)
                t = G.gvm_submit(r, G.GVM_K_VECADD, inp, out, 4096)
                if t < 0 or G.gvm_wait(r, t, 5_000_000_000) != 0 or not np.all(out == float(r * 10 + i)):
                    errs.append((r, i, G.gvm_last_error()))
                bar.wait()
            assert G.gvm_detach(r) == 0

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(nranks)]
        [t.start() for t in ths]
        [t.join() for t in ths]
        assert not errs, errs
        st = G.gvm_stats_json()
        assert st["requests_done"] == reps * nranks
        assert st["batches"] == reps, st["batches"]


def test_invalid_requests(ns_name):
    with Manager(ns_name, nranks=1, shm_bytes_per_rank=1 << 20):
        x = np.zeros(16, np.float32)
        assert G.gvm_submit(0, 1, x, x, 4) == G.GVM_ESTATE          # not attached
        assert G.gvm_attach_ns(ns_name, 0) == 0
        assert G.gvm_attach_ns(ns_name, 0) == G.GVM_ESTATE          # twice
        assert G.gvm_submit(0, 1, x, x, 0) == G.GVM_EINVAL          # n == 0
        assert G.gvm_submit(0, 99, x, x, 4) == G.GVM_EINVAL         # unknown kernel
        assert G.gvm_submit(0, 1, None, x, 4) == G.GVM_EINVAL       # no input
        assert G.gvm_submit(0, 1, x, x, 1 << 20) == G.GVM_ENOMEM    # larger than the space
        assert G.gvm_submit_ex(0, 1, x, x, 4, 1 << 8) == G.GVM_EINVAL  # unknown flag
        # resident input that was never uploaded
        t = G.gvm_submit_ex(0, 1, None, x, 4, G.GVM_F_IN_RESIDENT)
        assert t > 0 and G.gvm_wait(0, t, 2_000_000_000) == G.GVM_ESTATE
        assert G.gvm_wait(0, 12345, 1000) == G.GVM_EINVAL            # unknown ticket
        assert G.gvm_attach_ns(ns_name, 5) == G.GVM_EINVAL           # rank >= nranks
        G.gvm_detach(0)


def test_resident_and_zero_copy(ns_name):
    with Manager(ns_name, nranks=1):
        assert G.gvm_attach_ns(ns_name, 0) == 0
        n = 1000
        view = G.gvm_rank_buffer(0, 3 * n * 4)
        view[: 2 * n] = np.arange(2 * n, dtype=np.float32)
        out_view = view[2 * n: 3 * n]
        t = G.gvm_submit(0, 1, view[: 2 * n], out_view, n)          # zero copy both ways
        assert G.gvm_wait(0, t, 2_000_000_000) == 0
        assert np.array_equal(out_view, np.arange(n, dtype=np.float32))
        out = np.zeros(n, np.float32)
        t = G.gvm_submit_ex(0, 1, None, out, n, G.GVM_F_IN_RESIDENT)  # reuse the device input
        assert G.gvm_wait(0, t, 2_000_000_000) == 0
        assert np.array_equal(out, np.arange(n, dtype=np.float32))
        t = G.gvm_submit_ex(0, 1, None, None, n, G.GVM_F_IN_RESIDENT | G.GVM_F_OUT_RESIDENT)
        assert G.gvm_wait(0, t, 2_000_000_000) == 0
        # a different size invalidates the resident input
        t = G.gvm_submit_ex(0, 1, None, out, n - 1, G.GVM_F_IN_RESIDENT)
        assert G.gvm_wait(0, t, 2_000_000_000) == G.GVM_ESTATE
        G.gvm_detach(0)


def test_serving_budget_admission_and_eviction(ns_name):
    # 8 ranks, budget of 2 MiB: at most a few resident slots; every request
    # must still complete, with its own data, and the peak stays in budget
    budget = 2 << 20
    with Manager(ns_name, nranks=8, mode=G.GVM_MODE_SERVING, hbm_budget_bytes=budget, max_inflight=3):
        errs, ends = [], []

        def rank(r):
            assert G.gvm_attach_ns(ns_name, r) == 0
            for i in range(20):
                n = 20000 + 1000 * ((r + i) % 7)
                inp = np.full(2 * n, float(100 * r + i), np.float32)
                out = np.zeros(n, np.float32)
                t = G.gvm_submit(r, 1, inp, out, n)
                st, ts = G.gvm_wait_timed(r, t, 10_000_000_000)
                if st != 0 or not np.all(out == float(100 * r + i)):
                    errs.append((r, i, st))
                ends.append((ts[1], ts[4], (r, t), 2 * 4096 * ((n * 12 + 4095) // 4096)))
            G.gvm_detach(r)

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(8)]
        [t.start() for t in ths]
        [t.join() for t in ths]
        assert not errs, errs
        st = G.gvm_stats_json()
        assert st["requests_done"] == 160
        assert 0 < st["peak_device_bytes"] <= budget
        # no more than max_inflight requests between admission and completion
        events = [(a, "admit", k, 1) for a, _, k, _ in ends] + [(d, "complete", k, 1) for _, d, k, _ in ends]
        assert sv.check_budget(events, 3) <= 3
        sv.check_lifecycle([k for _, _, k, _ in ends], events)


def test_forked_rank_processes(ns_name):
    with Manager(ns_name, nranks=4):
        jobs = [(1, 0, 5000, 0, False), (2, 0, 777, 1, False), (3, 0, 33, 2, False)]
        res = spmd.run_processes(spmd.rank_program, [(ns_name, r, jobs, True) for r in range(4)], timeout_s=60)
        for r, rr in enumerate(res):
            assert rr["attach"] == 0 and rr["detach"] == 0
            for (k, cfg, n, req, integer), jr in zip(jobs, rr["results"]):
                assert jr["status"] == 0, jr
                x = spmd.make_input(k, cfg, r, n, req, integer)
                assert np.array_equal(jr["out"], expect_loopback(k, x, n))


def test_forked_ranks_zero_copy(ns_name):
    with Manager(ns_name, nranks=2):
        jobs = [(1, 0, 3000, 0, False), (3, 0, 40, 0, False)]
        res = spmd.run_processes(spmd.rank_program, [(ns_name, r, jobs, True, True) for r in range(2)], timeout_s=60)
        for r, rr in enumerate(res):
            for (k, cfg, n, req, integer), jr in zip(jobs, rr["results"]):
                assert jr["status"] == 0
                assert np.array_equal(jr["out"], expect_loopback(k, spmd.make_input(k, cfg, r, n, req), n))


def _submit_then_hang(ns, rank, ready):
    assert G.gvm_attach_ns(ns, rank) == 0
    x = np.ones(8, np.float32)
    o = np.zeros(4, np.float32)
    G.gvm_submit(rank, 1, x, o, 4)
    ready.set()
    time.sleep(60)


def test_dead_rank_is_reclaimed(ns_name):
    with Manager(ns_name, nranks=2, batch_window_us=30_000_000):
        ctx = spmd.context()
        ready = ctx.Event()
        p = ctx.Process(target=_submit_then_hang, args=(ns_name, 0, ready), daemon=True)
        p.start()
        assert ready.wait(20)
        os.kill(p.pid, signal.SIGKILL)
        p.join()
        # the manager notices, drops the request and frees the VGPU
        deadline = time.time() + 5
        rc = G.GVM_ESTATE
        while time.time() < deadline:
            rc = G.gvm_attach_ns(ns_name, 0)
            if rc == 0:
                break
            time.sleep(0.05)
        assert rc == 0, G.gvm_last_error()
        x = np.arange(8, dtype=np.float32)
        o = np.zeros(4, np.float32)
        t = G.gvm_submit(0, 1, x, o, 4)
        # rank 1 is not attached, so the barrier is only rank 0
        assert G.gvm_wait(0, t, 5_000_000_000) == 0 and np.array_equal(o, x[:4])
        G.gvm_detach(0)


def _manager_process(ns, ready):
    cfg = loop_cfg(ns, nranks=2, batch_window_us=60_000_000)
    assert G.gvm_init(cfg) == 0
    ready.set()
    time.sleep(120)


def test_dead_manager_reported(ns_name):
    ctx = spmd.context()
    ready = ctx.Event()
    p = ctx.Process(target=_manager_process, args=(ns_name, ready), daemon=True)
    p.start()
    try:
        assert ready.wait(20)
        assert G.gvm_attach_ns(ns_name, 0) == 0
        assert G.gvm_attach_ns(ns_name, 1) == 0
        x = np.ones(8, np.float32)
        o = np.zeros(4, np.float32)
        t = G.gvm_submit(0, 1, x, o, 4)   # held by the barrier (rank 1 silent, long window)
        assert t > 0
        assert G.gvm_wait(0, t, 100_000_000) == G.GVM_ETIMEDOUT
        os.kill(p.pid, signal.SIGKILL)
        p.join()
        t0 = time.time()
        assert G.gvm_wait(0, t, 10_000_000_000) == G.GVM_EDEAD
        assert time.time() - t0 < 2.0
        assert G.gvm_detach(0) == 0
        assert G.gvm_detach(1) == 0
    finally:
        if p.is_alive():
            os.kill(p.pid, signal.SIGKILL)
        for f in glob.glob(f"/dev/shm/{ns_name}.*"):
            os.unlink(f)


def test_shutdown_removes_shared_memory(ns_name):
    with Manager(ns_name, nranks=3):
        assert len(glob.glob(f"/dev/shm/{ns_name}.*")) == 4
        assert G.gvm_attach_ns(ns_name, 1) == 0
    assert glob.glob(f"/dev/shm/{ns_name}.*") == []
    # a second manager in the same process after shutdown
    with Manager(ns_name, nranks=1):
        assert G.gvm_attach_ns(ns_name, 0) == 0
        assert G.gvm_init(loop_cfg(ns_name + "x")) == G.GVM_ESTATE  # one manager per process


def test_hip_backend_fails_loudly_without_gpu(ns_name):
    if os.path.exists("/dev/kfd"):
        pytest.skip("a GPU driver is present")
    cfg = G.gvm_config_default(nranks=1, shm_bytes_per_rank=1 << 20, hbm_budget_bytes=16 << 20, name=ns_name)
    assert G.gvm_init(cfg) == G.GVM_EDEVICE
    assert "HIP" in G.gvm_last_error() or "device" in G.gvm_last_error()
    assert glob.glob(f"/dev/shm/{ns_name}.*") == []


def test_graph_replay_not_combined_with_cu_partition(ns_name):
    cfg = loop_cfg(ns_name, use_graphs=1, mode=G.GVM_MODE_SERVING, latency_cus=64)
    assert G.gvm_init(cfg) == G.GVM_EINVAL
    assert "use_graphs" in G.gvm_last_error()


def _popcount(words):
    return sum(bin(w).count("1") for w in words)


@pytest.mark.parametrize("m", range(1, 8))
def test_cu_partition_masks_cover_every_xcd(m):
    # the two CU-masked partitions are disjoint, cover all 256 CUs, and give
    # every XCD the same share whether XCDs own CUs by i % 8 or by i / 32
    lat, bulk = G.gvm_cu_partition_masks(32 * m)
    assert len(lat) == len(bulk) == 8
    assert all((a & b) == 0 for a, b in zip(lat, bulk))
    assert all((a | b) == 0xFFFFFFFF for a, b in zip(lat, bulk))
    assert _popcount(lat) == 32 * m and _popcount(bulk) == 256 - 32 * m

    def bit(words, i):
        return (words[i // 32] >> (i % 32)) & 1

    for xcd_of in (lambda i: i % 8, lambda i: i // 32):
        for x in range(8):
            cus = [i for i in range(256) if xcd_of(i) == x]
            assert sum(bit(lat, i) for i in cus) == 4 * m
            assert sum(bit(bulk, i) for i in cus) == 32 - 4 * m


@pytest.mark.parametrize("bad", [0, 16, 33, 256, 512])
def test_cu_partition_masks_reject_bad_sizes(bad):
    with pytest.raises(G.GvmError):
        G.gvm_cu_partition_masks(bad)


def test_cu_partition_config_checks(ns_name):
    # serving mode only, multiples of 32 below 256
    for kw in (dict(latency_cus=64), dict(latency_cus=48, mode=G.GVM_MODE_SERVING),
               dict(latency_cus=256, mode=G.GVM_MODE_SERVING)):
        assert G.gvm_init(loop_cfg(ns_name, **kw)) == G.GVM_EINVAL
        assert "latency_cus" in G.gvm_last_error()


def test_cu_partition_serving_routes_both_classes(ns_name):
    # small requests (latency class) and large ones (the rest) from the same
    # ranks: each launches in its own class and gets its own data back
    with Manager(ns_name, nranks=4, mode=G.GVM_MODE_SERVING, latency_cus=64, shm_bytes_per_rank=64 << 20,
                 hbm_budget_bytes=256 << 20):
        errs = []

        def rank(r):
            assert G.gvm_attach_ns(ns_name, r) == 0
            for i in range(6):
                n = 1000 + r if i % 2 == 0 else (1 << 22) + r   # ~0 us vs ~10 us of vector add
                k = G.GVM_K_VECADD if i % 3 else G.GVM_K_SGEMM
                if k == G.GVM_K_SGEMM:
                    n = 64 if i % 2 == 0 else 1024               # ~0 us vs ~20 us
                inp = np.arange(G.in_elems(k, n), dtype=np.float32) + 7 * r + i
                out = np.zeros(G.out_elems(k, n), np.float32)
                t = G.gvm_submit(r, k, inp, out, n)
                st = G.gvm_wait(r, t, 30_000_000_000)
                if st != 0 or not np.array_equal(out, expect_loopback(k, inp, n)):
                    errs.append((r, i, st))
            G.gvm_detach(r)

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(4)]
        [t.start() for t in ths]
        [t.join() for t in ths]
        assert not errs, errs
        assert G.gvm_stats_json()["requests_done"] == 24


@pytest.mark.parametrize("n, expect", [(20_000, "grouped"), (400_000, "ps2")])
def test_auto_policy_size_rule(ns_name, n, expect):
    # AUTO: one grouped launch when every request's copies are small (kept on
    # the kernel's stream), PS-2 once a request moves more than 1 MiB
    with Manager(ns_name, nranks=4, policy=G.GVM_POLICY_AUTO, batch_window_us=10_000_000,
                 shm_bytes_per_rank=16 << 20):
        bar = threading.Barrier(4)
        errs = []

        def rank(r):
            assert G.gvm_attach_ns(ns_name, r) == 0
            bar.wait()
            inp = np.arange(2 * n, dtype=np.float32) + r
            out = np.zeros(n, np.float32)
            t = G.gvm_submit(r, G.GVM_K_VECADD, inp, out, n)
            if G.gvm_wait(r, t, 30_000_000_000) != 0 or not np.array_equal(out, expect_loopback(1, inp, n)):
                errs.append(r)
            G.gvm_detach(r)

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(4)]
        [t.start() for t in ths]
        [t.join() for t in ths]
        assert not errs
        pl = G.gvm_stats_json()["device"]["policy_launches"]
    other = "ps2" if expect == "grouped" else "grouped"
    assert pl[expect] >= 1 and pl[other] == 0, pl


def test_tile_configuration_names_match_the_compiled_table():
    # the tuner's names and count, the kernel's configuration table, the
    # launch switch and the size table must describe the same configurations
    import re
    from paper_1511_07658_amd import tune
    csrc = os.path.join(os.path.dirname(G.__file__), "csrc")
    src = open(os.path.join(csrc, "sgemm.hip")).read()
    rows = re.findall(r"\{(\d+), (\d+), (\d+), (\d+), (\d+), (\d+), (true|false)\}", src)
    assert [int(r[0]) for r in rows] == list(range(tune.NUM_CONFIGS))
    assert len(tune.CONFIG_NAMES) == tune.NUM_CONFIGS
    for (idx, bm, bn, bk, wm, wn, bt), name in zip(rows, tune.CONFIG_NAMES):
        m = re.match(r"(\d+)x(\d+)x(\d+)([TR])", name)
        assert m and m.groups() == (bm, bn, bk, "T" if bt == "true" else "R"), (idx, name)
    cases = [int(c) for c in re.findall(r"case (\d+): return launch_cfg<", src)]
    assert cases == list(range(tune.NUM_CONFIGS))
    # the launch switch instantiates the same shape as the table row
    for c, (bm, bn, bk, wm, wn, bt) in zip(cases, re.findall(
            r"case \d+: return launch_cfg<(\d+), (\d+), (\d+), (\d+), (\d+), (true|false)", src)):
        assert (bm, bn, bk, wm, wn, bt) == rows[c][1:], c
    table = open(os.path.join(csrc, "gemm_tiles.inc")).read()
    for n, c in re.findall(r"\{(\d+)u, (\d+)\}", table):
        assert 0 <= int(c) < tune.NUM_CONFIGS, (n, c)
    mix = int(re.search(r"constexpr int kMixConfig = (\d+);", open(os.path.join(csrc, "device_hip.cpp")).read()).group(1))
    assert 0 <= mix < tune.NUM_CONFIGS


def test_tuner_merges_sweeps_by_mean_time(tmp_path):
    # two saved sweeps: the mean time decides, a configuration timed in one
    # sweep only keeps that time, ties to 0.1 us go to the lower index, and
    # neighbouring sizes with one winner share a table row
    from paper_1511_07658_amd import tune
    a, b, c = tune.CONFIG_NAMES[3], tune.CONFIG_NAMES[16], tune.CONFIG_NAMES[27]
    s1 = {"512": {"best": 3, "us": {a: 10.0, b: 12.0}}, "1024": {"best": 16, "us": {b: 134.0, c: 137.0}},
          "2048": {"best": 3, "us": {a: 50.0, b: 50.04}}}
    s2 = {"512": {"best": 16, "us": {a: 11.0, b: 9.5}}, "1024": {"best": 27, "us": {b: 137.0, c: 133.0}},
          "1536": {"best": 27, "us": {c: 40.0}}}
    m = tune.merge_sweeps([s1, s2])
    assert m[512]["best"] == 3 and m[512]["us"][a] == 10.5 and m[512]["us"][b] == 10.75
    assert m[1024]["best"] == 27 and m[1024]["us"][c] == 135.0
    assert m[1536]["best"] == 27
    assert m[2048]["best"] == 3  # 50.0 and 50.04 tie at 0.1 us
    import re
    path = tmp_path / "tiles.inc"
    tune.write_table(m, path=str(path))
    rows = re.findall(r"\{(\d+)u, (\d+)\}", path.read_text())
    assert rows == [("512", "3"), ("1536", "27"), (str(1 << 30), "3")]


def test_serving_pipelines_two_requests_of_a_rank(ns_name):
    """Serving mode admits a rank's second plain request while its first is
    still in flight (its copy-in overlaps the first's copies and device
    work); every result still carries its own bytes, and a resident-input
    request afterwards either finds the latest request's input or is refused
    with GVM_ESTATE, never other bytes."""
    with Manager(ns_name, nranks=1, shm_bytes_per_rank=64 << 20, hbm_budget_bytes=256 << 20,
                 mode=G.GVM_MODE_SERVING, copy_threads=1):
        assert G.gvm_attach_ns(ns_name, 0) == 0
        overlapped = 0
        n = 2 << 20
        per = 3 * n                                  # input (2n) and output (n) of one request
        view = G.gvm_rank_buffer(0, 2 * per * 4)     # both requests zero-copy in the rank's space
        for rep in range(10):
            ins, outs = [], []
            for i in range(2):
                x = view[i * per: i * per + 2 * n]
                x[:] = np.arange(2 * n, dtype=np.float32) + 7 * rep + i
                ins.append(x.copy())
                outs.append(view[i * per + 2 * n: (i + 1) * per])
            tk = [G.check(G.gvm_submit(0, G.GVM_K_VECADD, view[i * per: i * per + 2 * n], outs[i], n), "submit")
                  for i in range(2)]
            ts = [G.gvm_wait_timed(0, t, 10_000_000_000) for t in tk]
            for i in range(2):
                assert ts[i][0] == 0 and np.array_equal(outs[i], ins[i][:n])
            # the second admitted (ts[1]) before the first was posted (ts[0])
            overlapped += ts[1][1][1] < ts[0][1][4]
            o = np.empty(n, np.float32)
            t = G.gvm_submit_ex(0, G.GVM_K_VECADD, None, o, n, G.GVM_F_IN_RESIDENT)
            assert t >= 0
            rc = G.gvm_wait(0, t, 10_000_000_000)
            assert rc in (0, G.GVM_ESTATE)
            if rc == 0:
                assert np.array_equal(o, ins[1][:n])
        assert overlapped > 0
        assert G.gvm_detach(0) == 0
