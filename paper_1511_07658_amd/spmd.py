"""SPMD rank processes for the GVM: the emulated SPMD method of Section 6
(the same program started in N processes), with ranks that never touch the
GPU and reach it only through the manager's shared memory.

Processes are forked from a multiprocessing fork server.  Call ``prestart()``
before anything in the calling process touches the GPU, so that the server
(and every rank forked from it) is a clean GPU-free process.
"""

from __future__ import annotations

import hashlib
import multiprocessing as mp
import os
import signal
import time
from multiprocessing import forkserver

import numpy as np

from . import gvm as G
from . import workloads as wl

_CTX = None


def context():
    global _CTX
    if _CTX is None:
        _CTX = mp.get_context("forkserver")
    return _CTX


def prestart():
    """Start the fork server now (while this process is GPU-free)."""
    context()
    forkserver.ensure_running()


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def make_input(kernel_id: int, config: int, rank: int, n: int, request: int = 0, integer: bool = False):
    """Packed input of one request, drawn from the seeded generators."""
    if kernel_id in (G.GVM_K_VECADD, G.GVM_K_VECMUL):
        return wl.pack_request(kernel_id, *wl.vecadd_inputs(config, rank, n, request))
    if kernel_id == G.GVM_K_BLACKSCHOLES:
        return wl.pack_request(kernel_id, *wl.bs_inputs(config, rank, n, request))
    if kernel_id == G.GVM_K_SGEMM:
        gen = wl.sgemm_int_inputs if integer else wl.sgemm_inputs
        return wl.pack_request(kernel_id, *gen(config, rank, n, request))
    if kernel_id == G.GVM_K_EP:
        return wl.ep_request(wl.ep_key(config, rank, request))
    raise ValueError(kernel_id)


def rank_program(ns: str, rank: int, jobs, return_outputs: bool = False, zero_copy: bool = False,
                 barrier=None, timeout_s: float = 120.0):
    """Attach as ``rank``, run ``jobs`` = [(kernel_id, config, n, request, integer), ...]
    one after another and return per-job {status, digest, out?, ts}."""
    rc = G.gvm_attach_ns(ns, rank)
    if rc != 0:
        return {"attach": rc, "error": G.gvm_last_error(), "results": []}
    if barrier is not None:
        barrier.wait()
    results = []
    for (k, cfg, n, req, integer) in jobs:
        x = make_input(k, cfg, rank, n, req, integer)
        out_n = G.out_elems(k, n)
        if zero_copy:
            view = G.gvm_rank_buffer(rank, (x.size + out_n) * 4)
            view[: x.size] = x
            inb = view[: x.size]
            outb = view[x.size: x.size + out_n]
        else:
            inb = x
            outb = np.empty(out_n, np.float32)
        t = G.gvm_submit(rank, k, inb, outb, n)
        if t < 0:
            results.append({"status": int(t), "error": G.gvm_last_error()})
            continue
        st, ts = G.gvm_wait_timed(rank, t, int(timeout_s * 1e9))
        res = {"status": st, "ts": ts}
        if st == 0:
            o = np.array(outb, copy=True)
            res["digest"] = digest(o)
            if return_outputs:
                res["out"] = o
        else:
            res["error"] = G.gvm_last_error()
        results.append(res)
    rc = G.gvm_detach(rank)
    return {"attach": 0, "detach": rc, "results": results}


def _entry(q, fn, args, kwargs):
    try:
        q.put((os.getpid(), fn(*args, **kwargs), None))
    except BaseException as e:  # report, never hang the parent
        q.put((os.getpid(), None, repr(e)))


def run_processes(fn, arg_list, kwargs_list=None, timeout_s: float = 300.0):
    """Run ``fn(*args)`` in one forked process per entry of ``arg_list``;
    returns the results in order.  Stragglers are killed at the timeout."""
    ctx = context()
    q = ctx.Queue()
    procs = []
    kwargs_list = kwargs_list or [{}] * len(arg_list)
    for args, kw in zip(arg_list, kwargs_list):
        p = ctx.Process(target=_entry, args=(q, fn, tuple(args), dict(kw)), daemon=True)
        p.start()
        procs.append(p)
    by_pid = {}
    deadline = time.time() + timeout_s
    while len(by_pid) < len(procs) and time.time() < deadline:
        try:
            pid, res, err = q.get(timeout=max(0.1, deadline - time.time()))
        except Exception:
            break
        by_pid[pid] = (res, err)
    for p in procs:
        p.join(timeout=max(0.1, deadline - time.time()))
        if p.is_alive():
            os.kill(p.pid, signal.SIGKILL)
            p.join()
    out = []
    for p in procs:
        res, err = by_pid.get(p.pid, (None, "no result (timeout or crash)"))
        if err:
            raise RuntimeError(f"rank process {p.pid} failed: {err}")
        out.append(res)
    return out
