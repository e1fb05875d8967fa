"""The per-request trace dump (gvm_trace_dump) on the loopback backend: a
valid Chrome trace-event JSON file with one track per rank and, for every
answered request, its stage slices in order (queued, copy-in, device,
copy-out) whose ends and starts chain without gaps; a reset empties it; no
manager means GVM_ESTATE."""

import json
import threading

import numpy as np

from paper_1511_07658_amd import gvm as G


def test_trace_dump_chrome_json(ns_name, tmp_path):
    cfg = G.gvm_config_default(nranks=3, shm_bytes_per_rank=4 << 20, hbm_budget_bytes=64 << 20,
                               backend=G.GVM_BACKEND_LOOPBACK, batch_window_us=500, mode=G.GVM_MODE_SERVING,
                               name=ns_name)
    G.check(G.gvm_init(cfg), "gvm_init")
    try:
        def rank(r):
            G.check(G.gvm_attach_ns(ns_name, r), "attach")
            for i, (k, n) in enumerate([(1, 1000 + r), (2, 500), (3, 33), (1, 70000)]):
                x = np.arange(G.in_elems(k, n), dtype=np.float32)
                o = np.empty(G.out_elems(k, n), np.float32)
                t = G.check(G.gvm_submit(r, k, x, o, n), "submit")
                G.check(G.gvm_wait(r, t, 5_000_000_000), "wait")
            G.check(G.gvm_detach(r), "detach")

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(3)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        path = str(tmp_path / "trace.json")
        assert G.gvm_trace_dump(path) == 0, G.gvm_last_error()
        with open(path) as f:
            doc = json.load(f)
        ev = doc["traceEvents"]
        assert doc["otherData"]["requests_traced"] == 12 == doc["otherData"]["requests_in_file"]
        tracks = {e["tid"] for e in ev if e["ph"] == "M" and e["name"] == "thread_name"}
        assert tracks == {0, 1, 2}
        slices = [e for e in ev if e["ph"] == "X"]
        by_req = {}
        for e in slices:
            by_req.setdefault((e["tid"], e["args"]["ticket"]), []).append(e)
        assert len(by_req) == 12
        for key, es in by_req.items():
            es.sort(key=lambda e: e["ts"])
            assert [e["name"] for e in es] == ["queued", "copy-in", "device", "copy-out"], key
            for a, b in zip(es, es[1:]):
                assert abs(a["ts"] + a["dur"] - b["ts"]) < 1e-2, (key, a, b)
            assert all(e["dur"] >= 0 and e["args"]["status"] == 0 for e in es)
        assert G.gvm_stats_reset() == 0
        assert G.gvm_trace_dump(path) == 0
        with open(path) as f:
            assert json.load(f)["otherData"]["requests_in_file"] == 0
        assert G.gvm_trace_dump(str(tmp_path / "no" / "such" / "dir.json")) == G.GVM_ESYS
    finally:
        G.gvm_shutdown()
    assert G.gvm_trace_dump(str(tmp_path / "x.json")) == G.GVM_ESTATE
