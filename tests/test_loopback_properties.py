"""Property tests of the manager's host protocol on the loopback backend (no
GPU): for random rank counts, modes, policies, kernel mixes and request
sizes (hypothesis), every request finishes with status 0 and every rank gets
back exactly its own bytes (the loopback device returns the first
output-sized bytes of the request's input, zero-padded), in submission
order per rank, whatever else is in the batch."""

import threading

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_1511_07658_amd import gvm as G

KERNELS = [G.GVM_K_VECADD, G.GVM_K_BLACKSCHOLES, G.GVM_K_SGEMM, G.GVM_K_VECMUL, G.GVM_K_EP]
MAX_N = {G.GVM_K_VECADD: 300_000, G.GVM_K_VECMUL: 300_000, G.GVM_K_BLACKSCHOLES: 200_000, G.GVM_K_SGEMM: 300,
         G.GVM_K_EP: 1 << 22}

request = st.tuples(st.sampled_from(KERNELS), st.floats(0.0, 1.0))
plan = st.fixed_dictionaries({
    "ranks": st.integers(1, 6),
    "mode": st.sampled_from([G.GVM_MODE_BATCH, G.GVM_MODE_SERVING]),
    "policy": st.sampled_from([G.GVM_POLICY_AUTO, G.GVM_POLICY_PS1, G.GVM_POLICY_PS2, G.GVM_POLICY_GROUPED]),
    "budget_mib": st.sampled_from([8, 32, 256]),
    "requests": st.lists(st.lists(request, min_size=1, max_size=5), min_size=6, max_size=6),
    "outstanding": st.integers(1, 3),
})

_ns = [0]


def size_of(k, f):
    return max(1, int(round(f * MAX_N[k])))


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(plan)
def test_every_rank_gets_its_own_bytes(p):
    _ns[0] += 1
    name = f"gvm.prop.{threading.get_ident() % 100000}.{_ns[0]}"
    cfg = G.gvm_config_default(nranks=p["ranks"], shm_bytes_per_rank=8 << 20, hbm_budget_bytes=p["budget_mib"] << 20,
                               backend=G.GVM_BACKEND_LOOPBACK, batch_window_us=300, mode=p["mode"],
                               policy=p["policy"], copy_threads=2, name=name)
    G.check(G.gvm_init(cfg), "gvm_init")
    errs = []
    try:
        def rank(r):
            G.check(G.gvm_attach_ns(name, r), "attach")
            live = []
            for i, (k, f) in enumerate(p["requests"][r]):
                n = size_of(k, f)
                inp = np.random.default_rng([r, i, n]).standard_normal(G.in_elems(k, n)).astype(np.float32)
                out = np.full(G.out_elems(k, n), np.nan, np.float32)
                t = G.gvm_submit(r, k, inp, out, n)
                if t < 0:
                    errs.append((r, i, k, n, t, G.gvm_last_error()))
                    continue
                live.append((t, k, n, inp, out))
                while len(live) >= p["outstanding"] or (i == len(p["requests"][r]) - 1 and live):
                    t0, k0, n0, x0, o0 = live.pop(0)
                    rc = G.gvm_wait(r, t0, 20_000_000_000)
                    m = G.out_elems(k0, n0)
                    want = x0[:m] if x0.size >= m else np.concatenate([x0, np.zeros(m - x0.size, np.float32)])
                    if rc != 0 or not np.array_equal(o0.view(np.uint32), want.view(np.uint32)):
                        errs.append((r, k0, n0, rc, G.gvm_last_error()))
            G.check(G.gvm_detach(r), "detach")

        ths = [threading.Thread(target=rank, args=(r,)) for r in range(p["ranks"])]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
    finally:
        G.gvm_shutdown()
    assert not errs, errs[:5]
