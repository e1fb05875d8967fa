"""Served results against the oracle: a short run of the serving
configuration (64 open-loop ranks, Poisson arrivals at 2000 requests/s in
total, vector add up to 2^24, Black-Scholes up to 4M options, SGEMM up to
2048^2, a 64 GiB HBM budget, resident buffers) through the load generator.
Every request must finish with status 0, and a seeded sample of the results
(every 40th request of each rank, those of at most 8 MiB) is checked against
the oracle with the same bars as the batch tests: vector add bit-exact,
Black-Scholes relative L2 <= 1e-5 per output vector, SGEMM relative
Frobenius error <= 1e-4 against float64."""

import numpy as np
import pytest

from oracle import kernels as ok
from paper_1511_07658_amd import gvm as G
from paper_1511_07658_amd import loadgen
from paper_1511_07658_amd import workloads as wl

pytestmark = pytest.mark.gpu

R32 = float(np.float32(wl.BS_RATE))
V32 = float(np.float32(wl.BS_VOLATILITY))


def test_serving_64_ranks_results_match_oracle():
    a = loadgen.parse_args(["--ranks", "64", "--rate", "2000", "--duration", "2.5", "--warmup", "0.5", "--no-plain",
                            "--sample-every", "40"])
    print("serving: 64 ranks, 2000 req/s, 2.5 s", flush=True)
    result, samples = loadgen.run(a)
    g = result["gvm"]
    print({k: g[k] for k in ("requests", "ok", "failed", "p50_ms", "p99_ms", "sampled_results")}, flush=True)
    assert g["failed"] == 0 and g["ok"] == g["requests"] > 0, g
    assert g["sampled_results"] >= 40, g["sampled_results"]
    kinds = set()
    for rank, got in samples.items():
        if not got:
            continue
        pool = loadgen._Inputs(rank)
        for idx, k, n, out in got:
            kinds.add(k)
            if k == G.GVM_K_VECADD:
                ref = ok.vecadd_f32(pool.a[:n], pool.b[:n])
                assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (rank, idx, n)
            elif k == G.GVM_K_BLACKSCHOLES:
                call, put = ok.black_scholes_f64(pool.S[:n], pool.K[:n], pool.T[:n], R32, V32)
                for got_v, ref in ((out[:n], call), (out[n:], put)):
                    rel = np.linalg.norm(got_v.astype(np.float64) - ref) / np.linalg.norm(ref)
                    assert rel <= 1e-5, (rank, idx, n, rel)
            else:
                A = pool.A[:n * n].reshape(n, n)
                B = pool.B[:n * n].reshape(n, n)
                ref = ok.sgemm_f64(A, B)
                rel = np.linalg.norm(out.reshape(n, n).astype(np.float64) - ref) / np.linalg.norm(ref)
                assert rel <= 1e-4, (rank, idx, n, rel)
    assert kinds == {G.GVM_K_VECADD, G.GVM_K_BLACKSCHOLES, G.GVM_K_SGEMM}, kinds
