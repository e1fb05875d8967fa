"""The load generator's open-loop ranks and its result sampling, on the
loopback backend (no GPU): every request of a short Poisson trace finishes
with status 0, and every sampled result holds the first output-sized bytes
of the request's own packed input, which is what the loopback device
returns.  The same sampling feeds the oracle check of served results on the
GPU (test_gpu_serving_oracle.py)."""

import numpy as np

from paper_1511_07658_amd import gvm as G
from paper_1511_07658_amd import loadgen


def test_loopback_serving_samples_carry_own_bytes():
    a = loadgen.parse_args(["--ranks", "4", "--rate", "120", "--duration", "0.8", "--warmup", "0.1", "--loopback",
                            "--sample-every", "1", "--copy-threads", "2"])
    result, samples = loadgen.run(a)
    g = result["gvm"]
    assert g["failed"] == 0 and g["ok"] == g["requests"] > 0, g
    assert g["sampled_results"] > 0
    for rank, got in samples.items():
        pool = loadgen._Inputs(rank)
        for idx, k, n, out in got:
            assert loadgen.sampled(rank, idx, k, n, 1)
            x = pool.packed(k, n)
            want = x[:G.out_elems(k, n)]
            assert np.array_equal(out.view(np.uint32), want.view(np.uint32)), (rank, idx, k, n)
