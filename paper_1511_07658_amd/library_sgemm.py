"""The vendor library's FP32 GEMM on the same shapes as the grouped SGEMM.

A point of comparison for the hand-written kernel, not part of the path:
eight independent n x n FP32 products, as eight ranks submit them, run as
one batched library call (``torch.bmm`` on contiguous [8, n, n] tensors,
which ROCm's PyTorch hands to hipBLASLt or rocBLAS).  TF32-style reduced
precision is switched off, and each size's result is checked against a
float64 product on the CPU so that a reduced-precision path would show.

Prints one JSON object per size: mean device time per call (HIP events
around ``--iters`` calls on the current stream) and TFLOP/s.

    python -m paper_1511_07658_amd.library_sgemm [--sizes 256,512,1024,2048] [--batch 8]
"""

from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch


def run(n: int, batch: int, iters: int, warmup: int) -> dict:
    g = torch.Generator(device="cpu").manual_seed(1511 + n)
    a = torch.rand(batch, n, n, generator=g, dtype=torch.float32) * 2 - 1
    b = torch.rand(batch, n, n, generator=g, dtype=torch.float32) * 2 - 1
    da, db = a.cuda().contiguous(), b.cuda().contiguous()
    dc = torch.empty_like(da)
    for _ in range(warmup):
        torch.bmm(da, db, out=dc)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        torch.bmm(da, db, out=dc)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / iters
    # error of the first product against float64 on the CPU
    ref = a[0].double().numpy() @ b[0].double().numpy()
    got = dc[0].cpu().double().numpy()
    rel = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    flop = 2.0 * batch * n ** 3
    return {"n": n, "batch": batch, "us_per_call": round(us, 2), "TFLOPs": round(flop / us * 1e-6, 2),
            "max_rel_err_vs_f64": rel}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="256,512,768,1024,1536,2048")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("library_sgemm: needs a GPU", file=sys.stderr)
        return 2
    torch.backends.cuda.matmul.allow_tf32 = False
    torch.backends.cudnn.allow_tf32 = False
    print(json.dumps({"device": torch.cuda.get_device_name(0), "torch": torch.__version__,
                      "hip": torch.version.hip}), flush=True)
    for n in (int(x) for x in a.sizes.split(",")):
        print(json.dumps(run(n, a.batch, a.iters, a.warmup)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
