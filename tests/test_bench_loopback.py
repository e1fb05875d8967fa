"""bench.py's control flow on the loopback backend (no GPU): the default
workload's 32 rank processes run the warm-up, the timed steps with copies
and the resident steps, and the line carries the contract's keys.  The
numbers themselves mean nothing here (the loopback device computes no
kernel)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_on_loopback():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--loopback", "--steps", "2", "--warmup", "1",
                        "--resident-steps", "2", "--no-cpu-baseline", "--serving-seconds", "0"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=600, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-3000:]
    lines = [x for x in p.stdout.splitlines() if x.strip()]
    assert len(lines) == 1, p.stdout
    line = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "device_phase", "latency_us"):
        assert k in line, k
    assert line["config"]["name"] == "mixed32" and line["config"]["ranks"] == 32
    assert line["unit"] == "GFLOP/s" and line["n_gpus"] == 1 and line["steps"] == 2
    assert line["results_unchanged_by_virtualization"] is True
    assert line["roofline"]["bound"] == "mfma"
    # the resident leg's untimed steps cover about 60 ms of estimated device work
    sys.path.insert(0, ROOT)
    import bench
    w = bench.resident_warmup_steps(bench.rank_specs("mixed32"))
    assert line["device_phase"]["warmup_steps"] == w and 40 <= w <= 200


def test_resident_warmup_covers_the_clock_climb():
    sys.path.insert(0, ROOT)
    import bench
    for name in ("mixed32", "sgemm8", "vecadd16", "bs16", "ep8", "vecadd4"):
        specs = bench.rank_specs(name)
        w = bench.resident_warmup_steps(specs)
        assert 3 <= w <= 5000, (name, w)
    # 8 x 1024^2 SGEMM: 17.18 GFLOP at 110 TFLOP/s is 156 us, plus 50 us per step
    assert bench.resident_warmup_steps(bench.rank_specs("sgemm8")) == 292
    assert bench.resident_warmup_steps(bench.rank_specs("sgemm8"), target_ms=0.1) == 3


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2 and "one GPU only" in p.stderr
