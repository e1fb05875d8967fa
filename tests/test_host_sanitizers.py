"""Host code under the compiler's sanitizers, on the CPU.

The manager's host side runs a service thread, a pool of staging-copy
threads, rank threads or processes, lock-free single-producer rings in shared
memory and futex doorbells.  tests/cpp/host_stress.cpp drives all of it on
the loopback backend (no GPU, no HIP runtime): several rank threads submit
seeded random requests of every kernel id in batch and serving mode under
each enqueue policy, with copy-in and zero-copy inputs, non-blocking
submission and all three kinds of wait, while a reader polls the
statistics; every result is checked byte for byte.  It is built twice from
the host sources with g++:

* ``-fsanitize=address,undefined`` (out-of-bounds and use-after-free
  accesses, leaks, undefined behaviour), and
* ``-fsanitize=thread`` (data races between the threads).

Either build must report nothing and every request must come back intact.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_07658_amd", "csrc")
HOST_SOURCES = ["manager.cpp", "rank.cpp", "shm.cpp", "common.cpp", "copy_pool.cpp", "abi.cpp",
                "batch_plan.cpp", "device_loopback.cpp"]

SANITIZERS = {
    "address": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
    "thread": ["-fsanitize=thread"],
}

# (mode, policy, ranks, requests per rank); mode 0 batch, 1 serving; policy
# 0 auto, 1 PS-1, 2 PS-2, 3 grouped
RUNS = [(0, 3, 6, 40), (0, 2, 4, 30), (1, 0, 8, 60), (1, 1, 5, 30)]


def build(tmp_path, kind):
    out = tmp_path / kind
    out.mkdir()
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
             f"-I{ROOT}/include", f"-I{CSRC}", *SANITIZERS[kind]]
    srcs = [os.path.join(CSRC, s) for s in HOST_SOURCES] + [
        os.path.join(ROOT, "tests", "cpp", "no_hip_device.cpp"), os.path.join(ROOT, "tests", "cpp", "host_stress.cpp")]

    def compile_one(src):
        obj = str(out / (os.path.basename(src) + ".o"))
        p = subprocess.run(["g++", *flags, "-c", src, "-o", obj], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                           text=True)
        assert p.returncode == 0, p.stdout
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(out / "host_stress")
    subprocess.run(["g++", *flags, *objs, "-o", exe, "-lrt", "-lpthread", "-ldl"], check=True)
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("kind", sorted(SANITIZERS))
def test_host_protocol_under_sanitizer(tmp_path, kind):
    exe = build(tmp_path, kind)
    env = dict(os.environ, GVM_PIECE_MB="1",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    for seed, (mode, policy, ranks, requests) in enumerate(RUNS):
        p = subprocess.run([exe, str(mode), str(policy), str(ranks), str(requests), str(seed)], env=env,
                           stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=240)
        assert p.returncode == 0, p.stdout[-6000:]
        assert "Sanitizer" not in p.stdout and "runtime error" not in p.stdout, p.stdout[-6000:]
        assert p.stdout.strip().endswith("0 failures"), p.stdout[-2000:]
