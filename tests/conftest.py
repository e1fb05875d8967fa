import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    # Rank processes are forked from a server started now, before any test
    # touches the GPU, so that they are GPU-free processes.
    from paper_1511_07658_amd import spmd

    spmd.prestart()


_counter = [0]


@pytest.fixture
def ns_name():
    """A fresh shared-memory namespace for one test."""
    _counter[0] += 1
    return f"gvmt.{os.getpid()}.{_counter[0]}"
