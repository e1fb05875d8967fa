"""GPU virtualization manager (GVM) for many SPMD ranks on one MI355X.

The native library ``libgvm.so`` (built from ``csrc/``) holds the whole path:
the daemon side (one HIP context, streams, device arena, pinned staging,
kernels for gfx950) and the rank side (POSIX shared-memory request rings).
``paper_1511_07658_amd.gvm`` is a thin ctypes binding with the same names as
the C-ABI declared in ``include/gvm.h``.
"""

__all__ = ["gvm", "workloads"]
