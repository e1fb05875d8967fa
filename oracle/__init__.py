"""CPU oracle for the GPU virtualization manager (GVM) hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the GVM path computes, written from the paper
(Li, Narayana, El-Ghazawi, "Efficient Resource Sharing Through GPU
Virtualization on Accelerated High Performance Computing Systems").
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product package never imports it and shares
no code with it; both sides see the same inputs only through the seeded
generators in ``paper_1511_07658_amd.workloads``, which hold none of the
method's arithmetic.

Modules
-------
kernels  per-rank kernels of Table 3 (VecAdd, VecMul, MM, BlackScholes),
         in float64 unless the definition fixes binary32 (vector add/multiply)
model    the execution model of Section 4: Eq. 1 to Eq. 11, the C-I / IO-I
         classification and the programming-style rule
des      a discrete-event schedule of the stream rules of Section 4.2.1,
         used as brute force against the closed forms of Section 4.2.3
serving  invariant checks of a serving event log (admission budget, each
         ticket completed once); host-logic checker, no kernel arithmetic

Pins (what ties each function to something other than itself) live in
``tests/test_oracle_*.py``; every function here is pinned, none is
"parity unpinned".
"""
