"""ORACLE: test infrastructure only.

A plain, slow, FP64 CPU implementation of the least-squares h-p spectral
element method of Husain's thesis (arXiv 1110.2316): the discrete functional
R^{N,W} of Ch. 4 (eq 4.1-4.8), its normal equations (Sec. 5.3), the
block-diagonal preconditioner of Sec. 5.2, PCG (Ch. 6 intro) and the relative
H^1 error (Ch. 6 intro).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It shares no code with the HIP
library in ``paper_1110_2316_amd``; both read the same mesh descriptions and
manufactured problems from ``workloads``.
"""
