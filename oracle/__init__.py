"""CPU FP64 oracle for mixed-precision GADI (arXiv 2512.21164).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; the only common module is ``workloads`` (seeded random inputs).

It is deliberately plain and slow: the operator is assembled as a SciPy CSR
matrix from Kronecker sums of 1-D tridiagonal matrices, and Algorithm 1 is run
step by step in NumPy, in float64 unless a lower inner precision is being
emulated.

Modules
-------
problems      PDE discretizations (Section 5.2-5.4), assembly, HSS splitting.
lowprec       round-to-nearest-even storage rounding to BF16 / FP32.
gadi_ref      Algorithm 1, the two-step form of Section 2.1, inner CG / CGNE,
              backward and forward errors (Section 3).
closed_forms  Toeplitz eigenvalues, conditioning, contraction factors and the
              dense iteration matrix T_F of Section 2.1 for tiny grids.

Parity status: every function here is pinned by tests in ``tests/`` against
closed forms, identities of the paper or dense direct solves; none is
"parity unpinned".
"""
