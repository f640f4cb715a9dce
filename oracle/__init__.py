"""Plain FP64 CPU oracle for the axisymmetric modal FMM.

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library.  Parity of individual routines is pinned by tests/test_oracle_*.py.
"""
