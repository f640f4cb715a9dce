"""MI355X (gfx950) axisymmetric modal FMM: the hot path of Carley's FMM for
axisymmetric domains (arXiv 2301.01179) behind a C ABI (include/axf.h).

Importing the package loads nothing; ``axf`` holds the ctypes binding and
``inputs`` the seeded workload generators."""
