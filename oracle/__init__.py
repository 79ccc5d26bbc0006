"""Test infrastructure: the FP64 CPU oracle for graph-form ADMM.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU library shares no code with it.
"""
