"""Graph-form ADMM (POGS method) on MI355X: hand-written HIP kernels behind a C ABI.

``paper_1503_08366_amd.pogs`` is the ctypes binding to ``libpogs.so`` (built
by ``paper_1503_08366_amd.build``); ``paper_1503_08366_amd.workloads`` holds
seeded synthetic problem generators.  Importing the package loads nothing
native; the binding loads the library on first use and raises if it is
missing.
"""
__all__ = ["pogs", "workloads", "build"]
