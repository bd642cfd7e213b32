"""Balanced k-means geometric partitioning (arXiv:1805.01208) on MI355X.

The compute path lives in ``libbkm.so`` (HIP kernels for gfx950 behind a C
ABI declared in ``include/bkm.h``); :mod:`paper_1805_01208_amd.bkm` is the
thin ctypes binding to it.  :mod:`paper_1805_01208_amd.workloads` holds the
seeded synthetic inputs.  Importing the package loads nothing.
"""
