"""MI355X-native AFN-preconditioned CG for regularized Gaussian kernel systems.

The compute path is libafn.so (HIP for gfx950, C-ABI in include/afn.h);
``afn`` is its argument-marshalling binding and ``workloads`` holds the seeded
synthetic inputs.  Importing the package loads nothing; the library is loaded
on the first call.
"""
__all__ = ["afn", "workloads", "build"]
