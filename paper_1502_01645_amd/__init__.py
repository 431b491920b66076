"""MI355X (gfx950) hot path of the anti-lopsided NNLS method (arXiv 1502.01645).

The compute lives in libnnls.so (HIP kernels behind the C ABI of include/nnls.h); `nnls` is its
Python binding and `workloads` the seeded synthetic inputs.  Importing the package does not
load the library; the first call into `nnls` does, and raises if it is not built.
"""
__all__ = ["nnls", "workloads"]
