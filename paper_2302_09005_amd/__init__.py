"""MI355X-native batched Finite Volume patch update (arXiv 2302.09005 hot path).

``fv`` is the Python binding of the C ABI in ``include/fv.h`` (HIP kernels for
gfx950); ``workloads`` builds seeded synthetic inputs.
"""
__all__ = ["fv", "workloads"]
