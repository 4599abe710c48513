"""MI355X (gfx950) CRISP query engine: hand-written HIP kernels behind a C ABI.

``engine`` holds the Python binding (device memory and streams through torch,
every computation in ``libcrisp.so``).
"""
__all__ = ["engine"]
