"""MI355X-native tip decomposition of bipartite graphs (RECEIPT, arXiv 2010.08695).

The compute path lives in ``libtip.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/tip.h``); ``tip`` is its thin ctypes binding.
"""
__all__ = ["tip", "graphgen"]
