"""MI355X-native max-flow / min-cut on the Lawler expansion of hypergraphs.

The compute path lives in the HIP shared library ``libhyperflow.so``
(sources in ``csrc/``, C ABI in ``include/hyperflow.h``); ``hyperflow``
is the thin ctypes binding over it.  ``inputs`` draws seeded synthetic
workloads.  Importing the package does not load the library; the first
call into ``hyperflow`` does, and fails loudly if it was not built.
"""

__all__ = ["inputs", "hyperflow"]
