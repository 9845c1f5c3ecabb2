"""MI355X-native particle-in-cell step for condensed-matter quantum plasmas.

The compute path is the HIP library ``libpic.so`` (hand-written gfx950 kernels
behind a C ABI declared in ``include/pic.h``); ``paper_2501_07465_amd.pic`` is the
thin ctypes binding.  Importing the package does not load the library; the
binding loads it on first use and raises if it is missing.
"""
__all__ = ["pic", "workloads"]
