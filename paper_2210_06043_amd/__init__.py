"""MI355X-native LBM-IB capillary adhesion solver (arXiv 2210.06043).

The compute path is the HIP library ``libcapib.so`` (C-ABI declared in
``include/capib.h``); ``capib`` is its thin ctypes binding and ``inputs``
builds seeded synthetic workloads.  Submodules are imported on demand so that
importing the package never loads the library by itself.
"""
__all__ = ["capib", "inputs"]
