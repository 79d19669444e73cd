"""MI355X-native parallel ADMM for robust quadratic resource allocation.

The solver itself is the HIP library ``libadmm.so`` (C ABI in
``include/admm.h``); ``admm`` is its thin ctypes binding and ``workloads``
draws seeded synthetic inputs.  Importing this package loads nothing.
"""
__all__ = ["admm", "workloads"]
