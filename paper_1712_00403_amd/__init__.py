"""MI355X-native Fast-Diagonalization (FD) preconditioner apply.

The compute path is the HIP library ``libfd.so`` (C ABI declared in
``include/fd.h``); ``paper_1712_00403_amd.fd`` is its thin ctypes binding.
Importing this package loads nothing; ``paper_1712_00403_amd.workloads``
holds the seeded synthetic workloads and carries no arithmetic of the method.
"""
__all__ = ["fd", "workloads"]
