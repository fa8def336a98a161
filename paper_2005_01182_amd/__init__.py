"""MI355X-native batched Kuhn-Munkres solver for assignment and integer optimal transport.

``otkm`` is the ctypes binding of the HIP library (loaded on first use);
``workloads`` builds the seeded synthetic inputs.
"""
__all__ = ["otkm", "workloads"]
