"""MI355X-native implicit CP-ALS time step (Boelens, Venturi & Tartakovsky, Section 3.1).

The arithmetic lives in the HIP library ``libcpals.so`` (``csrc/``); ``binding`` is a thin
ctypes layer over its C ABI, ``workloads`` holds the seeded synthetic inputs.
"""
__all__ = ["workloads", "binding"]
