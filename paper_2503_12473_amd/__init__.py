"""MI355X-native OECDG: HIP kernels behind a C ABI (include/oecdg.h).

Modules
-------
inputs   seeded synthetic workloads (problem descriptions, projected initial data)
_lib     ctypes binding of liboecdg.so
api      the OECDG handle on torch tensors
"""
__all__ = ["inputs"]
