"""MI355X-native Jacobi-preconditioned conjugate gradients for CSR FEM systems.

The HIP library (libjpcg.so, built from csrc/ for gfx950) does all the work;
this package binds its C-ABI (include/jpcg.h) with ctypes and uses torch only
for device tensors and streams.
"""
from . import capi  # noqa: F401
from .solver import Batch, DeviceCSR, Solver, q1_apply, q1_assemble  # noqa: F401
