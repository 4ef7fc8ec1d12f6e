"""MI355X-native orbit pass of the energy-conserving relativistic GM-HC-CN potential PIC step.

The compute path is the HIP library ``libgmhc.so`` behind the C-ABI declared in
``include/gmhc.h``; :mod:`paper_2609_36383_amd.gmhc` is its thin ctypes binding.
The native library is loaded on first use and its absence is an error.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
