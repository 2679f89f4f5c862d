"""MI355X-native Monte Carlo line-transfer pass (hot path of the Kratos-linerad method).

The compute path is the HIP library ``libkrt.so`` behind the C ABI declared in
``include/krt.h``; :mod:`paper_2608_09340_amd.krt` is a thin ctypes binding
with the same names.  :mod:`paper_2608_09340_amd.workloads` builds the seeded
synthetic media.
"""
from . import workloads  # noqa: F401
