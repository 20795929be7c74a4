"""MI355X-native mixed-frame relativistic SHDOM source iteration
(Tominaga, Shibata & Blinnikov 2015).

The solver is the HIP library ``librrt.so`` behind the C ABI in
``include/rrt.h``; ``binding`` is its thin ctypes wrapper.
"""
from .workloads import MEC2_KEV  # noqa: F401
