"""MI355X-native random batch sum-of-Gaussians (RBSOG) electrostatic force path.

The compute path is the HIP library ``librbsog.so`` (built from ``csrc/``)
behind the C ABI declared in ``include/rbsog.h``; ``rbsog`` is its thin ctypes
binding and ``workloads`` builds seeded synthetic systems.
"""
