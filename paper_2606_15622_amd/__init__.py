"""MI355X-native cubic Fokker-Planck particle step.

The GPU library (``libfpgpu.so``, built from ``csrc/``) holds every step of the path;
``fpgpu`` is its ctypes binding (argument marshalling only) and ``inputs`` the seeded
synthetic workloads.  Importing this package loads nothing; ``fpgpu.load()`` loads the
library and raises if it is missing.
"""
