"""MI355X-native D2Q9 lattice-Boltzmann step with velocity-interpolation-based
bounce-back walls (arXiv:1903.01111).

The compute path is the C-ABI library built from ``csrc/`` (HIP for gfx950);
``binding`` wraps it with ctypes.  ``workloads`` holds seeded synthetic inputs.
Importing this package loads nothing; ``binding`` loads the library on first use.
"""
__all__ = ["workloads", "binding"]
