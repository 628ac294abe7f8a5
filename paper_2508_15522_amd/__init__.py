"""MI355X-native GridFF hot path (arXiv 2508.15522): tricubic B-spline grid
interpolation of Pauli/London/Coulomb substrate channels, fused with an
intramolecular field and FIRE/NVE steps over many replicas, in HIP for gfx950.

The C ABI is include/gridff.h; ``gridff`` is its ctypes binding."""
from . import gridff  # noqa: F401

__all__ = ["gridff"]
