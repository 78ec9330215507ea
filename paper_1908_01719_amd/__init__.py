"""MI355X-native finite-element Bloch-Torrey simulator (diffusion MRI signal).

The computation lives in libdmri.so (HIP kernels for gfx950 behind the C ABI
of include/dmri.h); `binding` is a thin ctypes layer over it. Importing the
package does not load the library; `Simulator(...)` does, and raises if the
library has not been built.
"""

from .binding import DmriError, Simulator, load  # noqa: F401

__all__ = ["Simulator", "DmriError", "load"]
