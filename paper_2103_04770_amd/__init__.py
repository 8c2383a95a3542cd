"""MI355X (gfx950) staggered FFT solver for non-local ductile damage on
periodic voxel RVEs (Magri, Lucarini, Lemoine, Adam, Segurado, CMAME).

The compute runs in the HIP library libfftg.so (C ABI in include/fftg.h);
this module only marshals arguments: torch tensors own the device memory and
the stream, and their pointers are handed to the library.  There is no CPU
fallback: importing `Solver` without a built library raises.
"""
from .binding import (FFTGError, Solver, phase_table, FP64, FP32_REFINED, ROTATED, SPECTRAL,  # noqa: F401
                      lib_path, load_library)
from . import microstructure  # noqa: F401
from .driver import LoadDriver  # noqa: F401
