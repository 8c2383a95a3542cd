"""MI355X (gfx950) staggered FFT solver for non-local ductile damage on
periodic voxel RVEs (Magri, Lucarini, Lemoine, Adam, Segurado, CMAME).

The compute runs in the HIP library libfftg.so (C ABI in include/fftg.h);
this module only marshals arguments: torch tensors own the device memory and
the stream, and their pointers are handed to the library.  There is no CPU
fallback: importing `Solver` without a built library raises.

  binding       Solver: one handle per grid (solves, staggered increments,
                adjoints, the adaptive driver, profiling entry points)
  autograd      torch.autograd wrappers: the one-pass chain, a converged
                increment, a whole load path (path_gradient, staggered_path)
  driver        LoadDriver: variable increments, checkpoint / resume, and the
                gradient of the path a run took (keep_states)
  batch         RVEBatch: many RVEs of uneven sizes advanced together
  run           one JSON configuration -> a JSON-lines log per increment
  microstructure seeded synthetic RVEs, material tables and load paths
  profiling     rocprofv3 summaries (kernel statistics, HBM counters, rates)
"""
from .binding import (FFTGError, Solver, phase_table, FP64, FP32_REFINED, ROTATED, SPECTRAL,  # noqa: F401
                      lib_path, load_library)
from . import microstructure  # noqa: F401
from .driver import LoadDriver  # noqa: F401
