"""Independent CPU FP64 checker for the staggered FFT non-local damage solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import or run anything in this package.  The
GPU library never calls it and shares no code, table or constant with it.

It is a plain, slow, vectorised numpy/scipy implementation of what the paper
computes, written to be checked against the paper by eye:

  spectral   discrete frequencies and the rotated-scheme derivative symbols
             (Sec. 3.2.1)
  mandel     Mandel vector <-> tensor helpers
  material   J2 return mapping on the effective stress with frozen damage,
             consistent tangent, linear damage laws (Sec. 2.1.2, Sec. 2.2.3,
             appendix A.2)
  gtn        Gurson-Tvergaard-Needleman matrix at frozen porosity and its
             porosity update (Sec. 2.1.1, non-local Gurson extension,
             appendix A.1)
  galerkin   FFT-Galerkin projection with mixed macroscopic control, the
             Newton + CG mechanical solver (Sec. 3.2.2)
  helmholtz  generalised Helmholtz operator in Fourier space and its
             preconditioned CG (Sec. 3.2.3, Algorithm 2)
  staggered  one load increment of the iterated staggered scheme
             (Sec. 3.2, Algorithm 1)
  driver     variable load increments with cutbacks (a reading of Sec. 4.2)
  adjoint    implicit adjoints of the converged solves, of a converged
             staggered increment and of a whole load path (gradients in the
             per-phase lengths)

Transforms use scipy.fft on the full complex spectrum (spectral.fftn /
spectral.ifftn, threaded over the process's cores) as a library primitive; Krylov solvers run in the plain real-space (mechanics) or
full-spectrum Hermitian (Helmholtz) inner product.
"""
from . import spectral, mandel, gtn, material, galerkin, helmholtz, staggered  # noqa: F401
