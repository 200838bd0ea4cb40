"""CPU oracle for the DDA hot path — TEST INFRASTRUCTURE, not part of the product.

Plain, slow, double-precision numpy code written from the paper (Yurkin, Maltsev &
Hoekstra, "The discrete dipole approximation for simulation of light scattering by
particles much larger than the wavelength", 2007) and from the literature it cites
for formulas it uses but does not print.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the GPU library never
does, and this package imports nothing from the GPU library.

Modules
  dda  — lattice, polarizabilities (CM, RR, LDR, CLDR; per material), Green's tensor,
         interaction matrix (dense and direct sum), incident field (plane wave, focused
         beam), QMR, Bi-CG, Bi-CGSTAB and CGNR, cross sections, far field, Mueller,
         asymmetry parameter, orientation averages (fixed and adaptive Romberg, Mueller).
  mie  — Mie theory for a homogeneous sphere (the exact reference the paper compares to).
  convnet — the learned-initial-guess network: forward, masked loss, exact gradient, and the
         features / target / guess maps between a DDA solution and the network's grid.

Parity status of each function is stated in its docstring ("pinned by ..." or
"parity unpinned").
"""
from . import convnet, dda, mie  # noqa: F401
