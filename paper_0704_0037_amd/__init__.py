"""MI355X-native DDA hot path: FFT interaction-matrix product and complex-symmetric QMR /
Bi-CGSTAB, as HIP kernels for gfx950 behind a C-ABI library (include/dda.h).

Importing this package loads nothing; `paper_0704_0037_amd.dda` binds the built library.
"""
