"""CPU oracle for the extension + volume-potential path (test infrastructure).

This package is a plain, slow, independent FP64 / extended-precision
implementation of what the GPU path computes.  It is test infrastructure:
only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the GPU library and never
consumes its outputs.

Modules
-------
cheb       first-kind Chebyshev nodes, coefficients, evaluation (Section 4).
stencil    the universal stencil X = X_S u X_Sbar u G and the interpolation
           matrix A_{X,G} in the flat Gaussian limit (Section 3.1, 3.2).
geometry   leaf nodes, tree checks, interior masks and extension lists
           (Section 4).
extension  the cut-leaf extension and its resampling (Sections 3.2, 4.1).
volume     direct quadrature of the log-kernel volume potential over the
           leaves (Section 1, volume potential; Section 4.1).
"""
