"""FP64 CPU oracle for stochastic multi-dimensional deconvolution.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may call it.
It shares no code with the GPU path (no kernels, tables, helpers or layouts).

Modules
  direct   -- the definition: time-domain circular convolution / correlation sums
              (Theory section, MDC integral and its matrix form; the finite-sum
              functional and its mini-batch gradient), brute-force DFT.
  freq     -- the same operator through numpy's FFT and complex128 matmuls, for
              sizes where the direct sums are too slow (validated against direct).
  optim    -- masks, the reciprocity preconditioner, SGD / Adam / Nesterov updates,
              the batch schedule and the RMSE of the Examples section.
  stepsize -- Landweber bound and largest singular value (Appendix B).

Every function works in float64 and documents the passage of the paper it
follows.  Functions without an independent pin say "parity unpinned".
"""
from . import direct, freq, optim, stepsize  # noqa: F401
