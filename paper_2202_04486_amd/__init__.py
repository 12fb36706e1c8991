"""MI355X-native stochastic multi-dimensional deconvolution (HIP kernels for gfx950).

The compute path is the C-ABI library libmdd.so (include/mdd.h); this package
is its thin Python binding:

  native    ctypes declarations of the C ABI
  plan      `Plan`: sizes + workspace + stream, entry points with the ABI's names
  autograd  `MDC`: torch.autograd.Function over mdc_forward / mdc_adjoint
  solver    host-side epoch loop (batch schedule, SGD / Adam / Nesterov steps,
            step size from the largest singular value, checkpoint / resume)
"""
from .native import MddError  # noqa: F401


def __getattr__(name):
    if name == "Plan":
        from .plan import Plan
        return Plan
    raise AttributeError(name)
