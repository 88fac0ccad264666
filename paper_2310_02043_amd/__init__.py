"""MI355X-native view-independent adjoint light tracing.

The hot path (BVH build, primal light tracing, objective, adjoint light
tracing, gradient reduction) runs in the HIP kernels of ``liblt.so`` behind
the C ABI declared in ``include/lt.h``; ``native.Context`` is its thin Python
binding and ``autograd.LightTraceFn`` exposes the primal pass as a
differentiable torch function whose backward is the adjoint kernel.
"""
from .native import Context, LtError, TraceCfg, load  # noqa: F401
