"""Differentiable light tracing for torch.

``LightTraceFn.apply(params, tracer)`` runs the primal light-tracing kernel
(Alg. 1) and returns texel irradiance E [n_layouts, K]; its backward runs the
adjoint light-tracing kernel (Alg. 2) with the incoming dL/dE as the adjoint
source and returns dL/dparams [L, 6].  ``LightTraceRGBFn`` is the colour form
(channel weights [L, 3] as a second input, E [n_layouts, 3, K]) and
``LightTraceDirFn`` the directional form (hemispherical-harmonic
coefficients of the reflected radiance, E [n_layouts, (order+1)^2, K]);
``LightTraceRVFn`` takes the orientation as a rotation vector (params
[L, 7] = x, y, z, theta, P; Sec. 4.4.2).  Whether the adjoint replays the
forward's paths (correlated evaluation, as the paper uses for validation) or
a fresh set (decorrelated, as it uses for optimisation) is the tracer's
``correlated`` flag (Sec. 4.3).  Both passes run on the current torch stream.
"""
from __future__ import annotations

import torch

from .native import Context

DECORRELATE = 0x9E3779B97F4A7C15


class LightTracer:
    """Holds a liblt context with one scene and one luminaire set, and the
    per-call configuration of the forward / adjoint passes."""

    def __init__(self, scene_arrays, lights_static, layout_offsets, paths_per_layout: int, max_hits: int,
                 seed: int = 1, correlated: bool = True, graph: bool = False, device: int = 0,
                 linear: bool = False):
        verts, tris, tri_patch, patches = scene_arrays
        self.ctx = Context(device)
        self.n_texels = self.ctx.upload_scene(verts, tris, tri_patch, patches)
        self.ctx.set_lights(lights_static, layout_offsets)
        self.paths_per_layout = int(paths_per_layout)
        self.max_hits = int(max_hits)
        self.seed = int(seed)
        self.correlated = bool(correlated)
        self.graph = bool(graph)
        self.linear = bool(linear)      # piecewise-linear texel basis (else box)
        self._S = None
        self.device = torch.device("cuda", device)
        # learned emission proposal (a LearnedProposal); it is trained on the
        # adjoint's gradient contributions and used by the adjoint pass, and by
        # the forward pass only if proposal_forward is set
        self.proposal = None
        self.alpha_plain = 0.2
        self.proposal_forward = False

    def cfg(self, seed=None, adjoint=False):
        prop = self.proposal is not None and (adjoint or self.proposal_forward)
        return self.ctx.cfg(self.seed if seed is None else seed, self.paths_per_layout, self.max_hits,
                            graph=self.graph, proposal=prop, alpha_plain=self.alpha_plain, linear=self.linear)

    def adjoint_seed(self, seed=None):
        s = self.seed if seed is None else seed
        return s if self.correlated else (s ^ DECORRELATE)

    def scratch(self):
        n = (self.ctx.n_layouts, self.n_texels)
        if self._S is None or tuple(self._S.shape) != n:
            self._S = torch.empty(n, dtype=torch.int64, device=self.device)
        return self._S

    def autotune(self, params, cache_path=None) -> float:
        """Pick the launch tuning for this scene and path count (lt_autotune);
        a matching entry of `cache_path` is reused."""
        p = params.detach().contiguous().float()
        E = torch.empty((self.ctx.n_layouts, self.n_texels), dtype=torch.float32, device=self.device)
        g = torch.randn_like(E)
        grad = torch.empty_like(p)
        return self.ctx.autotune(p, self.ctx.cfg(self.seed, self.paths_per_layout, self.max_hits), self.scratch(), E,
                                 g, grad, cache_path=cache_path)

    def __call__(self, params, seed=None):
        return LightTraceFn.apply(params, self, seed)

    def rgb(self, params, colour, seed=None):
        """Colour mode: E [n_layouts, 3, K] from luminaire parameters [L,6]
        and channel weights [L,3], differentiable in both."""
        return LightTraceRGBFn.apply(params, colour, self, seed)

    def rotvec(self, params7, seed=None):
        """Orientation as a rotation vector: E [n_layouts, K] from params
        [L,7] = (x, y, z, theta, P), differentiable in all seven."""
        return LightTraceRVFn.apply(params7, self, seed)

    def directional(self, params, order: int, samples: int, seed=None):
        """Directional texels: hemispherical-harmonic coefficients of the
        reflected radiance [n_layouts, (order+1)^2, K] (glossy BRDF per patch
        from ctx.set_glossy), differentiable in the luminaire parameters."""
        return LightTraceDirFn.apply(params, self, int(order), int(samples), seed)


class LightTraceFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params, tracer: LightTracer, seed=None):
        p = params.detach().contiguous().float()
        E, _ = tracer.ctx.trace_forward(p, tracer.cfg(seed), S=tracer.scratch())
        fctx.save_for_backward(p)
        fctx.tracer = tracer
        fctx.seed = seed
        return E

    @staticmethod
    def backward(fctx, grad_E):
        (p,) = fctx.saved_tensors
        tracer = fctx.tracer
        g = grad_E.contiguous().float()
        prop = tracer.proposal
        hist = prop.hist if prop is not None and prop.collect else None
        grad = tracer.ctx.trace_adjoint(p, g, tracer.cfg(tracer.adjoint_seed(fctx.seed), adjoint=True),
                                         bin_hist=hist)
        return grad, None, None


class LightTraceRGBFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params, colour, tracer: LightTracer, seed=None):
        p = params.detach().contiguous().float()
        c = colour.detach().contiguous().float()
        E, _ = tracer.ctx.trace_forward_rgb(p, c, tracer.cfg(seed))
        fctx.save_for_backward(p, c)
        fctx.tracer = tracer
        fctx.seed = seed
        return E

    @staticmethod
    def backward(fctx, grad_E):
        p, c = fctx.saved_tensors
        tracer = fctx.tracer
        g = grad_E.contiguous().float()
        prop = tracer.proposal
        hist = prop.hist if prop is not None and prop.collect else None
        grad, grad_c = tracer.ctx.trace_adjoint_rgb(p, c, g, tracer.cfg(tracer.adjoint_seed(fctx.seed), adjoint=True),
                                                    bin_hist=hist)
        return grad, grad_c, None, None


class LightTraceRVFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params, tracer: LightTracer, seed=None):
        p = params.detach().contiguous().float()
        E, _ = tracer.ctx.trace_forward_rv(p, tracer.cfg(seed), S=tracer.scratch())
        fctx.save_for_backward(p)
        fctx.tracer = tracer
        fctx.seed = seed
        return E

    @staticmethod
    def backward(fctx, grad_E):
        (p,) = fctx.saved_tensors
        tracer = fctx.tracer
        g = grad_E.contiguous().float()
        grad = tracer.ctx.trace_adjoint_rv(p, g, tracer.cfg(tracer.adjoint_seed(fctx.seed), adjoint=True))
        return grad, None, None


class LightTraceDirFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params, tracer: LightTracer, order, samples, seed=None):
        p = params.detach().contiguous().float()
        E, _ = tracer.ctx.trace_forward_dir(p, tracer.cfg(seed), order, samples)
        fctx.save_for_backward(p)
        fctx.tracer = tracer
        fctx.seed = seed
        fctx.order, fctx.samples = order, samples
        return E

    @staticmethod
    def backward(fctx, grad_E):
        (p,) = fctx.saved_tensors
        tracer = fctx.tracer
        g = grad_E.contiguous().float()
        prop = tracer.proposal
        hist = prop.hist if prop is not None and prop.collect else None
        grad = tracer.ctx.trace_adjoint_dir(p, g, tracer.cfg(tracer.adjoint_seed(fctx.seed), adjoint=True),
                                            fctx.order, fctx.samples, bin_hist=hist)
        return grad, None, None, None, None


def band_weights(order: int, w00: float = 0.1, device=None):
    """Per-coefficient weights alpha_l of Eq. objective for directional texels,
    [(order+1)^2]: the order-0 band (undirected light) weighted w00 against
    1 for the directional bands (the paper's glossy-coin example uses 0.1)."""
    n = (order + 1) ** 2
    w = torch.ones(n, dtype=torch.float32, device=device)
    w[0] = w00
    return w


def directional_alpha(band, alpha_k, n_layouts: int):
    """alpha_l [NC] times alpha_k [K], expanded to the directional texel
    layout [n_layouts, NC, K]: the per-element weight lt_objective takes."""
    K = alpha_k.shape[-1]
    return (band[None, :, None] * alpha_k.reshape(1, 1, K)).expand(n_layouts, band.numel(), K).contiguous()


def chromaticity(colour):
    """Channel weights projected to r + g + b = 1 (Sec. 4.4.3: optimising
    chromaticity at constant intensity); differentiating through it applies
    the projection's Jacobian to the gradient."""
    return colour / colour.sum(-1, keepdim=True)


def objective(E, E_target, texel_area, alpha=None):
    """O = 1/2 sum_k A_k alpha_k (E_k - E*_k)^2 (Eq. objective) in torch; alpha
    broadcasts against E (per texel, or alpha_k alpha_l for directional texels)."""
    w = texel_area if alpha is None else texel_area * alpha
    d = E - E_target
    return 0.5 * torch.sum(w * d * d, dtype=torch.float64)
