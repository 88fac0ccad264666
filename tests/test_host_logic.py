"""Host-side logic of the package on the CPU (no GPU, no liblt calls).

* the Adam optimisation loop against a linear stand-in for the tracer: it
  recovers the parameters, never moves a masked coordinate and stays inside
  the bounds;
* the plain lobe's hemi-octahedral cell masses against an independent
  quadrature in spherical coordinates;
* the proposal network's training target: normalisation, running average,
  square root and plain-lobe floor;
* the directional objective's band weights and the chromaticity projection.
"""
import math

import numpy as np
import pytest
import torch


class LinearTracer:
    """E = M p (per layout, K texels) with autograd, standing in for the
    light tracer in the optimisation loop."""

    def __init__(self, M):
        self.M = M
        self.device = torch.device("cpu")
        self.proposal = None
        self.seed = 0
        self.correlated = True

    def __call__(self, p, seed=None):
        return (self.M @ p.reshape(-1)).reshape(1, -1)


def test_optimize_recovers_linear_model():
    from paper_2310_02043_amd.optimize import optimize
    g = torch.Generator().manual_seed(0)
    L, K = 3, 200
    M = torch.randn(K, 6 * L, generator=g, dtype=torch.float32)
    p_true = torch.tensor([[1.0, 2.0, 2.85, 0.05, -0.05, 40.0]] * L)
    p_true[:, 0] += torch.arange(L, dtype=torch.float32)
    target = (M @ p_true.reshape(-1)).reshape(1, -1)
    p0 = p_true.clone()
    p0[:, 0] += 0.4
    p0[:, 1] -= 0.3
    p0[:, 3:5] += 0.08
    p0[:, 5] *= 1.2
    area = torch.ones(K)
    lo = [0.0, 0.0, 0.0, -0.15, -0.15, 1.0]
    hi = [10.0, 10.0, 3.0, 0.15, 0.15, 200.0]
    p, hist = optimize(LinearTracer(M), p0, target, area, 400, lr=0.05, scale=[1, 1, 1, 0.5, 0.5, 10.0],
                       mask=[1, 1, 0, 1, 1, 1], lo=lo, hi=hi)
    assert hist[-1]["objective"] < 1e-4 * hist[0]["objective"]
    assert torch.all(p[:, 2] == p0[:, 2])
    free = [0, 1, 3, 4, 5]
    assert torch.allclose(p[:, free], p_true[:, free], atol=2e-2, rtol=1e-3)
    lo_t, hi_t = torch.tensor(lo), torch.tensor(hi)
    assert torch.all(p >= lo_t - 1e-6) and torch.all(p <= hi_t + 1e-6)


def test_optimize_projects_into_bounds():
    """A target outside the box: the iterate ends on the bound, not past it."""
    from paper_2310_02043_amd.optimize import optimize
    L, K = 1, 6
    M = torch.eye(6)
    target = torch.tensor([[5.0, 5.0, 2.85, 0.4, -0.4, 50.0]])
    p0 = torch.tensor([[5.0, 5.0, 2.85, 0.0, 0.0, 50.0]])
    p, _ = optimize(LinearTracer(M), p0, target, torch.ones(K), 200, lr=0.05, scale=[1, 1, 1, 0.5, 0.5, 10.0],
                    lo=[0, 0, 0, -0.15, -0.15, 1], hi=[10, 10, 3, 0.15, 0.15, 200])
    assert abs(float(p[0, 3]) - 0.15) < 1e-6 and abs(float(p[0, 4]) + 0.15) < 1e-6


def test_optimize_quadratic_power():
    """P = w^2 / 2 with w optimised (Sec. 4.4.3): recovers the parameters, the
    power stays positive when the linear form would overshoot below zero, and
    dO/dP reaches the optimiser through the chain rule (the first step's
    direction in P matches the linear form's)."""
    from paper_2310_02043_amd.optimize import optimize
    g = torch.Generator().manual_seed(1)
    L, K = 2, 120
    M = torch.randn(K, 6 * L, generator=g, dtype=torch.float32)
    p_true = torch.tensor([[1.0, 2.0, 2.85, 0.05, -0.05, 3.0], [2.5, 1.0, 2.85, -0.02, 0.04, 60.0]])
    target = (M @ p_true.reshape(-1)).reshape(1, -1)
    p0 = p_true.clone()
    p0[:, 0] += 0.3
    p0[:, 5] = torch.tensor([12.0, 45.0])
    lo = [0.0, 0.0, 0.0, -0.15, -0.15, 0.0]
    hi = [10.0, 10.0, 3.0, 0.15, 0.15, 200.0]
    kw = dict(scale=[1, 1, 1, 0.5, 0.5, 10.0], mask=[1, 1, 0, 1, 1, 1], lo=lo, hi=hi)
    p, hist = optimize(LinearTracer(M), p0, target, torch.ones(K), 600, lr=0.05, power="quadratic", **kw)
    assert hist[-1]["objective"] < 1e-4 * hist[0]["objective"]
    assert torch.allclose(p[:, [0, 1, 3, 4, 5]], p_true[:, [0, 1, 3, 4, 5]], atol=3e-2, rtol=1e-3)
    # one step each way: same sign of the change in P
    p_lin, _ = optimize(LinearTracer(M), p0, target, torch.ones(K), 1, lr=0.05, **kw)
    p_quad, _ = optimize(LinearTracer(M), p0, target, torch.ones(K), 1, lr=0.05, power="quadratic", **kw)
    assert torch.equal(torch.sign(p_lin[:, 5] - p0[:, 5]), torch.sign(p_quad[:, 5] - p0[:, 5]))
    # a huge step: linear P is clipped at the bound 0, quadratic P stays >= 0 without it
    lo0 = list(lo)
    lo0[5] = -1e9
    p_big, _ = optimize(LinearTracer(M), p0, target, torch.ones(K), 30, lr=3.0, power="quadratic",
                        scale=kw["scale"], mask=kw["mask"], lo=lo0, hi=hi)
    assert torch.all(p_big[:, 5] >= 0)


def test_band_weights_and_chromaticity():
    """Per-band objective weights: order-0 band at w00, the rest 1, expanded
    as alpha_k alpha_l over [layouts, (order+1)^2, K]; the torch objective with
    them equals the weighted sum written out.  The chromaticity projection
    sums to one and is invariant to scaling the colour."""
    from paper_2310_02043_amd.autograd import band_weights, chromaticity, directional_alpha, objective
    w = band_weights(2, 0.1)
    assert w.shape == (9,) and float(w[0]) == pytest.approx(0.1) and torch.all(w[1:] == 1.0)
    ak = torch.linspace(0.5, 2.0, 7)
    al = directional_alpha(w, ak, 2)
    assert al.shape == (2, 9, 7) and al.is_contiguous()
    assert torch.allclose(al[1, 0], 0.1 * ak) and torch.equal(al[0, 4], ak)
    g = torch.Generator().manual_seed(3)
    E, Et, A = torch.rand(2, 9, 7, generator=g), torch.rand(2, 9, 7, generator=g), torch.rand(7, generator=g)
    ref = 0.5 * sum(float(A[k] * al[j, c, k] * (E[j, c, k] - Et[j, c, k]) ** 2)
                    for j in range(2) for c in range(9) for k in range(7))
    assert float(objective(E, Et, A, alpha=al)) == pytest.approx(ref, rel=1e-6)
    c = torch.tensor([[0.9, 0.7, 0.4], [2.0, 1.0, 1.0]])
    cp = chromaticity(c)
    assert torch.allclose(cp.sum(-1), torch.ones(2)) and torch.allclose(chromaticity(3.0 * c), cp)
