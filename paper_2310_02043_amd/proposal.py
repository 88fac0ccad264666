"""Learned emission proposal driver (an extension beyond the paper).

Holds the proposal network's FP32 master weights, their BF16 copy, Adam
moments and the per-light embeddings on the device, and drives the two
kernels of liblt: inference (BF16 MFMA) into the sampler's cell tables, and a
training step toward a target derived from the histogram of gradient
contributions by emission cell that the tracer's adjoint pass fills
(lt_trace_adjoint with d_bin_hist): the square root of each cell's share of
the histogrammed second moment (the variance-optimal cell probabilities).  The
sampler mixes the learned cells with the plain lobe (probability
alpha_plain) under one-sample MIS, so gradients stay unbiased; point lights
keep the plain sampler.
"""
from __future__ import annotations

import numpy as np
import torch

from .native import MLP_BINS, MLP_IN, MLP_WEIGHTS

HID, NPAR, NEMB = 64, 6, 16
_LAYERS = [(HID, MLP_IN), (HID,), (HID, HID), (HID,), (MLP_BINS, HID), (MLP_BINS,)]


def _bf16_bits(a: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest even."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def plain_cell_mass(lobe_n, sub: int = 8) -> np.ndarray:
    """Probability of each of the 32 x 32 hemi-octahedral cells under the plain
    cos^n lobe, (n + 1)/(2 pi) cos^n(theta) d(omega) with d(omega) =
    du dv / (2 |p|^3), by midpoint quadrature on sub x sub points per cell.
    Returns [L, 1024] (rows sum to 1)."""
    n = np.asarray(lobe_n, np.float64).reshape(-1, 1)
    k = (np.arange(32 * sub) + 0.5) / (16.0 * sub) - 1.0
    uu, vv = np.meshgrid(k, k, indexing="xy")          # [v, u]
    x, y = (uu + vv) / 2, (uu - vv) / 2
    z = 1.0 - np.abs(x) - np.abs(y)
    r = np.sqrt(x * x + y * y + z * z)
    cz = z / r
    dw = (1.0 / (16.0 * sub)) ** 2 / (2.0 * r ** 3)
    dens = (n[:, :, None] + 1.0) / (2 * np.pi) * cz[None] ** n[:, :, None] * dw[None]
    m = dens.reshape(-1, 32, sub, 32, sub).sum((2, 4)).reshape(-1, 1024)
    return m / m.sum(1, keepdims=True)


def training_target(hist, h_avg, decay: float, plain_mass=None, floor: float = 0.0, prior: float = 0.0):
    """Training target of the proposal network from one adjoint histogram.

    hist [L,1024] estimates, per cell, the second moment A_b of the scaled
    gradient integrand; the variance-optimal cell probabilities are
    proportional to sqrt(A_b).  Each light's histogram is normalised (a light
    with an empty histogram gets uniform cells) and folded into the running
    average h_avg (weight `decay` on the old average); with `prior` > 0 the
    average is shrunk toward the plain lobe's second moments (plain cell
    masses squared) before the square root; the result is mixed with the
    plain lobe's cell masses by `floor`.  Returns (target, new h_avg)."""
    h = hist.double()
    tot = h.sum(1, keepdim=True)
    hn = torch.where(tot > 0, h / tot.clamp_min(1e-300), torch.full_like(h, 1.0 / h.shape[1]))
    h_avg = hn if h_avg is None else decay * h_avg + (1 - decay) * hn
    a = h_avg
    if prior > 0 and plain_mass is not None:
        pm2 = plain_mass ** 2
        a = (1.0 - prior) * a + prior * pm2 / pm2.sum(1, keepdim=True)
    r = torch.sqrt(a)
    target = r / r.sum(1, keepdim=True)
    if plain_mass is not None and floor > 0:
        target = (1.0 - floor) * target + floor * plain_mass
    return target, h_avg


class LearnedProposal:
    def __init__(self, ctx, param_lo, param_hi, seed: int = 0, lr: float = 2e-3, alpha_plain: float = 0.2,
                 sigma_decay: float = 0.9, hist_decay: float = 0.9, lobe_n=None, plain_floor: float = 0.3,
                 prior: float = 0.0):
        self.ctx = ctx
        self.L = ctx.n_lights
        self.alpha_plain = float(alpha_plain)
        self.lr = float(lr)
        self.step = 0
        self.sigma_decay = sigma_decay
        self.hist_decay = hist_decay
        self.h_avg = None
        # share of the plain lobe's cell masses in the training target: the
        # learned cells then never fall far below the plain lobe, which bounds
        # the MIS weight of every sample
        self.plain_floor = float(plain_floor)
        self.prior = float(prior)
        self.plain_mass = None
        if lobe_n is not None and (plain_floor > 0 or prior > 0):
            self.plain_mass = torch.tensor(plain_cell_mass(lobe_n), dtype=torch.float64,
                                           device=torch.device("cuda", ctx.device))
        dev = torch.device("cuda", ctx.device)
        rng = np.random.default_rng(seed)
        parts = []
        for shp in _LAYERS:
            if len(shp) == 2:
                parts.append(rng.normal(0.0, np.sqrt(2.0 / shp[1]), shp).ravel())
            else:
                parts.append(np.zeros(shp))
        w = np.concatenate(parts).astype(np.float32)
        w[-MLP_BINS - MLP_BINS * HID:-MLP_BINS] *= 0.1   # start close to uniform cells
        assert w.size == MLP_WEIGHTS
        self.w = torch.tensor(w, device=dev)
        self.mw = torch.zeros_like(self.w)
        self.vw = torch.zeros_like(self.w)
        self.wb = torch.tensor(_bf16_bits(w).view(np.int16), device=dev)
        x = np.zeros((self.L, MLP_IN), np.float32)
        x[:, NPAR:NPAR + NEMB] = rng.normal(0.0, 0.5, (self.L, NEMB))
        self.x = torch.tensor(x, device=dev)
        self.mx = torch.zeros_like(self.x)
        self.vx = torch.zeros_like(self.x)
        self.lo = torch.tensor(np.asarray(param_lo, np.float32), device=dev)
        self.hi = torch.tensor(np.asarray(param_hi, np.float32), device=dev)
        self.sig2 = None
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.hist = torch.zeros((self.L, MLP_BINS), dtype=torch.float32, device=dev)
        self.collect = True     # whether the next adjoint pass fills self.hist

    def refresh(self, params):
        """Normalise the luminaire parameters into x and rebuild the sampler tables."""
        with torch.no_grad():
            self.x[:, :NPAR] = 2.0 * (params.detach() - self.lo) / (self.hi - self.lo) - 1.0
        self.ctx.mlp_infer(self.wb, self.x)

    def update_scale(self, grad, mask=None):
        """Running RMS of each light's gradient components (the histogram's
        units); components outside `mask` [6] do not enter the histogram."""
        g2 = grad.detach().float() ** 2
        self.sig2 = g2 if self.sig2 is None else self.sigma_decay * self.sig2 + (1 - self.sigma_decay) * g2
        inv = 1.0 / torch.sqrt(self.sig2 + 1e-30)
        inv = torch.where(torch.isfinite(inv), inv, torch.zeros_like(inv))
        if mask is not None:
            inv = inv * torch.as_tensor(mask, dtype=inv.dtype, device=inv.device)
        inv = inv.contiguous()
        self.ctx.proposal_set_scale(inv)

    def train(self, hist=None, steps: int = 4):
        """Fit the cell distribution to the adjoint histogram (training_target)."""
        h = (self.hist if hist is None else hist).double()
        target, self.h_avg = training_target(h, self.h_avg, self.hist_decay, self.plain_mass, self.plain_floor,
                                             self.prior)
        target = target.float().contiguous()
        for _ in range(steps):
            self.step += 1
            self.ctx.mlp_train(self.w, self.mw, self.vw, self.wb, self.x, self.mx, self.vx, target, self.step,
                               self.lr, loss=self.loss)
        return float(self.loss.item())
