"""Learned emission proposal driver (an extension beyond the paper).

The proposal network, its Adam state, the running averages and the
training target all live in the liblt context (lt_proposal_set); this
module draws the initial weights, hands them over, and passes pointers for
the three calls of an optimisation step: refresh (normalise the luminaire
parameters and run the BF16 MFMA inference into the sampler's cell tables),
update_scale (the histogram's per-component units from the last gradient)
and train (from the histogram of gradient contributions by emission cell
that the tracer's adjoint pass fills, lt_trace_adjoint with d_bin_hist: the
target is the square root of each cell's share of the histogrammed second
moment, the variance-optimal cell probabilities, mixed with the plain lobe).
The sampler mixes the learned cells with the plain lobe (probability
alpha_plain) under one-sample MIS, so gradients stay unbiased; point lights
and soft-edged spots keep the plain sampler.
"""
from __future__ import annotations

import numpy as np
import torch

from .native import MLP_BINS, MLP_IN, MLP_WEIGHTS

HID, NPAR, NEMB = 64, 6, 16
_LAYERS = [(HID, MLP_IN), (HID,), (HID, HID), (HID,), (MLP_BINS, HID), (MLP_BINS,)]


class LearnedProposal:
    def __init__(self, ctx, param_lo, param_hi, seed: int = 0, lr: float = 2e-3, alpha_plain: float = 0.2,
                 sigma_decay: float = 0.9, hist_decay: float = 0.9, plain_floor: float = 0.3):
        self.ctx = ctx
        self.L = ctx.n_lights
        self.alpha_plain = float(alpha_plain)
        self.lr = float(lr)
        dev = torch.device("cuda", ctx.device)
        # He-normal initial weights, zero biases; the output layer scaled down
        # so that the first cell distribution is close to uniform
        rng = np.random.default_rng(seed)
        parts = []
        for shp in _LAYERS:
            if len(shp) == 2:
                parts.append(rng.normal(0.0, np.sqrt(2.0 / shp[1]), shp).ravel())
            else:
                parts.append(np.zeros(shp))
        w = np.concatenate(parts).astype(np.float32)
        w[-MLP_BINS - MLP_BINS * HID:-MLP_BINS] *= 0.1
        assert w.size == MLP_WEIGHTS
        emb = rng.normal(0.0, 0.5, (self.L, NEMB)).astype(np.float32)
        ctx.proposal_set(torch.tensor(w, device=dev), torch.tensor(emb, device=dev), param_lo, param_hi,
                         hist_decay=hist_decay, plain_floor=plain_floor, sigma_decay=sigma_decay)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.hist = torch.zeros((self.L, MLP_BINS), dtype=torch.float32, device=dev)
        self.collect = True     # whether the next adjoint pass fills self.hist

    def refresh(self, params):
        """Rebuild the sampler tables for the luminaire parameters [L,6]."""
        self.ctx.proposal_refresh(params.detach().float().contiguous())

    def update_scale(self, grad, mask=None):
        """Running RMS of each light's gradient components (the histogram's
        units); components outside `mask` [6] do not enter the histogram."""
        self.ctx.proposal_update_scale(grad.detach().float().contiguous(), mask)

    def train(self, hist=None, steps: int = 4):
        """Fit the cell distribution to the adjoint histogram; returns the loss."""
        self.ctx.proposal_train_step(self.hist if hist is None else hist, self.lr, steps, loss=self.loss)
        return float(self.loss.item())
