"""Proposal-network oracle (numpy) -- TEST INFRASTRUCTURE.

The emission proposal is an extension beyond the paper (which leaves
importance sampling to future work, Sec. 7): a small MLP from a light's
normalised parameters and learned embedding to probabilities over the 32 x 32
cells of the hemi-octahedral map of its emission hemisphere.  This module
writes the network out plainly in float64:

* inference mirrors the kernel's rounding points (weights, inputs and hidden
  activations rounded to bfloat16, accumulation in higher precision);
* a training step is cross-entropy to a target distribution, backpropagated
  by hand, followed by Adam (beta1 0.9, beta2 0.999, eps 1e-8);
* the training target from an adjoint histogram of the scaled gradient's
  second moment per cell: the variance-optimal cell probabilities are
  proportional to the square root of that moment, averaged over passes and
  mixed with the plain cos^n lobe's cell masses (a midpoint quadrature of
  the lobe over each cell of the hemi-octahedral map).
"""
from __future__ import annotations

import numpy as np

IN, HID, BINS, NPAR, NEMB = 32, 64, 1024, 6, 16
OFF_W1 = 0
OFF_B1 = OFF_W1 + HID * IN
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + BINS * HID
N_WEIGHTS = OFF_B3 + BINS


def unpack(w):
    w = np.asarray(w, np.float64)
    return (w[OFF_W1:OFF_B1].reshape(HID, IN), w[OFF_B1:OFF_W2], w[OFF_W2:OFF_B2].reshape(HID, HID),
            w[OFF_B2:OFF_W3], w[OFF_W3:OFF_B3].reshape(BINS, HID), w[OFF_B3:N_WEIGHTS])


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16_bits(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def infer(w, x):
    """Logits and cell probabilities with bfloat16 weights / activations."""
    wb = bf16_round(np.asarray(w, np.float32)).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(wb)
    xb = bf16_round(np.asarray(x, np.float32)).astype(np.float64)
    h1 = bf16_round(np.maximum(xb @ W1.T + b1, 0.0).astype(np.float32)).astype(np.float64)
    h2 = bf16_round(np.maximum(h1 @ W2.T + b2, 0.0).astype(np.float32)).astype(np.float64)
    z = h2 @ W3.T + b3
    e = np.exp(z - z.max(1, keepdims=True))
    p = e / e.sum(1, keepdims=True)
    return z, p


def _bf16_choices(v, a, mag, tol):
    """The bfloat16 values a hidden unit may round to.  v is the float64
    activation after ReLU, a the pre-activation, mag the sum of the absolute
    terms of its dot product: FP32 accumulation in any order stays within
    tol * mag of the exact sum, so when a rounding tie (or, through ReLU, zero)
    lies that close both neighbouring values are admissible."""
    def rnd(t):
        return float(bf16_round(np.float32(t))[0])
    out = {rnd(v)}
    if abs(a) <= tol * mag:
        out |= {0.0, rnd(max(a + tol * mag, 0.0))}
    if v > 0.0:
        for d in (-tol * mag, tol * mag):
            out.add(rnd(max(v + d, 0.0)))
    return sorted(out)


def infer_alternatives(w, x, tol=2.0 ** -18, max_alternatives=1024):
    """Per light, the logits and cell probabilities for every admissible
    bfloat16 rounding of its hidden activations (see _bf16_choices); tol
    2^-18 bounds FP32 accumulation over the 64 terms of a hidden unit.  A
    light with more than max_alternatives combinations gets None."""
    wb = bf16_round(np.asarray(w, np.float32)).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(wb)
    xb = bf16_round(np.asarray(x, np.float32)).astype(np.float64)
    rows = []
    for r in range(xb.shape[0]):
        def layer(hin, W, b):
            a = W @ hin + b
            mag = np.abs(W) @ np.abs(hin) + np.abs(b)
            return [_bf16_choices(max(a[i], 0.0), a[i], mag[i], tol) for i in range(a.size)]

        def expand(choices, limit):
            combos = [[]]
            for c in choices:
                combos = [cc + [v] for cc in combos for v in c]
                if len(combos) > limit:
                    return None
            return [np.asarray(cc) for cc in combos]

        h1s = expand(layer(xb[r], W1, b1), max_alternatives)
        outs = []
        for h1 in (h1s or []):
            h2s = expand(layer(h1, W2, b2), max_alternatives)
            if h2s is None or len(outs) + len(h2s) > max_alternatives:
                outs = None
                break
            for h2 in h2s:
                z = W3 @ h2 + b3
                e = np.exp(z - z.max())
                outs.append((z, e / e.sum()))
        rows.append(outs if h1s is not None and outs else None)
    return rows


def loss_and_grad(w, x, target):
    """Mean cross-entropy over lights and its gradient w.r.t. the weights and
    the embedding columns of x (full precision)."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    x = np.asarray(x, np.float64)
    t = np.asarray(target, np.float64)
    L = x.shape[0]
    a1 = x @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    lse = z.max(1, keepdims=True) + np.log(np.exp(z - z.max(1, keepdims=True)).sum(1, keepdims=True))
    loss = float(-(t * (z - lse)).sum() / L)
    dz = (np.exp(z - lse) - t) / L
    gW3 = dz.T @ h2
    gb3 = dz.sum(0)
    dh2 = (dz @ W3) * (a2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ W2) * (a1 > 0)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(0)
    gx = dh1 @ W1
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    gx_emb = np.zeros_like(x)
    gx_emb[:, NPAR:NPAR + NEMB] = gx[:, NPAR:NPAR + NEMB]
    return loss, g, gx_emb


def adam(w, m, v, g, step, lr):
    m = 0.9 * m + 0.1 * g
    v = 0.999 * v + 0.001 * g * g
    c1 = 1.0 - 0.9 ** step
    c2 = 1.0 - 0.999 ** step
    return w - lr * (m / c1) / (np.sqrt(v / c2) + 1e-8), m, v


def cdf_table(pdf):
    """Inclusive prefix sums (float64, then float32) with the last entry exactly 1."""
    c = np.cumsum(np.asarray(pdf, np.float64), axis=1)
    c = c / c[:, -1:]
    out = c.astype(np.float32)
    out[:, -1] = 1.0
    return out


def plain_cell_mass(lobe_n, sub: int = 8):
    """Probability of each 32 x 32 hemi-octahedral cell (index v * 32 + u)
    under the plain lobe (n + 1)/(2 pi) cos^n(theta) d(omega), with
    d(omega) = du dv / (2 |p|^3) for p = ((u+v)/2, (u-v)/2, 1-|.|-|.|):
    midpoint rule on sub x sub points per cell, each light's row normalised."""
    out = []
    h = 1.0 / (16.0 * sub)
    c = -1.0 + (np.arange(32 * sub) + 0.5) * h
    v, u = np.meshgrid(c, c, indexing="ij")
    x, y = (u + v) / 2.0, (u - v) / 2.0
    z = 1.0 - np.abs(x) - np.abs(y)
    r = np.sqrt(x * x + y * y + z * z)
    dw = h * h / (2.0 * r ** 3)
    for n in np.atleast_1d(np.asarray(lobe_n, np.float64)):
        dens = (n + 1.0) / (2.0 * np.pi) * (z / r) ** n * dw
        m = dens.reshape(32, sub, 32, sub).sum(axis=(1, 3)).reshape(1024)
        out.append(m / m.sum())
    return np.asarray(out)


def training_target(hist, h_avg, decay, plain_mass=None, floor=0.0):
    """Target cell probabilities from one adjoint histogram hist [L,1024]
    (per cell, an estimate of the second moment of the scaled gradient
    integrand).  Each row is normalised (an empty row counts as uniform) and
    folded into the running average h_avg with weight `decay` on the old
    average (h_avg None: the first pass); the target is the normalised square
    root of the average, mixed with the plain lobe's masses by `floor`.
    Returns (target, new h_avg), float64."""
    h = np.asarray(hist, np.float64)
    tot = h.sum(axis=1, keepdims=True)
    hn = np.where(tot > 0, h / np.where(tot > 0, tot, 1.0), 1.0 / h.shape[1])
    a = hn if h_avg is None else decay * np.asarray(h_avg, np.float64) + (1.0 - decay) * hn
    r = np.sqrt(a)
    t = r / r.sum(axis=1, keepdims=True)
    if plain_mass is not None and floor > 0:
        t = (1.0 - floor) * t + floor * np.asarray(plain_mass, np.float64)
    return t, a
