"""Lighting optimisation loop (Sec. 6: a gradient-based optimiser updates the
luminaire parameters while the primal and adjoint passes run on the GPU; the
paper uses ADAM with beta1 = 0.9, beta2 = 0.999).

The parameters are optimised in scaled units, p = p0 + q * scale, so one Adam
step moves every free coordinate by about lr * scale (metres, radians,
watts).  With power="quadratic" the power is P = w^2 / 2 and w is the
optimised coordinate (Sec. 4.4.3 parametrises intensity this way so that it
cannot turn negative); its scale is then the step in P at the initial
power.  Coordinates outside `mask` stay fixed (ceiling luminaires keep their
mounting height), and every step is projected back into [lo, hi].  Each
iteration traces a fresh seed; the adjoint pass uses a decorrelated seed
(Sec. 4.3).  With a LearnedProposal attached to the tracer, the adjoint pass
samples emission from it; every `train_every` steps the adjoint pass also
histograms its contributions by emission direction and the proposal network
takes a few training steps on them.

    python -m paper_2310_02043_amd.optimize --workload office --steps 100 [--proposal]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from .autograd import LightTracer, objective


def optimize(tracer: LightTracer, params0, target, texel_area, steps: int, lr: float = 0.1, scale=None,
             mask=None, lo=None, hi=None, alpha=None, seed: int = 1, train_every: int = 1,
             proposal_train_steps: int = 4, proposal_warmup: int = 30, warmup_paths: int = 1 << 24,
             callback=None, power: str = "linear"):
    """Minimise O(E(p)) = 1/2 sum_k A_k alpha_k (E_k - E*_k)^2 over the luminaire
    parameters [L,6].  Returns (params, history); history holds each
    iteration's objective (from its own forward pass) and wall time.

    With a proposal, `proposal_warmup` adjoint passes of `warmup_paths` paths
    at the initial parameters train it before the first step (their time is
    part of the first iteration's)."""
    dev = tracer.device
    p0 = params0.detach().to(dev).float()
    ones = torch.ones(6, device=dev)
    sc = ones if scale is None else torch.as_tensor(scale, dtype=torch.float32, device=dev)
    mk = ones if mask is None else torch.as_tensor(mask, dtype=torch.float32, device=dev)
    lo_t = None if lo is None else torch.as_tensor(lo, dtype=torch.float32, device=dev)
    hi_t = None if hi is None else torch.as_tensor(hi, dtype=torch.float32, device=dev)
    if power not in ("linear", "quadratic"):
        raise ValueError("power must be 'linear' or 'quadratic'")
    quad = power == "quadratic"
    w0 = torch.sqrt(2.0 * p0[:, 5]) if quad else None
    sw = (sc[5] / w0.clamp_min(1e-6)) if quad else None      # w step per unit of q, per light

    def params_of(qq):
        p = p0 + qq * sc
        if quad:
            w = w0 + qq[:, 5] * sw
            p = torch.cat([p[:, :5], (0.5 * w * w)[:, None]], 1)
        return p

    def project(qq):
        p = torch.maximum(torch.minimum(p0 + qq * sc, hi_t), lo_t)
        out = (p - p0) / sc
        if quad:
            w = (w0 + qq[:, 5] * sw).clamp(torch.sqrt(2.0 * lo_t[5].clamp_min(0.0)), torch.sqrt(2.0 * hi_t[5]))
            out[:, 5] = (w - w0) / sw
        return out

    q = torch.zeros_like(p0, requires_grad=True)
    opt = torch.optim.Adam([q], lr=lr, betas=(0.9, 0.999))
    prop = tracer.proposal
    hist = []
    correlated = tracer.correlated
    tracer.correlated = False
    t_warm = time.perf_counter()
    if prop is not None and proposal_warmup > 0:
        with torch.no_grad():
            E = tracer(p0.contiguous(), seed ^ 0x5A5A)
            w = texel_area if alpha is None else texel_area * alpha
            g = (w * (E - target)).contiguous()
        for k in range(proposal_warmup):
            prop.refresh(p0)
            cfg = tracer.ctx.cfg(seed + 104729 * (k + 1), warmup_paths, tracer.max_hits, proposal=True,
                                 alpha_plain=tracer.alpha_plain)
            gr = tracer.ctx.trace_adjoint(p0.contiguous(), g, cfg, bin_hist=prop.hist)
            prop.update_scale(gr, mask=mk)
            prop.train(steps=proposal_train_steps)
    for it in range(steps):
        t0 = t_warm if it == 0 else time.perf_counter()
        tracer.seed = seed + 7919 * it
        p = params_of(q).contiguous()
        p.retain_grad()
        if prop is not None:
            prop.refresh(p)
            prop.collect = (it % train_every) == 0
        E = tracer(p)
        O = objective(E, target, texel_area, alpha)
        opt.zero_grad()
        O.backward()
        with torch.no_grad():
            grad_p = p.grad.detach().clone()
            q.grad.mul_(mk)
        opt.step()
        with torch.no_grad():
            if lo_t is not None:
                q.copy_(project(q))
        if prop is not None and prop.collect:
            prop.update_scale(grad_p, mask=mk)
            prop.train(steps=proposal_train_steps)
        Ov = float(O.item())
        if dev.type == "cuda":
            torch.cuda.synchronize(dev)
        rec = {"iter": it, "objective": Ov, "seconds": time.perf_counter() - t0,
               "grad_rms": grad_p.pow(2).mean(0).sqrt().tolist()}
        hist.append(rec)
        if callback is not None:
            callback(rec)
    if prop is not None:
        prop.collect = True
    tracer.correlated = correlated
    with torch.no_grad():
        return params_of(q.detach()), hist


def evaluate(tracer: LightTracer, params, target, texel_area, paths: int, seed: int = 0xE7A1):
    """Objective of `params` from one forward pass of `paths` paths."""
    n = tracer.paths_per_layout
    tracer.paths_per_layout = paths
    try:
        with torch.no_grad():
            E = tracer(params.contiguous(), seed)
            return float(objective(E, target, texel_area).item())
    finally:
        tracer.paths_per_layout = n


WORKLOADS = {
    # name: (generator, Adam steps, lr, per-parameter scale, free mask)
    "office": ("office", 100, 0.1, [1.0, 1.0, 1.0, 0.5, 0.5, 10.0], [1, 1, 0, 1, 1, 1]),
    "building": ("building_floor", 200, 0.1, [1.0, 1.0, 1.0, 0.5, 0.5, 10.0], [1, 1, 0, 1, 1, 1]),
}


def main(argv=None):
    import lt_inputs as li
    from .proposal import LearnedProposal
    ap = argparse.ArgumentParser(description="Adam lighting optimisation through the adjoint light tracer")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="office")
    ap.add_argument("--steps", type=int, default=0)
    ap.add_argument("--paths", type=int, default=0)
    ap.add_argument("--proposal", action="store_true", help="learned emission proposal in the adjoint pass")
    ap.add_argument("--alpha-plain", type=float, default=0.2)
    ap.add_argument("--eval-paths", type=int, default=1 << 28)
    ap.add_argument("--target-paths", type=int, default=1 << 28)
    ap.add_argument("--json", type=str, default="")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--power", choices=["linear", "quadratic"], default="linear",
                    help="optimise P directly or w with P = w^2 / 2")
    a = ap.parse_args(argv)
    gen, steps, lr, scale, mask = WORKLOADS[a.workload]
    steps = a.steps or steps
    wl = getattr(li, gen)()
    sc, lights = wl["scene"], wl["lights"]
    N = a.paths or wl["paths"]
    tracer = LightTracer((sc.verts, sc.tris, sc.tri_patch, sc.patches), lights.static, lights.layout_offsets,
                         N, wl["max_hits"], seed=wl["seed"], correlated=False)
    dev = tracer.device
    area = torch.tensor(sc.texel_area(), device=dev)
    pt = torch.tensor(wl["params_target"], device=dev)
    tracer.paths_per_layout = a.target_paths
    with torch.no_grad():
        target = tracer(pt, wl["seed_target"]).clone()
    tracer.paths_per_layout = N
    H = float(sc.verts[:, 2].max())
    W, D = float(sc.verts[:, 0].max()), float(sc.verts[:, 1].max())
    # tilts within +-0.15 rad keep every corner of a 0.6 m luminaire mounted
    # 0.15 m below the ceiling at least 6 cm under it: rays that graze the
    # ceiling from a luminaire at distance h have first-hit derivative terms of
    # size 1/h, so a luminaire touching the ceiling makes the gradient's
    # variance unbounded
    lo = [0.5, 0.5, 0.0, -0.15, -0.15, 1.0]
    hi = [W - 0.5, D - 0.5, H, 0.15, 0.15, 200.0]
    if a.proposal:
        tracer.proposal = LearnedProposal(tracer.ctx, lo, hi, alpha_plain=a.alpha_plain)
        tracer.alpha_plain = a.alpha_plain
    p0 = torch.tensor(lights.params, device=dev)
    if not a.no_autotune:
        tracer.autotune(p0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.cache"))
    O0 = evaluate(tracer, p0, target, area, a.eval_paths)
    print(f"{a.workload}: {sc.n_tris} triangles, {sc.n_texels} texels, {lights.n_lights} luminaires, "
          f"{N} paths x {wl['max_hits']} hits, proposal={a.proposal}; O(p0) = {O0:.6g}", flush=True)

    def cb(r):
        if r["iter"] % 10 == 0 or r["iter"] == steps - 1:
            print(f"  iter {r['iter']:4d}  O {r['objective']:.6g}  {r['seconds'] * 1000:.1f} ms", flush=True)

    t0 = time.perf_counter()
    p, hist = optimize(tracer, p0, target, area, steps, lr=lr, scale=scale, mask=mask, lo=lo, hi=hi,
                       seed=wl["seed"], callback=cb, power=a.power)
    wall = time.perf_counter() - t0
    O1 = evaluate(tracer, p, target, area, a.eval_paths)
    Opt = evaluate(tracer, pt, target, area, a.eval_paths, seed=0xE7A2)
    it_ms = np.array([r["seconds"] for r in hist[1:]]) * 1000.0
    out = {"workload": a.workload, "proposal": a.proposal, "steps": steps, "paths": N,
           "objective_initial": O0, "objective_final": O1, "objective_at_target_params": Opt,
           "ms_per_iteration_median": float(np.median(it_ms)) if it_ms.size else None,
           "wall_seconds": wall, "param_abs_error_final": (p - pt).abs().mean(0).tolist(),
           "param_abs_error_initial": (p0 - pt).abs().mean(0).tolist(),
           "objective_trace": [round(r["objective"], 6) for r in hist]}
    print(json.dumps({k: v for k, v in out.items() if k != "objective_trace"}), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(out, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
