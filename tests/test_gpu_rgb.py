"""Colour mode on the GPU vs the CPU oracle (Sec. 4.4.3, intensity and
colour), through the C ABI: per-luminaire channel weights of the flux,
per-patch channel albedos, channel-planar texels [n_layouts, 3, K], and the
gradient w.r.t. the channel weights.  Bars as for the grey tracer: texels
rel-L2 <= 1e-4, gradients 1e-3 relative; the tests report how close they are.
"""
import sys

import numpy as np
import pytest

import lt_inputs as li
from tuning_cache import bench_tuning

pytestmark = pytest.mark.gpu

TEX_BAR, GRAD_BAR = 1e-4, 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), 1e-6 * np.abs(ref).max() + 1e-30)
    return float(np.max(np.abs(x - ref) / scale))


def run_rgb(torch, oracle_lib, scene, lights, seed, N, B, use_bvh, tuning=None):
    from paper_2310_02043_amd import Context
    rng = np.random.default_rng(seed)
    alb = rng.uniform(0.3, 0.8, (scene.n_patches, 3)).astype(np.float32)
    col = rng.dirichlet([2.0, 2.0, 2.0], lights.n_lights).astype(np.float32)
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    if tuning:
        ctx.set_tuning(**tuning)
    ctx.set_albedo_rgb(alb)
    osc = oracle_lib.OracleScene(scene, use_bvh=use_bvh, albedo_rgb=alb)
    ol = oracle_lib.OracleLights(lights, col)
    p_d = torch.tensor(lights.params, device="cuda")
    c_d = torch.tensor(col, device="cuda")
    cfg = ctx.cfg(seed, N, B)
    E_d, S_d = ctx.trace_forward_rgb(p_d, c_d, cfg)
    assert ctx.sync() == 0
    S_ref, _ = oracle_lib.forward(osc, ol, lights.params, seed, N, B)
    E_ref = oracle_lib.fixed_to_float(S_ref)
    r = rel_l2(E_d.cpu().numpy(), E_ref)
    say(f"  texels: rel-L2 {r:.2e}, bit-identical {np.mean(S_d.cpu().numpy() == S_ref) * 100:.4f} %")
    assert r <= TEX_BAR
    Et = np.stack([np.stack([li.painted_target(scene, float(np.mean(E_ref[j, ch])) * 1.5 + 1e-3, seed=3 * j + ch)
                             for ch in range(3)]) for j in range(lights.n_layouts)])
    O_ref, g_ref = oracle_lib.objective(E_ref, Et, scene.texel_area())
    O_d, g_d = ctx.objective(E_d, torch.tensor(Et, device="cuda"))
    assert abs(O_d.item() / O_ref - 1) < 1e-4
    grad_ref, grad_c_ref, _ = oracle_lib.adjoint_rgb(osc, ol, lights.params, seed, N, B, g_ref)
    grad_d, grad_c_d = ctx.trace_adjoint_rgb(p_d, c_d, torch.tensor(g_ref, device="cuda"), cfg)
    assert ctx.sync() == 0
    e1 = max_rel(grad_d.cpu().numpy(), grad_ref)
    e2 = max_rel(grad_c_d.cpu().numpy(), grad_c_ref)
    say(f"  gradient: max rel err {e1:.2e}; colour gradient {e2:.2e}")
    assert e1 <= GRAD_BAR and e2 <= GRAD_BAR
    return ctx


def test_rgb_box_room_full(torch_dev, oracle_lib):
    """Closed room with two boxes at full size (2^20 paths, 3 hits), random
    channel albedos and channel weights."""
    c1 = li.box_room()
    run_rgb(torch_dev, oracle_lib, c1["scene"], c1["lights"], c1["seed"], c1["paths"], c1["max_hits"], False)


def test_rgb_office_reduced(torch_dev, oracle_lib):
    """The 200k-triangle office at 2^18 paths, 5 hits, 16 area lights, with
    the launch tuning bench.py uses."""
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    run_rgb(torch_dev, oracle_lib, sc, lights, c2["seed"], 1 << 18, c2["max_hits"], True,
            tuning=bench_tuning(sc, lights, c2["paths"], c2["max_hits"]))


def test_rgb_batched_layouts(torch_dev, oracle_lib):
    """Room set: 64 layouts of 4..48 lights in one launch, 2^14 paths per layout."""
    c3 = li.room_set()
    run_rgb(torch_dev, oracle_lib, c3["scene"], c3["lights"], c3["seed"], 1 << 14, c3["max_hits"], True)


def test_rgb_autograd_and_chromaticity(torch_dev):
    """The colour autograd function's backward equals the direct colour
    adjoint, and through the chromaticity projection c / (r + g + b) the
    colour gradient is orthogonal to c (scaling c leaves the projection
    unchanged)."""
    torch = torch_dev
    from paper_2310_02043_amd.autograd import LightTracer, chromaticity, objective
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    tr = LightTracer((sc.verts, sc.tris, sc.tri_patch, sc.patches), lights.static, lights.layout_offsets,
                     1 << 20, 3, seed=9)
    tr.ctx.set_albedo_rgb(np.random.default_rng(1).uniform(0.3, 0.8, (sc.n_patches, 3)).astype(np.float32))
    A = torch.tensor(sc.texel_area(), device="cuda")
    Et = torch.tensor(np.stack([li.painted_target(sc, 8.0, seed=s) for s in range(3)])[None], device="cuda")
    p = torch.tensor(lights.params, device="cuda", requires_grad=True)
    c = torch.tensor([[0.9, 0.7, 0.4]], device="cuda", requires_grad=True)
    E = tr.rgb(p, chromaticity(c))
    O = objective(E, Et, A)
    O.backward()
    g = (A * (E.detach() - Et)).contiguous()
    cp = chromaticity(c.detach()).contiguous()
    ref_p, ref_c = tr.ctx.trace_adjoint_rgb(p.detach(), cp, g, tr.cfg())
    torch.cuda.synchronize()
    rel = (p.grad - ref_p).abs().max().item() / ref_p.abs().max().item()
    say("  autograd vs direct colour adjoint:", rel)
    assert rel < 1e-5
    # chain rule through the projection: J^T ref_c with J = (I - cp 1^T) / sum(c)
    jt = (ref_c - (ref_c * cp).sum(-1, keepdim=True)) / c.detach().sum(-1, keepdim=True)
    assert torch.allclose(c.grad, jt, rtol=1e-5, atol=1e-6 * jt.abs().max().item())
    assert abs(float((c.grad * c.detach()).sum())) <= 1e-5 * float(c.grad.abs().sum() * c.detach().abs().sum())


def test_rgb_invalid_arguments(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd import Context
    from paper_2310_02043_amd.native import LtError
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    ctx = Context(0)
    ctx.upload_scene(sc.verts, sc.tris, sc.tri_patch, sc.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    p_d = torch.tensor(lights.params, device="cuda")
    c_d = torch.ones((lights.n_lights, 3), device="cuda")
    with pytest.raises(LtError):
        ctx.trace_forward_rgb(p_d, c_d, ctx.cfg(1, 1 << 12, 3, linear=True))     # box basis only
    with pytest.raises(LtError):
        ctx.set_albedo_rgb(np.full((sc.n_patches, 3), 1.5, np.float32))          # albedo outside [0, 1]
