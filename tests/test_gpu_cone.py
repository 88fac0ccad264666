"""Cone-angle gradients of soft-edged spots on the GPU vs the CPU oracle
(supplement, spot light: the fall-off differentiated w.r.t. the inner and
outer cone angles with x_1 fixed, at constant power), through the C ABI.
Gradients at the gradient bar (1e-3 relative); the six ordinary gradient
components must equal the plain adjoint's exactly (same per-path terms, same
summation order)."""
import sys

import numpy as np
import pytest

import lt_inputs as li
from lt_inputs.scenes import make_lights, POINT, SPOT, RECT, SOFT

pytestmark = pytest.mark.gpu

GRAD_BAR = 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def max_rel(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), 1e-6 * np.abs(ref).max() + 1e-30)
    return float(np.max(np.abs(x - ref) / scale))


def run_cone(torch, oracle_lib, scene, lights, seed, N, B, use_bvh):
    from paper_2310_02043_amd import Context
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    osc, ol = oracle_lib.OracleScene(scene, use_bvh=use_bvh), oracle_lib.OracleLights(lights)
    p_d = torch.tensor(lights.params, device="cuda")
    cfg = ctx.cfg(seed, N, B)
    S_ref, _ = oracle_lib.forward(osc, ol, lights.params, seed, N, B)
    E_ref = oracle_lib.fixed_to_float(S_ref)
    Et = np.stack([li.painted_target(scene, float(np.mean(E_ref[j])) * 1.5 + 1e-3, seed=j)
                   for j in range(lights.n_layouts)])
    _, g = oracle_lib.objective(E_ref, Et, scene.texel_area())
    g_d = torch.tensor(g, device="cuda")
    grad_d, gc_d = ctx.trace_adjoint_cone(p_d, g_d, cfg)
    plain = ctx.trace_adjoint(p_d, g_d, cfg)
    assert ctx.sync() == 0
    grad_ref, gc_ref, _ = oracle_lib.adjoint_cone(osc, ol, lights.params, seed, N, B, g)
    # the same per-path contributions to the six parameters; the plain adjoint
    # sums them per tile in FP64 in a second pass, this kernel per lane in FP32
    # first
    e0 = max_rel(grad_d.cpu().numpy(), plain.cpu().numpy())
    say(f"  position, tilt and power vs the plain adjoint: max rel diff {e0:.2e}")
    assert e0 <= 1e-5
    soft = lights.static["type"] == SOFT
    assert np.all(gc_d.cpu().numpy()[~soft] == 0.0)
    e1 = max_rel(grad_d.cpu().numpy(), grad_ref)
    e2 = max_rel(gc_d.cpu().numpy()[soft], gc_ref[soft])
    say(f"  gradient: max rel err {e1:.2e}; cone-angle gradient {e2:.2e} "
        f"({gc_d.cpu().numpy()[soft].ravel()[:4]})")
    assert e1 <= GRAD_BAR and e2 <= GRAD_BAR


def test_cone_box_room_mixed_lights(torch_dev, oracle_lib):
    """Closed room with two boxes at full size (2^20 paths, 3 hits): two
    soft-edged spots (one with no inner cone) beside a spot, a point light
    and a rectangle."""
    sc = li.box_room()["scene"]
    lights = make_lights([SOFT, SPOT, SOFT, POINT, RECT], [0.0, 3.0, 0.0, 0.0, 1.0],
                         [(0.3, 0.8), (0, 0), (0.0, 0.6), (0, 0), (0.5, 0.3)], [0, 0, 0, 0, 0],
                         [[2.8, 0.9, 2.3, 0.25, -0.1, 40.0], [1.0, 1.0, 2.0, 0.1, 0.2, 50.0],
                          [1.5, 2.2, 2.2, -0.2, 0.15, 30.0], [3.0, 2.0, 1.8, 0, 0, 30.0],
                          [2.0, 1.5, 2.4, -0.2, 0.3, 70.0]])
    run_cone(torch_dev, oracle_lib, sc, lights, 0xC1, 1 << 20, 3, False)


def test_cone_batched_layouts(torch_dev, oracle_lib):
    """Two layouts in one launch over the office's BVH at 2^18 paths per
    layout, 5 hits: soft-edged spots of different cones and a rectangle."""
    c2 = li.office()
    sc = c2["scene"]
    lights = make_lights([SOFT, RECT, SOFT, SOFT], [0.0, 2.0, 0.0, 0.0],
                         [(0.4, 0.9), (0.6, 0.6), (0.2, 0.5), (0.0, 1.1)], [0, 0, 1, 1],
                         [[5.0, 4.0, 2.7, 0.1, 0.05, 60.0], [12.0, 8.0, 2.85, 0.0, 0.0, 40.0],
                          [20.0, 10.0, 2.6, -0.1, 0.2, 50.0], [8.0, 15.0, 2.7, 0.05, -0.05, 35.0]])
    run_cone(torch_dev, oracle_lib, sc, lights, 0xC2, 1 << 18, c2["max_hits"], True)


def test_cone_invalid_arguments(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd import Context
    from paper_2310_02043_amd.native import LtError
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    ctx = Context(0)
    ctx.upload_scene(sc.verts, sc.tris, sc.tri_patch, sc.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    p_d = torch.tensor(lights.params, device="cuda")
    g = torch.zeros((lights.n_layouts, sc.n_texels), device="cuda")
    with pytest.raises(LtError):
        ctx.trace_adjoint_cone(p_d, g, ctx.cfg(1, 1 << 12, 3, linear=True))      # box basis only
