"""Object-space path tracing with next-event estimation on the GPU vs the
CPU oracle (the comparison estimator of Sec. 6), through the C ABI.

Both sides draw the same samples and follow the same arithmetic, so texel
means are compared at the texel bar (rel-L2 <= 1e-4) and gradients at the
gradient bar (1e-3 relative); the tests report how close they are.
"""
import sys

import numpy as np
import pytest

import lt_inputs as li
from lt_inputs.scenes import make_lights, POINT, SPOT, RECT, SOFT

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


def make_ctx(scene, lights):
    from paper_2310_02043_amd import Context
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    return ctx


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_pt(torch, oracle_lib, scene, lights, seed, M, B, use_bvh):
    ctx = make_ctx(scene, lights)
    osc, ol = oracle_lib.OracleScene(scene, use_bvh=use_bvh), oracle_lib.OracleLights(lights)
    p_d = torch.tensor(lights.params, device="cuda")
    cfg = ctx.cfg(seed, 1 << 16, B)
    E_d, S_d = ctx.pt_forward(p_d, cfg, M)
    assert ctx.sync() == 0
    S_ref, _ = oracle_lib.path_trace(osc, ol, lights.params, seed, M, B)
    E_ref = oracle_lib.fixed_to_float(S_ref)
    r = rel_l2(E_d.cpu().numpy(), E_ref)
    say(f"  texels: rel-L2 {r:.2e}, bit-identical {np.mean(S_d.cpu().numpy() == S_ref) * 100:.4f} %")
    assert r <= TEX_BAR
    Et = np.stack([li.painted_target(scene, float(np.mean(E_ref[j])) * 1.5 + 1e-3, seed=j)
                   for j in range(lights.n_layouts)])
    _, g = oracle_lib.objective(E_ref, Et, scene.texel_area())
    _, grad_ref = oracle_lib.path_trace(osc, ol, lights.params, seed, M, B, dOdE=g)
    grad_d = ctx.pt_adjoint(p_d, torch.tensor(g, device="cuda"), cfg, M)
    assert ctx.sync() == 0
    gg = grad_d.cpu().numpy()
    scale = np.maximum(np.abs(grad_ref), 1e-6 * np.abs(grad_ref).max() + 1e-30)
    e = float(np.max(np.abs(gg - grad_ref) / scale))
    say(f"  gradient: max rel err {e:.2e}")
    assert e <= GRAD_BAR
    return ctx


def test_pt_box_room_mixed_lights(torch_dev, oracle_lib):
    """Closed room with two boxes, all four luminaire types, 8 samples per
    texel, 3 path vertices."""
    sc = li.box_room()["scene"]
    lights = make_lights([SPOT, POINT, RECT, SOFT], [3.0, 0.0, 1.0, 0.0], [(0, 0), (0, 0), (0.5, 0.3), (0.3, 0.8)],
                         [0, 0, 0, 0], [[1.0, 1.0, 2.0, 0.1, 0.2, 50.0], [3.0, 2.0, 1.8, 0, 0, 30.0],
                                        [2.0, 1.5, 2.4, -0.2, 0.3, 70.0], [2.8, 0.9, 2.3, 0.25, -0.1, 40.0]])
    run_pt(torch_dev, oracle_lib, sc, lights, 0xB0, 8, 3, use_bvh=False)


def test_pt_office_reduced(torch_dev, oracle_lib):
    """The 200k-triangle office (3.98M texels, 16 area lights), one sample per
    texel, 3 path vertices."""
    c2 = li.office()
    run_pt(torch_dev, oracle_lib, c2["scene"], c2["lights"], 0xB1, 1, 3, use_bvh=True)


def test_pt_batched_layouts(torch_dev, oracle_lib):
    """Room set: 64 layouts of 4..48 point and spot lights, one launch per
    layout, one sample per texel, 2 path vertices."""
    c3 = li.room_set()
    run_pt(torch_dev, oracle_lib, c3["scene"], c3["lights"], 0xB2, 1, 2, use_bvh=True)


def test_pt_crossing_slivers(torch_dev, oracle_lib):
    """Narrow quads crossing around the point light (every box of the tree
    contains it, so traversals toward and from it run deep into the
    traversal stack's overflow area), one sample per texel, 3 path
    vertices."""
    sc, c = li.crossing_slivers(n_dirs=4096)
    lights = make_lights([POINT], [0.0], [(0, 0)], [0], [[c[0], c[1], c[2], 0, 0, 10.0]])
    run_pt(torch_dev, oracle_lib, sc, lights, 0xB3, 1, 3, use_bvh=True)


def test_pt_invalid_arguments(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd.native import LtError
    c1 = li.box_room()
    ctx = make_ctx(c1["scene"], c1["lights"])
    p_d = torch.tensor(c1["lights"].params, device="cuda")
    with pytest.raises(LtError):
        ctx.pt_forward(p_d, ctx.cfg(1, 1 << 10, 3), 0)                    # no samples
    with pytest.raises(LtError):
        ctx.pt_forward(p_d, ctx.cfg(1, 1 << 10, 3, linear=True), 4)       # flags are not taken
    with pytest.raises(LtError):
        ctx.pt_forward(p_d, ctx.cfg(1, 1 << 10, 0), 4)                    # max_hits 0
