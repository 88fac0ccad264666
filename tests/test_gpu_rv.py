"""Rotation-vector orientation on the GPU vs the CPU oracle (Sec. 4.4.2,
Rodrigues' formula), through the C ABI: texels and dO/d(x, y, z, theta, P).
Bars as for the tilt-angle tracer: texels rel-L2 <= 1e-4, gradients 1e-3
relative; the tests report how close they are.
"""
import sys

import numpy as np
import pytest

import lt_inputs as li
from lt_inputs.scenes import make_lights, POINT, SPOT, RECT, SOFT
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


def run_rv(torch, oracle_lib, scene, lights, p7, seed, N, B, use_bvh, tuning=None):
    from paper_2310_02043_amd import Context
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    if tuning:
        ctx.set_tuning(**tuning)
    osc = oracle_lib.OracleScene(scene, use_bvh=use_bvh)
    ol = oracle_lib.OracleLights(lights, rotvec=True)
    p_d = torch.tensor(p7, device="cuda")
    cfg = ctx.cfg(seed, N, B)
    E_d, S_d = ctx.trace_forward_rv(p_d, cfg)
    assert ctx.sync() == 0
    S_ref, _ = oracle_lib.forward(osc, ol, p7, seed, N, B)
    E_ref = oracle_lib.fixed_to_float(S_ref)
    r = rel_l2(E_d.cpu().numpy(), E_ref)
    say(f"  texels: rel-L2 {r:.2e}, bit-identical {np.mean(S_d.cpu().numpy() == S_ref) * 100:.4f} %")
    assert r <= TEX_BAR
    Et = np.stack([li.painted_target(scene, float(np.mean(E_ref[j])) * 1.5 + 1e-3, seed=j)
                   for j in range(lights.n_layouts)])
    _, g_ref = oracle_lib.objective(E_ref, Et, scene.texel_area())
    grad_ref, _ = oracle_lib.adjoint_rv(osc, ol, p7, seed, N, B, g_ref)
    grad_d = ctx.trace_adjoint_rv(p_d, torch.tensor(g_ref, device="cuda"), cfg)
    assert ctx.sync() == 0
    e = max_rel(grad_d.cpu().numpy(), grad_ref)
    say(f"  gradient: max rel err {e:.2e}")
    assert e <= GRAD_BAR


def test_rv_box_room_mixed_lights(torch_dev, oracle_lib):
    """Box room with a spot, a rectangle (roll about its normal included), a
    soft-edged spot and a point light at random rotation vectors (one below
    the small-angle threshold), 2^18 paths, 3 hits."""
    sc = li.box_room()["scene"]
    p7 = np.array([[1.0, 1.0, 2.0, 0.15, -0.2, 0.3, 50.0], [2.0, 1.5, 2.4, -0.25, 0.1, 0.8, 70.0],
                   [2.8, 0.9, 2.3, 1e-8, 2e-8, -1e-8, 40.0], [3.0, 2.0, 1.8, 0.0, 0.0, 0.0, 30.0]], np.float32)
    lights = make_lights([SPOT, RECT, SOFT, POINT], [3.0, 1.0, 0.0, 0.0], [(0, 0), (0.5, 0.3), (0.3, 0.8), (0, 0)],
                         [0, 0, 0, 0], p7[:, :6])
    run_rv(torch_dev, oracle_lib, sc, lights, p7, 0x7A1, (1 << 18) + 5, 3, False)


def test_rv_office_reduced(torch_dev, oracle_lib):
    """The 200k-triangle office (16 area lights) at 2^18 paths and 5 hits with
    the launch tuning bench.py uses, its tilt angles given as rotation
    vectors plus a roll."""
    from scipy.spatial.transform import Rotation
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    p = lights.params
    p7 = np.zeros((lights.n_lights, 7), np.float32)
    for l in range(lights.n_lights):
        R = Rotation.from_euler("YX", [float(p[l, 4]), float(p[l, 3])]).as_matrix()
        roll = Rotation.from_rotvec([0.0, 0.0, 0.05 * (l % 5)]).as_matrix()
        p7[l, :3] = p[l, :3]
        p7[l, 3:6] = Rotation.from_matrix(R @ roll).as_rotvec()
        p7[l, 6] = p[l, 5]
    run_rv(torch_dev, oracle_lib, sc, lights, p7, c2["seed"], 1 << 18, c2["max_hits"], True,
           tuning=bench_tuning(sc, lights, c2["paths"], c2["max_hits"]))


def test_rv_invalid_arguments(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd import Context
    from paper_2310_02043_amd.native import LtError
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    ctx = Context(0)
    ctx.upload_scene(sc.verts, sc.tris, sc.tri_patch, sc.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    p_d = torch.zeros((lights.n_lights, 7), device="cuda")
    p_d[:, 2] = 2.0
    p_d[:, 6] = 10.0
    with pytest.raises(LtError):
        ctx.trace_forward_rv(p_d, ctx.cfg(1, 1 << 12, 3, linear=True))      # box basis only
