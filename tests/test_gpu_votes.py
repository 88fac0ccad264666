"""Gradient-contribution map (Sec. gradVis) on the GPU vs the CPU oracle.

The map of light l and parameter j holds, per texel, the sum of the paths'
contributions to dO/dp_j whose first surface hit lies in that texel.  Both
sides form every path's contribution in the same FP32 arithmetic and sum in
FP64 (the GPU in no fixed order), so the bars are those of the texel values
(rel-L2 <= 1e-4) and of the gradient (1e-3); the tests report how close they
actually are.  At the benchmark's full size, where the oracle cannot trace
every path, the map is checked against properties that hold at any size: it
sums to the gradient, it leaves the gradient of the plain adjoint pass
unchanged, and it equals the first-hit histogram of the per-path
contributions replayed one by one (the replay kernel is itself checked
against the oracle path by path).
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


def make_ctx(scene, lights, tuning=None):
    from paper_2310_02043_amd import Context
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    if tuning:
        ctx.set_tuning(**tuning)
    return ctx


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def target_grad(oracle_lib, osc, ol, scene, lights, params, seed, N, B):
    S, _ = oracle_lib.forward(osc, ol, params, seed, N, B)
    E = oracle_lib.fixed_to_float(S)
    Et = np.stack([li.painted_target(scene, float(np.mean(E[j])) * 1.5 + 1e-3, seed=j)
                   for j in range(lights.n_layouts)])
    return oracle_lib.objective(E, Et, scene.texel_area())[1]


def compare(torch, oracle_lib, ctx, osc, ol, params, seed, N, B, g, light, params_to_check, graph=False,
            linear=False):
    p_d = torch.tensor(params, device="cuda")
    g_d = torch.tensor(g, device="cuda")
    cfg = ctx.cfg(seed, N, B, graph=graph, linear=linear)
    for j in params_to_check:
        v_ref, grad_ref, _ = oracle_lib.votes(osc, ol, params, seed, N, B, g, light, j)
        v_d, grad_d = ctx.gradient_votes(p_d, g_d, cfg, light, j)
        assert ctx.sync() == 0
        v = v_d.cpu().numpy()
        gr = grad_d.cpu().numpy()[light].astype(np.float64)
        r = rel_l2(v, v_ref)
        exact = float(np.mean(v == v_ref))
        scale = float(np.abs(v).sum())
        say(f"  light {light} param {j}: map rel-L2 {r:.2e} (bit-identical texels {exact * 100:.2f} %), "
            f"sum vs gradient {abs(v.sum() - gr[j]) / scale:.1e}")
        assert r <= TEX_BAR
        assert abs(v.sum() - gr[j]) <= 1e-5 * scale
        rel = np.abs(gr - grad_ref) / np.maximum(np.abs(grad_ref), 1e-6 * np.abs(grad_ref).max() + 1e-30)
        assert float(rel.max()) <= GRAD_BAR


@pytest.mark.parametrize("basis", ["box", "linear"])
def test_votes_box_room_full(torch_dev, oracle_lib, basis):
    """Closed room with two boxes at full size (2^20 paths, 3 hits), every
    parameter, with the box and the piecewise-linear texel basis (the map
    still names the texel that contains the first hit)."""
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    osc, ol = oracle_lib.OracleScene(sc, basis=basis), oracle_lib.OracleLights(lights)
    g = target_grad(oracle_lib, osc, ol, sc, lights, lights.params, c1["seed"], c1["paths"], c1["max_hits"])
    ctx = make_ctx(sc, lights)
    compare(torch_dev, oracle_lib, ctx, osc, ol, lights.params, c1["seed"], c1["paths"], c1["max_hits"], g, 0,
            range(6), linear=basis == "linear")


@pytest.mark.parametrize("graph", [False, True])
def test_votes_office_reduced(torch_dev, oracle_lib, graph):
    """The 200k-triangle office at 2^18 paths and 5 hits with the launch tuning
    bench.py uses, two luminaires, position and power; eager and through a
    captured graph replayed twice."""
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    N, B = 1 << 18, c2["max_hits"]
    osc, ol = oracle_lib.OracleScene(sc, use_bvh=True), oracle_lib.OracleLights(lights)
    g = target_grad(oracle_lib, osc, ol, sc, lights, lights.params, c2["seed"], N, B)
    ctx = make_ctx(sc, lights, bench_tuning(sc, lights, c2["paths"], B))
    for light in (3, 12):
        reps = 2 if graph else 1
        for _ in range(reps):
            compare(torch_dev, oracle_lib, ctx, osc, ol, lights.params, c2["seed"], N, B, g, light, (0, 5),
                    graph=graph)


def test_votes_office_full_size(torch_dev, oracle_lib):
    """Bench launch configuration (2^26 paths, 5 hits): the map sums to the
    gradient, leaves the adjoint gradient bit-identical, and equals the
    first-hit histogram of all of the light's paths replayed one by one."""
    torch = torch_dev
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    N, B = c2["paths"], c2["max_hits"]
    tuning = bench_tuning(sc, lights, N, B)
    assert tuning is not None
    ctx = make_ctx(sc, lights, tuning)
    p_d = torch.tensor(lights.params, device="cuda")
    cfg = ctx.cfg(c2["seed"], N, B)
    E_d, _ = ctx.trace_forward(p_d, cfg)
    Et_d = torch.tensor(li.painted_target(sc, 0.5, seed=0)[None], device="cuda")
    _, g_d = ctx.objective(E_d, Et_d)
    grad_plain = ctx.trace_adjoint(p_d, g_d, cfg).cpu().numpy()
    light, j = 7, 3
    v_d, grad_d = ctx.gradient_votes(p_d, g_d, cfg, light, j)
    assert ctx.sync() == 0
    # the same per-path contributions; the plain adjoint sums them per tile in
    # FP64 in a second pass, the map's kernel per lane in FP32 first
    gv = grad_d.cpu().numpy().astype(np.float64)
    gp = grad_plain.astype(np.float64)
    e = float(np.max(np.abs(gv - gp) / np.maximum(np.abs(gp), 1e-6 * np.abs(gp).max())))
    say(f"  gradient beside the map vs the plain adjoint: max rel diff {e:.2e}")
    assert e <= 1e-5
    v = v_d.cpu().numpy()
    scale = float(np.abs(v).sum())
    say(f"  sum of the map {v.sum():.6e} vs gradient {grad_plain[light, j]:.6e}")
    assert abs(v.sum() - float(grad_plain[light, j])) <= 1e-5 * scale
    nl = N // lights.n_lights + (1 if light < N % lights.n_lights else 0)
    _, tex, con = ctx.record_paths(p_d, cfg, 0, light, 0, nl, dOdE=g_d)
    first = tex[:, 0].long()
    ok = first >= 0
    ref = torch.zeros(sc.n_texels, dtype=torch.float64, device="cuda")
    ref.index_add_(0, first[ok], con[ok, j].double())
    r = rel_l2(v, ref.cpu().numpy())
    say(f"  replayed first-hit histogram vs the map: rel-L2 {r:.2e}")
    assert r <= 1e-6


def test_votes_invalid_arguments(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd.native import LtError
    c1 = li.box_room()
    ctx = make_ctx(c1["scene"], c1["lights"])
    p_d = torch.tensor(c1["lights"].params, device="cuda")
    g_d = torch.zeros((1, c1["scene"].n_texels), dtype=torch.float32, device="cuda")
    cfg = ctx.cfg(1, 1 << 12, 3)
    with pytest.raises(LtError):
        ctx.gradient_votes(p_d, g_d, cfg, 1, 0)      # one light only
    with pytest.raises(LtError):
        ctx.gradient_votes(p_d, g_d, cfg, 0, 6)      # six parameters
    with pytest.raises(LtError):
        ctx.gradient_votes(p_d, g_d, cfg, -1, 0)
