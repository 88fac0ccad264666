"""Directional texels with a glossy BRDF on the GPU vs the CPU oracle
(Eq. directionalCoeffs with n = 1 to 3 and the first hit's BRDF terms of the
adjoint), through the C ABI.  Bars as for the irradiance texels: texel
coefficients rel-L2 <= 1e-4, gradients 1e-3 relative; the tests report how
close they are.
"""
import sys

import numpy as np
import pytest

import lt_inputs as li
from lt_inputs.scenes import make_lights, POINT, SPOT, RECT
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


def run_dir(torch, oracle_lib, scene, lights, seed, N, B, order, samples, use_bvh, tuning=None):
    from paper_2310_02043_amd import Context
    rng = np.random.default_rng(seed)
    gl = np.stack([rng.uniform(0.0, 0.5, scene.n_patches), rng.uniform(2.0, 40.0, scene.n_patches)], 1)
    gl[:, 0] = np.minimum(gl[:, 0], 0.95 - scene.patches["albedo"])
    gl = gl.astype(np.float32)
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    if tuning:
        ctx.set_tuning(**tuning)
    ctx.set_glossy(gl)
    osc = oracle_lib.OracleScene(scene, use_bvh=use_bvh, glossy=gl, dir_order=order, dir_samples=samples)
    ol = oracle_lib.OracleLights(lights)
    p_d = torch.tensor(lights.params, device="cuda")
    cfg = ctx.cfg(seed, N, B)
    E_d, S_d = ctx.trace_forward_dir(p_d, cfg, order, samples)
    assert ctx.sync() == 0
    S_ref, _ = oracle_lib.forward(osc, ol, lights.params, seed, N, B)
    E_ref = oracle_lib.fixed_to_float(S_ref)
    r = rel_l2(E_d.cpu().numpy(), E_ref)
    say(f"  coefficients: rel-L2 {r:.2e}, bit-identical {np.mean(S_d.cpu().numpy() == S_ref) * 100:.4f} %")
    assert r <= TEX_BAR
    NC = (order + 1) ** 2
    Et = np.stack([np.stack([li.painted_target(scene, float(np.mean(np.abs(E_ref[j, c]))) * 1.5 + 1e-3,
                                               seed=NC * j + c) for c in range(NC)])
                   for j in range(lights.n_layouts)]).astype(np.float32)
    _, g_ref = oracle_lib.objective(E_ref, Et, scene.texel_area())
    grad_ref, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, N, B, g_ref)
    grad_d = ctx.trace_adjoint_dir(p_d, torch.tensor(g_ref, device="cuda"), cfg, order, samples)
    assert ctx.sync() == 0
    e = max_rel(grad_d.cpu().numpy(), grad_ref)
    say(f"  gradient: max rel err {e:.2e}")
    assert e <= GRAD_BAR


@pytest.mark.parametrize("order", [2, 3])
def test_dir_box_room_full(torch_dev, oracle_lib, order):
    """Closed room with two boxes at full size (2^20 paths, 3 hits), glossy
    patches, orders 2 and 3, 4 local samples per hit."""
    c1 = li.box_room()
    run_dir(torch_dev, oracle_lib, c1["scene"], c1["lights"], c1["seed"], c1["paths"], c1["max_hits"], order, 4,
            False)


def test_dir_mixed_lights_order1(torch_dev, oracle_lib):
    """Box room with a point light, a spot and a rectangle (whose origin shift
    enters the BRDF terms), order 1, 3 local samples (an odd count)."""
    sc = li.box_room()["scene"]
    lights = make_lights([POINT, SPOT, RECT], [0.0, 3.0, 1.0], [(0, 0), (0, 0), (0.5, 0.3)], [0, 0, 0],
                         [[3.0, 2.0, 1.8, 0, 0, 30.0], [1.0, 1.0, 2.0, 0.1, 0.2, 50.0],
                          [2.0, 1.5, 2.4, -0.2, 0.3, 70.0]])
    run_dir(torch_dev, oracle_lib, sc, lights, 0x5D1, (1 << 18) + 7, 3, 1, 3, False)


def test_dir_office_reduced(torch_dev, oracle_lib):
    """The 200k-triangle office at 2^18 paths, 5 hits, order 3, 2 local
    samples, with the launch tuning bench.py uses."""
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    run_dir(torch_dev, oracle_lib, sc, lights, c2["seed"], 1 << 18, c2["max_hits"], 3, 2, True,
            tuning=bench_tuning(sc, lights, c2["paths"], c2["max_hits"]))


def test_dir_invalid_arguments(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd import Context
    from paper_2310_02043_amd.native import LtError
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    ctx = Context(0)
    ctx.upload_scene(sc.verts, sc.tris, sc.tri_patch, sc.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    p_d = torch.tensor(lights.params, device="cuda")
    cfg = ctx.cfg(1, 1 << 12, 3)
    with pytest.raises(LtError):
        ctx.trace_forward_dir(p_d, cfg, 4, 4)                                   # order above 3
    with pytest.raises(LtError):
        ctx.trace_forward_dir(p_d, cfg, 1, 0)                                   # no local samples
    with pytest.raises(LtError):
        ctx.trace_forward_dir(p_d, ctx.cfg(1, 1 << 12, 3, linear=True), 1, 4)   # box basis only
    with pytest.raises(LtError):
        ctx.set_glossy(np.full((sc.n_patches, 2), 2.0, np.float32))             # specular albedo above 1


def _glossy_tracer(torch, scene, lights, paths, B, seed=9):
    from paper_2310_02043_amd.autograd import LightTracer
    gl = np.stack([np.full(scene.n_patches, 0.4), np.full(scene.n_patches, 16.0)], 1)
    gl[:, 0] = np.minimum(gl[:, 0], 0.95 - scene.patches["albedo"])
    tr = LightTracer((scene.verts, scene.tris, scene.tri_patch, scene.patches), lights.static, lights.layout_offsets,
                     paths, B, seed=seed, correlated=False)
    tr.ctx.set_glossy(gl.astype(np.float32))
    return tr


def test_dir_autograd_band_weights(torch_dev):
    """The directional autograd function's backward equals the direct
    directional adjoint with dO/dL = A alpha_k alpha_l (L - L*); the objective
    kernel with the expanded band weights (order-0 band at 0.1) agrees with
    the torch objective, and its order-0 dO/dL is 0.1 of the unweighted one."""
    torch = torch_dev
    from paper_2310_02043_amd.autograd import band_weights, directional_alpha, objective
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    tr = _glossy_tracer(torch, sc, lights, 1 << 20, 3)
    order, ns = 2, 4
    A = torch.tensor(sc.texel_area(), device="cuda")
    band = band_weights(order, 0.1, device="cuda")
    alpha = directional_alpha(band, torch.ones_like(A), 1)
    p = torch.tensor(lights.params, device="cuda", requires_grad=True)
    E = tr.directional(p, order, ns)
    Et = (E.detach() * 1.3 + 1e-3).contiguous()
    O = objective(E, Et, A, alpha=band[:, None])
    O.backward()
    g = (A * band[:, None] * (E.detach() - Et)).contiguous()
    ref = tr.ctx.trace_adjoint_dir(p.detach(), g, tr.cfg(tr.adjoint_seed(), adjoint=True), order, ns)
    torch.cuda.synchronize()
    rel = (p.grad - ref).abs().max().item() / ref.abs().max().item()
    say("  autograd vs direct directional adjoint:", rel)
    assert rel < 1e-5
    O_d, g_d = tr.ctx.objective(E.detach().contiguous(), Et, alpha)
    _, g_1 = tr.ctx.objective(E.detach().contiguous(), Et)
    torch.cuda.synchronize()
    assert abs(O_d.item() / O.item() - 1) < 1e-5
    assert torch.allclose(g_d, g, rtol=1e-6, atol=1e-7 * g.abs().max().item())
    assert torch.allclose(g_d[:, 0], 0.1 * g_1[:, 0], rtol=1e-6, atol=1e-7 * g_1.abs().max().item())
    assert torch.equal(g_d[:, 1:], g_1[:, 1:])


def test_dir_adam_recovers_spot(torch_dev):
    """Inverse directional lighting in the box room (glossy surfaces, order 2,
    order-0 band weighted 0.1): from a spot moved by 0.36 m and tilted by
    0.13 rad, Adam on the light-tracing gradients (fresh paths per step,
    decorrelated adjoint) brings the objective to within 1.5x of its value at
    the true parameters and the position to within 0.1 m."""
    torch = torch_dev
    from paper_2310_02043_amd.autograd import band_weights, objective
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    order, ns, B = 2, 4, 3
    tr = _glossy_tracer(torch, sc, lights, 1 << 18, B)
    A = torch.tensor(sc.texel_area(), device="cuda")
    band = band_weights(order, 0.1, device="cuda")[:, None]
    pt = torch.tensor(lights.params, device="cuda")
    with torch.no_grad():
        Et = tr.directional(pt, order, ns, seed=0x77).clone()
        O_true = objective(tr.directional(pt, order, ns, seed=999), Et, A, band).item()
    p0 = pt.clone()
    p0[0, 0] += 0.3
    p0[0, 1] -= 0.25
    p0[0, 3] += 0.12
    p = p0.clone().requires_grad_(True)
    lr = torch.tensor([0.02, 0.02, 0.02, 0.01, 0.01, 0.0], device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    O_first = None
    for it in range(80):
        p.grad = None
        O = objective(tr.directional(p, order, ns, seed=100 + it), Et, A, band)
        O.backward()
        O_first = O.item() if O_first is None else O_first
        with torch.no_grad():
            m.mul_(0.9).add_(0.1 * p.grad)
            v.mul_(0.999).add_(0.001 * p.grad * p.grad)
            p -= lr * (m / (1 - 0.9 ** (it + 1))) / ((v / (1 - 0.999 ** (it + 1))).sqrt() + 1e-8)
    pos_err = (p.detach() - pt)[0, :3].norm().item()
    say(f"  objective {O_first:.2f} -> {O.item():.2f} (true parameters {O_true:.2f}), position error "
        f"{(p0 - pt)[0, :3].norm().item():.3f} -> {pos_err:.3f} m")
    assert O.item() < 1.5 * O_true and pos_err < 0.1
