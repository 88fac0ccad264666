"""GPU path vs the CPU oracle, element by element on identical seeded inputs.

Everything on the GPU side goes through the C ABI (liblt.so).  Oracle inputs
and expected values come only from the generators and the oracle.  Bars
(from the method's target): texel irradiance rel-L2 <= 1e-4, gradient
components <= 1e-3 relative, hit sequences identical on >= 99.99 % of paths.
The arithmetic contract makes the two sides bit-identical in practice; the
tests also report how many texels / paths match exactly.
"""
import math
import sys

import numpy as np
import pytest

import lt_inputs as li
from lt_inputs.scenes import make_lights, POINT, SPOT, RECT, SOFT
from tuning_cache import bench_tuning

pytestmark = pytest.mark.gpu

TEX_BAR, GRAD_BAR, PATH_BAR = 1e-4, 1e-3, 0.9999


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_ctx(torch, scene, lights):
    from paper_2310_02043_amd import Context
    ctx = Context(0)
    K = ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    assert K == scene.n_texels
    ctx.set_lights(lights.static, lights.layout_offsets)
    return ctx


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def grad_rel(g_gpu, g_ref):
    g_gpu = np.asarray(g_gpu, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    scale = np.maximum(np.abs(g_ref), 1e-6 * np.abs(g_ref).max() + 1e-30)
    return float(np.max(np.abs(g_gpu - g_ref) / scale))


def run_case(torch, oracle_lib, scene, lights, params, seed, ppl, B, use_bvh, check_grad=True, target=None,
             graph=False, tuning=None, linear=False):
    ctx = make_ctx(torch, scene, lights)
    if tuning:
        ctx.set_tuning(**tuning)
    osc = oracle_lib.OracleScene(scene, use_bvh=use_bvh, basis="linear" if linear else "box")
    ol = oracle_lib.OracleLights(lights)
    p_d = torch.tensor(params, device="cuda")
    cfg = ctx.cfg(seed, ppl, B, graph=graph, linear=linear)
    E_d, S_d = ctx.trace_forward(p_d, cfg)
    assert ctx.sync() == 0
    S_ref, miss_ref = oracle_lib.forward(osc, ol, params, seed, ppl, B)
    S_gpu = S_d.cpu().numpy()
    E_ref = oracle_lib.fixed_to_float(S_ref)
    exact = float((S_gpu == S_ref).mean())
    r = rel_l2(E_d.cpu().numpy(), E_ref)
    say(f"  texels: rel-L2 {r:.3e}, bit-identical {exact * 100:.4f} %")
    assert r <= TEX_BAR
    out = dict(ctx=ctx, E_ref=E_ref, S_ref=S_ref, exact=exact, p_d=p_d, osc=osc, ol=ol)
    if check_grad:
        Et = target if target is not None else np.stack(
            [li.painted_target(scene, float(np.mean(E_ref[j])) * 1.5 + 1e-3, seed=j) for j in range(lights.n_layouts)])
        O_ref, g_ref = oracle_lib.objective(E_ref, Et, scene.texel_area())
        grad_ref, _ = oracle_lib.adjoint(osc, ol, params, seed, ppl, B, g_ref)
        g_d = torch.tensor(g_ref, device="cuda")
        grad_d = ctx.trace_adjoint(p_d, g_d, cfg)
        ctx.sync()
        e = grad_rel(grad_d.cpu().numpy(), grad_ref)
        say(f"  gradient: max rel err {e:.3e}")
        assert e <= GRAD_BAR
        out.update(g_ref=g_ref, grad_ref=grad_ref, Et=Et, O_ref=O_ref, g_d=g_d)
    return out


@pytest.mark.parametrize("basis", ["box", "linear"])
def test_box_room_full(torch_dev, oracle_lib, basis):
    """Closed 4x3x2.5 m room + two boxes, spot cos^4, 2^20 paths, 3 hits (full
    size), with the box and the piecewise-linear texel basis."""
    torch = torch_dev
    c1 = li.box_room()
    say("box_room full: paths", c1["paths"], "basis", basis)
    run_case(torch, oracle_lib, c1["scene"], c1["lights"], c1["lights"].params, c1["seed"], c1["paths"],
             c1["max_hits"], use_bvh=False, linear=basis == "linear")


@pytest.mark.parametrize("basis", ["box", "linear"])
def test_box_room_hit_sequences(torch_dev, oracle_lib, basis):
    """Every path of the box room replayed one by one: hit sequences and
    per-path adjoint contributions (whose gather depends on the basis)."""
    torch = torch_dev
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    ctx = make_ctx(torch, sc, lights)
    p_d = torch.tensor(lights.params, device="cuda")
    N, B = c1["paths"], c1["max_hits"]
    lin = basis == "linear"
    cfg = ctx.cfg(c1["seed"], N, B, linear=lin)
    g = np.random.default_rng(4).normal(size=(1, sc.n_texels)).astype(np.float32)
    prim_d, tex_d, con_d = ctx.record_paths(p_d, cfg, 0, 0, 0, N, dOdE=torch.tensor(g, device="cuda"))
    prim_ref, tex_ref, con_ref = oracle_lib.record(oracle_lib.OracleScene(sc, basis=basis),
                                                   oracle_lib.OracleLights(lights), lights.params, c1["seed"], N, B,
                                                   0, 0, 0, N, dOdE=g)
    same = np.all(prim_d.cpu().numpy() == prim_ref, 1) & np.all(tex_d.cpu().numpy() == tex_ref, 1)
    say(f"  identical hit sequences: {same.mean() * 100:.4f} % of {N}")
    assert same.mean() >= PATH_BAR
    c = con_d.cpu().numpy()
    r = rel_l2(c[same], con_ref[same])
    say(f"  per-path contributions rel-L2 {r:.2e}, bit-identical {np.mean(c == con_ref) * 100:.4f} %")
    assert r <= 1e-5


def test_objective_matches(torch_dev, oracle_lib):
    torch = torch_dev
    c1 = li.box_room()
    sc = c1["scene"]
    ctx = make_ctx(torch, sc, c1["lights"])
    rng = np.random.default_rng(3)
    E = rng.uniform(0, 40, (1, sc.n_texels)).astype(np.float32)
    Et = li.painted_target(sc, 20.0)[None]
    al = rng.uniform(0, 2, E.shape).astype(np.float32)
    O_ref, g_ref = oracle_lib.objective(E, Et, sc.texel_area(), al)
    O_d, g_d = ctx.objective(torch.tensor(E, device="cuda"), torch.tensor(Et, device="cuda"),
                             torch.tensor(al, device="cuda"))
    assert abs(O_d.item() / O_ref - 1) < 1e-12
    assert np.array_equal(g_d.cpu().numpy(), g_ref)


@pytest.mark.parametrize("launch", ["default", "bench"])
def test_office_reduced_paths(torch_dev, oracle_lib, launch):
    """The full 200k-triangle office at 2^18 paths (oracle-sized), 5 hits, 16
    area lights, with the default launch tuning and with the one bench.py
    times (the same kernel instance and tile, refill and scheduling settings)."""
    torch = torch_dev
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    tuning = bench_tuning(sc, lights, c2["paths"], c2["max_hits"]) if launch == "bench" else None
    say("office reduced: tris", sc.n_tris, "texels", sc.n_texels, "tuning", tuning)
    assert launch == "default" or tuning is not None
    run_case(torch, oracle_lib, sc, lights, lights.params, c2["seed"], 1 << 18, c2["max_hits"], use_bvh=True,
             tuning=tuning)


@pytest.mark.parametrize("basis", ["box", "linear"])
def test_office_full_size_sampled(torch_dev, oracle_lib, basis):
    """Bench launch configuration (2^26 paths, 5 hits): sampled paths vs the
    oracle one by one, plus the power identity sum_l P_l dO/dP_l = sum_k g_k E_k,
    with the box and the piecewise-linear texel basis."""
    full_size_sampled(torch_dev, oracle_lib, li.office(), linear=basis == "linear")


def test_building_full_size_sampled(torch_dev, oracle_lib):
    """Building floor in the bench launch configuration (2M triangles, 16M
    texels, 128 luminaires, 2^28 paths, 6 hits): sampled paths vs the oracle
    one by one, plus the power identity."""
    full_size_sampled(torch_dev, oracle_lib, li.building_floor())


def test_room_set_full_size_sampled(torch_dev, oracle_lib):
    """Room set in the bench launch configuration (64 layouts of 4-48 lights,
    2^22 paths per layout, 4 hits): sampled paths of random layouts vs the
    oracle one by one, the power identity over all layouts, and all paths of
    one light replayed against the adjoint kernel."""
    full_size_sampled(torch_dev, oracle_lib, li.room_set())


@pytest.mark.parametrize("workload", ["office", "building", "room_set"])
def test_full_size_one_luminaire_exact(torch_dev, oracle_lib, workload):
    """The forward kernel at the bench's full size and launch tuning (office:
    2^26 paths, 5 hits; building floor: 2^28 paths, 6 hits; room set: 64
    layouts x 2^22 paths, 4 hits, a luminaire of layout 37), bit for bit
    against the oracle for one luminaire's paths.  S is an integer sum, so
    the difference of two full launches, one with every luminaire and one
    with this luminaire rejected (negative power: it traces nothing), is
    exactly its share; the oracle traces its paths alone, the others at zero
    power.  The adjoint launch at the same size gives that luminaire's
    gradient row from its own paths only, so the oracle's adjoint of the
    luminaire alone (the same dO/dE) must agree with it to the gradient
    bar."""
    torch = torch_dev
    from paper_2310_02043_amd.native import LtError, LT_EINVAL
    c = {"office": li.office, "building": li.building_floor, "room_set": li.room_set}[workload]()
    sc, lights = c["scene"], c["lights"]
    N, B, seed = c["paths"], c["max_hits"], c["seed"]
    ctx = make_ctx(torch, sc, lights)
    tuning = bench_tuning(sc, lights, N, B)
    assert tuning is not None
    ctx.set_tuning(**tuning)
    say(f"{workload}: {sc.n_tris} triangles, {lights.n_lights} luminaires, {N} paths, tuning {tuning}")
    l = 5 if workload != "room_set" else int(lights.layout_offsets[37]) + 2
    p = np.asarray(lights.params, np.float32).copy()
    cfg = ctx.cfg(seed, N, B)
    _, S_all = ctx.trace_forward(torch.tensor(p, device="cuda"), cfg)
    assert ctx.sync() == 0
    S_all = S_all.cpu().numpy().copy()
    p_wo = p.copy()
    p_wo[l, 5] = -1.0
    _, S_wo = ctx.trace_forward(torch.tensor(p_wo, device="cuda"), cfg)
    with pytest.raises(LtError) as ei:
        ctx.sync()
    assert ei.value.code == LT_EINVAL
    S_l = S_all - S_wo.cpu().numpy()
    only = p.copy()
    only[:, 5] = 0.0
    only[l, 5] = p[l, 5]
    osc = oracle_lib.OracleScene(sc, use_bvh=True)
    S_ref, _ = oracle_lib.forward(osc, oracle_lib.OracleLights(lights), only, seed, N, B)
    say(f"  luminaire {l}: {np.count_nonzero(S_ref)} texels reached, "
        f"bit-identical {np.mean(S_l == S_ref) * 100:.4f} %")
    assert np.count_nonzero(S_ref) > 0
    assert np.array_equal(S_l, S_ref)
    E_all = oracle_lib.fixed_to_float(S_all)
    Et = np.stack([li.painted_target(sc, float(np.mean(E_all[j])) * 1.5 + 1e-3, seed=3 + j)
                   for j in range(lights.n_layouts)])
    _, g = oracle_lib.objective(E_all, Et, sc.texel_area())
    grad_d = ctx.trace_adjoint(torch.tensor(p, device="cuda"), torch.tensor(g, device="cuda"), cfg)
    assert ctx.sync() == 0
    grad_ref, _ = oracle_lib.adjoint(osc, oracle_lib.OracleLights(lights), only, seed, N, B, g)
    e = grad_rel(grad_d.cpu().numpy()[l], grad_ref[l])
    say(f"  luminaire {l}: gradient row max rel err {e:.3e}")
    assert e <= GRAD_BAR


@pytest.mark.parametrize("variant", ["linear", "colour"])
def test_office_full_size_one_luminaire_variants(torch_dev, oracle_lib, variant):
    """The office at full size (2^26 paths, 5 hits) and bench tuning with the
    piecewise-linear texel basis or in colour (per-luminaire channel weights,
    per-patch channel albedo): one luminaire's texels, isolated as the
    integer difference of a launch with every luminaire and one with it
    rejected, bit-identical to the oracle's for that luminaire alone."""
    torch = torch_dev
    from paper_2310_02043_amd.native import LtError, LT_EINVAL
    c = li.office()
    sc, lights = c["scene"], c["lights"]
    N, B, seed = c["paths"], c["max_hits"], c["seed"]
    ctx = make_ctx(torch, sc, lights)
    ctx.set_tuning(**bench_tuning(sc, lights, N, B))
    if variant == "colour":
        rng = np.random.default_rng(seed)
        alb = rng.uniform(0.3, 0.8, (sc.n_patches, 3)).astype(np.float32)
        col = rng.dirichlet([2.0, 2.0, 2.0], lights.n_lights).astype(np.float32)
        ctx.set_albedo_rgb(alb)
        c_d = torch.tensor(col, device="cuda")
        cfg = ctx.cfg(seed, N, B)

        def fwd(pp):
            return ctx.trace_forward_rgb(torch.tensor(pp, device="cuda"), c_d, cfg)[1]

        osc = oracle_lib.OracleScene(sc, use_bvh=True, albedo_rgb=alb)
        ol = oracle_lib.OracleLights(lights, col)
    else:
        cfg = ctx.cfg(seed, N, B, linear=True)

        def fwd(pp):
            return ctx.trace_forward(torch.tensor(pp, device="cuda"), cfg)[1]

        osc = oracle_lib.OracleScene(sc, use_bvh=True, basis="linear")
        ol = oracle_lib.OracleLights(lights)
    l = 9
    p = np.asarray(lights.params, np.float32).copy()
    S_all = fwd(p).cpu().numpy().copy()
    assert ctx.sync() == 0
    p_wo = p.copy()
    p_wo[l, 5] = -1.0
    S_wo = fwd(p_wo).cpu().numpy()
    with pytest.raises(LtError) as ei:
        ctx.sync()
    assert ei.value.code == LT_EINVAL
    only = p.copy()
    only[:, 5] = 0.0
    only[l, 5] = p[l, 5]
    S_ref, _ = oracle_lib.forward(osc, ol, only, seed, N, B)
    S_l = S_all - S_wo
    say(f"office {variant}: luminaire {l}, {np.count_nonzero(S_ref)} texel values reached, "
        f"bit-identical {np.mean(S_l == S_ref) * 100:.4f} %")
    assert np.count_nonzero(S_ref) > 0
    assert np.array_equal(S_l, S_ref)


def full_size_sampled(torch, oracle_lib, c2, linear=False):
    sc, lights = c2["scene"], c2["lights"]
    ctx = make_ctx(torch, sc, lights)
    N, B = c2["paths"], c2["max_hits"]
    tuning = bench_tuning(sc, lights, N, B)
    assert tuning is not None
    ctx.set_tuning(**tuning)
    say("  tuning", tuning)
    osc = oracle_lib.OracleScene(sc, use_bvh=True, basis="linear" if linear else "box")
    ol = oracle_lib.OracleLights(lights)
    p_d = torch.tensor(lights.params, device="cuda")
    cfg = ctx.cfg(c2["seed"], N, B, linear=linear)
    E_d, S_d = ctx.trace_forward(p_d, cfg)
    assert ctx.sync() == 0
    nly = lights.n_layouts
    Et_d = torch.tensor(np.stack([li.painted_target(sc, 0.5, seed=j) for j in range(nly)]), device="cuda")
    O_d, g_d = ctx.objective(E_d, Et_d)
    grad_d = ctx.trace_adjoint(p_d, g_d, cfg)
    ctx.sync()
    lhs = float(np.sum(lights.params[:, 5].astype(np.float64) * grad_d.cpu().numpy()[:, 5].astype(np.float64)))
    rhs = float(torch.sum(g_d.double() * E_d.double()).item())
    say(f"  power identity: {lhs:.6e} vs {rhs:.6e}")
    assert abs(lhs / rhs - 1) < 1e-4
    offs = np.asarray(lights.layout_offsets)

    def paths_of(gl):
        j = int(np.searchsorted(offs, gl, side="right") - 1)
        L, l = int(offs[j + 1] - offs[j]), int(gl - offs[j])
        return j, l, N // L + (1 if l < N % L else 0)

    rng = np.random.default_rng(9)
    g_np = g_d.cpu().numpy()
    n_same = n_tot = 0
    for gl in rng.choice(lights.n_lights, 4, replace=False):
        j, l, nl = paths_of(int(gl))
        first = int(rng.integers(0, nl - 4096))
        prim_d, tex_d, con_d = ctx.record_paths(p_d, cfg, j, l, first, 4096, dOdE=g_d)
        prim_r, tex_r, con_r = oracle_lib.record(osc, ol, lights.params, c2["seed"], N, B, j, l, first, 4096,
                                                 dOdE=g_np)
        same = np.all(prim_d.cpu().numpy() == prim_r, 1) & np.all(tex_d.cpu().numpy() == tex_r, 1)
        n_same += int(same.sum())
        n_tot += same.size
        c = con_d.cpu().numpy()
        assert rel_l2(c[same], con_r[same]) < 1e-5
    say(f"  sampled identical hit sequences: {n_same}/{n_tot}")
    assert n_same / n_tot >= PATH_BAR
    # every path of one light replayed one by one (the per-path kernel checked
    # against the oracle above) sums to the tuned adjoint kernel's gradient
    gl = int(rng.integers(0, lights.n_lights))
    j, l, nl = paths_of(gl)
    _, _, con_all = ctx.record_paths(p_d, cfg, j, l, 0, nl, dOdE=g_d)
    tot = con_all.double().sum(0).cpu().numpy()
    ref = grad_d.cpu().numpy()[gl].astype(np.float64)
    err = float(np.max(np.abs(tot - ref)) / np.max(np.abs(ref)))
    say(f"  light {gl}: all {nl} replayed paths vs the adjoint kernel, max rel err {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("launch", ["default", "bench"])
def test_batched_layouts_reduced(torch_dev, oracle_lib, launch):
    """Room set with 64 layouts of 4..48 lights in one launch (2^14 paths per
    layout), with the default launch tuning and with the one bench.py times."""
    torch = torch_dev
    c3 = li.room_set()
    tuning = bench_tuning(c3["scene"], c3["lights"], c3["paths"], c3["max_hits"]) if launch == "bench" else None
    say("room_set: layouts", c3["lights"].n_layouts, "lights", c3["lights"].n_lights, "tuning", tuning)
    assert launch == "default" or tuning is not None
    run_case(torch, oracle_lib, c3["scene"], c3["lights"], c3["lights"].params, c3["seed"], 1 << 14,
             c3["max_hits"], use_bvh=True, tuning=tuning)


@pytest.mark.parametrize("case", ["box_room", "room_set_64_layouts"])
def test_graph_replay_matches_eager_and_oracle(torch_dev, oracle_lib, case):
    """The forward and adjoint sequences captured as hipGraphs and replayed
    into fixed buffers (so every call after the first replays the cached
    graph): S, E and the gradient bit-identical to an eager run on every
    replay, with unrelated eager work between replays, and the eager run
    bit-identical (texels) / within 1e-3 (gradient) of the oracle.  Inputs
    changed in place between replays (dO/dE doubled, a luminaire moved) must
    be seen by the replay, so a graph holding stale pointers or sizes fails."""
    torch = torch_dev
    if case == "box_room":
        c = li.box_room()
        ppl, use_bvh = 1 << 18, False
    else:
        c = li.room_set()
        ppl, use_bvh = 1 << 14, True
    sc, lights, B, seed = c["scene"], c["lights"], c["max_hits"], 77
    say(f"graph replay: {case}, {lights.n_layouts} layouts, {ppl} paths per layout")
    ctx = make_ctx(torch, sc, lights)
    nl, K = lights.n_layouts, sc.n_texels
    p_d = torch.tensor(lights.params, device="cuda")
    S = torch.empty((nl, K), dtype=torch.int64, device="cuda")
    E = torch.empty((nl, K), dtype=torch.float32, device="cuda")
    grad = torch.empty((lights.n_lights, 6), dtype=torch.float32, device="cuda")
    # eager reference and the oracle
    cfg_e, cfg_g = ctx.cfg(seed, ppl, B), ctx.cfg(seed, ppl, B, graph=True)
    ctx.trace_forward(p_d, cfg_e, S=S, E=E)
    S_e, E_e = S.clone(), E.clone()
    osc, ol = oracle_lib.OracleScene(sc, use_bvh=use_bvh), oracle_lib.OracleLights(lights)
    S_ref, _ = oracle_lib.forward(osc, ol, lights.params, seed, ppl, B)
    assert np.array_equal(S_e.cpu().numpy(), S_ref)
    Et = np.stack([li.painted_target(sc, float(np.mean(oracle_lib.fixed_to_float(S_ref)[j])) * 1.5 + 1e-3, seed=j)
                   for j in range(nl)])
    _, g_ref = oracle_lib.objective(oracle_lib.fixed_to_float(S_ref), Et, sc.texel_area())
    g = torch.tensor(g_ref, device="cuda")
    ctx.trace_adjoint(p_d, g, cfg_e, grad=grad)
    G_e = grad.clone()
    grad_ref, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, ppl, B, g_ref)
    e = grad_rel(G_e.cpu().numpy(), grad_ref)
    say(f"  eager gradient vs oracle: max rel err {e:.3e}")
    assert e <= GRAD_BAR
    for rep in range(4):
        S.fill_(-1)
        E.fill_(float("nan"))
        grad.fill_(float("nan"))
        ctx.trace_forward(p_d, cfg_g, S=S, E=E)
        torch.cuda.synchronize()
        assert torch.equal(S, S_e) and torch.equal(E, E_e), rep
        ctx.trace_adjoint(p_d, g, cfg_g, grad=grad)
        torch.cuda.synchronize()
        assert torch.equal(grad, G_e), rep
        _ = (E * 2).sum().item()   # unrelated eager work between replays
    assert ctx.sync() == 0
    # the replay reads its inputs through the captured pointers: new contents
    # are seen (the adjoint is linear in dO/dE and doubling is exact in FP32)
    g.mul_(2.0)
    ctx.trace_adjoint(p_d, g, cfg_g, grad=grad)
    torch.cuda.synchronize()
    assert torch.equal(grad, 2.0 * G_e)
    p_d[0, 0] += 0.05
    ctx.trace_forward(p_d, cfg_g, S=S, E=E)
    S_moved = S.clone()
    ctx.trace_forward(p_d, cfg_e, S=S, E=E)
    torch.cuda.synchronize()
    assert torch.equal(S_moved, S) and not torch.equal(S_moved, S_e)
    assert ctx.sync() == 0


def test_autotune_search_parity(torch_dev, oracle_lib, tmp_path):
    """lt_autotune's coordinate search (no cache entry) on the box room picks
    a launch shape; traced with it, texels are bit-identical to the oracle's
    and the gradient within 1e-3; the choice is written to the cache file and
    a second context reads it back instead of searching."""
    torch = torch_dev
    c1 = li.box_room()
    sc, lights, B, seed = c1["scene"], c1["lights"], c1["max_hits"], c1["seed"]
    ppl = c1["paths"]
    ctx = make_ctx(torch, sc, lights)
    p_d = torch.tensor(lights.params, device="cuda")
    S = torch.empty((1, sc.n_texels), dtype=torch.int64, device="cuda")
    E = torch.empty((1, sc.n_texels), dtype=torch.float32, device="cuda")
    g = torch.randn((1, sc.n_texels), device="cuda")
    grad = torch.empty((lights.n_lights, 6), dtype=torch.float32, device="cuda")
    cache = str(tmp_path / "tuning.cache")
    before = ctx.get_tuning().as_dict()
    best = ctx.autotune(p_d, ctx.cfg(seed, ppl, B), S, E, g, grad, cache_path=cache)
    chosen = ctx.get_tuning().as_dict()
    say(f"  autotune: {before} -> {chosen} ({best:.3f} ms fwd+adj)")
    assert best > 0.0
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1
    cfg = ctx.cfg(seed, ppl, B)
    ctx.trace_forward(p_d, cfg, S=S, E=E)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    S_ref, _ = oracle_lib.forward(osc, ol, lights.params, seed, ppl, B)
    assert np.array_equal(S.cpu().numpy(), S_ref)
    E_ref = oracle_lib.fixed_to_float(S_ref)
    _, g_ref = oracle_lib.objective(E_ref, li.painted_target(sc, 20.0)[None], sc.texel_area())
    grad_ref, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, ppl, B, g_ref)
    gr = ctx.trace_adjoint(p_d, torch.tensor(g_ref, device="cuda"), cfg)
    assert ctx.sync() == 0
    e = grad_rel(gr.cpu().numpy(), grad_ref)
    say(f"  tuned launch: texels bit-identical, gradient max rel err {e:.3e}")
    assert e <= GRAD_BAR
    ctx2 = make_ctx(torch, sc, lights)
    best2 = ctx2.autotune(p_d, ctx2.cfg(seed, ppl, B), S, E, g, grad, cache_path=cache)
    assert ctx2.get_tuning().as_dict() == chosen and abs(best2 - best) < 1e-2
    assert len(open(cache).read().strip().splitlines()) == 1


@pytest.mark.parametrize("case", ["ragged", "one_path_per_light", "single_hit", "point_closed_box",
                                  "tiny_scene", "rect_many_lights", "soft_spots", "linear_ragged"])
def test_edge_cases(torch_dev, oracle_lib, case):
    torch = torch_dev
    if case == "ragged":
        sc = li.box_room()["scene"]
        lights = make_lights([SPOT, POINT, RECT], [3.0, 0.0, 2.0], [(0, 0), (0, 0), (0.5, 0.3)], [0, 0, 0],
                             [[1.0, 1.0, 2.0, 0.1, 0.2, 50.0], [3.0, 2.0, 1.8, 0, 0, 30.0],
                              [2.0, 1.5, 2.4, -0.2, 0.3, 70.0]])
        ppl, B = 100_003, 3
    elif case == "one_path_per_light":
        sc = li.box_room()["scene"]
        lights = make_lights([SPOT, POINT], [3.0, 0.0], [(0, 0), (0, 0)], [0, 1],
                             [[1.0, 1.0, 2.0, 0.1, 0.2, 50.0], [3.0, 2.0, 1.8, 0, 0, 30.0]])
        ppl, B = 1, 3
    elif case == "single_hit":
        sc = li.plane_scene(half=3.0, res=32)
        lights = make_lights([POINT], [0.0], [(0, 0)], [0], [[0.2, 0.1, 1.0, 0, 0, 10.0]])
        ppl, B = 1 << 16, 1
    elif case == "point_closed_box":
        sc = li.closed_box(albedo=0.7)
        lights = make_lights([POINT], [0.0], [(0, 0)], [0], [[0.9, 0.8, 0.4, 0, 0, 10.0]])
        ppl, B = 1 << 16, 8
    elif case == "tiny_scene":
        sb = li.SceneBuilder()
        sb.quads([-1.0, -1.0, 0.0], [2.0, 0, 0], [0, 2.0, 0], 0.5, res=(3, 5))
        sc = sb.build("one_quad", fixed_res=(3, 5))
        lights = make_lights([SPOT], [1.0], [(0, 0)], [0], [[0.0, 0.0, 1.0, 0.0, 0.0, 5.0]])
        ppl, B = 5000, 2
    elif case == "linear_ragged":
        # piecewise-linear basis on odd patch resolutions and a 1 x n strip
        sb = li.SceneBuilder()
        sb.quads([-2.0, -2.0, 0.0], [4.0, 0, 0], [0, 4.0, 0], 0.6, res=(7, 5))
        sb.quads([-2.0, -2.0, 2.5], [4.0, 0, 0], [0, 4.0, 0], 0.7, res=(1, 9))
        sc = sb.build("floor_ceiling_ragged")
        lights = make_lights([SPOT, POINT], [2.0, 0.0], [(0, 0), (0, 0)], [0, 0],
                             [[0.3, 0.2, 1.5, 0.1, -0.1, 40.0], [-0.5, 0.4, 1.0, 0, 0, 20.0]])
        ppl, B = 50_001, 3
    elif case == "soft_spots":
        # the supplement's soft-edged spots: a narrow ring, a pure fall-off
        # over the hemisphere, a hard-edged cone, beside a cos^n spot
        sc = li.box_room()["scene"]
        lights = make_lights([SOFT, SOFT, SOFT, SPOT], [0.0, 0.0, 0.0, 2.0],
                             [(0.5, 0.55), (0.0, 1.5707963), (0.6, 0.6001), (0, 0)], [0, 0, 0, 0],
                             [[1.2, 1.1, 2.3, 0.2, -0.1, 40.0], [2.9, 2.0, 1.6, -0.3, 0.2, 25.0],
                              [2.0, 1.0, 2.4, 0.0, 0.3, 60.0], [3.1, 0.8, 2.2, 0.1, 0.1, 30.0]])
        ppl, B = (1 << 18) + 3, 4
    else:
        sc = li.box_room()["scene"]
        n = 40
        rng = np.random.default_rng(2)
        ps = [[rng.uniform(0.5, 3.5), rng.uniform(0.5, 2.5), rng.uniform(1.5, 2.4), rng.uniform(-0.3, 0.3),
               rng.uniform(-0.3, 0.3), rng.uniform(5, 20)] for _ in range(n)]
        lights = make_lights([RECT] * n, rng.uniform(1, 6, n), [(0.3, 0.2)] * n, [0] * n, ps)
        ppl, B = 40 * 1000 + 17, 4
    say("edge case", case)
    out = run_case(torch, oracle_lib, sc, lights, lights.params, 0xE0 + len(case), ppl, B, use_bvh=False,
                   linear=case == "linear_ragged")
    if case == "point_closed_box":
        assert out["S_ref"].sum() > 0


def _guaranteed_stack_depth(nodes, point):
    """Stack entries a traversal from `point` must hold at some moment: each
    internal child whose stored box contains the point is entered at
    distance 0, and such children are visited in slot order, the others
    waiting on the stack; so descending into the r-th of m such children
    leaves m - 1 - r entries below it, and the deepest root-to-leaf sum of
    these is reached whatever the closest-hit distance (children the ray
    enters farther away only add)."""
    from test_gpu_bvh import decode
    lo, hi, ni, _, first_child, _ = decode(nodes)

    def deepest(node):
        inside = [k for k in range(int(ni[node])) if np.all(lo[node, k] <= point) and np.all(point <= hi[node, k])]
        return max([len(inside) - 1 - r + deepest(int(first_child[node] + k)) for r, k in enumerate(inside)],
                   default=0)

    return deepest(0)


@pytest.mark.parametrize("lds_depth", [16, 32])
def test_crossing_slivers_overflow_stack(torch_dev, oracle_lib, lds_depth):
    """15550 narrow 2 m x 2 cm quads in random directions, each passing 1 cm
    beside and 1 cm above a point light: every triangle's box, hence every
    box of the tree, contains the light, so a segment from it pushes three
    children at every
    level and its traversal stack runs past its LDS entries (checked on the
    device's own tree) into the wave's overflow area.  Forward bit-identical,
    gradients to the bar, with 16 and 32 LDS entries."""
    torch = torch_dev
    sc, pl = li.crossing_slivers()
    lights = make_lights([POINT], [0.0], [(0, 0)], [0], [[pl[0], pl[1], pl[2], 0, 0, 10.0]])
    ctx = make_ctx(torch, sc, lights)
    nodes, _ = ctx.bvh()
    depth = _guaranteed_stack_depth(nodes, pl)
    say(f"crossing slivers: {sc.n_tris} triangles, {nodes.shape[0]} nodes, stack depth from the light >= {depth}")
    assert depth > 16
    out = run_case(torch, oracle_lib, sc, lights, lights.params, 0x57AC, 1 << 13, 3, use_bvh=True,
                   tuning=dict(lds_depth=lds_depth))
    assert out["exact"] == 1.0


def _translated(scene, off):
    """The same scene moved by off (vertices and patch origins)."""
    import dataclasses
    patches = scene.patches.copy()
    patches["origin"] = (patches["origin"].astype(np.float64) + off).astype(np.float32)
    verts = (scene.verts.astype(np.float64) + off).astype(np.float32)
    return dataclasses.replace(scene, verts=verts, patches=patches)


def _two_far_rooms(dx):
    """Two closed box rooms dx apart along x, one spot in each."""
    import dataclasses
    a = li.box_room()["scene"]
    b = _translated(a, np.array([dx, 0.0, 0.0]))
    patches = np.concatenate([a.patches, b.patches])
    patches["texel_base"][a.n_patches:] += a.n_texels
    return dataclasses.replace(a, name="two_far_rooms", verts=np.concatenate([a.verts, b.verts]),
                               tris=np.concatenate([a.tris, b.tris + a.verts.shape[0]]),
                               tri_patch=np.concatenate([a.tri_patch, b.tri_patch + a.n_patches]),
                               patches=patches, n_texels=2 * a.n_texels)


@pytest.mark.parametrize("case", ["office_far_from_origin", "rooms_90km_apart"])
def test_compact_node_precision(torch_dev, oracle_lib, case):
    """The wide nodes keep child planes as f16 offsets from a bf16 origin,
    rounded outward.  Scenes that stress that encoding must still give the
    oracle's hits: an office of 20k triangles moved 4.6 km from the origin
    (bf16 origin steps of 16-32 m, f16 offsets up to tens of metres), and two
    rooms 90 km apart (the root's offsets beyond the f16 range, stored as
    65504 / +inf).  Texels, gradients and sampled hit sequences vs the oracle."""
    torch = torch_dev
    if case == "office_far_from_origin":
        c = li.office(target_tris=20_000, target_texels=200_000, n_lights=4)
        off = np.array([4096.3, -2048.7, 517.1])
        sc = _translated(c["scene"], off)
        prm = c["lights"].params.astype(np.float64)
        prm[:, :3] += off
        lights = make_lights([RECT] * 4, c["lights"].static["lobe_n"], [(0.6, 0.6)] * 4, [0] * 4,
                             prm.astype(np.float32))
        ppl, B, use_bvh = 1 << 16, 4, True
    else:
        sc = _two_far_rooms(90_000.0)
        lights = make_lights([SPOT, SPOT], [3.0, 2.0], [(0, 0), (0, 0)], [0, 0],
                             [[1.0, 1.0, 2.0, 0.1, 0.2, 50.0], [90_002.0, 1.5, 2.2, -0.1, 0.2, 40.0]])
        ppl, B, use_bvh = 1 << 16, 3, False
    say("compact-node precision case", case, sc.n_tris, "triangles")
    out = run_case(torch, oracle_lib, sc, lights, lights.params, 0xC0DE, ppl, B, use_bvh=use_bvh)
    ctx, p_d = out["ctx"], out["p_d"]
    cfg = ctx.cfg(0xC0DE, ppl, B)
    g = out["g_ref"]
    n_same = n_tot = 0
    for l in range(lights.n_lights):
        prim_d, tex_d, _ = ctx.record_paths(p_d, cfg, 0, l, 0, 2048, dOdE=torch.tensor(g, device="cuda"))
        prim_r, tex_r, _ = oracle_lib.record(out["osc"], out["ol"], lights.params, 0xC0DE, ppl, B, 0, l, 0, 2048,
                                             dOdE=g)
        same = np.all(prim_d.cpu().numpy() == prim_r, 1) & np.all(tex_d.cpu().numpy() == tex_r, 1)
        n_same += int(same.sum())
        n_tot += same.size
    say(f"  identical hit sequences: {n_same}/{n_tot}")
    assert n_same / n_tot >= PATH_BAR
    assert out["S_ref"].sum() > 0


def test_invalid_arguments_raise(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd.native import LtError
    c1 = li.box_room()
    ctx = make_ctx(torch, c1["scene"], c1["lights"])
    p_d = torch.tensor(c1["lights"].params, device="cuda")
    with pytest.raises(LtError):
        ctx.trace_forward(p_d, ctx.cfg(1, 1 << 10, 0))            # max_hits 0
    with pytest.raises(LtError):
        ctx.trace_forward(p_d, ctx.cfg(1, 0, 3))                  # fewer paths than lights
    with pytest.raises(LtError):
        ctx.record_paths(p_d, ctx.cfg(1, 100, 3), 0, 0, 90, 20)   # range beyond the light's paths
    bad = c1["scene"].patches.copy()
    bad["texel_base"][1] += 1
    with pytest.raises(LtError):
        ctx.upload_scene(c1["scene"].verts, c1["scene"].tris, c1["scene"].tri_patch, bad)
    far = c1["scene"].verts.copy()
    far[0, 0] = 2e8                                            # beyond the coordinate bound
    with pytest.raises(LtError):
        ctx.upload_scene(far, c1["scene"].tris, c1["scene"].tri_patch, c1["scene"].patches)


@pytest.mark.parametrize("bad", ["negative_power", "nan_position", "inf_tilt", "zero_power"])
def test_invalid_luminaire_parameters_flagged(torch_dev, oracle_lib, bad):
    """Luminaire parameters are checked on the device by every trace call: a
    NaN or infinite parameter or a power P <= 0 raises the parameter status,
    which lt_sync reports as LT_EINVAL (once: the status is then cleared), and
    that luminaire traces nothing.  Texels equal the oracle's with that
    luminaire's power set to zero (bit-identical), the other luminaires'
    gradients match the oracle's, and its own gradient row is exactly zero."""
    torch = torch_dev
    from paper_2310_02043_amd.native import LtError, LT_EINVAL
    sc = li.box_room()["scene"]
    params = np.array([[1.0, 1.0, 2.0, 0.1, 0.2, 50.0], [3.0, 2.0, 1.8, 0, 0, 30.0],
                       [2.0, 1.5, 2.4, -0.2, 0.3, 70.0]], np.float32)
    lights = make_lights([SPOT, POINT, RECT], [3.0, 0.0, 2.0], [(0, 0), (0, 0), (0.5, 0.3)], [0, 0, 0], params)
    bad_light = {"negative_power": 1, "nan_position": 2, "inf_tilt": 0, "zero_power": 2}[bad]
    p_bad = params.copy()
    if bad == "negative_power":
        p_bad[1, 5] = -30.0
    elif bad == "nan_position":
        p_bad[2, 0] = np.nan
    elif bad == "inf_tilt":
        p_bad[0, 3] = np.inf
    else:
        p_bad[2, 5] = 0.0
    say(f"invalid luminaire: {bad} on light {bad_light}")
    ctx = make_ctx(torch, sc, lights)
    ppl, B, seed = 30_001, 3, 0x1BAD
    cfg = ctx.cfg(seed, ppl, B)
    p_d = torch.tensor(p_bad, device="cuda")
    E_d, S_d = ctx.trace_forward(p_d, cfg)
    with pytest.raises(LtError) as ei:
        ctx.sync()
    assert ei.value.code == LT_EINVAL
    assert ctx.sync() == 0
    p_ref = params.copy()
    p_ref[bad_light, 5] = 0.0
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    S_ref, _ = oracle_lib.forward(osc, ol, p_ref, seed, ppl, B)
    assert np.array_equal(S_d.cpu().numpy(), S_ref)
    assert np.isfinite(E_d.cpu().numpy()).all()
    E_ref = oracle_lib.fixed_to_float(S_ref)
    _, g_ref = oracle_lib.objective(E_ref, li.painted_target(sc, 10.0)[None], sc.texel_area())
    grad = ctx.trace_adjoint(p_d, torch.tensor(g_ref, device="cuda"), cfg).cpu().numpy()
    with pytest.raises(LtError):
        ctx.sync()
    assert np.all(grad[bad_light] == 0.0)
    grad_ref, _ = oracle_lib.adjoint(osc, ol, p_ref, seed, ppl, B, g_ref)
    ok = [l for l in range(3) if l != bad_light]
    e = grad_rel(grad[ok], grad_ref[ok])
    say(f"  other luminaires' gradients: max rel err {e:.3e}")
    assert e <= GRAD_BAR
    # the rotation-vector form: a non-finite rotation vector gives a zero row, not NaN
    p7 = np.concatenate([params[:, :3], np.zeros((3, 3), np.float32), params[:, 5:]], 1)
    p7[bad_light, 3] = np.nan
    g7 = ctx.trace_adjoint_rv(torch.tensor(p7, device="cuda"), torch.tensor(g_ref, device="cuda"), cfg).cpu().numpy()
    with pytest.raises(LtError):
        ctx.sync()
    assert np.all(g7[bad_light] == 0.0) and np.isfinite(g7).all()
    # valid parameters again: no status
    ctx.trace_forward(torch.tensor(params, device="cuda"), cfg)
    assert ctx.sync() == 0


@pytest.mark.parametrize("case", ["box_room", "plane_two_lights"])
def test_trace_stats_counts(torch_dev, oracle_lib, case):
    """The instrumented forward kernel (lt_trace_stats, the algorithmic work
    counts the roofline uses) computes the same texels as the oracle and
    counts exactly the oracle's hits and misses (segments = hits + misses),
    with node visits and triangle tests recorded."""
    torch = torch_dev
    if case == "box_room":
        c1 = li.box_room()
        sc, lights, ppl, B = c1["scene"], c1["lights"], 1 << 16, c1["max_hits"]
    else:
        sc = li.plane_scene(half=2.0, res=16)
        lights = make_lights([SPOT, POINT], [2.0, 0.0], [(0, 0), (0, 0)], [0, 0],
                             [[0.2, -0.1, 1.5, 0.2, 0.1, 20.0], [-0.5, 0.4, 1.0, 0, 0, 10.0]])
        ppl, B = 20_011, 2
    say(f"trace stats: {case}, {ppl} paths, {B} hits")
    ctx = make_ctx(torch, sc, lights)
    p_d = torch.tensor(lights.params, device="cuda")
    seed = 0x57A7
    cfg = ctx.cfg(seed, ppl, B)
    S = torch.empty((1, sc.n_texels), dtype=torch.int64, device="cuda")
    st = ctx.trace_stats(p_d, cfg, S)
    assert ctx.sync() == 0
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    S_ref, miss_ref = oracle_lib.forward(osc, ol, lights.params, seed, ppl, B)
    assert np.array_equal(S.cpu().numpy(), S_ref)
    hits = 0
    off = lights.layout_offsets
    for l in range(lights.n_lights):
        n_l = ppl // (off[1] - off[0]) + (l < ppl % (off[1] - off[0]))
        prim, _, _ = oracle_lib.record(osc, ol, lights.params, seed, ppl, B, 0, l, 0, n_l)
        hits += int((prim >= 0).sum())
    say(f"  {st}; oracle hits {hits}, misses {int(miss_ref)}")
    assert st["hits"] == hits and st["misses"] == int(miss_ref)
    assert st["segments"] == hits + int(miss_ref)
    assert st["nodes"] > 0 and st["tri_tests"] >= hits and st["wave_iters"] > 0
    assert 0 < st["active_lanes"] <= 64 * st["wave_iters"]
