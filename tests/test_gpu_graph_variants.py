"""Graph capture of the method's variants: colour, directional texels and
rotation vectors, each forward and adjoint captured once and replayed three
times into the same buffers with eager work in between; every replay must
equal the eager result exactly (texel sums are fixed point; the adjoint's
partial sums are reduced in a fixed order)."""
import sys

import numpy as np
import pytest

import lt_inputs as li

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_variants_graph_replay(torch_dev):
    torch = torch_dev
    from scipy.spatial.transform import Rotation
    from paper_2310_02043_amd import Context
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    ctx = Context(0)
    ctx.upload_scene(sc.verts, sc.tris, sc.tri_patch, sc.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    rng = np.random.default_rng(4)
    ctx.set_albedo_rgb(rng.uniform(0.3, 0.8, (sc.n_patches, 3)).astype(np.float32))
    gl = np.stack([rng.uniform(0.0, 0.3, sc.n_patches), rng.uniform(2.0, 30.0, sc.n_patches)], 1)
    ctx.set_glossy(gl.astype(np.float32))
    L, K = lights.n_lights, sc.n_texels
    p = torch.tensor(lights.params, device="cuda")
    col = torch.tensor([[0.5, 0.3, 0.2]] * L, device="cuda")
    p6 = lights.params.astype(np.float64)
    th = np.stack([Rotation.from_euler("YX", [q[4], q[3]]).as_rotvec() for q in p6])
    p7 = torch.tensor(np.concatenate([p6[:, :3], th, p6[:, 5:6]], 1).astype(np.float32), device="cuda")
    g1 = torch.randn((1, K), device="cuda")
    g3 = torch.randn((1, 3, K), device="cuda")
    g9 = torch.randn((1, 9, K), device="cuda")
    eager, graph = ctx.cfg(0x6B, 1 << 18, 3), ctx.cfg(0x6B, 1 << 18, 3, graph=True)

    def run(cfg, out=None):
        o = out or {}
        r = {}
        r["rgb_E"], _ = ctx.trace_forward_rgb(p, col, cfg, S=o.get("rgb_S"), E=o.get("rgb_E"))
        r["rgb_g"], r["rgb_c"] = ctx.trace_adjoint_rgb(p, col, g3, cfg, grad=o.get("rgb_g"),
                                                       grad_colour=o.get("rgb_c"))
        r["dir_E"], _ = ctx.trace_forward_dir(p, cfg, 2, 3, S=o.get("dir_S"), E=o.get("dir_E"))
        r["dir_g"] = ctx.trace_adjoint_dir(p, g9, cfg, 2, 3, grad=o.get("dir_g"))
        r["rv_E"], _ = ctx.trace_forward_rv(p7, cfg, S=o.get("rv_S"), E=o.get("rv_E"))
        r["rv_g"] = ctx.trace_adjoint_rv(p7, g1, cfg, grad=o.get("rv_g"))
        return r

    ref = {k: v.clone() for k, v in run(eager).items()}
    assert ctx.sync() == 0
    out = {k: torch.empty_like(v) for k, v in ref.items()}
    out["rgb_S"] = torch.empty((1, 3, K), dtype=torch.int64, device="cuda")
    out["dir_S"] = torch.empty((1, 9, K), dtype=torch.int64, device="cuda")
    out["rv_S"] = torch.empty((1, K), dtype=torch.int64, device="cuda")
    for rep in range(3):
        got = run(graph, out)
        assert ctx.sync() == 0
        say(f"  replay {rep}")
        for k in ref:
            assert torch.equal(got[k], ref[k]), k
        ctx.trace_forward(p, eager)          # eager work between the replays
        torch.cuda.synchronize()
