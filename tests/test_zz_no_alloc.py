"""The allocation-free adjoint entry point (lt_trace_adjoint_noalloc) against
lt_trace_adjoint through the C ABI: the same gradient (the same per-path
contributions over the same work tiles; lt_trace_adjoint sums them per tile
in FP64 in a second pass, the allocation-free form per lane in FP32 first,
whose rounding, on luminaires with few paths and cancelling contributions,
reaches a few 1e-4 of a component: the gradient bar, 1e-3, applies) on two
calls in a row, the second
with a smaller input, on the box room and the 64-layout room set (1695
luminaires of uneven counts: the device-built tile table); a request too
large for its fixed scratch is refused with an error."""
import numpy as np
import pytest

import lt_inputs as li

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(torch, scene, lights):
    from paper_2310_02043_amd import Context
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    return ctx


@pytest.mark.parametrize("case", ["box_room", "room_set_64_layouts"])
def test_noalloc_adjoint_matches_adjoint(torch_dev, case):
    torch = torch_dev
    if case == "box_room":
        c = li.box_room()
        sizes = [1 << 20, 1 << 16]
    else:
        c = li.room_set()
        sizes = [1 << 14, 3001]
    sc, lights, B = c["scene"], c["lights"], c["max_hits"]
    ctx = _ctx(torch, sc, lights)
    p = torch.tensor(lights.params, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(11)
    g = torch.randn((lights.n_layouts, sc.n_texels), device="cuda", generator=gen)
    for k, ppl in enumerate(sizes):
        say(f"no-alloc adjoint: {case}, call {k + 1}, {ppl} paths per layout, {lights.n_lights} lights")
        cfg = ctx.cfg(0xA110C + k, ppl, B)
        grad_na = torch.full((lights.n_lights, 6), float("nan"), device="cuda")
        ctx.trace_adjoint_noalloc(p, g, cfg, grad_na)
        torch.cuda.synchronize()
        assert ctx.sync() == 0
        ref = ctx.trace_adjoint(p, g, cfg)
        torch.cuda.synchronize()
        a, b = grad_na.cpu().numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64)
        scale = np.maximum(np.abs(b), 1e-6 * np.abs(b).max())
        err = float(np.max(np.abs(a - b) / scale))
        say(f"  max rel diff to lt_trace_adjoint {err:.3e}")
        assert np.isfinite(a).all() and err <= 1e-3


def test_noalloc_refuses_oversized_work(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd.native import LtError
    c = li.room_set()
    sc, lights = c["scene"], c["lights"]
    ctx = _ctx(torch, sc, lights)
    ctx.set_tuning(tile_paths=64)
    p = torch.tensor(lights.params, device="cuda")
    g = torch.zeros((lights.n_layouts, sc.n_texels), device="cuda")
    grad = torch.empty((lights.n_lights, 6), device="cuda")
    with pytest.raises(LtError, match="too large"):
        ctx.trace_adjoint_noalloc(p, g, ctx.cfg(1, 1 << 22, c["max_hits"]), grad)
    with pytest.raises(LtError):
        ctx.trace_adjoint_noalloc(p, g, ctx.cfg(1, 1 << 12, c["max_hits"], graph=True), grad)
    # a fitting call on the same context still works afterwards
    ctx.trace_adjoint_noalloc(p, g, ctx.cfg(1, 1 << 12, c["max_hits"]), grad)
    assert ctx.sync() == 0
