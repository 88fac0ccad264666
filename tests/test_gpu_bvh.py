"""The compact 4-wide BVH as built on the device, read back through the C ABI
and checked in float64: every slot's stored box (bf16 origin + f16 offsets,
rounded outward) contains the triangles beneath it with at least half the
build's padding to spare, every triangle is the leaf of exactly one slot and
every node but the root the child of exactly one slot.  (The traversal's
hits rely on this containment; the parity tests compare the hits
themselves.)"""
import numpy as np
import pytest

import lt_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def decode(nodes):
    """[n, 64] u8 -> slot boxes lo, hi [n, 4, 3] f64, internal / leaf counts,
    first child, first triangle."""
    half = nodes.view(np.uint16).reshape(-1, 32)
    f16 = nodes.view(np.float16).reshape(-1, 32).astype(np.float64)
    words = nodes.view(np.uint32).reshape(-1, 16)
    lo = np.stack([f16[:, 0:4], f16[:, 8:12], f16[:, 16:20]], 2)
    hi = np.stack([f16[:, 4:8], f16[:, 12:16], f16[:, 20:24]], 2)
    origin = (half[:, 24:27].astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    counts = half[:, 27].astype(np.int64)
    ni, nl = counts & 15, (counts >> 4) & 15
    return (origin[:, None, :] + lo, origin[:, None, :] + hi, ni, nl, words[:, 14].astype(np.int64),
            words[:, 15].astype(np.int64))


def check_bvh(scene, nodes, tris):
    n = nodes.shape[0]
    lo, hi, ni, nl, first_child, first_tri = decode(nodes)
    v = scene.verts.astype(np.float64)
    amax = float(np.abs(v).max())
    ext = float((v.max(0) - v.min(0)).max())
    pad = 1e-5 * (amax + ext + 1.0)
    # triangles from their stored rows: v0, v0 + e1, v0 + e2
    rows = tris.reshape(-1, 3, 4).astype(np.float64)
    t0 = rows[:, 0, :3]
    tlo = np.minimum(np.minimum(t0, t0 + rows[:, 1, :3]), t0 + rows[:, 2, :3])
    thi = np.maximum(np.maximum(t0, t0 + rows[:, 1, :3]), t0 + rows[:, 2, :3])
    ids = tris.view(np.int32).reshape(-1, 3, 4)[:, 0, 3]
    assert np.all((ni + nl >= 1) & (ni + nl <= 4))
    slot = np.arange(4)[None, :]
    used = slot < (ni + nl)[:, None]
    assert np.all(lo[~used] == np.inf) and np.all(hi[~used] == -np.inf)
    child_refs = np.zeros(n, np.int64)
    tri_refs = np.zeros(rows.shape[0], np.int64)
    sub_lo = np.full((n, 3), np.inf)
    sub_hi = np.full((n, 3), -np.inf)
    worst = np.inf
    # children have larger indices than their parent (level order): reverse sweep
    for i in range(n - 1, -1, -1):
        for k in range(int(ni[i] + nl[i])):
            if k < ni[i]:
                c = int(first_child[i] + k)
                assert i < c < n
                child_refs[c] += 1
                blo, bhi = sub_lo[c], sub_hi[c]
            else:
                t = int(first_tri[i] + k - ni[i])
                assert 0 <= t < rows.shape[0]
                tri_refs[t] += 1
                blo, bhi = tlo[t], thi[t]
            margin = min(float(np.min(blo - lo[i, k])), float(np.min(hi[i, k] - bhi)))
            worst = min(worst, margin)
            sub_lo[i] = np.minimum(sub_lo[i], blo)
            sub_hi[i] = np.maximum(sub_hi[i], bhi)
    assert child_refs[0] == 0 and np.all(child_refs[1:] == 1)
    if scene.n_tris > 1:
        assert np.all(tri_refs == 1)
        assert sorted(ids.tolist()) == list(range(scene.n_tris))
    print(f"  {n} nodes, {rows.shape[0]} leaf triangles; least containment margin {worst:.3e} "
          f"(padding {pad:.3e})", flush=True)
    assert worst >= 0.5 * pad


def _translated(scene, off):
    import dataclasses
    patches = scene.patches.copy()
    patches["origin"] = (patches["origin"].astype(np.float64) + off).astype(np.float32)
    return dataclasses.replace(scene, verts=(scene.verts.astype(np.float64) + off).astype(np.float32),
                               patches=patches)


@pytest.mark.parametrize("case", ["box_room", "office", "office_far_from_origin", "single_quad"])
def test_bvh_boxes_contain_their_triangles(torch_dev, case):
    from paper_2310_02043_amd import Context
    if case == "box_room":
        sc = li.box_room()["scene"]
    elif case == "office":
        sc = li.office()["scene"]
    elif case == "office_far_from_origin":
        sc = _translated(li.office(target_tris=20_000, target_texels=200_000, n_lights=4)["scene"],
                         np.array([4096.3, -2048.7, 517.1]))
    else:
        sb = li.SceneBuilder()
        sb.quads([-1.0, -1.0, 0.0], [2.0, 0, 0], [0, 2.0, 0], 0.5, res=(3, 5))
        sc = sb.build("one_quad", fixed_res=(3, 5))
    print("BVH check", case, sc.n_tris, "triangles", flush=True)
    ctx = Context(0)
    ctx.upload_scene(sc.verts, sc.tris, sc.tri_patch, sc.patches)
    nodes, tris = ctx.bvh()
    check_bvh(sc, nodes, tris)
