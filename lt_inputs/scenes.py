"""Procedural scenes, luminaires and painted targets (all seeded).

Geometry model: every surface is a planar rectangle ("patch") with origin o,
orthogonal edges e_u, e_v, a texel grid of res_u x res_v cells and an albedo.
Each patch is two triangles (o, o+e_u, o+e_u+e_v) and (o, o+e_u+e_v, o+e_v).
Texels are numbered texel_base + j*res_u + i.  The per-patch float32
constants (unit normal, 1/|e_u|^2, 1/|e_v|^2, texel area and its reciprocal)
are computed here once in float64 and rounded, so that no consumer recomputes
them.

Luminaire parameters are p = (c_x, c_y, c_z, alpha, beta, P): centre, two
tilt angles and emitted power in W.  Static attributes are the type
(0 isotropic point, 1 cos^n spot, 2 cos^n rectangle), the lobe exponent n,
the rectangle size and the layout the light belongs to.
"""
from __future__ import annotations

import dataclasses
import numpy as np

PATCH_DTYPE = np.dtype([
    ("origin", "<f4", (3,)), ("e_u", "<f4", (3,)), ("e_v", "<f4", (3,)),
    ("normal", "<f4", (3,)),
    ("inv_len2_u", "<f4"), ("inv_len2_v", "<f4"),
    ("texel_area", "<f4"), ("inv_texel_area", "<f4"), ("albedo", "<f4"),
    ("res_u", "<i4"), ("res_v", "<i4"), ("pad", "<i4"),
    ("texel_base", "<i8"),
], align=True)
assert PATCH_DTYPE.itemsize == 88

LIGHT_DTYPE = np.dtype([
    ("type", "<i4"), ("lobe_n", "<f4"), ("size_w", "<f4"), ("size_h", "<f4"),
    ("layout", "<i4"),
], align=True)
assert LIGHT_DTYPE.itemsize == 20

POINT, SPOT, RECT, SOFT = 0, 1, 2, 3   # SOFT: soft-edged spot, size = (inner, outer) cone half-angle


@dataclasses.dataclass
class Scene:
    name: str
    verts: np.ndarray        # [V,3] f32
    tris: np.ndarray         # [T,3] i32
    tri_patch: np.ndarray    # [T] i32
    patches: np.ndarray      # [P] PATCH_DTYPE
    n_texels: int

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_patches(self) -> int:
        return int(self.patches.shape[0])

    def patch_floats(self) -> np.ndarray:
        """[P,17] f32: origin, e_u, e_v, normal, inv_len2_u, inv_len2_v,
        texel_area, inv_texel_area, albedo."""
        p = self.patches
        return np.ascontiguousarray(np.concatenate([
            p["origin"], p["e_u"], p["e_v"], p["normal"],
            p["inv_len2_u"][:, None], p["inv_len2_v"][:, None],
            p["texel_area"][:, None], p["inv_texel_area"][:, None],
            p["albedo"][:, None]], axis=1).astype(np.float32))

    def patch_res(self) -> np.ndarray:
        return np.ascontiguousarray(
            np.stack([self.patches["res_u"], self.patches["res_v"]], 1).astype(np.int32))

    def patch_base(self) -> np.ndarray:
        return np.ascontiguousarray(self.patches["texel_base"].astype(np.int64))

    def texel_area(self) -> np.ndarray:
        """[K] f32 area of every texel (copied from its patch)."""
        cnt = (self.patches["res_u"].astype(np.int64) * self.patches["res_v"])
        return np.repeat(self.patches["texel_area"], cnt).astype(np.float32)

    def texel_patch(self) -> np.ndarray:
        cnt = (self.patches["res_u"].astype(np.int64) * self.patches["res_v"])
        return np.repeat(np.arange(self.n_patches, dtype=np.int32), cnt)

    def bounds(self):
        return self.verts.min(0), self.verts.max(0)


@dataclasses.dataclass
class Lights:
    static: np.ndarray          # [L] LIGHT_DTYPE
    layout_offsets: np.ndarray  # [n_layouts+1] i32
    params: np.ndarray          # [L,6] f32 (c_x, c_y, c_z, alpha, beta, P)

    @property
    def n_lights(self) -> int:
        return int(self.static.shape[0])

    @property
    def n_layouts(self) -> int:
        return int(self.layout_offsets.shape[0] - 1)


def make_lights(types, lobe_n, sizes, layout_of, params) -> Lights:
    L = len(types)
    st = np.zeros(L, LIGHT_DTYPE)
    st["type"] = np.asarray(types, np.int32)
    st["lobe_n"] = np.asarray(lobe_n, np.float32)
    sz = np.asarray(sizes, np.float32).reshape(L, 2)
    st["size_w"] = sz[:, 0]
    st["size_h"] = sz[:, 1]
    lay = np.asarray(layout_of, np.int32)
    st["layout"] = lay
    assert np.all(np.diff(lay) >= 0), "lights must be grouped by layout"
    n_layouts = int(lay.max()) + 1 if L else 0
    offs = np.zeros(n_layouts + 1, np.int32)
    offs[1:] = np.cumsum(np.bincount(lay, minlength=n_layouts))
    return Lights(st, offs, np.asarray(params, np.float32).reshape(L, 6).copy())


class SceneBuilder:
    """Accumulates rectangular patches; texel resolution is assigned at the end."""

    def __init__(self):
        self.o, self.eu, self.ev, self.alb, self.res = [], [], [], [], []

    def quads(self, o, eu, ev, albedo, res=None):
        o = np.atleast_2d(np.asarray(o, np.float64))
        n = o.shape[0]
        eu = np.broadcast_to(np.asarray(eu, np.float64), (n, 3))
        ev = np.broadcast_to(np.asarray(ev, np.float64), (n, 3))
        self.o.append(o)
        self.eu.append(np.array(eu))
        self.ev.append(np.array(ev))
        self.alb.append(np.broadcast_to(np.asarray(albedo, np.float64), (n,)).copy())
        if res is None:
            self.res.append(np.full((n, 2), -1, np.int64))
        else:
            self.res.append(np.broadcast_to(np.asarray(res, np.int64), (n, 2)).copy())

    def boxes(self, lo, hi, albedo, res=None, skip_bottom=False):
        """Axis-aligned boxes [lo,hi] as 6 (or 5) outward-facing patches each."""
        lo = np.atleast_2d(np.asarray(lo, np.float64))
        hi = np.atleast_2d(np.asarray(hi, np.float64))
        n = lo.shape[0]
        alb = np.broadcast_to(np.asarray(albedo, np.float64), (n,))
        s = hi - lo
        z0 = np.zeros(n)
        X = np.stack([s[:, 0], z0, z0], 1)
        Y = np.stack([z0, s[:, 1], z0], 1)
        Z = np.stack([z0, z0, s[:, 2]], 1)
        x0, y0, z0_, x1, y1, z1 = lo[:, 0], lo[:, 1], lo[:, 2], hi[:, 0], hi[:, 1], hi[:, 2]
        faces = [
            (np.stack([x0, y0, z0_], 1), Z, Y),   # -x
            (np.stack([x1, y0, z0_], 1), Y, Z),   # +x
            (np.stack([x0, y0, z0_], 1), X, Z),   # -y
            (np.stack([x0, y1, z0_], 1), Z, X),   # +y
            (np.stack([x0, y0, z1], 1), X, Y),    # +z
        ]
        if not skip_bottom:
            faces.append((np.stack([x0, y0, z0_], 1), Y, X))  # -z
        for o, eu, ev in faces:
            self.quads(o, eu, ev, alb, res)

    def tiled_rect(self, o, eu, ev, nu, nv, albedo):
        """Rectangle o + [0,1]e_u + [0,1]e_v split into nu x nv patches."""
        o = np.asarray(o, np.float64)
        eu = np.asarray(eu, np.float64)
        ev = np.asarray(ev, np.float64)
        ii, jj = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
        oo = o + (ii.reshape(-1, 1) / nu) * eu + (jj.reshape(-1, 1) / nv) * ev
        self.quads(oo, eu / nu, ev / nv, albedo)

    def n_patches(self) -> int:
        return int(sum(a.shape[0] for a in self.o))

    def build(self, name, texel_density=None, target_texels=None, fixed_res=None) -> Scene:
        o = np.concatenate(self.o)
        eu = np.concatenate(self.eu)
        ev = np.concatenate(self.ev)
        alb = np.concatenate(self.alb)
        res = np.concatenate(self.res)
        lu = np.linalg.norm(eu, axis=1)
        lv = np.linalg.norm(ev, axis=1)
        assert np.all(np.abs(np.einsum("ij,ij->i", eu, ev)) <= 1e-9 * lu * lv + 1e-12), \
            "patch edges must be orthogonal"
        if fixed_res is not None:
            res = np.where(res < 0, np.asarray(fixed_res, np.int64), res)
        if np.any(res < 0):
            if texel_density is None:
                area = float(np.sum(lu * lv))
                texel_density = np.sqrt(area / float(target_texels))
            auto = np.stack([np.maximum(1, np.rint(lu / texel_density)),
                             np.maximum(1, np.rint(lv / texel_density))], 1).astype(np.int64)
            res = np.where(res < 0, auto, res)
        P = o.shape[0]
        nrm = np.cross(eu, ev)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        cnt = res[:, 0] * res[:, 1]
        base = np.zeros(P, np.int64)
        base[1:] = np.cumsum(cnt)[:-1]
        tarea = lu * lv / cnt
        pt = np.zeros(P, PATCH_DTYPE)
        pt["origin"] = o
        pt["e_u"] = eu
        pt["e_v"] = ev
        pt["normal"] = nrm
        pt["inv_len2_u"] = 1.0 / (lu * lu)
        pt["inv_len2_v"] = 1.0 / (lv * lv)
        pt["texel_area"] = tarea
        pt["inv_texel_area"] = 1.0 / tarea
        pt["albedo"] = alb
        pt["res_u"] = res[:, 0]
        pt["res_v"] = res[:, 1]
        pt["texel_base"] = base
        # vertices: 4 per patch, in float32
        v = np.stack([o, o + eu, o + eu + ev, o + ev], 1).reshape(-1, 3).astype(np.float32)
        q = np.arange(P, dtype=np.int64) * 4
        tris = np.concatenate([np.stack([q, q + 1, q + 2], 1),
                               np.stack([q, q + 2, q + 3], 1)], 1).reshape(-1, 3)
        tri_patch = np.repeat(np.arange(P), 2)
        return Scene(name, np.ascontiguousarray(v), tris.astype(np.int32),
                     tri_patch.astype(np.int32), pt, int(cnt.sum()))


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _place_boxes(rng, n, region_lo, region_hi, size_lo, size_hi, z_base, avoid, margin, max_tries=200):
    """Rejection-sample n non-overlapping footprints (with margin) inside a region."""
    out = []
    placed = list(avoid)
    for _ in range(n):
        for _t in range(max_tries):
            sx, sy = rng.uniform(size_lo[0], size_hi[0]), rng.uniform(size_lo[1], size_hi[1])
            x0 = rng.uniform(region_lo[0] + margin, region_hi[0] - margin - sx)
            y0 = rng.uniform(region_lo[1] + margin, region_hi[1] - margin - sy)
            fp = (x0, y0, x0 + sx, y0 + sy)
            if all(fp[2] + margin <= a[0] or a[2] + margin <= fp[0] or
                   fp[3] + margin <= a[1] or a[3] + margin <= fp[1] for a in placed):
                sz = rng.uniform(size_lo[2], size_hi[2])
                out.append(((x0, y0, z_base), (x0 + sx, y0 + sy, z_base + sz)))
                placed.append(fp)
                break
    return out


def texel_centers(scene: Scene, patch_ids=None) -> np.ndarray:
    """[K,3] f32 world-space centre of every texel (or of the given patches' texels)."""
    p = scene.patches if patch_ids is None else scene.patches[patch_ids]
    out = []
    for q in range(p.shape[0]):
        ru, rv = int(p["res_u"][q]), int(p["res_v"][q])
        i = (np.arange(ru) + 0.5) / ru
        j = (np.arange(rv) + 0.5) / rv
        jj, ii = np.meshgrid(j, i, indexing="ij")
        c = (p["origin"][q].astype(np.float64) + ii.reshape(-1, 1) * p["e_u"][q]
             + jj.reshape(-1, 1) * p["e_v"][q])
        out.append(c.astype(np.float32))
    return np.concatenate(out) if out else np.zeros((0, 3), np.float32)


def _texel_centers_fast(scene: Scene) -> np.ndarray:
    """Vectorised texel centres for large scenes (same values as texel_centers)."""
    p = scene.patches
    cnt = p["res_u"].astype(np.int64) * p["res_v"]
    pid = np.repeat(np.arange(p.shape[0]), cnt)
    local = np.arange(scene.n_texels, dtype=np.int64) - np.repeat(p["texel_base"], cnt)
    ru = p["res_u"][pid].astype(np.int64)
    i = local % ru
    j = local // ru
    fu = (i + 0.5) / ru
    fv = (j + 0.5) / p["res_v"][pid]
    c = (p["origin"][pid].astype(np.float64) + fu[:, None] * p["e_u"][pid]
         + fv[:, None] * p["e_v"][pid])
    return c.astype(np.float32)


def painted_target(scene: Scene, level: float, seed: int = 0, up_weight: float = 1.0,
                   other_weight: float = 0.25, wavelength: float = 4.0) -> np.ndarray:
    """A 'painted' target irradiance E* [K] f32 (W/m^2).

    Up-facing surfaces receive `level` modulated by a smooth seeded pattern,
    every other surface `other_weight * level`.  This stands in for the user's
    painted target on the texels.
    """
    rng = np.random.default_rng(seed)
    c = _texel_centers_fast(scene).astype(np.float64)
    nz = np.repeat(scene.patches["normal"][:, 2],
                   scene.patches["res_u"].astype(np.int64) * scene.patches["res_v"])
    ph = rng.uniform(0, 2 * np.pi, 2)
    k = 2 * np.pi / wavelength
    pattern = 0.75 + 0.25 * np.cos(k * c[:, 0] + ph[0]) * np.cos(k * c[:, 1] + ph[1])
    w = np.where(nz > 0.5, up_weight, other_weight)
    return (level * w * pattern).astype(np.float32)


def perturb_params(params: np.ndarray, seed: int, sigma_xy=0.5, tilt=0.2, power=(0.7, 1.3),
                   lo=None, hi=None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = params.astype(np.float64).copy()
    L = p.shape[0]
    p[:, 0:2] += rng.normal(0.0, sigma_xy, (L, 2))
    p[:, 3:5] += rng.uniform(-tilt, tilt, (L, 2))
    p[:, 5] *= rng.uniform(power[0], power[1], L)
    if lo is not None:
        p[:, 0:3] = np.clip(p[:, 0:3], lo, hi)
    return p.astype(np.float32)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

class _TallGeometry:
    """Footprints of the scene's triangles that reach within `reach` of the
    ceiling (walls, columns; the ceiling itself excluded), for keeping
    ceiling luminaires clear of them."""

    def __init__(self, scene: Scene, H: float, reach: float = 0.5):
        v = scene.verts[scene.tris]
        zmax, zmin = v[:, :, 2].max(1), v[:, :, 2].min(1)
        tall = (zmax >= H - reach) & (zmin < H - 1e-3)
        self.lo = v[tall][:, :, :2].min(1)
        self.hi = v[tall][:, :, :2].max(1)

    def clear(self, x: float, y: float, half: float) -> bool:
        return not np.any((self.lo[:, 0] < x + half) & (self.hi[:, 0] > x - half) &
                          (self.lo[:, 1] < y + half) & (self.hi[:, 1] > y - half))


def _clear_luminaires(rng, tall, params, jitter, half, lo, hi, fallback=None, tries=256):
    """Re-draw the (x, y) jitter of every luminaire whose square of half-width
    `half` touches tall geometry (a luminaire overlapping a column or wall
    emits from inside it); after `tries` draws it takes the fallback
    position."""
    p = params.copy()
    for k in range(p.shape[0]):
        x0, y0 = p[k, 0], p[k, 1]
        for _ in range(tries):
            if tall.clear(p[k, 0], p[k, 1], half):
                break
            p[k, 0] = np.clip(x0 + rng.uniform(-jitter[0], jitter[0]), lo[0], hi[0])
            p[k, 1] = np.clip(y0 + rng.uniform(-jitter[1], jitter[1]), lo[1], hi[1])
        else:
            if fallback is not None and not tall.clear(p[k, 0], p[k, 1], half):
                p[k, :2] = fallback[k, :2]
    return p


def box_room(seed: int = 1, res: int = 32):
    """Closed 4 x 3 x 2.5 m room (12 triangles) plus two seeded boxes (24
    triangles); every quad carries res x res texels; albedo U[0.5,0.8] per
    surface.  One cos^4 spot light of 100 W in the upper half of the room."""
    rng = np.random.default_rng(seed)
    sb = SceneBuilder()
    W, D, H = 4.0, 3.0, 2.5
    n_room = 6
    sb.boxes([0, 0, 0], [W, D, H], rng.uniform(0.5, 0.8, 1), res=(res, res))
    # two boxes on the floor: footprint 0.4-1.2 m, height 0.3-1.2 m, 0.1 m margin
    bx = _place_boxes(rng, 2, (0, 0), (W, D), (0.4, 0.4, 0.3), (1.2, 1.2, 1.2), 0.0, [], 0.1)
    assert len(bx) == 2
    for lo, hi in bx:
        sb.boxes(lo, hi, rng.uniform(0.5, 0.8, 1), res=(res, res))
    scene = sb.build("box_room", fixed_res=(res, res))
    # per-surface albedo: the room has 6 surfaces, each box 6
    alb = rng.uniform(0.5, 0.8, scene.n_patches).astype(np.float32)
    scene.patches["albedo"] = alb
    assert scene.n_patches == n_room + 12

    def spot(r):
        return [r.uniform(0.2, W - 0.2), r.uniform(0.2, D - 0.2), r.uniform(1.25, 2.45),
                r.uniform(-0.35, 0.35), r.uniform(-0.35, 0.35), 100.0]

    p_init = spot(rng)
    p_target = spot(np.random.default_rng(seed + 1000))
    lights = make_lights([SPOT], [4.0], [(0.0, 0.0)], [0], [p_init])
    return dict(scene=scene, lights=lights, params_target=np.asarray([p_target], np.float32),
                paths=1 << 20, max_hits=3, seed=0x1234 + seed, seed_target=0xBEEF + seed)


def _furnished_floor(rng, sb, W, D, H, n_cols, desk_grid, cabinets, wall_tile):
    """Shell + columns + desk clusters + cabinets; returns list of footprints used."""
    alb = lambda n=1: rng.uniform(0.3, 0.8, n)  # noqa: E731
    sb.tiled_rect([0, 0, 0], [W, 0, 0], [0, D, 0], int(W), int(D), 0.5)          # floor
    sb.tiled_rect([0, 0, H], [0, D, 0], [W, 0, 0], int(D), int(W), 0.8)          # ceiling
    nw = max(1, int(round(W / wall_tile)))
    nd = max(1, int(round(D / wall_tile)))
    sb.tiled_rect([0, 0, 0], [0, 0, H], [W, 0, 0], 1, nw, 0.7)                   # y=0 wall
    sb.tiled_rect([0, D, 0], [W, 0, 0], [0, 0, H], nw, 1, 0.7)                   # y=D wall
    sb.tiled_rect([0, 0, 0], [0, D, 0], [0, 0, H], nd, 1, 0.7)                   # x=0 wall
    sb.tiled_rect([W, 0, 0], [0, 0, H], [0, D, 0], 1, nd, 0.7)                   # x=W wall
    used = []
    # columns on a regular grid
    cx = np.linspace(0, W, n_cols[0] + 2)[1:-1]
    cy = np.linspace(0, D, n_cols[1] + 2)[1:-1]
    for x in cx:
        for y in cy:
            sb.boxes([x - 0.2, y - 0.2, 0], [x + 0.2, y + 0.2, H], alb(), skip_bottom=True)
            used.append((x - 0.5, y - 0.5, x + 0.5, y + 0.5))
    desk_tops = []
    gx, gy = desk_grid
    sx, sy = W / gx, D / gy
    for i in range(gx):
        for j in range(gy):
            x0 = i * sx + rng.uniform(0.4, 0.8)
            y0 = j * sy + rng.uniform(0.8, 1.1)
            if x0 + 3.4 > W - 0.3 or y0 + 2.4 > D - 0.3:
                continue
            fp = (x0, y0 - 0.6, x0 + 3.4, y0 + 2.4)
            if any(not (fp[2] <= a[0] or a[2] <= fp[0] or fp[3] <= a[1] or a[3] <= fp[1]) for a in used):
                continue
            used.append(fp)
            a = alb()
            # partition between the two desk rows, 1.2-1.6 m tall
            ph = rng.uniform(1.2, 1.6)
            sb.boxes([x0, y0 + 0.875, 0], [x0 + 3.4, y0 + 0.925, ph], a, skip_bottom=True)
            sb.boxes([x0 + 1.675, y0, 0], [x0 + 1.725, y0 + 1.8, ph * 0.8], a, skip_bottom=True)
            for dx in (0.0, 1.75):
                for dy, flip in ((0.0, 0), (0.95, 1)):
                    bx, by = x0 + dx, y0 + dy
                    top = [bx, by, 0.72], [bx + 1.6, by + 0.8, 0.75]
                    sb.boxes(*top, alb())
                    desk_tops.append((bx, by, bx + 1.6, by + 0.8))
                    for lx, ly in ((0.02, 0.02), (1.53, 0.02), (0.02, 0.73), (1.53, 0.73)):
                        sb.boxes([bx + lx, by + ly, 0], [bx + lx + 0.05, by + ly + 0.05, 0.72],
                                 0.3, skip_bottom=True)
                    my = by + (0.65 if flip == 0 else 0.1)
                    sb.boxes([bx + 0.5, my, 0.75], [bx + 1.05, my + 0.05, 1.1], 0.1)       # monitor
                    sb.boxes([bx + 0.72, my, 0.75], [bx + 0.83, my + 0.12, 0.78], 0.2)     # stand
                    cyc = by - 0.55 if flip == 0 else by + 0.9
                    sb.boxes([bx + 0.55, cyc, 0.42], [bx + 1.0, cyc + 0.45, 0.5], alb())   # seat
                    sb.boxes([bx + 0.55, cyc + (0.4 if flip == 0 else 0.0), 0.5],
                             [bx + 1.0, cyc + (0.45 if flip == 0 else 0.05), 1.0], alb())  # back
                    sb.boxes([bx + 0.75, cyc + 0.2, 0.0], [bx + 0.8, cyc + 0.25, 0.42], 0.2,
                             skip_bottom=True)                                               # post
    cab = []
    for _ in range(cabinets):
        side = rng.integers(4)
        w = rng.uniform(0.6, 1.2)
        if side < 2:
            x = rng.uniform(0.3, W - 0.3 - w)
            y = 0.02 if side == 0 else D - 0.47
            lo, hi = [x, y, 0], [x + w, y + 0.45, rng.uniform(1.0, 2.0)]
        else:
            y = rng.uniform(0.3, D - 0.3 - w)
            x = 0.02 if side == 2 else W - 0.47
            lo, hi = [x, y, 0], [x + 0.45, y + w, rng.uniform(1.0, 2.0)]
        sb.boxes(lo, hi, alb(), skip_bottom=True)
        cab.append((lo, hi))
    return desk_tops, cab


def _clutter(rng, sb, n, desk_tops, cabinets, W, D):
    """n small boxes: on desk tops, on cabinets and on the floor."""
    if n <= 0:
        return
    kind = rng.uniform(size=n)
    lo = np.zeros((n, 3))
    hi = np.zeros((n, 3))
    s = rng.uniform(0.04, 0.3, (n, 3))
    dt = np.asarray(desk_tops, np.float64) if desk_tops else np.zeros((1, 4))
    on_desk = kind < 0.6
    idx = rng.integers(0, dt.shape[0], n)
    u = rng.uniform(size=(n, 2))
    x = dt[idx, 0] + u[:, 0] * np.maximum(dt[idx, 2] - dt[idx, 0] - s[:, 0], 0)
    y = dt[idx, 1] + u[:, 1] * np.maximum(dt[idx, 3] - dt[idx, 1] - s[:, 1], 0)
    lo[on_desk] = np.stack([x, y, np.full(n, 0.75)], 1)[on_desk]
    floor = ~on_desk
    fx = rng.uniform(0.3, W - 0.6, n)
    fy = rng.uniform(0.3, D - 0.6, n)
    lo[floor] = np.stack([fx, fy, np.zeros(n)], 1)[floor]
    if cabinets:
        cb = rng.uniform(size=n) < 0.25
        cidx = rng.integers(0, len(cabinets), n)
        clo = np.asarray([c[0] for c in cabinets])[cidx]
        chi = np.asarray([c[1] for c in cabinets])[cidx]
        sel = floor & cb
        uu = rng.uniform(size=(n, 2))
        lo[sel] = np.stack([clo[:, 0] + uu[:, 0] * np.maximum(chi[:, 0] - clo[:, 0] - s[:, 0], 0),
                            clo[:, 1] + uu[:, 1] * np.maximum(chi[:, 1] - clo[:, 1] - s[:, 1], 0),
                            chi[:, 2]], 1)[sel]
    s[:, 2] = np.where(floor, s[:, 2] * 2.0, s[:, 2])
    hi = lo + s
    sb.boxes(lo, hi, rng.uniform(0.2, 0.85, n), skip_bottom=True)


def office(seed: int = 2, target_tris: int = 200_000, target_texels: int = 4_000_000,
           n_lights: int = 16, paths: int = 1 << 26, max_hits: int = 5):
    """30 x 20 x 3 m open-plan office: 1 m floor/ceiling tiles, columns, desk
    clusters with partitions, wall cabinets and clutter boxes up to
    target_tris; texel density sqrt(total area / target_texels); 16
    rectangular 0.6 x 0.6 m cos^n luminaires (n ~ U[1,8], P ~ U[30,60] W)
    on a jittered 4 x 4 grid 0.15 m below the ceiling (pendant fittings: a
    tilted 0.6 m emitter stays below the ceiling plane), facing down, each
    0.25 m or more from columns and walls."""
    rng = np.random.default_rng(seed)
    W, D, H = 30.0, 20.0, 3.0
    sb = SceneBuilder()
    grid = (8, 6) if target_tris >= 100_000 else (4, 3)
    desk_tops, cabs = _furnished_floor(rng, sb, W, D, H, (4, 2), grid, 40, 1.0)
    n_now = 2 * sb.n_patches()
    # clutter boxes have 5 faces = 10 triangles
    _clutter(rng, sb, max(0, (target_tris - n_now) // 10), desk_tops, cabs, W, D)
    scene = sb.build("office", target_texels=target_texels)
    g = int(round(np.sqrt(n_lights)))
    gx, gy = g, int(np.ceil(n_lights / g))
    params, lobe = [], []
    for k in range(n_lights):
        i, j = k % gx, k // gx
        x = (i + 0.5) * W / gx + rng.uniform(-1.0, 1.0)
        y = (j + 0.5) * D / gy + rng.uniform(-0.7, 0.7)
        params.append([x, y, H - 0.15, 0.0, 0.0, rng.uniform(30, 60)])
        lobe.append(rng.uniform(1.0, 8.0))
    params = np.asarray(params, np.float32)
    # ground truth and start both keep 0.25 m between a luminaire and any
    # column or wall
    tall = _TallGeometry(scene, H)
    params = _clear_luminaires(rng, tall, params, (1.0, 1.0), 0.55, (0.5, 0.5), (W - 0.5, D - 0.5))
    lights = make_lights([RECT] * n_lights, lobe, [(0.6, 0.6)] * n_lights, [0] * n_lights, params)
    init = perturb_params(params, seed + 7, lo=[0.5, 0.5, H - 0.15], hi=[W - 0.5, D - 0.5, H - 0.15])
    init = _clear_luminaires(rng, tall, init, (0.5, 0.5), 0.55, (0.5, 0.5), (W - 0.5, D - 0.5), params)
    lights.params[:] = init
    return dict(scene=scene, lights=lights, params_target=params, paths=paths,
                max_hits=max_hits, seed=0x5EED0 + seed, seed_target=0x7A46E7 + seed)


def room_set(seed: int = 3, target_tris: int = 50_000, target_texels: int = 250_000,
             n_layouts: int = 64, paths_per_layout: int = 1 << 22, max_hits: int = 4,
             min_lights: int = 4, max_lights: int = 48):
    """Four connected 6 x 5 x 3 m rooms (2 x 2, interior walls with door gaps)
    plus furniture boxes up to target_tris, traced for n_layouts candidate
    lighting layouts with U{4..48} lights each (point/spot 50/50, spot n ~
    U[1,8], P ~ U[5,40] W)."""
    rng = np.random.default_rng(seed)
    W, D, H = 12.0, 10.0, 3.0
    sb = SceneBuilder()
    sb.tiled_rect([0, 0, 0], [W, 0, 0], [0, D, 0], 12, 10, 0.5)
    sb.tiled_rect([0, 0, H], [0, D, 0], [W, 0, 0], 10, 12, 0.8)
    sb.tiled_rect([0, 0, 0], [0, 0, H], [W, 0, 0], 1, 12, 0.7)
    sb.tiled_rect([0, D, 0], [W, 0, 0], [0, 0, H], 12, 1, 0.7)
    sb.tiled_rect([0, 0, 0], [0, D, 0], [0, 0, H], 10, 1, 0.7)
    sb.tiled_rect([W, 0, 0], [0, 0, H], [0, D, 0], 1, 10, 0.7)
    # interior walls x=6 and y=5, 0.1 m thick, one 1 m door gap per half
    t = 0.05
    for (a0, a1) in ((0.0, 1.5), (2.5, 6.5), (7.5, 10.0)):
        sb.boxes([6 - t, a0, 0], [6 + t, a1, H], 0.7, skip_bottom=True)
    for (a0, a1) in ((0.0, 2.0), (3.0, 8.5), (9.5, 12.0)):
        sb.boxes([a0, 5 - t, 0], [a1, 5 + t, H], 0.7, skip_bottom=True)
    n_now = 2 * sb.n_patches()
    n_box = max(0, (target_tris - n_now) // 10)
    rooms = [(0, 0, 6, 5), (6, 0, 12, 5), (0, 5, 6, 10), (6, 5, 12, 10)]
    ridx = rng.integers(0, 4, n_box)
    r = np.asarray(rooms, np.float64)[ridx]
    s = rng.uniform(0.05, 0.5, (n_box, 3))
    s[:, 2] = rng.uniform(0.05, 1.2, n_box)
    x = r[:, 0] + 0.15 + rng.uniform(size=n_box) * (r[:, 2] - r[:, 0] - 0.3 - s[:, 0])
    y = r[:, 1] + 0.15 + rng.uniform(size=n_box) * (r[:, 3] - r[:, 1] - 0.3 - s[:, 1])
    lo = np.stack([x, y, np.zeros(n_box)], 1)
    sb.boxes(lo, lo + s, rng.uniform(0.2, 0.85, n_box), skip_bottom=True)
    scene = sb.build("room_set", target_texels=target_texels)
    types, lobes, sizes, lay, params = [], [], [], [], []
    counts = rng.integers(min_lights, max_lights + 1, n_layouts)
    for j in range(n_layouts):
        for _ in range(int(counts[j])):
            ty = SPOT if rng.uniform() < 0.5 else POINT
            rm = rooms[rng.integers(4)]
            types.append(ty)
            lobes.append(rng.uniform(1.0, 8.0) if ty == SPOT else 0.0)
            sizes.append((0.0, 0.0))
            lay.append(j)
            params.append([rng.uniform(rm[0] + 0.3, rm[2] - 0.3), rng.uniform(rm[1] + 0.3, rm[3] - 0.3),
                           rng.uniform(1.5, 2.8),
                           rng.uniform(-0.5, 0.5) if ty == SPOT else 0.0,
                           rng.uniform(-0.5, 0.5) if ty == SPOT else 0.0,
                           rng.uniform(5.0, 40.0)])
    lights = make_lights(types, lobes, sizes, lay, params)
    return dict(scene=scene, lights=lights, paths=paths_per_layout, max_hits=max_hits,
                seed=0xC0FFEE + seed, counts=counts)


def building_floor(seed: int = 5, target_tris: int = 2_000_000, target_texels: int = 16_000_000,
                   n_lights: int = 128, paths: int = 1 << 28, max_hits: int = 6):
    """80 x 60 x 3.2 m building floor: a grid of rooms along corridors (walls
    as thin boxes with door gaps), desks and clutter up to target_tris;
    128 rectangular cos^n luminaires below the ceiling."""
    rng = np.random.default_rng(seed)
    W, D, H = 80.0, 60.0, 3.2
    sb = SceneBuilder()
    desk_tops, cabs = _furnished_floor(rng, sb, W, D, H, (8, 6), (20, 16), 200, 2.0)
    t = 0.06
    # corridor walls every 10 m in x, rooms along y with door gaps
    for xw in np.arange(10.0, W, 10.0):
        for y0 in np.arange(0.0, D, 6.0):
            sb.boxes([xw - t, y0, 0], [xw + t, y0 + 4.8, H], 0.7, skip_bottom=True)
    for yw in np.arange(12.0, D, 12.0):
        for x0 in np.arange(0.0, W, 10.0):
            sb.boxes([x0 + 1.2, yw - t, 0], [x0 + 10.0, yw + t, H], 0.7, skip_bottom=True)
    n_now = 2 * sb.n_patches()
    _clutter(rng, sb, max(0, (target_tris - n_now) // 10), desk_tops, cabs, W, D)
    scene = sb.build("building_floor", target_texels=target_texels)
    gx, gy = 16, int(np.ceil(n_lights / 16))
    params, lobe = [], []
    for k in range(n_lights):
        i, j = k % gx, k // gx
        params.append([(i + 0.5) * W / gx + rng.uniform(-1, 1), (j + 0.5) * D / gy + rng.uniform(-1, 1),
                       H - 0.15, 0.0, 0.0, rng.uniform(30, 60)])
        lobe.append(rng.uniform(1.0, 8.0))
    params = np.asarray(params, np.float32)
    tall = _TallGeometry(scene, H)
    params = _clear_luminaires(rng, tall, params, (1.0, 1.0), 0.55, (0.5, 0.5), (W - 0.5, D - 0.5))
    lights = make_lights([RECT] * n_lights, lobe, [(0.6, 0.6)] * n_lights, [0] * n_lights, params)
    init = perturb_params(params, seed + 7, lo=[0.5, 0.5, H - 0.15], hi=[W - 0.5, D - 0.5, H - 0.15])
    lights.params[:] = _clear_luminaires(rng, tall, init, (0.5, 0.5), 0.55, (0.5, 0.5), (W - 0.5, D - 0.5),
                                         params)
    return dict(scene=scene, lights=lights, params_target=params, paths=paths,
                max_hits=max_hits, seed=0xF100 + seed, seed_target=0xF200 + seed)


def plane_scene(half: float = 10.0, res: int = 64, albedo: float = 0.5) -> Scene:
    """One square patch [-half,half]^2 at z=0, facing +z, res x res texels."""
    sb = SceneBuilder()
    sb.quads([-half, -half, 0.0], [2 * half, 0, 0], [0, 2 * half, 0], albedo, res=(res, res))
    return sb.build("plane", fixed_res=(res, res))


def closed_box(size=(2.0, 1.5, 1.0), res: int = 16, albedo=0.6) -> Scene:
    """A closed box room with uniform (scalar) or per-face albedo."""
    sb = SceneBuilder()
    sb.boxes([0, 0, 0], list(size), 0.6, res=(res, res))
    s = sb.build("closed_box", fixed_res=(res, res))
    s.patches["albedo"] = np.broadcast_to(np.asarray(albedo, np.float32), (s.n_patches,))
    return s


def random_scene_tiny(seed: int, n_quads: int = 24, extent: float = 2.0) -> Scene:
    """Randomly oriented small quads in a cube (for brute-force traversal checks)."""
    rng = np.random.default_rng(seed)
    sb = SceneBuilder()
    for _ in range(n_quads):
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        b = np.cross(a, rng.normal(size=3))
        b /= np.linalg.norm(b)
        o = rng.uniform(-extent, extent, 3)
        sb.quads(o, a * rng.uniform(0.2, 1.5), b * rng.uniform(0.2, 1.5), rng.uniform(0.3, 0.9),
                 res=(4, 4))
    return sb.build("tiny_%d" % seed, fixed_res=(4, 4))


def crossing_slivers(seed: int = 0x5C1, n_dirs: int = 16384, centre=(2.0, 2.0, 1.5), half: float = 1.0,
                     off: float = 0.01, width: float = 0.02, albedo: float = 0.7):
    """Narrow quads (2 half x width) in random directions whose every component
    is at least 0.2, each passing `off` beside and `off` above `centre`, so
    that every triangle's bounding box contains the centre (an adversarial
    tree for a traversal stack: a point light placed there enters every box
    at distance 0).  Returns (scene, centre)."""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n_dirs, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    u = u[np.all(np.abs(u) >= 0.2, axis=1)][: n_dirs // 2]
    u = np.concatenate([u, -u[:, [1, 2, 0]]])
    v = np.cross(u, rng.normal(size=u.shape))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    nrm = np.cross(u, v)
    c = np.asarray(centre, np.float64)
    sb = SceneBuilder()
    sb.quads(c - half * u + off * v - off * nrm, 2 * half * u, width * v, albedo, res=(2, 1))
    return sb.build("crossing_slivers", fixed_res=(2, 1)), c
