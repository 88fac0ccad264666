"""CPU oracle for view-independent adjoint light tracing -- TEST INFRASTRUCTURE.

Only tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (``paper_2310_02043_amd``) never
imports, links or runs it.  The heavy lifting is plain C in ``lt_oracle.c``
(FP32 path arithmetic under the written contract, FP64 reductions, int64
fixed-point texels); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lt_oracle.c")
_LIB = os.path.join(_HERE, "liblt_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fvisibility=hidden", "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("verts", C.c_void_p), ("tris", C.c_void_p), ("tri_patch", C.c_void_p),
                ("n_tris", C.c_int64), ("pf", C.c_void_p), ("pres", C.c_void_p), ("pbase", C.c_void_p),
                ("n_patches", C.c_int32), ("n_texels", C.c_int64), ("basis", C.c_int32), ("bvh", C.c_void_p),
                ("albedo_rgb", C.c_void_p), ("glossy", C.c_void_p), ("dir_order", C.c_int32),
                ("dir_samples", C.c_int32)]


class _Proposal(C.Structure):
    _fields_ = [("pdf", C.c_void_p), ("cdf", C.c_void_p), ("alpha", C.c_float), ("inv_sigma", C.c_void_p),
                ("hist", C.c_void_p)]


class Proposal:
    """Binned emission proposal tables (pdf, cdf [L,1024] f32), plain-lobe
    probability alpha, and for the adjoint histogram inv_sigma [L,6]."""

    def __init__(self, pdf, cdf, alpha, inv_sigma=None, with_hist=False):
        self.pdf = np.ascontiguousarray(pdf, np.float32)
        self.cdf = np.ascontiguousarray(cdf, np.float32)
        L = self.pdf.shape[0]
        self.inv_sigma = np.ascontiguousarray(np.ones((L, 6)) if inv_sigma is None else inv_sigma, np.float32)
        self.hist = np.zeros((L, 1024), np.float64) if with_hist else None
        self.c = _Proposal(self.pdf.ctypes.data, self.cdf.ctypes.data, float(alpha), self.inv_sigma.ctypes.data,
                           None if self.hist is None else self.hist.ctypes.data)


def _prop(p):
    return None if p is None else C.byref(p.c)


class _Lights(C.Structure):
    _fields_ = [("type", C.c_void_p), ("lobe_n", C.c_void_p), ("size", C.c_void_p),
                ("layout_offsets", C.c_void_p), ("n_lights", C.c_int32), ("n_layouts", C.c_int32),
                ("colour", C.c_void_p), ("rotvec", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_philox.argtypes = [P, P, P]
        L.or_sincos2pi.argtypes = [C.c_float, P, P]
        L.or_log2.argtypes = [C.c_float]
        L.or_log2.restype = C.c_float
        L.or_exp2.argtypes = [C.c_float]
        L.or_exp2.restype = C.c_float
        L.or_sincos_f64.argtypes = [C.c_double, P, P]
        L.or_bvh_build.argtypes = [P, P, C.c_int64, C.c_double]
        L.or_bvh_build.restype = P
        L.or_bvh_free.argtypes = [P]
        L.or_intersect_batch.argtypes = [P, P, C.c_int64, P, P, P]
        L.or_forward.argtypes = [P, P, P, C.c_uint64, C.c_int64, C.c_int, C.c_int64, C.c_int, P, P]
        L.or_forward.restype = C.c_int64
        L.or_adjoint.argtypes = [P, P, P, C.c_uint64, C.c_int64, C.c_int, C.c_int64, C.c_int, P, P, P, P]
        L.or_adjoint.restype = C.c_int64
        L.or_votes.argtypes = [P, P, P, C.c_uint64, C.c_int64, C.c_int, C.c_int64, C.c_int, P, P, C.c_int,
                               C.c_int, P, P]
        L.or_votes.restype = C.c_int64
        L.or_pt.argtypes = [P, P, P, C.c_uint64, C.c_int, C.c_int, C.c_int, P, P, P]
        L.or_pt.restype = None
        L.or_hsh.argtypes = [C.c_int, C.c_float, C.c_float, C.c_float, P]
        L.or_hsh.restype = C.c_int
        L.or_brdf.argtypes = [C.c_float, C.c_float, C.c_float, P, P, P]
        L.or_brdf.restype = C.c_float
        L.or_tangent.argtypes = [P, P, P, C.c_uint64, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int, P]
        L.or_tangent.restype = C.c_int64
        L.or_adjoint_rv.argtypes = [P, P, P, C.c_uint64, C.c_int64, C.c_int, C.c_int, P, P]
        L.or_adjoint_rv.restype = C.c_int64
        L.or_adjoint_cone.argtypes = [P, P, P, C.c_uint64, C.c_int64, C.c_int, C.c_int, P, P, P]
        L.or_adjoint_cone.restype = C.c_int64
        L.or_first_hit_dlog_cone.argtypes = [P, P, C.c_int, P, P, P, P]
        L.or_rotvec.argtypes = [P, P, P]
        L.or_record.argtypes = [P, P, P, C.c_uint64, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int64,
                                C.c_int64, P, P, P, P, P]
        L.or_fixed_to_float.argtypes = [P, C.c_int64, P]
        L.or_objective.argtypes = [P, P, P, P, C.c_int64, C.c_int64, P]
        L.or_objective.restype = C.c_double
        L.or_light_frames.argtypes = [P, P, C.c_int64, P]
        L.or_first_hit_dlog.argtypes = [P, P, C.c_int, P, P, P, C.c_float, C.c_float, P]
        L.or_num_threads.restype = C.c_int
        L.or_dir_block.argtypes = [C.c_uint32, C.c_uint32]
        L.or_dir_block.restype = C.c_uint32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


class OracleScene:
    """Holds the scene arrays (and optionally the oracle's own BVH).  basis:
    "box" (one texel per hit) or "linear" (piecewise-linear nodes at the
    texel centres, Eq. pwLin)."""

    def __init__(self, scene, use_bvh: bool = False, basis: str = "box", albedo_rgb=None, glossy=None,
                 dir_order: int = -1, dir_samples: int = 4):
        self.scene = scene
        self.verts = np.ascontiguousarray(scene.verts, np.float32)
        self.tris = np.ascontiguousarray(scene.tris, np.int32)
        self.tri_patch = np.ascontiguousarray(scene.tri_patch, np.int32)
        self.pf = scene.patch_floats()
        self.pres = scene.patch_res()
        self.pbase = scene.patch_base()
        self.n_texels = int(scene.n_texels)
        self._bvh = None
        if use_bvh:
            lo, hi = self.verts.min(0).astype(np.float64), self.verts.max(0).astype(np.float64)
            pad = 1e-5 * (float(np.abs(np.concatenate([lo, hi])).max()) + float((hi - lo).max()) + 1.0)
            self._bvh = lib().or_bvh_build(self.verts.ctypes.data, self.tris.ctypes.data,
                                           int(self.tris.shape[0]), pad)
        self.c = _Scene(self.verts.ctypes.data, self.tris.ctypes.data, self.tri_patch.ctypes.data,
                        int(self.tris.shape[0]), self.pf.ctypes.data, self.pres.ctypes.data,
                        self.pbase.ctypes.data, int(self.pf.shape[0]), self.n_texels,
                        {"box": 0, "linear": 1}[basis], self._bvh)
        # per-patch channel albedos for the colour mode (else the scalar albedo)
        self.albedo_rgb = None if albedo_rgb is None else np.ascontiguousarray(albedo_rgb, np.float32).reshape(-1, 3)
        if self.albedo_rgb is not None:
            assert self.albedo_rgb.shape[0] == self.pf.shape[0]
            self.c.albedo_rgb = self.albedo_rgb.ctypes.data
        # directional texels (HSH order 0..3, N' local samples) and a glossy BRDF
        # (per patch: specular albedo, Phong exponent)
        self.glossy = None if glossy is None else np.ascontiguousarray(glossy, np.float32).reshape(-1, 2)
        if self.glossy is not None:
            self.c.glossy = self.glossy.ctypes.data
        assert -1 <= dir_order <= 3 and dir_samples >= 1
        self.dir_order = int(dir_order)
        self.n_coef = (dir_order + 1) ** 2 if dir_order >= 0 else 0
        self.c.dir_order = int(dir_order)
        self.c.dir_samples = int(dir_samples)

    def __del__(self):
        if self._bvh is not None and _lib is not None:
            _lib.or_bvh_free(self._bvh)
            self._bvh = None


class OracleLights:
    """Luminaire statics; with `colour` ([L,3] channel weights of the flux)
    the tracer runs in colour mode: texel arrays [n_layouts, 3, K]."""

    def __init__(self, lights, colour=None, rotvec: bool = False):
        st = lights.static
        self.type = np.ascontiguousarray(st["type"], np.int32)
        self.lobe = np.ascontiguousarray(st["lobe_n"], np.float32)
        self.size = np.ascontiguousarray(np.stack([st["size_w"], st["size_h"]], 1), np.float32)
        self.offs = np.ascontiguousarray(lights.layout_offsets, np.int32)
        self.n_lights = int(st.shape[0])
        self.n_layouts = int(self.offs.shape[0] - 1)
        self.c = _Lights(self.type.ctypes.data, self.lobe.ctypes.data, self.size.ctypes.data,
                         self.offs.ctypes.data, self.n_lights, self.n_layouts)
        self.colour = None if colour is None else np.ascontiguousarray(colour, np.float32).reshape(self.n_lights, 3)
        if self.colour is not None:
            self.c.colour = self.colour.ctypes.data
        # orientation as a rotation vector: params [L,7] = x, y, z, theta, P
        self.rotvec = bool(rotvec)
        self.c.rotvec = int(self.rotvec)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def dir_block(h: int, j: int) -> int:
    """Generator block of the directional mode's local sample j at hit h."""
    return int(lib().or_dir_block(h, j))


def sincos2pi(u):
    s, c = C.c_float(), C.c_float()
    lib().or_sincos2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def log2(x):
    return lib().or_log2(float(x))


def exp2(x):
    return lib().or_exp2(float(x))


def sincos_f64(x):
    s, c = C.c_double(), C.c_double()
    lib().or_sincos_f64(float(x), C.byref(s), C.byref(c))
    return s.value, c.value


def intersect(osc: OracleScene, rays: np.ndarray, skip=None):
    rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 6)
    n = rays.shape[0]
    t = np.zeros(n, np.float32)
    prim = np.zeros(n, np.int64)
    sk = None if skip is None else np.ascontiguousarray(skip, np.int32)
    lib().or_intersect_batch(C.byref(osc.c), rays.ctypes.data, n, _p(sk), t.ctypes.data, prim.ctypes.data)
    return t, prim


def forward(osc: OracleScene, ol: OracleLights, params, seed: int, paths_per_layout: int, max_hits: int,
            limit_per_light: int = 0, n_threads: int = 0, proposal: Proposal = None):
    """Alg. 1: returns (S [n_layouts,K] int64 ([n_layouts,3,K] in colour
    mode), misses).  Luminaires of zero power add nothing and are not traced
    (their paths count no misses)."""
    prm = np.ascontiguousarray(params, np.float32)
    shape = (ol.n_layouts, osc.n_texels) if ol.colour is None else (ol.n_layouts, 3, osc.n_texels)
    if osc.dir_order >= 0:
        shape = (ol.n_layouts, osc.n_coef, osc.n_texels)
    S = np.zeros(shape, np.int64)
    m = lib().or_forward(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                         int(paths_per_layout), int(max_hits), int(limit_per_light), int(n_threads),
                         _prop(proposal), S.ctypes.data)
    return S, int(m)


def adjoint(osc: OracleScene, ol: OracleLights, params, seed: int, paths_per_layout: int, max_hits: int,
            dOdE, limit_per_light: int = 0, n_threads: int = 0, proposal: Proposal = None):
    """Alg. 2: returns (grad [L,6] float64, misses); with a proposal holding a
    histogram, fills proposal.hist.  Grey mode only (see adjoint_rgb).
    Luminaires of zero power are not traced and get a zero row."""
    if ol.colour is not None:
        raise ValueError("colour mode: use adjoint_rgb")
    if ol.rotvec:
        raise ValueError("rotation vectors: use adjoint_rv")
    prm = np.ascontiguousarray(params, np.float32)
    per = osc.n_coef if osc.dir_order >= 0 else 1
    g = np.ascontiguousarray(dOdE, np.float32).reshape(ol.n_layouts, per * osc.n_texels)
    out = np.zeros((ol.n_lights, 6), np.float64)
    if proposal is not None and proposal.hist is not None:
        proposal.hist[:] = 0.0
    m = lib().or_adjoint(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                         int(paths_per_layout), int(max_hits), int(limit_per_light), int(n_threads),
                         _prop(proposal), g.ctypes.data, out.ctypes.data, None)
    return out, int(m)


def adjoint_rgb(osc: OracleScene, ol: OracleLights, params, seed: int, paths_per_layout: int, max_hits: int,
                dOdE, limit_per_light: int = 0, n_threads: int = 0, proposal: Proposal = None):
    """Colour mode, dOdE [n_layouts,3,K]: returns (grad [L,6], grad_colour
    [L,3] = dO/d(channel weights), misses)."""
    if ol.colour is None:
        raise ValueError("grey mode: use adjoint")
    prm = np.ascontiguousarray(params, np.float32)
    g = np.ascontiguousarray(dOdE, np.float32).reshape(ol.n_layouts, 3, osc.n_texels)
    out = np.zeros((ol.n_lights, 6), np.float64)
    outc = np.zeros((ol.n_lights, 3), np.float64)
    if proposal is not None and proposal.hist is not None:
        proposal.hist[:] = 0.0
    m = lib().or_adjoint(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                         int(paths_per_layout), int(max_hits), int(limit_per_light), int(n_threads),
                         _prop(proposal), g.ctypes.data, out.ctypes.data, outc.ctypes.data)
    return out, outc, int(m)


def votes(osc: OracleScene, ol: OracleLights, params, seed: int, paths_per_layout: int, max_hits: int,
          dOdE, light: int, param: int, limit_per_light: int = 0, n_threads: int = 0, proposal: Proposal = None):
    """Gradient-contribution map (Sec. gradVis) of global light `light` and
    parameter `param`: returns (vote [K] float64 over the texels of the
    light's layout, grad [6] float64 of that light, misses)."""
    if ol.colour is not None or ol.rotvec:
        raise ValueError("the contribution map takes grey light with tilt angles only")
    prm = np.ascontiguousarray(params, np.float32)
    g = np.ascontiguousarray(dOdE, np.float32).reshape(ol.n_layouts, osc.n_texels)
    vote = np.zeros(osc.n_texels, np.float64)
    grad = np.zeros(6, np.float64)
    if not (0 <= light < ol.n_lights and 0 <= param < 6):
        raise ValueError("light or parameter out of range")
    m = lib().or_votes(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                       int(paths_per_layout), int(max_hits), int(limit_per_light), int(n_threads),
                       _prop(proposal), g.ctypes.data, int(light), int(param), vote.ctypes.data, grad.ctypes.data)
    return vote, grad, int(m)


def path_trace(osc: OracleScene, ol: OracleLights, params, seed: int, samples_per_texel: int, max_hits: int,
               dOdE=None, n_threads: int = 0):
    """Object-space path tracing with next-event estimation: returns
    (S [n_layouts,K] int64, grad [L,6] float64 or None when dOdE is None).
    Grey only."""
    if ol.colour is not None or ol.rotvec:
        raise ValueError("the path tracer takes grey light with tilt angles only")
    prm = np.ascontiguousarray(params, np.float32)
    S = np.zeros((ol.n_layouts, osc.n_texels), np.int64)
    g = None if dOdE is None else np.ascontiguousarray(dOdE, np.float32).reshape(ol.n_layouts, osc.n_texels)
    grad = None if dOdE is None else np.zeros((ol.n_lights, 6), np.float64)
    if osc.n_texels * samples_per_texel >= 1 << 32:
        raise ValueError("more than 2^32 samples per layout")
    lib().or_pt(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                int(samples_per_texel), int(max_hits), int(n_threads), _p(g), S.ctypes.data, _p(grad))
    return S, grad


def adjoint_rv(osc: OracleScene, ol: OracleLights, params, seed: int, paths_per_layout: int, max_hits: int,
               dOdE, n_threads: int = 0):
    """Rotation-vector orientation (params [L,7] = x, y, z, theta, P):
    returns (grad [L,7] float64, misses)."""
    if not ol.rotvec:
        raise ValueError("build OracleLights with rotvec=True")
    prm = np.ascontiguousarray(params, np.float32)
    g = np.ascontiguousarray(dOdE, np.float32).reshape(ol.n_layouts, osc.n_texels)
    out = np.zeros((ol.n_lights, 7), np.float64)
    m = lib().or_adjoint_rv(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                            int(paths_per_layout), int(max_hits), int(n_threads), g.ctypes.data, out.ctypes.data)
    return out, int(m)


def tangent(osc: OracleScene, ol: OracleLights, params, seed: int, paths_per_layout: int, max_hits: int,
            light: int, param: int, n_threads: int = 0):
    """Direct-differentiation map of global light `light` and parameter
    `param`: dE_k/dp_j [K] int64 Q31.32 over the texels of its layout."""
    if ol.colour is not None or ol.rotvec or osc.dir_order >= 0:
        raise ValueError("the direct-differentiation map takes grey light, tilt angles, irradiance texels")
    if not (0 <= light < ol.n_lights and 0 <= param < 6):
        raise ValueError("light or parameter out of range")
    prm = np.ascontiguousarray(params, np.float32)
    T = np.zeros(osc.n_texels, np.int64)
    lib().or_tangent(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                     int(paths_per_layout), int(max_hits), int(n_threads), int(light), int(param), T.ctypes.data)
    return T


def rotvec(theta):
    """The oracle's rotation matrix and exponential-map Jacobian of theta."""
    th = np.ascontiguousarray(theta, np.float64)
    R = np.zeros(9)
    J = np.zeros(9)
    lib().or_rotvec(th.ctypes.data, R.ctypes.data, J.ctypes.data)
    return R.reshape(3, 3), J.reshape(3, 3)


def record(osc: OracleScene, ol: OracleLights, params, seed: int, paths_per_layout: int, max_hits: int,
           layout: int, light: int, first: int, count: int, dOdE=None, proposal: Proposal = None):
    if ol.colour is not None or ol.rotvec:
        raise ValueError("path records take grey light with tilt angles only")
    prm = np.ascontiguousarray(params, np.float32)
    prim = np.zeros((count, max_hits), np.int32)
    tex = np.zeros((count, max_hits), np.int32)
    g = None if dOdE is None else np.ascontiguousarray(dOdE, np.float32)
    contrib = None if dOdE is None else np.zeros((count, 6), np.float32)
    lib().or_record(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                    int(paths_per_layout), int(max_hits), int(layout), int(light), int(first), int(count),
                    _prop(proposal), prim.ctypes.data, tex.ctypes.data, _p(g), _p(contrib))
    return prim, tex, contrib


def hsh(order: int, ct, cp, sp):
    """The oracle's hemispherical harmonics at one direction (local frame)."""
    out = np.zeros(16, np.float32)
    n = lib().or_hsh(int(order), float(ct), float(cp), float(sp), out.ctypes.data)
    return out[:n]


def brdf(rho_d, rho_s, e, wi, wo):
    """The oracle's BRDF and its gradient w.r.t. wi (local frame)."""
    a = np.ascontiguousarray(wi, np.float32)
    b = np.ascontiguousarray(wo, np.float32)
    gr = np.zeros(3, np.float32)
    f = lib().or_brdf(float(rho_d), float(rho_s), float(e), a.ctypes.data, b.ctypes.data, gr.ctypes.data)
    return float(f), gr


def fixed_to_float(S):
    S = np.ascontiguousarray(S, np.int64)
    E = np.zeros(S.shape, np.float32)
    lib().or_fixed_to_float(S.ctypes.data, S.size, E.ctypes.data)
    return E


def objective(E, Et, A, alpha=None):
    E = np.ascontiguousarray(E, np.float32)
    Et = np.ascontiguousarray(Et, np.float32)
    A = np.ascontiguousarray(A, np.float32)
    al = None if alpha is None else np.ascontiguousarray(alpha, np.float32)
    g = np.zeros(E.shape, np.float32)
    O = lib().or_objective(E.ctypes.data, Et.ctypes.data, _p(al), A.ctypes.data, A.size, E.size, g.ctypes.data)
    return O, g


def light_frames(ol: OracleLights, params, paths_per_layout: int):
    prm = np.ascontiguousarray(params, np.float32)
    out = np.zeros((ol.n_lights, 29), np.float32)
    lib().or_light_frames(C.byref(ol.c), prm.ctypes.data, int(paths_per_layout), out.ctypes.data)
    return out


def first_hit_dlog(ol: OracleLights, params, light: int, x1, y, n1, au=0.0, av=0.0):
    """dlog of the first-hit kernel: [6] (x, y, z, alpha, beta, P), or [7]
    (x, y, z, world rotation, P) with rotation-vector orientation."""
    prm = np.ascontiguousarray(params, np.float32)
    a = [np.ascontiguousarray(v, np.float32) for v in (x1, y, n1)]
    out = np.zeros(7 if ol.rotvec else 6, np.float32)
    lib().or_first_hit_dlog(C.byref(ol.c), prm.ctypes.data, int(light), a[0].ctypes.data, a[1].ctypes.data,
                            a[2].ctypes.data, float(au), float(av), out.ctypes.data)
    return out


def first_hit_dlog_cone(ol: OracleLights, params, light: int, x1, y, n1):
    """dlog of the first-hit kernel with the cone angles: [8] (x, y, z, alpha,
    beta, P, theta_in, theta_out); the last two are 0 unless soft-edged spot."""
    prm = np.ascontiguousarray(params, np.float32)
    a = [np.ascontiguousarray(v, np.float32) for v in (x1, y, n1)]
    out = np.zeros(8, np.float32)
    lib().or_first_hit_dlog_cone(C.byref(ol.c), prm.ctypes.data, int(light), a[0].ctypes.data, a[1].ctypes.data,
                                 a[2].ctypes.data, out.ctypes.data)
    return out


def adjoint_cone(osc: OracleScene, ol: OracleLights, params, seed: int, paths_per_layout: int, max_hits: int,
                 dOdE, n_threads: int = 0):
    """Adjoint with the soft-edged spots' cone angles: (grad [L,6],
    grad_cone [L,2] = dO/d(theta_in, theta_out), misses)."""
    if ol.colour is not None or ol.rotvec or osc.dir_order >= 0 or osc.c.basis != 0:
        raise ValueError("cone-angle gradients take grey light, tilt angles, box irradiance texels")
    prm = np.ascontiguousarray(params, np.float32)
    g = np.ascontiguousarray(dOdE, np.float32)
    grad = np.zeros((ol.n_lights, 6))
    gc = np.zeros((ol.n_lights, 2))
    m = lib().or_adjoint_cone(C.byref(osc.c), C.byref(ol.c), prm.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF,
                              int(paths_per_layout), int(max_hits), int(n_threads), g.ctypes.data,
                              grad.ctypes.data, gc.ctypes.data)
    return grad, gc, m


def num_threads() -> int:
    return int(lib().or_num_threads())
