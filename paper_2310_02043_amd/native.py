"""ctypes binding of liblt.so (argument marshalling only).

Every step of the light-tracing path runs in the HIP kernels of liblt.so.
This module loads the in-tree library (raising if it has not been built),
passes device pointers of torch tensors and the current torch stream, and
turns error codes into exceptions.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblt.so")

LT_OK, LT_EINVAL, LT_ENOMEM, LT_EHIP, LT_ESTATE, LT_EOVERFLOW = 0, -1, -2, -3, -4, -5
LT_FLAG_GRAPH, LT_FLAG_PROPOSAL, LT_FLAG_LINEAR = 1, 2, 4

EXPORTED = [
    "lt_create", "lt_destroy", "lt_last_error", "lt_set_stream", "lt_sync", "lt_scene_upload",
    "lt_set_lights", "lt_trace_forward", "lt_objective", "lt_trace_adjoint", "lt_gradient_votes",
    "lt_pt_forward", "lt_pt_adjoint", "lt_set_albedo_rgb", "lt_trace_forward_rgb", "lt_trace_adjoint_rgb",
    "lt_set_glossy", "lt_trace_forward_dir", "lt_trace_adjoint_dir", "lt_trace_forward_rv", "lt_trace_adjoint_rv",
    "lt_trace_tangent", "lt_fd_map", "lt_trace_adjoint_cone",
    "lt_record_paths",
    "lt_trace_stats", "lt_get_tuning", "lt_set_tuning", "lt_autotune", "lt_info_get", "lt_set_timing",
    "lt_timing_read", "lt_proposal_set_table", "lt_proposal_get_table", "lt_proposal_set_scale",
    "lt_proposal_mlp_infer",
    "lt_proposal_mlp_train", "lt_proposal_set", "lt_proposal_refresh", "lt_proposal_update_scale",
    "lt_proposal_train_step", "lt_proposal_get_net", "lt_trace_adjoint_noalloc", "lt_bvh_copy",
]
MLP_WEIGHTS, MLP_IN, MLP_BINS = 72832, 32, 1024

PATCH_ITEMSIZE = 88
LIGHT_ITEMSIZE = 20


class LtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblt error {code}: {msg}")
        self.code = code


class TraceCfg(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("paths_per_layout", C.c_int64), ("max_hits", C.c_int32),
                ("flags", C.c_uint32), ("alpha_plain", C.c_float), ("reserved", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("xcd_remap", C.c_int32), ("tile_paths", C.c_int32),
                ("refill_threshold", C.c_int32), ("lds_depth", C.c_int32), ("tri_share", C.c_int32),
                ("reserved", C.c_int32 * 2)]

    def as_dict(self):
        return {k: getattr(self, k) for k in ("waves_per_block", "xcd_remap", "tile_paths",
                                               "refill_threshold", "lds_depth", "tri_share")}


class ProposalCfg(C.Structure):
    _fields_ = [("param_lo", C.c_float * 6), ("param_hi", C.c_float * 6), ("hist_decay", C.c_float),
                ("plain_floor", C.c_float), ("sigma_decay", C.c_float), ("reserved", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n_tris", C.c_int64), ("n_patches", C.c_int64), ("n_texels", C.c_int64),
                ("bvh_nodes", C.c_int32), ("bvh_depth", C.c_int32), ("device_bytes", C.c_int64),
                ("n_lights", C.c_int32), ("n_layouts", C.c_int32)]


_lib = None


def load():
    """Load liblt.so; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: the HIP library must be built before use")
    L = C.CDLL(LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    L.lt_create.argtypes = [C.c_int, P, C.POINTER(P)]
    L.lt_destroy.argtypes = [P]
    L.lt_destroy.restype = None
    L.lt_last_error.argtypes = [P]
    L.lt_last_error.restype = C.c_char_p
    L.lt_set_stream.argtypes = [P, P]
    L.lt_sync.argtypes = [P, C.POINTER(C.c_uint32)]
    L.lt_scene_upload.argtypes = [P, P, I64, P, P, I64, P, I32, C.POINTER(I64)]
    L.lt_set_lights.argtypes = [P, P, I32, P, I32]
    L.lt_trace_forward.argtypes = [P, C.POINTER(TraceCfg), P, P, P]
    L.lt_objective.argtypes = [P, P, P, P, I64, P, P]
    L.lt_trace_adjoint.argtypes = [P, C.POINTER(TraceCfg), P, P, P, P]
    L.lt_trace_adjoint_noalloc.argtypes = [P, C.POINTER(TraceCfg), P, P, P]
    L.lt_gradient_votes.argtypes = [P, C.POINTER(TraceCfg), P, P, I32, I32, P, P]
    L.lt_pt_forward.argtypes = [P, C.POINTER(TraceCfg), P, I32, P, P]
    L.lt_set_albedo_rgb.argtypes = [P, P]
    L.lt_set_glossy.argtypes = [P, P]
    L.lt_trace_forward_rv.argtypes = [P, C.POINTER(TraceCfg), P, P, P]
    L.lt_trace_tangent.argtypes = [P, C.POINTER(TraceCfg), P, I32, I32, P, P]
    L.lt_fd_map.argtypes = [P, C.POINTER(TraceCfg), P, I32, I32, C.c_float, P, P, P]
    L.lt_trace_adjoint_cone.argtypes = [P, C.POINTER(TraceCfg), P, P, P, P]
    L.lt_trace_adjoint_rv.argtypes = [P, C.POINTER(TraceCfg), P, P, P]
    L.lt_trace_forward_dir.argtypes = [P, C.POINTER(TraceCfg), P, I32, I32, P, P]
    L.lt_trace_adjoint_dir.argtypes = [P, C.POINTER(TraceCfg), P, I32, I32, P, P, P]
    L.lt_trace_forward_rgb.argtypes = [P, C.POINTER(TraceCfg), P, P, P, P]
    L.lt_trace_adjoint_rgb.argtypes = [P, C.POINTER(TraceCfg), P, P, P, P, P, P]
    L.lt_pt_adjoint.argtypes = [P, C.POINTER(TraceCfg), P, I32, P, P]
    L.lt_record_paths.argtypes = [P, C.POINTER(TraceCfg), P, I32, I32, I64, I64, P, P, P, P]
    L.lt_trace_stats.argtypes = [P, C.POINTER(TraceCfg), P, P, C.POINTER(I64)]
    L.lt_get_tuning.argtypes = [P, C.POINTER(Tuning)]
    L.lt_set_tuning.argtypes = [P, C.POINTER(Tuning)]
    L.lt_autotune.argtypes = [P, C.POINTER(TraceCfg), P, P, P, P, P, C.c_char_p, C.POINTER(C.c_float)]
    L.lt_info_get.argtypes = [P, C.POINTER(Info)]
    L.lt_bvh_copy.argtypes = [P, P, I64, P, I64]
    L.lt_set_timing.argtypes = [P, C.c_int]
    L.lt_proposal_set_table.argtypes = [P, P, P]
    L.lt_proposal_set_scale.argtypes = [P, P]
    L.lt_proposal_get_table.argtypes = [P, P, P]
    L.lt_proposal_mlp_infer.argtypes = [P, P, P, P]
    L.lt_proposal_mlp_train.argtypes = [P, P, P, P, P, P, P, P, P, I32, C.c_float, P, P]
    L.lt_proposal_set.argtypes = [P, P, P, C.POINTER(ProposalCfg)]
    L.lt_proposal_refresh.argtypes = [P, P]
    L.lt_proposal_update_scale.argtypes = [P, P, P]
    L.lt_proposal_train_step.argtypes = [P, P, C.c_float, I32, P, P]
    L.lt_proposal_get_net.argtypes = [P, P, P]
    L.lt_timing_read.argtypes = [P, C.POINTER(C.c_double), C.POINTER(I32), C.POINTER(C.c_double), C.POINTER(I32)]
    for name in EXPORTED:
        if name not in ("lt_destroy", "lt_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """One liblt context on a torch CUDA (HIP) device."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.lt_create(device, C.c_void_p(torch.cuda.current_stream(device).cuda_stream), C.byref(h))
        if rc != LT_OK:
            raise LtError(rc, "lt_create failed")
        self.h = h
        self.n_texels = 0
        self.n_lights = 0
        self.n_layouts = 0
        self.layout_offsets = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.lt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != LT_OK:
            raise LtError(rc, self.lib.lt_last_error(self.h).decode())

    def _stream(self):
        self._check(self.lib.lt_set_stream(
            self.h, C.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)))

    # -- scene / lights ------------------------------------------------------
    def upload_scene(self, verts, tris, tri_patch, patches) -> int:
        v = np.ascontiguousarray(verts, np.float32)
        t = np.ascontiguousarray(tris, np.int32)
        tp = np.ascontiguousarray(tri_patch, np.int32)
        p = np.ascontiguousarray(patches)
        assert p.dtype.itemsize == PATCH_ITEMSIZE, "patch records must be 88-byte lt_patch structs"
        K = C.c_int64()
        self._stream()
        self._check(self.lib.lt_scene_upload(self.h, v.ctypes.data, v.shape[0], t.ctypes.data, tp.ctypes.data,
                                             t.shape[0], p.ctypes.data, p.shape[0], C.byref(K)))
        self.n_texels = int(K.value)
        return self.n_texels

    def set_lights(self, static, layout_offsets):
        s = np.ascontiguousarray(static)
        assert s.dtype.itemsize == LIGHT_ITEMSIZE
        o = np.ascontiguousarray(layout_offsets, np.int32)
        self._stream()
        self._check(self.lib.lt_set_lights(self.h, s.ctypes.data, s.shape[0], o.ctypes.data, o.shape[0] - 1))
        self.n_lights = int(s.shape[0])
        self.n_layouts = int(o.shape[0] - 1)
        self.layout_offsets = o.copy()

    # -- tracing -------------------------------------------------------------
    @staticmethod
    def cfg(seed, paths_per_layout, max_hits, graph=False, proposal=False, alpha_plain=0.2, linear=False):
        flags = (LT_FLAG_GRAPH if graph else 0) | (LT_FLAG_PROPOSAL if proposal else 0) | \
            (LT_FLAG_LINEAR if linear else 0)
        return TraceCfg(int(seed) & 0xFFFFFFFFFFFFFFFF, int(paths_per_layout), int(max_hits), flags,
                        float(alpha_plain), 0)

    def _dev(self, t, dtype, shape):
        torch = self._torch
        assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
        assert tuple(t.shape) == tuple(shape), (tuple(t.shape), shape)
        return t

    def trace_forward(self, params, cfg, S=None, E=None):
        torch = self._torch
        dev = params.device
        n = (self.n_layouts, self.n_texels)
        self._dev(params, torch.float32, (self.n_lights, 6))
        if S is None:
            S = torch.empty(n, dtype=torch.int64, device=dev)
        if E is None:
            E = torch.empty(n, dtype=torch.float32, device=dev)
        self._dev(S, torch.int64, n)
        self._dev(E, torch.float32, n)
        self._stream()
        self._check(self.lib.lt_trace_forward(self.h, C.byref(cfg), _ptr(params), _ptr(S), _ptr(E)))
        return E, S

    def objective(self, E, Et, alpha=None, g=None, O=None):
        torch = self._torch
        n = E.numel()
        self._dev(E, torch.float32, E.shape)
        self._dev(Et, torch.float32, E.shape)
        if alpha is not None:
            self._dev(alpha, torch.float32, E.shape)
        if g is None:
            g = torch.empty_like(E)
        if O is None:
            O = torch.empty(1, dtype=torch.float64, device=E.device)
        self._stream()
        self._check(self.lib.lt_objective(self.h, _ptr(E), _ptr(Et), _ptr(alpha), n, _ptr(O), _ptr(g)))
        return O, g

    def trace_adjoint(self, params, dOdE, cfg, grad=None, bin_hist=None):
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        self._dev(dOdE, torch.float32, (self.n_layouts, self.n_texels))
        if grad is None:
            grad = torch.empty((self.n_lights, 6), dtype=torch.float32, device=params.device)
        self._dev(grad, torch.float32, (self.n_lights, 6))
        self._stream()
        self._check(self.lib.lt_trace_adjoint(self.h, C.byref(cfg), _ptr(params), _ptr(dOdE), _ptr(grad),
                                              _ptr(bin_hist)))
        return grad

    def trace_adjoint_noalloc(self, params, dOdE, cfg, grad):
        """lt_trace_adjoint_noalloc: the adjoint pass with no device allocation
        (grad [L,6] f32 must be given)."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        self._dev(dOdE, torch.float32, (self.n_layouts, self.n_texels))
        self._dev(grad, torch.float32, (self.n_lights, 6))
        self._stream()
        self._check(self.lib.lt_trace_adjoint_noalloc(self.h, C.byref(cfg), _ptr(params), _ptr(dOdE), _ptr(grad)))
        return grad

    def gradient_votes(self, params, dOdE, cfg, light, param, vote=None, grad=None):
        """Gradient-contribution map of global light `light` and parameter
        `param` (0..5): returns (vote [K] float64, grad [L,6] float32)."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        self._dev(dOdE, torch.float32, (self.n_layouts, self.n_texels))
        if vote is None:
            vote = torch.empty(self.n_texels, dtype=torch.float64, device=params.device)
        self._dev(vote, torch.float64, (self.n_texels,))
        if grad is None:
            grad = torch.empty((self.n_lights, 6), dtype=torch.float32, device=params.device)
        self._dev(grad, torch.float32, (self.n_lights, 6))
        self._stream()
        self._check(self.lib.lt_gradient_votes(self.h, C.byref(cfg), _ptr(params), _ptr(dOdE), int(light),
                                               int(param), _ptr(vote), _ptr(grad)))
        return vote, grad

    def set_albedo_rgb(self, albedo):
        """Per-patch channel albedos [n_patches,3] for the colour mode (host)."""
        import numpy as np
        a = np.ascontiguousarray(albedo, np.float32)
        self._check(self.lib.lt_set_albedo_rgb(self.h, a.ctypes.data))

    def trace_forward_rgb(self, params, colour, cfg, S=None, E=None):
        """Colour mode: channel weights colour [L,3]; returns (E, S) with
        texels [n_layouts,3,K]."""
        torch = self._torch
        n = (self.n_layouts, 3, self.n_texels)
        self._dev(params, torch.float32, (self.n_lights, 6))
        self._dev(colour, torch.float32, (self.n_lights, 3))
        if S is None:
            S = torch.empty(n, dtype=torch.int64, device=params.device)
        if E is None:
            E = torch.empty(n, dtype=torch.float32, device=params.device)
        self._dev(S, torch.int64, n)
        self._dev(E, torch.float32, n)
        self._stream()
        self._check(self.lib.lt_trace_forward_rgb(self.h, C.byref(cfg), _ptr(params), _ptr(colour), _ptr(S),
                                                  _ptr(E)))
        return E, S

    def trace_adjoint_rgb(self, params, colour, dOdE, cfg, grad=None, grad_colour=None, bin_hist=None):
        """Colour mode adjoint: returns (grad [L,6], grad_colour [L,3])."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        self._dev(colour, torch.float32, (self.n_lights, 3))
        self._dev(dOdE, torch.float32, (self.n_layouts, 3, self.n_texels))
        if grad is None:
            grad = torch.empty((self.n_lights, 6), dtype=torch.float32, device=params.device)
        if grad_colour is None:
            grad_colour = torch.empty((self.n_lights, 3), dtype=torch.float32, device=params.device)
        self._stream()
        self._check(self.lib.lt_trace_adjoint_rgb(self.h, C.byref(cfg), _ptr(params), _ptr(colour), _ptr(dOdE),
                                                  _ptr(grad), _ptr(grad_colour), _ptr(bin_hist)))
        return grad, grad_colour

    def trace_tangent(self, params, cfg, light, param, D=None, T=None):
        """Direct-differentiation map dE/dp_j of global light `light` over the
        texels of its layout: ([K] float32, [K] int64 Q31.32 sums)."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        if T is None:
            T = torch.empty(self.n_texels, dtype=torch.int64, device=params.device)
        if D is None:
            D = torch.empty(self.n_texels, dtype=torch.float32, device=params.device)
        self._dev(T, torch.int64, (self.n_texels,))
        self._dev(D, torch.float32, (self.n_texels,))
        self._stream()
        self._check(self.lib.lt_trace_tangent(self.h, C.byref(cfg), _ptr(params), int(light), int(param), _ptr(T),
                                              _ptr(D)))
        return D, T

    def trace_adjoint_cone(self, params, dOdE, cfg, grad=None, gcone=None):
        """Adjoint with the soft-edged spots' cone angles: (grad [L,6],
        grad_cone [L,2] = dO/d(theta_in, theta_out))."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        self._dev(dOdE, torch.float32, (self.n_layouts, self.n_texels))
        if grad is None:
            grad = torch.empty((self.n_lights, 6), dtype=torch.float32, device=params.device)
        if gcone is None:
            gcone = torch.empty((self.n_lights, 2), dtype=torch.float32, device=params.device)
        self._dev(grad, torch.float32, (self.n_lights, 6))
        self._dev(gcone, torch.float32, (self.n_lights, 2))
        self._stream()
        self._check(self.lib.lt_trace_adjoint_cone(self.h, C.byref(cfg), _ptr(params), _ptr(dOdE), _ptr(grad),
                                                   _ptr(gcone)))
        return grad, gcone

    def fd_map(self, params, cfg, light, param, h, F=None, Sp=None, Sm=None):
        """Central-difference map (E(p_j + h) - E(p_j - h)) / step of global
        light `light` over the texels of its layout, common random numbers:
        [K] float32."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        n = (self.n_layouts, self.n_texels)
        if Sp is None:
            Sp = torch.empty(n, dtype=torch.int64, device=params.device)
        if Sm is None:
            Sm = torch.empty(n, dtype=torch.int64, device=params.device)
        if F is None:
            F = torch.empty(self.n_texels, dtype=torch.float32, device=params.device)
        self._dev(Sp, torch.int64, n)
        self._dev(Sm, torch.int64, n)
        self._dev(F, torch.float32, (self.n_texels,))
        self._stream()
        self._check(self.lib.lt_fd_map(self.h, C.byref(cfg), _ptr(params), int(light), int(param), float(h), _ptr(Sp),
                                       _ptr(Sm), _ptr(F)))
        return F

    def trace_forward_rv(self, params, cfg, S=None, E=None):
        """Rotation-vector orientation, params [L,7] = (x, y, z, theta, P): (E, S)."""
        torch = self._torch
        n = (self.n_layouts, self.n_texels)
        self._dev(params, torch.float32, (self.n_lights, 7))
        if S is None:
            S = torch.empty(n, dtype=torch.int64, device=params.device)
        if E is None:
            E = torch.empty(n, dtype=torch.float32, device=params.device)
        self._dev(S, torch.int64, n)
        self._dev(E, torch.float32, n)
        self._stream()
        self._check(self.lib.lt_trace_forward_rv(self.h, C.byref(cfg), _ptr(params), _ptr(S), _ptr(E)))
        return E, S

    def trace_adjoint_rv(self, params, dOdE, cfg, grad=None):
        """Rotation-vector adjoint: dO/d(x, y, z, theta, P) [L,7]."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 7))
        self._dev(dOdE, torch.float32, (self.n_layouts, self.n_texels))
        if grad is None:
            grad = torch.empty((self.n_lights, 7), dtype=torch.float32, device=params.device)
        self._dev(grad, torch.float32, (self.n_lights, 7))
        self._stream()
        self._check(self.lib.lt_trace_adjoint_rv(self.h, C.byref(cfg), _ptr(params), _ptr(dOdE), _ptr(grad)))
        return grad

    def set_glossy(self, glossy):
        """Per-patch (specular albedo, Phong exponent) [n_patches,2] for the
        directional texels (host)."""
        import numpy as np
        a = np.ascontiguousarray(glossy, np.float32)
        self._check(self.lib.lt_set_glossy(self.h, a.ctypes.data))

    def trace_forward_dir(self, params, cfg, order, samples, S=None, E=None):
        """Directional texels: returns (L, S), [n_layouts, (order+1)^2, K]
        hemispherical-harmonic coefficients of the reflected radiance."""
        torch = self._torch
        n = (self.n_layouts, (order + 1) ** 2, self.n_texels)
        self._dev(params, torch.float32, (self.n_lights, 6))
        if S is None:
            S = torch.empty(n, dtype=torch.int64, device=params.device)
        if E is None:
            E = torch.empty(n, dtype=torch.float32, device=params.device)
        self._dev(S, torch.int64, n)
        self._dev(E, torch.float32, n)
        self._stream()
        self._check(self.lib.lt_trace_forward_dir(self.h, C.byref(cfg), _ptr(params), int(order), int(samples),
                                                  _ptr(S), _ptr(E)))
        return E, S

    def trace_adjoint_dir(self, params, dOdE, cfg, order, samples, grad=None, bin_hist=None):
        """Directional adjoint: dOdE [n_layouts, (order+1)^2, K] -> grad [L,6]."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        self._dev(dOdE, torch.float32, (self.n_layouts, (order + 1) ** 2, self.n_texels))
        if grad is None:
            grad = torch.empty((self.n_lights, 6), dtype=torch.float32, device=params.device)
        self._stream()
        self._check(self.lib.lt_trace_adjoint_dir(self.h, C.byref(cfg), _ptr(params), int(order), int(samples),
                                                  _ptr(dOdE), _ptr(grad), _ptr(bin_hist)))
        return grad

    def pt_forward(self, params, cfg, samples_per_texel, S=None, E=None):
        """Object-space path tracing with next-event estimation: (E, S)."""
        torch = self._torch
        n = (self.n_layouts, self.n_texels)
        self._dev(params, torch.float32, (self.n_lights, 6))
        if S is None:
            S = torch.empty(n, dtype=torch.int64, device=params.device)
        if E is None:
            E = torch.empty(n, dtype=torch.float32, device=params.device)
        self._dev(S, torch.int64, n)
        self._dev(E, torch.float32, n)
        self._stream()
        self._check(self.lib.lt_pt_forward(self.h, C.byref(cfg), _ptr(params), int(samples_per_texel), _ptr(S),
                                           _ptr(E)))
        return E, S

    def pt_adjoint(self, params, dOdE, cfg, samples_per_texel, grad=None):
        """Gradient of sum_k dOdE_k E_k for the path tracer: [L,6]."""
        torch = self._torch
        self._dev(params, torch.float32, (self.n_lights, 6))
        self._dev(dOdE, torch.float32, (self.n_layouts, self.n_texels))
        if grad is None:
            grad = torch.empty((self.n_lights, 6), dtype=torch.float32, device=params.device)
        self._dev(grad, torch.float32, (self.n_lights, 6))
        self._stream()
        self._check(self.lib.lt_pt_adjoint(self.h, C.byref(cfg), _ptr(params), int(samples_per_texel), _ptr(dOdE),
                                           _ptr(grad)))
        return grad

    def record_paths(self, params, cfg, layout, light, first, count, dOdE=None):
        torch = self._torch
        dev = params.device
        prim = torch.empty((count, cfg.max_hits), dtype=torch.int32, device=dev)
        tex = torch.empty((count, cfg.max_hits), dtype=torch.int32, device=dev)
        contrib = None
        if dOdE is not None:
            self._dev(dOdE, torch.float32, (self.n_layouts, self.n_texels))
            contrib = torch.empty((count, 6), dtype=torch.float32, device=dev)
        self._stream()
        self._check(self.lib.lt_record_paths(self.h, C.byref(cfg), _ptr(params), int(layout), int(light),
                                             int(first), int(count), _ptr(prim), _ptr(tex), _ptr(dOdE),
                                             _ptr(contrib)))
        return prim, tex, contrib

    def trace_stats(self, params, cfg, S=None):
        torch = self._torch
        if S is None:
            S = torch.empty((self.n_layouts, self.n_texels), dtype=torch.int64, device=params.device)
        out = (C.c_int64 * 8)()
        self._stream()
        self._check(self.lib.lt_trace_stats(self.h, C.byref(cfg), _ptr(params), _ptr(S), out))
        keys = ("segments", "nodes", "tri_tests", "hits", "misses", "wave_iters", "active_lanes", "phases")
        return dict(zip(keys, [int(x) for x in out]))

    def sync(self) -> int:
        f = C.c_uint32()
        self._check(self.lib.lt_sync(self.h, C.byref(f)))
        return int(f.value)

    def get_tuning(self) -> Tuning:
        t = Tuning()
        self._check(self.lib.lt_get_tuning(self.h, C.byref(t)))
        return t

    def set_tuning(self, **kw):
        t = self.get_tuning()
        for k, v in kw.items():
            setattr(t, k, int(v))
        self._check(self.lib.lt_set_tuning(self.h, C.byref(t)))

    def autotune(self, params, cfg, S, E, dOdE, grad, cache_path=None) -> float:
        best = C.c_float()
        cp = None if cache_path is None else cache_path.encode()
        self._stream()
        self._check(self.lib.lt_autotune(self.h, C.byref(cfg), _ptr(params), _ptr(S), _ptr(E), _ptr(dOdE),
                                         _ptr(grad), cp, C.byref(best)))
        return float(best.value)

    # -- emission proposal ---------------------------------------------------
    def proposal_set_table(self, pdf, cdf):
        torch = self._torch
        self._dev(pdf, torch.float32, (self.n_lights, MLP_BINS))
        self._dev(cdf, torch.float32, (self.n_lights, MLP_BINS))
        self._stream()
        self._check(self.lib.lt_proposal_set_table(self.h, _ptr(pdf), _ptr(cdf)))

    def proposal_get_table(self):
        torch = self._torch
        pdf = torch.empty((self.n_lights, MLP_BINS), dtype=torch.float32, device=f"cuda:{self.device}")
        cdf = torch.empty_like(pdf)
        self._stream()
        self._check(self.lib.lt_proposal_get_table(self.h, _ptr(pdf), _ptr(cdf)))
        return pdf, cdf

    def proposal_set_scale(self, inv_sigma):
        self._dev(inv_sigma, self._torch.float32, (self.n_lights, 6))
        self._stream()
        self._check(self.lib.lt_proposal_set_scale(self.h, _ptr(inv_sigma)))

    def mlp_infer(self, w_bf16, x, logits=None):
        torch = self._torch
        self._dev(w_bf16, torch.int16, (MLP_WEIGHTS,))
        self._dev(x, torch.float32, (self.n_lights, MLP_IN))
        self._stream()
        self._check(self.lib.lt_proposal_mlp_infer(self.h, _ptr(w_bf16), _ptr(x), _ptr(logits)))

    def mlp_train(self, w, mw, vw, w_bf16, x, mx, vx, target, step, lr, loss=None, grad_out=None):
        torch = self._torch
        for t in (w, mw, vw):
            self._dev(t, torch.float32, (MLP_WEIGHTS,))
        self._dev(w_bf16, torch.int16, (MLP_WEIGHTS,))
        for t in (x, mx, vx):
            self._dev(t, torch.float32, (self.n_lights, MLP_IN))
        self._dev(target, torch.float32, (self.n_lights, MLP_BINS))
        self._stream()
        self._check(self.lib.lt_proposal_mlp_train(self.h, _ptr(w), _ptr(mw), _ptr(vw), _ptr(w_bf16), _ptr(x),
                                                   _ptr(mx), _ptr(vx), _ptr(target), int(step), float(lr),
                                                   _ptr(loss), _ptr(grad_out)))

    def proposal_set(self, w, embed, param_lo, param_hi, hist_decay=0.9, plain_floor=0.3, sigma_decay=0.9):
        """Hand the network (FP32 weights [MLP_WEIGHTS], embeddings [L,16]) to the context."""
        torch = self._torch
        self._dev(w, torch.float32, (MLP_WEIGHTS,))
        self._dev(embed, torch.float32, (self.n_lights, 16))
        cfg = ProposalCfg()
        cfg.param_lo[:] = [float(v) for v in param_lo]
        cfg.param_hi[:] = [float(v) for v in param_hi]
        cfg.hist_decay, cfg.plain_floor, cfg.sigma_decay = float(hist_decay), float(plain_floor), float(sigma_decay)
        self._stream()
        self._check(self.lib.lt_proposal_set(self.h, _ptr(w), _ptr(embed), C.byref(cfg)))

    def proposal_refresh(self, params):
        self._dev(params, self._torch.float32, (self.n_lights, 6))
        self._stream()
        self._check(self.lib.lt_proposal_refresh(self.h, _ptr(params)))

    def proposal_update_scale(self, grad, mask=None):
        self._dev(grad, self._torch.float32, (self.n_lights, 6))
        m = None if mask is None else (C.c_float * 6)(*[float(v) for v in mask])
        self._stream()
        self._check(self.lib.lt_proposal_update_scale(self.h, _ptr(grad), m))

    def proposal_train_step(self, hist, lr, steps, loss=None, target_out=None):
        torch = self._torch
        self._dev(hist, torch.float32, (self.n_lights, MLP_BINS))
        if target_out is not None:
            self._dev(target_out, torch.float32, (self.n_lights, MLP_BINS))
        self._stream()
        self._check(self.lib.lt_proposal_train_step(self.h, _ptr(hist), float(lr), int(steps), _ptr(loss),
                                                    _ptr(target_out)))

    def proposal_get_net(self):
        torch = self._torch
        w = torch.empty(MLP_WEIGHTS, dtype=torch.float32, device=f"cuda:{self.device}")
        x = torch.empty((self.n_lights, MLP_IN), dtype=torch.float32, device=f"cuda:{self.device}")
        self._stream()
        self._check(self.lib.lt_proposal_get_net(self.h, _ptr(w), _ptr(x)))
        return w, x

    def set_timing(self, enable: bool):
        self._check(self.lib.lt_set_timing(self.h, 1 if enable else 0))

    def timing_read(self):
        """(forward kernel ms summed, launches, adjoint kernel ms summed, launches)."""
        f, a = C.c_double(), C.c_double()
        nf, na = C.c_int32(), C.c_int32()
        self._check(self.lib.lt_timing_read(self.h, C.byref(f), C.byref(nf), C.byref(a), C.byref(na)))
        return f.value, nf.value, a.value, na.value

    def bvh(self):
        """The acceleration structure on the host: (nodes [n, 64] u8, triangles
        [m, 12] f32 rows, the ids and patch ids as int bits)."""
        import numpy as np
        n = self.info()["bvh_nodes"]
        m = max(self.info()["n_tris"], 2)
        nodes = np.zeros((n, 64), np.uint8)
        tris = np.zeros((m, 12), np.float32)
        self._check(self.lib.lt_bvh_copy(self.h, nodes.ctypes.data, nodes.nbytes, tris.ctypes.data, tris.nbytes))
        if self.info()["n_tris"] > 1:
            tris = tris[: self.info()["n_tris"]]
        return nodes, tris

    def info(self) -> dict:
        i = Info()
        self._check(self.lib.lt_info_get(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}
