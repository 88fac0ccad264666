"""Independent closed forms and quadratures used to pin the oracle.

Nothing here calls the oracle or the GPU path.  Everything is float64 numpy
written from radiometry: solid angles of rectangles, Gauss-Legendre
integration of an emitter's irradiance over texels, and the log-irradiance
of a luminaire at a fixed receiver point (for derivative checks).
"""
import math

import numpy as np


def rot_y(b):
    c, s = np.cos(b), np.sin(b)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def frame(alpha, beta):
    """Light frame R = R_y(beta) R_x(alpha): axis d = R(0,0,-1), t = R e_x, b = R e_y."""
    R = rot_y(beta) @ rot_x(alpha)
    return R @ np.array([0, 0, -1.0]), R[:, 0], R[:, 1]


def corner_solid_angle(a, b, h):
    """Solid angle of the rectangle [0,a] x [0,b] (signed) seen from height h."""
    return np.arctan(a * b / (h * np.sqrt(a * a + b * b + h * h)))


def rect_solid_angle(x0, x1, y0, y1, h):
    f = corner_solid_angle
    return f(x1, y1, h) - f(x0, y1, h) - f(x1, y0, h) + f(x0, y0, h)


def corner_form_factor(a, b, h):
    """Differential-area (facing the plane) to corner rectangle [0,a]x[0,b] on a
    parallel plane at distance h (signed in a, b)."""
    X, Y = a / h, b / h
    sx, sy = np.sqrt(1 + X * X), np.sqrt(1 + Y * Y)
    return (X / sx * np.arctan(Y / sx) + Y / sy * np.arctan(X / sy)) / (2 * np.pi)


def rect_form_factor(x0, x1, y0, y1, h):
    f = corner_form_factor
    return f(x1, y1, h) - f(x0, y1, h) - f(x1, y0, h) + f(x0, y0, h)


def gauss_legendre(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w   # on [0,1]


def plane_texels(half, res):
    """Texel rectangles of plane_scene: x-index i runs along +x, j along +y."""
    edges = np.linspace(-half, half, res + 1)
    i = np.arange(res)
    x0, x1 = edges[i], edges[i + 1]
    X0, Y0 = np.meshgrid(x0, x0, indexing="xy")
    X1, Y1 = np.meshgrid(x1, x1, indexing="xy")
    # texel k = j*res + i  -> rows j (y), columns i (x)
    return X0.ravel(), X1.ravel(), Y0.ravel(), Y1.ravel()


def soft_profile(c, th_in, th_out):
    """Soft-edged spot: relative intensity as a function of cos(theta), and
    its integral over the sphere divided by 2 pi."""
    ci, co = math.cos(th_in), math.cos(th_out)
    a = np.where(c >= ci, 1.0, np.where(c > co, ((c - co) / (ci - co)) ** 2, 0.0))
    # int_{co}^{1} a dc = (1 - ci) + (ci - co) / 3
    return a, (1 - ci) + (ci - co) / 3


def lobe_density(kind, n, d, w, size=None, profile_power=1):
    """Direction pdf of a luminaire (per steradian) for unit directions w
    (soft-edged spot with profile_power 2: its profile squared over the same
    normalisation, for second moments)."""
    if kind == 0:
        return np.full(w.shape[:-1], 1.0 / (4 * np.pi))
    c = w @ d
    if kind == 3:
        a, norm = soft_profile(c, size[0], size[1])
        return a ** profile_power / (2 * np.pi * norm)
    return np.where(c > 0, (n + 1) / (2 * np.pi) * np.clip(c, 0, None) ** n, 0.0)


def plane_hit_probability(kind, n, p, size, half, res, q_tex=6, q_light=4, profile_power=1):
    """Probability that one emitted path first hits each texel of the z=0
    plane_scene (texel order k = j*res + i)."""
    c = np.asarray(p[:3], np.float64)
    d, t, b = frame(p[3], p[4])
    x0, x1, y0, y1 = plane_texels(half, res)
    gx, gw = gauss_legendre(q_tex)
    pts_u, pts_w = np.meshgrid(gx, gx, indexing="ij"), np.outer(gw, gw)
    fu, fv = pts_u[0].ravel(), pts_u[1].ravel()
    wq = pts_w.ravel()
    X = x0[:, None] + (x1 - x0)[:, None] * fu[None, :]
    Y = y0[:, None] + (y1 - y0)[:, None] * fv[None, :]
    area = ((x1 - x0) * (y1 - y0))[:, None]
    if kind == 2:
        lx, lw = gauss_legendre(q_light)
        su, sv = np.meshgrid(lx, lx, indexing="ij")
        sw = np.outer(lw, lw).ravel()
        au = (su.ravel() - 0.5) * size[0]
        av = (sv.ravel() - 0.5) * size[1]
        origins = c[None, :] + au[:, None] * t[None, :] + av[:, None] * b[None, :]
    else:
        origins = c[None, :]
        sw = np.ones(1)
    prob = np.zeros(X.shape[0])
    for o, ow in zip(origins, sw):
        v = np.stack([X - o[0], Y - o[1], -np.full_like(X, o[2])], -1)
        r = np.linalg.norm(v, axis=-1)
        w = v / r[..., None]
        dens = lobe_density(kind, n, d, w, size, profile_power)
        cos_i = o[2] / r          # receiver normal +z, emitter above
        prob += ow * np.sum(dens * cos_i / r ** 2 * wq[None, :] * area, axis=1)
    return prob


def linear_node_weights(u, res):
    """Piecewise-linear hats on a row of `res` texels over [0, 1]: nodes at
    the texel centres (i + 1/2)/res, the two outermost hats extended flat to
    the border so that the weights sum to one.  Returns (i0, i1, w0, w1)."""
    f = u * res - 0.5
    i0 = np.floor(f)
    w1 = f - i0
    i0 = i0.astype(np.int64)
    return np.clip(i0, 0, res - 1), np.clip(i0 + 1, 0, res - 1), 1.0 - w1, w1


def plane_node_moments(kind, n, p, size, half, res, q=4):
    """First and second moments, per node of the piecewise-linear basis on the
    z = 0 plane_scene, of one emitted path's first-hit weight w_k(x):
    m1_k = int phi_k(x) pdf(x) dA, m2_k = int phi_k(x)^2 pdf(x) dA, with pdf
    the first-hit density per unit area.  Each texel is split at its centre
    into four cells on which the hats are smooth, each integrated by
    Gauss-Legendre with q x q points."""
    c = np.asarray(p[:3], np.float64)
    d, t, b = frame(p[3], p[4])
    gx, gw = gauss_legendre(q)
    h = 2 * half / res
    # sub-cell corners along one axis: every half texel
    edges = -half + 0.5 * h * np.arange(2 * res + 1)
    xs = (edges[:-1, None] + 0.5 * h * gx[None, :]).ravel()          # points along x
    ws = np.broadcast_to(0.5 * h * gw[None, :], (2 * res, q)).ravel()
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    W = np.outer(ws, ws)
    v = np.stack([X - c[0], Y - c[1], -np.full_like(X, c[2])], -1)
    r = np.linalg.norm(v, axis=-1)
    w = v / r[..., None]
    pdf = lobe_density(kind, n, d, w, size) * (c[2] / r) / r ** 2 * W
    i0, i1, a0, a1 = linear_node_weights((X + half) / (2 * half), res)
    j0, j1, b0, b1 = linear_node_weights((Y + half) / (2 * half), res)
    m1 = np.zeros(res * res)
    m2 = np.zeros(res * res)
    for ii, aa in ((i0, a0), (i1, a1)):
        for jj, bb in ((j0, b0), (j1, b1)):
            np.add.at(m1, (jj * res + ii).ravel(), (pdf * aa * bb).ravel())
    # phi_k^2: sum the weights landing on the same node first (clamped borders)
    for k_of, wt in _node_sums(i0, i1, a0, a1, j0, j1, b0, b1, res):
        np.add.at(m2, k_of.ravel(), (pdf * wt * wt).ravel())
    return m1, m2


def _node_sums(i0, i1, a0, a1, j0, j1, b0, b1, res):
    """Per sample point, the (node, total weight) pairs after merging corners
    that the border clamp maps onto the same node."""
    ks = [(j * res + i, wa * wb) for i, wa in ((i0, a0), (i1, a1)) for j, wb in ((j0, b0), (j1, b1))]
    out = []
    for n_, (k, wk) in enumerate(ks):
        tot = wk.copy()
        first = np.ones(k.shape, bool)
        for m_, (k2, w2) in enumerate(ks):
            if m_ < n_:
                first &= k2 != k
            elif m_ > n_:
                tot = tot + np.where(k2 == k, w2, 0.0)
        out.append((k, np.where(first, tot, 0.0)))
    return out


def hsh_basis(order, ct, phi):
    """2pi-normalised hemispherical harmonics (integral of H^2 over the
    hemisphere = 2 pi) from scipy's associated Legendre functions of
    x = 2 cos(theta) - 1, with the Condon-Shortley phase removed; index
    l^2 + l + m, cos(m phi) for m > 0, sin(|m| phi) for m < 0."""
    from scipy.special import lpmv
    x = 2.0 * np.asarray(ct, np.float64) - 1.0
    out = []
    for l in range(order + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            P = lpmv(am, l, x) * (-1.0) ** am
            if m == 0:
                K = math.sqrt(2 * l + 1)
                out.append(K * P)
            else:
                K = math.sqrt(2 * (2 * l + 1) * math.factorial(l - am) / math.factorial(l + am))
                out.append(K * P * (np.cos(am * phi) if m > 0 else np.sin(am * phi)))
    return np.stack(out, -1)


def phong_brdf(rho_d, rho_s, e, wi, wo):
    """Lambertian + normalised Phong, normal = z: f = rho_d/pi + rho_s (e+2)/(2 pi)
    max(0, r.wo)^e with r the mirror direction of wi."""
    r = np.stack([-wi[..., 0], -wi[..., 1], wi[..., 2]], -1)
    ro = np.clip(np.sum(r * wo, -1), 0.0, None)
    return rho_d / math.pi + rho_s * (e + 2) / (2 * math.pi) * ro ** e


def plane_direct_coefficients(n_lobe, p, half, res, rho_d, rho_s, e, order, q_tex=4, q_ct=24, n_phi=48):
    """Expected exitant-radiance coefficients per texel of the z = 0 plane
    (normal +z, local frame = world) under a cos^n spot, direct light only,
    times A_k / P: int_texel pdf(x) F_lm(w_in(x)) dA with pdf the first-hit
    density per unit area and F_lm(w_in) = 1/(2 pi) int f(w_in, w) H_lm(w) dw,
    both by quadrature."""
    c = np.asarray(p[:3], np.float64)
    d, t, b = frame(p[3], p[4])
    gx, gw = gauss_legendre(q_tex)
    x0, x1, y0, y1 = plane_texels(half, res)
    fu, fv = np.meshgrid(gx, gx, indexing="ij")
    wq = np.outer(gw, gw).ravel()
    X = x0[:, None] + (x1 - x0)[:, None] * fu.ravel()[None, :]
    Y = y0[:, None] + (y1 - y0)[:, None] * fv.ravel()[None, :]
    area = ((x1 - x0) * (y1 - y0))[:, None]
    v = np.stack([X - c[0], Y - c[1], -np.full_like(X, c[2])], -1)
    r = np.linalg.norm(v, axis=-1)
    w = v / r[..., None]
    pdf = lobe_density(1, n_lobe, d, w) * (c[2] / r) / r ** 2            # per unit area
    wi = -w                                                             # towards the light
    cg, cw = gauss_legendre(q_ct)
    ph = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    CT, PH = np.meshgrid(cg, ph, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    wo = np.stack([ST * np.cos(PH), ST * np.sin(PH), CT], -1).reshape(-1, 3)
    ww = (np.repeat(cw, n_phi) * (2 * math.pi / n_phi))                   # dw = d(ct) dphi
    H = hsh_basis(order, CT.ravel(), PH.ravel())                          # [Q, NC]
    f = phong_brdf(rho_d, rho_s, e, wi.reshape(-1, 1, 3), wo[None, :, :])  # [texels*q, Q]
    F = (f * ww[None, :]) @ H / (2 * math.pi)                            # [texels*q, NC]
    F = F.reshape(X.shape[0], X.shape[1], -1)
    return np.einsum("kq,kqc->kc", pdf * wq[None, :] * area, F)          # [K, NC] per unit flux


def log_irradiance(kind, n, p, x1, n1, au=0.0, av=0.0, size=None, R=None):
    """log of the first-hit irradiance kernel at receiver x1 with unit normal
    n1 (facing the light), up to p-independent constants: a luminaire of power
    P with direction pdf ~ cos^n about its axis, origin c + a_u t + a_v b."""
    c = np.asarray(p[:3], np.float64)
    if R is None:
        d, t, b = frame(p[3], p[4])
    else:       # an explicit frame: axis -R e_z, tangents R e_x, R e_y
        d, t, b = -R[:, 2], R[:, 0], R[:, 1]
    y = c + au * t + av * b
    v = np.asarray(x1, np.float64) - y
    r = np.linalg.norm(v)
    w = v / r
    val = np.log(p[5]) + np.log(-np.dot(n1, w)) - 2 * np.log(r)
    if kind == 3:
        # intensity P a(cos) / (2 pi norm): the normalisation depends on the cones
        a, norm = soft_profile(np.dot(d, w), size[0], size[1])
        val += np.log(a) - np.log(norm)
    elif kind != 0:
        val += n * np.log(np.dot(d, w))
    return val
