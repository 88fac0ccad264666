"""Pins of the CPU oracle against closed forms, invariants and brute force.

None of these compares the oracle with another implementation of itself:
each check is fixed by radiometry or mathematics (solid angles, form factors,
energy conservation, linearity in power, finite differences of an
independently written irradiance function, brute-force intersection,
statistical properties of the generator, and the generator's published
known-answer vectors).
"""
import math

import numpy as np
import pytest

import lt_inputs as li
from lt_inputs.scenes import make_lights, POINT, SPOT, RECT, SOFT
import closed_forms as cf


# --------------------------------------------------------------------------
# generator and own transcendentals
# --------------------------------------------------------------------------

def test_philox_known_answers(oracle_lib):
    """The generator is the canonical Philox4x32-10: the known-answer vectors
    published with it (Salmon, Moraes, Dror and Shaw, SC'11, Random123 test
    suite) for an all-zero, an all-ones and a pi-digit counter and key."""
    kat = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
           ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, out in kat:
        assert [int(x) for x in oracle_lib.philox(list(ctr), list(key))] == list(out), (ctr, key)


def test_philox_avalanche(oracle_lib):
    """Counter-based generation needs outputs of neighbouring counters and
    keys to be unrelated: flipping any one counter or key bit flips each
    output bit with probability 1/2 (binomial bound over all 192 inputs)."""
    rng = np.random.default_rng(11)
    flips = []
    for _ in range(4):
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2 ** 32, 2, dtype=np.uint64)]
        base = np.asarray(oracle_lib.philox(ctr, key), np.uint64)
        for word in range(6):
            for bit in range(32):
                c, k = list(ctr), list(key)
                if word < 4:
                    c[word] ^= 1 << bit
                else:
                    k[word - 4] ^= 1 << bit
                out = np.asarray(oracle_lib.philox(c, k), np.uint64)
                flips.append(sum(bin(int(x)).count("1") for x in (out ^ base)))
    f = np.asarray(flips, np.float64)
    n = f.size * 128
    assert abs(f.sum() / n - 0.5) < 5 * math.sqrt(0.25 / n)
    assert f.min() > 128 * 0.25 and f.max() < 128 * 0.75


def test_philox_uniformity(oracle_lib):
    n = 1 << 14
    u = np.empty(4 * n)
    for i in range(n):
        x = oracle_lib.philox([i, 7, 3, 0], [0x1234, 0x5678])
        u[4 * i:4 * i + 4] = (x >> 8).astype(np.float64) * 2.0 ** -24
    assert u.min() >= 0.0 and u.max() <= 1.0 - 2.0 ** -24
    h, _ = np.histogram(u, bins=128, range=(0, 1))
    e = u.size / 128
    chi2 = ((h - e) ** 2 / e).sum()
    assert abs(chi2 - 127) < 6 * math.sqrt(2 * 127)
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5 / math.sqrt(u.size)


def test_directional_sample_uniforms_do_not_repeat(oracle_lib):
    """The directional mode's local samples (up to 64 per hit, two per
    generator draw) take their own generator blocks at every hit: over all
    hits a path can have (1..64) and all sample indices, the (block, half)
    pairs are distinct and never coincide with the emission (0), proposal (1)
    or bounce (1 + h) blocks, and the uniform pairs drawn for one path are all
    different.  Consecutive hits sharing samples would correlate a path's
    bounces (no bias, more variance)."""
    seen = set()
    for h in range(1, 65):
        for j in range(64):
            b = oracle_lib.dir_block(h, j)
            assert b > 65
            seen.add((b, j & 1))
    assert len(seen) == 64 * 64
    key = [0x1234567, 0x89ABCDE]
    pairs = set()
    for h in range(1, 9):
        for j in range(0, 64, 2):
            x = oracle_lib.philox([42, (3 << 16) | 5, oracle_lib.dir_block(h, j), 0], key)
            pairs.add((int(x[0]), int(x[1])))
            pairs.add((int(x[2]), int(x[3])))
    assert len(pairs) == 8 * 64


def test_sincos2pi(oracle_lib):
    us = np.concatenate([np.arange(0, 1 << 24, 997) * 2.0 ** -24, [0.0, 0.25, 0.5, 0.75, 1 - 2.0 ** -24]])
    for u in us[::7]:
        s, c = oracle_lib.sincos2pi(u)
        assert abs(s - math.sin(2 * math.pi * u)) < 2.5e-7
        assert abs(c - math.cos(2 * math.pi * u)) < 2.5e-7
    # exact quadrant points
    assert oracle_lib.sincos2pi(0.0) == (0.0, 1.0)
    assert oracle_lib.sincos2pi(0.25) == (1.0, -0.0) or oracle_lib.sincos2pi(0.25)[0] == 1.0


def test_log2_exp2(oracle_lib):
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(0, 1, 4000), 2.0 ** -rng.uniform(0, 24, 4000)]).astype(np.float32)
    xs = xs[xs > 0]
    for x in xs[::3]:
        ref = math.log2(float(x))
        assert abs(oracle_lib.log2(x) - ref) <= 3e-7 * max(1.0, abs(ref))
    ys = rng.uniform(-40, 0, 3000).astype(np.float32)
    for y in ys[::3]:
        ref = 2.0 ** float(y)
        assert abs(oracle_lib.exp2(y) - ref) <= 3e-7 * ref
    assert oracle_lib.log2(1.0) == 0.0 and oracle_lib.exp2(0.0) == 1.0
    assert oracle_lib.log2(0.5) == -1.0 and oracle_lib.exp2(-3.0) == 0.125


def test_sincos_f64(oracle_lib):
    for x in np.linspace(-12.0, 12.0, 1001):
        s, c = oracle_lib.sincos_f64(x)
        assert abs(s - math.sin(x)) < 4e-16 and abs(c - math.cos(x)) < 4e-16


# --------------------------------------------------------------------------
# P3: BVH closest hit == brute force
# --------------------------------------------------------------------------

def _random_rays(rng, n, lo, hi):
    o = rng.uniform(lo, hi, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([o, d], 1).astype(np.float32)


@pytest.mark.parametrize("seed", range(4))
def test_bvh_equals_brute_force(oracle_lib, seed):
    sc = li.random_scene_tiny(seed, n_quads=32)
    brute = oracle_lib.OracleScene(sc, use_bvh=False)
    bvh = oracle_lib.OracleScene(sc, use_bvh=True)
    rng = np.random.default_rng(seed)
    rays = _random_rays(rng, 1 << 13, -2.5, 2.5)
    skip = rng.integers(-1, sc.n_patches, rays.shape[0]).astype(np.int32)
    t0, p0 = oracle_lib.intersect(brute, rays, skip)
    t1, p1 = oracle_lib.intersect(bvh, rays, skip)
    assert np.array_equal(p0, p1)
    assert np.array_equal(t0.view(np.uint32), t1.view(np.uint32))
    assert (p0 >= 0).mean() > 0.1


def test_bvh_equals_brute_force_room(oracle_lib):
    c1 = li.box_room()
    sc = c1["scene"]
    brute = oracle_lib.OracleScene(sc, use_bvh=False)
    bvh = oracle_lib.OracleScene(sc, use_bvh=True)
    rays = _random_rays(np.random.default_rng(5), 1 << 13, [0.01, 0.01, 0.01], [3.99, 2.99, 2.49])
    t0, p0 = oracle_lib.intersect(brute, rays)
    t1, p1 = oracle_lib.intersect(bvh, rays)
    assert np.array_equal(p0, p1) and np.array_equal(t0, t1)
    assert (p0 >= 0).all()    # closed room: every ray hits


def test_skip_patch_prevents_self_hit(oracle_lib):
    sc = li.plane_scene(half=1.0, res=4)
    osc = oracle_lib.OracleScene(sc)
    rays = np.array([[0.1, 0.2, 0.0, 0.3, 0.1, 0.9], [0.1, 0.2, 0.5, 0.0, 0.0, -1.0]], np.float32)
    t, p = oracle_lib.intersect(osc, rays, np.array([0, -1], np.int32))
    assert p[0] == -1 and p[1] >= 0 and abs(t[1] - 0.5) < 1e-6


# --------------------------------------------------------------------------
# P1: emitters over a plane, B = 1 (closed-form / quadrature texel probabilities)
# --------------------------------------------------------------------------

def _hit_counts(oracle_lib, kind, n, p, size, half, res, N):
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([kind], [n], [size], [0], [p])
    S, misses = oracle_lib.forward(oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights),
                                   lights.params, 0xABC, N, 1)
    E = oracle_lib.fixed_to_float(S)[0].astype(np.float64)
    A = sc.texel_area().astype(np.float64)
    counts = E * A / (p[5] / N)
    return counts, misses


def _binomial_check(counts, prob, N, min_expect=50.0, zmax=5.5):
    m = N * prob >= min_expect
    assert m.sum() > 200
    z = (counts[m] - N * prob[m]) / np.sqrt(N * prob[m] * (1 - prob[m]))
    chi2 = float((z ** 2).sum())
    dof = int(m.sum())
    assert np.abs(z).max() < zmax, np.abs(z).max()
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof), (chi2, dof)


def test_point_light_over_plane(oracle_lib):
    """E = I cos(theta)/r^2 with I = P/(4 pi): texel hit probability = Omega/(4 pi)."""
    half, res, N, h = 10.0, 64, 1 << 20, 2.0
    p = [0.3, -0.2, h, 0.0, 0.0, 100.0]
    counts, misses = _hit_counts(oracle_lib, POINT, 0.0, p, (0, 0), half, res, N)
    assert np.abs(counts - np.rint(counts)).max() < 2e-3    # whole paths per texel
    x0, x1, y0, y1 = cf.plane_texels(half, res)
    omega = cf.rect_solid_angle(x0 - p[0], x1 - p[0], y0 - p[1], y1 - p[1], h)
    _binomial_check(counts, omega / (4 * np.pi), N)
    p_hit = omega.sum() / (4 * np.pi)
    assert abs((N - misses) - N * p_hit) < 6 * math.sqrt(N * p_hit * (1 - p_hit))


def test_tilted_spot_over_plane(oracle_lib):
    half, res, N = 4.0, 48, 1 << 20
    p = [0.5, 0.3, 1.5, 0.2, -0.15, 80.0]
    counts, misses = _hit_counts(oracle_lib, SPOT, 4.0, p, (0, 0), half, res, N)
    prob = cf.plane_hit_probability(SPOT, 4.0, p, None, half, res)
    _binomial_check(counts, prob, N)


def test_rect_light_over_plane(oracle_lib):
    half, res, N = 4.0, 40, 1 << 20
    p = [-0.4, 0.2, 1.2, 0.25, 0.1, 60.0]
    counts, misses = _hit_counts(oracle_lib, RECT, 1.5, p, (0.8, 0.5), half, res, N)
    prob = cf.plane_hit_probability(RECT, 1.5, p, (0.8, 0.5), half, res)
    _binomial_check(counts, prob, N)


def test_soft_spot_over_plane(oracle_lib):
    """Soft-edged spot: directions uniform over the outer cap, each path's
    flux weighted by the fall-off.  The flux reaching each texel has mean
    P * (its share of the normalised intensity profile) and variance
    (P^2/N) (k_cap m2_k - m_k^2), both by quadrature of the profile."""
    half, res, N = 2.0, 40, 1 << 20
    th = (0.3, 0.75)
    p = [0.4, -0.3, 1.3, 0.25, -0.15, 70.0]
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([SOFT], [0.0], [th], [0], [p])
    S, _ = oracle_lib.forward(oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights), lights.params,
                              0x50F7, N, 1)
    flux = oracle_lib.fixed_to_float(S)[0].astype(np.float64) * sc.texel_area().astype(np.float64)
    m1 = cf.plane_hit_probability(SOFT, 0.0, p, th, half, res, q_tex=6)
    # second moment: the same quadrature with the profile squared
    ci, co = math.cos(th[0]), math.cos(th[1])
    _, norm = cf.soft_profile(1.0, *th)
    kcap = (1 - co) / norm
    m2 = cf.plane_hit_probability(SOFT, 0.0, p, th, half, res, q_tex=6, profile_power=2)
    var = p[5] ** 2 / N * (kcap * m2 - m1 ** 2)
    m = m1 * N >= 50
    assert m.sum() > 300
    z = (flux[m] - p[5] * m1[m]) / np.sqrt(var[m])
    assert np.abs(z).max() < 5.5, np.abs(z).max()
    assert abs(float((z ** 2).sum()) - m.sum()) < 6 * math.sqrt(2 * m.sum())


def test_soft_spot_total_flux(oracle_lib):
    """In a closed box every first hit lands: the splatted flux is the sum of
    the per-path weights, whose mean is P (the normalisation of the profile)
    and whose variance is (P^2/N)(k_cap m2 - 1) with the closed forms
    int a dc = (1 - ci) + (ci - co)/3 and int a^2 dc = (1 - ci) + (ci - co)/5."""
    N, P = 1 << 20, 30.0
    for th in ((0.2, 0.6), (0.0, 1.0), (0.5, 0.55)):
        sc = li.closed_box()
        lights = make_lights([SOFT], [0.0], [th], [0], [[1.0, 0.75, 0.5, 0.3, -0.2, P]])
        S, misses = oracle_lib.forward(oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights),
                                       lights.params, 0x77 + int(th[1] * 100), N, 1)
        assert misses == 0
        total = float(np.sum(S[0].astype(np.float64) * 2.0 ** -32 * sc.texel_area().astype(np.float64)))
        ci, co = math.cos(th[0]), math.cos(th[1])
        norm = (1 - ci) + (ci - co) / 3
        m2 = ((1 - ci) + (ci - co) / 5) / norm
        kcap = (1 - co) / norm
        sigma = P * math.sqrt((kcap * m2 - 1) / N)
        assert abs(total - P) < 5 * sigma + 1e-6 * P, (th, total, sigma)


def test_linear_basis_over_plane(oracle_lib):
    """Piecewise-linear basis (nodes at texel centres): the flux each node
    receives has mean P m1_k and variance (P^2/N)(m2_k - m1_k^2), with m1, m2
    the first-hit density integrated against the hat and its square; and the
    hats sum to one, so the total equals the box basis' total path by path."""
    half, res, N = 2.0, 24, 1 << 20
    p = [0.35, -0.25, 1.2, 0.2, -0.1, 60.0]
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([SPOT], [3.0], [(0, 0)], [0], [p])
    ol = oracle_lib.OracleLights(lights)
    S_lin, _ = oracle_lib.forward(oracle_lib.OracleScene(sc, basis="linear"), ol, lights.params, 0x11B, N, 1)
    S_box, _ = oracle_lib.forward(oracle_lib.OracleScene(sc), ol, lights.params, 0x11B, N, 1)
    A = sc.texel_area().astype(np.float64)
    flux = S_lin[0].astype(np.float64) * 2.0 ** -32 * A
    tot_box = float((S_box[0].astype(np.float64) * 2.0 ** -32 * A).sum())
    assert abs(flux.sum() / tot_box - 1) < 1e-6
    m1, m2 = cf.plane_node_moments(SPOT, 3.0, p, None, half, res)
    m = m1 * N >= 50
    assert m.sum() > 200
    z = (flux[m] - p[5] * m1[m]) / np.sqrt(p[5] ** 2 / N * (m2[m] - m1[m] ** 2))
    assert np.abs(z).max() < 5.5, np.abs(z).max()
    assert abs(float((z ** 2).sum()) - m.sum()) < 6 * math.sqrt(2 * m.sum())


def test_linear_basis_closed_box(oracle_lib):
    rho, B, N, P = 0.6, 5, 1 << 17, 50.0
    sc = li.closed_box(albedo=rho)
    lights = make_lights([POINT, SOFT], [0.0, 0.0], [(0, 0), (0.2, 0.7)], [0, 0],
                         [[0.7, 0.6, 0.5, 0, 0, P], [1.3, 0.9, 0.8, 0.3, -0.2, 2 * P]])
    ol = oracle_lib.OracleLights(lights)
    S, misses = oracle_lib.forward(oracle_lib.OracleScene(sc, basis="linear"), ol, lights.params, 0x98, N, B)
    S_box, _ = oracle_lib.forward(oracle_lib.OracleScene(sc), ol, lights.params, 0x98, N, B)
    assert misses == 0
    A = sc.texel_area().astype(np.float64)
    total = float(np.sum(A * S[0].astype(np.float64) * 2.0 ** -32))
    total_box = float(np.sum(A * S_box[0].astype(np.float64) * 2.0 ** -32))
    assert abs(total / total_box - 1) < 1e-6
    assert not np.array_equal(S, S_box)


def test_linear_basis_direct_gradient_vs_quadrature(oracle_lib):
    """B = 1 with the linear basis: the adjoint gathers dO/dE with the same
    hat weights, so its mean is sum_k g_k d/dp (P m1_k(p) / A_k).  Coarse
    texels under a narrow spot make the hat and box expectations differ by
    many standard errors, so a gather with box weights would fail."""
    half, res, N, n = 2.0, 8, 1 << 20, 8.0
    p = np.array([0.3, -0.2, 1.0, 0.3, -0.2, 40.0])
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([SPOT], [n], [(0, 0)], [0], [p])
    A = float(sc.texel_area()[0])
    ii, jj = np.meshgrid(np.arange(res), np.arange(res), indexing="xy")
    sign = np.where((ii + jj).ravel() % 2 == 0, 1.0, -1.0)
    g = (sign * np.random.default_rng(17).uniform(0.5, 1.0, sc.n_texels)).astype(np.float32)
    ref, ref_box = np.zeros(6), np.zeros(6)
    for c in range(6):
        h = 1e-4
        pp, pm = p.copy(), p.copy()
        pp[c] += h
        pm[c] -= h
        Ep = cf.plane_node_moments(SPOT, n, pp, None, half, res, q=8)[0] * pp[5] / A
        Em = cf.plane_node_moments(SPOT, n, pm, None, half, res, q=8)[0] * pm[5] / A
        ref[c] = np.dot(g.astype(np.float64), (Ep - Em) / (2 * h))
        Bp = cf.plane_hit_probability(SPOT, n, pp, None, half, res, q_tex=12) * pp[5] / A
        Bm = cf.plane_hit_probability(SPOT, n, pm, None, half, res, q_tex=12) * pm[5] / A
        ref_box[c] = np.dot(g.astype(np.float64), (Bp - Bm) / (2 * h))
    osc, ol = oracle_lib.OracleScene(sc, basis="linear"), oracle_lib.OracleLights(lights)
    _, _, contrib = oracle_lib.record(osc, ol, lights.params, 0xD7, N, 1, 0, 0, 0, N, g[None])
    c64 = contrib.astype(np.float64)
    est = c64.sum(0)
    sigma = c64.std(0) * math.sqrt(N)
    assert np.max(np.abs(ref - ref_box) / sigma) > 10
    for c in range(6):
        assert abs(est[c] - ref[c]) < 4.5 * sigma[c] + 1e-3 * abs(ref[c]), (c, est[c], ref[c], sigma[c])
    grad, _ = oracle_lib.adjoint(osc, ol, lights.params, 0xD7, N, 1, g[None])
    assert np.allclose(grad[0], est, rtol=1e-9, atol=1e-12 * np.abs(c64).sum())


# --------------------------------------------------------------------------
# object-space path tracing with next-event estimation (comparison estimator)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [POINT, SPOT, RECT, SOFT])
def test_path_trace_direct_over_plane(oracle_lib, kind):
    """One vertex per sample (direct light only): the texel means agree with
    the quadrature of the emitter's irradiance over each texel, to within the
    noise that two seeds show."""
    half, res, M = 3.0, 16, 64
    n = {SPOT: 3.0, RECT: 1.5}.get(kind, 0.0)
    size = {RECT: (0.8, 0.5), SOFT: (0.3, 0.8)}.get(kind, (0, 0))
    p = [0.4, -0.3, 1.3, 0.25 if kind else 0.0, -0.15 if kind else 0.0, 70.0]
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([kind], [n], [size], [0], [p])
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    A = float(sc.texel_area()[0])
    ref = cf.plane_hit_probability(kind, n, p, size, half, res, q_tex=8, q_light=8) * p[5] / A
    Es = [oracle_lib.fixed_to_float(oracle_lib.path_trace(osc, ol, lights.params, sd, M, 1)[0])[0].astype(np.float64)
          for sd in (0x71, 0x72)]
    err = np.linalg.norm((Es[0] + Es[1]) / 2 - ref)
    noise = np.linalg.norm(Es[0] - Es[1]) / 2
    assert err < 1.6 * noise + 1e-4 * np.linalg.norm(ref), (err, noise)


def test_path_trace_matches_light_trace(oracle_lib):
    """Box room with bounces (B = 3) and three luminaires: path tracing and
    light tracing estimate the same texel irradiance; per-patch flux totals
    agree within the noise that two seeds of each show."""
    sc = li.box_room()["scene"]
    lights = make_lights([SPOT, POINT, RECT], [3.0, 0.0, 1.0], [(0, 0), (0, 0), (0.5, 0.3)], [0, 0, 0],
                         [[1.0, 1.0, 2.0, 0.1, 0.2, 50.0], [3.0, 2.0, 1.8, 0, 0, 30.0],
                          [2.0, 1.5, 2.4, -0.2, 0.3, 70.0]])
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    A = sc.texel_area().astype(np.float64)
    patch = np.repeat(np.arange(sc.n_patches), sc.patch_res().prod(1))

    def patch_flux(S):
        f = S[0].astype(np.float64) * 2.0 ** -32 * A
        return np.bincount(patch, weights=f, minlength=sc.n_patches)

    pt = [patch_flux(oracle_lib.path_trace(osc, ol, lights.params, sd, 8, 3)[0]) for sd in (1, 2)]
    lt = [patch_flux(oracle_lib.forward(osc, ol, lights.params, sd, 1 << 21, 3)[0]) for sd in (3, 4)]
    err = np.linalg.norm((pt[0] + pt[1]) / 2 - (lt[0] + lt[1]) / 2)
    noise = math.sqrt(np.sum((pt[0] - pt[1]) ** 2) + np.sum((lt[0] - lt[1]) ** 2)) / 2
    assert err < 3 * noise, (err, noise)
    assert np.linalg.norm(pt[0] - lt[0]) < 0.05 * np.linalg.norm(lt[0])


def test_path_trace_gradient_is_the_estimators_derivative(oracle_lib):
    """In a convex room no shadow ray is ever blocked and no sample moves with
    the lights, so one seed's estimate is a smooth function of p: its
    gradient of sum_k g_k E_k equals central differences of that sum with the
    same seed, for every luminaire type and parameter."""
    sb = li.SceneBuilder()
    sb.boxes([0, 0, 0], [4.0, 3.0, 2.5], 0.6, res=(12, 12))
    sc = sb.build("empty_room", fixed_res=(12, 12))
    p = np.array([[1.2, 1.0, 2.1, 0.2, -0.15, 40.0], [2.9, 1.8, 2.2, -0.1, 0.25, 30.0],
                  [2.0, 2.2, 2.3, 0.15, 0.1, 50.0], [1.0, 2.1, 1.8, 0.0, 0.0, 20.0]], np.float32)
    # profiles without kinks (cos^n with n >= 2, a soft-edged spot with no
    # inner cone), so a difference step never straddles a kink of the intensity
    lights = make_lights([SPOT, RECT, SOFT, POINT], [3.0, 2.0, 0.0, 0.0], [(0, 0), (0.6, 0.4), (0.0, 0.9), (0, 0)],
                         [0, 0, 0, 0], p)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    g = np.random.default_rng(21).normal(size=(1, sc.n_texels)).astype(np.float32)
    seed, M, B = 0x3C, 4, 3
    _, grad = oracle_lib.path_trace(osc, ol, p, seed, M, B, dOdE=g)

    def lin(pp):
        S, _ = oracle_lib.path_trace(osc, ol, pp, seed, M, B)
        return float(np.dot(g[0].astype(np.float64), S[0].astype(np.float64) * 2.0 ** -32))

    for l in range(4):
        for c in range(6):
            if lights.static["type"][l] == POINT and c in (3, 4):
                assert grad[l, c] == 0.0
                continue
            h = {5: 0.2}.get(c, 1e-3)
            pp, pm = p.copy(), p.copy()
            pp[l, c] += h
            pm[l, c] -= h
            fd = (lin(pp) - lin(pm)) / (float(pp[l, c]) - float(pm[l, c]))
            assert abs(fd - grad[l, c]) <= 2e-3 * abs(grad[l, c]) + 1e-4 * np.abs(grad).max(), (l, c, fd, grad[l, c])


# --------------------------------------------------------------------------
# colour (per-channel flux weights and albedos)
# --------------------------------------------------------------------------

def test_rgb_closed_box_energy(oracle_lib):
    """Per channel, a closed box with albedo rho_ch absorbs exactly the flux
    sum_l P_l c_l,ch (1 - rho_ch^B) / (1 - rho_ch)."""
    rho = np.array([0.5, 0.6, 0.72])
    B, N = 5, 1 << 17
    sc = li.closed_box(albedo=0.6)
    alb = np.broadcast_to(rho.astype(np.float32), (sc.n_patches, 3)).copy()
    P = np.array([30.0, 55.0])
    col = np.array([[0.2, 0.3, 0.5], [0.6, 0.25, 0.15]], np.float32)
    lights = make_lights([POINT, SPOT], [0.0, 2.0], [(0, 0)] * 2, [0, 0],
                         [[0.7, 0.6, 0.5, 0, 0, P[0]], [1.3, 0.9, 0.8, 0.3, -0.2, P[1]]])
    S, misses = oracle_lib.forward(oracle_lib.OracleScene(sc, albedo_rgb=alb), oracle_lib.OracleLights(lights, col),
                                   lights.params, 0x3B, N, B)
    assert misses == 0 and S.shape == (1, 3, sc.n_texels)
    A = sc.texel_area().astype(np.float64)
    for ch in range(3):
        total = float(np.sum(A * S[0, ch].astype(np.float64) * 2.0 ** -32))
        expect = float(np.dot(P, col[:, ch])) * (1 - rho[ch] ** B) / (1 - rho[ch])
        assert abs(total / expect - 1) < 1e-6, (ch, total, expect)


def _rgb_case(oracle_lib):
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    rng = np.random.default_rng(12)
    alb = rng.uniform(0.3, 0.8, (sc.n_patches, 3)).astype(np.float32)
    col = np.array([[0.5, 0.3, 0.2]], np.float32)
    return sc, lights, alb, col


def test_rgb_channels_are_grey_runs(oracle_lib):
    """One path geometry for all channels: channel ch equals c_ch times the
    grey tracer run with albedo rho_ch, and the geometric gradient is
    sum_ch c_ch times the grey gradients with dO/dE_ch."""
    sc, lights, alb, col = _rgb_case(oracle_lib)
    N, B, seed = 1 << 15, 3, 0x77
    ol_rgb = oracle_lib.OracleLights(lights, col)
    S, _ = oracle_lib.forward(oracle_lib.OracleScene(sc, albedo_rgb=alb), ol_rgb, lights.params, seed, N, B)
    g = np.random.default_rng(2).normal(size=(1, 3, sc.n_texels)).astype(np.float32)
    grad, grad_c, _ = oracle_lib.adjoint_rgb(oracle_lib.OracleScene(sc, albedo_rgb=alb), ol_rgb, lights.params,
                                             seed, N, B, g)
    ol = oracle_lib.OracleLights(lights)
    ref_grad = np.zeros(6)
    for ch in range(3):
        sc_ch = li.scenes.Scene(**{**sc.__dict__})
        sc_ch.patches = sc.patches.copy()
        sc_ch.patches["albedo"] = alb[:, ch]
        osc_ch = oracle_lib.OracleScene(sc_ch)
        S_g, _ = oracle_lib.forward(osc_ch, ol, lights.params, seed, N, B)
        E_rgb = S[0, ch].astype(np.float64)
        E_g = S_g[0].astype(np.float64) * float(col[0, ch])
        assert np.linalg.norm(E_rgb - E_g) <= 1e-6 * np.linalg.norm(E_g)
        gr, _ = oracle_lib.adjoint(osc_ch, ol, lights.params, seed, N, B, g[:, ch])
        ref_grad += float(col[0, ch]) * gr[0]
    assert np.allclose(grad[0], ref_grad, rtol=1e-5, atol=1e-6 * np.abs(ref_grad).max())


def test_rgb_colour_gradient(oracle_lib):
    """E is linear in the channel weights, so dO/dc of O = sum g E matches
    central differences exactly (up to rounding); and sum_ch c_ch dO/dc_ch =
    P dO/dP, both being sum over paths of the colour-weighted adjoint times
    Phi_r."""
    sc, lights, alb, col = _rgb_case(oracle_lib)
    N, B, seed = 1 << 14, 3, 0x5D
    osc = oracle_lib.OracleScene(sc, albedo_rgb=alb)
    g = np.random.default_rng(3).normal(size=(1, 3, sc.n_texels)).astype(np.float32)
    grad, grad_c, _ = oracle_lib.adjoint_rgb(osc, oracle_lib.OracleLights(lights, col), lights.params, seed, N, B, g)

    def lin(cc):
        S, _ = oracle_lib.forward(osc, oracle_lib.OracleLights(lights, cc), lights.params, seed, N, B)
        return float(np.sum(g.astype(np.float64) * S.astype(np.float64) * 2.0 ** -32))

    for ch in range(3):
        h = 0.05
        cp, cm = col.copy(), col.copy()
        cp[0, ch] += h
        cm[0, ch] -= h
        fd = (lin(cp) - lin(cm)) / (float(cp[0, ch]) - float(cm[0, ch]))
        assert abs(fd - grad_c[0, ch]) <= 1e-5 * np.abs(grad_c).max(), (ch, fd, grad_c[0, ch])
    lhs = float(np.dot(col[0].astype(np.float64), grad_c[0]))
    rhs = float(lights.params[0, 5]) * grad[0, 5]
    assert abs(lhs / rhs - 1) < 1e-5


# --------------------------------------------------------------------------
# directional texels (hemispherical harmonics) and a glossy BRDF
# --------------------------------------------------------------------------

def test_hsh_orthonormal(oracle_lib):
    """The oracle's harmonics: integral of H_i H_j over the hemisphere is
    2 pi delta_ij, and they agree with scipy's associated Legendre functions."""
    cg, cw = cf.gauss_legendre(16)
    n_phi = 64
    ph = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    Hs, W = [], []
    for ct, w in zip(cg, cw):
        for f in ph:
            Hs.append(oracle_lib.hsh(3, ct, math.cos(f), math.sin(f)).astype(np.float64))
            W.append(w * 2 * math.pi / n_phi)
    Hs, W = np.array(Hs), np.array(W)
    G = (Hs * W[:, None]).T @ Hs
    assert np.allclose(G, 2 * math.pi * np.eye(16), atol=4e-5)
    CT, PH = np.meshgrid(cg, ph, indexing="ij")
    ref = cf.hsh_basis(3, CT.ravel(), PH.ravel())
    assert np.allclose(Hs, ref, atol=4e-6)
    for order in range(3):     # lower orders are prefixes
        n = (order + 1) ** 2
        assert np.array_equal(oracle_lib.hsh(order, 0.3, 0.6, 0.8), oracle_lib.hsh(3, 0.3, 0.6, 0.8)[:n])


def test_brdf_normalisation_and_gradient(oracle_lib):
    """At normal incidence the normalised Phong lobe reflects exactly rho_s
    (int (e+2)/(2 pi) cos^e cos dw = 1); the gradient w.r.t. w_in matches
    central differences."""
    cg, cw = cf.gauss_legendre(64)
    n_phi = 32
    tot = 0.0
    for ct, w in zip(cg, cw):
        st = math.sqrt(1 - ct * ct)
        for k in range(n_phi):
            f = (k + 0.5) * 2 * math.pi / n_phi
            fv, _ = oracle_lib.brdf(0.3, 0.5, 12.0, [0, 0, 1], [st * math.cos(f), st * math.sin(f), ct])
            tot += fv * ct * w * 2 * math.pi / n_phi
    assert abs(tot - 0.8) < 1e-4
    rng = np.random.default_rng(4)
    for _ in range(20):
        wi = rng.normal(size=3); wi[2] = abs(wi[2]) + 0.3; wi /= np.linalg.norm(wi)
        wo = np.array([-wi[0], -wi[1], wi[2]]) + 0.2 * rng.normal(size=3); wo[2] = abs(wo[2]); wo /= np.linalg.norm(wo)
        f0, gr = oracle_lib.brdf(0.2, 0.6, 7.0, wi, wo)
        for c in range(3):
            h = 1e-3
            a, b = wi.copy(), wi.copy()
            a[c] += h
            b[c] -= h
            fd = (oracle_lib.brdf(0.2, 0.6, 7.0, a, wo)[0] - oracle_lib.brdf(0.2, 0.6, 7.0, b, wo)[0]) / (2 * h)
            assert abs(fd - gr[c]) < 2e-3 * (abs(fd) + 1.0), (c, fd, gr[c])


def test_directional_lambertian_is_irradiance(oracle_lib):
    """With a Lambertian surface the exitant radiance is isotropic: the
    order-0 coefficient is (rho / pi) E_k of the irradiance tracer on the same
    paths, and the higher ones average out."""
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    N, B, seed = 1 << 15, 3, 0x61
    ol = oracle_lib.OracleLights(lights)
    S_d, _ = oracle_lib.forward(oracle_lib.OracleScene(sc, dir_order=2, dir_samples=4), ol, lights.params, seed, N, B)
    S_e, _ = oracle_lib.forward(oracle_lib.OracleScene(sc), ol, lights.params, seed, N, B)
    rho = np.repeat(sc.patches["albedo"].astype(np.float64), sc.patch_res().prod(1))
    L0 = S_d[0, 0].astype(np.float64)
    ref = rho / math.pi * S_e[0].astype(np.float64)
    assert np.linalg.norm(L0 - ref) <= 2e-6 * np.linalg.norm(ref)
    hi = S_d[0, 1:].astype(np.float64)
    assert abs(hi.sum()) < 0.02 * np.abs(hi).sum()


def _glossy_plane(half, res):
    sc = li.plane_scene(half=half, res=res, albedo=0.3)
    return sc, np.array([[0.5, 16.0]], np.float32)


def test_directional_glossy_direct_over_plane(oracle_lib):
    """Direct light on a glossy plane: every coefficient's texel mean (order
    3, 16 harmonics) agrees with the quadrature of the reflected radiance's
    projection, within the noise two seeds show, in total and order by order."""
    half, res, N = 2.0, 8, 1 << 18
    sc, gl = _glossy_plane(half, res)
    p = [0.3, -0.2, 1.2, 0.3, -0.15, 50.0]
    lights = make_lights([SPOT], [3.0], [(0, 0)], [0], [p])
    osc = oracle_lib.OracleScene(sc, glossy=gl, dir_order=3, dir_samples=8)
    ol = oracle_lib.OracleLights(lights)
    A = float(sc.texel_area()[0])
    ref = cf.plane_direct_coefficients(3.0, p, half, res, 0.3, 0.5, 16.0, 3).T * p[5] / A   # [16, K]
    Ls = [oracle_lib.fixed_to_float(oracle_lib.forward(osc, ol, lights.params, sd, N, 1)[0])[0].astype(np.float64)
          for sd in (0x91, 0x92)]
    # all coefficients, then each order's block on its own
    for sl in (slice(0, 16), slice(0, 1), slice(1, 4), slice(4, 9), slice(9, 16)):
        err = np.linalg.norm((Ls[0][sl] + Ls[1][sl]) / 2 - ref[sl])
        noise = np.linalg.norm(Ls[0][sl] - Ls[1][sl]) / 2
        assert err < 1.6 * noise + 1e-4 * np.linalg.norm(ref[sl]), (sl, err, noise)
    assert np.linalg.norm(ref[9:]) > 0.05 * np.linalg.norm(ref)     # order 3 carries signal here


def test_directional_glossy_direct_gradient(oracle_lib):
    """Direct light on a glossy plane: the adjoint's mean over seeds matches
    the derivative of the quadrature expectation of sum g_lm,k L_lm,k; the
    first hit's BRDF projection term carries most of the position gradient."""
    half, res, N, n_seeds = 2.0, 8, 1 << 16, 8
    sc, gl = _glossy_plane(half, res)
    p = np.array([0.3, -0.2, 1.2, 0.3, -0.15, 50.0])
    lights = make_lights([SPOT], [3.0], [(0, 0)], [0], [p])
    osc = oracle_lib.OracleScene(sc, glossy=gl, dir_order=2, dir_samples=8)
    ol = oracle_lib.OracleLights(lights)
    A = float(sc.texel_area()[0])
    g = np.random.default_rng(6).normal(size=(9, sc.n_texels)).astype(np.float32)
    ref = np.zeros(6)
    for c in range(6):
        h = 1e-4
        pp, pm = p.copy(), p.copy()
        pp[c] += h
        pm[c] -= h
        Ep = cf.plane_direct_coefficients(3.0, pp, half, res, 0.3, 0.5, 16.0, 2).T * pp[5] / A
        Em = cf.plane_direct_coefficients(3.0, pm, half, res, 0.3, 0.5, 16.0, 2).T * pm[5] / A
        ref[c] = float(np.sum(g.astype(np.float64) * (Ep - Em))) / (2 * h)
    grads = np.array([oracle_lib.adjoint(osc, ol, lights.params, 0xA0 + s, N, 1, g[None])[0][0]
                      for s in range(n_seeds)])
    mean, se = grads.mean(0), grads.std(0, ddof=1) / math.sqrt(n_seeds)
    for c in range(6):
        assert abs(mean[c] - ref[c]) < 5 * se[c] + 3e-3 * abs(ref[c]), (c, mean[c], ref[c], se[c])


def test_directional_glossy_bounce_gradient(oracle_lib):
    """Light reflected by a glossy floor onto a Lambertian ceiling, dO/dL on
    the ceiling only (B = 2): the floor's bounce weight pi f(w_in, w_out)
    changes with the incident direction while the floor point stays fixed,
    so the adjoint needs the BRDF term.  Its mean over seeds matches
    seed-averaged central differences with common random numbers."""
    sb = li.SceneBuilder()
    sb.quads([-2.0, -2.0, 0.0], [4.0, 0, 0], [0, 4.0, 0], 0.3, res=(1, 1))
    sb.quads([-2.0, -2.0, 2.5], [4.0, 0, 0], [0, 4.0, 0], 0.7, res=(2, 2))
    sc = sb.build("glossy_floor_ceiling")
    gl = np.array([[0.5, 10.0], [0.0, 1.0]], np.float32)
    p = np.array([[0.2, -0.1, 1.4, 0.25, -0.1, 60.0]], np.float32)
    lights = make_lights([SPOT], [3.0], [(0, 0)], [0], p)
    osc = oracle_lib.OracleScene(sc, glossy=gl, dir_order=1, dir_samples=2)
    ol = oracle_lib.OracleLights(lights)
    g = np.zeros((1, 4, sc.n_texels), np.float32)
    g[0, 0, 1:] = np.array([1.0, 0.7, 1.3, 0.9], np.float32)
    N, B, n_seeds = 1 << 16, 2, 16

    def lin(pp, seed):
        S, _ = oracle_lib.forward(osc, ol, pp, seed, N, B)
        return float(np.sum(g.astype(np.float64) * S.astype(np.float64) * 2.0 ** -32))

    diffs, adjs = [], []
    for s_ in range(n_seeds):
        seed = 0xC0 + 31 * s_
        adj = oracle_lib.adjoint(osc, ol, p, seed, N, B, g)[0][0]
        fd = np.zeros(5)
        for c in range(5):
            h = 2e-3
            pp, pm = p.copy(), p.copy()
            pp[0, c] += h
            pm[0, c] -= h
            fd[c] = (lin(pp, seed) - lin(pm, seed)) / (float(pp[0, c]) - float(pm[0, c]))
        diffs.append(fd - adj[:5])
        adjs.append(adj[:5])
    D, G = np.array(diffs), np.array(adjs)
    se = D.std(0, ddof=1) / math.sqrt(n_seeds)
    gm = np.abs(G.mean(0))
    for c in range(5):
        assert abs(D[:, c].mean()) < 4.5 * se[c] + 0.02 * gm[c], (c, D[:, c].mean(), se[c], gm[c])


# --------------------------------------------------------------------------
# orientation as a rotation vector (Rodrigues)
# --------------------------------------------------------------------------

def test_rotvec_frame_and_jacobian(oracle_lib):
    """The oracle's Rodrigues matrix equals scipy's rotation of the same
    vector, and its Jacobian maps a change of theta to the world rotation it
    causes: R(theta + h e_i) R(theta)^T = exp([h J e_i]x) to first order."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(30)
    for th in [np.array([0.3, -0.2, 0.5]), rng.normal(size=3) * 1.2, np.array([2.5, 0.1, -0.4])]:
        R, J = oracle_lib.rotvec(th)
        assert np.allclose(R, Rotation.from_rotvec(th).as_matrix(), atol=1e-12)
        for i in range(3):
            h = 1e-6
            tp, tm = th.copy(), th.copy()
            tp[i] += h
            tm[i] -= h
            dw = (Rotation.from_rotvec(tp) * Rotation.from_rotvec(tm).inv()).as_rotvec() / (2 * h)
            assert np.allclose(dw, J[:, i], atol=1e-7), (th, i, dw, J[:, i])
    R0, J0 = oracle_lib.rotvec(np.zeros(3))
    assert np.array_equal(R0, np.eye(3)) and np.array_equal(J0, np.eye(3))


@pytest.mark.parametrize("kind", [SPOT, RECT, SOFT])
def test_rotvec_first_hit_derivative(oracle_lib, kind):
    """dlog of the first-hit kernel w.r.t. the rotation vector (the world
    rotation terms mapped by J^T) vs central differences of an independent
    log-irradiance whose frame comes from scipy's rotation of theta."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(40 + kind)
    n = {SPOT: 3.5, RECT: 1.5}.get(kind, 0.0)
    size = {RECT: (0.6, 0.4), SOFT: (0.0, 1.2)}.get(kind, (0, 0))
    done = 0
    while done < 20:
        th = rng.normal(size=3) * 0.3      # tilts the default axis -z
        p7 = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(1.5, 2.5), *th, rng.uniform(10, 100)])
        lights = make_lights([kind], [n], [size], [0], [p7[:6]])
        ol = oracle_lib.OracleLights(lights, rotvec=True)
        x1 = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5), 0.0])
        n1 = np.array([0.0, 0.0, 1.0])
        au = rng.uniform(-0.5, 0.5) * size[0] if kind == RECT else 0.0
        av = rng.uniform(-0.5, 0.5) * size[1] if kind == RECT else 0.0
        R = Rotation.from_rotvec(p7[3:6]).as_matrix()
        d, t, b = -R[:, 2], R[:, 0], R[:, 1]
        y = p7[:3] + au * t + av * b
        cw = float(np.dot(d, (x1 - y) / np.linalg.norm(x1 - y)))
        if cw < 0.2:
            continue
        done += 1
        pp7 = p7.astype(np.float32)[None]
        dl = oracle_lib.first_hit_dlog(ol, pp7, 0, x1.astype(np.float32), y.astype(np.float32),
                                       n1.astype(np.float32), au, av).astype(np.float64)
        _, J = oracle_lib.rotvec(pp7[0, 3:6].astype(np.float64))
        dth = J.T @ dl[3:6]
        pf = pp7[0].astype(np.float64)

        def logE(q):
            Rq = Rotation.from_rotvec(q[3:6]).as_matrix()
            return cf.log_irradiance(kind, n, [q[0], q[1], q[2], 0.0, 0.0, q[6]], x1, n1, au, av, size, R=Rq)

        for c in range(7):
            h = 1e-6 * max(1.0, abs(pf[c]))
            qp, qm = pf.copy(), pf.copy()
            qp[c] += h
            qm[c] -= h
            fd = (logE(qp) - logE(qm)) / (2 * h)
            got = dth[c - 3] if 3 <= c < 6 else dl[c]
            assert abs(got - fd) <= 3e-4 * (abs(fd) + 1.0), (kind, c, got, fd)


def test_rotvec_agrees_with_tilt_angles(oracle_lib):
    """The same frame given as tilt angles and as a rotation vector traces
    the same paths: equal texels, and the tilt derivatives are the world-
    rotation gradient along the rotations the tilts generate (R_y(beta) e_x
    for alpha, e_y for beta)."""
    from scipy.spatial.transform import Rotation
    c1 = li.box_room()
    sc = c1["scene"]
    p6 = np.array([[1.2, 1.0, 2.1, 0.25, -0.2, 40.0], [2.8, 1.9, 2.3, -0.1, 0.3, 60.0]], np.float32)
    lights = make_lights([SPOT, RECT], [3.0, 1.0], [(0, 0), (0.5, 0.3)], [0, 0], p6)
    p7 = np.zeros((2, 7), np.float32)
    for l in range(2):
        R = cf.rot_y(float(p6[l, 4])) @ cf.rot_x(float(p6[l, 3]))
        p7[l, :3] = p6[l, :3]
        p7[l, 3:6] = Rotation.from_matrix(R).as_rotvec()
        p7[l, 6] = p6[l, 5]
    osc = oracle_lib.OracleScene(sc)
    ol6, ol7 = oracle_lib.OracleLights(lights), oracle_lib.OracleLights(lights, rotvec=True)
    N, B, seed = 1 << 16, 3, 0x7E
    S6, _ = oracle_lib.forward(osc, ol6, p6, seed, N, B)
    S7, _ = oracle_lib.forward(osc, ol7, p7, seed, N, B)
    E6, E7 = oracle_lib.fixed_to_float(S6), oracle_lib.fixed_to_float(S7)
    assert np.linalg.norm(E7 - E6) <= 1e-4 * np.linalg.norm(E6)
    g = np.random.default_rng(5).normal(size=(1, sc.n_texels)).astype(np.float32)
    G6, _ = oracle_lib.adjoint(osc, ol6, p6, seed, N, B, g)
    G7, _ = oracle_lib.adjoint_rv(osc, ol7, p7, seed, N, B, g)
    scale = np.abs(G6).max()
    assert np.allclose(G7[:, :3], G6[:, :3], atol=2e-3 * scale) and np.allclose(G7[:, 6], G6[:, 5], rtol=1e-3)
    for l in range(2):
        _, J = oracle_lib.rotvec(p7[l, 3:6].astype(np.float64))
        gw = np.linalg.solve(J.T, G7[l, 3:6])
        ax_a = cf.rot_y(float(p6[l, 4])) @ np.array([1.0, 0, 0])
        assert abs(gw @ ax_a - G6[l, 3]) <= 2e-3 * scale, (l, gw @ ax_a, G6[l, 3])
        assert abs(gw[1] - G6[l, 4]) <= 2e-3 * scale, (l, gw[1], G6[l, 4])


# --------------------------------------------------------------------------
# direct-differentiation map (the comparison beside the contribution map)
# --------------------------------------------------------------------------

def test_tangent_dotted_with_g_is_the_adjoint(oracle_lib):
    """sum_k g_k dE_k/dp_j over the direct-differentiation map of light l is
    the adjoint gradient dO/dp_j of that light: both sum, over the light's
    paths, (Phi_h / A) g at every hit times the first hit's dlog_j."""
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    N, B, seed = 1 << 15, 3, 0x2E
    g = np.random.default_rng(8).normal(size=(1, sc.n_texels)).astype(np.float32)
    grad, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, N, B, g)
    for j in range(6):
        T = oracle_lib.tangent(osc, ol, lights.params, seed, N, B, 0, j).astype(np.float64) * 2.0 ** -32
        lhs = float(np.dot(g[0].astype(np.float64), T))
        assert abs(lhs - grad[0, j]) <= 1e-5 * abs(grad[0, j]) + 1e-9 * np.abs(grad[0]).max(), (j, lhs, grad[0, j])


def test_tangent_direct_vs_quadrature(oracle_lib):
    """Direct light on a plane: the map's texel means are the derivative of
    the texel's expected irradiance (quadrature, central differences)."""
    half, res, N = 3.0, 16, 1 << 18
    p = np.array([0.3, -0.2, 1.4, 0.3, -0.2, 40.0])
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([SPOT], [2.5], [(0, 0)], [0], [p])
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    A = float(sc.texel_area()[0])
    for j in (0, 3, 5):
        h = 1e-4
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        ref = (cf.plane_hit_probability(SPOT, 2.5, pp, None, half, res, q_tex=5) * pp[5] -
               cf.plane_hit_probability(SPOT, 2.5, pm, None, half, res, q_tex=5) * pm[5]) / (2 * h * A)
        Ts = [oracle_lib.tangent(osc, ol, lights.params, sd, N, 1, 0, j).astype(np.float64) * 2.0 ** -32
              for sd in (0x31, 0x32)]
        err = np.linalg.norm((Ts[0] + Ts[1]) / 2 - ref)
        noise = np.linalg.norm(Ts[0] - Ts[1]) / 2
        assert err < 1.6 * noise + 1e-4 * np.linalg.norm(ref), (j, err, noise)


def test_tangent_responds_at_the_target(oracle_lib):
    """Indirect-only target (downward spot under a ceiling, B = 2): the direct
    differentiation map responds on the ceiling, where the light arrives,
    while the adjoint contribution map sits on the floor (the paper's
    contrast between the two)."""
    sb = li.SceneBuilder()
    sb.quads([-8.0, -8.0, 0.0], [16.0, 0, 0], [0, 16.0, 0], 0.6, res=(16, 16))
    sb.quads([-4.0, -4.0, 2.5], [8.0, 0, 0], [0, 8.0, 0], 0.7, res=(16, 16))
    sc = sb.build("floor_ceiling", fixed_res=(16, 16))
    p = np.array([[0.5, -0.3, 1.5, 0.2, 0.1, 100.0]], np.float32)
    lights = make_lights([SPOT], [3.0], [(0, 0)], [0], p)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    g = np.zeros((1, sc.n_texels), np.float32)
    g[0, 256:] = 1.0
    T = oracle_lib.tangent(osc, ol, p, 0x99, 1 << 15, 2, 0, 0).astype(np.float64)
    vote, grad, _ = oracle_lib.votes(osc, ol, p, 0x99, 1 << 15, 2, g, 0, 0)
    assert np.count_nonzero(T[256:]) > 100 and np.all(vote[256:] == 0.0)
    assert abs(float(np.dot(g[0], T * 2.0 ** -32)) / vote.sum() - 1) < 1e-5


def test_cosine_bounce_floor_to_ceiling(oracle_lib):
    """Second hits on a parallel ceiling: floor first-hit density times the
    differential form factor to each ceiling texel (cosine-weighted bounce, rho)."""
    H, h, rho, N = 2.5, 1.5, 0.5, 1 << 20
    sb = li.SceneBuilder()
    sb.quads([-15.0, -15.0, 0.0], [30.0, 0, 0], [0, 30.0, 0], rho, res=(8, 8))
    sb.quads([-6.0, -6.0, H], [12.0, 0, 0], [0, 12.0, 0], 0.7, res=(24, 24))
    sc = sb.build("floor_ceiling", fixed_res=(8, 8))
    light = [0.2, -0.3, h, 0.0, 0.0, 100.0]
    lights = make_lights([SPOT], [4.0], [(0, 0)], [0], [light])
    S, _ = oracle_lib.forward(oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights),
                              lights.params, 0x77, N, 2)
    E = oracle_lib.fixed_to_float(S)[0].astype(np.float64)
    A = sc.texel_area().astype(np.float64)
    ceil = slice(64, 64 + 576)
    counts = E[ceil] * A[ceil] / (light[5] / N * rho)
    # floor first-hit density (per m^2) on a grid, truncated at |x|,|y| <= 8 m
    g = np.arange(-8.0 + 0.04, 8.0, 0.08)
    FX, FY = np.meshgrid(g, g, indexing="xy")
    fx = FX.ravel() - light[0]
    fy = FY.ravel() - light[1]
    r = np.sqrt(fx * fx + fy * fy + h * h)
    dens = (4 + 1) / (2 * np.pi) * (h / r) ** 4 * (h / r) / r ** 2 * 0.08 ** 2
    edges = np.linspace(-6.0, 6.0, 25)
    prob = np.zeros(576)
    for j in range(24):
        for i in range(24):
            F = cf.rect_form_factor(edges[i] - FX.ravel(), edges[i + 1] - FX.ravel(),
                                    edges[j] - FY.ravel(), edges[j + 1] - FY.ravel(), H)
            prob[j * 24 + i] = np.sum(dens * F)
    _binomial_check(counts, prob, N, min_expect=100.0)


# --------------------------------------------------------------------------
# P2: energy conservation in closed boxes
# --------------------------------------------------------------------------

def test_closed_box_uniform_albedo(oracle_lib):
    rho, B, N, P = 0.6, 5, 1 << 18, 50.0
    sc = li.closed_box(albedo=rho)
    lights = make_lights([POINT, SPOT], [0.0, 3.0], [(0, 0)] * 2, [0, 0],
                         [[0.7, 0.6, 0.5, 0, 0, P], [1.3, 0.9, 0.8, 0.3, -0.2, 2 * P]])
    S, misses = oracle_lib.forward(oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights),
                                   lights.params, 0x99, N, B)
    assert misses == 0
    A = sc.texel_area().astype(np.float64)
    total = float(np.sum(A * S[0].astype(np.float64) * 2.0 ** -32))
    expect = 3 * P * (1 - rho ** B) / (1 - rho)
    assert abs(total / expect - 1) < 1e-6, total / expect - 1


def test_closed_box_absorbs_all_flux(oracle_lib):
    B, N, P = 64, 1 << 16, 10.0
    alb = np.array([0.55, 0.6, 0.65, 0.7, 0.75, 0.5], np.float32)
    sc = li.closed_box(albedo=alb)
    lights = make_lights([SPOT], [2.0], [(0, 0)], [0], [[1.0, 0.7, 0.6, 0.4, 0.1, P]])
    S, misses = oracle_lib.forward(oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights),
                                   lights.params, 0x5, N, B)
    assert misses == 0
    A = sc.texel_area().astype(np.float64)
    rho_k = np.repeat(alb.astype(np.float64), 256)
    absorbed = float(np.sum((1 - rho_k) * A * S[0].astype(np.float64) * 2.0 ** -32))
    assert abs(absorbed / P - 1) < 1e-5 + 0.75 ** B


def test_zero_power_luminaire_adds_nothing(oracle_lib):
    """Alg. 1 gives every path of a luminaire the flux P / N: at zero power
    all its splats are zero, so the forward pass that skips it equals one
    that traces it at a power too small to reach one fixed-point unit, and
    the other luminaires' texels are those of the full run less its share."""
    sc = li.closed_box(albedo=0.6)
    base = [[0.7, 0.6, 0.5, 0, 0, 40.0], [1.3, 0.9, 0.8, 0.3, -0.2, 60.0], [1.0, 1.2, 0.9, -0.1, 0.2, 30.0]]
    lights = make_lights([POINT, SPOT, POINT], [0.0, 3.0, 0.0], [(0, 0)] * 3, [0, 0, 0], base)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    N, B, seed = 3 * 4096 + 2, 4, 0x2E0

    def fwd(p1):
        p = lights.params.copy()
        p[1, 5] = p1
        return oracle_lib.forward(osc, ol, p, seed, N, B)[0]

    S_zero, S_tiny, S_full = fwd(0.0), fwd(1e-30), fwd(60.0)
    assert np.array_equal(S_zero, S_tiny)
    assert np.count_nonzero(S_full - S_zero) > 0
    only = lights.params.copy()
    only[0, 5] = only[2, 5] = 0.0
    S_only = oracle_lib.forward(osc, ol, only, seed, N, B)[0]
    assert np.array_equal(S_full - S_zero, S_only)
    # the adjoint: each luminaire's row sums its own paths only, so the other
    # rows are unchanged (up to the threads' summation order) and the
    # zero-power row is zero
    g = oracle_lib.fixed_to_float(S_full).astype(np.float32) - 1.0
    p_zero = lights.params.copy()
    p_zero[1, 5] = 0.0
    G_full, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, N, B, g)
    G_zero, _ = oracle_lib.adjoint(osc, ol, p_zero, seed, N, B, g)
    assert np.all(G_zero[1] == 0.0) and np.any(G_full[1] != 0.0)
    assert np.allclose(G_zero[[0, 2]], G_full[[0, 2]], rtol=1e-12, atol=0.0)


# --------------------------------------------------------------------------
# objective and fixed point
# --------------------------------------------------------------------------

def test_fixed_point_exact(oracle_lib):
    S = np.array([0, 1 << 32, 3 << 31, -(5 << 32), 1], np.int64)
    E = oracle_lib.fixed_to_float(S)
    assert E.tolist() == [0.0, 1.0, 1.5, -5.0, 2.0 ** -32]


def test_objective_definition(oracle_lib):
    rng = np.random.default_rng(1)
    K = 300
    A = rng.uniform(0.01, 0.2, K).astype(np.float32)
    Et = rng.uniform(0, 5, K).astype(np.float32)
    al = rng.uniform(0, 2, K).astype(np.float32)
    O0, g0 = oracle_lib.objective(Et, Et, A, al)
    assert O0 == 0.0 and not g0.any()
    E = (Et + rng.normal(0, 0.5, K)).astype(np.float32)
    O, g = oracle_lib.objective(E, Et, A, al)
    assert O > 0
    # g = dO/dE by central differences in the exact arithmetic of the sum
    for k in rng.choice(K, 10, replace=False):
        h = 1e-2
        Ep, Em = E.copy(), E.copy()
        Ep[k] += h
        Em[k] -= h
        fd = (oracle_lib.objective(Ep, Et, A, al)[0] - oracle_lib.objective(Em, Et, A, al)[0]) / \
            (float(Ep[k]) - float(Em[k]))
        assert abs(fd - g[k]) <= 1e-5 * (abs(g[k]) + 1e-3)
    # quadratic scaling
    O2, _ = oracle_lib.objective((Et + 2 * (E - Et)).astype(np.float32), Et, A, al)
    assert abs(O2 / O - 4) < 1e-5


# --------------------------------------------------------------------------
# derivatives: first-hit dlog vs FD of an independent log-irradiance
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [POINT, SPOT, RECT, SOFT])
def test_first_hit_derivative(oracle_lib, kind):
    rng = np.random.default_rng(10 + kind)
    n = 0.0 if kind in (POINT, SOFT) else 3.5
    size = {RECT: (0.6, 0.4), SOFT: (0.3, 1.2)}.get(kind, (0, 0))
    done = 0
    while done < 20:
        p = [rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(1.5, 2.5),
             rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), rng.uniform(10, 100)]
        if kind == POINT:
            p[3] = p[4] = 0.0
        lights = make_lights([kind], [n], [size], [0], [p])
        ol = oracle_lib.OracleLights(lights)
        pf = np.asarray(lights.params[0], np.float64)
        x1 = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5), 0.0])
        n1 = np.array([0.0, 0.0, 1.0])
        au = rng.uniform(-0.5, 0.5) * size[0] if kind == RECT else 0.0
        av = rng.uniform(-0.5, 0.5) * size[1] if kind == RECT else 0.0
        d, t, b = cf.frame(pf[3], pf[4])
        y = pf[:3] + au * t + av * b
        if kind == SOFT:
            # inside the outer cone and away from the inner cone's kink
            cw = float(np.dot(d, (x1 - y) / np.linalg.norm(x1 - y)))
            if cw <= math.cos(size[1]) + 1e-3 or abs(cw - math.cos(size[0])) < 1e-3:
                continue
        done += 1
        dl = oracle_lib.first_hit_dlog(ol, lights.params, 0, x1.astype(np.float32), y.astype(np.float32),
                                       n1.astype(np.float32), au, av).astype(np.float64)
        for c in range(6):
            hstep = 1e-6 * max(1.0, abs(pf[c]))
            pp, pm = pf.copy(), pf.copy()
            pp[c] += hstep
            pm[c] -= hstep
            fd = (cf.log_irradiance(kind, n, pp, x1, n1, au, av, size) -
                  cf.log_irradiance(kind, n, pm, x1, n1, au, av, size)) / (2 * hstep)
            if kind == POINT and c in (3, 4):
                assert dl[c] == 0.0
                continue
            assert abs(dl[c] - fd) <= 2e-4 * (abs(fd) + 1.0), (kind, c, dl[c], fd)


def test_light_frame_convention(oracle_lib):
    rng = np.random.default_rng(3)
    P = rng.uniform(-1.2, 1.2, (8, 2))
    params = np.zeros((8, 6), np.float32)
    params[:, 3:5] = P
    params[:, 5] = 1.0
    lights = make_lights([SPOT] * 8, [1.0] * 8, [(0, 0)] * 8, [0] * 8, params)
    fr = oracle_lib.light_frames(oracle_lib.OracleLights(lights), lights.params, 1000)
    for k in range(8):
        d, t, b = cf.frame(float(params[k, 3]), float(params[k, 4]))
        assert np.allclose(fr[k, 3:6], d, atol=3e-7) and np.allclose(fr[k, 6:9], t, atol=3e-7)
        assert np.allclose(fr[k, 9:12], b, atol=3e-7)
        assert fr[k, 28] == 125 and abs(fr[k, 27] - 1.0 / 125) < 1e-9   # 1000 paths over 8 lights


# --------------------------------------------------------------------------
# P5: intensity identity  dO/dP = (1/P) sum_k g_k E_k
# --------------------------------------------------------------------------

def test_intensity_identity(oracle_lib):
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    N, B, seed = 1 << 17, 3, 0x42
    S, _ = oracle_lib.forward(osc, ol, lights.params, seed, N, B)
    E = oracle_lib.fixed_to_float(S)
    Et = li.painted_target(sc, 20.0, seed=4)[None]
    O, g = oracle_lib.objective(E, Et, sc.texel_area())
    grad, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, N, B, g)
    P = float(lights.params[0, 5])
    expect = float(np.sum(g.astype(np.float64) * E.astype(np.float64))) / P
    assert abs(grad[0, 5] / expect - 1) < 2e-5


def test_record_matches_adjoint(oracle_lib):
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    N, B, seed = 1 << 12, 3, 0x43
    g = np.random.default_rng(0).normal(size=(1, sc.n_texels)).astype(np.float32)
    grad, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, N, B, g)
    prim, tex, contrib = oracle_lib.record(osc, ol, lights.params, seed, N, B, 0, 0, 0, N, g)
    assert np.allclose(contrib.astype(np.float64).sum(0), grad[0], rtol=1e-9, atol=1e-12)
    assert (prim[:, 0] >= 0).all() and (tex >= -1).all()


# --------------------------------------------------------------------------
# P7: direct-only gradient vs quadrature derivative (plane, B = 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [POINT, SPOT, RECT, SOFT])
def test_direct_gradient_vs_quadrature(oracle_lib, kind):
    half, res, N = 3.0, 24, 1 << 18
    n = 2.5 if kind in (SPOT, RECT) else 0.0
    size = {RECT: (0.7, 0.4), SOFT: (0.35, 0.9)}.get(kind, (0, 0))
    p = np.array([0.3, -0.2, 1.4, 0.3 if kind else 0.0, -0.2 if kind else 0.0, 40.0])
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([kind], [n], [size], [0], [p])
    A = float(sc.texel_area()[0])
    rng = np.random.default_rng(7)
    g = rng.uniform(-1, 1, sc.n_texels).astype(np.float32)

    def expected_E(pp):
        return cf.plane_hit_probability(kind, n, pp, size, half, res, q_tex=5, q_light=5) * pp[5] / A

    ref = np.zeros(6)
    for c in range(6):
        h = 1e-4
        pp, pm = p.copy(), p.copy()
        pp[c] += h
        pm[c] -= h
        ref[c] = np.dot(g.astype(np.float64), (expected_E(pp) - expected_E(pm)) / (2 * h))
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    prim, tex, contrib = oracle_lib.record(osc, ol, lights.params, 0xD1, N, 1, 0, 0, 0, N, g[None])
    c64 = contrib.astype(np.float64)
    est = c64.sum(0)
    sigma = c64.std(0) * math.sqrt(N)
    for c in range(6):
        if kind == POINT and c in (3, 4):
            assert est[c] == 0.0
            continue
        assert abs(est[c] - ref[c]) < 4.5 * sigma[c] + 1e-3 * abs(ref[c]), (c, est[c], ref[c], sigma[c])


# --------------------------------------------------------------------------
# gradient-contribution map (Sec. gradVis)
# --------------------------------------------------------------------------

def test_votes_power_direct_equals_forward(oracle_lib):
    """B = 1, parameter P: every path's contribution is g_k invA_k Phi_r / P,
    so the map equals g_k E_k / P with E_k from the primal splat."""
    sc = li.plane_scene(half=3.0, res=24)
    p = np.array([[0.3, -0.2, 1.4, 0.2, -0.1, 40.0]], np.float32)
    lights = make_lights([SPOT], [2.5], [(0, 0)], [0], p)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    N, seed = 1 << 16, 0x5150
    g = np.random.default_rng(3).uniform(-1, 1, (1, sc.n_texels)).astype(np.float32)
    S, _ = oracle_lib.forward(osc, ol, p, seed, N, 1)
    E = oracle_lib.fixed_to_float(S)[0].astype(np.float64)
    vote, grad, _ = oracle_lib.votes(osc, ol, p, seed, N, 1, g, 0, 5)
    ref = g[0].astype(np.float64) * E / float(p[0, 5])
    assert (E > 0).sum() > 300
    assert np.all(np.abs(vote - ref) <= 2e-6 * np.abs(ref) + 1e-15)
    assert abs(vote.sum() / grad[5] - 1) < 1e-9


def test_votes_partition_the_gradient(oracle_lib):
    """Box room, B = 3, every parameter: the map is the first-hit texel
    histogram of the per-path contributions (recorded path by path) and sums
    to the light's gradient."""
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    N, B, seed = 1 << 13, 3, 0x77
    g = np.random.default_rng(5).normal(size=(1, sc.n_texels)).astype(np.float32)
    grad_all, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, N, B, g)
    prim, tex, contrib = oracle_lib.record(osc, ol, lights.params, seed, N, B, 0, 0, 0, N, g)
    first = tex[:, 0]
    for j in range(6):
        vote, grad, _ = oracle_lib.votes(osc, ol, lights.params, seed, N, B, g, 0, j)
        assert np.allclose(grad, grad_all[0], rtol=1e-12, atol=0)
        ok = first >= 0
        ref = np.bincount(first[ok], weights=contrib[ok, j].astype(np.float64), minlength=sc.n_texels)
        scale = np.abs(contrib[:, j]).astype(np.float64).sum()
        assert np.all(np.abs(vote - ref) <= 1e-12 * scale)
        assert abs(vote.sum() - grad[j]) <= 1e-12 * scale
        assert np.count_nonzero(vote) == np.count_nonzero(np.bincount(first[ok], minlength=sc.n_texels))


def test_votes_sit_at_the_first_hit(oracle_lib):
    """A target that only indirect light reaches: a downward spot under a
    ceiling, dO/dE non-zero on the ceiling alone.  The contributions are
    drawn on the floor, where the paths first hit, and none on the ceiling."""
    sb = li.SceneBuilder()
    sb.quads([-8.0, -8.0, 0.0], [16.0, 0, 0], [0, 16.0, 0], 0.6, res=(16, 16))
    sb.quads([-4.0, -4.0, 2.5], [8.0, 0, 0], [0, 8.0, 0], 0.7, res=(16, 16))
    sc = sb.build("floor_ceiling", fixed_res=(16, 16))
    p = np.array([[0.5, -0.3, 1.5, 0.2, 0.1, 100.0]], np.float32)
    lights = make_lights([SPOT], [3.0], [(0, 0)], [0], p)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    g = np.zeros((1, sc.n_texels), np.float32)
    g[0, 256:] = 1.0
    vote, grad, _ = oracle_lib.votes(osc, ol, p, 0x99, 1 << 15, 2, g, 0, 0)
    assert np.all(vote[256:] == 0.0)
    assert np.count_nonzero(vote[:256]) > 100
    assert grad[0] != 0.0 and abs(vote.sum() / grad[0] - 1) < 1e-9


@pytest.mark.parametrize("kind", [SPOT, RECT])
def test_votes_direct_vs_quadrature_per_texel(oracle_lib, kind):
    """B = 1: the expected map is g_k times the derivative of the texel's
    expected irradiance (the texel is fixed, so differentiation passes under
    the integral over it); checked texel by texel against central differences
    of the independent quadrature, with the per-texel variance estimated from
    the recorded paths."""
    half, res, N = 3.0, 16, 1 << 18
    n = 2.5
    size = (0.7, 0.4) if kind == RECT else (0, 0)
    p = np.array([0.3, -0.2, 1.4, 0.3, -0.2, 40.0])
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([kind], [n], [size], [0], [p])
    A = float(sc.texel_area()[0])
    g = np.random.default_rng(9).uniform(0.2, 1.0, sc.n_texels).astype(np.float32)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    seed = 0xE1
    _, tex, contrib = oracle_lib.record(osc, ol, lights.params, seed, N, 1, 0, 0, 0, N, g[None])
    first = tex[:, 0]
    ok = first >= 0
    counts = np.bincount(first[ok], minlength=sc.n_texels)
    m = counts >= 200
    assert m.sum() > 60

    def expected_E(pp):
        return cf.plane_hit_probability(kind, n, pp, size, half, res, q_tex=5, q_light=5) * pp[5] / A

    zs = []
    for j in range(6):
        vote, _, _ = oracle_lib.votes(osc, ol, lights.params, seed, N, 1, g[None], 0, j)
        h = 1e-4
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        ref = g.astype(np.float64) * (expected_E(pp) - expected_E(pm)) / (2 * h)
        c = contrib[ok, j].astype(np.float64)
        var = np.bincount(first[ok], weights=c * c, minlength=sc.n_texels) - vote ** 2 / N
        z = (vote[m] - ref[m]) / np.sqrt(var[m])
        assert np.abs(z).max() < 5.5, (j, np.abs(z).max())
        zs.append(z)
    z = np.concatenate(zs)
    assert abs(float((z ** 2).mean()) - 1) < 6 * math.sqrt(2 / z.size) + 0.05


# --------------------------------------------------------------------------
# P6: adjoint vs central finite differences with common random numbers
# --------------------------------------------------------------------------

@pytest.mark.slow
def test_adjoint_vs_fd_common_random_numbers(oracle_lib):
    """Occluder-free closed room (the box room without its boxes), B = 3.

    For each seed the central difference uses the same seed at p +- h
    (correlated evaluation) and the adjoint uses it too; a single seed's FD is
    dominated by texel-boundary crossings, so the check is on the mean of the
    difference over seeds against its standard error (and < 3 % of the
    gradient).  The power component agrees per seed to 1e-4."""
    rng = np.random.default_rng(11)
    sb = li.SceneBuilder()
    sb.boxes([0, 0, 0], [4.0, 3.0, 2.5], 0.6, res=(32, 32))
    sc = sb.build("empty_room", fixed_res=(32, 32))
    sc.patches["albedo"] = rng.uniform(0.5, 0.8, 6).astype(np.float32)
    p = np.array([[1.7, 1.4, 2.0, 0.25, -0.2, 100.0]], np.float32)
    lights = make_lights([SPOT], [4.0], [(0, 0)], [0], p)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    N, B, h = 1 << 20, 3, 0.03
    A = sc.texel_area()
    Et = li.painted_target(sc, 30.0, seed=2, wavelength=3.0)[None]
    diffs, grads = [], []
    for s in range(8):
        seed = 0xF00D + 977 * s
        S, _ = oracle_lib.forward(osc, ol, p, seed, N, B)
        _, g = oracle_lib.objective(oracle_lib.fixed_to_float(S), Et, A)
        grad, _ = oracle_lib.adjoint(osc, ol, p, seed, N, B, g)

        def O_at(pp):
            S_, _ = oracle_lib.forward(osc, ol, pp, seed, N, B)
            return oracle_lib.objective(oracle_lib.fixed_to_float(S_), Et, A)[0]

        fd = []
        for c in range(6):
            hh = h * (100.0 if c == 5 else 1.0)
            pp, pm = p.copy(), p.copy()
            pp[0, c] += hh
            pm[0, c] -= hh
            fd.append((O_at(pp) - O_at(pm)) / (float(pp[0, c]) - float(pm[0, c])))
        assert abs(fd[5] / grad[0, 5] - 1) < 1e-4
        diffs.append(np.array(fd[:5]) - grad[0, :5])
        grads.append(grad[0, :5])
    D, G = np.array(diffs), np.array(grads)
    se = D.std(0, ddof=1) / math.sqrt(D.shape[0])
    gm = np.abs(G.mean(0))
    for c in range(5):
        assert abs(D[:, c].mean()) < 4 * se[c] + 1e-3 * gm[c], (c, D[:, c].mean(), se[c])
        if gm[c] > 0.1 * gm.max():
            assert abs(D[:, c].mean()) < 0.03 * gm[c]


# --------------------------------------------------------------------------
# emission proposal: MIS unbiasedness, hemi-octahedral Jacobian, MLP backprop
# --------------------------------------------------------------------------

def test_hemi_octahedral_cells_cover_the_hemisphere():
    """Sum over cells of the cell solid angle (du dv / (2 |p|^3)) = 2 pi."""
    g = (np.arange(512) + 0.5) / 512 * 2 - 1
    U, V = np.meshgrid(g, g)
    xp, yp = (U + V) / 2, (U - V) / 2
    zp = 1 - np.abs(xp) - np.abs(yp)
    dA = (2.0 / 512) ** 2
    omega = np.sum(dA / (2 * np.sqrt(xp ** 2 + yp ** 2 + zp ** 2) ** 3))
    assert abs(omega / (2 * np.pi) - 1) < 1e-4
    assert zp.min() >= 0


def _random_table(rng, L, peaky=3.0):
    logits = rng.normal(0, peaky, (L, 1024))
    p = np.exp(logits - logits.max(1, keepdims=True))
    return (p / p.sum(1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("kind", [SPOT, RECT])
def test_proposal_direct_gradient_unbiased(oracle_lib, kind):
    """With a random proposal table and alpha = 0.2 the first-hit gradient is
    still the quadrature derivative (plane, B = 1)."""
    from oracle.proposal import cdf_table
    half, res, N = 3.0, 24, 1 << 18
    n = 2.5
    size = (0.7, 0.4) if kind == RECT else (0, 0)
    p = np.array([0.3, -0.2, 1.4, 0.3, -0.2, 40.0])
    sc = li.plane_scene(half=half, res=res)
    lights = make_lights([kind], [n], [size], [0], [p])
    A = float(sc.texel_area()[0])
    rng = np.random.default_rng(17)
    g = rng.uniform(-1, 1, sc.n_texels).astype(np.float32)
    pdf = _random_table(rng, 1)
    prop = oracle_lib.Proposal(pdf, cdf_table(pdf), 0.2)

    def expected_E(pp):
        return cf.plane_hit_probability(kind, n, pp, size, half, res, q_tex=5, q_light=5) * pp[5] / A

    ref = np.zeros(6)
    for c in range(6):
        h = 1e-4
        pp, pm = p.copy(), p.copy()
        pp[c] += h
        pm[c] -= h
        ref[c] = np.dot(g.astype(np.float64), (expected_E(pp) - expected_E(pm)) / (2 * h))
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    _, _, contrib = oracle_lib.record(osc, ol, lights.params, 0xD7, N, 1, 0, 0, 0, N, g[None], proposal=prop)
    c64 = contrib.astype(np.float64)
    est, sigma = c64.sum(0), c64.std(0) * math.sqrt(N)
    for c in range(6):
        assert abs(est[c] - ref[c]) < 4.5 * sigma[c] + 1e-3 * abs(ref[c]), (c, est[c], ref[c], sigma[c])
    # texel expectation: the irradiance of the whole plane is unchanged
    S, _ = oracle_lib.forward(osc, ol, lights.params, 0xD8, N, 1, proposal=prop)
    tot = float(oracle_lib.fixed_to_float(S)[0].astype(np.float64).sum() * A)
    tot_ref = float(expected_E(p).sum() * A)
    assert abs(tot / tot_ref - 1) < 0.02


def test_proposal_histogram_signal(oracle_lib):
    """The adjoint histogram adds |c_r * inv_sigma|^2 * q / (512 |p|^3) into the
    path's emission cell.  With a uniform cell table and a vanishing plain
    share, q / (512 |p|^3) is (1 - alpha) / 1024 up to the plain share's
    alpha * p_plain / (512 |p|^3) <= 1e-8, so the histogram total is fixed by the
    recorded contributions."""
    from oracle.proposal import cdf_table
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    rng = np.random.default_rng(2)
    pdf = np.full((1, 1024), 1.0 / 1024, np.float32)
    inv_sigma = rng.uniform(0.5, 2.0, (1, 6)).astype(np.float32)
    alpha = 1e-6
    prop = oracle_lib.Proposal(pdf, cdf_table(pdf), alpha, inv_sigma=inv_sigma, with_hist=True)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    g = rng.normal(size=(1, sc.n_texels)).astype(np.float32)
    N = 1 << 12
    grad, _ = oracle_lib.adjoint(osc, ol, lights.params, 9, N, 3, g, proposal=prop)
    hist_total = float(prop.hist.sum())
    _, _, contrib = oracle_lib.record(osc, ol, lights.params, 9, N, 3, 0, 0, 0, N, g, proposal=prop)
    m2 = ((contrib.astype(np.float64) * inv_sigma) ** 2).sum(1)
    assert abs(hist_total / (m2.sum() * (1 - alpha) / 1024) - 1) < 1e-4
    assert np.allclose(contrib.astype(np.float64).sum(0), grad[0], rtol=1e-9, atol=1e-12)


def test_proposal_histogram_sampler_independent(oracle_lib):
    """Per cell, the histogram's expectation does not depend on the sampler:
    a poor random table with a small plain share and the plain-heavy mixture
    give the same cell sums within their statistical error (seed averages,
    coarse 8 x 8 blocks of cells)."""
    from oracle.proposal import cdf_table
    c1 = li.box_room()
    sc, lights = c1["scene"], c1["lights"]
    rng = np.random.default_rng(4)
    g = (rng.normal(size=(1, sc.n_texels)) + 0.5).astype(np.float32)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    inv_sigma = np.ones((1, 6), np.float32)
    runs = {}
    for name, pdf, alpha in (("random", _random_table(rng, 1), 0.1),
                             ("plain-heavy", np.full((1, 1024), 1.0 / 1024, np.float32), 0.9)):
        H = []
        for s in range(12):
            prop = oracle_lib.Proposal(pdf, cdf_table(pdf), alpha, inv_sigma=inv_sigma, with_hist=True)
            oracle_lib.adjoint(osc, ol, lights.params, 100 + s, 1 << 14, 3, g, proposal=prop)
            H.append(prop.hist[0].reshape(8, 4, 8, 4).sum((1, 3)).ravel())
        runs[name] = np.array(H)
    a, b = runs["random"], runs["plain-heavy"]
    se = np.sqrt(a.var(0, ddof=1) / len(a) + b.var(0, ddof=1) / len(b))
    big = a.mean(0) + b.mean(0) > 1e-3 * (a.mean(0) + b.mean(0)).max()
    z = np.abs(a.mean(0) - b.mean(0))[big] / np.maximum(se[big], 1e-30)
    assert np.median(z) < 1.5 and z.max() < 6.0, (np.median(z), z.max())
    assert abs(a.sum(1).mean() / b.sum(1).mean() - 1) < 0.1


def test_mlp_backprop_matches_finite_differences():
    from oracle import proposal as op
    rng = np.random.default_rng(3)
    L = 5
    w = rng.normal(0, 0.2, op.N_WEIGHTS)
    x = np.zeros((L, op.IN))
    x[:, :op.NPAR + op.NEMB] = rng.normal(0, 1, (L, op.NPAR + op.NEMB))
    t = rng.dirichlet(np.ones(op.BINS), L)
    loss, g, gx = op.loss_and_grad(w, x, t)
    for k in list(rng.choice(op.N_WEIGHTS, 25, replace=False)) + [op.OFF_B1 + 3, op.OFF_B3 + 7]:
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (op.loss_and_grad(wp, x, t)[0] - op.loss_and_grad(wm, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 + 1e-5 * abs(g[k])
    for (r, c) in [(0, 6), (2, 13), (4, 21)]:
        xp, xm = x.copy(), x.copy()
        xp[r, c] += 1e-6
        xm[r, c] -= 1e-6
        fd = (op.loss_and_grad(w, xp, t)[0] - op.loss_and_grad(w, xm, t)[0]) / 2e-6
        assert abs(fd - gx[r, c]) < 1e-6 + 1e-5 * abs(gx[r, c])
    # a softmax cross-entropy lower bound: loss >= entropy of the target
    assert loss >= float(-(t * np.log(t)).sum() / L) - 1e-9


def _cell_mass_spherical(n, res=32, nt=400, nph=800):
    """Independent check: integrate (n+1)/(2 pi) cos^n theta over the
    hemisphere in (theta, phi) and bin each direction into its hemi-octahedral
    cell (u = x' + y', v = x' - y' with (x', y') = (x, y) / (|x| + |y| + z))."""
    th = (np.arange(nt) + 0.5) * (math.pi / 2) / nt
    ph = (np.arange(nph) + 0.5) * (2 * math.pi) / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    x, y, z = np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)
    s = np.abs(x) + np.abs(y) + z
    u, v = (x + y) / s, (x - y) / s
    iu = np.clip(np.floor((u + 1) * res / 2).astype(int), 0, res - 1)
    iv = np.clip(np.floor((v + 1) * res / 2).astype(int), 0, res - 1)
    w = (n + 1) / (2 * math.pi) * z ** n * np.sin(T) * (math.pi / 2 / nt) * (2 * math.pi / nph)
    m = np.zeros(res * res)
    np.add.at(m, (iv * res + iu).ravel(), w.ravel())
    return m


@pytest.mark.parametrize("n", [0.0, 1.0, 4.0])
def test_plain_cell_mass(n):
    """The plain lobe's cell masses (midpoint rule on the hemi-octahedral
    map, its Jacobian 1/(2|p|^3)) against an independent integration of the
    lobe over the hemisphere in (theta, phi), each direction binned into its
    cell: rows sum to one and 4 x 4 blocks of cells agree."""
    from oracle import proposal as op
    m = op.plain_cell_mass([n], sub=16)[0]
    ref = _cell_mass_spherical(n)
    assert abs(m.sum() - 1) < 1e-12 and abs(ref.sum() - 1) < 2e-3
    mb = m.reshape(8, 4, 8, 4).sum((1, 3))
    rb = ref.reshape(8, 4, 8, 4).sum((1, 3))
    assert np.max(np.abs(mb - rb)) < 2e-3


def test_plain_cell_mass_vs_sampled_lobe():
    """Directions drawn from the cos^n lobe by inverting its CDF (cos theta =
    u^(1/(n+1))) fall into the cells with the quadrature's probabilities
    (chi-square over the cells)."""
    from oracle import proposal as op
    rng = np.random.default_rng(17)
    for n in (1.0, 5.0):
        N = 2_000_000
        ct = rng.uniform(0, 1, N) ** (1.0 / (n + 1.0))
        ph = rng.uniform(0, 2 * math.pi, N)
        st = np.sqrt(1 - ct * ct)
        x, y = st * np.cos(ph), st * np.sin(ph)
        s = np.abs(x) + np.abs(y) + ct
        iu = np.clip(np.floor((x / s + y / s + 1) * 16).astype(int), 0, 31)
        iv = np.clip(np.floor((x / s - y / s + 1) * 16).astype(int), 0, 31)
        cnt = np.bincount(iv * 32 + iu, minlength=1024)
        e = op.plain_cell_mass([n])[0] * N
        keep = e > 20
        chi2 = ((cnt[keep] - e[keep]) ** 2 / e[keep]).sum()
        dof = keep.sum() - 1
        assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof), (n, chi2, dof)


def test_training_target():
    """The proposal's training target: per light, the normalised square root
    of the running average of the normalised histogram (the variance-optimal
    cell probabilities for a second-moment histogram), an empty row counting
    as uniform, mixed with the plain lobe's masses; a histogram equal to the
    plain masses squared gives back the plain masses for any mixing share."""
    from oracle import proposal as op
    h = np.zeros((2, 4))
    h[0] = [4.0, 0.0, 1.0, 11.0]
    t, avg = op.training_target(h, None, 0.5)
    r = np.sqrt(np.array([4.0, 0.0, 1.0, 11.0]) / 16)
    assert np.allclose(t[0], r / r.sum()) and np.allclose(t[1], 0.25)
    h2 = np.array([[0.0, 0.0, 0.0, 8.0], [1.0, 1.0, 1.0, 1.0]])
    pm = np.array([[0.1, 0.2, 0.3, 0.4]] * 2)
    t2, avg2 = op.training_target(h2, avg, 0.75, pm, 0.3)
    a = 0.75 * avg + 0.25 * (h2 / h2.sum(1, keepdims=True))
    r2 = np.sqrt(a)
    assert np.allclose(avg2, a)
    assert np.allclose(t2, 0.7 * r2 / r2.sum(1, keepdims=True) + 0.3 * pm)
    assert np.allclose(t2.sum(1), 1.0)
    pmc = op.plain_cell_mass([0.0, 3.0])
    for floor in (0.0, 0.3, 1.0):
        t3, _ = op.training_target(7.0 * pmc ** 2, None, 0.9, pmc, floor)
        assert np.allclose(t3, pmc, rtol=1e-12, atol=0)


def test_mlp_admissible_roundings():
    """The set of admissible bfloat16 roundings of the hidden activations
    (what FP32 accumulation in an unknown order may produce) always holds
    the nominal round-to-nearest-even network, and is exactly it when the
    accumulation bound is zero; a network that truncates its activations to
    bfloat16 instead is admissible for almost no light."""
    from oracle import proposal as op
    rng = np.random.default_rng(9)
    L = 24
    w = rng.normal(0, 0.15, op.N_WEIGHTS).astype(np.float32)
    x = np.zeros((L, op.IN), np.float32)
    x[:, :op.NPAR + op.NEMB] = rng.normal(0, 1, (L, op.NPAR + op.NEMB))
    z, p = op.infer(w, x)
    alts = op.infer_alternatives(w, x)
    exact = op.infer_alternatives(w, x, tol=0.0)
    for r in range(L):
        assert min(np.abs(zz - z[r]).max() for zz, _ in alts[r]) < 1e-12
        assert len(exact[r]) == 1 and np.abs(exact[r][0][0] - z[r]).max() < 1e-12
    # truncation instead of rounding to nearest even
    def trunc(a):
        u = np.ascontiguousarray(a, np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
        return u.view(np.float32).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = op.unpack(op.bf16_round(w).astype(np.float64))
    xb = op.bf16_round(x).astype(np.float64)
    h1 = trunc(np.maximum(xb @ W1.T + b1, 0.0).astype(np.float32))
    h2 = trunc(np.maximum(h1 @ W2.T + b2, 0.0).astype(np.float32))
    zt = h2 @ W3.T + b3
    ok = sum(min(np.abs(zz - zt[r]).max() / np.abs(zz).max() for zz, _ in alts[r]) <= 1e-5 for r in range(L))
    assert ok <= 1


def test_tangent_vs_central_differences_convex_room(oracle_lib):
    """In a convex room (no shadow edges to sweep) the direct-differentiation
    map and central differences of the primal with common random numbers
    estimate the same derivative: their seed means agree patch by patch
    within the noise the seeds show, for a spot's x and tilt, while the
    derivative itself stands well above that noise."""
    sb = li.SceneBuilder()
    sb.boxes([0, 0, 0], [4.0, 3.0, 2.5], 0.6, res=(12, 12))
    sc = sb.build("empty_room", fixed_res=(12, 12))
    p = np.array([[1.6, 1.2, 2.0, 0.3, -0.2, 40.0]], np.float32)
    lights = make_lights([SPOT], [3.0], [(0, 0)], [0], p)
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    N, B, n_seeds = 1 << 16, 3, 8
    ends = np.cumsum(sc.patch_res().prod(1))
    starts = np.concatenate([[0], ends[:-1]])
    A = sc.texel_area().astype(np.float64)

    def per_patch(E):           # d(flux)/dp of each patch
        return np.add.reduceat(E * A, starts)

    for j, h in ((0, 0.05), (3, 0.02)):
        T, F = [], []
        for s in range(n_seeds):
            seed = 0x600 + s
            T.append(per_patch(oracle_lib.tangent(osc, ol, p, seed, N, B, 0, j).astype(np.float64) * 2.0 ** -32))
            pp, pm = p.copy(), p.copy()
            pp[0, j] += h
            pm[0, j] -= h
            Sp, _ = oracle_lib.forward(osc, ol, pp, seed, N, B)
            Sm, _ = oracle_lib.forward(osc, ol, pm, seed, N, B)
            step = float(np.float64(pp[0, j]) - np.float64(pm[0, j]))
            F.append(per_patch((Sp[0] - Sm[0]).astype(np.float64) * 2.0 ** -32 / step))
        T, F = np.array(T), np.array(F)
        noise = math.sqrt(np.sum(T.var(0, ddof=1) + F.var(0, ddof=1)) / n_seeds)
        err = np.linalg.norm(T.mean(0) - F.mean(0))
        assert err < 3 * noise, (j, err, noise)
        assert np.linalg.norm(T.mean(0)) > 5 * noise, (j, np.linalg.norm(T.mean(0)), noise)


# --------------------------------------------------------------------------
# soft-edged spot: derivatives w.r.t. the cone angles
# --------------------------------------------------------------------------

@pytest.mark.parametrize("size", [(0.3, 1.2), (0.0, 0.7), (0.5, 0.55)])
def test_cone_first_hit_derivative(oracle_lib, size):
    """dlog of the first-hit kernel w.r.t. (theta_in, theta_out) at constant
    power vs central differences of an independent log-intensity (profile and
    normalisation) in the fixed direction of x_1, in the fall-off ring and
    inside the inner cone; the other six entries are those of the plain call."""
    rng = np.random.default_rng(int(size[1] * 100))
    ci, co = math.cos(size[0]), math.cos(size[1])
    done, ring = 0, 0
    while done < 24:
        p = [rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(1.5, 2.5),
             rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), rng.uniform(10, 100)]
        lights = make_lights([SOFT], [0.0], [size], [0], [p])
        ol = oracle_lib.OracleLights(lights)
        pf = np.asarray(lights.params[0], np.float64)
        d, t, b = cf.frame(pf[3], pf[4])
        y = pf[:3]
        # a direction inside the outer cone (half of them in the ring), a
        # receiver along it facing back towards the light
        ct = rng.uniform(co, ci) if (done % 3 != 2 or size[0] == 0) else rng.uniform(ci, 1.0)
        if ct <= co + 1e-3 or abs(ct - ci) < 1e-3:
            continue
        ph = rng.uniform(0, 2 * math.pi)
        st = math.sqrt(1 - ct * ct)
        w = ct * d + st * (math.cos(ph) * t + math.sin(ph) * b)
        x1 = y + rng.uniform(0.5, 3.0) * w
        n1 = -w + rng.normal(size=3) * 0.2
        n1 /= np.linalg.norm(n1)
        cw = float(np.dot(d, (x1 - y) / np.linalg.norm(x1 - y)))
        done += 1
        ring += cw < math.cos(size[0])
        args = (x1.astype(np.float32), y.astype(np.float32), n1.astype(np.float32))
        dl = oracle_lib.first_hit_dlog_cone(ol, lights.params, 0, *args).astype(np.float64)
        assert np.array_equal(dl[:6], oracle_lib.first_hit_dlog(ol, lights.params, 0, *args))
        for c in range(2):
            h = 1e-6
            sp, sm = list(size), list(size)
            sp[c] += h
            sm[c] -= h
            if sm[0] < 0:           # theta_in = 0: one-sided
                sm[0] = 0.0
            fd = (cf.log_irradiance(SOFT, 0.0, pf, x1, n1, size=sp) -
                  cf.log_irradiance(SOFT, 0.0, pf, x1, n1, size=sm)) / (sp[c] - sm[c])
            assert abs(dl[6 + c] - fd) <= 2e-4 * (abs(fd) + 1.0), (size, c, cw, dl[6 + c], fd)
    assert ring == 16 if size[0] > 0 else ring == done


def test_cone_gradient_vs_quadrature(oracle_lib):
    """Direct light of a soft-edged spot on a plane: the seed mean of the
    adjoint's dO/d(theta_in, theta_out) matches central differences of the
    quadrature expectation of O's linear part sum_k g_k E_k in the cone
    angles (at constant power), and the position and tilt gradients of the
    cone call equal the plain adjoint's."""
    half, res, N, n_seeds = 3.0, 12, 1 << 16, 8
    sc = li.plane_scene(half=half, res=res)
    p = np.array([0.3, -0.2, 1.4, 0.25, -0.15, 40.0])
    size = (0.35, 0.9)
    lights = make_lights([SOFT], [0.0], [size], [0], [p])
    osc, ol = oracle_lib.OracleScene(sc), oracle_lib.OracleLights(lights)
    A = float(sc.texel_area()[0])
    # weight on the texels near the axis: widening either cone at constant
    # power moves flux away from them
    d, _, _ = cf.frame(p[3], p[4])
    xa = p[:2] + d[:2] * (p[2] / -d[2])
    x0, x1, y0, y1 = cf.plane_texels(half, res)
    cx, cy = (x0 + x1) / 2, (y0 + y1) / 2
    g = np.exp(-((cx - xa[0]) ** 2 + (cy - xa[1]) ** 2) / 0.5).astype(np.float32)[None]
    ref = np.zeros(2)
    for c in range(2):
        h = 1e-4
        sp, sm = list(size), list(size)
        sp[c] += h
        sm[c] -= h
        # the inner cone's kink crosses texels: a fine rule (converged to 1e-3)
        Ep = cf.plane_hit_probability(SOFT, 0.0, p, sp, half, res, q_tex=64) * p[5] / A
        Em = cf.plane_hit_probability(SOFT, 0.0, p, sm, half, res, q_tex=64) * p[5] / A
        ref[c] = float(np.dot(g[0].astype(np.float64), Ep - Em)) / (2 * h)
    runs = [oracle_lib.adjoint_cone(osc, ol, lights.params, 0xC0 + s, N, 1, g) for s in range(n_seeds)]
    gc = np.array([r[1][0] for r in runs])
    mean, se = gc.mean(0), gc.std(0, ddof=1) / math.sqrt(n_seeds)
    for c in range(2):
        assert abs(mean[c] - ref[c]) < 4 * se[c] + 2e-3 * abs(ref[c]), (c, mean[c], ref[c], se[c])
        assert abs(ref[c]) > 8 * se[c], (c, ref[c], se[c])
    g0, _ = oracle_lib.adjoint(osc, ol, lights.params, 0xC0, N, 1, g)
    assert np.allclose(runs[0][0], g0, rtol=1e-9, atol=0)      # FP64 sums in thread order
