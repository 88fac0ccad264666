/*
 * Light-tracing oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU implementation of view-independent adjoint light tracing
 * (Lipp et al., "View-Independent Adjoint Light Tracing for Lighting Design
 * Optimization").  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product library never does.  It shares no
 * code with the GPU path: the two sides implement the same written arithmetic
 * contract (FP32 path arithmetic in a fixed operation order, no contraction,
 * IEEE division and square root, own transcendental polynomials, Philox4x32-10)
 * independently.
 *
 * What it computes, with the passage each step follows:
 *   - Primal light tracing, Alg. 1 (Sec. 4.2): per light N_l rays, each
 *     carrying flux Phi_r = P / N_l; at every hit the incident flux is splatted
 *     into the hit texel as irradiance (Eq. directionalCoeffs with n = 0,
 *     H_0^0 = 1 and the box basis of the mass-lumped projection, supplement
 *     Eq. spatialRep / appdxSpatialCoeffs); the path continues with a
 *     cosine-weighted bounce and Phi_{i+1} = Phi_i * rho (Eq. indirectFlux for
 *     a Lambertian BRDF f = rho/pi sampled with pdf cos/pi).
 *   - Objective, Eq. objective with alpha_l = 1: O = 1/2 sum_k A_k alpha_k
 *     (E_k - E*_k)^2, and its derivative g_k = dO/dE_k.
 *   - Adjoint light tracing, Alg. 2 (Sec. 4.3): the same paths replayed from
 *     the counter-based generator; the adjoint state dO/dPhi_r accumulates
 *     g_k * dE_k/dPhi_i * dPhi_i/dPhi_r at every hit (Eq. adjointFlux); at the
 *     first hit dPhi_r/dp is formed with x_1 held fixed (Sec. 4.3 "constant
 *     sample", Sec. 4.4.2 Eq. posDeriv, rotation and area-light terms of the
 *     supplement, generalised to a cos^n lobe); at path end
 *     dO/dp += dO/dPhi_r * dPhi_r/dp (Eq. objGradAdjoint, first term; the BRDF
 *     terms vanish for Lambertian surfaces, Eq. dLdp discussion).
 *   - Texel basis: box (one texel per hit) or the piecewise-linear basis of
 *     Eq. pwLin with nodes at the texel centres (bilinear weights, four
 *     splats per hit, the adjoint gathering with the same weights).
 *   - Directional texels (Eq. directionalCoeffs with n = 1, 2): each hit
 *     projects its reflected radiance, (Phi / A) f(w_in, w), on 2pi-normalised
 *     hemispherical harmonics with N' uniform local samples; a glossy
 *     (Lambertian + normalised Phong) BRDF; the bounce stays cosine-sampled
 *     with weight pi f; the adjoint adds the first hit's BRDF terms (Eq. dLdp:
 *     its projection and its bounce weight change with the incident
 *     direction while x_1 stays fixed).
 *   - Orientation as a rotation vector (Sec. 4.4.2, Rodrigues' formula with
 *     the small-angle form near zero): the first-hit derivative w.r.t. a
 *     world rotation of the luminaire, mapped to the rotation vector by the
 *     transposed Jacobian of the exponential map.
 *   - Colour: per-luminaire channel weights of the flux and per-patch channel
 *     albedos; three channel-planar texel arrays per layout, one path
 *     geometry for all channels, and the gradient w.r.t. the channel weights
 *     (Sec. 4.4.3, intensity and colour).
 *   - Luminaires: point, cos^n spot, cos^n rectangle, and the supplement's
 *     soft-edged spot (quadratic fall-off in cos theta between the inner and
 *     outer cone, directions uniform over the outer cap, weighted).
 *   - Object-space path tracing with next-event estimation (the comparison
 *     estimator of Sec. 6) on the same texels, and its gradient.
 *   - Direct-differentiation map, the comparison beside it: dE_k/dp_j with
 *     the first hits held fixed, splatted at every hit.
 *   - Gradient-contribution map (Sec. gradVis): the same adjoint pass over
 *     one light's paths, each path adding its contribution to dO/dp_j into
 *     the texel of its first surface hit.
 *
 * Pins (tests/test_oracle_pins.py): closed forms, invariants, brute force and
 * finite differences for every step above; the generator against the
 * published Philox4x32-10 known-answer vectors.
 *
 * Floating point: path arithmetic is FP32 because the kernels compute in FP32
 * and FP32 decides integers here (which triangle is hit, which texel, the
 * fixed-point code of a splat); texel sums are exact int64 fixed point
 * (Q31.32); reductions over paths and texels are FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from Salmon, Moraes, Dror, Shaw, "Parallel random numbers:  */
/* as easy as 1, 2, 3" (SC'11): 10 rounds of two 32x32->64 multiplies with    */
/* a Weyl-sequence key schedule.                                              */
/* ------------------------------------------------------------------------- */
EXPORT void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 24 high bits of a 32-bit word as a float in [0, 1 - 2^-24]. */
static float unit_float(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

static void draw4(uint64_t seed, uint32_t i, uint32_t stream, uint32_t block, float u[4])
{
    uint32_t ctr[4] = {i, stream, block, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    or_philox(ctr, key, r);
    for (int c = 0; c < 4; ++c) u[c] = unit_float(r[c]);
}

/* Generator block of the directional mode's local sample j at hit h (the N'
 * local samples of Alg. 1): one Philox draw serves two samples, and each hit
 * owns 32 consecutive blocks from 0x100 on, so up to 64 samples per hit never
 * share uniforms with another hit's samples, with the emission (0), proposal
 * (1) or bounce (1 + h) draws. */
EXPORT uint32_t or_dir_block(uint32_t h, uint32_t j) { return 0x100u + 32u * h + (j >> 1); }

/* ------------------------------------------------------------------------- */
/* Own transcendentals (FP32 contract).                                       */
/* ------------------------------------------------------------------------- */

/* sin and cos of 2*pi*u for u in [0,1): quadrant from round(4u), remainder
 * x = (4u - q) * pi/2 in [-pi/4, pi/4], Taylor polynomials in Horner form. */
EXPORT void or_sincos2pi(float u, float* s_out, float* c_out)
{
    const float HALF_PI = (float)1.57079632679489661923;
    float q4 = u * 4.0f;
    float qf = rintf(q4);
    float r = q4 - qf;
    float x = r * HALF_PI;
    float x2 = x * x;
    float ps = (float)(1.0 / 362880.0);
    ps = ps * x2 + (float)(-1.0 / 5040.0);
    ps = ps * x2 + (float)(1.0 / 120.0);
    ps = ps * x2 + (float)(-1.0 / 6.0);
    ps = ps * x2;
    float s = x + x * ps;
    float pc = (float)(1.0 / 3628800.0);
    pc = pc * x2 + (float)(-1.0 / 40320.0);
    pc = pc * x2 + (float)(1.0 / 720.0);
    pc = pc * x2 + (float)(-1.0 / 24.0);
    pc = pc * x2 + (float)(1.0 / 2.0);
    float c = 1.0f - pc * x2;
    int q = ((int)qf) & 3;
    float so, co;
    if (q == 0) { so = s; co = c; }
    else if (q == 1) { so = c; co = -s; }
    else if (q == 2) { so = -s; co = -c; }
    else { so = -c; co = s; }
    *s_out = so;
    *c_out = co;
}

/* log2 of a positive normal float: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
 * ln m = 2 atanh(s), s = (m-1)/(m+1), odd series to s^11. */
EXPORT float or_log2(float x)
{
    const float SQRT_HALF = (float)0.70710678118654752440;
    const float INV_LN2 = (float)1.44269504088896340736;
    int e;
    float m = frexpf(x, &e);
    if (m < SQRT_HALF) {
        m = m * 2.0f;
        e = e - 1;
    }
    float f = m - 1.0f;
    float s = f / (m + 1.0f);
    float s2 = s * s;
    float p = (float)(1.0 / 11.0);
    p = p * s2 + (float)(1.0 / 9.0);
    p = p * s2 + (float)(1.0 / 7.0);
    p = p * s2 + (float)(1.0 / 5.0);
    p = p * s2 + (float)(1.0 / 3.0);
    p = p * s2;
    float h = s + s * p;
    float ln_m = h + h;
    return (float)e + ln_m * INV_LN2;
}

/* 2^y: k = round(y), f = y - k in [-1/2, 1/2], e^(f ln2) by Taylor to degree 7. */
EXPORT float or_exp2(float y)
{
    const float LN2 = (float)0.69314718055994530942;
    float k = rintf(y);
    float f = y - k;
    float z = f * LN2;
    float p = (float)(1.0 / 5040.0);
    p = p * z + (float)(1.0 / 720.0);
    p = p * z + (float)(1.0 / 120.0);
    p = p * z + (float)(1.0 / 24.0);
    p = p * z + (float)(1.0 / 6.0);
    p = p * z + 0.5f;
    p = p * z + 1.0f;
    p = p * z + 1.0f;
    return ldexpf(p, (int)k);
}

/* sin and cos of an arbitrary angle in FP64 (used for the light frame only):
 * k = round(x 2/pi), r = (x - k P1) - k P2 with pi/2 = P1 + P2 (P1 has 33
 * significant bits), Taylor polynomials to r^17 / r^18. */
EXPORT void or_sincos_f64(double x, double* s_out, double* c_out)
{
    const double TWO_OVER_PI = 6.36619772367581382433e-01;
    const double P1 = 1.57079632673412561417e+00;
    const double P2 = 6.07710050650619224932e-11;
    double k = rint(x * TWO_OVER_PI);
    double r = (x - k * P1) - k * P2;
    double r2 = r * r;
    double ps = -1.0 / 355687428096000.0;       /* -1/17! */
    ps = ps * r2 + 1.0 / 1307674368000.0;       /* 1/15! */
    ps = ps * r2 - 1.0 / 6227020800.0;          /* -1/13! */
    ps = ps * r2 + 1.0 / 39916800.0;            /* 1/11! */
    ps = ps * r2 - 1.0 / 362880.0;              /* -1/9! */
    ps = ps * r2 + 1.0 / 5040.0;                /* 1/7! */
    ps = ps * r2 - 1.0 / 120.0;                 /* -1/5! */
    ps = ps * r2 + 1.0 / 6.0;                   /* 1/3! */
    double s = r - r * (r2 * ps);
    double pc = 1.0 / 6402373705728000.0;       /* 1/18! */
    pc = pc * r2 - 1.0 / 20922789888000.0;      /* -1/16! */
    pc = pc * r2 + 1.0 / 87178291200.0;         /* 1/14! */
    pc = pc * r2 - 1.0 / 479001600.0;           /* -1/12! */
    pc = pc * r2 + 1.0 / 3628800.0;             /* 1/10! */
    pc = pc * r2 - 1.0 / 40320.0;               /* -1/8! */
    pc = pc * r2 + 1.0 / 720.0;                 /* 1/6! */
    pc = pc * r2 - 1.0 / 24.0;                  /* -1/4! */
    pc = pc * r2 + 0.5;                         /* 1/2! */
    double c = 1.0 - r2 * pc;
    int q = (int)(((long long)k) & 3);
    if (q == 0) { *s_out = s; *c_out = c; }
    else if (q == 1) { *s_out = c; *c_out = -s; }
    else if (q == 2) { *s_out = -s; *c_out = -c; }
    else { *s_out = -c; *c_out = s; }
}

/* ------------------------------------------------------------------------- */
/* Scene                                                                      */
/* ------------------------------------------------------------------------- */
typedef struct {
    const float* verts;       /* [V,3] */
    const int32_t* tris;      /* [T,3] */
    const int32_t* tri_patch; /* [T] */
    int64_t n_tris;
    const float* pf;          /* [P,17] origin, e_u, e_v, normal, inv_len2_u, inv_len2_v,
                                 texel_area, inv_texel_area, albedo */
    const int32_t* pres;      /* [P,2] res_u, res_v */
    const int64_t* pbase;     /* [P] first texel */
    int32_t n_patches;
    int64_t n_texels;
    int32_t basis;            /* 0 box (one texel per hit), 1 piecewise-linear nodes at texel centres */
    const void* bvh;          /* or_bvh* or NULL for brute force */
    const float* albedo_rgb;  /* [P,3] per-channel albedo (colour mode), or NULL: the scalar albedo */
    const float* glossy;      /* [P,2] specular albedo, Phong exponent (directional mode), or NULL */
    int32_t dir_order;        /* directional texels: HSH order 0..3, or -1 (irradiance texels) */
    int32_t dir_samples;      /* local exitant samples per hit (directional mode) */
} or_scene;

typedef struct {
    const int32_t* type;      /* [L] 0 point, 1 spot (cos^n), 2 rectangle, 3 soft-edged spot */
    const float* lobe_n;      /* [L] */
    const float* size;        /* [L,2] rectangle w, h; soft-edged spot: inner, outer cone angle */
    const int32_t* layout_offsets; /* [n_layouts+1] */
    int32_t n_lights;
    int32_t n_layouts;
    const float* colour;      /* [L,3] channel weights (colour mode: texels [n_layouts,3,K]), or NULL */
    int32_t rotvec;           /* orientation as a rotation vector: params [L,7] = x, y, z, theta, P */
} or_lights;

/* Learned emission proposal (beyond the paper, which leaves importance
 * sampling to future work, Sec. 7): per light a distribution over 32 x 32
 * cells of the hemi-octahedral map of the emission hemisphere, mixed with the
 * plain lobe under one-sample MIS (defensive mixture).  pdf/cdf: [L,1024]. */
typedef struct {
    const float* pdf;        /* bin probabilities pi_b */
    const float* cdf;        /* inclusive prefix sums of pdf */
    float alpha;             /* probability of the plain lobe */
    const float* inv_sigma;  /* [L,6] scale of the histogram signal (adjoint) */
    double* hist;            /* [L,1024] adjoint histogram (adjoint, may be NULL): per
                              * path, |c_r * inv_sigma|^2 * q / (512 |p|^3) into
                              * its emission cell (q: the mixture density of
                              * the emitted direction, |p|: the norm of its
                              * point on the octahedron) */
} or_proposal;

static float dot3(const float* a, const float* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

/* Moeller-Trumbore ray/triangle test, barycentric bounds widened by 2^-20.
 * Returns 1 and t on a hit with t > 0. */
static int ray_triangle(const float* o, const float* d, const float* v0, const float* v1, const float* v2,
                        float* t_out)
{
    const float EPS = 0x1p-20f;
    float e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    float e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    float p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    float det = dot3(e1, p);
    if (det == 0.0f) return 0;
    float inv = 1.0f / det;
    float s[3] = {o[0] - v0[0], o[1] - v0[1], o[2] - v0[2]};
    float u = dot3(s, p) * inv;
    if (u < -EPS || u > 1.0f + EPS) return 0;
    float q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    float v = dot3(d, q) * inv;
    if (v < -EPS || u + v > 1.0f + EPS) return 0;
    float t = dot3(e2, q) * inv;
    if (!(t > 0.0f)) return 0;
    *t_out = t;
    return 1;
}

/* closest hit = lexicographic minimum of (t, primitive id) */
static void consider(const or_scene* S, int64_t prim, const float* o, const float* d, int32_t skip_patch,
                     float* tb, int64_t* pb)
{
    if (S->tri_patch[prim] == skip_patch) return;
    const int32_t* tr = S->tris + 3 * prim;
    float t;
    if (!ray_triangle(o, d, S->verts + 3 * tr[0], S->verts + 3 * tr[1], S->verts + 3 * tr[2], &t)) return;
    if (t < *tb || (t == *tb && prim < *pb)) {
        *tb = t;
        *pb = prim;
    }
}

/* ---- a plain median-split BVH (oracle-own; checked against brute force) --- */
typedef struct {
    double lo[3], hi[3];
    int64_t left, right;   /* children, or -1 for a leaf */
    int64_t first, count;  /* leaf primitive range in `order` */
} obnode;

typedef struct {
    obnode* nodes;
    int64_t n_nodes;
    int64_t* order;
    double pad;
} or_bvh;

static void tri_bounds(const float* verts, const int32_t* tr, double lo[3], double hi[3])
{
    for (int c = 0; c < 3; ++c) {
        double a = verts[3 * tr[0] + c], b = verts[3 * tr[1] + c], e = verts[3 * tr[2] + c];
        lo[c] = fmin(a, fmin(b, e));
        hi[c] = fmax(a, fmax(b, e));
    }
}

typedef struct { const double* key; } sort_ctx_t;
static const double* g_sort_key;
static int cmp_idx(const void* a, const void* b)
{
    double ka = g_sort_key[*(const int64_t*)a], kb = g_sort_key[*(const int64_t*)b];
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    int64_t ia = *(const int64_t*)a, ib = *(const int64_t*)b;
    return (ia > ib) - (ia < ib);
}

static int64_t build_rec(or_bvh* B, const float* verts, const int32_t* tris, const double* cen,
                         double* key, int64_t first, int64_t count)
{
    int64_t id = B->n_nodes++;
    obnode* n = &B->nodes[id];
    for (int c = 0; c < 3; ++c) { n->lo[c] = INFINITY; n->hi[c] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = first; i < first + count; ++i) {
        double lo[3], hi[3];
        int64_t p = B->order[i];
        tri_bounds(verts, tris + 3 * p, lo, hi);
        for (int c = 0; c < 3; ++c) {
            n->lo[c] = fmin(n->lo[c], lo[c]);
            n->hi[c] = fmax(n->hi[c], hi[c]);
            clo[c] = fmin(clo[c], cen[3 * p + c]);
            chi[c] = fmax(chi[c], cen[3 * p + c]);
        }
    }
    for (int c = 0; c < 3; ++c) { n->lo[c] -= B->pad; n->hi[c] += B->pad; }
    if (count <= 4) {
        n->left = n->right = -1;
        n->first = first;
        n->count = count;
        return id;
    }
    int ax = 0;
    for (int c = 1; c < 3; ++c)
        if (chi[c] - clo[c] > chi[ax] - clo[ax]) ax = c;
    for (int64_t i = first; i < first + count; ++i) key[B->order[i]] = cen[3 * B->order[i] + ax];
    g_sort_key = key;
    qsort(B->order + first, (size_t)count, sizeof(int64_t), cmp_idx);
    int64_t half = count / 2;
    int64_t l = build_rec(B, verts, tris, cen, key, first, half);
    int64_t r = build_rec(B, verts, tris, cen, key, first + half, count - half);
    n = &B->nodes[id];
    n->left = l;
    n->right = r;
    n->first = n->count = 0;
    return id;
}

/* Build the oracle's BVH.  Node boxes are padded by `pad` (metres) so the
 * FP64 slab test below can never reject a box that holds an accepted hit. */
EXPORT void* or_bvh_build(const float* verts, const int32_t* tris, int64_t n_tris, double pad)
{
    or_bvh* B = (or_bvh*)calloc(1, sizeof(or_bvh));
    B->nodes = (obnode*)calloc((size_t)(2 * n_tris + 1), sizeof(obnode));
    B->order = (int64_t*)malloc((size_t)n_tris * sizeof(int64_t));
    B->pad = pad;
    double* cen = (double*)malloc((size_t)n_tris * 3 * sizeof(double));
    double* key = (double*)malloc((size_t)n_tris * sizeof(double));
    for (int64_t p = 0; p < n_tris; ++p) {
        B->order[p] = p;
        for (int c = 0; c < 3; ++c)
            cen[3 * p + c] = ((double)verts[3 * tris[3 * p] + c] + verts[3 * tris[3 * p + 1] + c] +
                              verts[3 * tris[3 * p + 2] + c]) / 3.0;
    }
    if (n_tris > 0) build_rec(B, verts, tris, cen, key, 0, n_tris);
    free(cen);
    free(key);
    return B;
}

EXPORT void or_bvh_free(void* p)
{
    or_bvh* B = (or_bvh*)p;
    if (!B) return;
    free(B->nodes);
    free(B->order);
    free(B);
}

static int box_hit(const obnode* n, const double* o, const double* inv, double tmax)
{
    double t0 = 0.0, t1 = tmax;
    for (int c = 0; c < 3; ++c) {
        double a = (n->lo[c] - o[c]) * inv[c], b = (n->hi[c] - o[c]) * inv[c];
        if (a > b) { double tmp = a; a = b; b = tmp; }
        if (a > t0) t0 = a;
        if (b < t1) t1 = b;
    }
    return t0 <= t1;
}

/* Closest hit of ray (o, d) skipping every triangle of patch skip_patch.
 * Returns the primitive or -1 for a miss. */
static int64_t intersect(const or_scene* S, const float* o, const float* d, int32_t skip_patch, float* t_out)
{
    float tb = INFINITY;
    int64_t pb = -1;
    if (!S->bvh) {
        for (int64_t p = 0; p < S->n_tris; ++p) consider(S, p, o, d, skip_patch, &tb, &pb);
    } else {
        const or_bvh* B = (const or_bvh*)S->bvh;
        double od[3], inv[3];
        for (int c = 0; c < 3; ++c) {
            od[c] = o[c];
            double dc = d[c];
            inv[c] = 1.0 / (dc != 0.0 ? dc : (signbit(dc) ? -1e-300 : 1e-300));
        }
        int64_t stack[256];
        int sp = 0;
        if (B->n_nodes > 0) stack[sp++] = 0;
        while (sp > 0) {
            const obnode* n = &B->nodes[stack[--sp]];
            double tmax = isinf(tb) ? INFINITY : (double)tb;
            if (!box_hit(n, od, inv, tmax)) continue;
            if (n->left < 0) {
                for (int64_t i = n->first; i < n->first + n->count; ++i)
                    consider(S, B->order[i], o, d, skip_patch, &tb, &pb);
            } else {
                stack[sp++] = n->left;
                stack[sp++] = n->right;
            }
        }
    }
    *t_out = tb;
    return pb;
}

/* batch entry for the brute-force / BVH equivalence pin */
EXPORT void or_intersect_batch(const or_scene* S, const float* rays, int64_t n, const int32_t* skip,
                               float* t_out, int64_t* prim_out)
{
    for (int64_t i = 0; i < n; ++i)
        prim_out[i] = intersect(S, rays + 6 * i, rays + 6 * i + 3, skip ? skip[i] : -1, &t_out[i]);
}

/* ------------------------------------------------------------------------- */
/* Luminaires: frame R = R_y(beta) R_x(alpha), axis d = R(0,0,-1),            */
/* tangent t = R(1,0,0), bitangent b = R(0,1,0), and their angle derivatives. */
/* ------------------------------------------------------------------------- */
typedef struct {
    int type;
    float n, w, h;
    float ci, co;          /* soft-edged spot: cosines of the inner and outer cone */
    float c[3], d[3], t[3], b[3];
    float dd_da[3], dd_db[3], dt_db[3], db_da[3], db_db[3];
    float P, phi_r;
    int64_t n_paths;
    int rgb;               /* colour mode */
    float col[3];          /* channel weights of the flux */
    int rv;                /* rotation-vector orientation (7 parameters) */
    int cone;              /* soft-edged spot: also differentiate the cone angles (dl[6], dl[7]) */
    float ki, ko;          /* dlog I_e / d(theta_in), d(theta_out) at constant power */
    float kri, kq, so;     /* 2 sin(theta_in) / (ci - co), 2 / (ci - co), sin(theta_out) */
} olight;

/* Rodrigues' formula R = I + sin(phi)/phi K + (1 - cos(phi))/phi^2 K^2, K = [theta]x,
 * phi = |theta|, with the linear small-angle form I + K near zero (Sec. 4.4.2). */
static void rodrigues(const double* th, double R[9])
{
    double K[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    double f2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
    double A = 1.0, Bc = 0.0;
    if (f2 >= 1e-12) {
        double f = sqrt(f2), sf, cf;
        or_sincos_f64(f, &sf, &cf);
        A = sf / f;
        Bc = (1.0 - cf) / f2;
    }
    for (int i = 0; i < 9; ++i) R[i] = ((i % 4 == 0) ? 1.0 : 0.0) + A * K[i] + Bc * K2[i];
}

/* d theta of a world rotation: R(theta + dtheta) = exp([J dtheta]x) R(theta) with
 * J = I + (1 - cos phi)/phi^2 K + (phi - sin phi)/phi^3 K^2 (I near zero, where the
 * small-angle form is used); gradients map as g_theta = J^T g_omega. */
static void rot_jacobian(const double* th, double J[9])
{
    double K[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    double f2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
    double a = 0.0, b = 0.0;
    if (f2 >= 1e-12) {
        double f = sqrt(f2), sf, cf;
        or_sincos_f64(f, &sf, &cf);
        a = (1.0 - cf) / f2;
        b = (f - sf) / (f2 * f);
    }
    for (int i = 0; i < 9; ++i) J[i] = ((i % 4 == 0) ? 1.0 : 0.0) + a * K[i] + b * K2[i];
}

static void light_setup(const or_lights* Ls, const float* params, int gl, int64_t n_paths, olight* L)
{
    const float* p = params + (Ls->rotvec ? 7 : 6) * gl;
    L->cone = 0;
    L->type = Ls->type[gl];
    L->n = Ls->lobe_n[gl];
    L->w = Ls->size[2 * gl];
    L->h = Ls->size[2 * gl + 1];
    for (int c = 0; c < 3; ++c) L->c[c] = p[c];
    double sa_d, ca_d, sb_d, cb_d;
    or_sincos_f64((double)p[3], &sa_d, &ca_d);
    or_sincos_f64((double)p[4], &sb_d, &cb_d);
    float sa = (float)sa_d, ca = (float)ca_d, sb = (float)sb_d, cb = (float)cb_d;
    L->d[0] = -(sb * ca); L->d[1] = sa; L->d[2] = -(cb * ca);
    L->t[0] = cb; L->t[1] = 0.0f; L->t[2] = -sb;
    L->b[0] = sb * sa; L->b[1] = ca; L->b[2] = cb * sa;
    L->dd_da[0] = sb * sa; L->dd_da[1] = ca; L->dd_da[2] = cb * sa;
    L->dd_db[0] = -(cb * ca); L->dd_db[1] = 0.0f; L->dd_db[2] = sb * ca;
    L->dt_db[0] = -sb; L->dt_db[1] = 0.0f; L->dt_db[2] = -cb;
    L->db_da[0] = sb * ca; L->db_da[1] = -sa; L->db_da[2] = cb * ca;
    L->db_db[0] = cb * sa; L->db_db[1] = 0.0f; L->db_db[2] = -(sb * sa);
    L->rv = Ls->rotvec != 0;
    if (L->rv) {
        /* world frame from the rotation vector: d = R(0,0,-1), t = R e_x, b = R e_y */
        double th[3] = {(double)p[3], (double)p[4], (double)p[5]}, R[9];
        rodrigues(th, R);
        for (int c = 0; c < 3; ++c) {
            L->d[c] = (float)(-R[3 * c + 2]);
            L->t[c] = (float)R[3 * c];
            L->b[c] = (float)R[3 * c + 1];
            L->dd_da[c] = L->dd_db[c] = L->dt_db[c] = L->db_da[c] = L->db_db[c] = 0.0f;
        }
    }
    const float Pw = p[L->rv ? 6 : 5];
    L->P = Pw;
    L->n_paths = n_paths;
    L->phi_r = Pw / (float)n_paths;
    L->ci = 1.0f;
    L->co = 0.0f;
    L->rgb = Ls->colour != NULL;
    for (int c = 0; c < 3; ++c) L->col[c] = Ls->colour ? Ls->colour[3 * gl + c] : 1.0f;
    if (L->type == 3) {
        /* soft-edged spot (supplement, spot light): constant intensity inside
         * the inner cone, a = ((cos - cos_out) / (cos_in - cos_out))^2 out to
         * the outer cone, nothing beyond.  Directions are drawn uniformly
         * over the outer cone's cap and weighted by a, so with P the total
         * flux, Phi_r = (P / N) a (1 - cos_out) / ((1 - cos_in) + (cos_in - cos_out) / 3). */
        double si_d, ci_d, so_d, co_d;
        or_sincos_f64((double)L->w, &si_d, &ci_d);
        or_sincos_f64((double)L->h, &so_d, &co_d);
        L->ci = (float)ci_d;
        L->co = (float)co_d;
        double den = (1.0 - ci_d) + (ci_d - co_d) / 3.0;
        float kcap = (float)((1.0 - co_d) / den);
        L->phi_r = L->phi_r * kcap;
        /* cone-angle derivatives at constant P: I_e = P / (2 pi den) gives
         * dlog I_e/dci = (2/3)/den and dlog I_e/dco = (1/3)/den; with
         * dci = -sin(theta_in) dtheta_in, dco = -sin(theta_out) dtheta_out */
        L->ki = (float)(-(si_d * (2.0 / 3.0)) / den);
        L->ko = (float)(-(so_d * (1.0 / 3.0)) / den);
        L->kq = (float)(2.0 / (ci_d - co_d));
        L->kri = (float)(2.0 * si_d / (ci_d - co_d));
        L->so = (float)so_d;
    }
}

static int64_t paths_of_light(int64_t n_layout, int n_in_layout, int l)
{
    return n_layout / n_in_layout + ((int64_t)l < n_layout % n_in_layout ? 1 : 0);
}

/* ---- one path ------------------------------------------------------------ */
typedef struct {
    int64_t* S;            /* forward: texel accumulators of this layout (or NULL) */
    const float* g;        /* adjoint: dO/dE of this layout (or NULL) */
    double* acc;           /* adjoint: per-light gradient accumulator [6] */
    double* acc_col;       /* adjoint, colour mode: gradient w.r.t. the channel weights [3] */
    float* contrib;        /* record: per-path contribution [6] (or NULL) */
    double* vote;          /* votes: per-texel map of one parameter's contributions (or NULL) */
    int64_t* tangent;      /* direct differentiation: dE_k/dp_j splats of this layout (or NULL) */
    int tangent_param;
    int vote_param;        /* votes: which of the six parameters */
    int32_t* rec_prim;     /* record: [B] (or NULL) */
    int32_t* rec_texel;    /* record: [B] */
    int64_t misses;
} path_io;

/* dlog of the first-hit irradiance kernel w.r.t. (c, alpha, beta, P), x_1 fixed:
 * log E = log P + n log(d.w) + log(-n1.w) - 2 log r + const, w = (x1 - y)/r. */
static void first_hit_dlog(const olight* L, const float* x1, const float* y, const float* n1, float au,
                           float av, float* dl)
{
    /* rotation-vector mode: dl[7] = (position, world-rotation, power) */
    const int np = L->rv ? 7 : 6;
    for (int c = 0; c < np - 1; ++c) dl[c] = 0.0f;
    dl[np - 1] = 1.0f / L->P;
    if (L->cone) dl[6] = dl[7] = 0.0f;
    float v[3] = {x1[0] - y[0], x1[1] - y[1], x1[2] - y[2]};
    float r2 = dot3(v, v);
    if (r2 <= 1e-12f) return;
    float r = sqrtf(r2);
    float inv_r = 1.0f / r;
    float w[3] = {v[0] * inv_r, v[1] * inv_r, v[2] * inv_r};
    if (L->cone && L->type == 3) {
        /* log a = 2 log(ce - co) - 2 log(ci - co) in the fall-off ring, 0
         * inside the inner cone; the intensity's log-derivatives in the
         * direction of x_1, which stays fixed */
        float cw = dot3(L->d, w);
        int ring = cw > L->co && cw < L->ci;
        dl[6] = ring ? L->ki + L->kri : L->ki;
        dl[7] = ring ? L->ko + L->so * (2.0f / (cw - L->co) - L->kq) : L->ko;
    }
    float c1 = -dot3(n1, w);
    if (c1 <= 1e-6f) return;
    float k1 = 1.0f / (r * c1);
    float k3 = 2.0f * inv_r;
    float G[3];
    if (L->type == 0) {
        for (int c = 0; c < 3; ++c) G[c] = (n1[c] + c1 * w[c]) * k1 + w[c] * k3;
        for (int c = 0; c < 3; ++c) dl[c] = G[c];
        return;
    }
    float ce = dot3(L->d, w);
    if (ce <= 1e-6f) return;
    /* ka, kd: the derivative of log I along cos(theta) = d.w, divided by r
     * and not; cos^n lobe: n / cos, soft-edged spot: 2 / (cos - cos_out) in
     * its fall-off ring and 0 inside the inner cone */
    float ka, kd;
    if (L->type == 3) {
        float lg = (ce > L->co && ce < L->ci) ? 2.0f / (ce - L->co) : 0.0f;
        ka = lg / r;
        kd = lg;
    } else {
        ka = L->n / (r * ce);
        kd = L->n / ce;
    }
    for (int c = 0; c < 3; ++c) {
        float t1 = -((L->d[c] - ce * w[c]) * ka);
        float t2 = (n1[c] + c1 * w[c]) * k1;
        float t3 = w[c] * k3;
        G[c] = (t1 + t2) + t3;
    }
    if (L->rv) {
        /* rotating the luminaire about its centre by d_omega turns d into
         * d + d_omega x d and moves the origin by d_omega x (y - c):
         * dlog/d_omega = kd (d x w) + (y - c) x G */
        float yc[3], dw[3], yg[3];
        for (int c = 0; c < 3; ++c) yc[c] = L->type == 2 ? au * L->t[c] + av * L->b[c] : 0.0f;
        dw[0] = L->d[1] * w[2] - L->d[2] * w[1];
        dw[1] = L->d[2] * w[0] - L->d[0] * w[2];
        dw[2] = L->d[0] * w[1] - L->d[1] * w[0];
        yg[0] = yc[1] * G[2] - yc[2] * G[1];
        yg[1] = yc[2] * G[0] - yc[0] * G[2];
        yg[2] = yc[0] * G[1] - yc[1] * G[0];
        for (int c = 0; c < 3; ++c) {
            dl[c] = G[c];
            dl[3 + c] = dw[c] * kd + yg[c];
        }
        return;
    }
    float ra = dot3(L->dd_da, w) * kd;
    float rb = dot3(L->dd_db, w) * kd;
    if (L->type == 2) {
        float dya[3], dyb[3];
        for (int c = 0; c < 3; ++c) {
            dya[c] = av * L->db_da[c];
            dyb[c] = au * L->dt_db[c] + av * L->db_db[c];
        }
        ra = dot3(G, dya) + ra;
        rb = dot3(G, dyb) + rb;
    }
    dl[0] = G[0]; dl[1] = G[1]; dl[2] = G[2];
    dl[3] = ra; dl[4] = rb;
}

/* ---- directional texels and a glossy BRDF -------------------------------- */

/* 2pi-normalised hemispherical harmonics (the integral of H^2 over the
 * hemisphere is 2 pi, H_0^0 = 1) up to order 2, as associated Legendre
 * functions of x = 2 cos(theta) - 1 times cos / sin of m phi; index
 * l^2 + l + m.  Returns the number of functions. */
EXPORT int or_hsh(int order, float ct, float cp, float sp, float* H)
{
    float x = 2.0f * ct - 1.0f;
    float s1 = sqrtf(fmaxf(0.0f, 1.0f - x * x));
    H[0] = 1.0f;
    if (order >= 1) {
        H[1] = (1.7320508075688772f * s1) * sp;
        H[2] = 1.7320508075688772f * x;
        H[3] = (1.7320508075688772f * s1) * cp;
    }
    /* cos/sin of 2 phi and 3 phi by the angle-addition formulas */
    float c2 = 2.0f * (cp * cp) - 1.0f, s2 = 2.0f * (sp * cp);
    float q = 1.0f - x * x;
    if (order >= 2) {
        H[4] = (1.9364916731037085f * q) * s2;
        H[5] = ((3.872983346207417f * x) * s1) * sp;
        H[6] = 2.23606797749979f * ((3.0f * (x * x) - 1.0f) * 0.5f);
        H[7] = ((3.872983346207417f * x) * s1) * cp;
        H[8] = (1.9364916731037085f * q) * c2;
    }
    if (order >= 3) {
        /* l = 3: P3 = (5x^3 - 3x)/2, P3^1 = 3/2 (5x^2 - 1) s1, P3^2 = 15 x q,
         * P3^3 = 15 q s1 (no Condon-Shortley sign), each times its norm */
        float c3 = c2 * cp - s2 * sp, s3 = s2 * cp + c2 * sp;
        float w1 = 5.0f * (x * x) - 1.0f;
        H[9] = ((2.091650066335189f * q) * s1) * s3;
        H[10] = ((5.123475382979799f * x) * q) * s2;
        H[11] = ((1.620185174601965f * w1) * s1) * sp;
        H[12] = 2.6457513110645907f * (((5.0f * (x * x) - 3.0f) * x) * 0.5f);
        H[13] = ((1.620185174601965f * w1) * s1) * cp;
        H[14] = ((5.123475382979799f * x) * q) * c2;
        H[15] = ((2.091650066335189f * q) * s1) * c3;
    }
    return (order + 1) * (order + 1);
}

/* Lambertian plus normalised Phong lobe, in the local frame (normal = z):
 * f = rho_d / pi + rho_s (e + 2) / (2 pi) max(0, r.wo)^e with r the mirror
 * direction of wi; grad = df/dwi (wi as a free vector). */
EXPORT float or_brdf(float rho_d, float rho_s, float e, const float* wi, const float* wo, float* grad)
{
    float f = rho_d * 0.3183098861837907f;
    if (grad) grad[0] = grad[1] = grad[2] = 0.0f;
    if (rho_s > 0.0f) {
        float ro = (-(wi[0] * wo[0]) - wi[1] * wo[1]) + wi[2] * wo[2];
        if (ro > 0.0f) {
            float ks = (rho_s * (e + 2.0f)) * 0.15915494309189533f;
            float pw = or_exp2(e * or_log2(ro));
            f = f + ks * pw;
            if (grad) {
                float gk = (ks * e) * (pw / ro);
                grad[0] = -(gk * wo[0]);
                grad[1] = -(gk * wo[1]);
                grad[2] = gk * wo[2];
            }
        }
    }
    return f;
}

/* the bounce's orthonormal basis about the oriented normal (Duff et al. 2017) */
static void local_frame(const float* no, float* b1, float* b2)
{
    float sign = copysignf(1.0f, no[2]);
    float a = -1.0f / (sign + no[2]);
    float bxy = (no[0] * no[1]) * a;
    b1[0] = 1.0f + ((sign * no[0]) * no[0]) * a; b1[1] = sign * bxy; b1[2] = -(sign * no[0]);
    b2[0] = bxy; b2[1] = sign + (no[1] * no[1]) * a; b2[2] = -no[1];
}

/* The state a light path carries from hit to hit. */
typedef struct {
    float o[3], dir[3];    /* current ray */
    int32_t skip;          /* patch the ray leaves (never hit again by it) */
    float y[3];            /* emission point */
    float au, av;          /* area light: the emission point's offsets along t and b */
    float phi_r;           /* flux the path carries from the light (Phi_r) */
    int ebin;              /* proposal: cell of the emission direction (or -1) */
    float wq;              /* proposal: density of the emission over its cell's (u, v) measure */
    float T;               /* throughput, Phi_h / Phi_r */
    float Tc[3];           /* colour: channel throughputs */
    float s_r;             /* adjoint: sum over hits of g_k Phi_h / (A_k Phi_r) */
    float sc[3];           /* colour adjoint: the same per channel */
    float dphi[8];         /* adjoint: Phi_r dlog/dp_j of the first hit */
    float tdl;             /* direct differentiation: dlog/dp_j of the first hit */
    int hits;
    int64_t k1;            /* texel of the first hit */
    /* directional texels: T2 the bounce-weight product after the first hit,
     * Rd the adjoint sum of the later hits weighted by it, Qw / Dw the
     * first hit's projection and bounce-weight derivatives w.r.t. the
     * incident direction, om1 / inv_r1 that direction and 1 / distance, and
     * the current hit's incident direction and local frame */
    float T2, Rd;
    float Qw[3], Dw[3], om1[3], inv_r1;
    float wi_loc[3], fb1[3], fb2[3];
} path_state;

/* A surface hit: position, the normal facing the incident ray, patch, texel
 * (box basis) and, for the piecewise-linear basis, the four nodes and their
 * bilinear weights. */
typedef struct {
    float x[3], no[3];
    int32_t q;
    const float* pf;       /* the patch's float record */
    int64_t k;
    float inv_a;
    int64_t kb[4];
    float wb[4];
} hit_point;

/* Emission (Alg. 1 "generate exitant ray"): origin y, direction, flux
 * Phi_r; with a proposal the direction comes from the plain cos^n lobe with
 * probability alpha, else from the binned proposal, and Phi_r = (P/N)
 * p_plain / q (one-sample MIS). */
static void emit_path(const olight* L, uint64_t seed, uint32_t i, uint32_t stream, int gl, const or_proposal* prop,
                      path_state* ps)
{
    ps->phi_r = L->phi_r;
    ps->ebin = -1;
    ps->wq = 0.0f;
    float u[4];
    draw4(seed, i, stream, 0u, u);
    for (int c = 0; c < 3; ++c) ps->y[c] = L->c[c];
    ps->au = 0.0f;
    ps->av = 0.0f;
    float* dir = ps->dir;
    if (L->type == 0) {
        float z = 1.0f - 2.0f * u[2];
        float rr = sqrtf(fmaxf(0.0f, 1.0f - z * z));
        float sp, cp;
        or_sincos2pi(u[3], &sp, &cp);
        dir[0] = rr * cp; dir[1] = rr * sp; dir[2] = z;
    } else if (L->type == 3) {
        /* uniform over the outer cone's cap, weighted by the fall-off */
        float ct = 1.0f - u[2] * (1.0f - L->co);
        float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
        float sp, cp;
        or_sincos2pi(u[3], &sp, &cp);
        float a = st * cp, bb = st * sp;
        if (ct < L->ci) {
            float f = (ct - L->co) / (L->ci - L->co);
            ps->phi_r = ps->phi_r * (f * f);
        }
        for (int c = 0; c < 3; ++c) dir[c] = (a * L->t[c] + bb * L->b[c]) + ct * L->d[c];
    } else {
        float ct = 0.0f;
        if (u[2] > 0.0f) ct = or_exp2(or_log2(u[2]) / (L->n + 1.0f));
        float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
        float sp, cp;
        or_sincos2pi(u[3], &sp, &cp);
        float a = st * cp, bb = st * sp;
        if (prop) {
            float w[4];
            draw4(seed, i, stream, 1u, w);
            const float* pdf = prop->pdf + 1024 * (int64_t)gl;
            const float* cdf = prop->cdf + 1024 * (int64_t)gl;
            float lz, pl3;
            if (w[0] < prop->alpha) {
                /* the plain lobe's direction, and its cell of the
                 * hemi-octahedral map */
                lz = ct;
                float s = (fabsf(a) + fabsf(bb)) + lz;
                float xp = a / s, yp = bb / s;
                int iu = (int)floorf(((xp + yp) + 1.0f) * 16.0f);
                int iv = (int)floorf(((xp - yp) + 1.0f) * 16.0f);
                if (iu < 0) iu = 0;
                if (iu > 31) iu = 31;
                if (iv < 0) iv = 0;
                if (iv > 31) iv = 31;
                ps->ebin = iv * 32 + iu;
                pl3 = 1.0f / ((s * s) * s);
            } else {
                /* a cell by inverse CDF, a uniform point in it */
                int lo = 0, hi = 1023;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (w[1] < cdf[mid]) hi = mid;
                    else lo = mid + 1;
                }
                ps->ebin = lo;
                float uu = -1.0f + ((float)(lo & 31) + w[2]) * 0.0625f;
                float vv = -1.0f + ((float)(lo >> 5) + w[3]) * 0.0625f;
                float xp = (uu + vv) * 0.5f, yp = (uu - vv) * 0.5f;
                float zp = (1.0f - fabsf(xp)) - fabsf(yp);
                float nrm = sqrtf((xp * xp + yp * yp) + zp * zp);
                float inv = 1.0f / nrm;
                a = xp * inv;
                bb = yp * inv;
                lz = zp * inv;
                ct = lz;
                pl3 = (nrm * nrm) * nrm;
            }
            float pw = 1.0f;
            if (L->n != 0.0f) pw = lz > 0.0f ? or_exp2(L->n * or_log2(lz)) : 0.0f;
            float p_plain = ((L->n + 1.0f) * (float)0.15915494309189533577) * pw;
            float p_learn = (pdf[ps->ebin] * 512.0f) * pl3;
            float q = prop->alpha * p_plain + (1.0f - prop->alpha) * p_learn;
            ps->phi_r = q > 0.0f ? ps->phi_r * (p_plain / q) : 0.0f;
            ps->wq = q / (512.0f * pl3);
        }
        for (int c = 0; c < 3; ++c) dir[c] = (a * L->t[c] + bb * L->b[c]) + ct * L->d[c];
        if (L->type == 2) {
            ps->au = (u[0] - 0.5f) * L->w;
            ps->av = (u[1] - 0.5f) * L->h;
            for (int c = 0; c < 3; ++c) ps->y[c] = (L->c[c] + ps->au * L->t[c]) + ps->av * L->b[c];
        }
    }
}

/* The hit point of the ray at distance t on triangle prim: its patch, texel
 * (box basis), piecewise-linear nodes (Eq. pwLin on the texel grid: nodes at
 * the texel centres, bilinear hats clamped at the patch border so that they
 * sum to one; the mass-lumped weight of every node is the texel area,
 * supplement Eq. appdxSpatialCoeffs) and the normal facing the ray. */
static void locate_hit(const or_scene* S, const float* o, const float* dir, float t, int64_t prim, hit_point* hp)
{
    for (int c = 0; c < 3; ++c) hp->x[c] = o[c] + t * dir[c];
    const int32_t q = S->tri_patch[prim];
    const float* pf = S->pf + 17 * (int64_t)q;
    hp->q = q;
    hp->pf = pf;
    float du[3] = {hp->x[0] - pf[0], hp->x[1] - pf[1], hp->x[2] - pf[2]};
    float su = dot3(du, pf + 3) * pf[12];
    float sv = dot3(du, pf + 6) * pf[13];
    int32_t ru = S->pres[2 * q], rv = S->pres[2 * q + 1];
    int32_t iu = (int32_t)floorf(su * (float)ru);
    int32_t iv = (int32_t)floorf(sv * (float)rv);
    if (iu < 0) iu = 0;
    if (iu > ru - 1) iu = ru - 1;
    if (iv < 0) iv = 0;
    if (iv > rv - 1) iv = rv - 1;
    hp->k = S->pbase[q] + (int64_t)iv * ru + iu;
    hp->inv_a = pf[15];
    if (S->basis == 1) {
        float fu = su * (float)ru - 0.5f, fv = sv * (float)rv - 0.5f;
        float fu0 = floorf(fu), fv0 = floorf(fv);
        float au1 = fu - fu0, av1 = fv - fv0;
        float au0 = 1.0f - au1, av0 = 1.0f - av1;
        int32_t i0 = (int32_t)fu0, j0 = (int32_t)fv0;
        int32_t i1 = i0 + 1, j1 = j0 + 1;
        i0 = i0 < 0 ? 0 : (i0 > ru - 1 ? ru - 1 : i0);
        i1 = i1 < 0 ? 0 : (i1 > ru - 1 ? ru - 1 : i1);
        j0 = j0 < 0 ? 0 : (j0 > rv - 1 ? rv - 1 : j0);
        j1 = j1 < 0 ? 0 : (j1 > rv - 1 ? rv - 1 : j1);
        hp->kb[0] = S->pbase[q] + (int64_t)j0 * ru + i0; hp->wb[0] = au0 * av0;
        hp->kb[1] = S->pbase[q] + (int64_t)j0 * ru + i1; hp->wb[1] = au1 * av0;
        hp->kb[2] = S->pbase[q] + (int64_t)j1 * ru + i0; hp->wb[2] = au0 * av1;
        hp->kb[3] = S->pbase[q] + (int64_t)j1 * ru + i1; hp->wb[3] = au1 * av1;
    }
    const float* nq = pf + 9;
    float nd = dot3(nq, dir);
    if (nd < 0.0f) { hp->no[0] = nq[0]; hp->no[1] = nq[1]; hp->no[2] = nq[2]; }
    else { hp->no[0] = -nq[0]; hp->no[1] = -nq[1]; hp->no[2] = -nq[2]; }
}

static void splat(int64_t* S, int64_t k, float val)
{
    long long code = llrintf(val * 4294967296.0f);
#ifdef _OPENMP
#pragma omp atomic
#endif
    S[k] += code;
}

/* Directional texels at hit h: exitant radiance coefficients (HSH of order
 * dir_order, N' local samples of the BRDF lobe) splatted, and for the
 * adjoint the projected dO/dL sum and, at the first hit, the BRDF terms
 * that move with the incident direction. */
static void directional_hit(const or_scene* S, const olight* L, uint64_t seed, uint32_t i, uint32_t stream, int h,
                            const hit_point* hp, path_io* io, path_state* ps)
{
    const int64_t K = S->n_texels, k = hp->k;
    const int NC = (S->dir_order + 1) * (S->dir_order + 1);
    const float inv_np = 1.0f / (float)S->dir_samples;
    const int NP = L->rv ? 7 : (L->cone ? 8 : 6);
    const float* gl_ = S->glossy ? S->glossy + 2 * (int64_t)hp->q : NULL;
    float rs = gl_ ? gl_[0] : 0.0f, ex = gl_ ? gl_[1] : 1.0f;
    local_frame(hp->no, ps->fb1, ps->fb2);
    float wiw[3] = {-ps->dir[0], -ps->dir[1], -ps->dir[2]};
    ps->wi_loc[0] = dot3(ps->fb1, wiw); ps->wi_loc[1] = dot3(ps->fb2, wiw); ps->wi_loc[2] = dot3(hp->no, wiw);
    float acc_c[16] = {0};
    float pd = 0.0f, ql[3] = {0, 0, 0};
    for (int j = 0; j < S->dir_samples; ++j) {
        float us[4];
        draw4(seed, i, stream, or_dir_block((uint32_t)h, (uint32_t)j), us);
        float ua = (j & 1) ? us[2] : us[0], ub = (j & 1) ? us[3] : us[1];
        float ct = ua;
        float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
        float sp, cp;
        or_sincos2pi(ub, &sp, &cp);
        float wo[3] = {st * cp, st * sp, ct};
        float H[16];
        or_hsh(S->dir_order, ct, cp, sp, H);
        float gr[3];
        float f = or_brdf(hp->pf[16], rs, ex, ps->wi_loc, wo, (io->g && h == 1) ? gr : NULL);
        if (io->S)
            for (int c = 0; c < NC; ++c) acc_c[c] = acc_c[c] + f * H[c];
        if (io->g) {
            float G = 0.0f;
            for (int c = 0; c < NC; ++c) G = G + io->g[c * K + k] * H[c];
            pd = pd + f * G;
            if (h == 1)
                for (int c = 0; c < 3; ++c) ql[c] = ql[c] + G * gr[c];
        }
    }
    if (io->S) {
        float base = (ps->phi_r * ps->T) * hp->inv_a;
        for (int c = 0; c < NC; ++c) splat(io->S, c * K + k, (base * acc_c[c]) * inv_np);
    }
    if (io->g) {
        float P = (pd * inv_np) * hp->inv_a;
        ps->s_r = ps->s_r + P * ps->T;
        if (h >= 2) ps->Rd = ps->Rd + P * ps->T2;
        if (h == 1) {
            ps->k1 = k;
            float dl[8];
            first_hit_dlog(L, hp->x, ps->y, hp->no, ps->au, ps->av, dl);
            for (int c = 0; c < NP; ++c) ps->dphi[c] = ps->phi_r * dl[c];
            float sq = (inv_np * hp->inv_a);
            for (int c = 0; c < 3; ++c)
                ps->Qw[c] = ((ql[0] * sq) * ps->fb1[c] + (ql[1] * sq) * ps->fb2[c]) + (ql[2] * sq) * hp->no[c];
            float v1[3] = {ps->y[0] - hp->x[0], ps->y[1] - hp->x[1], ps->y[2] - hp->x[2]};
            float r1 = sqrtf(dot3(v1, v1));
            ps->inv_r1 = 1.0f / r1;
            for (int c = 0; c < 3; ++c) ps->om1[c] = v1[c] * ps->inv_r1;
        }
    }
}

/* Irradiance splats of a hit (Alg. 1): Phi_h / A_k into the hit texel, or
 * its bilinear shares into the four nodes; in colour, one per channel. */
static void splat_hit(const or_scene* S, const olight* L, const hit_point* hp, path_io* io, const path_state* ps)
{
    const int64_t K = S->n_texels;
    if (L->rgb) {
        for (int ch = 0; ch < 3; ++ch) splat(io->S, ch * K + hp->k, ((ps->phi_r * L->col[ch]) * ps->Tc[ch]) * hp->inv_a);
    } else {
        float val = (ps->phi_r * ps->T) * hp->inv_a;
        if (S->basis == 1) {
            for (int c = 0; c < 4; ++c) splat(io->S, hp->kb[c], val * hp->wb[c]);
        } else {
            splat(io->S, hp->k, val);
        }
    }
}

/* Direct (forward-mode) differentiation with x_1 held fixed: every hit of
 * the path adds d(Phi_h / A)/dp_j = (Phi_h / A) dlog_j of its first hit, in
 * its own texel. */
static void tangent_hit(const olight* L, int h, const hit_point* hp, path_io* io, path_state* ps)
{
    if (h == 1) {
        float dl[8];
        first_hit_dlog(L, hp->x, ps->y, hp->no, ps->au, ps->av, dl);
        ps->tdl = dl[io->tangent_param];
    }
    splat(io->tangent, hp->k, ((ps->phi_r * ps->T) * hp->inv_a) * ps->tdl);
}

/* Adjoint at a hit (Alg. 2, Eq. adjointFlux): g_k Phi_h / (A_k Phi_r) added
 * to the path's sum (bilinear gather for the linear basis, per channel in
 * colour); at the first hit, dlog Phi_r/dp with x_1 held fixed. */
static void adjoint_hit(const or_scene* S, const olight* L, int h, const hit_point* hp, path_io* io,
                        path_state* ps)
{
    const int64_t K = S->n_texels, k = hp->k;
    const int NP = L->rv ? 7 : (L->cone ? 8 : 6);
    if (L->rgb) {
        for (int ch = 0; ch < 3; ++ch) ps->sc[ch] = ps->sc[ch] + (io->g[ch * K + k] * hp->inv_a) * ps->Tc[ch];
    } else {
        float gk = io->g[k];
        if (S->basis == 1)
            gk = ((hp->wb[0] * io->g[hp->kb[0]] + hp->wb[1] * io->g[hp->kb[1]]) + hp->wb[2] * io->g[hp->kb[2]]) +
                 hp->wb[3] * io->g[hp->kb[3]];
        ps->s_r = ps->s_r + (gk * hp->inv_a) * ps->T;
    }
    if (h == 1) {
        ps->k1 = k;
        float dl[8];
        first_hit_dlog(L, hp->x, ps->y, hp->no, ps->au, ps->av, dl);
        for (int c = 0; c < NP; ++c) ps->dphi[c] = ps->phi_r * dl[c];
    }
}

/* Cosine-weighted bounce about the oriented normal (Malley's method in the
 * Duff et al. 2017 orthonormal basis); Phi_{h+1} = Phi_h rho, or the glossy
 * BRDF's bounce weight pi f for directional texels. */
static void bounce(const or_scene* S, uint64_t seed, uint32_t i, uint32_t stream, int h, const hit_point* hp,
                   path_state* ps)
{
    const float* no = hp->no;
    float ub[4];
    draw4(seed, i, stream, 1u + (uint32_t)h, ub);
    float sign = copysignf(1.0f, no[2]);
    float a = -1.0f / (sign + no[2]);
    float bxy = (no[0] * no[1]) * a;
    float b1[3] = {1.0f + ((sign * no[0]) * no[0]) * a, sign * bxy, -(sign * no[0])};
    float b2[3] = {bxy, sign + (no[1] * no[1]) * a, -no[1]};
    float rr = sqrtf(ub[0]);
    float sp, cp;
    or_sincos2pi(ub[1], &sp, &cp);
    float lx = rr * cp, ly = rr * sp;
    float lz = sqrtf(fmaxf(0.0f, 1.0f - ub[0]));
    for (int c = 0; c < 3; ++c) ps->dir[c] = (lx * b1[c] + ly * b2[c]) + lz * no[c];
    for (int c = 0; c < 3; ++c) ps->o[c] = hp->x[c];
    ps->skip = hp->q;
    if (S->dir_order >= 0) {
        const float* gl_ = S->glossy ? S->glossy + 2 * (int64_t)hp->q : NULL;
        float wo[3] = {dot3(ps->fb1, ps->dir), dot3(ps->fb2, ps->dir), dot3(no, ps->dir)};
        float gr[3];
        float fbv = or_brdf(hp->pf[16], gl_ ? gl_[0] : 0.0f, gl_ ? gl_[1] : 1.0f, ps->wi_loc, wo, gr);
        float wb = fbv * 3.14159265358979f;
        if (h == 1) {
            for (int c = 0; c < 3; ++c)
                ps->Dw[c] = ((gr[0] * 3.14159265358979f) * ps->fb1[c] + (gr[1] * 3.14159265358979f) * ps->fb2[c]) +
                            (gr[2] * 3.14159265358979f) * no[c];
        } else {
            ps->T2 = ps->T2 * wb;
        }
        ps->T = ps->T * wb;
    } else {
        ps->T = ps->T * hp->pf[16];
    }
    for (int ch = 0; ch < 3; ++ch) ps->Tc[ch] = ps->Tc[ch] * (S->albedo_rgb ? S->albedo_rgb[3 * hp->q + ch] : hp->pf[16]);
}

/* End of a path (Eq. objGradAdjoint, first term): dO/dp_j += s_r Phi_r
 * dlog_j (plus, for directional texels, the first hit's BRDF terms through
 * the incident direction); in colour the geometric terms take the
 * colour-weighted sum and dO/dcol_ch = s_ch Phi_r; the contribution map and
 * the proposal's histogram take the path's share. */
static void finish_path(const olight* L, int gl, const or_proposal* prop, const or_scene* S, path_io* io,
                        path_state* ps)
{
    const int NP = L->rv ? 7 : (L->cone ? 8 : 6);
    if (io->g && ps->hits >= 1 && L->rgb) {
        ps->s_r = (ps->sc[0] * L->col[0] + ps->sc[1] * L->col[1]) + ps->sc[2] * L->col[2];
        if (io->acc_col)
            for (int ch = 0; ch < 3; ++ch) io->acc_col[ch] += (double)(ps->sc[ch] * ps->phi_r);
    }
    if (io->g && ps->hits >= 1) {
        float cr[8];
        float ub_[3] = {0, 0, 0};
        float dya[3] = {0, 0, 0}, dyb[3] = {0, 0, 0};
        if (S->dir_order >= 0) {
            /* d/dy of the first hit's projection and bounce weight through the
             * incident direction om1 = (y - x_1)/|y - x_1| */
            float v[3];
            for (int c = 0; c < 3; ++c) v[c] = ps->Qw[c] + ps->Rd * ps->Dw[c];
            float wv = dot3(ps->om1, v);
            for (int c = 0; c < 3; ++c) ub_[c] = (v[c] - ps->om1[c] * wv) * ps->inv_r1;
            if (L->type == 2)
                for (int c = 0; c < 3; ++c) {
                    dya[c] = ps->av * L->db_da[c];
                    dyb[c] = ps->au * L->dt_db[c] + ps->av * L->db_db[c];
                }
        }
        float extra[6] = {ub_[0], ub_[1], ub_[2], dot3(ub_, dya), dot3(ub_, dyb), 0.0f};
        for (int c = 0; c < NP; ++c) {
            cr[c] = ps->s_r * ps->dphi[c];
            if (S->dir_order >= 0) cr[c] = cr[c] + ps->phi_r * extra[c];
            if (io->acc) io->acc[c] += (double)cr[c];
            if (io->contrib && c < 6) io->contrib[c] = cr[c];
        }
        if (io->vote) {
            /* the path's share of dO/dp_j goes to the texel of its first
             * surface hit (Sec. gradVis) */
#ifdef _OPENMP
#pragma omp atomic
#endif
            io->vote[ps->k1] += (double)cr[io->vote_param];
        }
        if (prop && prop->hist && ps->ebin >= 0) {
            const float* is = prop->inv_sigma + 6 * (int64_t)gl;
            float m2 = 0.0f;
            for (int c = 0; c < 6; ++c) {
                float z = cr[c] * is[c];
                m2 = m2 + z * z;
            }
            double v = (double)(m2 * ps->wq);
#ifdef _OPENMP
#pragma omp atomic
#endif
            prop->hist[1024 * (int64_t)gl + ps->ebin] += v;
        }
    } else if (io->contrib) {
        for (int c = 0; c < 6; ++c) io->contrib[c] = 0.0f;
    }
}

/* One light path of light gl: emission, then up to B hits, each splatting
 * its flux (forward), adding its share of the adjoint sum (adjoint), its
 * direct-differentiation splat or its record, then bouncing; the adjoint
 * quantities are accumulated at the end of the path. */
static void trace_path(const or_scene* S, const olight* L, int layout, int l_local, int gl, uint32_t i, uint64_t seed,
                       int B, const or_proposal* prop_in, path_io* io)
{
    const uint32_t stream = ((uint32_t)layout << 16) | (uint32_t)l_local;
    const or_proposal* prop = (prop_in && prop_in->pdf && (L->type == 1 || L->type == 2)) ? prop_in : NULL;
    path_state ps;
    memset(&ps, 0, sizeof(ps));
    emit_path(L, seed, i, stream, gl, prop, &ps);
    for (int c = 0; c < 3; ++c) ps.o[c] = ps.y[c];
    ps.skip = -1;
    ps.T = 1.0f;
    ps.k1 = -1;
    ps.T2 = 1.0f;
    for (int ch = 0; ch < 3; ++ch) ps.Tc[ch] = 1.0f;
    const int dirm = S->dir_order >= 0;
    for (int h = 1; h <= B; ++h) {
        float t;
        int64_t prim = intersect(S, ps.o, ps.dir, ps.skip, &t);
        if (prim < 0) {
            io->misses++;
            break;
        }
        ps.hits = h;
        hit_point hp;
        locate_hit(S, ps.o, ps.dir, t, prim, &hp);
        if (dirm) directional_hit(S, L, seed, i, stream, h, &hp, io, &ps);
        else if (io->S) splat_hit(S, L, &hp, io, &ps);
        if (io->tangent) tangent_hit(L, h, &hp, io, &ps);
        if (io->g && !dirm) adjoint_hit(S, L, h, &hp, io, &ps);
        if (io->rec_prim) {
            io->rec_prim[h - 1] = (int32_t)prim;
            io->rec_texel[h - 1] = (int32_t)hp.k;
        }
        if (h == B) break;
        bounce(S, seed, i, stream, h, &hp, &ps);
    }
    finish_path(L, gl, prop, S, io, &ps);
}

/* ------------------------------------------------------------------------- */
/* Entry points                                                               */
/* ------------------------------------------------------------------------- */

/* Primal light tracing (Alg. 1).  S_out: [n_layouts, K] int64, overwritten.
 * limit_per_light > 0 traces only the first paths of each light (still with
 * Phi_r = P / N_l of the full path count). */
EXPORT int64_t or_forward(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed,
                          int64_t paths_per_layout, int max_hits, int64_t limit_per_light, int n_threads,
                          const or_proposal* prop, int64_t* S_out)
{
    /* colour mode: [n_layouts, 3, K] */
    const int64_t stride = (S->dir_order >= 0 ? (S->dir_order + 1) * (S->dir_order + 1) : (Ls->colour ? 3 : 1)) *
                           S->n_texels;
    memset(S_out, 0, (size_t)(stride * Ls->n_layouts) * sizeof(int64_t));
    int64_t misses = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    for (int j = 0; j < Ls->n_layouts; ++j) {
        int l0 = Ls->layout_offsets[j], l1 = Ls->layout_offsets[j + 1];
        for (int gl = l0; gl < l1; ++gl) {
            olight L;
            int64_t nl = paths_of_light(paths_per_layout, l1 - l0, gl - l0);
            light_setup(Ls, params, gl, nl, &L);
            /* a luminaire of zero power carries flux P / N = 0 on every path
             * (Alg. 1), so each of its splats is zero: it is not traced */
            if (L.P == 0.0f) continue;
            int64_t lim = (limit_per_light > 0 && limit_per_light < nl) ? limit_per_light : nl;
            int64_t m = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : m)
#endif
            for (int64_t i = 0; i < lim; ++i) {
                path_io io;
                memset(&io, 0, sizeof(io));
                io.S = S_out + (int64_t)j * stride;
                trace_path(S, &L, j, gl - l0, gl, (uint32_t)i, seed, max_hits, prop, &io);
                m += io.misses;
            }
            misses += m;
        }
    }
    return misses;
}

/* Adjoint light tracing (Alg. 2).  dOdE: [n_layouts, K] ([n_layouts, 3, K]
 * in colour mode); grad_out: [L,6] FP64; grad_colour: [L,3] FP64 in colour
 * mode (may be NULL). */
EXPORT int64_t or_adjoint(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed,
                          int64_t paths_per_layout, int max_hits, int64_t limit_per_light, int n_threads,
                          const or_proposal* prop, const float* dOdE, double* grad_out, double* grad_colour)
{
    const int64_t stride = (S->dir_order >= 0 ? (S->dir_order + 1) * (S->dir_order + 1) : (Ls->colour ? 3 : 1)) *
                           S->n_texels;
    if (Ls->rotvec) return -1;   /* or_adjoint_rv */
    int64_t misses = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    for (int j = 0; j < Ls->n_layouts; ++j) {
        int l0 = Ls->layout_offsets[j], l1 = Ls->layout_offsets[j + 1];
        for (int gl = l0; gl < l1; ++gl) {
            olight L;
            int64_t nl = paths_of_light(paths_per_layout, l1 - l0, gl - l0);
            light_setup(Ls, params, gl, nl, &L);
            if (L.P == 0.0f) {
                /* zero power: the replayed paths (Alg. 2 follows Alg. 1's)
                 * carry no flux and dO/dP is a 0/0 form there, so the
                 * luminaire is not traced and its row is zero */
                for (int c = 0; c < 6; ++c) grad_out[6 * (int64_t)gl + c] = 0.0;
                if (grad_colour)
                    for (int c = 0; c < 3; ++c) grad_colour[3 * (int64_t)gl + c] = 0.0;
                continue;
            }
            int64_t lim = (limit_per_light > 0 && limit_per_light < nl) ? limit_per_light : nl;
            double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, c0 = 0, c1 = 0, c2 = 0;
            int64_t m = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : a0, a1, a2, a3, a4, a5, c0, c1, c2, m)
#endif
            for (int64_t i = 0; i < lim; ++i) {
                double acc[6] = {0, 0, 0, 0, 0, 0};
                double accc[3] = {0, 0, 0};
                path_io io;
                memset(&io, 0, sizeof(io));
                io.g = dOdE + (int64_t)j * stride;
                io.acc = acc;
                io.acc_col = accc;
                trace_path(S, &L, j, gl - l0, gl, (uint32_t)i, seed, max_hits, prop, &io);
                a0 += acc[0]; a1 += acc[1]; a2 += acc[2]; a3 += acc[3]; a4 += acc[4]; a5 += acc[5];
                c0 += accc[0]; c1 += accc[1]; c2 += accc[2];
                m += io.misses;
            }
            double* g = grad_out + 6 * (int64_t)gl;
            g[0] = a0; g[1] = a1; g[2] = a2; g[3] = a3; g[4] = a4; g[5] = a5;
            if (grad_colour) {
                double* gc = grad_colour + 3 * (int64_t)gl;
                gc[0] = c0; gc[1] = c1; gc[2] = c2;
            }
            misses += m;
        }
    }
    return misses;
}

/* Adjoint light tracing with rotation-vector orientation (Sec. 4.4.2):
 * params [L,7] = (x, y, z, theta, P); grad_out [L,7] FP64 = dO/d(x, y, z,
 * theta, P), the per-path world-rotation derivatives mapped through J^T. */
/* Adjoint with the soft-edged spots' cone angles: grad_out [L,6] as
 * or_adjoint, grad_cone [L,2] = dO/d(theta_in, theta_out) (0 for other
 * luminaire types).  Grey, box basis, irradiance texels, tilt angles. */
EXPORT int64_t or_adjoint_cone(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed,
                               int64_t paths_per_layout, int max_hits, int n_threads, const float* dOdE,
                               double* grad_out, double* grad_cone)
{
    if (Ls->rotvec || Ls->colour || S->dir_order >= 0 || S->basis != 0) return -1;
    int64_t misses = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    for (int j = 0; j < Ls->n_layouts; ++j) {
        int l0 = Ls->layout_offsets[j], l1 = Ls->layout_offsets[j + 1];
        for (int gl = l0; gl < l1; ++gl) {
            olight L;
            int64_t nl = paths_of_light(paths_per_layout, l1 - l0, gl - l0);
            light_setup(Ls, params, gl, nl, &L);
            L.cone = 1;
            double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0, a7 = 0;
            int64_t m = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : a0, a1, a2, a3, a4, a5, a6, a7, m)
#endif
            for (int64_t i = 0; i < nl; ++i) {
                double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                path_io io;
                memset(&io, 0, sizeof(io));
                io.g = dOdE + (int64_t)j * S->n_texels;
                io.acc = acc;
                trace_path(S, &L, j, gl - l0, gl, (uint32_t)i, seed, max_hits, NULL, &io);
                a0 += acc[0]; a1 += acc[1]; a2 += acc[2]; a3 += acc[3];
                a4 += acc[4]; a5 += acc[5]; a6 += acc[6]; a7 += acc[7];
                m += io.misses;
            }
            a[0] = a0; a[1] = a1; a[2] = a2; a[3] = a3; a[4] = a4; a[5] = a5; a[6] = a6; a[7] = a7;
            for (int c = 0; c < 6; ++c) grad_out[6 * (int64_t)gl + c] = a[c];
            grad_cone[2 * (int64_t)gl] = a[6];
            grad_cone[2 * (int64_t)gl + 1] = a[7];
            misses += m;
        }
    }
    return misses;
}

EXPORT void or_first_hit_dlog_cone(const or_lights* Ls, const float* params, int gl, const float* x1,
                                   const float* y, const float* n1, float* dl)
{
    olight L;
    light_setup(Ls, params, gl, 1, &L);
    L.cone = 1;
    first_hit_dlog(&L, x1, y, n1, 0.0f, 0.0f, dl);
}

EXPORT int64_t or_adjoint_rv(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed,
                             int64_t paths_per_layout, int max_hits, int n_threads, const float* dOdE,
                             double* grad_out)
{
    if (!Ls->rotvec || Ls->colour || S->dir_order >= 0) return -1;
    int64_t misses = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    for (int j = 0; j < Ls->n_layouts; ++j) {
        int l0 = Ls->layout_offsets[j], l1 = Ls->layout_offsets[j + 1];
        for (int gl = l0; gl < l1; ++gl) {
            olight L;
            int64_t nl = paths_of_light(paths_per_layout, l1 - l0, gl - l0);
            light_setup(Ls, params, gl, nl, &L);
            double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0;
            int64_t m = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : a0, a1, a2, a3, a4, a5, a6, m)
#endif
            for (int64_t i = 0; i < nl; ++i) {
                double acc[7] = {0, 0, 0, 0, 0, 0, 0};
                path_io io;
                memset(&io, 0, sizeof(io));
                io.g = dOdE + (int64_t)j * S->n_texels;
                io.acc = acc;
                trace_path(S, &L, j, gl - l0, gl, (uint32_t)i, seed, max_hits, NULL, &io);
                a0 += acc[0]; a1 += acc[1]; a2 += acc[2]; a3 += acc[3]; a4 += acc[4]; a5 += acc[5]; a6 += acc[6];
                m += io.misses;
            }
            const float* p = params + 7 * gl;
            double th[3] = {(double)p[3], (double)p[4], (double)p[5]}, J[9];
            rot_jacobian(th, J);
            double* g = grad_out + 7 * (int64_t)gl;
            g[0] = a0; g[1] = a1; g[2] = a2; g[6] = a6;
            for (int c = 0; c < 3; ++c) g[3 + c] = (J[c] * a3 + J[3 + c] * a4) + J[6 + c] * a5;
            misses += m;
        }
    }
    return misses;
}

/* Direct-differentiation map (the comparison of Sec. gradVis): dE_k/dp_j of
 * light gl's paths with every first hit held fixed, as Q31.32 fixed point in
 * tangent_out [K] (texels of the light's layout), overwritten.  Summed
 * against dO/dE it gives the adjoint gradient dO/dp_j of that light. */
EXPORT int64_t or_tangent(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed,
                          int64_t paths_per_layout, int max_hits, int n_threads, int gl, int param,
                          int64_t* tangent_out)
{
    if (Ls->colour || Ls->rotvec || S->dir_order >= 0 || S->basis != 0) return -1;
    int j = 0;
    while (Ls->layout_offsets[j + 1] <= gl) ++j;
    int l0 = Ls->layout_offsets[j], l1 = Ls->layout_offsets[j + 1];
    memset(tangent_out, 0, (size_t)S->n_texels * sizeof(int64_t));
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    olight L;
    int64_t nl = paths_of_light(paths_per_layout, l1 - l0, gl - l0);
    light_setup(Ls, params, gl, nl, &L);
    int64_t m = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : m)
#endif
    for (int64_t i = 0; i < nl; ++i) {
        path_io io;
        memset(&io, 0, sizeof(io));
        io.tangent = tangent_out;
        io.tangent_param = param;
        trace_path(S, &L, j, gl - l0, gl, (uint32_t)i, seed, max_hits, NULL, &io);
        m += io.misses;
    }
    return m;
}

/* the rotation-vector frame and Jacobian, for the pins */
EXPORT void or_rotvec(const double* th, double* R, double* J)
{
    rodrigues(th, R);
    rot_jacobian(th, J);
}

/* Gradient-contribution map of one light gl and one parameter j (Sec.
 * gradVis): the adjoint pass of Alg. 2 over the paths of that light, where
 * each path adds its contribution to dO/dp_j into the texel of its first
 * surface hit.  vote_out: [K] FP64 over the texels of the light's layout,
 * overwritten; grad_out: [6] FP64, the light's gradient (the map sums to
 * grad_out[j]). */
EXPORT int64_t or_votes(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed,
                        int64_t paths_per_layout, int max_hits, int64_t limit_per_light, int n_threads,
                        const or_proposal* prop, const float* dOdE, int gl, int param, double* vote_out,
                        double* grad_out)
{
    if (Ls->colour) return -1;   /* grey only */
    int j = 0;
    while (Ls->layout_offsets[j + 1] <= gl) ++j;
    int l0 = Ls->layout_offsets[j], l1 = Ls->layout_offsets[j + 1];
    memset(vote_out, 0, (size_t)S->n_texels * sizeof(double));
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    olight L;
    int64_t nl = paths_of_light(paths_per_layout, l1 - l0, gl - l0);
    light_setup(Ls, params, gl, nl, &L);
    int64_t lim = (limit_per_light > 0 && limit_per_light < nl) ? limit_per_light : nl;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
    int64_t m = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : a0, a1, a2, a3, a4, a5, m)
#endif
    for (int64_t i = 0; i < lim; ++i) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        path_io io;
        memset(&io, 0, sizeof(io));
        io.g = dOdE + (int64_t)j * S->n_texels;
        io.acc = acc;
        io.vote = vote_out;
        io.vote_param = param;
        trace_path(S, &L, j, gl - l0, gl, (uint32_t)i, seed, max_hits, prop, &io);
        a0 += acc[0]; a1 += acc[1]; a2 += acc[2]; a3 += acc[3]; a4 += acc[4]; a5 += acc[5];
        m += io.misses;
    }
    grad_out[0] = a0; grad_out[1] = a1; grad_out[2] = a2; grad_out[3] = a3; grad_out[4] = a4; grad_out[5] = a5;
    return m;
}

/* ------------------------------------------------------------------------- */
/* Object-space path tracing with next-event estimation: the comparison     */
/* estimator of Sec. 6 (after Stam 2020), built on the same texels: sample   */
/* points uniformly in each texel, connect every path vertex to one light   */
/* chosen uniformly (shadow ray), continue with the light tracer's cosine    */
/* bounce.  Its gradient differentiates each light connection with the       */
/* vertex held fixed, which is the first-hit derivative above evaluated at   */
/* that vertex.                                                               */
/* ------------------------------------------------------------------------- */

/* radiant intensity of light L towards unit direction w (from its origin),
 * with L->phi_r = P (or P kcap for the soft-edged spot: n_paths = 1) */
static float light_intensity(const olight* L, const float* w)
{
    if (L->type == 0) return L->phi_r * 0.07957747154594767f;
    float ce = dot3(L->d, w);
    if (L->type == 3) {
        if (!(ce > L->co)) return 0.0f;
        float a = 1.0f;
        if (ce < L->ci) {
            float f = (ce - L->co) / (L->ci - L->co);
            a = f * f;
        }
        return (L->phi_r * a) * (0.15915494309189533f / (1.0f - L->co));
    }
    if (!(ce > 0.0f)) return 0.0f;
    float pw = 1.0f;
    if (L->n != 0.0f) pw = or_exp2(L->n * or_log2(ce));
    return L->phi_r * (((L->n + 1.0f) * 0.15915494309189533f) * pw);
}

/* one light connection from vertex v (patch qv, unit normal nq); side < 0:
 * either side (the one facing the light), else the side of normal nside.
 * Returns the unoccluded-or-zero irradiance term I cos / r^2 and, for the
 * gradient, the light's derivative factors with v fixed. */
static float connect_light(const or_scene* S, const olight* L, const float* v, int32_t qv, const float* nq,
                           const float* nside, const float* ul, float dl[6])
{
    float y[3] = {L->c[0], L->c[1], L->c[2]};
    float au = 0.0f, av = 0.0f;
    if (L->type == 2) {
        au = (ul[0] - 0.5f) * L->w;
        av = (ul[1] - 0.5f) * L->h;
        for (int c = 0; c < 3; ++c) y[c] = (L->c[c] + au * L->t[c]) + av * L->b[c];
    }
    float vec[3] = {v[0] - y[0], v[1] - y[1], v[2] - y[2]};
    float r2 = dot3(vec, vec);
    if (!(r2 > 1e-12f)) return 0.0f;
    float r = sqrtf(r2);
    float inv_r = 1.0f / r;
    float w[3] = {vec[0] * inv_r, vec[1] * inv_r, vec[2] * inv_r};
    float n1[3];
    if (nside) {
        n1[0] = nside[0]; n1[1] = nside[1]; n1[2] = nside[2];
    } else if (dot3(nq, w) < 0.0f) {
        n1[0] = nq[0]; n1[1] = nq[1]; n1[2] = nq[2];
    } else {
        n1[0] = -nq[0]; n1[1] = -nq[1]; n1[2] = -nq[2];
    }
    float cv = -dot3(n1, w);
    if (!(cv > 0.0f)) return 0.0f;
    float I = light_intensity(L, w);
    if (!(I > 0.0f)) return 0.0f;
    float C = (I * cv) / r2;
    /* shadow ray from v towards the light sample */
    float sd[3] = {-w[0], -w[1], -w[2]};
    float t;
    int64_t prim = intersect(S, v, sd, qv, &t);
    if (prim >= 0 && t < r * 0.9999f) return 0.0f;
    if (dl) first_hit_dlog(L, v, y, n1, au, av, dl);
    return C;
}

/* One layout's samples: M per texel, vertex 0 uniform in the texel, up to
 * max_hits - 1 bounces.  Forward: S_out [K] int64 (Q31.32 of the texel's
 * mean irradiance).  With dOdE [K]: grad_out [L,6] FP64 += sum_k dO/dE_k
 * dE_k/dp. */
static void pt_layout(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed, int M,
                      int max_hits, int j, const int32_t* texel_patch, const float* dOdE, int64_t* S_out,
                      double* grad_out)
{
    int l0 = Ls->layout_offsets[j], l1 = Ls->layout_offsets[j + 1];
    int nl = l1 - l0;
    olight* Lt = (olight*)malloc(sizeof(olight) * (size_t)nl);
    for (int l = 0; l < nl; ++l) light_setup(Ls, params, l0 + l, 1, &Lt[l]);
    const uint32_t stream = ((uint32_t)j << 16) | 0xFFFFu;
    const float inv_m = 1.0f / (float)M;
    const float fl = (float)nl;
    const int64_t total = S->n_texels * (int64_t)M;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < total; ++i) {
        int64_t k = i / M;
        int32_t q = texel_patch[k];
        const float* pf = S->pf + 17 * (int64_t)q;
        int32_t ru = S->pres[2 * q];
        int64_t loc = k - S->pbase[q];
        int32_t iu = (int32_t)(loc % ru), iv = (int32_t)(loc / ru);
        float u[4];
        draw4(seed, (uint32_t)i, stream, 0u, u);
        float su = ((float)iu + u[0]) / (float)ru;
        float sv = ((float)iv + u[1]) / (float)S->pres[2 * q + 1];
        float x[3];
        for (int c = 0; c < 3; ++c) x[c] = (pf[c] + su * pf[3 + c]) + sv * pf[6 + c];
        const float* nq = pf + 9;
        float gk = dOdE ? dOdE[k] * inv_m : 0.0f;
        float e = 0.0f;
        float T = 1.0f;
        float v[3] = {x[0], x[1], x[2]};
        int32_t qv = q;
        float nside[3];
        int have_side = 0;
        for (int h = 0; h < max_hits; ++h) {
            /* light connection at vertex h */
            float ul[4];
            draw4(seed, (uint32_t)i, stream, 1u + 2u * (uint32_t)h, ul);
            int ls = (int)(ul[0] * fl);
            if (ls > nl - 1) ls = nl - 1;
            float dl[6];
            const float* nqv = S->pf + 17 * (int64_t)qv + 9;
            float C = connect_light(S, &Lt[ls], v, qv, nqv, have_side ? nside : NULL, ul + 1, dOdE ? dl : NULL);
            if (C > 0.0f) {
                float we = (T * fl) * C;
                e = e + we;
                if (dOdE) {
                    double* g = grad_out + 6 * (int64_t)(l0 + ls);
                    for (int c = 0; c < 6; ++c) {
                        double cr = (double)((gk * we) * dl[c]);
#ifdef _OPENMP
#pragma omp atomic
#endif
                        g[c] += cr;
                    }
                }
            }
            if (h == max_hits - 1) break;
            /* bounce: at vertex 0 a side drawn with probability 1/2 (weight 2),
             * later the side facing the incoming ray */
            float no[3];
            if (!have_side) {
                float sg = u[2] < 0.5f ? 1.0f : -1.0f;
                for (int c = 0; c < 3; ++c) no[c] = sg * nq[c];
                T = T * 2.0f;
            } else {
                for (int c = 0; c < 3; ++c) no[c] = nside[c];
            }
            float ub[4];
            draw4(seed, (uint32_t)i, stream, 2u + 2u * (uint32_t)h, ub);
            float sign = copysignf(1.0f, no[2]);
            float a = -1.0f / (sign + no[2]);
            float bxy = (no[0] * no[1]) * a;
            float b1[3] = {1.0f + ((sign * no[0]) * no[0]) * a, sign * bxy, -(sign * no[0])};
            float b2[3] = {bxy, sign + (no[1] * no[1]) * a, -no[1]};
            float rr = sqrtf(ub[0]);
            float sp, cp;
            or_sincos2pi(ub[1], &sp, &cp);
            float lx = rr * cp, ly = rr * sp;
            float lz = sqrtf(fmaxf(0.0f, 1.0f - ub[0]));
            float dir[3];
            for (int c = 0; c < 3; ++c) dir[c] = (lx * b1[c] + ly * b2[c]) + lz * no[c];
            float t;
            int64_t prim = intersect(S, v, dir, qv, &t);
            if (prim < 0) break;
            float xn[3];
            for (int c = 0; c < 3; ++c) xn[c] = v[c] + t * dir[c];
            int32_t qn = S->tri_patch[prim];
            const float* pn = S->pf + 17 * (int64_t)qn;
            float nd = dot3(pn + 9, dir);
            for (int c = 0; c < 3; ++c) nside[c] = nd < 0.0f ? pn[9 + c] : -pn[9 + c];
            have_side = 1;
            T = T * pn[16];
            for (int c = 0; c < 3; ++c) v[c] = xn[c];
            qv = qn;
        }
        if (S_out) {
            long long code = llrintf((e * inv_m) * 4294967296.0f);
#ifdef _OPENMP
#pragma omp atomic
#endif
            S_out[k] += code;
        }
    }
    free(Lt);
}

EXPORT void or_pt(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed, int M, int max_hits,
                  int n_threads, const float* dOdE, int64_t* S_out, double* grad_out)
{
    if (Ls->colour) return;   /* grey only */
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    int32_t* texel_patch = (int32_t*)malloc(sizeof(int32_t) * (size_t)S->n_texels);
    for (int32_t q = 0; q < S->n_patches; ++q) {
        int64_t n = (int64_t)S->pres[2 * q] * S->pres[2 * q + 1];
        for (int64_t k = 0; k < n; ++k) texel_patch[S->pbase[q] + k] = q;
    }
    if (S_out) memset(S_out, 0, (size_t)(S->n_texels * Ls->n_layouts) * sizeof(int64_t));
    if (grad_out) memset(grad_out, 0, sizeof(double) * 6 * (size_t)Ls->n_lights);
    for (int j = 0; j < Ls->n_layouts; ++j)
        pt_layout(S, Ls, params, seed, M, max_hits, j, texel_patch, dOdE ? dOdE + (int64_t)j * S->n_texels : NULL,
                  S_out ? S_out + (int64_t)j * S->n_texels : NULL, grad_out);
    free(texel_patch);
}

/* Hit sequences (primitive and texel per hit, -1 = none) of paths
 * [first, first+count) of one light; with dOdE also the per-path
 * contribution dO/dPhi_r * dPhi_r/dp [count,6]. */
EXPORT void or_record(const or_scene* S, const or_lights* Ls, const float* params, uint64_t seed,
                      int64_t paths_per_layout, int max_hits, int layout, int l_local, int64_t first,
                      int64_t count, const or_proposal* prop, int32_t* prim_out, int32_t* texel_out,
                      const float* dOdE, float* contrib)
{
    if (Ls->colour) return;   /* grey only */
    int l0 = Ls->layout_offsets[layout], l1 = Ls->layout_offsets[layout + 1];
    int gl = l0 + l_local;
    olight L;
    light_setup(Ls, params, gl, paths_of_light(paths_per_layout, l1 - l0, l_local), &L);
    for (int64_t r = 0; r < count; ++r) {
        path_io io;
        memset(&io, 0, sizeof(io));
        for (int h = 0; h < max_hits; ++h) {
            prim_out[r * max_hits + h] = -1;
            texel_out[r * max_hits + h] = -1;
        }
        io.rec_prim = prim_out + r * max_hits;
        io.rec_texel = texel_out + r * max_hits;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        if (dOdE) {
            io.g = dOdE + (int64_t)layout * S->n_texels;
            io.acc = acc;
            io.contrib = contrib + 6 * r;
        }
        trace_path(S, &L, layout, l_local, gl, (uint32_t)(first + r), seed, max_hits, prop, &io);
    }
}

/* E_k = S_k 2^-32 (Q31.32 fixed point to float through FP64). */
EXPORT void or_fixed_to_float(const int64_t* S, int64_t n, float* E)
{
    for (int64_t k = 0; k < n; ++k) E[k] = (float)((double)S[k] * 0x1p-32);
}

/* Eq. objective with alpha_l = 1: O = 1/2 sum_k A_k alpha_k (E_k - E*_k)^2
 * (FP64 sum); g_k = (A_k alpha_k)(E_k - E*_k) in FP32.  A is per texel and
 * repeats for every layout (n = n_layouts * K). */
EXPORT double or_objective(const float* E, const float* Et, const float* alpha, const float* A, int64_t K,
                           int64_t n, float* g)
{
    double O = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        float a = A[i % K];
        float al = alpha ? alpha[i] : 1.0f;
        if (g) g[i] = (a * al) * (E[i] - Et[i]);
        double e = (double)E[i] - (double)Et[i];
        O += (double)a * (double)al * e * e;
    }
    return 0.5 * O;
}

/* light frame as the oracle computes it: [L, 3+3+3+3+15+2] for the pins */
EXPORT void or_light_frames(const or_lights* Ls, const float* params, int64_t paths_per_layout, float* out)
{
    for (int j = 0; j < Ls->n_layouts; ++j) {
        int l0 = Ls->layout_offsets[j], l1 = Ls->layout_offsets[j + 1];
        for (int gl = l0; gl < l1; ++gl) {
            olight L;
            light_setup(Ls, params, gl, paths_of_light(paths_per_layout, l1 - l0, gl - l0), &L);
            float* o = out + 29 * (int64_t)gl;
            memcpy(o, L.c, 12); memcpy(o + 3, L.d, 12); memcpy(o + 6, L.t, 12); memcpy(o + 9, L.b, 12);
            memcpy(o + 12, L.dd_da, 12); memcpy(o + 15, L.dd_db, 12); memcpy(o + 18, L.dt_db, 12);
            memcpy(o + 21, L.db_da, 12); memcpy(o + 24, L.db_db, 12);
            o[27] = L.phi_r;
            o[28] = (float)L.n_paths;
        }
    }
}

/* the first-hit derivative alone, for the closed-form pins */
EXPORT void or_first_hit_dlog(const or_lights* Ls, const float* params, int gl, const float* x1,
                              const float* y, const float* n1, float au, float av, float* dl)
{
    olight L;
    light_setup(Ls, params, gl, 1, &L);
    first_hit_dlog(&L, x1, y, n1, au, av, dl);
}

EXPORT int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
