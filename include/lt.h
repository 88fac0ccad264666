/*
 * lt.h -- C ABI of the MI355X light-tracing library (liblt.so).
 *
 * The library implements the hot path of view-independent adjoint light
 * tracing (Lipp et al., "View-Independent Adjoint Light Tracing for Lighting
 * Design Optimization"): a primal light-tracing pass that splats the flux of
 * light paths into per-surface texels, and an adjoint pass that replays the
 * same paths and returns dO/dp for every luminaire parameter.  All work runs
 * in hand-written HIP kernels for gfx950.
 *
 * Conventions
 *   - Every function returns LT_OK (0) or a negative LT_E* code and never
 *     throws.  lt_last_error() gives a message owned by the context.
 *   - Arguments named h_* are host pointers, d_* are device pointers on the
 *     context's device.  The caller owns every d_* buffer; output buffers are
 *     overwritten completely (never accumulated into).  The context owns the
 *     scene, its BVH, the luminaire tables and all internal scratch.
 *   - All device work is enqueued on the context's stream (lt_set_stream) and
 *     is asynchronous; argument validation is synchronous.  Device-side
 *     conditions (fixed-point overflow) surface in lt_sync().
 *   - One context per host thread; calls on one context are not thread-safe.
 *
 * Paper notation: Phi_r flux per light ray, E_k irradiance of texel k (the
 * n = 0 coefficient of the radiance data structure up to the constant
 * rho_k / pi), A_k texel area, alpha_k texel weight, p = (c_x, c_y, c_z,
 * alpha, beta, P) per luminaire.
 */
#ifndef LT_H
#define LT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LT_OK 0
#define LT_EINVAL (-1)    /* bad argument (shape, range, NaN, missing state) */
#define LT_ENOMEM (-2)    /* device allocation failed */
#define LT_EHIP (-3)      /* HIP runtime error (message in lt_last_error) */
#define LT_ESTATE (-4)    /* call order violated (e.g. trace before upload) */
#define LT_EOVERFLOW (-5) /* a texel accumulator reached 2^62 (fixed point) */

/* lt_trace_cfg.flags */
#define LT_FLAG_GRAPH 1u    /* replay the launch sequence as a captured hipGraph */
#define LT_FLAG_PROPOSAL 2u /* sample emission from the learned proposal (MIS) */
/* piecewise-linear texel basis (Eq. pwLin with the supplement's mass-lumped
 * projection): nodes at the texel centres, bilinear hats clamped at each
 * patch border so that they sum to one; a hit splats into its four nearest
 * nodes and the adjoint gathers dO/dE with the same weights.  Without it a
 * hit splats into the one texel that contains it (box basis). */
#define LT_FLAG_LINEAR 4u

/* lt_sync flags_out bits */
#define LT_STATUS_OVERFLOW 1u  /* a texel accumulator reached 2^62 */
#define LT_STATUS_TRAVERSAL 2u /* a traversal exceeded its node-visit bound (malformed BVH) */
/* a luminaire parameter passed to a trace call was NaN or infinite, or its
 * power P was not positive; that luminaire traced no path (zero texel
 * contribution, zero gradient row) */
#define LT_STATUS_PARAMS 4u

typedef struct lt_ctx lt_ctx;

/* A planar rectangular surface patch with a res_u x res_v texel grid.
 * Triangles of the scene reference patches; a hit point x on patch q falls in
 * texel texel_base + j*res_u + i with
 *   i = clamp(floor(((x - origin).e_u * inv_len2_u) * res_u), 0, res_u-1)
 * and likewise j with e_v.  All constants are given (never recomputed). */
typedef struct {
    float origin[3];
    float e_u[3];
    float e_v[3];
    float normal[3];        /* unit normal of the plane (either side) */
    float inv_len2_u;       /* 1/|e_u|^2 */
    float inv_len2_v;       /* 1/|e_v|^2 */
    float texel_area;       /* A_k of each texel of the patch (m^2) */
    float inv_texel_area;   /* 1/A_k */
    float albedo;           /* Lambertian reflectance rho in [0,1] */
    int32_t res_u, res_v;
    int32_t pad;
    int64_t texel_base;     /* first texel index of the patch */
} lt_patch;                 /* 88 bytes */

/* Static luminaire attributes.  type: 0 isotropic point light (Phi_r = P/N),
 * 1 spot with radiant intensity P (n+1)/(2 pi) cos^n about its axis,
 * 2 rectangle size_w x size_h with the same cos^n lobe per unit area
 * (n = 1 is the paper's cosine area light), 3 soft-edged spot (supplement,
 * spot light): constant intensity inside the cone of half-angle size_w,
 * falling off as ((cos - cos_out) / (cos_in - cos_out))^2 out to size_h
 * (0 <= size_w < size_h <= pi/2, lobe_n 0), directions uniform over the
 * outer cone and weighted.  P is always the total emitted flux.  The
 * learned emission proposal applies to types 1 and 2 only.  Lights are
 * grouped by layout. */
typedef struct {
    int32_t type;
    float lobe_n;
    float size_w, size_h;
    int32_t layout;
} lt_light_static;          /* 20 bytes */

/* Per-call tracing configuration. */
typedef struct {
    uint64_t seed;             /* Philox key; the same seed replays the same paths */
    int64_t paths_per_layout;  /* N per layout, split evenly over its lights */
    int32_t max_hits;          /* B: hits per path (2 indirect bounces = 3) */
    uint32_t flags;            /* LT_FLAG_* */
    float alpha_plain;         /* one-sample MIS: probability of the plain lobe */
    int32_t reserved;
} lt_trace_cfg;                /* 32 bytes */

/* Launch tuning (chosen by lt_autotune or set by hand). */
typedef struct {
    int32_t waves_per_block;   /* 1, 2 or 4 waves per workgroup of the persistent trace launch */
    int32_t xcd_remap;         /* 1: eight work queues, one contiguous share of the tiles per XCD; a wave
                                  drains its XCD's queue first, then helps the others */
    int32_t tile_paths;        /* paths per work tile (multiple of 64), 0 = automatic */
    int32_t refill_threshold;  /* lanes that must finish a segment before hit processing */
    int32_t lds_depth;         /* traversal stack entries kept in LDS: 16 or 32 (the plain and
                                  colour adjoint keep at most 13 and 12, the most their
                                  occupancy leaves room for); the rest overflows to a
                                  device buffer the context sizes by the tree's depth */
    int32_t tri_share;         /* 1..8: a traversal iteration runs the queued triangle tests once at
                                  least tri_share/8 of the traversing lanes hold some (or all do),
                                  node steps otherwise; 0: both kinds in every iteration */
    int32_t reserved[2];
} lt_tuning;

typedef struct {
    int64_t n_tris, n_patches, n_texels;
    int32_t bvh_nodes, bvh_depth;   /* 4-wide nodes, levels */
    int64_t device_bytes;
    int32_t n_lights, n_layouts;
} lt_info;

/* Context on HIP device `device`; `hip_stream` (hipStream_t, may be NULL for
 * the null stream) receives all work. */
int lt_create(int device, void* hip_stream, lt_ctx** out);
void lt_destroy(lt_ctx* ctx);
const char* lt_last_error(const lt_ctx* ctx);
int lt_set_stream(lt_ctx* ctx, void* hip_stream);

/* Wait for the context's stream; report sticky device status bits
 * (LT_STATUS_*) and clear them.  Returns LT_EINVAL if LT_STATUS_PARAMS is
 * set (the parameter check of every trace call happens on the device, so a
 * rejected luminaire surfaces here), else LT_EOVERFLOW for LT_STATUS_OVERFLOW,
 * else LT_EHIP for LT_STATUS_TRAVERSAL. */
int lt_sync(lt_ctx* ctx, uint32_t* flags_out);

/* Scene upload and BVH build (supplies the acceleration structure the paper
 * takes from ray-tracing hardware, Sec. 6).  Host arrays: h_verts [n_verts,3]
 * f32, h_tris [n_tris,3] i32 vertex indices, h_tri_patch [n_tris] i32,
 * h_patches [n_patches].  Texel ranges of the patches must tile
 * [0, n_texels) in order; at most 2^26 triangles and a tree under 2^32 bytes
 * (the traversal addresses triangles and nodes by 32-bit byte offsets);
 * vertices finite and within 1e8 of the origin (so the slab test's
 * products with a reciprocal direction, up to 1e30 for an axis-parallel
 * ray, stay finite).  Builds the BVH on the device (Morton order, PLOC
 * clustering, collapse to a 4-wide tree) and the per-texel area table;
 * replaces any previous scene.  *n_texels_out receives K.  LT_EINVAL for
 * any violation. */
int lt_scene_upload(lt_ctx* ctx, const float* h_verts, int64_t n_verts, const int32_t* h_tris,
                    const int32_t* h_tri_patch, int64_t n_tris, const lt_patch* h_patches, int32_t n_patches,
                    int64_t* n_texels_out);

/* Luminaires (Sec. 4.4 and the supplement's light models): h_lights
 * [n_lights], h_layout_offsets [n_layouts+1] (lights of layout j are
 * [off[j], off[j+1]), every layout non-empty).  Parameters p are passed per
 * trace call. */
int lt_set_lights(lt_ctx* ctx, const lt_light_static* h_lights, int32_t n_lights,
                  const int32_t* h_layout_offsets, int32_t n_layouts);

/* Primal light tracing (Alg. 1, Eq. indirectFlux, Eq. directionalCoeffs with
 * n = 0): d_params [L,6] f32; d_S [n_layouts,K] i64 scratch (Q31.32 fixed-point
 * sums, zeroed by the call); d_E [n_layouts,K] f32 irradiance E_k = S_k 2^-32.
 * Every trace call checks the parameters on the device: a luminaire with a
 * NaN or infinite parameter or a power P <= 0 traces no path and raises
 * LT_STATUS_PARAMS, which lt_sync reports as LT_EINVAL. */
int lt_trace_forward(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int64_t* d_S, float* d_E);

/* Objective (Eq. objective, alpha_l = 1): O = 1/2 sum A_k alpha_k (E_k - E*_k)^2
 * over n = n_layouts*K texels; d_alpha may be NULL (all ones).  Writes d_O
 * (one f64) and d_g = dO/dE [n] f32. */
int lt_objective(lt_ctx* ctx, const float* d_E, const float* d_Etarget, const float* d_alpha, int64_t n,
                 double* d_O, float* d_g);

/* Adjoint light tracing (Alg. 2, Eq. adjointFlux, Eq. objGradAdjoint,
 * Eq. posDeriv and the rotation / area-light terms): replays the paths of
 * `cfg` (same seed = correlated evaluation) with d_dOdE [n_layouts,K] and
 * writes d_grad [L,6] f32 = dO/dp.  d_bin_hist [L,1024] f32 (may be NULL,
 * overwritten) receives per-light adjoint magnitudes binned by emission
 * direction (see lt_proposal_set_scale); rows of point lights and
 * soft-edged spots stay 0.  In the box basis, below 2^30 paths per layout
 * and while the records take at most an eighth of device memory it runs in
 * two passes: the trace leaves a 60-byte record per path (first hit,
 * origin, flux, adjoint sums, emission cell) in a context-owned device
 * buffer that grows to the largest path count seen (16 GB for 2^28 paths;
 * counted in lt_info's device_bytes), and a second kernel forms the
 * per-tile FP64 sums; otherwise in one pass.  lt_trace_adjoint_rgb runs
 * the same way. */
int lt_trace_adjoint(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE,
                     float* d_grad, float* d_bin_hist);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * adjoint pass of lt_trace_adjoint (same arguments without d_bin_hist, same
 * kernels and the same d_grad [L,6] f32 result, bit for bit) with every
 * buffer it needs beyond the inputs and outputs -- work-queue counters, the
 * work-tile table (built on the device), per-light ranges and path counts,
 * per-tile partial sums, the traversal-stack overflow area -- carved from
 * one fixed 64 MiB device array that the library holds per device until the
 * process ends.  Makes no allocation call.  LT_EINVAL when the work does not
 * fit that array (n_tiles * 64 B + L * 16 B plus the overflow area of at
 * least 64 waves; tiles of tile_paths paths), for LT_FLAG_GRAPH, and as
 * lt_trace_adjoint otherwise.  All calls on one device share the array,
 * which keeps the last call's contents (every region is rewritten before it
 * is read): calls that overlap in time on one device, from any context or
 * stream, race and must be serialised by the caller.  The context must have
 * a scene and luminaires (their set-up calls allocate, this one does not). */
int lt_trace_adjoint_noalloc(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE,
                             float* d_grad);

/* Gradient-contribution map (Sec. gradVis): the adjoint pass of
 * lt_trace_adjoint (same arguments, same d_grad [L,6] f32 output), which also
 * adds each path's contribution to dO/dp_j, j = `param` in 0..5 (x, y, z,
 * alpha, beta, P), of the global light `light` into the texel of the path's
 * first surface hit.  d_vote [K] f64 covers the texels of that light's layout,
 * is 16-byte aligned and is overwritten; it sums to d_grad[light][param] up
 * to rounding.  Summation order over paths is not fixed, so the map agrees
 * with a sequential sum to FP64 rounding only.  LT_EINVAL for a light or
 * parameter out of range. */
int lt_gradient_votes(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE,
                      int32_t light, int32_t param, double* d_vote, float* d_grad);

/* Direct-differentiation map, the comparison the paper sets beside the
 * contribution map (Sec. gradVis): d_D [K] f32 = dE_k/dp_j over the texels
 * of the layout of global light `light`, j = `param`, from that light's
 * paths with every first hit held fixed (each hit adds (Phi_h / A) times its
 * path's first-hit dlog_j to its own texel).  d_T [K] i64 scratch (Q31.32,
 * 16-byte aligned).  Unlike the contribution map it responds where light
 * arrives; sum_k dO/dE_k d_D[k] equals the adjoint's dO/dp_j of the light up
 * to rounding.  Plain emission, box basis, grey light, orientation as tilt
 * angles (j = 0..5 as in the parameter vector).  LT_EINVAL for proposal or
 * linear-basis flags, a light or parameter out of range, misaligned or NULL
 * buffers. */
int lt_trace_tangent(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int32_t light, int32_t param,
                     int64_t* d_T, float* d_D);

/* Central-difference map, the third image of the paper's gradient
 * comparison (Sec. gradVis): two primal passes with the same seed (common
 * random numbers) at p_j + h and p_j - h of global light `light` (FP32 sums),
 * d_F [K] f32 = (E_k(p+) - E_k(p-)) / ((p_j + h) - (p_j - h)) over the texels
 * of the light's layout, the step taken in FP64 from the two FP32 values and
 * the difference taken exactly on the int64 sums.  d_Sp, d_Sm [n_layouts,K]
 * i64 scratch (16-byte aligned), holding the two passes' sums afterwards.
 * Unlike the direct-differentiation map, hits move with p, so texels where a
 * shadow or patch edge sweeps respond too.  Plain emission, box basis, grey,
 * tilt angles; LT_EINVAL for h <= 0 or not finite, a light or parameter out
 * of range, proposal or linear-basis flags. */
int lt_fd_map(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int32_t light, int32_t param, float h,
              int64_t* d_Sp, int64_t* d_Sm, float* d_F);

/* Adjoint with the soft-edged spots' cone angles (supplement, spot light:
 * the derivatives of the fall-off w.r.t. the cone angles, with x_1 fixed).
 * d_grad [L,6] f32 as lt_trace_adjoint (the same sums); d_grad_cone [L,2] f32
 * = dO/d(theta_in, theta_out) in radians at constant total power P, 0 for
 * other luminaire types.  The angles themselves are the size_w / size_h of
 * lt_set_lights.  Plain emission, box basis, grey, tilt angles. */
int lt_trace_adjoint_cone(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE,
                          float* d_grad, float* d_grad_cone);

/* Colour (Sec. 4.4.3, intensity and colour).  A luminaire's flux is split
 * over three channels by weights d_colour [L,3] f32 (channel ch carries
 * P c_ch; the optimiser may keep r + g + b = 1, the chromaticity
 * projection); every patch reflects channel ch with its own albedo
 * (lt_set_albedo_rgb, h_albedo [n_patches,3] in [0,1], host pointer; after
 * lt_scene_upload each channel takes the patch's scalar albedo).  All
 * channels share one path geometry.  Texel arrays are channel-planar:
 * d_S, d_E, d_dOdE [n_layouts,3,K] (lt_objective takes n = n_layouts*3*K).
 * The adjoint returns d_grad [L,6] for the geometry and power, taking the
 * colour-weighted adjoint sum, and d_grad_colour [L,3] = dO/dc.  Box basis
 * only (LT_FLAG_LINEAR is refused); the contribution map, path records and
 * the path tracer are grey only. */
int lt_set_albedo_rgb(lt_ctx* ctx, const float* h_albedo);
int lt_trace_forward_rgb(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, const float* d_colour,
                         int64_t* d_S, float* d_E);
int lt_trace_adjoint_rgb(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, const float* d_colour,
                         const float* d_dOdE, float* d_grad, float* d_grad_colour, float* d_bin_hist);

/* Directional texels (Eq. directionalCoeffs with n = 1 to 3; Sec. 4.1) with a
 * glossy BRDF.  Each texel holds NC = (order+1)^2 coefficients of its
 * reflected radiance in 2pi-normalised hemispherical harmonics (the
 * integral of H^2 over the hemisphere is 2 pi, H_0^0 = 1; associated
 * Legendre functions of 2 cos(theta) - 1, index l^2 + l + m, cos m phi for
 * m > 0, sin |m| phi for m < 0), in the local frame of the side the light
 * arrives on (normal = z, tangents of the bounce's orthonormal basis, Duff et
 * al. 2017).  Each hit projects (Phi / A) f(w_in, w) with `samples` uniform
 * local directions.  BRDF per patch: Lambertian albedo (lt_patch.albedo)
 * plus a normalised Phong lobe rho_s (e+2)/(2 pi) cos^e about the mirror
 * direction (lt_set_glossy, h_glossy [n_patches,2] = (rho_s, e), host
 * pointer; Lambertian after lt_scene_upload).  Bounces stay cosine-sampled,
 * the throughput taking pi f.  Texel arrays d_S, d_E, d_dOdE
 * [n_layouts,NC,K]; lt_objective takes n = n_layouts*NC*K.  The adjoint
 * adds the first hit's BRDF terms: its projection and its bounce weight
 * depend on the incident direction, which moves with the luminaire while
 * x_1 stays fixed (Eq. dLdp).  order 0..3, samples 1..64, box basis, grey. */
int lt_set_glossy(lt_ctx* ctx, const float* h_glossy);

/* Orientation as a rotation vector (Sec. 4.4.2): d_params [L,7] = (x, y, z,
 * theta_x, theta_y, theta_z, P); the luminaire frame is R(theta) applied to
 * the default frame (axis -z, tangents +x, +y), R by Rodrigues' formula
 * (the linear small-angle form I + [theta]x below |theta| = 1e-6).  The
 * adjoint differentiates each path's first-hit kernel w.r.t. a world
 * rotation of the luminaire about its centre and maps the per-luminaire sum
 * to theta with the transposed Jacobian of the exponential map; d_grad
 * [L,7].  A rectangle's roll about its normal is a free direction here,
 * which the two tilt angles cannot express.  Plain emission and the box
 * basis only (LT_FLAG_PROPOSAL and LT_FLAG_LINEAR are refused); grey. */
int lt_trace_forward_rv(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int64_t* d_S, float* d_E);
int lt_trace_adjoint_rv(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE,
                        float* d_grad);
int lt_trace_forward_dir(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int32_t order, int32_t samples,
                         int64_t* d_S, float* d_E);
int lt_trace_adjoint_dir(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int32_t order, int32_t samples,
                         const float* d_dOdE, float* d_grad, float* d_bin_hist);

/* Object-space path tracing with next-event estimation: the comparison
 * estimator of Sec. 6 (after Stam 2020) on the same texels.  Each texel gets
 * samples_per_texel points drawn uniformly in it; every path vertex (the
 * point, then up to cfg->max_hits - 1 cosine bounces, the first on a side
 * drawn with probability 1/2) connects to one luminaire of its layout chosen
 * uniformly, through a shadow ray.  E_k is the mean over the texel's samples
 * of the irradiance estimates (both sides of the surface, like the light
 * tracer's splat).  cfg: seed and max_hits as for light tracing
 * (paths_per_layout is only checked against the luminaire counts); flags
 * must be 0.  At most 256 luminaires per layout and fewer than 2^32 samples
 * per layout (K samples_per_texel).  d_S [n_layouts,K] i64 scratch, d_E
 * [n_layouts,K] f32 out, as for lt_trace_forward. */
int lt_pt_forward(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int32_t samples_per_texel,
                  int64_t* d_S, float* d_E);

/* Gradient of sum_k dOdE_k E_k for the path tracer above with the same
 * samples (same seed): every luminaire connection differentiated with its
 * vertex held fixed (the first-hit derivative factors at that vertex; no
 * visibility terms).  d_dOdE [n_layouts,K] f32; d_grad [L,6] f32 out. */
int lt_pt_adjoint(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int32_t samples_per_texel,
                  const float* d_dOdE, float* d_grad);

/* Hit sequences of paths [first, first+count) of light `light` (index within
 * its layout `layout`): d_prim / d_texel [count, max_hits] i32, -1 where the
 * path ended.  With d_dOdE, d_contrib [count,6] f32 receives each path's
 * gradient contribution (may both be NULL). */
int lt_record_paths(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int32_t layout, int32_t light,
                    int64_t first, int64_t count, int32_t* d_prim, int32_t* d_texel, const float* d_dOdE,
                    float* d_contrib);

/* Work counters of one forward pass (instrumented kernel): segments traced,
 * BVH nodes visited (four box tests each), triangle tests, hits, misses,
 * traversal-loop wave iterations, active lanes summed over those iterations,
 * hit-processing phases. */
int lt_trace_stats(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int64_t* d_S,
                   int64_t h_counts_out[8]);

/* Learned emission proposal (an extension beyond the paper, which leaves
 * importance sampling to future work, Sec. 7).  Per light, a distribution
 * pi_b over the 32 x 32 cells of the hemi-octahedral map of the emission
 * hemisphere (cell (i, j) covers u in [-1 + i/16, -1 + (i+1)/16], v likewise,
 * direction p = ((u+v)/2, (u-v)/2, 1-|.|-|.|)/|p| in the light frame (t, b, d),
 * solid-angle density pi_b * 512 * |p|^3).  With LT_FLAG_PROPOSAL a spot or
 * rectangle emits from the plain cos^n lobe with probability alpha_plain and
 * from the cells otherwise, with Phi_r = (P/N) p_plain / q, q = alpha p_plain
 * + (1 - alpha) p_learn (one-sample MIS, unbiased for alpha > 0).  Point
 * lights always use the plain sampler.  d_pdf, d_cdf [L,1024] f32 (cdf =
 * inclusive prefix sums of pdf, non-decreasing, last entry 1) are copied into
 * the context, which also derives its inverse-CDF guide entries from d_cdf.
 * A learned sample takes the first cell b with u < cdf[b] (the last cell when
 * none); a table that is not non-decreasing gives unspecified (in-range)
 * cells. */
int lt_proposal_set_table(lt_ctx* ctx, const float* d_pdf, const float* d_cdf);
/* Copy the context's current proposal tables out (d_pdf, d_cdf [L,1024]). */
int lt_proposal_get_table(lt_ctx* ctx, float* d_pdf, float* d_cdf);

/* Per-light scale of the adjoint histogram signal: the adjoint pass adds
 * |c_r * inv_sigma|_2^2 * q / (512 |p|^3) of every path's gradient
 * contribution c_r into d_bin_hist[light][cell of its emission direction],
 * with q the solid-angle density the direction was drawn from (the mixture
 * with a proposal, the plain lobe otherwise) and p its point on the
 * octahedron.  Per cell b this estimates A_b / N independently of the
 * sampler, where A_b integrates the second moment of the scaled integrand
 * over the cell against d(omega) / (512 |p|^3); a sampler drawing cell b with
 * probability pi_b (uniform in (u, v) within it) has variance sum_b A_b / pi_b,
 * least for pi_b proportional to sqrt(A_b).  d_inv_sigma [L,6] f32. */
int lt_proposal_set_scale(lt_ctx* ctx, const float* d_inv_sigma);

/* The proposal network: per light x [32] = 6 normalised parameters, a 16-d
 * learned embedding, 10 zeros -> 64 ReLU -> 64 ReLU -> 1024 cell logits ->
 * softmax.  Weights (LT_MLP_WEIGHTS values): W1 [64][32], b1 [64], W2 [64][64],
 * b2 [64], W3 [1024][64], b3 [1024], row-major, output-major.
 * lt_proposal_mlp_infer: BF16 weights d_w_bf16 and inputs (rounded to BF16)
 * on MFMA with FP32 accumulate; writes the context's proposal tables (as
 * lt_proposal_set_table) and, if d_logits [L,1024] is not NULL, the logits.
 * d_x is [L,32] f32. */
#define LT_MLP_WEIGHTS 72832
#define LT_MLP_IN 32
int lt_proposal_mlp_infer(lt_ctx* ctx, const uint16_t* d_w_bf16, const float* d_x, float* d_logits);

/* One training step: cross-entropy between softmax(MLP(x)) and the target
 * cell distribution d_target [L,1024] (rows sum to 1), averaged over lights;
 * backward through the network and into the embedding columns 6..21 of d_x;
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias correction with `step` >= 1,
 * learning rate lr) on the FP32 master weights d_w with moments d_mw, d_vw
 * and on the embeddings with d_mx, d_vx; refreshes d_w_bf16.  d_loss (one
 * f32) and d_grad_out [LT_MLP_WEIGHTS + L*32] may be NULL. */
int lt_proposal_mlp_train(lt_ctx* ctx, float* d_w, float* d_mw, float* d_vw, uint16_t* d_w_bf16, float* d_x,
                          float* d_mx, float* d_vx, const float* d_target, int32_t step, float lr, float* d_loss,
                          float* d_grad_out);

/* The proposal network held by the context, so that a training step takes
 * only the adjoint histogram.  lt_proposal_set copies the FP32 master
 * weights d_w [LT_MLP_WEIGHTS] (layout as above) and the per-light
 * embeddings d_embed [L,16] into the context, zeroes the Adam moments,
 * derives the BF16 copy and computes the plain cos^n lobe's probability of
 * every cell (midpoint rule, 8 x 8 points per cell, FP64) for the training
 * target's floor; it replaces any earlier network and is dropped by
 * lt_set_lights.  cfg: the box that maps each parameter to the network input
 * 2 (p - lo)/(hi - lo) - 1 (finite, lo < hi), the running-average weights of
 * the histogram and of the squared gradients (in [0, 1)), and the plain
 * lobe's share of the target (in [0, 1]). */
typedef struct {
    float param_lo[6], param_hi[6];
    float hist_decay;   /* weight of the old average of the normalised histogram */
    float plain_floor;  /* share of the plain lobe's cell masses in the target */
    float sigma_decay;  /* weight of the old mean squared gradient component */
    int32_t reserved;
} lt_proposal_cfg;
int lt_proposal_set(lt_ctx* ctx, const float* d_w, const float* d_embed, const lt_proposal_cfg* cfg);
/* Network inputs from the luminaire parameters d_params [L,6] (the box of
 * lt_proposal_set), then inference into the sampling tables as
 * lt_proposal_mlp_infer. */
int lt_proposal_refresh(lt_ctx* ctx, const float* d_params);
/* Histogram units from one adjoint gradient d_grad [L,6]: the running mean
 * s of each squared component (the first call starts it), then the scale
 * 1/sqrt(s + 1e-30) times h_mask[c] (host [6], NULL = all ones; a component
 * with mask 0 does not enter the histogram), as lt_proposal_set_scale. */
int lt_proposal_update_scale(lt_ctx* ctx, const float* d_grad, const float* h_mask);
/* One training round from the adjoint histogram d_bin_hist [L,1024]
 * (lt_trace_adjoint): each light's row is normalised (an empty row counts as
 * uniform) and folded into the running average (the first call starts it);
 * the target is the normalised square root of that average (the
 * variance-optimal cell probabilities, see lt_proposal_set_scale), mixed with
 * the plain lobe's cell masses by plain_floor; then `steps` (0..1000) Adam
 * steps of lt_proposal_mlp_train toward it with learning rate lr on the
 * context's network (step count continuing across calls).  d_loss (one f32,
 * the last step's loss) and d_target_out [L,1024] f32 may be NULL.
 * Call lt_proposal_refresh afterwards to sample from the trained network. */
int lt_proposal_train_step(lt_ctx* ctx, const float* d_bin_hist, float lr, int32_t steps, float* d_loss,
                           float* d_target_out);
/* Copy the context's FP32 master weights d_w [LT_MLP_WEIGHTS] and network
 * inputs d_x [L,32] (normalised parameters, embeddings, zero padding) out;
 * either may be NULL. */
int lt_proposal_get_net(lt_ctx* ctx, float* d_w, float* d_x);

int lt_get_tuning(const lt_ctx* ctx, lt_tuning* out);
int lt_set_tuning(lt_ctx* ctx, const lt_tuning* t);

/* Time candidate launch shapes for forward+adjoint on this configuration and
 * keep the fastest; d_* are scratch buffers of the trace calls.  If
 * cache_path is not NULL the choice is appended there and reused when a
 * matching entry exists. */
int lt_autotune(lt_ctx* ctx, const lt_trace_cfg* cfg, const float* d_params, int64_t* d_S, float* d_E,
                const float* d_dOdE, float* d_grad, const char* cache_path, float* h_best_ms);

int lt_info_get(const lt_ctx* ctx, lt_info* out);

/* Copy the uploaded scene's acceleration structure to host memory, for
 * inspection (the structure the paper takes from ray-tracing hardware,
 * Sec. 6).  h_nodes receives the wide nodes (lt_info.bvh_nodes x 64 B: per
 * axis x, y, z the four slots' lower then upper planes as f16 offsets from
 * the node origin, rounded outward; then the origin as bf16 x, y, z, the
 * slot counts internal | leaves << 4, the first internal child's node index
 * and the first leaf's triangle slot; slots ordered internal, leaves,
 * unused), h_tris the leaf triangles (lt_info.n_tris x 48 B, 2 x 48 B for a
 * single-triangle scene: (v0, id), (v1 - v0, patch), (v2 - v0, 0) as f32 /
 * int bits, in leaf-slot order).  Byte sizes of the host buffers are passed
 * in; LT_EINVAL if there is no scene or a buffer is too small. */
int lt_bvh_copy(lt_ctx* ctx, void* h_nodes, int64_t nodes_bytes, void* h_tris, int64_t tris_bytes);

/* Kernel timing.  While enabled, HIP events are recorded on the launch stream
 * around every persistent trace kernel launched outside a graph;
 * lt_timing_read waits for them and returns the summed kernel durations (ms)
 * and launch counts of the forward and adjoint kernels since the last read. */
int lt_set_timing(lt_ctx* ctx, int enable);
int lt_timing_read(lt_ctx* ctx, double* fwd_ms, int32_t* n_fwd, double* adj_ms, int32_t* n_adj);

#ifdef __cplusplus
}
#endif
#endif /* LT_H */
