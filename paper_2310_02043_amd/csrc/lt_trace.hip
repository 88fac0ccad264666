// Primal and adjoint light-tracing kernels for gfx950.
//
// Alg. 1 (primal) and Alg. 2 (adjoint) of the paper, one launch over a grid
// of work tiles covering every layout.  A tile is a contiguous path range of
// one luminaire of one layout; its wave keeps 64 paths in flight and refills
// lanes whose path ended (ballot + mbcnt prefix count) until the tile is
// exhausted.  Hit processing (splat or adjoint gather, bounce, refill) runs
// once at least `refill_threshold` lanes have finished their current segment,
// so the BVH traversal loop stays converged.  Texel sums are int64 Q31.32
// fixed point (order-independent); adjoint contributions are summed per lane
// in path order (FP32) and per tile over the lanes in a fixed order (FP64), so
// both passes are deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lt_device.h"
#include "lt_internal.h"

namespace lt {

namespace {

struct Ray {
    float ox, oy, oz, dx, dy, dz;
    float ix, iy, iz, oix, oiy, oiz;   // safe reciprocal direction and origin * reciprocal
};

__device__ __forceinline__ void set_ray(Ray& r, V3 o, V3 d)
{
    r.ox = o.x; r.oy = o.y; r.oz = o.z;
    r.dx = d.x; r.dy = d.y; r.dz = d.z;
    // the slab test is conservative by the build's padding, so the hardware
    // reciprocal (1 ulp) serves; exact zeros are replaced so no 0 * inf appears
    const float tiny = 1e-30f;
    r.ix = __builtin_amdgcn_rcpf(d.x != 0.0f ? d.x : __builtin_copysignf(tiny, d.x));
    r.iy = __builtin_amdgcn_rcpf(d.y != 0.0f ? d.y : __builtin_copysignf(tiny, d.y));
    r.iz = __builtin_amdgcn_rcpf(d.z != 0.0f ? d.z : __builtin_copysignf(tiny, d.z));
    r.oix = o.x * r.ix;
    r.oiy = o.y * r.iy;
    r.oiz = o.z * r.iz;
}

// f16 halves of a packed word, widened exactly (the fma then takes the f16
// operand directly, v_fma_mix_f32)
__device__ __forceinline__ float f16lo(unsigned w) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xFFFFu)); }
__device__ __forceinline__ float f16hi(unsigned w) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16)); }

// Lane's entry i of its wave's traversal-stack overflow area (entries
// interleaved by lane): a 32-bit byte offset from the wave-uniform base,
// so the access takes the scalar-base form and the base costs no VGPRs.
__device__ __forceinline__ int* gst_slot(int* gst, int i)
{
    return (int*)((char*)gst + (((unsigned)i * 64u + (unsigned)__lane_id()) << 2));
}

struct Trav {
    float tb;
    int pb, qb;
    int node, sp;   // node < 0: nothing left to visit
    int steps;
    int lmask;      // slots of the last node step whose leaf triangle awaits its test
    int lrow;       // that node's first leaf-triangle row, less 3 x its internal-child count
};

// One traversal operation per lane and call: either up to two queued leaf
// triangle tests, or one node of the 4-wide tree (four box tests; hit leaf
// slots are queued as a bit mask, hit internal children sorted by entry
// distance, the nearest visited next and the others pushed far-to-near).
// Queued leaves are tested before the next node step, so the closest-hit
// bound tightens as early as before.
// mode 1 runs only a queued triangle test, mode 2 only a node step, mode 0
// whichever the lane has next.
template <int LDS_D, bool STATS>
__device__ __forceinline__ void trav_step(const Ray& r, int skip, Trav& s, bool& traversing,
                                          const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                          int* lst, int* gst, unsigned& n_nodes, unsigned& n_tris,
                                          int max_steps, bool& overrun, int mode = 0)
{
    if (mode == 1 && s.lmask == 0) return;
    if (mode == 2 && s.lmask != 0) return;
    if (s.lmask != 0) {
#pragma unroll
        for (int rep = 0; rep < 2; ++rep) {
            if (s.lmask == 0) break;
            // leaf slot k holds the triangle at row lrow + 3 k (48 B each)
            const int k = __builtin_ctz((unsigned)s.lmask);
            const float4* tp = (const float4*)((const char*)tris + ((unsigned)(s.lrow + 3 * k) << 4));
            tri_test(tp[0], tp[1], tp[2], v3(r.ox, r.oy, r.oz), v3(r.dx, r.dy, r.dz), skip, s.tb, s.pb, s.qb);
            if (STATS) ++n_tris;
            s.lmask &= s.lmask - 1;
        }
        if (s.lmask == 0 && s.node < 0) traversing = false;
        return;
    }
    // bounded: a segment visits each node at most once in a tree
    if (++s.steps > max_steps) {
        traversing = false;
        overrun = true;
        s.pb = -1;
        s.qb = -1;
        return;
    }
    // 32-bit byte offsets from the uniform node base (64 B per node; the
    // upload keeps the tree under 2^32 bytes), so the four loads share one
    // address with immediate offsets
    const char* nd = (const char*)nodes + ((unsigned)s.node << 6);
    const uint4 px = *(const uint4*)nd;
    const uint4 py = *(const uint4*)(nd + 16);
    const uint4 pz = *(const uint4*)(nd + 32);
    const uint4 hd = *(const uint4*)(nd + 48);
    if (STATS) ++n_nodes;
    // near and far planes per axis: the lower planes for a positive
    // direction component, the upper ones otherwise (two slots per word)
    const bool sx = __float_as_int(r.ix) < 0, sy = __float_as_int(r.iy) < 0, sz = __float_as_int(r.iz) < 0;
    const unsigned xn0 = sx ? px.z : px.x, xn1 = sx ? px.w : px.y, xf0 = sx ? px.x : px.z, xf1 = sx ? px.y : px.w;
    const unsigned yn0 = sy ? py.z : py.x, yn1 = sy ? py.w : py.y, yf0 = sy ? py.x : py.z, yf1 = sy ? py.y : py.w;
    const unsigned zn0 = sz ? pz.z : pz.x, zn1 = sz ? pz.w : pz.y, zf0 = sz ? pz.x : pz.z, zf1 = sz ? pz.y : pz.w;
    const float xn[4] = {f16lo(xn0), f16hi(xn0), f16lo(xn1), f16hi(xn1)}, xf[4] = {f16lo(xf0), f16hi(xf0), f16lo(xf1), f16hi(xf1)};
    const float yn[4] = {f16lo(yn0), f16hi(yn0), f16lo(yn1), f16hi(yn1)}, yf[4] = {f16lo(yf0), f16hi(yf0), f16lo(yf1), f16hi(yf1)};
    const float zn[4] = {f16lo(zn0), f16hi(zn0), f16lo(zn1), f16hi(zn1)}, zf[4] = {f16lo(zf0), f16hi(zf0), f16lo(zf1), f16hi(zf1)};
    // a plane at origin + h lies at distance h * ix + b, b = origin * ix - o * ix
    const float bx = __builtin_fmaf(__uint_as_float(hd.x << 16), r.ix, -r.oix);
    const float by = __builtin_fmaf(__uint_as_float(hd.x & 0xFFFF0000u), r.iy, -r.oiy);
    const float bz = __builtin_fmaf(__uint_as_float(hd.y << 16), r.iz, -r.oiz);
    const int ni = (int)((hd.y >> 16) & 15u);   // internal children, in the first slots
    const float tb = s.tb;
    // per slot: the entry distance as an unsigned key (non-negative floats
    // order as their bit patterns) with the slot in bits 8-9, all ones unless
    // the slot is an internal child whose box the ray enters; hit leaf slots
    // are queued by mask.  The build pads every box by a scene-relative
    // margin far above the rounding of this form, so the test is conservative.
    unsigned key[4];
    int lm = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float t0 = fmaxf(fmaxf(__builtin_fmaf(xn[k], r.ix, bx), __builtin_fmaf(yn[k], r.iy, by)),
                               fmaxf(__builtin_fmaf(zn[k], r.iz, bz), 0.0f));
        const float t1 = fminf(fminf(__builtin_fmaf(xf[k], r.ix, bx), __builtin_fmaf(yf[k], r.iy, by)),
                               fminf(__builtin_fmaf(zf[k], r.iz, bz), tb));
        const bool hit = t0 <= t1;   // unused slots hold inverted boxes
        const bool leaf = k >= ni;
        lm |= (hit && leaf) ? (1 << k) : 0;
        key[k] = (hit && !leaf) ? ((__float_as_uint(t0) & ~0x300u) | ((unsigned)k << 8)) : 0xFFFFFFFFu;
    }
    s.lmask = lm;
    s.lrow = 3 * ((int)hd.w - ni);
    // ascending sort of the four keys (five compare-exchanges)
    const unsigned a0 = min(key[0], key[1]), a1 = max(key[0], key[1]);
    const unsigned a2 = min(key[2], key[3]), a3 = max(key[2], key[3]);
    const unsigned e0 = min(a0, a2), p2 = max(a0, a2);
    const unsigned p1 = min(a1, a3), e3 = max(a1, a3);
    const unsigned e1 = min(p1, p2), e2 = max(p1, p2);
    const unsigned none = 0xFFFFFFFFu;
    const int first = (int)hd.z;   // internal child in slot k: node first + k
    if (e0 == none) {
        if (s.sp == 0) {
            s.node = -1;
        } else {
            --s.sp;
            // the LDS and the overflow read stay two accesses: merged, they
            // would become one generic (flat) access through the vector-memory
            // path (the empty asm statement keeps the branches distinct)
            if (s.sp < LDS_D) {
                s.node = lst[s.sp * 64];
                __asm__ volatile("");
            } else {
                s.node = *gst_slot(gst, s.sp - LDS_D);
            }
        }
    } else {
        s.node = first + (int)((e0 >> 8) & 3u);
        // the others far-to-near
        const unsigned ek[3] = {e3, e2, e1};
        if (s.sp + 3 <= LDS_D) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (ek[k] != none) {
                    lst[s.sp * 64] = first + (int)((ek[k] >> 8) & 3u);
                    ++s.sp;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (ek[k] != none) {
                    const int cv = first + (int)((ek[k] >> 8) & 3u);
                    if (s.sp < LDS_D) {
                        lst[s.sp * 64] = cv;
                        __asm__ volatile("");   // two stores, not one flat store
                    } else {
                        *gst_slot(gst, s.sp - LDS_D) = cv;
                    }
                    ++s.sp;
                }
            }
        }
    }
    if (s.node < 0 && s.lmask == 0) traversing = false;
}

__device__ __forceinline__ void start_segment(Trav& s)
{
    s.tb = __builtin_inff();
    s.pb = -1;
    s.qb = -1;
    s.node = 0;
    s.sp = 0;
    s.steps = 0;
    s.lmask = 0;
    s.lrow = 0;
}

// Emission (Alg. 1 "generate exitant ray"): origin y, direction, area
// offsets, flux phi and the emission direction's cell of the hemi-octahedral
// map (ebin, -1 for point lights).  With a proposal, the direction comes from
// the plain cos^n lobe with probability alpha and otherwise from the binned
// proposal (cell by inverse CDF, uniform jitter in the cell), and
// phi = (P/N) p_plain / (alpha p_plain + (1 - alpha) p_learn).  wq is the
// sample's density over the (u, v) measure of its cell, q / (512 |p|^3) with q
// the density it was drawn from: the adjoint histogram adds |c_r / sigma|^2 wq,
// whose expectation per cell does not depend on the sampler and is
// proportional to the square of the variance-optimal cell probability.
// r: the path's generator output at counter (pid, stream, 0, 0).
__device__ __forceinline__ void emit_from(const DevLight& L, const U4 r, uint32_t pid, uint32_t stream_id, uint32_t k0,
                                          uint32_t k1, const float* __restrict__ pdf, const float* __restrict__ cdf,
                                          const int* __restrict__ guide, float alpha, bool want_bin, V3& y, V3& dir,
                                          float& au, float& av, float& phi, int& ebin, float& wq)
{
    const float u0 = u24(r.x), u1 = u24(r.y), u2 = u24(r.z), u3 = u24(r.w);
    y = v3(L.c[0], L.c[1], L.c[2]);
    au = 0.0f;
    av = 0.0f;
    phi = L.phi_r;
    ebin = -1;
    wq = 0.0f;
    if (L.type == 0) {
        float sp, cp;
        sincos_2pi(u3, sp, cp);
        const float z = 1.0f - 2.0f * u2;
        const float rr = __builtin_sqrtf(fmaxf(0.0f, 1.0f - z * z));
        dir = v3(rr * cp, rr * sp, z);
        return;
    }
    if (L.type == 3) {
        // soft-edged spot: uniform over the outer cone's cap (L.h = its
        // cosine), the flux weighted by the fall-off towards it (L.w = the
        // inner cone's cosine)
        float sp, cp;
        sincos_2pi(u3, sp, cp);
        const float ct = 1.0f - u2 * (1.0f - L.h);
        const float st = __builtin_sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
        const float a = st * cp, bb = st * sp;
        if (ct < L.w) {
            const float f = (ct - L.h) / (L.w - L.h);
            phi = phi * (f * f);
        }
        dir = v3((a * L.t[0] + bb * L.b[0]) + ct * L.d[0], (a * L.t[1] + bb * L.b[1]) + ct * L.d[1],
                 (a * L.t[2] + bb * L.b[2]) + ct * L.d[2]);
        return;
    }
    // Component choice first: a sample from the learned cells never needs
    // the plain lobe's direction, only its density.
    bool plain = true;
    float w1 = 0.0f, w2 = 0.0f, w3 = 0.0f;
    if (pdf != nullptr) {
        const U4 r1 = philox10(pid, stream_id, 1u, 0u, k0, k1);
        plain = u24(r1.x) < alpha;
        w1 = u24(r1.y);
        w2 = u24(r1.z);
        w3 = u24(r1.w);
    }
    float ct, a, bb, pl3 = 0.0f;
    if (plain) {
        float sp, cp;
        sincos_2pi(u3, sp, cp);
        ct = u2 > 0.0f ? exp2_c(log2_c(u2) / (L.n + 1.0f)) : 0.0f;
        const float st = __builtin_sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
        a = st * cp;
        bb = st * sp;
        if (pdf != nullptr || want_bin) {
            const float s = (fabsf(a) + fabsf(bb)) + ct;
            const float xp = a / s, yp = bb / s;
            int iu = (int)__builtin_floorf(((xp + yp) + 1.0f) * 16.0f);
            int iv = (int)__builtin_floorf(((xp - yp) + 1.0f) * 16.0f);
            iu = iu < 0 ? 0 : (iu > 31 ? 31 : iu);
            iv = iv < 0 ? 0 : (iv > 31 ? 31 : iv);
            ebin = iv * 32 + iu;
            pl3 = 1.0f / ((s * s) * s);
        }
    } else {
        // Inverse CDF: the first cell whose inclusive prefix sum exceeds w1.
        // The guide entries bracket it (guide[j] = first cell whose sum
        // exceeds j/1024), so the search covers a few cells, not 1024.
        const int j = (int)(w1 * 1024.0f);
        int lo = guide[j], hi = guide[j + 1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (w1 < cdf[mid]) hi = mid;
            else lo = mid + 1;
        }
        ebin = lo;
        const float uu = -1.0f + ((float)(lo & 31) + w2) * 0.0625f;
        const float vv = -1.0f + ((float)(lo >> 5) + w3) * 0.0625f;
        const float xp = (uu + vv) * 0.5f, yp = (uu - vv) * 0.5f;
        const float zp = (1.0f - fabsf(xp)) - fabsf(yp);
        const float nrm = __builtin_sqrtf((xp * xp + yp * yp) + zp * zp);
        const float inv = 1.0f / nrm;
        a = xp * inv;
        bb = yp * inv;
        ct = zp * inv;
        pl3 = (nrm * nrm) * nrm;
    }
    if (pdf != nullptr || want_bin) {
        float pw = 1.0f;
        if (L.n != 0.0f) pw = ct > 0.0f ? exp2_c(L.n * log2_c(ct)) : 0.0f;
        const float p_plain = ((L.n + 1.0f) * (float)0.15915494309189533577) * pw;
        float q = p_plain;
        if (pdf != nullptr) {
            const float p_learn = (pdf[ebin] * 512.0f) * pl3;
            q = alpha * p_plain + (1.0f - alpha) * p_learn;
            phi = q > 0.0f ? phi * (p_plain / q) : 0.0f;
        }
        // histogram weight: the sample's density over the cell's (u, v)
        // measure, q / (512 |p|^3)
        wq = q / (512.0f * pl3);
    }
    dir = v3((a * L.t[0] + bb * L.b[0]) + ct * L.d[0], (a * L.t[1] + bb * L.b[1]) + ct * L.d[1],
             (a * L.t[2] + bb * L.b[2]) + ct * L.d[2]);
    if (L.type == 2) {
        au = (u0 - 0.5f) * L.w;
        av = (u1 - 0.5f) * L.h;
        y = v3((L.c[0] + au * L.t[0]) + av * L.b[0], (L.c[1] + au * L.t[1]) + av * L.b[1],
               (L.c[2] + au * L.t[2]) + av * L.b[2]);
    }
}

__device__ __forceinline__ void emit(const DevLight& L, uint32_t pid, uint32_t stream_id, uint32_t k0, uint32_t k1,
                                     const float* __restrict__ pdf, const float* __restrict__ cdf,
                                     const int* __restrict__ guide, float alpha, bool want_bin, V3& y, V3& dir,
                                     float& au, float& av, float& phi, int& ebin, float& wq)
{
    emit_from(L, philox10(pid, stream_id, 0u, 0u, k0, k1), pid, stream_id, k0, k1, pdf, cdf, guide, alpha, want_bin, y,
              dir, au, av, phi, ebin, wq);
}

// Cosine-weighted bounce about the oriented normal (Malley's method in the
// orthonormal basis of Duff et al. 2017); the flux update is Phi * rho.
__device__ __forceinline__ V3 cosine_dir(V3 no, float u0, float u1)
{
    const float sg = __builtin_copysignf(1.0f, no.z);
    const float a = -1.0f / (sg + no.z);
    const float bxy = (no.x * no.y) * a;
    const V3 b1 = v3(1.0f + ((sg * no.x) * no.x) * a, sg * bxy, -(sg * no.x));
    const V3 b2 = v3(bxy, sg + (no.y * no.y) * a, -no.y);
    const float rr = __builtin_sqrtf(u0);
    float sp, cp;
    sincos_2pi(u1, sp, cp);
    const float lx = rr * cp, ly = rr * sp;
    const float lz = __builtin_sqrtf(fmaxf(0.0f, 1.0f - u0));
    return v3((lx * b1.x + ly * b2.x) + lz * no.x, (lx * b1.y + ly * b2.y) + lz * no.y,
              (lx * b1.z + ly * b2.z) + lz * no.z);
}

__device__ __forceinline__ V3 bounce_dir(V3 no, uint32_t pid, uint32_t stream_id, uint32_t h, uint32_t k0,
                                         uint32_t k1)
{
    const U4 r = philox10(pid, stream_id, 1u + h, 0u, k0, k1);
    return cosine_dir(no, u24(r.x), u24(r.y));
}

// dlog of the first-hit irradiance kernel w.r.t. (c, alpha, beta, P) with x_1
// fixed (Sec. 4.3 constant sample; Eq. posDeriv generalised to a cos^n lobe,
// plus the rotation terms and the area-light origin shift of the supplement).
// RV: orientation as a rotation vector, dl[7] = (position, derivative w.r.t.
// a world rotation of the luminaire about its centre, power).
template <bool RV = false>
__device__ __forceinline__ void first_hit_dlog(const DevLight& L, V3 x1, V3 y, V3 n1, float au, float av,
                                               float* dl)
{
    constexpr int NPAR = RV ? 7 : 6;
    for (int c = 0; c < NPAR - 1; ++c) dl[c] = 0.0f;
    dl[NPAR - 1] = 1.0f / L.P;
    const V3 v = sub(x1, y);
    const float r2 = dot(v, v);
    if (r2 <= 1e-12f) return;
    const float r = __builtin_sqrtf(r2);
    const float inv_r = 1.0f / r;
    const V3 w = v3(v.x * inv_r, v.y * inv_r, v.z * inv_r);
    const float c1 = -dot(n1, w);
    if (c1 <= 1e-6f) return;
    const float k1 = 1.0f / (r * c1);
    const float k3 = 2.0f * inv_r;
    if (L.type == 0) {
        dl[0] = (n1.x + c1 * w.x) * k1 + w.x * k3;
        dl[1] = (n1.y + c1 * w.y) * k1 + w.y * k3;
        dl[2] = (n1.z + c1 * w.z) * k1 + w.z * k3;
        return;
    }
    const V3 d = v3(L.d[0], L.d[1], L.d[2]);
    const float ce = dot(d, w);
    if (ce <= 1e-6f) return;
    // derivative of log I along cos(theta), over r and not: n / cos for the
    // cos^n lobe; 2 / (cos - cos_out) in the soft-edged spot's fall-off ring
    float ka, kd;
    if (L.type == 3) {
        const float lg = (ce > L.h && ce < L.w) ? 2.0f / (ce - L.h) : 0.0f;
        ka = lg / r;
        kd = lg;
    } else {
        ka = L.n / (r * ce);
        kd = L.n / ce;
    }
    const V3 G = v3((-((d.x - ce * w.x) * ka) + (n1.x + c1 * w.x) * k1) + w.x * k3,
                    (-((d.y - ce * w.y) * ka) + (n1.y + c1 * w.y) * k1) + w.y * k3,
                    (-((d.z - ce * w.z) * ka) + (n1.z + c1 * w.z) * k1) + w.z * k3);
    if (RV) {
        // rotating by d_omega turns d into d + d_omega x d and moves the
        // origin by d_omega x (y - c): dlog/d_omega = kd (d x w) + (y - c) x G
        const V3 yc = L.type == 2 ? v3(au * L.t[0] + av * L.b[0], au * L.t[1] + av * L.b[1], au * L.t[2] + av * L.b[2])
                                  : v3(0.0f, 0.0f, 0.0f);
        const V3 dw = v3(d.y * w.z - d.z * w.y, d.z * w.x - d.x * w.z, d.x * w.y - d.y * w.x);
        const V3 yg = v3(yc.y * G.z - yc.z * G.y, yc.z * G.x - yc.x * G.z, yc.x * G.y - yc.y * G.x);
        dl[0] = G.x;
        dl[1] = G.y;
        dl[2] = G.z;
        dl[3] = dw.x * kd + yg.x;
        dl[4] = dw.y * kd + yg.y;
        dl[5] = dw.z * kd + yg.z;
        return;
    }
    float ra = dot(v3(L.dd_da[0], L.dd_da[1], L.dd_da[2]), w) * kd;
    float rb = dot(v3(L.dd_db[0], L.dd_db[1], L.dd_db[2]), w) * kd;
    if (L.type == 2) {
        const V3 dya = v3(av * L.db_da[0], av * L.db_da[1], av * L.db_da[2]);
        const V3 dyb = v3(au * L.dt_db[0] + av * L.db_db[0], au * L.dt_db[1] + av * L.db_db[1],
                          au * L.dt_db[2] + av * L.db_db[2]);
        ra = dot(G, dya) + ra;
        rb = dot(G, dyb) + rb;
    }
    dl[0] = G.x;
    dl[1] = G.y;
    dl[2] = G.z;
    dl[3] = ra;
    dl[4] = rb;
}

struct HitInfo {
    V3 x, no;
    long long k;
    float inva, rho;
    bool flip;   // no is the patch normal negated (the ray arrives from its back)
};

__device__ __forceinline__ HitInfo hit_info(const Ray& r, float tb, int qb, const DevPatch* __restrict__ patches)
{
    HitInfo hi;
    hi.x = v3(r.ox + tb * r.dx, r.oy + tb * r.dy, r.oz + tb * r.dz);
    const DevPatch& P = patches[qb];
    const float4 o = P.o_inva, eu = P.eu_ilu, ev = P.ev_ilv, nr = P.n_rho;
    const V3 du = sub(hi.x, xyz(o));
    const float su = dot(du, xyz(eu)) * eu.w;
    const float sv = dot(du, xyz(ev)) * ev.w;
    const int ru = P.res_u, rv = P.res_v;
    int iu = (int)__builtin_floorf(su * (float)ru);
    int iv = (int)__builtin_floorf(sv * (float)rv);
    iu = iu < 0 ? 0 : (iu > ru - 1 ? ru - 1 : iu);
    iv = iv < 0 ? 0 : (iv > rv - 1 ? rv - 1 : iv);
    hi.k = P.base + (long long)iv * ru + iu;
    hi.inva = o.w;
    hi.rho = nr.w;
    const V3 nq = xyz(nr);
    const float nd = dot(nq, v3(r.dx, r.dy, r.dz));
    hi.flip = !(nd < 0.0f);
    hi.no = hi.flip ? v3(-nq.x, -nq.y, -nq.z) : nq;
    return hi;
}

// Piecewise-linear basis (Eq. pwLin on the texel grid): the four nodes
// around the hit (texel centres, indices clamped at the patch border so the
// hats sum to one) and their bilinear weights.
__device__ __forceinline__ void linear_nodes(V3 x, int qb, const DevPatch* __restrict__ patches, long long kb[4],
                                             float wb[4])
{
    const DevPatch& P = patches[qb];
    const float4 o = P.o_inva, eu = P.eu_ilu, ev = P.ev_ilv;
    const V3 du = sub(x, xyz(o));
    const float su = dot(du, xyz(eu)) * eu.w;
    const float sv = dot(du, xyz(ev)) * ev.w;
    const int ru = P.res_u, rv = P.res_v;
    const float fu = su * (float)ru - 0.5f, fv = sv * (float)rv - 0.5f;
    const float fu0 = __builtin_floorf(fu), fv0 = __builtin_floorf(fv);
    const float au1 = fu - fu0, av1 = fv - fv0;
    const float au0 = 1.0f - au1, av0 = 1.0f - av1;
    int i0 = (int)fu0, j0 = (int)fv0;
    int i1 = i0 + 1, j1 = j0 + 1;
    i0 = i0 < 0 ? 0 : (i0 > ru - 1 ? ru - 1 : i0);
    i1 = i1 < 0 ? 0 : (i1 > ru - 1 ? ru - 1 : i1);
    j0 = j0 < 0 ? 0 : (j0 > rv - 1 ? rv - 1 : j0);
    j1 = j1 < 0 ? 0 : (j1 > rv - 1 ? rv - 1 : j1);
    kb[0] = P.base + (long long)j0 * ru + i0;
    kb[1] = P.base + (long long)j0 * ru + i1;
    kb[2] = P.base + (long long)j1 * ru + i0;
    kb[3] = P.base + (long long)j1 * ru + i1;
    wb[0] = au0 * av0;
    wb[1] = au1 * av0;
    wb[2] = au0 * av1;
    wb[3] = au1 * av1;
}

__device__ __forceinline__ float linear_gather(const float* __restrict__ g, const long long kb[4], const float wb[4])
{
    return ((wb[0] * g[kb[0]] + wb[1] * g[kb[1]]) + wb[2] * g[kb[2]]) + wb[3] * g[kb[3]];
}

// Soft-edged spot: dlog of the intensity in the fixed direction of x_1 w.r.t.
// the inner and outer cone angles at constant power.  cone = (dlog I_e/dtheta_in,
// dlog I_e/dtheta_out, 2/(ci - co), 2 sin(theta_in)/(ci - co), sin(theta_out));
// in the fall-off ring log a = 2 log(cos - co) - 2 log(ci - co) adds its terms.
__device__ __forceinline__ void cone_dlog(const DevLight& L, const float* __restrict__ cone, V3 x1, V3 y,
                                          float& d_in, float& d_out)
{
    d_in = 0.0f;
    d_out = 0.0f;
    if (L.type != 3) return;
    const V3 v = sub(x1, y);
    const float r2 = dot(v, v);
    if (r2 <= 1e-12f) return;
    const float r = __builtin_sqrtf(r2);
    const float inv_r = 1.0f / r;
    const V3 w = v3(v.x * inv_r, v.y * inv_r, v.z * inv_r);
    const float cw = dot(v3(L.d[0], L.d[1], L.d[2]), w);
    const bool ring = cw > L.h && cw < L.w;
    d_in = ring ? cone[0] + cone[3] : cone[0];
    d_out = ring ? cone[1] + cone[4] * (2.0f / (cw - L.h) - cone[2]) : cone[1];
}

// Directional texels: 2pi-normalised hemispherical harmonics up to order 3
// (associated Legendre functions of x = 2 cos(theta) - 1 times cos / sin of
// m phi, index l^2 + l + m), and a Lambertian + normalised Phong BRDF in the
// local frame (normal = z) with its gradient w.r.t. the incident direction.
__device__ __forceinline__ void hsh_eval(int order, float ct, float cp, float sp, float H[16])
{
    const float x = 2.0f * ct - 1.0f;
    const float s1 = __builtin_sqrtf(fmaxf(0.0f, 1.0f - x * x));
    H[0] = 1.0f;
    if (order >= 1) {
        H[1] = (1.7320508075688772f * s1) * sp;
        H[2] = 1.7320508075688772f * x;
        H[3] = (1.7320508075688772f * s1) * cp;
    }
    const float c2 = 2.0f * (cp * cp) - 1.0f, s2 = 2.0f * (sp * cp);
    const float q = 1.0f - x * x;
    if (order >= 2) {
        H[4] = (1.9364916731037085f * q) * s2;
        H[5] = ((3.872983346207417f * x) * s1) * sp;
        H[6] = 2.23606797749979f * ((3.0f * (x * x) - 1.0f) * 0.5f);
        H[7] = ((3.872983346207417f * x) * s1) * cp;
        H[8] = (1.9364916731037085f * q) * c2;
    }
    if (order >= 3) {
        // l = 3 with the (2l+1)-scaled norms: P3, 3/2 (5x^2-1) s1, 15 x q, 15 q s1
        const float c3 = c2 * cp - s2 * sp, s3 = s2 * cp + c2 * sp;
        const float w1 = 5.0f * (x * x) - 1.0f;
        H[9] = ((2.091650066335189f * q) * s1) * s3;
        H[10] = ((5.123475382979799f * x) * q) * s2;
        H[11] = ((1.620185174601965f * w1) * s1) * sp;
        H[12] = 2.6457513110645907f * (((5.0f * (x * x) - 3.0f) * x) * 0.5f);
        H[13] = ((1.620185174601965f * w1) * s1) * cp;
        H[14] = ((5.123475382979799f * x) * q) * c2;
        H[15] = ((2.091650066335189f * q) * s1) * c3;
    }
}

__device__ __forceinline__ float brdf_local(float rho_d, float rho_s, float e, V3 wi, V3 wo, bool want_grad, V3& grad)
{
    float f = rho_d * 0.3183098861837907f;
    grad = v3(0.0f, 0.0f, 0.0f);
    if (rho_s > 0.0f) {
        const float ro = (-(wi.x * wo.x) - wi.y * wo.y) + wi.z * wo.z;
        if (ro > 0.0f) {
            const float ks = (rho_s * (e + 2.0f)) * 0.15915494309189533f;
            const float pw = exp2_c(e * log2_c(ro));
            f = f + ks * pw;
            if (want_grad) {
                const float gk = (ks * e) * (pw / ro);
                grad = v3(-(gk * wo.x), -(gk * wo.y), gk * wo.z);
            }
        }
    }
    return f;
}

// the bounce's orthonormal basis about the oriented normal
__device__ __forceinline__ void local_frame(V3 no, V3& b1, V3& b2)
{
    const float sg = __builtin_copysignf(1.0f, no.z);
    const float a = -1.0f / (sg + no.z);
    const float bxy = (no.x * no.y) * a;
    b1 = v3(1.0f + ((sg * no.x) * no.x) * a, sg * bxy, -(sg * no.x));
    b2 = v3(bxy, sg + (no.y * no.y) * a, -no.y);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------------------
// The forward / adjoint kernel: one persistent launch over the work tiles of
// every layout.  The grid holds as many waves as the chip keeps resident;
// each wave takes one tile at a time from a work queue (an atomic ticket per
// tile) until the queue is drained, so the traversal-stack overflow area is
// sized by resident waves, not by tiles.  No loop carries lane-divergent
// code across its back edge, so every wave-wide operation (ballot, shuffle)
// runs on a converged wave.
// ---------------------------------------------------------------------------

// The adjoint keeps its per-path first-hit derivative factors and running
// sums in LDS.  MODE selects at compile time, leaving the other instances
// as they were: 0 the box texel basis, 1 the piecewise-linear basis (four
// splats / a four-node gather per hit), 2 colour (three channel-planar
// texel arrays; the green and blue throughputs and adjoint sums live in
// LDS beside the red ones in registers), 30 + n directional texels of
// harmonic order n (hemispherical-harmonic coefficients of the reflected
// radiance and a glossy BRDF; the adjoint's first-hit BRDF terms live in
// LDS), 4 rotation-vector orientation (seven derivatives), 5 the
// direct-differentiation map of one luminaire (forward only), 6 the
// soft-edged spots' cone angles (adjoint, eight derivatives).
template <bool ADJ, bool STATS, int WPB, int LDS_D, int MODE>
// Occupancy floor per instance: the forward pass with the box basis runs
// eight waves per SIMD (64 VGPRs; the one spilled value is read only when a
// proposal samples the emission), with the linear basis seven (at eight it
// would spill its LDS stack address, read on every push and pop), the plain
// adjoint six (80 VGPRs; with kAdjLdsDepth stack entries in LDS, 6.5 KB per
// wave), the other instances five, the directional ones four.
__global__ void __launch_bounds__(WPB * 64)
    __attribute__((amdgpu_waves_per_eu(MODE >= 30 ? 4
                                                  : (!ADJ && !STATS && MODE == 0 ? 8
                                                     : (!STATS && ((!ADJ && MODE == 1) || MODE == 7) ? 7
                                                                                    : (ADJ && !STATS && (MODE == 0 || MODE == 8) ? 6 : 5))))))
    k_trace(TraceArgs a)
{
    constexpr bool DIR = MODE >= 30;               // directional texels of order MODE - 30
    constexpr int DORD = DIR ? MODE - 30 : 0;
    // MODE 7 (grey) and 8 (colour): the first pass of the two-pass adjoint
    // (box basis, no map): each path leaves a first-hit record and its
    // adjoint sums instead of adding its contribution to the tile's sums
    constexpr bool REC = ADJ && (MODE == 7 || MODE == 8);   // 8: the same in colour
    constexpr bool RGB = MODE == 2 || MODE == 8;
    // the plain and the colour adjoint keep kAdjLdsDepth / kColAdjLdsDepth
    // stack entries in LDS: their per-lane state takes the rest of the
    // budget of six (plain) or five (colour) waves per SIMD; the overflow
    // part of the stack is sized for the smaller
    constexpr int LDS_A = MODE == 2 ? kColAdjLdsDepth : kAdjLdsDepth;
    constexpr int LDS_S = (ADJ && (MODE == 0 || MODE == 2) && LDS_D > LDS_A) ? LDS_A : LDS_D;
    __shared__ int s_stack[WPB * LDS_S * 64];
    // adjoint per-lane state read once per path (first-hit derivative
    // factors, running contribution sums), kept in LDS instead of registers
    constexpr int NPAR = MODE == 4 ? 7 : (MODE == 6 ? 8 : 6);   // 4: rotation vector, 6: cone angles
    __shared__ float s_adj[ADJ && !REC ? WPB * 2 * NPAR * 64 : 1];
    // adjoint with a gradient-contribution map (grey irradiance, box or
    // linear basis): texel of the first hit
    constexpr bool VOTES = ADJ && MODE <= 1;
    __shared__ int s_k1[VOTES ? WPB * 64 : 1];
    // colour: per lane T_g, T_b, s_g, s_b and the three channel-weight sums
    __shared__ float s_rgb[RGB ? WPB * 7 * 64 : 1];
    // directional: forward, the hit's 16 coefficient sums; adjoint T2, R,
    // Q[3], D[3], w_in1[3], 1/r1 and the hit texel's 16 dO/dL values
    constexpr int DIRW = ADJ ? 28 : 16;
    __shared__ float s_dir[DIR ? WPB * DIRW * 64 : 1];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    float* adj = s_adj + (ADJ && !REC ? wib * 2 * NPAR * 64 + lane : 0);
    int k1_reg = 0;
    int* k1 = VOTES ? s_k1 + wib * 64 + lane : &k1_reg;
    float* rgbs = s_rgb + (RGB ? wib * 7 * 64 + lane : 0);
    float* dst = s_dir + (DIR ? wib * DIRW * 64 + lane : 0);
    // persistent wave: its slot owns one traversal-stack overflow area, and
    // it takes work tiles from the queue(s) until they are drained
    const long long gw = (long long)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(wib);
    if (gw >= a.gstack_waves) return;
    int* lst = s_stack + wib * LDS_S * 64 + lane;
    int* gst = a.gstack + gw * (long long)a.gdepth * 64;   // the wave's overflow area
    const int B = a.max_hits;
    const int thresh = a.refill_threshold;
    // with XCD-aware queues, workgroup b runs on XCD b % 8 and starts on that
    // XCD's contiguous share of the tiles, then helps with the others
    const int nq = a.n_queues;
    const int q0 = nq > 1 ? (int)(blockIdx.x % (unsigned)nq) : 0;
    int taken = 0;   // tiles this wave took: never more than exist, so the loop always ends
    for (int qi = 0; qi < nq; ++qi) {
    const int q = (q0 + qi) % nq;
    for (;;) {
    if (++taken > a.n_tiles) {
        if (lane == 0) atomicOr(a.flags, kStatusTraversal);
        break;
    }
    // one ticket per wave: every lane takes part in the atomic (lane 0 adds
    // 1, the others 0), so no lane-divergent branch precedes the read of
    // lane 0's result; a branch there lets the compiler thread the other
    // lanes' path into the loop and read the ticket under a partial mask
    const unsigned old_q = atomicAdd(a.queue + q, lane == 0 ? 1u : 0u);
    const int ticket = __builtin_amdgcn_readfirstlane((int)old_q);
    if (ticket >= a.q_len[q]) break;
    const int tile = a.q_first[q] + ticket;
    if (MODE == 5 && a.tiles[tile].x != a.tan_light) continue;   // other luminaires add nothing
    {
        const int4 ti = a.tiles[tile];
        const DevLight& L = a.lights[ti.x];
        const uint32_t first = (uint32_t)ti.y;
        const int count = L.invalid ? 0 : ti.z;   // a rejected luminaire traces nothing
        const uint32_t stream_id = ((uint32_t)ti.w << 16) | (uint32_t)L.l_local;
        constexpr int NC = DIR ? (DORD + 1) * (DORD + 1) : 1;
        const long long rowK = (RGB ? 3 : (DIR ? NC : 1)) * a.K;
        const float inv_np = DIR ? 1.0f / (float)a.dir_samples : 0.0f;
        long long* S = ADJ ? nullptr : a.S + (long long)ti.w * rowK;
        const float* g = ADJ ? a.g + (long long)ti.w * rowK : nullptr;
        float c0 = 1.0f, c1 = 1.0f, c2 = 1.0f;   // channel weights of the flux
        if (RGB) {
            c0 = a.colour[3 * ti.x];
            c1 = a.colour[3 * ti.x + 1];
            c2 = a.colour[3 * ti.x + 2];
#pragma unroll
            for (int c = 4; c < 7; ++c) rgbs[c * 64] = 0.0f;
        }
        const bool prop_on = a.prop_pdf != nullptr && (L.type == 1 || L.type == 2);
        const float* pdf = prop_on ? a.prop_pdf + 1024 * (long long)ti.x : nullptr;
        const float* cdf = prop_on ? a.prop_cdf + 1024 * (long long)ti.x : nullptr;
        const int* guide = prop_on ? a.prop_guide + 1025 * (long long)ti.x : nullptr;
        float* hist = (ADJ && a.bin_hist != nullptr && (L.type == 1 || L.type == 2)) ? a.bin_hist + 1024 * (long long)ti.x : nullptr;
        double* vote = (ADJ && a.vote != nullptr && ti.x == a.vote_light) ? a.vote : nullptr;
        // this luminaire's path 0 in the record planes, wave-uniform (the
        // host keeps a luminaire's paths under 2^30, so a path's byte offset
        // from it fits 32 bits)
        float* rec0 = nullptr;
        if (REC) {
            const long long rb = a.rec_base[ti.x];
            const long long rbu = ((long long)__builtin_amdgcn_readfirstlane((int)(rb >> 32)) << 32) |
                                  (long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(rb & 0xFFFFFFFFll));
            rec0 = a.rec + rbu;
        }

        int next = 0;          // paths of this tile handed out so far (uniform)
        bool alive = false;    // lane holds a path
        bool trav = false;     // lane is traversing its current segment
        uint32_t pid = 0;
        int h = 0, skip = -1, ebin = -1;
        float T = 1.0f, s_r = 0.0f, au = 0.0f, av = 0.0f, phi_r = 0.0f, wq = 0.0f;
        float tdl = 0.0f;      // direct differentiation: dlog_j of the first hit
        if (ADJ && !REC) {
#pragma unroll
            for (int c = 0; c < 2 * NPAR; ++c) adj[c * 64] = 0.0f;
        }
        unsigned miss = 0, n_seg = 0, n_nodes = 0, n_tris = 0, n_hits = 0;
        unsigned n_iter = 0, n_active = 0, n_phase = 0;   // wave-uniform counters
        bool overrun = false;
        Ray r;
        Trav s;
        start_segment(s);
        set_ray(r, v3(0, 0, 0), v3(0, 0, 1));

        // a lane that bounced at the last hit keeps its oriented normal (and
        // its ray and hit distance, which give the hit point) until the
        // phase's shared ray generation
        bool bnc = false;
        V3 bn = v3(0, 0, 1);
        for (;;) {
            // refill lanes without a path (ballot + prefix count)
            const bool need = !alive;
            const uint64_t m = ballot(need);
            bool newp = false;
            if (m != 0 && next < count) {
                const int slot = next + lanes_below(m);
                if (need && slot < count) {
                    pid = first + (uint32_t)slot;
                    newp = true;
                }
                next += __popcll(m);
            }
            // every lane starting a segment, a new path or a bounce, draws its
            // generator block once here: counter 0 for the emission, 1 + h for
            // the bounce after hit h
            if (newp || bnc) {
                const U4 ru = philox10(pid, stream_id, newp ? 0u : 1u + (uint32_t)h, 0u, a.key0, a.key1);
                V3 y, dir;
                if (newp) {
                    emit_from(L, ru, pid, stream_id, a.key0, a.key1, pdf, cdf, guide, a.alpha_plain, hist != nullptr, y,
                              dir, au, av, phi_r, ebin, wq);
                    if (REC && hist) {
                        // the emission cell and its weight, for the second
                        // pass's training histogram
                        const long long st = a.rec_stride;
                        *(float*)((char*)(rec0 + 11 * st) + (pid << 2)) = __int_as_float(ebin);
                        *(float*)((char*)(rec0 + 12 * st) + (pid << 2)) = wq;
                    }
                } else {
                    y = v3(r.ox + s.tb * r.dx, r.oy + s.tb * r.dy, r.oz + s.tb * r.dz);   // as in hit_info
                    dir = cosine_dir(bn, u24(ru.x), u24(ru.y));
                }
                set_ray(r, y, dir);
                start_segment(s);
                trav = true;
                bnc = false;
            }
            if (newp) {
                alive = true;
                h = 0;
                skip = -1;
                T = 1.0f;
                s_r = 0.0f;
                if (RGB) {
                    rgbs[0] = 1.0f;
                    rgbs[64] = 1.0f;
                    rgbs[128] = 0.0f;
                    rgbs[192] = 0.0f;
                }
                if (DIR && ADJ) {
                    dst[0] = 1.0f;
#pragma unroll
                    for (int c = 1; c < 8; ++c) dst[c * 64] = 0.0f;
                }
                if (STATS) ++n_seg;
            }
            // lanes holding a path: fixed while the traversal loop runs
            const uint64_t am = ballot(alive);
            if (am == 0) break;

            // traverse until enough lanes finished their segment
            for (;;) {
                const uint64_t tm = ballot(trav);
                if (tm == 0) break;
                if (__popcll(am & ~tm) >= thresh) break;
                if (STATS) {
                    ++n_iter;
                    n_active += (unsigned)__popcll(tm);
                }
                // one kind of operation per iteration: the queued triangle
                // tests once enough traversing lanes hold some (or all do),
                // node steps otherwise; either choice lets some lane progress
                int mode = 0;
                if (a.tri_share > 0) {
                    const int nq = __popcll(ballot(trav && s.lmask != 0));
                    const int nt = __popcll(tm);
                    mode = (nq > 0 && (nq == nt || nq * 8 >= nt * a.tri_share)) ? 1 : 2;
                }
                if (trav)
                    trav_step<LDS_S, STATS>(r, skip, s, trav, a.nodes, a.tris, lst, gst, n_nodes, n_tris,
                                            a.max_steps, overrun, mode);
            }

            // hit processing for lanes whose segment ended
            if (STATS) ++n_phase;
            if (alive && !trav) {
                bool end_path = false;
                if (s.pb < 0) {
                    ++miss;
                    end_path = true;
                } else {
                    ++h;
                    if (STATS) ++n_hits;
                    const HitInfo hi = hit_info(r, s.tb, s.qb, a.patches);
                    V3 fb1 = v3(0, 0, 0), fb2 = v3(0, 0, 0), wil = v3(0, 0, 0);
                    float2 gls = make_float2(0.0f, 1.0f);
                    if (MODE == 5) {
                        // d(Phi_h / A)/dp_j with the first hit held fixed
                        if (h == 1) {
                            float dl[6];
                            first_hit_dlog(L, hi.x, v3(r.ox, r.oy, r.oz), hi.no, au, av, dl);
                            tdl = dl[a.tan_param];
                        }
                        const long long qt =
                            (long long)__builtin_rintf((((phi_r * T) * hi.inva) * tdl) * 4294967296.0f);
                        __hip_atomic_fetch_add((unsigned long long*)(a.tangent + hi.k), (unsigned long long)qt,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else if (DIR) {
                        gls = a.glossy[s.qb];
                        local_frame(hi.no, fb1, fb2);
                        const V3 wiw = v3(-r.dx, -r.dy, -r.dz);
                        wil = v3(dot(fb1, wiw), dot(fb2, wiw), dot(hi.no, wiw));
#pragma unroll
                        for (int c = 0; c < 16; ++c)
                            if (c < NC) {
                                if (ADJ)
                                    dst[(12 + c) * 64] = g[c * a.K + hi.k];
                                else
                                    dst[c * 64] = 0.0f;
                            }
                        float pd = 0.0f;
                        V3 ql = v3(0, 0, 0);
                        U4 us = {0u, 0u, 0u, 0u};
                        for (int j = 0; j < a.dir_samples; ++j) {
                            if ((j & 1) == 0)
                                us = philox10(pid, stream_id, 0x100u + 32u * (uint32_t)h + (uint32_t)(j >> 1), 0u, a.key0,
                                              a.key1);
                            const float ua = (j & 1) ? u24(us.z) : u24(us.x);
                            const float ub = (j & 1) ? u24(us.w) : u24(us.y);
                            const float ct = ua;
                            const float st = __builtin_sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
                            float sp, cp;
                            sincos_2pi(ub, sp, cp);
                            const V3 wo = v3(st * cp, st * sp, ct);
                            float H[16];
                            hsh_eval(DORD, ct, cp, sp, H);
                            V3 gr;
                            const float f = brdf_local(hi.rho, gls.x, gls.y, wil, wo, ADJ && h == 1, gr);
                            if (!ADJ) {
#pragma unroll
                                for (int c = 0; c < 16; ++c)
                                    if (c < NC) dst[c * 64] = dst[c * 64] + f * H[c];
                            } else {
                                float G = 0.0f;
#pragma unroll
                                for (int c = 0; c < 16; ++c)
                                    if (c < NC) G = G + dst[(12 + c) * 64] * H[c];
                                pd = pd + f * G;
                                if (h == 1) ql = v3(ql.x + G * gr.x, ql.y + G * gr.y, ql.z + G * gr.z);
                            }
                        }
                        if (!ADJ) {
                            const float base = (phi_r * T) * hi.inva;
#pragma unroll
                            for (int c = 0; c < 16; ++c)
                                if (c < NC) {
                                    const long long qc =
                                        (long long)__builtin_rintf(((base * dst[c * 64]) * inv_np) * 4294967296.0f);
                                    __hip_atomic_fetch_add((unsigned long long*)(S + c * a.K + hi.k),
                                                           (unsigned long long)qc, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                                }
                        } else {
                            const float P = (pd * inv_np) * hi.inva;
                            s_r = s_r + P * T;
                            if (h >= 2) dst[64] = dst[64] + P * dst[0];
                            if (h == 1) {
                                float dl[6];
                                first_hit_dlog(L, hi.x, v3(r.ox, r.oy, r.oz), hi.no, au, av, dl);
#pragma unroll
                                for (int c = 0; c < 6; ++c) adj[c * 64] = phi_r * dl[c];
                                if (vote) *k1 = (int)hi.k;
                                const float sq = inv_np * hi.inva;
                                dst[128] = ((ql.x * sq) * fb1.x + (ql.y * sq) * fb2.x) + (ql.z * sq) * hi.no.x;
                                dst[192] = ((ql.x * sq) * fb1.y + (ql.y * sq) * fb2.y) + (ql.z * sq) * hi.no.y;
                                dst[256] = ((ql.x * sq) * fb1.z + (ql.y * sq) * fb2.z) + (ql.z * sq) * hi.no.z;
                                const V3 v1 = v3(r.ox - hi.x.x, r.oy - hi.x.y, r.oz - hi.x.z);
                                const float r1 = __builtin_sqrtf(dot(v1, v1));
                                const float ir1 = 1.0f / r1;
                                dst[512] = v1.x * ir1;
                                dst[576] = v1.y * ir1;
                                dst[640] = v1.z * ir1;
                                dst[704] = ir1;
                            }
                        }
                    } else if (!ADJ && RGB) {
                        const float v0 = ((phi_r * c0) * T) * hi.inva;
                        const float v1 = ((phi_r * c1) * rgbs[0]) * hi.inva;
                        const float v2 = ((phi_r * c2) * rgbs[64]) * hi.inva;
                        const long long q0 = (long long)__builtin_rintf(v0 * 4294967296.0f);
                        const long long q1 = (long long)__builtin_rintf(v1 * 4294967296.0f);
                        const long long q2 = (long long)__builtin_rintf(v2 * 4294967296.0f);
                        __hip_atomic_fetch_add((unsigned long long*)(S + hi.k), (unsigned long long)q0,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_add((unsigned long long*)(S + a.K + hi.k), (unsigned long long)q1,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_add((unsigned long long*)(S + 2 * a.K + hi.k), (unsigned long long)q2,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else if (!ADJ) {
                        const float val = (phi_r * T) * hi.inva;
                        if (MODE == 1) {
                            long long kb[4];
                            float wb[4];
                            linear_nodes(hi.x, s.qb, a.patches, kb, wb);
#pragma unroll
                            for (int c = 0; c < 4; ++c) {
                                const long long code = (long long)__builtin_rintf((val * wb[c]) * 4294967296.0f);
                                __hip_atomic_fetch_add((unsigned long long*)(S + kb[c]), (unsigned long long)code,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            }
                        } else {
                            const long long code = (long long)__builtin_rintf(val * 4294967296.0f);
                            __hip_atomic_fetch_add((unsigned long long*)(S + hi.k), (unsigned long long)code,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    } else if (!DIR) {
                        float gk;
                        if (MODE == 1) {
                            long long kb[4];
                            float wb[4];
                            linear_nodes(hi.x, s.qb, a.patches, kb, wb);
                            gk = linear_gather(g, kb, wb);
                        } else {
                            gk = g[hi.k];
                        }
                        s_r = s_r + (gk * hi.inva) * T;
                        if (RGB) {
                            rgbs[128] = rgbs[128] + (g[a.K + hi.k] * hi.inva) * rgbs[0];
                            rgbs[192] = rgbs[192] + (g[2 * a.K + hi.k] * hi.inva) * rgbs[64];
                        }
                        if (h == 1 && REC) {
                            // what the path's dlog needs, for the second pass
                            const long long st = a.rec_stride;
                            const unsigned off = pid << 2;
                            const float v[10] = {hi.x.x, hi.x.y, hi.x.z, r.ox, r.oy, r.oz,
                                                 __uint_as_float((unsigned)s.qb | (hi.flip ? 0x80000000u : 0u)),
                                                 au, av, phi_r};
#pragma unroll
                            for (int f = 0; f < 10; ++f) *(float*)((char*)(rec0 + f * st) + off) = v[f];
                        } else if (h == 1) {
                            float dl[NPAR];
                            first_hit_dlog<MODE == 4>(L, hi.x, v3(r.ox, r.oy, r.oz), hi.no, au, av, dl);
                            if constexpr (MODE == 6)
                                cone_dlog(L, a.cone + 5 * ti.x, hi.x, v3(r.ox, r.oy, r.oz), dl[6], dl[7]);
#pragma unroll
                            for (int c = 0; c < NPAR; ++c) adj[c * 64] = phi_r * dl[c];
                            if (vote) *k1 = (int)hi.k;
                        }
                    }
                    if (h >= B) {
                        end_path = true;
                    } else if (!DIR) {
                        // the new direction is drawn with the phase's emissions
                        bnc = true;
                        bn = hi.no;
                        skip = s.qb;
                        if (RGB) {
                            const float4 rho = a.rho_rgb[skip];
                            T = T * rho.x;
                            rgbs[0] = rgbs[0] * rho.y;
                            rgbs[64] = rgbs[64] * rho.z;
                        } else {
                            T = T * hi.rho;
                        }
                        if (STATS) ++n_seg;
                    } else {
                        const V3 nd = bounce_dir(hi.no, pid, stream_id, (uint32_t)h, a.key0, a.key1);
                        set_ray(r, hi.x, nd);
                        skip = s.qb;
                        start_segment(s);
                        trav = true;
                        if (RGB) {
                            const float4 rho = a.rho_rgb[skip];
                            T = T * rho.x;
                            rgbs[0] = rgbs[0] * rho.y;
                            rgbs[64] = rgbs[64] * rho.z;
                        } else if (DIR) {
                            const V3 wo = v3(dot(fb1, nd), dot(fb2, nd), dot(hi.no, nd));
                            V3 gr;
                            const float fbv = brdf_local(hi.rho, gls.x, gls.y, wil, wo, ADJ && h == 1, gr);
                            const float wb = fbv * 3.14159265358979f;
                            if (ADJ) {
                                if (h == 1) {
                                    const float pi = 3.14159265358979f;
                                    dst[320] = ((gr.x * pi) * fb1.x + (gr.y * pi) * fb2.x) + (gr.z * pi) * hi.no.x;
                                    dst[384] = ((gr.x * pi) * fb1.y + (gr.y * pi) * fb2.y) + (gr.z * pi) * hi.no.y;
                                    dst[448] = ((gr.x * pi) * fb1.z + (gr.y * pi) * fb2.z) + (gr.z * pi) * hi.no.z;
                                } else {
                                    dst[0] = dst[0] * wb;
                                }
                            }
                            T = T * wb;
                        } else {
                            T = T * hi.rho;
                        }
                        if (STATS) ++n_seg;
                    }
                }
                if (end_path) {
                    if (REC) {
                        // every path leaves its adjoint sum(s) (0 without a
                        // hit, which tells the second pass to skip its record)
                        *(float*)((char*)(rec0 + 10 * a.rec_stride) + (pid << 2)) = s_r;
                        if (RGB) {
                            *(float*)((char*)(rec0 + 13 * a.rec_stride) + (pid << 2)) = rgbs[128];
                            *(float*)((char*)(rec0 + 14 * a.rec_stride) + (pid << 2)) = rgbs[192];
                        }
                    } else if (ADJ && h >= 1) {
                        // colour: every channel shares the path, so the
                        // geometric terms take the colour-weighted adjoint
                        // sum, and dO/dc_ch gathers s_ch Phi_r
                        float se = s_r;
                        if (RGB) {
                            se = (s_r * c0 + rgbs[128] * c1) + rgbs[192] * c2;
                            rgbs[256] += s_r * phi_r;
                            rgbs[320] += rgbs[128] * phi_r;
                            rgbs[384] += rgbs[192] * phi_r;
                        }
                        // directional: d/dy of the first hit's projection and
                        // bounce weight through w_in1 = (y - x_1)/|y - x_1|
                        float ext[6] = {0, 0, 0, 0, 0, 0};
                        if (DIR) {
                            const float Rd = dst[64];
                            const V3 v = v3(dst[128] + Rd * dst[320], dst[192] + Rd * dst[384], dst[256] + Rd * dst[448]);
                            const V3 om = v3(dst[512], dst[576], dst[640]);
                            const float ir1 = dst[704];
                            const float wv = dot(om, v);
                            const V3 u = v3((v.x - om.x * wv) * ir1, (v.y - om.y * wv) * ir1, (v.z - om.z * wv) * ir1);
                            V3 dya = v3(0, 0, 0), dyb = v3(0, 0, 0);
                            if (L.type == 2) {
                                dya = v3(av * L.db_da[0], av * L.db_da[1], av * L.db_da[2]);
                                dyb = v3(au * L.dt_db[0] + av * L.db_db[0], au * L.dt_db[1] + av * L.db_db[1],
                                         au * L.dt_db[2] + av * L.db_db[2]);
                            }
                            ext[0] = u.x;
                            ext[1] = u.y;
                            ext[2] = u.z;
                            ext[3] = dot(u, dya);
                            ext[4] = dot(u, dyb);
                        }
                        float m2 = 0.0f;
#pragma unroll
                        for (int c = 0; c < NPAR; ++c) {
                            float cr = se * adj[c * 64];
                            if (DIR) cr = cr + phi_r * ext[c < 6 ? c : 0];
                            adj[(NPAR + c) * 64] += cr;
                            if (hist && c < 6) {
                                const float z = cr * a.inv_sigma[6 * ti.x + c];
                                m2 = m2 + z * z;
                            }
                        }
                        if (hist && ebin >= 0) atomicAdd(hist + ebin, m2 * wq);
                        // the path's share of dO/dp_j, placed at its first hit
                        if (vote) {
                            float cv = se * adj[a.vote_param * 64];
                            if (DIR) cv = cv + phi_r * ext[a.vote_param];
                            unsafeAtomicAdd(vote + *k1, (double)cv);
                        }
                    }
                    alive = false;
                }
            }
        }
        if (ADJ && !REC) {
            double acc[NPAR];
#pragma unroll
            for (int c = 0; c < NPAR; ++c) acc[c] = wave_sum((double)adj[(NPAR + c) * 64]);
            if (lane == 0) {
#pragma unroll
                for (int c = 0; c < NPAR; ++c) a.partials[(long long)tile * NPAR + c] = acc[c];
            }
            if (RGB) {
                double accc[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) accc[c] = wave_sum((double)rgbs[(4 + c) * 64]);
                if (lane == 0) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) a.partials_col[(long long)tile * 3 + c] = accc[c];
                }
            }
        }
        const unsigned wm = wave_sum(miss);
        if (lane == 0 && wm) atomicAdd(a.misses, (unsigned long long)wm);
        if (overrun) atomicOr(a.flags, kStatusTraversal);
        if (STATS) {
            const unsigned c0 = wave_sum(n_seg), c1 = wave_sum(n_nodes), c2 = wave_sum(n_tris),
                           c3 = wave_sum(n_hits);
            if (lane == 0) {
                atomicAdd(a.stats + 0, (unsigned long long)c0);
                atomicAdd(a.stats + 1, (unsigned long long)c1);
                atomicAdd(a.stats + 2, (unsigned long long)c2);
                atomicAdd(a.stats + 3, (unsigned long long)c3);
                atomicAdd(a.stats + 4, (unsigned long long)wm);
                atomicAdd(a.stats + 5, (unsigned long long)n_iter);
                atomicAdd(a.stats + 6, (unsigned long long)n_active);
                atomicAdd(a.stats + 7, (unsigned long long)n_phase);
            }
        }
    }
    }   // tiles of queue q
    }   // queues
}

// One path per thread (grid-stride): hit sequences and per-path adjoint
// contributions, with the same device functions as the tracing kernel.
template <int LDS_D>
__global__ void __launch_bounds__(256) k_record(RecordArgs a)
{
    __shared__ int s_stack[4 * LDS_D * 64];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const long long gw = (long long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(wib);
    int* lst = s_stack + wib * LDS_D * 64 + lane;
    int* gst = a.gstack + gw * (long long)a.gdepth * 64;   // the wave's overflow area
    const DevLight& L = a.lights[a.gl];
    const float* g = a.g ? a.g + (long long)a.layout * a.K : nullptr;
    const long long stride = (long long)gridDim.x * 256;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < a.count; idx += stride) {
        const uint32_t pid = (uint32_t)(a.first + idx);
        for (int hh = 0; hh < a.max_hits; ++hh) {
            a.prim[idx * a.max_hits + hh] = -1;
            a.texel[idx * a.max_hits + hh] = -1;
        }
        if (L.invalid) {
            if (a.contrib)
                for (int c = 0; c < 6; ++c) a.contrib[idx * 6 + c] = 0.0f;
            continue;
        }
        V3 y, dir;
        float au, av, phi_r;
        int ebin;
        float wq;
        const bool prop_on = a.prop_pdf != nullptr && (L.type == 1 || L.type == 2);
        emit(L, pid, a.stream_id, a.key0, a.key1, prop_on ? a.prop_pdf + 1024 * (long long)a.gl : nullptr,
             prop_on ? a.prop_cdf + 1024 * (long long)a.gl : nullptr,
             prop_on ? a.prop_guide + 1025 * (long long)a.gl : nullptr, a.alpha_plain, false, y, dir, au, av, phi_r,
             ebin, wq);
        Ray r;
        set_ray(r, y, dir);
        int skip = -1;
        float T = 1.0f, s_r = 0.0f;
        float dphi[6] = {0, 0, 0, 0, 0, 0};
        int h = 0;
        unsigned dummy0 = 0, dummy1 = 0;
        bool overrun = false;
        for (;;) {
            Trav s;
            start_segment(s);
            bool trav = true;
            while (trav)
                trav_step<LDS_D, false>(r, skip, s, trav, a.nodes, a.tris, lst, gst, dummy0, dummy1, a.max_steps,
                                        overrun);
            if (s.pb < 0) break;
            ++h;
            const HitInfo hi = hit_info(r, s.tb, s.qb, a.patches);
            a.prim[idx * a.max_hits + h - 1] = s.pb;
            a.texel[idx * a.max_hits + h - 1] = (int)hi.k;
            if (g) {
                float gk;
                if (a.linear) {
                    long long kb[4];
                    float wb[4];
                    linear_nodes(hi.x, s.qb, a.patches, kb, wb);
                    gk = linear_gather(g, kb, wb);
                } else {
                    gk = g[hi.k];
                }
                s_r = s_r + (gk * hi.inva) * T;
                if (h == 1) {
                    float dl[6];
                    first_hit_dlog(L, hi.x, v3(r.ox, r.oy, r.oz), hi.no, au, av, dl);
                    for (int c = 0; c < 6; ++c) dphi[c] = phi_r * dl[c];
                }
            }
            if (h >= a.max_hits) break;
            const V3 nd = bounce_dir(hi.no, pid, a.stream_id, (uint32_t)h, a.key0, a.key1);
            set_ray(r, hi.x, nd);
            skip = s.qb;
            T = T * hi.rho;
        }
        if (a.contrib) {
            for (int c = 0; c < 6; ++c) a.contrib[idx * 6 + c] = (g && h >= 1) ? s_r * dphi[c] : 0.0f;
        }
        if (overrun) atomicOr(a.flags, kStatusTraversal);
    }
}

// ---------------------------------------------------------------------------
// Object-space path tracing with next-event estimation, the comparison
// estimator of Sec. 6 (after Stam 2020) on the same texels: M points uniform
// in each texel; every path vertex connects to one luminaire of the layout
// chosen uniformly (shadow ray); the path continues with the light tracer's
// cosine bounce (at the texel point on a side drawn with probability 1/2).
// The gradient differentiates each connection with its vertex held fixed:
// the first-hit derivative factors evaluated at that vertex.
// ---------------------------------------------------------------------------

// radiant intensity towards unit direction w from the luminaire's origin
__device__ __forceinline__ float light_intensity(const DevLight& L, V3 w)
{
    if (L.type == 0) return L.P * 0.07957747154594767f;
    const float ce = dot(v3(L.d[0], L.d[1], L.d[2]), w);
    if (L.type == 3) {
        if (!(ce > L.h)) return 0.0f;
        float a = 1.0f;
        if (ce < L.w) {
            const float f = (ce - L.h) / (L.w - L.h);
            a = f * f;
        }
        return ((L.P * L.kcap) * a) * (0.15915494309189533f / (1.0f - L.h));
    }
    if (!(ce > 0.0f)) return 0.0f;
    float pw = 1.0f;
    if (L.n != 0.0f) pw = exp2_c(L.n * log2_c(ce));
    return L.P * (((L.n + 1.0f) * 0.15915494309189533f) * pw);
}

// closest hit along r (origin patch skipped) with t < tmax; per-lane loop
template <int LDS_D>
__device__ __forceinline__ void trace_lane(const Ray& r, int skip, float tmax, Trav& s, const float4* nodes,
                                           const float4* tris, int* lst, int* gst, int max_steps, bool& overrun)
{
    start_segment(s);
    s.tb = tmax;
    bool trav = true;
    unsigned d0 = 0, d1 = 0;
    while (trav) trav_step<LDS_D, false>(r, skip, s, trav, nodes, tris, lst, gst, d0, d1, max_steps, overrun);
}

template <bool ADJ, int LDS_D>
__global__ void __launch_bounds__(256) k_pt(PtArgs a)
{
    __shared__ int s_stack[4 * LDS_D * 64];
    __shared__ double s_grad[ADJ ? kPtMaxLights * 6 : 1];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const long long gw = (long long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(wib);
    int* lst = s_stack + wib * LDS_D * 64 + lane;
    int* gst = a.gstack + gw * (long long)a.gdepth * 64;   // the wave's overflow area
    if (ADJ) {
        for (int j = threadIdx.x; j < a.nl * 6; j += 256) s_grad[j] = 0.0;
        __syncthreads();
    }
    const uint32_t stream = ((uint32_t)a.layout << 16) | 0xFFFFu;
    const float inv_m = 1.0f / (float)a.M;
    const float fl = (float)a.nl;
    const long long total = a.K * a.M;
    const long long stride = (long long)gridDim.x * 256;
    bool overrun = false;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < total; idx += stride) {
        const long long k = idx / a.M;
        // patch of texel k: the last patch whose first texel is <= k
        int lo = 0, hi = a.n_patches - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.pbase[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        const int q = lo;
        const DevPatch& P = a.patches[q];
        const long long loc = k - P.base;
        const int iu = (int)(loc % P.res_u), iv = (int)(loc / P.res_u);
        const uint32_t pid = (uint32_t)idx;
        const U4 r0 = philox10(pid, stream, 0u, 0u, a.key0, a.key1);
        const float su = ((float)iu + u24(r0.x)) / (float)P.res_u;
        const float sv = ((float)iv + u24(r0.y)) / (float)P.res_v;
        const float4 o = P.o_inva, eu = P.eu_ilu, ev = P.ev_ilv;
        V3 v = v3((o.x + su * eu.x) + sv * ev.x, (o.y + su * eu.y) + sv * ev.y, (o.z + su * eu.z) + sv * ev.z);
        const V3 nq0 = xyz(P.n_rho);
        const float gk = ADJ ? a.g[k] * inv_m : 0.0f;
        float e = 0.0f, T = 1.0f;
        int qv = q;
        bool have_side = false;
        V3 nside = nq0;
        for (int h = 0; h < a.max_hits; ++h) {
            // connection to one luminaire chosen uniformly
            const U4 rl = philox10(pid, stream, 1u + 2u * (uint32_t)h, 0u, a.key0, a.key1);
            int ls = (int)(u24(rl.x) * fl);
            ls = ls > a.nl - 1 ? a.nl - 1 : ls;
            const DevLight& L = a.lights[ls];
            V3 y = v3(L.c[0], L.c[1], L.c[2]);
            float au = 0.0f, av = 0.0f;
            if (L.type == 2) {
                au = (u24(rl.y) - 0.5f) * L.w;
                av = (u24(rl.z) - 0.5f) * L.h;
                y = v3((L.c[0] + au * L.t[0]) + av * L.b[0], (L.c[1] + au * L.t[1]) + av * L.b[1],
                       (L.c[2] + au * L.t[2]) + av * L.b[2]);
            }
            const V3 vec = sub(v, y);
            const float r2 = dot(vec, vec);
            if (r2 > 1e-12f) {
                const float rd = __builtin_sqrtf(r2);
                const float inv_r = 1.0f / rd;
                const V3 w = v3(vec.x * inv_r, vec.y * inv_r, vec.z * inv_r);
                const V3 nqv = xyz(a.patches[qv].n_rho);
                V3 n1;
                if (have_side) n1 = nside;
                else n1 = dot(nqv, w) < 0.0f ? nqv : v3(-nqv.x, -nqv.y, -nqv.z);
                const float cv = -dot(n1, w);
                const float I = (cv > 0.0f && !L.invalid) ? light_intensity(L, w) : 0.0f;
                if (I > 0.0f) {
                    const float C = (I * cv) / r2;
                    Ray sr;
                    set_ray(sr, v, v3(-w.x, -w.y, -w.z));
                    Trav s;
                    trace_lane<LDS_D>(sr, qv, rd * 0.9999f, s, a.nodes, a.tris, lst, gst, a.max_steps, overrun);
                    if (s.pb < 0) {
                        const float we = (T * fl) * C;
                        e = e + we;
                        if (ADJ) {
                            float dl[6];
                            first_hit_dlog(L, v, y, n1, au, av, dl);
#pragma unroll
                            for (int c = 0; c < 6; ++c) atomicAdd(&s_grad[ls * 6 + c], (double)((gk * we) * dl[c]));
                        }
                    }
                }
            }
            if (h == a.max_hits - 1) break;
            // bounce: at the texel point a side drawn with probability 1/2
            // (weight 2), later the side facing the incoming ray
            V3 no;
            if (!have_side) {
                const float sg = u24(r0.z) < 0.5f ? 1.0f : -1.0f;
                no = v3(sg * nq0.x, sg * nq0.y, sg * nq0.z);
                T = T * 2.0f;
            } else {
                no = nside;
            }
            const U4 rb = philox10(pid, stream, 2u + 2u * (uint32_t)h, 0u, a.key0, a.key1);
            const V3 dir = cosine_dir(no, u24(rb.x), u24(rb.y));
            Ray br;
            set_ray(br, v, dir);
            Trav s;
            trace_lane<LDS_D>(br, qv, __builtin_inff(), s, a.nodes, a.tris, lst, gst, a.max_steps, overrun);
            if (s.pb < 0) break;
            const HitInfo hn = hit_info(br, s.tb, s.qb, a.patches);
            T = T * hn.rho;
            v = hn.x;
            qv = s.qb;
            nside = hn.no;
            have_side = true;
        }
        if (!ADJ) {
            const long long code = (long long)__builtin_rintf((e * inv_m) * 4294967296.0f);
            __hip_atomic_fetch_add((unsigned long long*)(a.S + k), (unsigned long long)code, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (overrun) atomicOr(a.flags, kStatusTraversal);
    if (ADJ) {
        __syncthreads();
        for (int j = threadIdx.x; j < a.nl * 6; j += 256)
            if (s_grad[j] != 0.0) atomicAdd(a.grad + j, s_grad[j]);
    }
}

__global__ void k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

// Central differences: the two parameter sets p +- h e_idx (FP32 sums) and
// the step actually taken, (p + h) - (p - h) in FP64.
__global__ void k_fd_params(const float* __restrict__ p, int n, int idx, float h, float* __restrict__ pp,
                            float* __restrict__ pm, double* __restrict__ den)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = p[i];
    const float vp = i == idx ? v + h : v;
    const float vm = i == idx ? v - h : v;
    pp[i] = vp;
    pm[i] = vm;
    if (i == idx) den[0] = (double)vp - (double)vm;
}

// F_k = (S+_k - S-_k) 2^-32 / den: the difference is exact on the fixed-point sums.
__global__ void k_fd_diff(const long long* __restrict__ Sp, const long long* __restrict__ Sm, long long K,
                          const double* __restrict__ den, float* __restrict__ F)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    const double d = den[0];
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += stride)
        F[k] = (float)(((double)(Sp[k] - Sm[k]) * 0x1p-32) / d);
}

// Luminaire setup: frame R = R_y(beta) R_x(alpha), derivatives, Phi_r = P/N_l.
// lstat_i = (type, layout, l_local, -), lstat_f = (n, w, h, N_l as float bits unused).
// Rodrigues' formula in FP64, R = I + sin(phi)/phi K + (1 - cos(phi))/phi^2 K^2,
// K = [theta]x, with the linear small-angle form I + K near zero (Sec. 4.4.2).
__device__ void rodrigues_f64(const double th[3], double R[9])
{
    const double K[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    const double f2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
    double A = 1.0, Bc = 0.0;
    if (f2 >= 1e-12) {
        const double f = __builtin_sqrt(f2);
        double sf, cf;
        sincos_f64(f, sf, cf);
        A = sf / f;
        Bc = (1.0 - cf) / f2;
    }
    for (int i = 0; i < 9; ++i) R[i] = ((i % 4 == 0) ? 1.0 : 0.0) + A * K[i] + Bc * K2[i];
}

// Jacobian of the exponential map: R(theta + dtheta) = exp([J dtheta]x) R(theta)
__device__ void rot_jacobian_f64(const double th[3], double J[9])
{
    const double K[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    const double f2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
    double a = 0.0, b = 0.0;
    if (f2 >= 1e-12) {
        const double f = __builtin_sqrt(f2);
        double sf, cf;
        sincos_f64(f, sf, cf);
        a = (1.0 - cf) / f2;
        b = (f - sf) / (f2 * f);
    }
    for (int i = 0; i < 9; ++i) J[i] = ((i % 4 == 0) ? 1.0 : 0.0) + a * K[i] + b * K2[i];
}

__global__ void k_light_setup(const float* __restrict__ params, const int4* __restrict__ si,
                              const float4* __restrict__ sf, const long long* __restrict__ npaths, int n,
                              DevLight* __restrict__ out, unsigned* __restrict__ flags, int rv,
                              float* __restrict__ cone)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    // a luminaire whose parameters are not all finite, or whose power is not
    // positive, raises the sticky parameter status and is set up from benign
    // stand-in values (origin 0, default frame, unit power) with no paths'
    // worth of flux: its work tiles then trace nothing, so no NaN or
    // out-of-range value reaches a fixed-point splat or a gradient sum
    const int np = rv ? 7 : 6;
    float p[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    bool ok = true;
    for (int c = 0; c < np; ++c) {
        p[c] = params[np * l + c];
        ok = ok && __builtin_isfinite(p[c]);
    }
    ok = ok && p[np - 1] > 0.0f;
    if (!ok) {
        atomicOr(flags, kStatusParams);
        for (int c = 0; c < np; ++c) p[c] = 0.0f;
        p[np - 1] = 1.0f;
    }
    double sa_d, ca_d, sb_d, cb_d;
    sincos_f64((double)p[3], sa_d, ca_d);
    sincos_f64((double)p[4], sb_d, cb_d);
    const float sa = (float)sa_d, ca = (float)ca_d, sb = (float)sb_d, cb = (float)cb_d;
    DevLight L;
    L.c[0] = p[0]; L.c[1] = p[1]; L.c[2] = p[2];
    L.d[0] = -(sb * ca); L.d[1] = sa; L.d[2] = -(cb * ca);
    L.t[0] = cb; L.t[1] = 0.0f; L.t[2] = -sb;
    L.b[0] = sb * sa; L.b[1] = ca; L.b[2] = cb * sa;
    L.dd_da[0] = sb * sa; L.dd_da[1] = ca; L.dd_da[2] = cb * sa;
    L.dd_db[0] = -(cb * ca); L.dd_db[1] = 0.0f; L.dd_db[2] = sb * ca;
    L.dt_db[0] = -sb; L.dt_db[1] = 0.0f; L.dt_db[2] = -cb;
    L.db_da[0] = sb * ca; L.db_da[1] = -sa; L.db_da[2] = cb * ca;
    L.db_db[0] = cb * sa; L.db_db[1] = 0.0f; L.db_db[2] = -(sb * sa);
    const int4 i4 = si[l];
    const float4 f4 = sf[l];
    const long long nl = npaths[l];
    if (rv) {
        // world frame from the rotation vector: d = R(0,0,-1), t = R e_x, b = R e_y
        const double th[3] = {(double)p[3], (double)p[4], (double)p[5]};
        double R[9];
        rodrigues_f64(th, R);
        for (int c = 0; c < 3; ++c) {
            L.d[c] = (float)(-R[3 * c + 2]);
            L.t[c] = (float)R[3 * c];
            L.b[c] = (float)R[3 * c + 1];
            L.dd_da[c] = L.dd_db[c] = L.dt_db[c] = L.db_da[c] = L.db_db[c] = 0.0f;
        }
    }
    const float Pw = p[rv ? 6 : 5];
    L.P = Pw;
    L.n_paths = nl;
    L.phi_r = Pw / (float)nl;
    L.n = f4.x;
    L.w = f4.y;
    L.h = f4.z;
    L.type = i4.x;
    L.kcap = 1.0f;
    if (L.type == 3) {
        // soft-edged spot: w, h carry the cosines of the inner and outer cone
        // angles; P is the total flux, so Phi_r = (P/N) kcap a(cos) with
        // kcap = (1 - cos_out) / ((1 - cos_in) + (cos_in - cos_out) / 3)
        double si_d, ci_d, so_d, co_d;
        sincos_f64((double)f4.y, si_d, ci_d);
        sincos_f64((double)f4.z, so_d, co_d);
        L.w = (float)ci_d;
        L.h = (float)co_d;
        const float kcap = (float)((1.0 - co_d) / ((1.0 - ci_d) + (ci_d - co_d) / 3.0));
        L.phi_r = L.phi_r * kcap;
        L.kcap = kcap;
        if (cone != nullptr) {
            // cone-angle derivatives at constant P: I_e = P / (2 pi den),
            // dlog I_e/dci = (2/3)/den, dlog I_e/dco = (1/3)/den, dci = -sin dtheta
            const double den = (1.0 - ci_d) + (ci_d - co_d) / 3.0;
            cone[5 * l + 0] = (float)(-(si_d * (2.0 / 3.0)) / den);
            cone[5 * l + 1] = (float)(-(so_d * (1.0 / 3.0)) / den);
            cone[5 * l + 2] = (float)(2.0 / (ci_d - co_d));
            cone[5 * l + 3] = (float)(2.0 * si_d / (ci_d - co_d));
            cone[5 * l + 4] = (float)so_d;
        }
    }
    L.layout = i4.y;
    L.l_local = i4.z;
    L.invalid = ok ? 0 : 1;
    if (!ok) L.phi_r = 0.0f;
    L.pad1 = 0;
    out[l] = L;
}

__global__ void k_fill_f32(float* __restrict__ p, long long n, float v)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_clear(long long* __restrict__ S, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    longlong2* S2 = (longlong2*)S;
    const long long n2 = n >> 1;
    for (long long j = i; j < n2; j += stride) S2[j] = make_longlong2(0, 0);
    if ((n & 1) && i == 0) S[n - 1] = 0;
}

// E_k = S_k 2^-32 through FP64; sticky overflow flag at |S| >= 2^62.
__global__ void k_finalize(const long long* __restrict__ S, float* __restrict__ E, long long n,
                           unsigned* __restrict__ flags)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool ovf = false;
    const long long n2 = n >> 1;
    const longlong2* S2 = (const longlong2*)S;
    float2* E2 = (float2*)E;
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n2; j += stride) {
        const longlong2 v = S2[j];
        ovf |= (v.x >= (1ll << 62)) | (v.x <= -(1ll << 62)) | (v.y >= (1ll << 62)) | (v.y <= -(1ll << 62));
        E2[j] = make_float2((float)((double)v.x * 0x1p-32), (float)((double)v.y * 0x1p-32));
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const long long v = S[n - 1];
        ovf |= (v >= (1ll << 62)) | (v <= -(1ll << 62));
        E[n - 1] = (float)((double)v * 0x1p-32);
    }
    if (ovf) atomicOr(flags, kStatusOverflow);
}

// O = 1/2 sum A_k alpha_k (E_k - E*_k)^2 (FP64, fixed grid + fixed tree),
// g_k = (A_k alpha_k)(E_k - E*_k).
__global__ void __launch_bounds__(256) k_objective(const float* __restrict__ E, const float* __restrict__ Et,
                                                  const float* __restrict__ alpha, const float* __restrict__ A,
                                                  long long K, long long n, float* __restrict__ g,
                                                  double* __restrict__ part)
{
    __shared__ double sh[256];
    double acc = 0.0;
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const float ak = A[i % K];
        const float al = alpha ? alpha[i] : 1.0f;
        const float e = E[i], et = Et[i];
        if (g) g[i] = (ak * al) * (e - et);
        const double de = (double)e - (double)et;
        acc += (double)ak * (double)al * de * de;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_objective_final(const double* __restrict__ part, int n_part,
                                                        double* __restrict__ O)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n_part; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *O = 0.5 * sh[0];
}

// Per-light gradient: ordered sum of the light's tile partials (one wave per light).
template <int NC>
__global__ void __launch_bounds__(64) k_grad_reduce(const double* __restrict__ partials,
                                                   const int2* __restrict__ range, int n_lights,
                                                   float* __restrict__ grad)
{
    const int l = blockIdx.x;
    if (l >= n_lights) return;
    const int2 rg = range[l];
    double acc[NC];
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (int t = rg.x + (int)threadIdx.x; t < rg.y; t += 64)
        for (int c = 0; c < NC; ++c) acc[c] += partials[(long long)t * NC + c];
    for (int c = 0; c < NC; ++c) acc[c] = wave_sum(acc[c]);
    if (threadIdx.x == 0)
        for (int c = 0; c < NC; ++c) grad[NC * l + c] = (float)acc[c];
}

// Second pass of the two-pass adjoint (Alg. 2's update at the end of a
// path): each recorded path of a tile contributes s_r (Phi_r dlog_r), the
// first hit's dlog from its record (the oriented normal is the patch's, or
// its negation), the same FP32 products as the one-pass kernel; the tile's
// sums are FP64, thread-strided in path order and then a fixed tree.  With
// the training histogram each path also adds its squared normalised
// contribution, weighted, to its emission cell, as the one-pass kernel does.
// In colour the record holds the three channels' sums: the geometric terms
// take their colour-weighted sum, and dO/dc_ch gathers s_ch Phi_r.
template <bool RGB>
__global__ void __launch_bounds__(256) k_rec_grad(const int4* __restrict__ tiles, const DevLight* __restrict__ lights,
                                                  const DevPatch* __restrict__ patches, const float* __restrict__ rec,
                                                  long long stride, const long long* __restrict__ rec_base,
                                                  float* __restrict__ bin_hist, const float* __restrict__ inv_sigma,
                                                  const float* __restrict__ colour, double* __restrict__ partials,
                                                  double* __restrict__ partials_col)
{
    constexpr int NA = RGB ? 9 : 6;
    __shared__ double sh[NA][256];
    const int4 ti = tiles[blockIdx.x];
    const DevLight& L = lights[ti.x];
    float* hist = (bin_hist != nullptr && (L.type == 1 || L.type == 2)) ? bin_hist + 1024 * (long long)ti.x : nullptr;
    double acc[NA];
#pragma unroll
    for (int c = 0; c < NA; ++c) acc[c] = 0.0;
    if (!L.invalid) {   // a rejected luminaire traced nothing, so its records are stale
        const long long base = rec_base[ti.x] + (long long)(uint32_t)ti.y;
        for (int i = threadIdx.x; i < ti.z; i += 256) {
            const long long j = base + i;
            float se = rec[10 * stride + j];
            if (RGB) {
                const float s_r = se, s_g = rec[13 * stride + j], s_b = rec[14 * stride + j];
                if (s_r == 0.0f && s_g == 0.0f && s_b == 0.0f) continue;   // no hit, or nothing to add
                const float phi = rec[9 * stride + j];
                se = (s_r * colour[3 * ti.x] + s_g * colour[3 * ti.x + 1]) + s_b * colour[3 * ti.x + 2];
                acc[6] += (double)(s_r * phi);
                acc[7] += (double)(s_g * phi);
                acc[8] += (double)(s_b * phi);
            } else if (se == 0.0f) {
                continue;   // no hit, or nothing to add
            }
            const V3 x1 = v3(rec[j], rec[stride + j], rec[2 * stride + j]);
            const V3 y = v3(rec[3 * stride + j], rec[4 * stride + j], rec[5 * stride + j]);
            const unsigned qf = __float_as_uint(rec[6 * stride + j]);
            const V3 nq = xyz(patches[qf & 0x7FFFFFFFu].n_rho);
            const V3 n1 = (qf >> 31) ? v3(-nq.x, -nq.y, -nq.z) : nq;
            const float phi_r = rec[9 * stride + j];
            float dl[6];
            first_hit_dlog(L, x1, y, n1, rec[7 * stride + j], rec[8 * stride + j], dl);
            float m2 = 0.0f;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const float cr = se * (phi_r * dl[c]);
                acc[c] += (double)cr;
                if (hist) {
                    const float z = cr * inv_sigma[6 * ti.x + c];
                    m2 = m2 + z * z;
                }
            }
            if (hist) {
                const int ebin = __float_as_int(rec[11 * stride + j]);
                if (ebin >= 0) atomicAdd(hist + ebin, m2 * rec[12 * stride + j]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NA; ++c) sh[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int c = 0; c < NA; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) partials[(long long)blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
    if (RGB && threadIdx.x >= 6 && threadIdx.x < 9)
        partials_col[(long long)blockIdx.x * 3 + threadIdx.x - 6] = sh[threadIdx.x][0];
}

// Per-texel area A_k from the patch table (binary search of texel_base).
__global__ void k_texel_area(const float* __restrict__ patch_area, const long long* __restrict__ base,
                             int n_patches, long long K, float* __restrict__ A)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += stride) {
        int lo = 0, hi = n_patches - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (base[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        A[k] = patch_area[lo];
    }
}

inline int nblocks(long long n, int b, int cap)
{
    long long x = (n + b - 1) / b;
    if (x > cap) x = cap;
    if (x < 1) x = 1;
    return (int)x;
}

// Persistent grid of one trace-kernel instance: as many waves as stay
// resident on n_cu CUs (its occupancy, queried once), no more than there are
// tiles or overflow-stack slots.
template <bool ADJ, bool STATS, int WPB, int LDS_D, int MODE>
void launch_persistent(const TraceArgs& a, int n_cu, hipStream_t st)
{
    static int per_cu = -1;
    if (per_cu < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<ADJ, STATS, WPB, LDS_D, MODE>, WPB * 64, 0) !=
                hipSuccess || nb < 1)
            nb = 1;
        per_cu = nb;
    }
    long long blocks = ((long long)a.n_tiles + WPB - 1) / WPB;
    blocks = std::min<long long>(blocks, (long long)n_cu * per_cu);
    blocks = std::min<long long>(blocks, a.gstack_waves / WPB);
    if (blocks < 1) blocks = 1;
    k_trace<ADJ, STATS, WPB, LDS_D, MODE><<<(unsigned)blocks, WPB * 64, 0, st>>>(a);
}

// Work tiles built on the device (the table the context otherwise builds on
// the host and uploads): light gl of a layout of Lj lights (si[gl].w) and
// local index l (si[gl].z) traces N = ppl / Lj + (l < ppl % Lj) paths in
// tiles of tp paths, lights in order.  One thread forms the per-light ranges
// (a prefix over the lights), then one thread per tile writes it.
__global__ void k_tile_ranges(const int4* __restrict__ si, int L, long long ppl, int tp, int2* __restrict__ range,
                              long long* __restrict__ npaths)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int acc = 0;
    for (int gl = 0; gl < L; ++gl) {
        const int4 s = si[gl];
        const long long n = ppl / s.w + ((long long)s.z < ppl % s.w ? 1 : 0);
        const int nt = (int)((n + tp - 1) / tp);
        range[gl] = make_int2(acc, acc + nt);
        npaths[gl] = n;
        acc += nt;
    }
}

__global__ void k_tile_fill(const int4* __restrict__ si, const int2* __restrict__ range,
                            const long long* __restrict__ npaths, int L, int tp, int n_tiles, int4* __restrict__ tiles)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    int lo = 0, hi = L - 1;   // the light whose range holds t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (range[mid].x <= t) lo = mid;
        else hi = mid - 1;
    }
    const long long f = (long long)(t - range[lo].x) * tp;
    const long long cnt = npaths[lo] - f < tp ? npaths[lo] - f : tp;
    tiles[t] = make_int4(lo, (int)(uint32_t)f, (int)cnt, si[lo].y);
}

__global__ void k_queue_reset(unsigned* __restrict__ q)
{
    if (threadIdx.x < 8) q[threadIdx.x] = 0u;
}

template <bool ADJ, int WPB, int MODE>
void launch_dir(const TraceArgs& a, int lds_depth, int n_cu, hipStream_t st)
{
    if (lds_depth == 16)
        launch_persistent<ADJ, false, WPB, 16, MODE>(a, n_cu, st);
    else
        launch_persistent<ADJ, false, WPB, 32, MODE>(a, n_cu, st);
}

template <bool ADJ, bool STATS, int WPB>
hipError_t launch_wpb(const TraceArgs& a, int lds_depth, int n_cu, hipStream_t st)
{
    if (a.tangent != nullptr && !ADJ && !STATS) {
        if (lds_depth == 16)
            launch_persistent<ADJ, STATS, WPB, 16, 5>(a, n_cu, st);
        else
            launch_persistent<ADJ, STATS, WPB, 32, 5>(a, n_cu, st);
    } else if (a.cone != nullptr && ADJ && !STATS) {
        if (lds_depth == 16)
            launch_persistent<ADJ, STATS, WPB, 16, 6>(a, n_cu, st);
        else
            launch_persistent<ADJ, STATS, WPB, 32, 6>(a, n_cu, st);
    } else if (a.rotvec && ADJ) {
        if (lds_depth == 16)
            launch_persistent<ADJ, STATS, WPB, 16, 4>(a, n_cu, st);
        else
            launch_persistent<ADJ, STATS, WPB, 32, 4>(a, n_cu, st);
    } else if (a.dir_order >= 0 && !STATS) {
        if constexpr (!STATS) {
            // the harmonic order as a compile-time constant: MODE 30 + order.
            // The directional adjoint holds 14 KB of LDS per wave, so a CU
            // fits 10 of its waves in two-wave blocks but 8 in four-wave ones.
            constexpr int DW = (ADJ && WPB == 4) ? 2 : WPB;
            switch (a.dir_order) {
                case 0: launch_dir<ADJ, DW, 30>(a, lds_depth, n_cu, st); break;
                case 1: launch_dir<ADJ, DW, 31>(a, lds_depth, n_cu, st); break;
                case 2: launch_dir<ADJ, DW, 32>(a, lds_depth, n_cu, st); break;
                default: launch_dir<ADJ, DW, 33>(a, lds_depth, n_cu, st); break;
            }
        }
    } else if (a.rgb && !STATS) {
        if constexpr (ADJ) {
            if (a.rec != nullptr) {
                if (lds_depth == 16)
                    launch_persistent<ADJ, STATS, WPB, 16, 8>(a, n_cu, st);
                else
                    launch_persistent<ADJ, STATS, WPB, 32, 8>(a, n_cu, st);
                return hipGetLastError();
            }
        }
        if (lds_depth == 16)
            launch_persistent<ADJ, STATS, WPB, 16, 2>(a, n_cu, st);
        else
            launch_persistent<ADJ, STATS, WPB, 32, 2>(a, n_cu, st);
    } else if (a.linear && !STATS) {
        if (lds_depth == 16)
            launch_persistent<ADJ, STATS, WPB, 16, 1>(a, n_cu, st);
        else
            launch_persistent<ADJ, STATS, WPB, 32, 1>(a, n_cu, st);
    } else if (ADJ && !STATS && a.rec != nullptr) {
        if constexpr (ADJ && !STATS) {
            if (lds_depth == 16)
                launch_persistent<ADJ, STATS, WPB, 16, 7>(a, n_cu, st);
            else
                launch_persistent<ADJ, STATS, WPB, 32, 7>(a, n_cu, st);
        }
    } else {
        if (lds_depth == 16)
            launch_persistent<ADJ, STATS, WPB, 16, 0>(a, n_cu, st);
        else
            launch_persistent<ADJ, STATS, WPB, 32, 0>(a, n_cu, st);
    }
    return hipGetLastError();
}

template <bool ADJ, bool STATS>
hipError_t launch_t(const TraceArgs& a, int wpb, int lds_depth, int n_cu, hipStream_t st)
{
    switch (wpb) {
        case 1: return launch_wpb<ADJ, STATS, 1>(a, lds_depth, n_cu, st);
        case 2: return launch_wpb<ADJ, STATS, 2>(a, lds_depth, n_cu, st);
        default: return launch_wpb<ADJ, STATS, 4>(a, lds_depth, n_cu, st);
    }
}

}  // namespace

hipError_t launch_trace(bool adjoint, bool stats, const TraceArgs& a, int waves_per_block, int lds_depth, int n_cu,
                        hipStream_t st)
{
    k_queue_reset<<<1, 64, 0, st>>>(a.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (adjoint) return launch_t<true, false>(a, waves_per_block, lds_depth, n_cu, st);
    if (stats) return launch_t<false, true>(a, waves_per_block, lds_depth, n_cu, st);
    return launch_t<false, false>(a, waves_per_block, lds_depth, n_cu, st);
}

hipError_t launch_build_tiles(const int4* si, int L, long long ppl, int tp, int n_tiles, int4* tiles, int2* range,
                              long long* npaths, hipStream_t st)
{
    k_tile_ranges<<<1, 64, 0, st>>>(si, L, ppl, tp, range, npaths);
    k_tile_fill<<<(n_tiles + 255) / 256, 256, 0, st>>>(si, range, npaths, L, tp, n_tiles, tiles);
    return hipGetLastError();
}

hipError_t launch_pt(bool adjoint, const PtArgs& a, int lds_depth, hipStream_t st)
{
    const int blocks = nblocks(a.K * a.M, 256, kPtBlocks);
    if (adjoint) {
        if (lds_depth == 16) k_pt<true, 16><<<blocks, 256, 0, st>>>(a);
        else k_pt<true, 32><<<blocks, 256, 0, st>>>(a);
    } else {
        if (lds_depth == 16) k_pt<false, 16><<<blocks, 256, 0, st>>>(a);
        else k_pt<false, 32><<<blocks, 256, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_fd_params(const float* p, int n, int idx, float h, float* pp, float* pm, double* den,
                            hipStream_t st)
{
    k_fd_params<<<(n + 255) / 256, 256, 0, st>>>(p, n, idx, h, pp, pm, den);
    return hipGetLastError();
}

hipError_t launch_fd_diff(const long long* Sp, const long long* Sm, long long K, const double* den, float* F,
                          hipStream_t st)
{
    k_fd_diff<<<nblocks(K, 256, 4096), 256, 0, st>>>(Sp, Sm, K, den, F);
    return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double* in, float* out, long long n, hipStream_t st)
{
    k_f64_to_f32<<<(int)((n + 255) / 256), 256, 0, st>>>(in, out, n);
    return hipGetLastError();
}

hipError_t launch_record(const RecordArgs& a, int lds_depth, hipStream_t st)
{
    const int blocks = nblocks(a.count, 256, kRecordBlocks);
    if (lds_depth == 16)
        k_record<16><<<blocks, 256, 0, st>>>(a);
    else
        k_record<32><<<blocks, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_light_setup(const float* params, const int4* si, const float4* sf, const long long* npaths,
                              int n_lights, DevLight* out, unsigned* flags, hipStream_t st, int rv, float* cone)
{
    k_light_setup<<<nblocks(n_lights, 64, 1 << 20), 64, 0, st>>>(params, si, sf, npaths, n_lights, out, flags, rv,
                                                                 cone);
    return hipGetLastError();
}

// per light: the seven partial sums of its tiles (FP64), the world-rotation
// components mapped to the rotation vector by J^T, written as f32
__global__ void __launch_bounds__(64) k_grad_reduce_rv(const double* __restrict__ partials,
                                                       const int2* __restrict__ range, const float* __restrict__ params,
                                                       int n_lights, float* __restrict__ grad)
{
    const int l = blockIdx.x;
    if (l >= n_lights) return;
    const int2 rg = range[l];
    double acc[7];
    for (int c = 0; c < 7; ++c) acc[c] = 0.0;
    for (int t = rg.x + (int)threadIdx.x; t < rg.y; t += 64)
        for (int c = 0; c < 7; ++c) acc[c] += partials[(long long)t * 7 + c];
    for (int c = 0; c < 7; ++c) acc[c] = wave_sum(acc[c]);
    if (threadIdx.x == 0) {
        double th[3] = {(double)params[7 * l + 3], (double)params[7 * l + 4], (double)params[7 * l + 5]};
        // a rejected luminaire (non-finite parameters) has zero partials; keep
        // its Jacobian finite so that its gradient row is zero, not NaN
        if (!(__builtin_isfinite(th[0]) && __builtin_isfinite(th[1]) && __builtin_isfinite(th[2])))
            th[0] = th[1] = th[2] = 0.0;
        double J[9];
        rot_jacobian_f64(th, J);
        grad[7 * l + 0] = (float)acc[0];
        grad[7 * l + 1] = (float)acc[1];
        grad[7 * l + 2] = (float)acc[2];
        for (int c = 0; c < 3; ++c) grad[7 * l + 3 + c] = (float)((J[c] * acc[3] + J[3 + c] * acc[4]) + J[6 + c] * acc[5]);
        grad[7 * l + 6] = (float)acc[6];
    }
}

// per light: the eight partial sums of its tiles (FP64) -> grad [L,6] and the
// cone-angle gradient [L,2]
__global__ void __launch_bounds__(64) k_grad_reduce_cone(const double* __restrict__ partials,
                                                         const int2* __restrict__ range, int n_lights,
                                                         float* __restrict__ grad, float* __restrict__ gcone)
{
    const int l = blockIdx.x;
    if (l >= n_lights) return;
    const int2 rg = range[l];
    double acc[8];
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    for (int t = rg.x + (int)threadIdx.x; t < rg.y; t += 64)
        for (int c = 0; c < 8; ++c) acc[c] += partials[(long long)t * 8 + c];
    for (int c = 0; c < 8; ++c) acc[c] = wave_sum(acc[c]);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 6; ++c) grad[6 * l + c] = (float)acc[c];
        gcone[2 * l] = (float)acc[6];
        gcone[2 * l + 1] = (float)acc[7];
    }
}

hipError_t launch_grad_reduce_cone(const double* partials, const int2* range, int n_lights, float* grad,
                                   float* gcone, hipStream_t st)
{
    k_grad_reduce_cone<<<n_lights, 64, 0, st>>>(partials, range, n_lights, grad, gcone);
    return hipGetLastError();
}

hipError_t launch_grad_reduce_rv(const double* partials, const int2* range, const float* params, int n_lights,
                                 float* grad, hipStream_t st)
{
    k_grad_reduce_rv<<<n_lights, 64, 0, st>>>(partials, range, params, n_lights, grad);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, long long n, float v, hipStream_t st)
{
    k_fill_f32<<<nblocks(n, 256, 4096), 256, 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_clear(long long* S, long long n, hipStream_t st)
{
    k_clear<<<nblocks(n / 2 + 1, 256, 4096), 256, 0, st>>>(S, n);
    return hipGetLastError();
}

hipError_t launch_finalize(const long long* S, float* E, long long n, unsigned* flags, hipStream_t st)
{
    k_finalize<<<nblocks(n / 2 + 1, 256, 4096), 256, 0, st>>>(S, E, n, flags);
    return hipGetLastError();
}

hipError_t launch_objective(const float* E, const float* Et, const float* alpha, const float* A, long long K,
                            long long n, float* g, double* partials, double* O, hipStream_t st)
{
    k_objective<<<kObjBlocks, 256, 0, st>>>(E, Et, alpha, A, K, n, g, partials);
    k_objective_final<<<1, 256, 0, st>>>(partials, kObjBlocks, O);
    return hipGetLastError();
}

hipError_t launch_rec_grad(const TraceArgs& a, double* partials, hipStream_t st)
{
    if (a.n_tiles > 0 && a.rgb)
        k_rec_grad<true><<<a.n_tiles, 256, 0, st>>>(a.tiles, a.lights, a.patches, a.rec, a.rec_stride, a.rec_base,
                                                    a.bin_hist, a.inv_sigma, a.colour, partials, a.partials_col);
    else if (a.n_tiles > 0)
        k_rec_grad<false><<<a.n_tiles, 256, 0, st>>>(a.tiles, a.lights, a.patches, a.rec, a.rec_stride, a.rec_base,
                                                     a.bin_hist, a.inv_sigma, nullptr, partials, nullptr);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double* partials, const int2* range, int n_lights, float* grad,
                              hipStream_t st)
{
    k_grad_reduce<6><<<n_lights, 64, 0, st>>>(partials, range, n_lights, grad);
    return hipGetLastError();
}

hipError_t launch_grad_reduce_col(const double* partials, const int2* range, int n_lights, float* grad,
                                  hipStream_t st)
{
    k_grad_reduce<3><<<n_lights, 64, 0, st>>>(partials, range, n_lights, grad);
    return hipGetLastError();
}

hipError_t launch_texel_area(const float* patch_area, const long long* base, int n_patches, long long K, float* A,
                             hipStream_t st)
{
    k_texel_area<<<nblocks(K, 256, 8192), 256, 0, st>>>(patch_area, base, n_patches, K, A);
    return hipGetLastError();
}

}  // namespace lt
