// Device-side building blocks of the light-tracing kernels (gfx950).
//
// Arithmetic contract (shared by specification with the test oracle, not by
// code): all path arithmetic is FP32 with this translation unit compiled
// without FP contraction, IEEE division and square root; dot products are
// (a.x*b.x + a.y*b.y) + a.z*b.z; transcendentals are the polynomials below.
// This makes the primal and adjoint passes replay bit-identical paths.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lt {

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                       uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// top 24 bits -> [0, 1 - 2^-24]
__device__ __forceinline__ float u24(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------
// Transcendentals of the contract.
// ---------------------------------------------------------------------------
// sin/cos(2 pi u): quadrant q = rint(4u), x = (4u - q) pi/2, Taylor in x^2.
__device__ __forceinline__ void sincos_2pi(float u, float& s_out, float& c_out)
{
    const float half_pi = (float)1.57079632679489661923;
    const float q4 = u * 4.0f;
    const float qf = __builtin_rintf(q4);
    const float x = (q4 - qf) * half_pi;
    const float z = x * x;
    float sp = (float)(1.0 / 362880.0);
    sp = sp * z + (float)(-1.0 / 5040.0);
    sp = sp * z + (float)(1.0 / 120.0);
    sp = sp * z + (float)(-1.0 / 6.0);
    sp = sp * z;
    const float sn = x + x * sp;
    float cp = (float)(1.0 / 3628800.0);
    cp = cp * z + (float)(-1.0 / 40320.0);
    cp = cp * z + (float)(1.0 / 720.0);
    cp = cp * z + (float)(-1.0 / 24.0);
    cp = cp * z + 0.5f;
    const float cs = 1.0f - cp * z;
    const int q = ((int)qf) & 3;
    // rotate (cos, sin) by q quarter turns
    const float s1 = (q & 1) ? cs : sn;
    const float c1 = (q & 1) ? sn : cs;
    s_out = (q & 2) ? -s1 : s1;
    c_out = ((q + 1) & 2) ? -c1 : c1;
}

// log2 for positive normal floats: mantissa in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh((m-1)/(m+1)) as an odd series to s^11.
__device__ __forceinline__ float log2_c(float x)
{
    int e;
    float m = __builtin_frexpf(x, &e);
    if (m < (float)0.70710678118654752440) {
        m = m * 2.0f;
        e = e - 1;
    }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float p = (float)(1.0 / 11.0);
    p = p * z + (float)(1.0 / 9.0);
    p = p * z + (float)(1.0 / 7.0);
    p = p * z + (float)(1.0 / 5.0);
    p = p * z + (float)(1.0 / 3.0);
    p = p * z;
    const float a = s + s * p;
    return (float)e + (a + a) * (float)1.44269504088896340736;
}

// 2^y: integer part by rint, fraction via Taylor of e^(f ln 2) to degree 7.
__device__ __forceinline__ float exp2_c(float y)
{
    const float k = __builtin_rintf(y);
    const float z = (y - k) * (float)0.69314718055994530942;
    float p = (float)(1.0 / 5040.0);
    p = p * z + (float)(1.0 / 720.0);
    p = p * z + (float)(1.0 / 120.0);
    p = p * z + (float)(1.0 / 24.0);
    p = p * z + (float)(1.0 / 6.0);
    p = p * z + 0.5f;
    p = p * z + 1.0f;
    p = p * z + 1.0f;
    return __builtin_ldexpf(p, (int)k);
}

// FP64 sin/cos of any angle (luminaire frames only): Cody-Waite reduction
// by pi/2 = P1 + P2, Taylor to r^17 / r^18.
__device__ __forceinline__ void sincos_f64(double x, double& s_out, double& c_out)
{
    const double k = __builtin_rint(x * 6.36619772367581382433e-01);
    const double r = (x - k * 1.57079632673412561417e+00) - k * 6.07710050650619224932e-11;
    const double z = r * r;
    double sp = -1.0 / 355687428096000.0;
    sp = sp * z + 1.0 / 1307674368000.0;
    sp = sp * z - 1.0 / 6227020800.0;
    sp = sp * z + 1.0 / 39916800.0;
    sp = sp * z - 1.0 / 362880.0;
    sp = sp * z + 1.0 / 5040.0;
    sp = sp * z - 1.0 / 120.0;
    sp = sp * z + 1.0 / 6.0;
    const double sn = r - r * (z * sp);
    double cp = 1.0 / 6402373705728000.0;
    cp = cp * z - 1.0 / 20922789888000.0;
    cp = cp * z + 1.0 / 87178291200.0;
    cp = cp * z - 1.0 / 479001600.0;
    cp = cp * z + 1.0 / 3628800.0;
    cp = cp * z - 1.0 / 40320.0;
    cp = cp * z + 1.0 / 720.0;
    cp = cp * z - 1.0 / 24.0;
    cp = cp * z + 0.5;
    const double cs = 1.0 - z * cp;
    const int q = (int)(((long long)k) & 3);
    const double s1 = (q & 1) ? cs : sn;
    const double c1 = (q & 1) ? sn : cs;
    s_out = (q & 2) ? -s1 : s1;
    c_out = ((q + 1) & 2) ? -c1 : c1;
}

// ---------------------------------------------------------------------------
// Small vector helpers with the contract's evaluation order.
// ---------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 xyz(float4 v) { return V3{v.x, v.y, v.z}; }

// ---------------------------------------------------------------------------
// Data layouts in HBM.
// ---------------------------------------------------------------------------
// BVH node of the 4-wide tree, 64 B = 4 rows of 16 B, slots ordered internal
// children, leaves, unused: per axis x, y, z the four slots' lower then upper
// planes as f16 offsets from the node origin (rounded outward; unused slots
// +inf / -inf); then the origin as bf16 x, y, z, the slot counts (internal |
// leaves << 4), the first internal child's node index and the first leaf's
// triangle slot (a node's children and its leaf triangles are consecutive).
// Triangle, 48 B: (v0, original id), (e1 = v1 - v0, patch), (e2 = v2 - v0, 0).

// Patch record, 80 B.
struct DevPatch {
    float4 o_inva;   // origin, 1/A_k
    float4 eu_ilu;   // e_u, 1/|e_u|^2
    float4 ev_ilv;   // e_v, 1/|e_v|^2
    float4 n_rho;    // normal, albedo
    int res_u, res_v;
    long long base;
};

// Luminaire record after per-call setup (frame, derivatives, flux per ray).
struct DevLight {
    float c[3], d[3], t[3], b[3];
    float dd_da[3], dd_db[3], dt_db[3], db_da[3], db_db[3];
    float P, phi_r, n, w, h;
    int type, layout, l_local;
    float kcap;  // soft-edged spot: flux scale of cap sampling (1 otherwise)
    long long n_paths;
    int invalid;  // parameters not finite or power not positive: the light adds nothing
    int pad1;
};  // 160 B

// Moeller-Trumbore with the contract's order; barycentric bounds widened by
// 2^-20; accepts t > 0 improving (t, prim) lexicographically.
__device__ __forceinline__ void tri_test(const float4 A, const float4 B, const float4 C, V3 o, V3 d, int skip,
                                         float& tb, int& pb, int& qb)
{
    const int prim = __float_as_int(A.w);
    const int patch = __float_as_int(B.w);
    if (patch == skip) return;
    const V3 v0 = xyz(A), e1 = xyz(B), e2 = xyz(C);
    const V3 p = cross(d, e2);
    const float det = dot(e1, p);
    if (det == 0.0f) return;
    const float inv = 1.0f / det;
    const V3 s = sub(o, v0);
    const float u = dot(s, p) * inv;
    const float eps = 0x1p-20f;
    if (u < -eps || u > 1.0f + eps) return;
    const V3 q = cross(s, e1);
    const float v = dot(d, q) * inv;
    if (v < -eps || u + v > 1.0f + eps) return;
    const float t = dot(e2, q) * inv;
    if (!(t > 0.0f)) return;
    if (t < tb || (t == tb && prim < pb)) {
        tb = t;
        pb = prim;
        qb = patch;
    }
}

}  // namespace lt
