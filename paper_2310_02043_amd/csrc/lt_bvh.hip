// Linear BVH build on the device.
//
// The paper traces rays with the ray-tracing units of its GPU (Sec. 6); the
// MI355X has none, so the scene's acceleration structure is built here:
// 63-bit Morton codes of triangle centroids, a bitonic sort of (code, index),
// the binary radix tree of Karras (HPG 2012) with index tie-breaking, and
// bottom-up bounds.  Output nodes hold both child boxes inline (64 B, one
// fetch = two box tests); leaves are single triangles stored in Morton order
// as (v0, id), (v1 - v0, patch), (v2 - v0, 0).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <float.h>
#include "lt_device.h"
#include "lt_internal.h"

namespace lt {

namespace {

__global__ void k_tri_setup(const float* __restrict__ verts, const int* __restrict__ tris, int n, float pad,
                            float4* __restrict__ lo, float4* __restrict__ hi, float4* __restrict__ cen)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    float mn[3], mx[3], ce[3];
    for (int k = 0; k < 3; ++k) {
        const float va = verts[3 * a + k], vb = verts[3 * b + k], vc = verts[3 * c + k];
        mn[k] = fminf(va, fminf(vb, vc)) - pad;
        mx[k] = fmaxf(va, fmaxf(vb, vc)) + pad;
        ce[k] = 0.5f * (fminf(va, fminf(vb, vc)) + fmaxf(va, fmaxf(vb, vc)));
    }
    lo[t] = make_float4(mn[0], mn[1], mn[2], 0.f);
    hi[t] = make_float4(mx[0], mx[1], mx[2], 0.f);
    cen[t] = make_float4(ce[0], ce[1], ce[2], 0.f);
}

// block-level min/max of centroids -> partial[2*block] = (min, max)
__global__ void k_bounds_partial(const float4* __restrict__ cen, int n, float4* __restrict__ part)
{
    __shared__ float smn[3][256], smx[3][256];
    float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float4 c = cen[i];
        mn[0] = fminf(mn[0], c.x); mn[1] = fminf(mn[1], c.y); mn[2] = fminf(mn[2], c.z);
        mx[0] = fmaxf(mx[0], c.x); mx[1] = fmaxf(mx[1], c.y); mx[2] = fmaxf(mx[2], c.z);
    }
    for (int k = 0; k < 3; ++k) {
        smn[k][threadIdx.x] = mn[k];
        smx[k][threadIdx.x] = mx[k];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 3; ++k) {
                smn[k][threadIdx.x] = fminf(smn[k][threadIdx.x], smn[k][threadIdx.x + s]);
                smx[k][threadIdx.x] = fmaxf(smx[k][threadIdx.x], smx[k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = make_float4(smn[0][0], smn[1][0], smn[2][0], 0.f);
        part[2 * blockIdx.x + 1] = make_float4(smx[0][0], smx[1][0], smx[2][0], 0.f);
    }
}

__device__ __forceinline__ uint64_t spread21(uint64_t x)
{
    x &= 0x1FFFFFull;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ void k_morton(const float4* __restrict__ cen, int n, int n_pow2, const float4* __restrict__ part,
                         int n_part, uint64_t* __restrict__ keys, int* __restrict__ vals)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pow2) return;
    if (i >= n) {
        keys[i] = ~0ull;
        vals[i] = 0x7fffffff;
        return;
    }
    float mn[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, mx[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int b = 0; b < n_part; ++b) {
        const float4 a = part[2 * b], c = part[2 * b + 1];
        mn[0] = fminf(mn[0], a.x); mn[1] = fminf(mn[1], a.y); mn[2] = fminf(mn[2], a.z);
        mx[0] = fmaxf(mx[0], c.x); mx[1] = fmaxf(mx[1], c.y); mx[2] = fmaxf(mx[2], c.z);
    }
    const float4 c = cen[i];
    const float cc[3] = {c.x, c.y, c.z};
    uint64_t code = 0;
    for (int k = 0; k < 3; ++k) {
        const float ext = mx[k] - mn[k];
        float f = ext > 0.f ? (cc[k] - mn[k]) / ext : 0.5f;
        f = fminf(fmaxf(f, 0.f), 1.f);
        uint64_t q = (uint64_t)fminf(f * 2097152.0f, 2097151.0f);
        code |= spread21(q) << (2 - k);
    }
    keys[i] = code;
    vals[i] = i;
}

// one compare-exchange stage of a bitonic sort on (key, val) pairs
__global__ void k_bitonic(uint64_t* __restrict__ keys, int* __restrict__ vals, int n_pow2, int j, int k)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pow2) return;
    const int ixj = i ^ j;
    if (ixj <= i) return;
    const uint64_t ka = keys[i], kb = keys[ixj];
    const int va = vals[i], vb = vals[ixj];
    const bool a_gt_b = (ka > kb) || (ka == kb && va > vb);
    const bool up = (i & k) == 0;
    if (a_gt_b == up) {
        keys[i] = kb; keys[ixj] = ka;
        vals[i] = vb; vals[ixj] = va;
    }
}

// common prefix length of sorted keys i and j (index tie-break), -1 outside
__device__ __forceinline__ int delta(const uint64_t* keys, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint64_t a = keys[i], b = keys[j];
    if (a != b) return __clzll((long long)(a ^ b));
    return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}

// Karras 2012: internal node i covers a key range; children are internal
// nodes or leaves (encoded as ~leaf).
__global__ void k_hierarchy(const uint64_t* __restrict__ keys, int n, int2* __restrict__ child,
                            int* __restrict__ parent_int, int* __restrict__ parent_leaf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(keys, n, i, i - d);
    int lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta(keys, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + (d < 0 ? d : 0);
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    int left, right;
    if (lo == gamma) {
        left = ~gamma;
        parent_leaf[gamma] = i;
    } else {
        left = gamma;
        parent_int[gamma] = i;
    }
    if (hi == gamma + 1) {
        right = ~(gamma + 1);
        parent_leaf[gamma + 1] = i;
    } else {
        right = gamma + 1;
        parent_int[gamma + 1] = i;
    }
    child[i] = make_int2(left, right);
}

__device__ __forceinline__ void child_box(int c, const float4* tlo, const float4* thi, const int* vals,
                                          const float4* nlo, const float4* nhi, float4& lo, float4& hi)
{
    if (c < 0) {
        const int t = vals[~c];
        lo = tlo[t];
        hi = thi[t];
    } else {
        lo = nlo[c];
        hi = nhi[c];
    }
}

// bottom-up bounds: the second thread to reach a node computes its box
__global__ void k_bounds_up(int n, const int2* __restrict__ child, const int* __restrict__ parent_int,
                            const int* __restrict__ parent_leaf, const int* __restrict__ vals,
                            const float4* __restrict__ tlo, const float4* __restrict__ thi, float4* nlo, float4* nhi,
                            int* flags)
{
    const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
    if (leaf >= n) return;
    int node = parent_leaf[leaf];
    while (node >= 0) {
        const int prev = __hip_atomic_fetch_add(&flags[node], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == 0) return;
        const int2 c = child[node];
        float4 al, ah, bl, bh;
        child_box(c.x, tlo, thi, vals, nlo, nhi, al, ah);
        child_box(c.y, tlo, thi, vals, nlo, nhi, bl, bh);
        nlo[node] = make_float4(fminf(al.x, bl.x), fminf(al.y, bl.y), fminf(al.z, bl.z), 0.f);
        nhi[node] = make_float4(fmaxf(ah.x, bh.x), fmaxf(ah.y, bh.y), fmaxf(ah.z, bh.z), 0.f);
        __atomic_thread_fence(__ATOMIC_RELEASE);
        node = node == 0 ? -1 : parent_int[node];
    }
}

__global__ void k_write_nodes(int n_int, const int2* __restrict__ child, const int* __restrict__ vals,
                              const float4* __restrict__ tlo, const float4* __restrict__ thi,
                              const float4* __restrict__ nlo, const float4* __restrict__ nhi,
                              float4* __restrict__ nodes)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_int) return;
    const int2 c = child[i];
    float4 al, ah, bl, bh;
    child_box(c.x, tlo, thi, vals, nlo, nhi, al, ah);
    child_box(c.y, tlo, thi, vals, nlo, nhi, bl, bh);
    nodes[4 * i + 0] = make_float4(al.x, ah.x, al.y, ah.y);
    nodes[4 * i + 1] = make_float4(bl.x, bh.x, bl.y, bh.y);
    nodes[4 * i + 2] = make_float4(al.z, ah.z, bl.z, bh.z);
    nodes[4 * i + 3] = make_float4(__int_as_float(c.x), __int_as_float(c.y), 0.f, 0.f);
}

__global__ void k_write_tris(int n, const int* __restrict__ vals, const float* __restrict__ verts,
                             const int* __restrict__ tris, const int* __restrict__ tri_patch,
                             float4* __restrict__ out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int t = vals[s];
    const int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    const float v0x = verts[3 * a], v0y = verts[3 * a + 1], v0z = verts[3 * a + 2];
    out[3 * s + 0] = make_float4(v0x, v0y, v0z, __int_as_float(t));
    out[3 * s + 1] = make_float4(verts[3 * b] - v0x, verts[3 * b + 1] - v0y, verts[3 * b + 2] - v0z,
                                 __int_as_float(tri_patch[t]));
    out[3 * s + 2] = make_float4(verts[3 * c] - v0x, verts[3 * c + 1] - v0y, verts[3 * c + 2] - v0z, 0.f);
}

// depth of every leaf (internal nodes on its root path) -> max
__global__ void k_depth(int n, const int* __restrict__ parent_int, const int* __restrict__ parent_leaf,
                        int* __restrict__ out)
{
    const int leaf = blockIdx.x * blockDim.x + threadIdx.x;
    if (leaf >= n) return;
    int d = 0;
    int node = parent_leaf[leaf];
    while (node >= 0 && d < (1 << 20)) {
        ++d;
        node = node == 0 ? -1 : parent_int[node];
    }
    atomicMax(out, d);
}

inline int blocks_for(long long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

// Builds nodes [max(n-1,1) * 4 float4] and leaf triangles [n * 3 float4].
// Device inputs: d_verts [V*3], d_tris [n*3], d_tri_patch [n].
hipError_t build_bvh(const float* d_verts, const int* d_tris, const int* d_tri_patch, int n, float pad,
                     hipStream_t st, float4** nodes_out, float4** tris_out, int* n_nodes_out, int* depth_out)
{
    *nodes_out = nullptr;
    *tris_out = nullptr;
    if (n < 1) return hipErrorInvalidValue;
    int n_pow2 = 1;
    while (n_pow2 < n) n_pow2 <<= 1;
    const int n_int = n - 1 > 0 ? n - 1 : 1;
    const int n_part = 256;
    float4 *tlo = nullptr, *thi = nullptr, *cen = nullptr, *part = nullptr, *nlo = nullptr, *nhi = nullptr;
    uint64_t* keys = nullptr;
    int *vals = nullptr, *pint = nullptr, *pleaf = nullptr, *flags = nullptr, *dmax = nullptr;
    int2* child = nullptr;
    float4 *nodes = nullptr, *otris = nullptr;
    const int2 single_leaf = make_int2(~0, ~0);
    hipError_t e = hipSuccess;
#define LT_TRY(x)                          \
    do {                                   \
        e = (x);                           \
        if (e != hipSuccess) goto cleanup; \
    } while (0)
    LT_TRY(hipMalloc(&tlo, sizeof(float4) * n));
    LT_TRY(hipMalloc(&thi, sizeof(float4) * n));
    LT_TRY(hipMalloc(&cen, sizeof(float4) * n));
    LT_TRY(hipMalloc(&part, sizeof(float4) * 2 * n_part));
    LT_TRY(hipMalloc(&keys, sizeof(uint64_t) * n_pow2));
    LT_TRY(hipMalloc(&vals, sizeof(int) * n_pow2));
    LT_TRY(hipMalloc(&child, sizeof(int2) * n_int));
    LT_TRY(hipMalloc(&pint, sizeof(int) * n_int));
    LT_TRY(hipMalloc(&pleaf, sizeof(int) * n));
    LT_TRY(hipMalloc(&flags, sizeof(int) * n_int));
    LT_TRY(hipMalloc(&nlo, sizeof(float4) * n_int));
    LT_TRY(hipMalloc(&nhi, sizeof(float4) * n_int));
    LT_TRY(hipMalloc(&dmax, sizeof(int)));
    LT_TRY(hipMalloc(&nodes, sizeof(float4) * 4 * n_int));
    LT_TRY(hipMalloc(&otris, sizeof(float4) * 3 * n));

    k_tri_setup<<<blocks_for(n, 256), 256, 0, st>>>(d_verts, d_tris, n, pad, tlo, thi, cen);
    k_bounds_partial<<<n_part, 256, 0, st>>>(cen, n, part);
    k_morton<<<blocks_for(n_pow2, 256), 256, 0, st>>>(cen, n, n_pow2, part, n_part, keys, vals);
    for (int k = 2; k <= n_pow2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1)
            k_bitonic<<<blocks_for(n_pow2, 256), 256, 0, st>>>(keys, vals, n_pow2, j, k);
    LT_TRY(hipGetLastError());
    if (n == 1) {
        // a single triangle: one node whose two children are that leaf
        LT_TRY(hipMemcpyAsync(child, &single_leaf, sizeof(int2), hipMemcpyHostToDevice, st));
        LT_TRY(hipMemsetAsync(pleaf, 0, sizeof(int), st));
    } else {
        k_hierarchy<<<blocks_for(n - 1, 256), 256, 0, st>>>(keys, n, child, pint, pleaf);
        LT_TRY(hipMemsetAsync(flags, 0, sizeof(int) * n_int, st));
        k_bounds_up<<<blocks_for(n, 256), 256, 0, st>>>(n, child, pint, pleaf, vals, tlo, thi, nlo, nhi, flags);
    }
    k_write_nodes<<<blocks_for(n_int, 256), 256, 0, st>>>(n_int, child, vals, tlo, thi, nlo, nhi, nodes);
    k_write_tris<<<blocks_for(n, 256), 256, 0, st>>>(n, vals, d_verts, d_tris, d_tri_patch, otris);
    LT_TRY(hipMemsetAsync(dmax, 0, sizeof(int), st));
    if (n > 1) k_depth<<<blocks_for(n, 256), 256, 0, st>>>(n, pint, pleaf, dmax);
    LT_TRY(hipGetLastError());
    LT_TRY(hipMemcpyAsync(depth_out, dmax, sizeof(int), hipMemcpyDeviceToHost, st));
    LT_TRY(hipStreamSynchronize(st));
    if (n == 1) *depth_out = 1;
    *nodes_out = nodes;
    *tris_out = otris;
    *n_nodes_out = n_int;
    nodes = nullptr;
    otris = nullptr;
cleanup:
    hipFree(tlo); hipFree(thi); hipFree(cen); hipFree(part); hipFree(keys); hipFree(vals);
    hipFree(child); hipFree(pint); hipFree(pleaf); hipFree(flags); hipFree(nlo); hipFree(nhi);
    hipFree(dmax); hipFree(nodes); hipFree(otris);
#undef LT_TRY
    return e;
}

}  // namespace lt
