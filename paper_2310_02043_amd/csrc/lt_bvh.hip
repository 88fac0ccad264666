// BVH build on the device.
//
// The paper traces rays with the ray-tracing units of its GPU (Sec. 6); the
// MI355X has none, so the scene's acceleration structure is built here:
// 63-bit Morton codes of triangle centroids, a bitonic sort of (code, index),
// then parallel locally-ordered clustering (PLOC, Meister and Bittner 2018):
// every cluster finds its nearest neighbour (smallest merged surface area)
// within a window of the Morton order, mutual nearest neighbours merge, the
// cluster list is compacted by a prefix sum, until one cluster is left.
// Internal nodes are numbered from the root (0) in reverse creation order.
// The binary tree is collapsed into a 4-wide tree whose nodes keep the four
// child boxes as f16 offsets from a node origin (64 B, four loads per node
// step); leaves are single triangles, stored so that the leaves of each wide
// node are consecutive, as (v0, id), (v1 - v0, patch), (v2 - v0, 0).
#include <hip/hip_runtime.h>
#include <utility>
#include <vector>
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

// ---- PLOC -------------------------------------------------------------------
__device__ __forceinline__ float half_area(float4 lo, float4 hi)
{
    const float dx = hi.x - lo.x, dy = hi.y - lo.y, dz = hi.z - lo.z;
    return dx * dy + dy * dz + dz * dx;
}

__global__ void k_ploc_init(int n, const int* __restrict__ vals, const float4* __restrict__ tlo,
                            const float4* __restrict__ thi, int* __restrict__ cid, float4* __restrict__ clo,
                            float4* __restrict__ chi)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int t = vals[s];
    cid[s] = ~s;
    clo[s] = tlo[t];
    chi[s] = thi[t];
}

// nearest neighbour within [i-R, i+R] by merged half surface area (ties: lower index)
__global__ void k_ploc_nn(int nc, int R, const float4* __restrict__ clo, const float4* __restrict__ chi,
                          int* __restrict__ nn)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const float4 a = clo[i], b = chi[i];
    const int j0 = i - R < 0 ? 0 : i - R;
    const int j1 = i + R > nc - 1 ? nc - 1 : i + R;
    float best = __builtin_inff();
    int bj = -1;
    for (int j = j0; j <= j1; ++j) {
        if (j == i) continue;
        const float4 c = clo[j], d = chi[j];
        const float ha = half_area(make_float4(fminf(a.x, c.x), fminf(a.y, c.y), fminf(a.z, c.z), 0.f),
                                   make_float4(fmaxf(b.x, d.x), fmaxf(b.y, d.y), fmaxf(b.z, d.z), 0.f));
        if (ha < best) {
            best = ha;
            bj = j;
        }
    }
    nn[i] = bj;
}

// flag = keep << 32 | merge  (mutual pair: the lower index keeps and merges)
__global__ void k_ploc_flags(int nc, const int* __restrict__ nn, unsigned long long* __restrict__ flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const int j = nn[i];
    const bool mutual = j >= 0 && nn[j] == i;
    const unsigned long long keep = (mutual && i > j) ? 0ull : 1ull;
    const unsigned long long merge = (mutual && i < j) ? 1ull : 0ull;
    flags[i] = (keep << 32) | merge;
}

__global__ void k_ploc_write(int nc, int n_int, int node_base, const int* __restrict__ nn,
                             const unsigned long long* __restrict__ flags, const unsigned long long* __restrict__ scan,
                             const int* __restrict__ cid, const float4* __restrict__ clo,
                             const float4* __restrict__ chi, int* __restrict__ oid, float4* __restrict__ olo,
                             float4* __restrict__ ohi, int2* __restrict__ child, float4* __restrict__ nlo,
                             float4* __restrict__ nhi, int* __restrict__ parent_int, int* __restrict__ parent_leaf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const unsigned long long f = flags[i];
    if (!(f >> 32)) return;
    const int p = (int)(scan[i] >> 32);
    if (f & 1ull) {
        const int j = nn[i];
        const int node = n_int - 1 - (node_base + (int)(scan[i] & 0xffffffffull));
        const int ca = cid[i], cb = cid[j];
        child[node] = make_int2(ca, cb);
        if (ca >= 0) parent_int[ca] = node;
        else parent_leaf[~ca] = node;
        if (cb >= 0) parent_int[cb] = node;
        else parent_leaf[~cb] = node;
        const float4 a = clo[i], b = chi[i], c = clo[j], d = chi[j];
        const float4 ul = make_float4(fminf(a.x, c.x), fminf(a.y, c.y), fminf(a.z, c.z), 0.f);
        const float4 uh = make_float4(fmaxf(b.x, d.x), fmaxf(b.y, d.y), fmaxf(b.z, d.z), 0.f);
        nlo[node] = ul;
        nhi[node] = uh;
        oid[p] = node;
        olo[p] = ul;
        ohi[p] = uh;
    } else {
        oid[p] = cid[i];
        olo[p] = clo[i];
        ohi[p] = chi[i];
    }
}

// ---- collapse of the binary tree into a 4-wide tree ------------------------
// Node of the wide tree, 64 B = 4 rows of 16 B (kNodeRows).  Its slots hold
// the internal children first, then the leaves, then unused slots.  Rows 0-2:
// for x, y and z the four slots' lower planes then their upper planes as f16
// offsets from the node origin, rounded outward (lower down, upper up) so
// that the stored box contains the child's box; unused slots hold +inf /
// -inf, a box no slab test hits.  Row 3: the origin as bf16 x, y, z (rounded
// down, at or below every child box; x | y << 16, then z | counts << 16 with
// counts = internal children | leaves << 4), the index of the first internal
// child (the others follow it), the slot of the first leaf triangle (the
// others follow it).
__device__ __forceinline__ void ref_box(int c, const float4* nlo, const float4* nhi, const int* vals,
                                        const float4* tlo, const float4* thi, float4& lo, float4& hi)
{
    if (c >= 0) {
        lo = nlo[c];
        hi = nhi[c];
    } else {
        const int t = vals[~c];
        lo = tlo[t];
        hi = thi[t];
    }
}

// Cost-optimal collapse of the binary tree into the 4-wide tree (the
// dynamic programme of Ylitie, Karras and Laine 2017 for four children).
// D(n, i) is the least surface-area cost of representing the subtree of n with
// at most i child slots of its wide parent: a leaf costs A(leaf) * kCostTri
// whatever i; D(n, 1) makes n a wide node, A(n) * kCostNode plus the best
// split of its four slots between its two binary children; D(n, i > 1) takes
// the better of D(n, i - 1) and the best split of i slots.  dp[n] holds
// D(n, 1..4); dec[n] holds the split of the wide node (bits 0..7) and of
// i = 2, 3, 4 slots (bits 8 (i - 1) .. 8 (i - 1) + 7; 0 = use i - 1 slots).
constexpr float kCostNode = 1.0f;
constexpr float kCostTri = 1.0f;

__device__ __forceinline__ void dp_of(int c, const float4* __restrict__ dp, const int* __restrict__ vals,
                                      const float4* __restrict__ tlo, const float4* __restrict__ thi, float d[4])
{
    if (c < 0) {
        const int t = vals[~c];
        const float a = half_area(tlo[t], thi[t]) * kCostTri;
        d[0] = d[1] = d[2] = d[3] = a;
    } else {
        const float4 v = dp[c];
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
    }
}

// Binary nodes [lo, hi) were all created in one merge round, after their
// children, so rounds are evaluated in creation order.
__global__ void k_collapse_dp(int lo, int hi, const int2* __restrict__ child, const float4* __restrict__ nlo,
                              const float4* __restrict__ nhi, const int* __restrict__ vals,
                              const float4* __restrict__ tlo, const float4* __restrict__ thi,
                              float4* __restrict__ dp, int* __restrict__ dec)
{
    const int n = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= hi) return;
    const int2 ch = child[n];
    float L[4], R[4];
    dp_of(ch.x, dp, vals, tlo, thi, L);
    dp_of(ch.y, dp, vals, tlo, thi, R);
    float bw = __builtin_inff();
    int kw = 1;
    for (int k = 1; k <= 3; ++k) {
        const float c = L[k - 1] + R[3 - k];
        if (c < bw) {
            bw = c;
            kw = k;
        }
    }
    float D[4];
    int code = kw;
    D[0] = half_area(nlo[n], nhi[n]) * kCostNode + bw;
    for (int i = 2; i <= 4; ++i) {
        float sb = __builtin_inff();
        int kb = 1;
        for (int k = 1; k < i; ++k) {
            const float c = L[k - 1] + R[i - k - 1];
            if (c < sb) {
                sb = c;
                kb = k;
            }
        }
        if (sb < D[i - 2]) {
            D[i - 1] = sb;
            code |= kb << (8 * (i - 1));
        } else {
            D[i - 1] = D[i - 2];
        }
    }
    dp[n] = make_float4(D[0], D[1], D[2], D[3]);
    dec[n] = code;
}

// Children of the wide node rooted at each level node: its four slots are
// distributed over binary descendants by the recorded decisions.
__global__ void k_collapse_open(int n_level, const int* __restrict__ level, const int2* __restrict__ child,
                                const int* __restrict__ dec, int* __restrict__ kids,
                                unsigned long long* __restrict__ cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_level) return;
    const int root = level[i];
    const int2 c0 = child[root];
    const int kw = dec[root] & 0xff;
    // (node, slots) pairs; their slots sum to at most 4, each at least 1
    int sn[4], ss[4], top = 0;
    sn[top] = c0.y; ss[top] = 4 - kw; ++top;
    sn[top] = c0.x; ss[top] = kw; ++top;
    int k[4] = {kEmptyChild, kEmptyChild, kEmptyChild, kEmptyChild};
    int m = 0;
    while (top > 0) {
        --top;
        const int c = sn[top], s = ss[top];
        if (c < 0 || s == 1) {
            if (m < 4) k[m++] = c;
            continue;
        }
        int d = (dec[c] >> (8 * (s - 1))) & 0xff;
        if (d >= s) d = 0;   // (never recorded: every split leaves each side a slot)
        if (d == 0) {
            sn[top] = c; ss[top] = s - 1; ++top;
        } else {
            const int2 cc = child[c];
            sn[top] = cc.y; ss[top] = s - d; ++top;
            sn[top] = cc.x; ss[top] = d; ++top;
        }
    }
    unsigned long long n_int = 0, n_leaf = 0;
    for (int q = 0; q < 4; ++q) {
        kids[4 * i + q] = k[q];
        n_int += (k[q] >= 0) ? 1ull : 0ull;
        n_leaf += (k[q] < 0 && k[q] != kEmptyChild) ? 1ull : 0ull;
    }
    cnt[i] = n_int | (n_leaf << 32);   // the prefix sum adds both halves
}

// Conservative conversions of a non-negative offset to f16: the largest f16
// not above x, and the smallest not below it (offsets beyond the f16 range
// become 65504 and +inf).
__device__ __forceinline__ unsigned short f16_down(double x)
{
    _Float16 h = (_Float16)(float)x;
    unsigned short b = __builtin_bit_cast(unsigned short, h);
    while ((double)__builtin_bit_cast(_Float16, b) > x) --b;   // x >= 0: positive encodings step down by one
    return b;
}

__device__ __forceinline__ unsigned short f16_up(double x)
{
    _Float16 h = (_Float16)(float)x;
    unsigned short b = __builtin_bit_cast(unsigned short, h);
    while ((double)__builtin_bit_cast(_Float16, b) < x) ++b;   // up to 0x7C00 = +inf
    return b;
}

__device__ __forceinline__ unsigned pack_f16(unsigned short a, unsigned short b)
{
    return (unsigned)a | ((unsigned)b << 16);
}

// The largest bf16 not above x (x finite): the upper half of its bits, one
// step further from zero for a negative x with a non-zero lower half.
__device__ __forceinline__ unsigned short bf16_down(float x)
{
    const unsigned u = __float_as_uint(x);
    unsigned short b = (unsigned short)(u >> 16);
    if ((int)u < 0 && (u & 0xFFFFu) != 0u) ++b;
    return b;
}

// Write the wide nodes of a level; internal children become the next level
// (from next_base + the node's internal-child offset), leaves take the
// triangle slots from leaf_base + the node's leaf offset (leaf_order[slot] =
// the leaf's Morton position).
__global__ void k_collapse_write(int n_level, int out_base, int next_base, int leaf_base, const int* __restrict__ kids,
                                 const unsigned long long* __restrict__ off, const float4* __restrict__ nlo,
                                 const float4* __restrict__ nhi, const int* __restrict__ vals,
                                 const float4* __restrict__ tlo, const float4* __restrict__ thi,
                                 float4* __restrict__ wide, int* __restrict__ next_level, int* __restrict__ leaf_order)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_level) return;
    const int ibase = (int)(off[i] & 0xffffffffull), lbase = (int)(off[i] >> 32);
    // slot order: internal children, leaves, unused
    int ord[4];
    int no = 0;
    for (int q = 0; q < 4; ++q)
        if (kids[4 * i + q] >= 0) ord[no++] = kids[4 * i + q];
    const int ni = no;
    for (int q = 0; q < 4; ++q) {
        const int c = kids[4 * i + q];
        if (c < 0 && c != kEmptyChild) ord[no++] = c;
    }
    const int nl = no - ni;
    while (no < 4) ord[no++] = kEmptyChild;
    float lo3[4][3], hi3[4][3];
    for (int q = 0; q < 4; ++q) {
        if (ord[q] == kEmptyChild) continue;
        float4 lo, hi;
        ref_box(ord[q], nlo, nhi, vals, tlo, thi, lo, hi);
        lo3[q][0] = lo.x; lo3[q][1] = lo.y; lo3[q][2] = lo.z;
        hi3[q][0] = hi.x; hi3[q][1] = hi.y; hi3[q][2] = hi.z;
    }
    for (int r = 0; r < ni; ++r) next_level[ibase + r] = ord[r];
    for (int j = 0; j < nl; ++j) leaf_order[leaf_base + lbase + j] = ~ord[ni + j];
    // origin: the least lower bound over the used slots, rounded down to bf16
    unsigned short ob[3];
    float o[3];
    for (int k = 0; k < 3; ++k) {
        float m = __builtin_inff();
        for (int q = 0; q < ni + nl; ++q) m = fminf(m, lo3[q][k]);
        if (m == __builtin_inff()) m = 0.0f;
        ob[k] = bf16_down(m);
        o[k] = __uint_as_float((unsigned)ob[k] << 16);
    }
    unsigned short ql[3][4], qh[3][4];
    for (int q = 0; q < 4; ++q)
        for (int k = 0; k < 3; ++k) {
            if (q >= ni + nl) {
                ql[k][q] = 0x7C00;   // +inf
                qh[k][q] = 0xFC00;   // -inf
            } else {
                ql[k][q] = f16_down((double)lo3[q][k] - (double)o[k]);
                qh[k][q] = f16_up((double)hi3[q][k] - (double)o[k]);
            }
        }
    float4* nd = wide + kNodeRows * (size_t)(out_base + i);
    for (int k = 0; k < 3; ++k)
        nd[k] = make_float4(__uint_as_float(pack_f16(ql[k][0], ql[k][1])), __uint_as_float(pack_f16(ql[k][2], ql[k][3])),
                            __uint_as_float(pack_f16(qh[k][0], qh[k][1])), __uint_as_float(pack_f16(qh[k][2], qh[k][3])));
    const unsigned counts = (unsigned)ni | ((unsigned)nl << 4);
    nd[3] = make_float4(__uint_as_float(pack_f16(ob[0], ob[1])), __uint_as_float(pack_f16(ob[2], (unsigned short)counts)),
                        __int_as_float(next_base + ibase), __int_as_float(leaf_base + lbase));
}

// ---- exclusive prefix sum of u64 (block-local, block sums, add) --------------
constexpr int kScanItems = 1024;   // 256 threads x 4

__global__ void __launch_bounds__(256) k_scan_local(const unsigned long long* __restrict__ in,
                                                   unsigned long long* __restrict__ out,
                                                   unsigned long long* __restrict__ sums, int n)
{
    __shared__ unsigned long long sh[256];
    const int base = blockIdx.x * kScanItems + threadIdx.x * 4;
    unsigned long long v[4], t = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = base + k < n ? in[base + k] : 0ull;
        t += v[k];
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned long long x = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned long long run = sh[threadIdx.x] - t;   // exclusive prefix of this thread
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = sh[255];
}

// single block: exclusive scan of the block sums in place; *total = sum
__global__ void __launch_bounds__(256) k_scan_sums(unsigned long long* __restrict__ sums, int nb,
                                                  unsigned long long* __restrict__ total)
{
    __shared__ unsigned long long sh[256];
    unsigned long long carry = 0;
    for (int c0 = 0; c0 < nb; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const unsigned long long v = i < nb ? sums[i] : 0ull;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const unsigned long long x = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0ull;
            __syncthreads();
            sh[threadIdx.x] += x;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + sh[threadIdx.x] - v;
        const unsigned long long chunk = sh[255];
        __syncthreads();
        carry += chunk;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(256) k_scan_add(unsigned long long* __restrict__ out,
                                                 const unsigned long long* __restrict__ sums, int n)
{
    const int base = blockIdx.x * kScanItems + threadIdx.x * 4;
    const unsigned long long s = sums[blockIdx.x];
    for (int k = 0; k < 4; ++k)
        if (base + k < n) out[base + k] += s;
}

__global__ void k_write_tris(int n, const int* __restrict__ leaf_order, const int* __restrict__ vals,
                             const float* __restrict__ verts, const int* __restrict__ tris,
                             const int* __restrict__ tri_patch, float4* __restrict__ out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int t = vals[leaf_order[s]];
    const int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    const float v0x = verts[3 * a], v0y = verts[3 * a + 1], v0z = verts[3 * a + 2];
    out[3 * s + 0] = make_float4(v0x, v0y, v0z, __int_as_float(t));
    out[3 * s + 1] = make_float4(verts[3 * b] - v0x, verts[3 * b + 1] - v0y, verts[3 * b + 2] - v0z,
                                 __int_as_float(tri_patch[t]));
    out[3 * s + 2] = make_float4(verts[3 * c] - v0x, verts[3 * c + 1] - v0y, verts[3 * c + 2] - v0z, 0.f);
}

inline int blocks_for(long long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

namespace {

// device buffer freed on scope exit unless released
template <typename T>
struct DevBuf {
    T* p = nullptr;
    hipError_t alloc(size_t n) { return hipMalloc(&p, sizeof(T) * (n > 0 ? n : 1)); }
    T* release()
    {
        T* q = p;
        p = nullptr;
        return q;
    }
    ~DevBuf() { hipFree(p); }
};

hipError_t scan_u64(const unsigned long long* in, unsigned long long* out, unsigned long long* sums,
                    unsigned long long* total, int n, hipStream_t st)
{
    const int nb = blocks_for(n, kScanItems);
    k_scan_local<<<nb, 256, 0, st>>>(in, out, sums, n);
    k_scan_sums<<<1, 256, 0, st>>>(sums, nb, total);
    k_scan_add<<<nb, 256, 0, st>>>(out, sums, n);
    return hipGetLastError();
}

}  // namespace

// Builds the 4-wide nodes [n_nodes * kNodeRows float4] and leaf triangles
// [n * 3 float4, 2 * 3 for a single triangle, which the root holds twice];
// *depth_out = number of wide levels.
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
    const int radius = kPlocRadius;
    int n_wide = 0, wide_levels = 0;
    std::vector<std::pair<int, int>> rounds;   // binary nodes created per merge round
    DevBuf<float4> tlo, thi, cen, part, nlo, nhi, clo[2], chi[2], nodes, otris;
    DevBuf<uint64_t> keys;
    DevBuf<unsigned long long> flags, scan, sums, total;
    DevBuf<int> vals, pint, pleaf, nn, cid[2];
    DevBuf<int2> child;
    hipError_t e;
#define LT_TRY(x)                      \
    do {                               \
        e = (x);                       \
        if (e != hipSuccess) return e; \
    } while (0)
    LT_TRY(tlo.alloc(n)); LT_TRY(thi.alloc(n)); LT_TRY(cen.alloc(n)); LT_TRY(part.alloc(2 * n_part));
    LT_TRY(keys.alloc(n_pow2)); LT_TRY(vals.alloc(n_pow2));
    LT_TRY(child.alloc(n_int)); LT_TRY(pint.alloc(n_int)); LT_TRY(pleaf.alloc(n));
    LT_TRY(nlo.alloc(n_int)); LT_TRY(nhi.alloc(n_int));
    const int n_leaves = n > 1 ? n : 2;   // every triangle is one leaf; a single one fills both root slots
    LT_TRY(nodes.alloc(kNodeRows * (size_t)n_int)); LT_TRY(otris.alloc(3 * (size_t)n_leaves));

    k_tri_setup<<<blocks_for(n, 256), 256, 0, st>>>(d_verts, d_tris, n, pad, tlo.p, thi.p, cen.p);
    k_bounds_partial<<<n_part, 256, 0, st>>>(cen.p, n, part.p);
    k_morton<<<blocks_for(n_pow2, 256), 256, 0, st>>>(cen.p, n, n_pow2, part.p, n_part, keys.p, vals.p);
    for (int k = 2; k <= n_pow2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1)
            k_bitonic<<<blocks_for(n_pow2, 256), 256, 0, st>>>(keys.p, vals.p, n_pow2, j, k);
    LT_TRY(hipGetLastError());
    if (n == 1) {
        // a single triangle: one node whose two children are that leaf
        const int2 single_leaf = make_int2(~0, ~0);
        LT_TRY(hipMemcpyAsync(child.p, &single_leaf, sizeof(int2), hipMemcpyHostToDevice, st));
        LT_TRY(hipStreamSynchronize(st));
    } else {
        for (int b = 0; b < 2; ++b) {
            LT_TRY(clo[b].alloc(n)); LT_TRY(chi[b].alloc(n)); LT_TRY(cid[b].alloc(n));
        }
        LT_TRY(nn.alloc(n)); LT_TRY(flags.alloc(n)); LT_TRY(scan.alloc(n));
        LT_TRY(sums.alloc(blocks_for(n, kScanItems))); LT_TRY(total.alloc(1));
        k_ploc_init<<<blocks_for(n, 256), 256, 0, st>>>(n, vals.p, tlo.p, thi.p, cid[0].p, clo[0].p, chi[0].p);
        int nc = n, node_base = 0, cur = 0, iter = 0;
        while (nc > 1) {
            if (++iter > 4 * n + 64) return hipErrorUnknown;   // every round merges at least one pair
            const int nx = cur ^ 1;
            k_ploc_nn<<<blocks_for(nc, 256), 256, 0, st>>>(nc, radius, clo[cur].p, chi[cur].p, nn.p);
            k_ploc_flags<<<blocks_for(nc, 256), 256, 0, st>>>(nc, nn.p, flags.p);
            LT_TRY(scan_u64(flags.p, scan.p, sums.p, total.p, nc, st));
            k_ploc_write<<<blocks_for(nc, 256), 256, 0, st>>>(nc, n_int, node_base, nn.p, flags.p, scan.p,
                                                              cid[cur].p, clo[cur].p, chi[cur].p, cid[nx].p,
                                                              clo[nx].p, chi[nx].p, child.p, nlo.p, nhi.p,
                                                              pint.p, pleaf.p);
            unsigned long long tot = 0;
            LT_TRY(hipMemcpyAsync(&tot, total.p, sizeof(tot), hipMemcpyDeviceToHost, st));
            LT_TRY(hipStreamSynchronize(st));
            const int kept = (int)(tot >> 32), merged = (int)(tot & 0xffffffffull);
            if (merged < 1 || kept != nc - merged) return hipErrorUnknown;
            rounds.push_back(std::make_pair(n_int - node_base - merged, n_int - node_base));
            node_base += merged;
            nc = kept;
            cur = nx;
        }
        if (node_base != n - 1) return hipErrorUnknown;
    }
    if (rounds.empty()) rounds.push_back(std::make_pair(0, 1));
    // collapse into the wide tree, level by level from the root
    {
        DevBuf<int> lvl[2], kids, dec, leaf_order;
        DevBuf<float4> dp;
        DevBuf<unsigned long long> cnt, off;
        LT_TRY(dec.alloc(n_int)); LT_TRY(dp.alloc(n_int));
        for (const auto& r : rounds) {
            if (r.first < 0 || r.second > n_int || r.first >= r.second) return hipErrorUnknown;
            k_collapse_dp<<<blocks_for(r.second - r.first, 256), 256, 0, st>>>(r.first, r.second, child.p, nlo.p,
                                                                               nhi.p, vals.p, tlo.p, thi.p, dp.p,
                                                                               dec.p);
        }
        LT_TRY(hipGetLastError());
        LT_TRY(lvl[0].alloc(n_int)); LT_TRY(lvl[1].alloc(n_int)); LT_TRY(kids.alloc(4 * (size_t)n_int));
        LT_TRY(cnt.alloc(n_int)); LT_TRY(off.alloc(n_int)); LT_TRY(leaf_order.alloc(n_leaves));
        if (!sums.p) LT_TRY(sums.alloc(blocks_for(n_int, kScanItems)));
        if (!total.p) LT_TRY(total.alloc(1));
        const int root = 0;
        LT_TRY(hipMemcpyAsync(lvl[0].p, &root, sizeof(int), hipMemcpyHostToDevice, st));
        int n_level = 1, out_base = 0, cur = 0, levels = 0;
        long long leaf_base = 0;
        while (n_level > 0) {
            if (++levels > n_int + 1) return hipErrorUnknown;
            k_collapse_open<<<blocks_for(n_level, 256), 256, 0, st>>>(n_level, lvl[cur].p, child.p, dec.p, kids.p,
                                                                      cnt.p);
            LT_TRY(scan_u64(cnt.p, off.p, sums.p, total.p, n_level, st));
            unsigned long long tot = 0;
            LT_TRY(hipMemcpyAsync(&tot, total.p, sizeof(tot), hipMemcpyDeviceToHost, st));
            LT_TRY(hipStreamSynchronize(st));
            const int next_base = out_base + n_level;
            const long long n_next = (long long)(tot & 0xffffffffull), n_lv = (long long)(tot >> 32);
            // before any write
            if (next_base + n_next > n_int || leaf_base + n_lv > n_leaves) return hipErrorUnknown;
            k_collapse_write<<<blocks_for(n_level, 256), 256, 0, st>>>(n_level, out_base, next_base, (int)leaf_base,
                                                                       kids.p, off.p, nlo.p, nhi.p, vals.p, tlo.p,
                                                                       thi.p, nodes.p, lvl[cur ^ 1].p, leaf_order.p);
            LT_TRY(hipGetLastError());
            out_base = next_base;
            leaf_base += n_lv;
            n_level = (int)n_next;
            cur ^= 1;
        }
        if (leaf_base != n_leaves) return hipErrorUnknown;   // every leaf slot written once
        n_wide = out_base;
        wide_levels = levels;
        k_write_tris<<<blocks_for(n_leaves, 256), 256, 0, st>>>(n_leaves, leaf_order.p, vals.p, d_verts, d_tris,
                                                                d_tri_patch, otris.p);
    }
    int depth = wide_levels;
    LT_TRY(hipGetLastError());
    LT_TRY(hipStreamSynchronize(st));
#undef LT_TRY
    *depth_out = depth;
    *nodes_out = nodes.release();
    *tris_out = otris.release();
    *n_nodes_out = n_wide;
    return hipSuccess;
}

}  // namespace lt
