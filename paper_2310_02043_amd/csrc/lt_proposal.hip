// Learned emission proposal: a small MLP per luminaire batch,
//   x [32] (6 normalised light parameters, 16-d light embedding, zero pad)
//   -> 64 ReLU -> 64 ReLU -> 1024 logits over the cells of the emission
//   hemisphere's hemi-octahedral map -> softmax = cell probabilities.
// Inference runs BF16 weights and activations on MFMA with FP32 accumulate
// (v_mfma_f32_16x16x16 bf16, 16 luminaires per block) and writes the
// sampler's pdf / cdf tables directly.  Training (cross-entropy to a target
// cell distribution, Adam) keeps FP32 master weights and refreshes the BF16
// copy; it is a small single-block kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "lt_internal.h"

namespace lt {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even float -> bf16 bits
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Y[16][N] = act(X[16][K] W^T + b); X in LDS (bf16, row stride ldx), W [N][K]
// bf16 in global memory, b [N] f32.  Each wave computes 16x16 output tiles
// tile = wave, wave + 4, ...; results to LDS, as bf16 (ldy) or f32 (ldz).
template <int K, bool RELU, bool F32OUT>
__device__ __forceinline__ void mfma_layer(const uint16_t* __restrict__ sx, int ldx, const uint16_t* __restrict__ W,
                                           const float* __restrict__ bias, int N, uint16_t* sy, int ldy, float* sz,
                                           int ldz)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    for (int tile = wave; tile < N / 16; tile += 4) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += 16) {
            bf16x4 a, b;
            const uint16_t* xa = sx + r16 * ldx + k0 + 4 * kq;
            const uint16_t* wb = W + (size_t)(tile * 16 + r16) * K + k0 + 4 * kq;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = (short)xa[i];
                b[i] = (short)wb[i];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        const int col = tile * 16 + r16;
        const float bcol = bias[col];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 4 * kq + i;
            float v = acc[i] + bcol;
            if (RELU) v = fmaxf(v, 0.0f);
            if (F32OUT) sz[row * ldz + col] = v;
            else sy[row * ldy + col] = to_bf16(v);
        }
    }
}

__global__ void __launch_bounds__(256) k_mlp_infer(const uint16_t* __restrict__ wb, const float* __restrict__ x,
                                                  int L, float* __restrict__ logits, float* __restrict__ pdf,
                                                  float* __restrict__ cdf)
{
    __shared__ uint16_t sx[16 * kMlpIn];
    __shared__ uint16_t sh1[16 * kMlpHidden];
    __shared__ uint16_t sh2[16 * kMlpHidden];
    __shared__ float sz[16 * kMlpBins];
    const int row0 = blockIdx.x * 16;
    for (int i = threadIdx.x; i < 16 * kMlpIn; i += 256) {
        const int r = i / kMlpIn, k = i % kMlpIn;
        sx[i] = row0 + r < L ? to_bf16(x[(size_t)(row0 + r) * kMlpIn + k]) : (uint16_t)0;
    }
    __syncthreads();
    const uint16_t* W1 = wb + kMlpOffW1;
    const uint16_t* W2 = wb + kMlpOffW2;
    const uint16_t* W3 = wb + kMlpOffW3;
    // biases are kept in bf16 as well; expand to f32 in LDS
    __shared__ float b1[kMlpHidden], b2[kMlpHidden], b3[kMlpBins];
    for (int i = threadIdx.x; i < kMlpBins; i += 256) b3[i] = from_bf16(wb[kMlpOffB3 + i]);
    if (threadIdx.x < kMlpHidden) {
        b1[threadIdx.x] = from_bf16(wb[kMlpOffB1 + threadIdx.x]);
        b2[threadIdx.x] = from_bf16(wb[kMlpOffB2 + threadIdx.x]);
    }
    __syncthreads();
    mfma_layer<kMlpIn, true, false>(sx, kMlpIn, W1, b1, kMlpHidden, sh1, kMlpHidden, nullptr, 0);
    __syncthreads();
    mfma_layer<kMlpHidden, true, false>(sh1, kMlpHidden, W2, b2, kMlpHidden, sh2, kMlpHidden, nullptr, 0);
    __syncthreads();
    mfma_layer<kMlpHidden, false, true>(sh2, kMlpHidden, W3, b3, kMlpBins, nullptr, 0, sz, kMlpBins);
    __syncthreads();
    // softmax and inclusive prefix per row: wave w owns rows w, w+4, w+8, w+12
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = wave; r < 16; r += 4) {
        const int row = row0 + r;
        if (row >= L) continue;   // wave-uniform
        const float* z = sz + r * kMlpBins + lane * 16;
        float m = -3.0e38f;
        for (int i = 0; i < 16; ++i) m = fmaxf(m, z[i]);
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        float e[16], run = 0.0f;
        for (int i = 0; i < 16; ++i) {
            e[i] = __expf(z[i] - m);
            run += e[i];
        }
        // exclusive scan of the lane sums
        float incl = run;
        for (int off = 1; off < 64; off <<= 1) {
            const float o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        const float total = __shfl(incl, 63);
        float pre = incl - run;
        const float inv = 1.0f / total;
        for (int i = 0; i < 16; ++i) {
            const size_t k = (size_t)row * kMlpBins + lane * 16 + i;
            pre += e[i];
            pdf[k] = e[i] * inv;
            cdf[k] = (lane == 63 && i == 15) ? 1.0f : pre * inv;
            if (logits) logits[k] = z[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Training step (FP32): forward with the master weights, cross-entropy to the
// target distribution (rows of t sum to 1), backward through the three
// layers and into the embedding columns of x, Adam (beta1 0.9, beta2 0.999,
// eps 1e-8), BF16 refresh.  One block of 1024 threads; activations in the
// scratch buffer.
// ---------------------------------------------------------------------------
struct TrainScratch {
    float *h1, *h2, *p, *dh2, *dh1, *gx;
};

__device__ __forceinline__ void adam(float& w, float& m, float& v, float g, float lr, float c1, float c2)
{
    m = 0.9f * m + 0.1f * g;
    v = 0.999f * v + 0.001f * g * g;
    w -= lr * (m / c1) / (__builtin_sqrtf(v / c2) + 1e-8f);
}

__global__ void __launch_bounds__(1024) k_mlp_train(float* __restrict__ w, float* __restrict__ mw,
                                                   float* __restrict__ vw, uint16_t* __restrict__ wb,
                                                   float* __restrict__ x, float* __restrict__ mx,
                                                   float* __restrict__ vx, const float* __restrict__ target, int L,
                                                   int step, float lr, TrainScratch sc, float* __restrict__ loss_out,
                                                   float* __restrict__ grad_out)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    float* W1 = w + kMlpOffW1;
    float* B1 = w + kMlpOffB1;
    float* W2 = w + kMlpOffW2;
    float* B2 = w + kMlpOffB2;
    float* W3 = w + kMlpOffW3;
    float* B3 = w + kMlpOffB3;
    const int H = kMlpHidden, NB = kMlpBins, NI = kMlpIn;
    __shared__ float red[1024];
    // forward
    for (int i = tid; i < L * H; i += nt) {
        const int r = i / H, j = i % H;
        float s = B1[j];
        for (int k = 0; k < NI; ++k) s += W1[j * NI + k] * x[r * NI + k];
        sc.h1[i] = fmaxf(s, 0.0f);
    }
    __syncthreads();
    for (int i = tid; i < L * H; i += nt) {
        const int r = i / H, j = i % H;
        float s = B2[j];
        for (int k = 0; k < H; ++k) s += W2[j * H + k] * sc.h1[r * H + k];
        sc.h2[i] = fmaxf(s, 0.0f);
    }
    __syncthreads();
    for (int i = tid; i < L * NB; i += nt) {
        const int r = i / NB, b = i % NB;
        float s = B3[b];
        for (int k = 0; k < H; ++k) s += W3[b * H + k] * sc.h2[r * H + k];
        sc.p[i] = s;
    }
    __syncthreads();
    // softmax rows, loss, dZ = (p - t) / L stored in p
    float lsum = 0.0f;
    for (int r = 0; r < L; ++r) {
        float m = -3.0e38f;
        for (int b = tid; b < NB; b += nt) m = fmaxf(m, sc.p[r * NB + b]);
        red[tid] = m;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
            __syncthreads();
        }
        m = red[0];
        __syncthreads();
        float e = 0.0f;
        for (int b = tid; b < NB; b += nt) e += __expf(sc.p[r * NB + b] - m);
        red[tid] = e;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        const float lse = m + __logf(red[0]);
        __syncthreads();
        for (int b = tid; b < NB; b += nt) {
            const float z = sc.p[r * NB + b];
            const float t = target[r * NB + b];
            if (t > 0.0f) lsum += -t * (z - lse);
            sc.p[r * NB + b] = (__expf(z - lse) - t) / (float)L;
        }
        __syncthreads();
    }
    red[tid] = lsum;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0 && loss_out) *loss_out = red[0] / (float)L;
    __syncthreads();
    const float c1 = 1.0f - __powf(0.9f, (float)step), c2 = 1.0f - __powf(0.999f, (float)step);
    // dH2 = dZ W3 (old W3), masked by ReLU
    for (int i = tid; i < L * H; i += nt) {
        const int r = i / H, j = i % H;
        float s = 0.0f;
        for (int b = 0; b < NB; ++b) s += sc.p[r * NB + b] * W3[b * H + j];
        sc.dh2[i] = sc.h2[i] > 0.0f ? s : 0.0f;
    }
    __syncthreads();
    // layer 3 update
    for (int i = tid; i < NB * (H + 1); i += nt) {
        const int b = i / (H + 1), j = i % (H + 1);
        float g = 0.0f;
        for (int r = 0; r < L; ++r) g += sc.p[r * NB + b] * (j < H ? sc.h2[r * H + j] : 1.0f);
        const int o = j < H ? kMlpOffW3 + b * H + j : kMlpOffB3 + b;
        if (grad_out) grad_out[o] = g;
        adam(w[o], mw[o], vw[o], g, lr, c1, c2);
    }
    // dH1 = dH2 W2 (old W2), masked
    for (int i = tid; i < L * H; i += nt) {
        const int r = i / H, k = i % H;
        float s = 0.0f;
        for (int j = 0; j < H; ++j) s += sc.dh2[r * H + j] * W2[j * H + k];
        sc.dh1[i] = sc.h1[i] > 0.0f ? s : 0.0f;
    }
    __syncthreads();
    for (int i = tid; i < H * (H + 1); i += nt) {
        const int j = i / (H + 1), k = i % (H + 1);
        float g = 0.0f;
        for (int r = 0; r < L; ++r) g += sc.dh2[r * H + j] * (k < H ? sc.h1[r * H + k] : 1.0f);
        const int o = k < H ? kMlpOffW2 + j * H + k : kMlpOffB2 + j;
        if (grad_out) grad_out[o] = g;
        adam(w[o], mw[o], vw[o], g, lr, c1, c2);
    }
    // embedding columns of x: dX = dH1 W1 (old W1), kept until x is no longer read
    for (int i = tid; i < L * kMlpEmbed; i += nt) {
        const int r = i / kMlpEmbed, k = kMlpParams + i % kMlpEmbed;
        float g = 0.0f;
        for (int j = 0; j < H; ++j) g += sc.dh1[r * H + j] * W1[j * NI + k];
        sc.gx[i] = g;
    }
    __syncthreads();
    // layer 1 update with the old x
    for (int i = tid; i < H * (NI + 1); i += nt) {
        const int j = i / (NI + 1), k = i % (NI + 1);
        float g = 0.0f;
        for (int r = 0; r < L; ++r) g += sc.dh1[r * H + j] * (k < NI ? x[r * NI + k] : 1.0f);
        const int o = k < NI ? kMlpOffW1 + j * NI + k : kMlpOffB1 + j;
        if (grad_out) grad_out[o] = g;
        adam(w[o], mw[o], vw[o], g, lr, c1, c2);
    }
    __syncthreads();
    for (int i = tid; i < L * kMlpEmbed; i += nt) {
        const int r = i / kMlpEmbed, k = kMlpParams + i % kMlpEmbed;
        const int o = r * NI + k;
        if (grad_out) grad_out[kMlpWeights + o] = sc.gx[i];
        adam(x[o], mx[o], vx[o], sc.gx[i], lr, c1, c2);
    }
    __syncthreads();
    for (int i = tid; i < kMlpWeights; i += nt) wb[i] = to_bf16(w[i]);
}

// ---------------------------------------------------------------------------
// Training target and network inputs, computed where the tables live.
// ---------------------------------------------------------------------------
// Block-wide FP64 sum over 256 threads (fixed tree, so the result is
// reproducible).
__device__ __forceinline__ double block_sum256(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double out = red[0];
    __syncthreads();
    return out;
}

// Cell masses of the plain cos^n lobe: midpoint rule on kPlainSub^2 points
// per cell of (n + 1)/(2 pi) cos^n(theta) d(omega), d(omega) = du dv / (2 |p|^3)
// on the hemi-octahedral map, normalised per light.  One block per light,
// four cells per thread, FP64.
constexpr int kPlainSub = 8;
__global__ void __launch_bounds__(256) k_plain_mass(const float* __restrict__ lobe_n, double* __restrict__ mass)
{
    __shared__ double red[256];
    const int l = blockIdx.x;
    const double n = (double)lobe_n[l];
    const double h = 1.0 / (16.0 * kPlainSub);
    double m[4], tot = 0.0;
    for (int c = 0; c < 4; ++c) {
        const int b = (int)threadIdx.x + 256 * c;
        const int iu = b & 31, iv = b >> 5;
        double acc = 0.0;
        for (int sv = 0; sv < kPlainSub; ++sv)
            for (int su = 0; su < kPlainSub; ++su) {
                const double u = -1.0 + ((double)(iu * kPlainSub + su) + 0.5) * h;
                const double v = -1.0 + ((double)(iv * kPlainSub + sv) + 0.5) * h;
                const double x = 0.5 * (u + v), y = 0.5 * (u - v);
                const double z = 1.0 - fabs(x) - fabs(y);
                const double r = sqrt(x * x + y * y + z * z);
                acc += (n + 1.0) * 0.15915494309189533577 * pow(z / r, n) * (h * h / (2.0 * r * r * r));
            }
        m[c] = acc;
        tot += acc;
    }
    tot = block_sum256(tot, red);
    for (int c = 0; c < 4; ++c) mass[1024 * (long long)l + threadIdx.x + 256 * c] = m[c] / tot;
}

// Training target of one pass: per light, the histogram row normalised (an
// empty row counts as uniform), folded into the running average (weight
// `decay` on the old one; `first` starts it), square root, normalised, then
// mixed with the plain lobe's cell masses by `floor`.  One block per light.
__global__ void __launch_bounds__(256) k_proposal_target(const float* __restrict__ hist, double* __restrict__ h_avg,
                                                        const double* __restrict__ pmass, int first, double decay,
                                                        double floor_w, float* __restrict__ target)
{
    __shared__ double red[256];
    const long long row = 1024 * (long long)blockIdx.x;
    double hv[4], tot = 0.0;
    for (int c = 0; c < 4; ++c) {
        hv[c] = (double)hist[row + threadIdx.x + 256 * c];
        tot += hv[c];
    }
    tot = block_sum256(tot, red);
    double r[4], rs = 0.0;
    for (int c = 0; c < 4; ++c) {
        const long long k = row + threadIdx.x + 256 * c;
        const double hn = tot > 0.0 ? hv[c] / tot : 1.0 / 1024.0;
        const double a = first ? hn : decay * h_avg[k] + (1.0 - decay) * hn;
        h_avg[k] = a;
        r[c] = sqrt(a);
        rs += r[c];
    }
    rs = block_sum256(rs, red);
    for (int c = 0; c < 4; ++c) {
        const long long k = row + threadIdx.x + 256 * c;
        double t = r[c] / rs;
        if (floor_w > 0.0) t = (1.0 - floor_w) * t + floor_w * pmass[k];
        target[k] = (float)t;
    }
}

// Network inputs: the six parameters mapped to [-1, 1] by the box [lo, hi].
__global__ void k_proposal_inputs(const float* __restrict__ params, int L, ParamBox box, float* __restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L * kMlpParams) return;
    const int l = i / kMlpParams, c = i % kMlpParams;
    x[l * kMlpIn + c] = (2.0f * (params[i] - box.lo[c])) / (box.hi[c] - box.lo[c]) - 1.0f;
}

// Histogram units: running mean of each light's squared gradient components
// (weight `decay` on the old mean), then 1/sqrt(mean + 1e-30) times the
// component mask (non-finite values become 0).
__global__ void k_proposal_scale(const float* __restrict__ grad, int n, float* __restrict__ sig2, int first,
                                 float decay, Param6 mask, float* __restrict__ inv_sigma)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g2 = grad[i] * grad[i];
    const float s = first ? g2 : decay * sig2[i] + (1.0f - decay) * g2;
    sig2[i] = s;
    float inv = 1.0f / __builtin_sqrtf(s + 1e-30f);
    if (!__builtin_isfinite(inv)) inv = 0.0f;
    inv_sigma[i] = inv * mask.v[i % kMlpParams];
}

__global__ void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wb, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = to_bf16(w[i]);
}

}  // namespace

hipError_t launch_to_bf16(const float* w, uint16_t* wb, int n, hipStream_t st)
{
    k_to_bf16<<<(n + 255) / 256, 256, 0, st>>>(w, wb, n);
    return hipGetLastError();
}

hipError_t launch_plain_mass(const float* lobe_n, int L, double* mass, hipStream_t st)
{
    k_plain_mass<<<L, 256, 0, st>>>(lobe_n, mass);
    return hipGetLastError();
}

hipError_t launch_proposal_target(const float* hist, int L, double* h_avg, const double* pmass, int first,
                                  double decay, double floor_w, float* target, hipStream_t st)
{
    k_proposal_target<<<L, 256, 0, st>>>(hist, h_avg, pmass, first, decay, floor_w, target);
    return hipGetLastError();
}

hipError_t launch_proposal_inputs(const float* params, int L, const ParamBox& box, float* x, hipStream_t st)
{
    const int n = L * kMlpParams;
    k_proposal_inputs<<<(n + 255) / 256, 256, 0, st>>>(params, L, box, x);
    return hipGetLastError();
}

hipError_t launch_proposal_scale(const float* grad, int L, float* sig2, int first, float decay, const Param6& mask,
                                 float* inv_sigma, hipStream_t st)
{
    const int n = L * kMlpParams;
    k_proposal_scale<<<(n + 255) / 256, 256, 0, st>>>(grad, n, sig2, first, decay, mask, inv_sigma);
    return hipGetLastError();
}

size_t mlp_train_scratch_floats(int L) { return (size_t)L * (4 * kMlpHidden + kMlpBins + kMlpEmbed); }

// Guide entries for the inverse-CDF lookup: guide[l][j] is the first cell
// whose inclusive prefix sum exceeds j/1024 (1023 when none does), and
// guide[l][1024] = 1023.  For u in [j/1024, (j+1)/1024) the cell sought lies
// in [guide[j], guide[j+1]], so a search over that range returns the same
// cell as a search over all 1024.
__global__ void k_guide_build(const float* __restrict__ cdf, int L, int* __restrict__ guide)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)L * 1025) return;
    const int l = (int)(idx / 1025), j = (int)(idx % 1025);
    int out = 1023;
    if (j < 1024) {
        const float* c = cdf + 1024 * (long long)l;
        const float t = (float)j * (1.0f / 1024.0f);
        int lo = 0, hi = 1023;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (c[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        out = lo;
    }
    guide[idx] = out;
}

hipError_t launch_guide_build(const float* cdf, int L, int* guide, hipStream_t st)
{
    const long long n = (long long)L * 1025;
    k_guide_build<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(cdf, L, guide);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const uint16_t* wb, const float* x, int L, float* logits, float* pdf, float* cdf,
                            hipStream_t st)
{
    k_mlp_infer<<<(L + 15) / 16, 256, 0, st>>>(wb, x, L, logits, pdf, cdf);
    return hipGetLastError();
}

hipError_t launch_mlp_train(float* w, float* mw, float* vw, uint16_t* wb, float* x, float* mx, float* vx,
                            const float* target, int L, int step, float lr, float* scratch, float* loss,
                            float* grad_out, hipStream_t st)
{
    TrainScratch sc;
    sc.h1 = scratch;
    sc.h2 = sc.h1 + (size_t)L * kMlpHidden;
    sc.dh2 = sc.h2 + (size_t)L * kMlpHidden;
    sc.dh1 = sc.dh2 + (size_t)L * kMlpHidden;
    sc.p = sc.dh1 + (size_t)L * kMlpHidden;
    sc.gx = sc.p + (size_t)L * kMlpBins;
    k_mlp_train<<<1, 1024, 0, st>>>(w, mw, vw, wb, x, mx, vx, target, L, step, lr, sc, loss, grad_out);
    return hipGetLastError();
}

}  // namespace lt
