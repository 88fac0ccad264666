// Internal interfaces between the C ABI layer and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "lt_device.h"

namespace lt {

constexpr int kMaxStackDepth = 128;   // BVH depth bound accepted at upload
constexpr int kObjBlocks = 1024;      // fixed grid of the objective reduction
constexpr int kRecordBlocks = 1024;   // grid of the path-recording kernel (4 waves each)
constexpr int kPtBlocks = 2048;       // grid of the path-tracing kernel (4 waves each)
constexpr int kPtMaxLights = 256;     // luminaires per layout the path tracer accepts
constexpr int kPlocRadius = 16;       // nearest-neighbour window of the BVH build
constexpr int kBvhWidth = 4;          // children per node of the traversed tree
constexpr int kEmptyChild = (int)0x80000000;  // unused child slot of a wide node
constexpr int kNodeRows = 4;                  // 16-byte rows per wide node
// traversal-stack entries in LDS of the plain adjoint: the most that six
// of its waves per SIMD (6.5 KB each with their per-lane state) fit in a
// CU's 160 KB
constexpr int kAdjLdsDepth = 13;
// the same for the colour adjoint at five waves per SIMD (7.75 KB each; at
// 13 entries, 8 KB, its fifth block no longer fits)
constexpr int kColAdjLdsDepth = 12;

// sticky device status bits (the LT_STATUS_* values of the C ABI)
constexpr unsigned kStatusOverflow = 1u;   // a texel accumulator reached 2^62
constexpr unsigned kStatusTraversal = 2u;  // a segment exceeded its node-visit bound
constexpr unsigned kStatusParams = 4u;     // a luminaire parameter was not finite or its power not positive

// emission-proposal MLP: x [32] -> 64 -> 64 -> 1024 cells
constexpr int kMlpParams = 6, kMlpEmbed = 16, kMlpIn = 32, kMlpHidden = 64, kMlpBins = 1024;
constexpr int kMlpOffW1 = 0;                                    // [64][32]
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpHidden * kMlpIn;      // [64]
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpHidden;               // [64][64]
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpHidden * kMlpHidden;  // [64]
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpHidden;               // [1024][64]
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpBins * kMlpHidden;    // [1024]
constexpr int kMlpWeights = kMlpOffB3 + kMlpBins;               // 72832

struct TraceArgs {
    const float4* nodes;
    const float4* tris;
    const DevPatch* patches;
    const DevLight* lights;
    const int4* tiles;          // (global light, first path, count, layout)
    int n_tiles;
    int max_hits;
    // work queues: queue q hands out tiles q_first[q] .. q_first[q] + q_len[q] - 1
    // through the ticket counter queue[q] (zeroed before every launch); one
    // queue, or eight contiguous shares (one per XCD) with XCD remapping
    unsigned* queue;
    int n_queues;
    int q_first[8], q_len[8];
    int xcd_remap;
    uint32_t key0, key1;
    long long* S;               // forward: [n_layouts, K]
    const float* g;             // adjoint: [n_layouts, K]
    long long K;
    double* partials;           // adjoint: [n_tiles, 6]
    unsigned long long* misses;
    unsigned long long* stats;  // instrumented kernel: 5 counters
    int* gstack;                // traversal stack overflow, [gstack_waves][gdepth][64]
    int gdepth;
    long long gstack_waves;     // persistent wave slots the overflow area covers
    int refill_threshold;
    int linear;                 // piecewise-linear texel basis (else box)
    int tri_share;              // eighths of the traversing lanes that select a triangle-test iteration
    int max_steps;              // node visits per segment before the segment is abandoned
    unsigned* flags;            // sticky status bits (2 = traversal step limit hit)
    // emission proposal (one-sample MIS with the plain lobe), may be null
    const float* prop_pdf;      // [L,1024] bin probabilities
    const float* prop_cdf;      // [L,1024] inclusive prefix sums
    const int* prop_guide;      // [L,1025] first cell whose prefix sum exceeds j/1024
    float alpha_plain;
    float* bin_hist;            // adjoint: [L,1024] histogram of |c_r / sigma| (may be null)
    const float* inv_sigma;     // [L,6]
    // direct-differentiation map of one luminaire and parameter: [K] Q31.32
    long long* tangent;
    int tan_light;
    int tan_param;
    // soft-edged spots' cone angles (adjoint: [n_tiles,8] partials), [L,5]
    // per-light constants written by the light setup, may be null
    const float* cone;
    // orientation as a rotation vector (adjoint: [n_tiles,7] partials)
    int rotvec;
    // directional texels: HSH order 0..2 (-1: irradiance texels), local
    // samples per hit, [P] per-patch (specular albedo, Phong exponent)
    int dir_order;
    int dir_samples;
    const float2* glossy;
    // colour mode: [L,3] channel weights, [P] per-patch channel albedo,
    // adjoint [n_tiles,3] partial sums of dO/dc
    int rgb;
    const float* colour;
    const float4* rho_rgb;
    double* partials_col;
    // adjoint: gradient-contribution map of one light and parameter (may be null)
    double* vote;               // [K] texels of the light's layout
    int vote_light;             // global light index
    int vote_param;             // 0..5
    // two-pass adjoint (grey, box basis): instead of the per-tile sums, each
    // path leaves a first-hit record, kRecFields planes of rec_stride floats
    // (x_1 xyz, origin y xyz, patch | flip << 31, a_u, a_v, Phi_r, s_r, with
    // the training histogram the emission cell and its weight, in colour the
    // green and blue sums), at index rec_base[light] + path; null otherwise
    float* rec;
    long long rec_stride;
    const long long* rec_base;
};

constexpr int kRecFields = 15;   // floats per path of the two-pass adjoint's records

// Object-space path tracing over the texels of one layout.
struct PtArgs {
    const float4* nodes;
    const float4* tris;
    const DevPatch* patches;
    const long long* pbase;     // first texel of each patch (ascending)
    int n_patches;
    const DevLight* lights;     // the layout's luminaires: lights[0 .. nl)
    int nl;
    int layout;
    long long K;
    int M;                      // samples per texel
    int max_hits;               // path vertices (the texel point and its bounces)
    uint32_t key0, key1;
    long long* S;               // forward: [K] Q31.32 texel means (accumulated)
    const float* g;             // adjoint: [K] dO/dE
    double* grad;               // adjoint: [nl,6] accumulated
    int* gstack;
    int gdepth;
    int max_steps;
    unsigned* flags;
};

struct RecordArgs {
    const float4* nodes;
    const float4* tris;
    const DevPatch* patches;
    const DevLight* lights;
    int gl, layout, max_hits;
    long long K;
    uint32_t stream_id;
    uint32_t key0, key1;
    long long first, count;
    int* prim;
    int* texel;
    const float* g;
    float* contrib;
    int linear;
    int* gstack;
    int gdepth;
    int max_steps;
    unsigned* flags;
    const float* prop_pdf;
    const float* prop_cdf;
    const int* prop_guide;
    float alpha_plain;
};

hipError_t build_bvh(const float* d_verts, const int* d_tris, const int* d_tri_patch, int n, float pad,
                     hipStream_t st, float4** nodes_out, float4** tris_out, int* n_nodes_out, int* depth_out);

// persistent launch: min(tiles, resident waves of the instance on n_cu CUs)
// waves, never more than a.gstack_waves; zeroes the queue counters first
hipError_t launch_trace(bool adjoint, bool stats, const TraceArgs& a, int waves_per_block, int lds_depth, int n_cu,
                        hipStream_t st);
hipError_t launch_record(const RecordArgs& a, int lds_depth, hipStream_t st);
// work tiles of paths_per_layout ppl in tiles of tp paths, built on the device
// from the static light table si (.y layout, .z index in it, .w lights in it)
hipError_t launch_build_tiles(const int4* si, int L, long long ppl, int tp, int n_tiles, int4* tiles, int2* range,
                              long long* npaths, hipStream_t st);
hipError_t launch_light_setup(const float* params, const int4* lstat_i, const float4* lstat_f,
                              const long long* npaths, int n_lights, DevLight* out, unsigned* flags,
                              hipStream_t st, int rv = 0, float* cone = nullptr);
hipError_t launch_grad_reduce_cone(const double* partials, const int2* range, int n_lights, float* grad,
                                   float* gcone, hipStream_t st);
hipError_t launch_grad_reduce_rv(const double* partials, const int2* range, const float* params, int n_lights,
                                 float* grad, hipStream_t st);
hipError_t launch_clear(long long* S, long long n_texels_total, hipStream_t st);
hipError_t launch_fill_f32(float* p, long long n, float v, hipStream_t st);
hipError_t launch_pt(bool adjoint, const PtArgs& a, int lds_depth, hipStream_t st);
hipError_t launch_grad_reduce_col(const double* partials, const int2* range, int n_lights, float* grad,
                                  hipStream_t st);
hipError_t launch_f64_to_f32(const double* in, float* out, long long n, hipStream_t st);
hipError_t launch_fd_params(const float* p, int n, int idx, float h, float* pp, float* pm, double* den,
                            hipStream_t st);
hipError_t launch_fd_diff(const long long* Sp, const long long* Sm, long long K, const double* den, float* F,
                          hipStream_t st);
hipError_t launch_finalize(const long long* S, float* E, long long n, unsigned* flags, hipStream_t st);
hipError_t launch_objective(const float* E, const float* Et, const float* alpha, const float* A, long long K,
                            long long n, float* g, double* partials, double* O, hipStream_t st);
hipError_t launch_grad_reduce(const double* partials, const int2* tile_range, int n_lights, float* grad,
                              hipStream_t st);
// second pass of the two-pass adjoint: per-tile FP64 partial sums [n_tiles, 6]
// of the recorded paths' contributions
hipError_t launch_rec_grad(const TraceArgs& a, double* partials, hipStream_t st);
// the box [lo, hi] that maps luminaire parameters to network inputs, and a
// per-parameter factor, passed by value
struct ParamBox {
    float lo[6], hi[6];
};
struct Param6 {
    float v[6];
};
size_t mlp_train_scratch_floats(int L);
hipError_t launch_plain_mass(const float* lobe_n, int L, double* mass, hipStream_t st);
hipError_t launch_to_bf16(const float* w, uint16_t* wb, int n, hipStream_t st);
hipError_t launch_proposal_target(const float* hist, int L, double* h_avg, const double* pmass, int first,
                                  double decay, double floor_w, float* target, hipStream_t st);
hipError_t launch_proposal_inputs(const float* params, int L, const ParamBox& box, float* x, hipStream_t st);
hipError_t launch_proposal_scale(const float* grad, int L, float* sig2, int first, float decay, const Param6& mask,
                                 float* inv_sigma, hipStream_t st);
hipError_t launch_guide_build(const float* cdf, int L, int* guide, hipStream_t st);
hipError_t launch_mlp_infer(const uint16_t* wb, const float* x, int L, float* logits, float* pdf, float* cdf,
                            hipStream_t st);
hipError_t launch_mlp_train(float* w, float* mw, float* vw, uint16_t* wb, float* x, float* mx, float* vx,
                            const float* target, int L, int step, float lr, float* scratch, float* loss,
                            float* grad_out, hipStream_t st);
hipError_t launch_texel_area(const float* patch_area, const long long* base, int n_patches, long long K,
                             float* A, hipStream_t st);

}  // namespace lt
