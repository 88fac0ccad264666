// C ABI of liblt.so: context, scene upload, luminaires, trace calls.
//
// Host code validates arguments synchronously, keeps the work-tile tables of
// the persistent kernels, and optionally replays each trace call as a captured
// hipGraph (no memset nodes are captured: counters and accumulators are
// cleared by kernels).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "lt.h"
#include "lt_device.h"
#include "lt_internal.h"

using namespace lt;

// Scratch of lt_trace_adjoint_noalloc: queue counters, work tiles, per-light
// ranges and path counts, per-tile partial sums and the traversal-stack
// overflow area, carved from one fixed device array so that the call needs no
// allocation.  Each device holds its own copy until the process ends; host
// code uses only the per-device address taken at lt_create, never the
// symbol itself.
constexpr size_t kNoAllocBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on `device` (current device), taken
// once per device; nullptr on failure.
void* scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
};

}  // namespace

struct lt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t gstream = nullptr;   // capture stream for graphs
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::string err;
    int n_cu = 256;
    int waves_per_cu = 32;           // hardware wave slots per CU
    size_t mem_total = 0;            // device memory (bytes), for the two-pass adjoint's record budget
    unsigned char* noalloc = nullptr;  // this device's scratch array (lt_trace_adjoint_noalloc)
    unsigned* d_queue = nullptr;     // work-queue ticket counters of the persistent trace kernels [8]

    // scene
    bool has_scene = false;
    float4* nodes = nullptr;
    float4* tris = nullptr;
    DevPatch* patches = nullptr;
    long long* pbase = nullptr;
    float* parea = nullptr;
    float* texel_area = nullptr;
    float4* rho_rgb = nullptr;       // per-patch channel albedo (colour mode)
    float2* glossy = nullptr;        // per-patch (specular albedo, Phong exponent) (directional mode)
    int n_nodes = 0, depth = 0, n_patches = 0;
    long long n_tris = 0, K = 0;
    uint64_t generation = 1;

    // luminaires
    bool has_lights = false;
    int L = 0, n_layouts = 0;
    std::vector<lt_light_static> lights;
    std::vector<int> offs;
    int4* d_si = nullptr;
    float4* d_sf = nullptr;
    DevLight* d_lights = nullptr;

    // tiles for (paths_per_layout, tile_paths)
    long long tiles_ppl = -1;
    int tiles_tp = -1;
    int4* d_tiles = nullptr;
    int n_tiles = 0;
    int2* d_range = nullptr;
    long long* d_npaths = nullptr;
    long long* d_rec_base = nullptr;  // two-pass adjoint: first record of each luminaire's paths [L]
    long long rec_paths = 0;          // paths of all layouts: records per field

    // scratch
    unsigned long long* d_misses = nullptr;
    unsigned* d_flags = nullptr;
    unsigned long long* d_stats = nullptr;
    double* d_objpart = nullptr;
    double* d_partials = nullptr;
    size_t partials_cap = 0;
    int* d_gstack = nullptr;
    size_t gstack_cap = 0;
    double* d_ptgrad = nullptr;      // path tracer: FP64 gradient accumulator [L,6]
    size_t ptgrad_cap = 0;
    double* d_partials_col = nullptr; // colour adjoint: [n_tiles,3] partial sums of dO/dc
    size_t partials_col_cap = 0;
    double* d_partials7 = nullptr;    // rotation-vector adjoint: [n_tiles,7] partial sums
    float* d_pfd = nullptr;           // central differences: p+ [L,6], p- [L,6], step (f64)
    int pfd_cap = 0;                  // lights d_pfd holds
    double* d_partials8 = nullptr;    // cone-angle adjoint: [n_tiles,8] partial sums
    size_t partials8_cap = 0;
    float* d_cone = nullptr;          // cone-angle adjoint: [L,5] per-light constants
    int cone_cap = 0;
    float* d_rec = nullptr;           // two-pass adjoint: first-hit records [kRecFields][rec_paths]
    size_t rec_cap = 0;               // floats d_rec holds
    size_t partials7_cap = 0;

    lt_tuning tune;
    std::vector<GraphEntry> graphs;

    // emission proposal tables (per light, 32 x 32 hemi-octahedral cells)
    bool has_proposal = false;
    float* prop_pdf = nullptr;
    float* prop_cdf = nullptr;
    int* prop_guide = nullptr;
    float* inv_sigma = nullptr;
    float* mlp_scratch = nullptr;
    size_t mlp_scratch_cap = 0;

    // proposal network owned by the context (lt_proposal_set): FP32 master
    // weights, Adam moments, BF16 copy, inputs [L,32] with the embeddings,
    // running histogram average and plain-lobe cell masses [L,1024] (FP64),
    // the last training target [L,1024], running squared gradients [L,6]
    bool has_net = false;
    float *net_w = nullptr, *net_mw = nullptr, *net_vw = nullptr;
    uint16_t* net_wb = nullptr;
    float *net_x = nullptr, *net_mx = nullptr, *net_vx = nullptr;
    double *net_havg = nullptr, *net_pmass = nullptr;
    float *net_target = nullptr, *net_sig2 = nullptr;
    int net_step = 0;
    bool net_havg_ok = false, net_sig2_ok = false;
    lt_proposal_cfg net_cfg;

    // kernel timing (events around trace kernels launched outside graphs)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> t_fwd, t_adj;
};

namespace {

int fail(lt_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, e_ == hipErrorOutOfMemory ? LT_ENOMEM : LT_EHIP,                  \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

// An executable graph may still run on the capture stream; wait for it
// before destroying any (or freeing a buffer a graph refers to).
void free_graphs(lt_ctx* c)
{
    if (c->gstream && !c->graphs.empty()) hipStreamSynchronize(c->gstream);
    for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

void free_net(lt_ctx* c)
{
    hipFree(c->net_w); hipFree(c->net_mw); hipFree(c->net_vw); hipFree(c->net_wb);
    hipFree(c->net_x); hipFree(c->net_mx); hipFree(c->net_vx);
    hipFree(c->net_havg); hipFree(c->net_pmass); hipFree(c->net_target); hipFree(c->net_sig2);
    c->net_w = c->net_mw = c->net_vw = nullptr;
    c->net_wb = nullptr;
    c->net_x = c->net_mx = c->net_vx = nullptr;
    c->net_havg = c->net_pmass = nullptr;
    c->net_target = c->net_sig2 = nullptr;
    c->has_net = false;
}

void free_scene(lt_ctx* c)
{
    hipFree(c->nodes); hipFree(c->tris); hipFree(c->patches); hipFree(c->pbase); hipFree(c->parea);
    hipFree(c->texel_area); hipFree(c->rho_rgb); hipFree(c->glossy);
    c->nodes = nullptr; c->tris = nullptr; c->patches = nullptr; c->pbase = nullptr; c->parea = nullptr;
    c->texel_area = nullptr; c->rho_rgb = nullptr; c->glossy = nullptr;
    c->has_scene = false;
}

void free_tiles(lt_ctx* c)
{
    hipFree(c->d_tiles); hipFree(c->d_range); hipFree(c->d_npaths); hipFree(c->d_rec_base);
    c->d_tiles = nullptr; c->d_range = nullptr; c->d_npaths = nullptr; c->d_rec_base = nullptr;
    c->rec_paths = 0;
    c->tiles_ppl = -1;
    c->tiles_tp = -1;
    c->n_tiles = 0;
}

lt_tuning default_tuning()
{
    lt_tuning t;
    memset(&t, 0, sizeof(t));
    t.waves_per_block = 4;
    t.xcd_remap = 0;
    t.tile_paths = 1024;
    t.refill_threshold = 32;
    t.lds_depth = 16;
    t.tri_share = 4;
    return t;
}

// Waves the device can hold resident at once (every CU full): the persistent
// trace kernels never launch more, so their traversal-stack overflow area is
// sized by this, not by the number of work tiles.
long long resident_waves(const lt_ctx* c) { return (long long)c->n_cu * c->waves_per_cu; }

long long paths_of_light(long long ppl, int n_in_layout, int l)
{
    return ppl / n_in_layout + ((long long)l < ppl % n_in_layout ? 1 : 0);
}

int effective_tile_paths(const lt_ctx* c, long long ppl)
{
    if (c->tune.tile_paths > 0) return c->tune.tile_paths;
    // about 64 tiles per CU: enough waves to fill the chip and balance the tail
    const long long total = ppl * (long long)c->n_layouts;
    long long tp = total / ((long long)c->n_cu * 64);
    tp = (tp / 64) * 64;
    if (tp < 64) tp = 64;
    if (tp > 8192) tp = 8192;
    return (int)tp;
}

int ensure_tiles(lt_ctx* c, long long ppl)
{
    const int tp = effective_tile_paths(c, ppl);
    if (c->tiles_ppl == ppl && c->tiles_tp == tp) return LT_OK;
    std::vector<int4> tiles;
    std::vector<int2> range(c->L);
    std::vector<long long> np(c->L), rb(c->L);
    long long total = 0;
    for (int j = 0; j < c->n_layouts; ++j) {
        const int l0 = c->offs[j], l1 = c->offs[j + 1];
        for (int gl = l0; gl < l1; ++gl) {
            const long long nl = paths_of_light(ppl, l1 - l0, gl - l0);
            if (nl > 0xFFFFFFFFll) return fail(c, LT_EINVAL, "more than 2^32 paths for one light");
            np[gl] = nl;
            rb[gl] = total;
            total += nl;
            range[gl].x = (int)tiles.size();
            for (long long f = 0; f < nl; f += tp) {
                const long long cnt = std::min<long long>(tp, nl - f);
                tiles.push_back(make_int4(gl, (int)(uint32_t)f, (int)cnt, j));
            }
            range[gl].y = (int)tiles.size();
        }
    }
    if (tiles.size() > (size_t)0x7fffffff) return fail(c, LT_EINVAL, "too many work tiles");
    free_tiles(c);
    free_graphs(c);
    HIPCHK(c, hipMalloc(&c->d_tiles, sizeof(int4) * std::max<size_t>(tiles.size(), 1)));
    HIPCHK(c, hipMalloc(&c->d_range, sizeof(int2) * c->L));
    HIPCHK(c, hipMalloc(&c->d_npaths, sizeof(long long) * c->L));
    HIPCHK(c, hipMalloc(&c->d_rec_base, sizeof(long long) * c->L));
    HIPCHK(c, hipMemcpy(c->d_rec_base, rb.data(), sizeof(long long) * c->L, hipMemcpyHostToDevice));
    c->rec_paths = total;
    HIPCHK(c, hipMemcpy(c->d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_range, range.data(), sizeof(int2) * c->L, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_npaths, np.data(), sizeof(long long) * c->L, hipMemcpyHostToDevice));
    c->n_tiles = (int)tiles.size();
    c->tiles_ppl = ppl;
    c->tiles_tp = tp;
    if (c->partials_cap < (size_t)c->n_tiles * 6) {
        hipFree(c->d_partials);
        c->d_partials = nullptr;
        c->partials_cap = 0;
        HIPCHK(c, hipMalloc(&c->d_partials, sizeof(double) * 6 * std::max(c->n_tiles, 1)));
        c->partials_cap = (size_t)std::max(c->n_tiles, 1) * 6;
    }
    return LT_OK;
}

// whether the two-pass adjoint's records for the current tiles' paths fit its
// budget, an eighth of device memory (36 GB on a 288 GB device); larger
// jobs take the one-pass kernel, which needs no per-path memory
bool rec_fits(const lt_ctx* c)
{
    return (size_t)kRecFields * sizeof(float) * (size_t)std::max(c->rec_paths, 1ll) <= c->mem_total / 8;
}

// the two-pass adjoint's record planes for the current tiles' paths
int ensure_rec(lt_ctx* c)
{
    const size_t need = (size_t)kRecFields * (size_t)std::max(c->rec_paths, 1ll);
    if (need <= c->rec_cap) return LT_OK;
    // the previous calls' passes may still read or write the old buffer
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_graphs(c);
    hipFree(c->d_rec);
    c->d_rec = nullptr;
    c->rec_cap = 0;
    HIPCHK(c, hipMalloc(&c->d_rec, sizeof(float) * need));
    c->rec_cap = need;
    return LT_OK;
}

// stack entries a segment can need: up to three pushes per level of the 4-wide tree
int stack_need(const lt_ctx* c) { return 3 * c->depth + 1; }
// overflow entries per lane: what the deepest segment can need beyond the
// smallest LDS part of any instance (the colour adjoint's)
int gstack_depth(const lt_ctx* c)
{
    return std::max(0, stack_need(c) - std::min({c->tune.lds_depth, kAdjLdsDepth, kColAdjLdsDepth}));
}

int ensure_gstack(lt_ctx* c, long long waves)
{
    const size_t need = (size_t)waves * (size_t)std::max(gstack_depth(c), 1) * 64;
    if (need <= c->gstack_cap) return LT_OK;
    free_graphs(c);
    hipFree(c->d_gstack);
    c->d_gstack = nullptr;
    c->gstack_cap = 0;
    HIPCHK(c, hipMalloc(&c->d_gstack, sizeof(int) * need));
    c->gstack_cap = need;
    return LT_OK;
}

int check_cfg(lt_ctx* c, const lt_trace_cfg* cfg)
{
    if (!c) return LT_EINVAL;
    if (!cfg) return fail(c, LT_EINVAL, "cfg is NULL");
    if (!c->has_scene) return fail(c, LT_ESTATE, "no scene uploaded");
    if (!c->has_lights) return fail(c, LT_ESTATE, "no luminaires set");
    if (cfg->max_hits < 1 || cfg->max_hits > 64) return fail(c, LT_EINVAL, "max_hits must be in [1, 64]");
    for (int j = 0; j < c->n_layouts; ++j)
        if (cfg->paths_per_layout < c->offs[j + 1] - c->offs[j])
            return fail(c, LT_EINVAL, "paths_per_layout smaller than the number of lights of a layout");
    if (cfg->flags & ~(LT_FLAG_GRAPH | LT_FLAG_PROPOSAL | LT_FLAG_LINEAR)) return fail(c, LT_EINVAL, "unknown flag");
    if (cfg->flags & LT_FLAG_PROPOSAL) {
        if (!c->has_proposal) return fail(c, LT_EINVAL, "no emission proposal loaded");
        if (!(cfg->alpha_plain > 0.0f && cfg->alpha_plain <= 1.0f))
            return fail(c, LT_EINVAL, "alpha_plain must be in (0, 1] (defensive mixture)");
    }
    return ensure_tiles(c, cfg->paths_per_layout);
}

// Launch a trace kernel; with timing on (and outside graph capture) bracket
// it by events on the same stream.
hipError_t timed_trace(lt_ctx* c, bool adjoint, bool capture, const TraceArgs& a, hipStream_t st)
{
    const bool t = c->timing && !capture;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (t) {
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        if (e != hipSuccess) return e;
    }
    hipError_t e = launch_trace(adjoint, false, a, c->tune.waves_per_block, c->tune.lds_depth, c->n_cu, st);
    if (t) {
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        (adjoint ? c->t_adj : c->t_fwd).push_back({e0, e1});
    }
    return e;
}

TraceArgs trace_args(lt_ctx* c, const lt_trace_cfg* cfg)
{
    TraceArgs a;
    memset(&a, 0, sizeof(a));
    a.nodes = c->nodes;
    a.tris = c->tris;
    a.patches = c->patches;
    a.lights = c->d_lights;
    a.tiles = c->d_tiles;
    a.n_tiles = c->n_tiles;
    a.max_hits = cfg->max_hits;
    a.xcd_remap = c->tune.xcd_remap;
    a.key0 = (uint32_t)cfg->seed;
    a.key1 = (uint32_t)(cfg->seed >> 32);
    a.K = c->K;
    a.misses = c->d_misses;
    a.stats = c->d_stats;
    a.gstack = c->d_gstack;
    a.gdepth = std::max(gstack_depth(c), 1);
    a.gstack_waves = (long long)(c->gstack_cap / ((size_t)a.gdepth * 64));
    // work queues: one over all tiles, or with XCD remapping eight contiguous
    // shares, one per XCD (workgroup b runs on XCD b % 8)
    a.queue = c->d_queue;
    a.n_queues = c->tune.xcd_remap ? 8 : 1;
    for (int q = 0; q < 8; ++q) {
        const long long lo = (long long)c->n_tiles * q / a.n_queues, hi = (long long)c->n_tiles * (q + 1) / a.n_queues;
        a.q_first[q] = q < a.n_queues ? (int)lo : 0;
        a.q_len[q] = q < a.n_queues ? (int)(hi - lo) : 0;
    }
    a.refill_threshold = c->tune.refill_threshold;
    a.tri_share = c->tune.tri_share;
    a.linear = (cfg->flags & LT_FLAG_LINEAR) ? 1 : 0;
    a.dir_order = -1;
    a.max_steps = 2 * c->n_nodes + 16;
    a.flags = c->d_flags;
    if (cfg->flags & LT_FLAG_PROPOSAL) {
        a.prop_pdf = c->prop_pdf;
        a.prop_cdf = c->prop_cdf;
        a.prop_guide = c->prop_guide;
        a.alpha_plain = cfg->alpha_plain;
    }
    a.inv_sigma = c->inv_sigma;
    return a;
}

// Run `body` directly on the context stream, or through a cached graph.
template <typename F>
int run_seq(lt_ctx* c, bool graph, const std::vector<uint64_t>& key, F body)
{
    if (!graph) {
        HIPCHK(c, body(c->stream));
        return LT_OK;
    }
    if (!c->gstream) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    }
    hipGraphExec_t exec = nullptr;
    for (auto& g : c->graphs)
        if (g.key == key) exec = g.exec;
    if (!exec) {
        hipGraph_t graph_h = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
        hipError_t e = body(c->gstream);
        hipError_t e2 = hipStreamEndCapture(c->gstream, &graph_h);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph_h) hipGraphDestroy(graph_h);
            return fail(c, LT_EHIP, std::string("graph capture failed: ") +
                                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipError_t e3 = hipGraphInstantiate(&exec, graph_h, nullptr, nullptr, 0);
        hipGraphDestroy(graph_h);
        if (e3 != hipSuccess) return fail(c, LT_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e3));
        if (c->graphs.size() >= 16) {
            hipStreamSynchronize(c->gstream);
            hipGraphExecDestroy(c->graphs.front().exec);
            c->graphs.erase(c->graphs.begin());
        }
        c->graphs.push_back(GraphEntry{key, exec});
    }
    HIPCHK(c, hipEventRecord(c->ev_in, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->gstream, c->ev_in, 0));
    HIPCHK(c, hipGraphLaunch(exec, c->gstream));
    HIPCHK(c, hipEventRecord(c->ev_out, c->gstream));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_out, 0));
    return LT_OK;
}

std::vector<uint64_t> make_key(lt_ctx* c, int kind, const lt_trace_cfg* cfg, std::initializer_list<const void*> ptrs)
{
    std::vector<uint64_t> k;
    k.push_back((uint64_t)kind);
    k.push_back(c->generation);
    k.push_back(cfg->seed);
    k.push_back((uint64_t)cfg->paths_per_layout);
    k.push_back((uint64_t)cfg->max_hits);
    k.push_back((uint64_t)cfg->flags);
    uint32_t ab;
    memcpy(&ab, &cfg->alpha_plain, 4);
    k.push_back((uint64_t)ab);
    k.push_back((uint64_t)c->tune.waves_per_block | ((uint64_t)c->tune.xcd_remap << 8) |
                ((uint64_t)c->tune.refill_threshold << 24) | ((uint64_t)c->tune.lds_depth << 40) |
                ((uint64_t)c->tune.tri_share << 56));
    k.push_back((uint64_t)c->tiles_tp);
    for (const void* p : ptrs) k.push_back((uint64_t)(uintptr_t)p);
    return k;
}

bool finite3(const float* v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

}  // namespace

extern "C" {

int lt_create(int device, void* hip_stream, lt_ctx** out)
{
    if (!out) return LT_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LT_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return LT_EHIP;
    lt_ctx* c = new lt_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->tune = default_tuning();
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0) {
        c->n_cu = prop.multiProcessorCount;
        if (prop.maxThreadsPerMultiProcessor >= 64) c->waves_per_cu = prop.maxThreadsPerMultiProcessor / 64;
        c->mem_total = prop.totalGlobalMem;
    }
    if (hipMalloc(&c->d_misses, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->d_flags, sizeof(unsigned)) != hipSuccess ||
        hipMalloc(&c->d_stats, sizeof(unsigned long long) * 8) != hipSuccess ||
        hipMalloc(&c->d_objpart, sizeof(double) * kObjBlocks) != hipSuccess ||
        hipMalloc(&c->d_queue, sizeof(unsigned) * 8) != hipSuccess) {
        lt_destroy(c);
        return LT_ENOMEM;
    }
    hipMemset(c->d_misses, 0, sizeof(unsigned long long));
    hipMemset(c->d_flags, 0, sizeof(unsigned));
    hipMemset(c->d_stats, 0, sizeof(unsigned long long) * 8);
    c->noalloc = (unsigned char*)scratch_address(device);
    hipDeviceSynchronize();
    *out = c;
    return LT_OK;
}

void lt_destroy(lt_ctx* c)
{
    if (!c) return;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    if (c->gstream) hipStreamSynchronize(c->gstream);
    free_graphs(c);
    free_scene(c);
    free_tiles(c);
    hipFree(c->d_si); hipFree(c->d_sf); hipFree(c->d_lights);
    hipFree(c->prop_pdf); hipFree(c->prop_cdf); hipFree(c->prop_guide); hipFree(c->inv_sigma); hipFree(c->mlp_scratch);
    free_net(c);
    hipFree(c->d_misses); hipFree(c->d_flags); hipFree(c->d_stats); hipFree(c->d_queue);
    hipFree(c->d_objpart); hipFree(c->d_partials); hipFree(c->d_gstack); hipFree(c->d_ptgrad);
    hipFree(c->d_partials_col); hipFree(c->d_partials7); hipFree(c->d_pfd);
    hipFree(c->d_partials8); hipFree(c->d_cone); hipFree(c->d_rec);
    if (c->ev_in) hipEventDestroy(c->ev_in);
    if (c->ev_out) hipEventDestroy(c->ev_out);
    if (c->gstream) hipStreamDestroy(c->gstream);
    delete c;
}

const char* lt_last_error(const lt_ctx* c) { return c ? c->err.c_str() : "null context"; }

int lt_set_stream(lt_ctx* c, void* hip_stream)
{
    if (!c) return LT_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return LT_OK;
}

int lt_sync(lt_ctx* c, uint32_t* flags_out)
{
    if (!c) return LT_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->gstream) HIPCHK(c, hipStreamSynchronize(c->gstream));
    unsigned f = 0;
    HIPCHK(c, hipMemcpy(&f, c->d_flags, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (f) HIPCHK(c, hipMemset(c->d_flags, 0, sizeof(unsigned)));
    if (flags_out) *flags_out = f;
    if (f & LT_STATUS_PARAMS)
        return fail(c, LT_EINVAL, "a luminaire parameter was not finite or its power not positive "
                                  "(that luminaire contributed nothing)");
    if (f & LT_STATUS_OVERFLOW) return fail(c, LT_EOVERFLOW, "texel accumulator overflow (|S| >= 2^62)");
    if (f & LT_STATUS_TRAVERSAL) return fail(c, LT_EHIP, "BVH traversal exceeded its step bound");
    return LT_OK;
}

int lt_scene_upload(lt_ctx* c, const float* h_verts, int64_t n_verts, const int32_t* h_tris,
                    const int32_t* h_tri_patch, int64_t n_tris, const lt_patch* h_patches, int32_t n_patches,
                    int64_t* n_texels_out)
{
    if (!c) return LT_EINVAL;
    if (!h_verts || !h_tris || !h_tri_patch || !h_patches) return fail(c, LT_EINVAL, "NULL scene array");
    if (n_verts < 3 || n_tris < 1 || n_patches < 1) return fail(c, LT_EINVAL, "empty scene");
    // the traversal addresses triangles (48 B) and nodes (64 B) by 32-bit byte offsets
    if (n_tris > (1ll << 26) || n_verts > (1ll << 31) - 1) return fail(c, LT_EINVAL, "scene too large");
    double amax = 0.0, lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < n_verts; ++v) {
        if (!finite3(h_verts + 3 * v)) return fail(c, LT_EINVAL, "non-finite vertex");
        for (int k = 0; k < 3; ++k) {
            const double x = h_verts[3 * v + k];
            amax = std::max(amax, fabs(x));
            lo[k] = std::min(lo[k], x);
            hi[k] = std::max(hi[k], x);
        }
    }
    // an axis-parallel ray's reciprocal direction is up to 1e30; the slab
    // test's products with coordinates must stay finite
    if (amax > 1e8) return fail(c, LT_EINVAL, "vertex coordinates beyond 1e8 in magnitude");
    for (int64_t t = 0; t < n_tris; ++t) {
        for (int k = 0; k < 3; ++k)
            if (h_tris[3 * t + k] < 0 || h_tris[3 * t + k] >= n_verts)
                return fail(c, LT_EINVAL, "triangle vertex index out of range");
        if (h_tri_patch[t] < 0 || h_tri_patch[t] >= n_patches)
            return fail(c, LT_EINVAL, "triangle patch index out of range");
    }
    std::vector<DevPatch> dp(n_patches);
    std::vector<long long> base(n_patches);
    std::vector<float> area(n_patches);
    long long K = 0;
    for (int q = 0; q < n_patches; ++q) {
        const lt_patch& p = h_patches[q];
        if (p.res_u < 1 || p.res_v < 1) return fail(c, LT_EINVAL, "patch resolution < 1");
        if (p.texel_base != K) return fail(c, LT_EINVAL, "patch texel ranges must tile [0, K) in order");
        if (!finite3(p.origin) || !finite3(p.e_u) || !finite3(p.e_v) || !finite3(p.normal) ||
            !(p.inv_len2_u > 0) || !(p.inv_len2_v > 0) || !isfinite(p.inv_len2_u) || !isfinite(p.inv_len2_v) ||
            !(p.texel_area > 0) || !(p.inv_texel_area > 0) || !isfinite(p.inv_texel_area) ||
            !(p.albedo >= 0.0f && p.albedo <= 1.0f))
            return fail(c, LT_EINVAL, "invalid patch constants");
        K += (long long)p.res_u * p.res_v;
        dp[q].o_inva = make_float4(p.origin[0], p.origin[1], p.origin[2], p.inv_texel_area);
        dp[q].eu_ilu = make_float4(p.e_u[0], p.e_u[1], p.e_u[2], p.inv_len2_u);
        dp[q].ev_ilv = make_float4(p.e_v[0], p.e_v[1], p.e_v[2], p.inv_len2_v);
        dp[q].n_rho = make_float4(p.normal[0], p.normal[1], p.normal[2], p.albedo);
        dp[q].res_u = p.res_u;
        dp[q].res_v = p.res_v;
        dp[q].base = p.texel_base;
        base[q] = p.texel_base;
        area[q] = p.texel_area;
    }
    if (K > 0x7fffffffll) return fail(c, LT_EINVAL, "more than 2^31-1 texels");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_graphs(c);
    free_scene(c);
    float* d_verts = nullptr;
    int *d_tris = nullptr, *d_tp = nullptr;
    HIPCHK(c, hipMalloc(&d_verts, sizeof(float) * 3 * n_verts));
    HIPCHK(c, hipMalloc(&d_tris, sizeof(int) * 3 * n_tris));
    HIPCHK(c, hipMalloc(&d_tp, sizeof(int) * n_tris));
    HIPCHK(c, hipMemcpy(d_verts, h_verts, sizeof(float) * 3 * n_verts, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(d_tris, h_tris, sizeof(int) * 3 * n_tris, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(d_tp, h_tri_patch, sizeof(int) * n_tris, hipMemcpyHostToDevice));
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k]);
    const float pad = (float)(1e-5 * (amax + ext + 1.0));
    int depth = 0, n_nodes = 0;
    hipError_t e = build_bvh(d_verts, d_tris, d_tp, (int)n_tris, pad, c->stream, &c->nodes, &c->tris, &n_nodes, &depth);
    hipFree(d_verts);
    hipFree(d_tris);
    hipFree(d_tp);
    if (e != hipSuccess) return fail(c, LT_EHIP, std::string("BVH build: ") + hipGetErrorString(e));
    if (3 * depth + 1 > kMaxStackDepth) {
        free_scene(c);
        return fail(c, LT_EINVAL, "BVH deeper than the traversal stack bound");
    }
    if ((long long)n_nodes * 16 * kNodeRows > (1ll << 32)) {
        free_scene(c);
        return fail(c, LT_EINVAL, "BVH larger than 2^32 bytes");
    }
    HIPCHK(c, hipMalloc(&c->patches, sizeof(DevPatch) * n_patches));
    HIPCHK(c, hipMalloc(&c->pbase, sizeof(long long) * n_patches));
    HIPCHK(c, hipMalloc(&c->parea, sizeof(float) * n_patches));
    HIPCHK(c, hipMalloc(&c->texel_area, sizeof(float) * K));
    HIPCHK(c, hipMemcpy(c->patches, dp.data(), sizeof(DevPatch) * n_patches, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->pbase, base.data(), sizeof(long long) * n_patches, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->parea, area.data(), sizeof(float) * n_patches, hipMemcpyHostToDevice));
    {
        // colour mode: every channel takes the patch's albedo until set otherwise
        std::vector<float4> rr(n_patches);
        for (int q = 0; q < n_patches; ++q) rr[q] = make_float4(h_patches[q].albedo, h_patches[q].albedo, h_patches[q].albedo, 0.f);
        HIPCHK(c, hipMalloc(&c->rho_rgb, sizeof(float4) * n_patches));
        HIPCHK(c, hipMemcpy(c->rho_rgb, rr.data(), sizeof(float4) * n_patches, hipMemcpyHostToDevice));
        // directional mode: Lambertian until set otherwise
        std::vector<float2> gg(n_patches, make_float2(0.0f, 1.0f));
        HIPCHK(c, hipMalloc(&c->glossy, sizeof(float2) * n_patches));
        HIPCHK(c, hipMemcpy(c->glossy, gg.data(), sizeof(float2) * n_patches, hipMemcpyHostToDevice));
    }
    HIPCHK(c, launch_texel_area(c->parea, c->pbase, n_patches, K, c->texel_area, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->n_nodes = n_nodes;
    c->depth = depth;
    c->n_tris = n_tris;
    c->n_patches = n_patches;
    c->K = K;
    c->has_scene = true;
    c->generation++;
    if (n_texels_out) *n_texels_out = K;
    return LT_OK;
}

int lt_set_lights(lt_ctx* c, const lt_light_static* h_lights, int32_t n_lights, const int32_t* h_offs,
                  int32_t n_layouts)
{
    if (!c) return LT_EINVAL;
    if (!h_lights || !h_offs || n_lights < 1 || n_layouts < 1) return fail(c, LT_EINVAL, "no luminaires");
    if (n_layouts > 65535 || n_lights > (1 << 24)) return fail(c, LT_EINVAL, "too many layouts or lights");
    if (h_offs[0] != 0 || h_offs[n_layouts] != n_lights) return fail(c, LT_EINVAL, "bad layout offsets");
    for (int j = 0; j < n_layouts; ++j) {
        if (h_offs[j + 1] <= h_offs[j]) return fail(c, LT_EINVAL, "empty layout or unordered offsets");
        if (h_offs[j + 1] - h_offs[j] > 65535) return fail(c, LT_EINVAL, "too many lights in a layout");
    }
    std::vector<int4> si(n_lights);
    std::vector<float4> sf(n_lights);
    for (int j = 0; j < n_layouts; ++j)
        for (int l = h_offs[j]; l < h_offs[j + 1]; ++l) {
            const lt_light_static& s = h_lights[l];
            if (s.type < 0 || s.type > 3) return fail(c, LT_EINVAL, "unknown light type");
            if (s.layout != j) return fail(c, LT_EINVAL, "light layout does not match the offsets");
            if (!(s.lobe_n >= 0.0f) || !isfinite(s.lobe_n) || ((s.type == 0 || s.type == 3) && s.lobe_n != 0.0f))
                return fail(c, LT_EINVAL, "invalid lobe exponent");
            if (s.type == 3 && !(s.size_w >= 0.0f && s.size_h > s.size_w && s.size_h <= 1.5707963f))
                return fail(c, LT_EINVAL, "soft-edged spot needs 0 <= inner < outer <= pi/2");
            if (s.type == 2 && !(s.size_w > 0.0f && s.size_h > 0.0f && isfinite(s.size_w) && isfinite(s.size_h)))
                return fail(c, LT_EINVAL, "invalid rectangle size");
            si[l] = make_int4(s.type, j, l - h_offs[j], h_offs[j + 1] - h_offs[j]);
            sf[l] = make_float4(s.lobe_n, s.size_w, s.size_h, 0.f);
        }
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_graphs(c);
    free_tiles(c);
    hipFree(c->d_si); hipFree(c->d_sf); hipFree(c->d_lights);
    hipFree(c->prop_pdf); hipFree(c->prop_cdf); hipFree(c->prop_guide); hipFree(c->inv_sigma);
    c->d_si = nullptr; c->d_sf = nullptr; c->d_lights = nullptr;
    c->prop_pdf = nullptr; c->prop_cdf = nullptr; c->prop_guide = nullptr; c->inv_sigma = nullptr;
    free_net(c);
    c->has_lights = false;
    c->has_proposal = false;
    HIPCHK(c, hipMalloc(&c->d_si, sizeof(int4) * n_lights));
    HIPCHK(c, hipMalloc(&c->d_sf, sizeof(float4) * n_lights));
    HIPCHK(c, hipMalloc(&c->d_lights, sizeof(DevLight) * n_lights));
    HIPCHK(c, hipMemcpy(c->d_si, si.data(), sizeof(int4) * n_lights, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_sf, sf.data(), sizeof(float4) * n_lights, hipMemcpyHostToDevice));
    HIPCHK(c, hipMalloc(&c->prop_pdf, sizeof(float) * 1024 * (size_t)n_lights));
    HIPCHK(c, hipMalloc(&c->prop_cdf, sizeof(float) * 1024 * (size_t)n_lights));
    HIPCHK(c, hipMalloc(&c->prop_guide, sizeof(int) * 1025 * (size_t)n_lights));
    HIPCHK(c, hipMalloc(&c->inv_sigma, sizeof(float) * 6 * (size_t)n_lights));
    {
        std::vector<float> ones(6 * (size_t)n_lights, 1.0f);
        HIPCHK(c, hipMemcpy(c->inv_sigma, ones.data(), sizeof(float) * ones.size(), hipMemcpyHostToDevice));
    }
    c->lights.assign(h_lights, h_lights + n_lights);
    c->offs.assign(h_offs, h_offs + n_layouts + 1);
    c->L = n_lights;
    c->n_layouts = n_layouts;
    c->has_lights = true;
    c->generation++;
    return LT_OK;
}

int lt_trace_forward(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int64_t* d_S, float* d_E)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_S || !d_E) return fail(c, LT_EINVAL, "NULL device buffer");
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_E & 7) || ((uintptr_t)d_params & 3))
        return fail(c, LT_EINVAL, "d_S must be 16-byte and d_E 8-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.S = (long long*)d_S;
    const long long n = c->K * c->n_layouts;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess) e = launch_clear(a.S, n, st);
        if (e == hipSuccess) e = timed_trace(c, false, graph, a, st);
        if (e == hipSuccess) e = launch_finalize(a.S, d_E, n, c->d_flags, st);
        return e;
    };
    return run_seq(c, graph, make_key(c, 1, cfg, {d_params, d_S, d_E}), body);
}

int lt_objective(lt_ctx* c, const float* d_E, const float* d_Et, const float* d_alpha, int64_t n, double* d_O,
                 float* d_g)
{
    if (!c) return LT_EINVAL;
    if (!c->has_scene) return fail(c, LT_ESTATE, "no scene uploaded");
    if (!d_E || !d_Et || !d_O) return fail(c, LT_EINVAL, "NULL device buffer");
    if (n <= 0 || n % c->K != 0) return fail(c, LT_EINVAL, "n must be a positive multiple of the texel count");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_objective(d_E, d_Et, d_alpha, c->texel_area, c->K, n, d_g, c->d_objpart, d_O, c->stream));
    return LT_OK;
}

int lt_trace_adjoint(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE, float* d_grad,
                     float* d_bin_hist)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_dOdE || !d_grad) return fail(c, LT_EINVAL, "NULL device buffer");
    if (d_bin_hist && ((uintptr_t)d_bin_hist & 15)) return fail(c, LT_EINVAL, "d_bin_hist must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.g = d_dOdE;
    a.partials = c->d_partials;
    a.bin_hist = d_bin_hist;
    // in the box basis, below 2^30 paths per layout (a luminaire's records
    // then lie within 32-bit byte offsets) and within the record budget the
    // adjoint runs in two passes:
    // the trace records each path's first hit and adjoint sum, a second
    // kernel forms the paths' contributions, the tiles' sums and the
    // training histogram
    const bool two_pass = !(cfg->flags & LT_FLAG_LINEAR) && cfg->paths_per_layout < (1ll << 30) && rec_fits(c);
    if (two_pass) {
        rc = ensure_rec(c);
        if (rc) return rc;
        a.rec = c->d_rec;
        a.rec_stride = c->rec_paths;
        a.rec_base = c->d_rec_base;
    }
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess && d_bin_hist) e = launch_fill_f32(d_bin_hist, (long long)c->L * 1024, 0.0f, st);
        if (e == hipSuccess) e = timed_trace(c, true, graph, a, st);
        if (e == hipSuccess && two_pass) e = launch_rec_grad(a, c->d_partials, st);
        if (e == hipSuccess) e = launch_grad_reduce(c->d_partials, c->d_range, c->L, d_grad, st);
        return e;
    };
    return run_seq(c, graph, make_key(c, 2, cfg, {d_params, d_dOdE, d_grad, d_bin_hist}), body);
}

int lt_trace_adjoint_noalloc(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE,
                             float* d_grad)
{
    if (!c) return LT_EINVAL;
    if (!cfg) return fail(c, LT_EINVAL, "cfg is NULL");
    if (!c->has_scene) return fail(c, LT_ESTATE, "no scene uploaded");
    if (!c->has_lights) return fail(c, LT_ESTATE, "no luminaires set");
    if (!d_params || !d_dOdE || !d_grad) return fail(c, LT_EINVAL, "NULL device buffer");
    if (cfg->max_hits < 1 || cfg->max_hits > 64) return fail(c, LT_EINVAL, "max_hits must be in [1, 64]");
    if (cfg->flags & ~(LT_FLAG_PROPOSAL | LT_FLAG_LINEAR))
        return fail(c, LT_EINVAL, "unknown flag (graph replay allocates; it is not available here)");
    if (cfg->flags & LT_FLAG_PROPOSAL) {
        if (!c->has_proposal) return fail(c, LT_EINVAL, "no emission proposal loaded");
        if (!(cfg->alpha_plain > 0.0f && cfg->alpha_plain <= 1.0f))
            return fail(c, LT_EINVAL, "alpha_plain must be in (0, 1] (defensive mixture)");
    }
    if (!c->noalloc) return fail(c, LT_EHIP, "no scratch address for this device");
    // the tile table, counted on the host without storing it
    const long long ppl = cfg->paths_per_layout;
    const int tp = effective_tile_paths(c, ppl);
    long long n_tiles = 0;
    for (int j = 0; j < c->n_layouts; ++j) {
        const int nl = c->offs[j + 1] - c->offs[j];
        if (ppl < nl) return fail(c, LT_EINVAL, "paths_per_layout smaller than the number of lights of a layout");
        for (int l = 0; l < nl; ++l) {
            const long long n = paths_of_light(ppl, nl, l);
            if (n > 0xFFFFFFFFll) return fail(c, LT_EINVAL, "more than 2^32 paths for one light");
            n_tiles += (n + tp - 1) / tp;
        }
    }
    // scratch layout, every region 256-byte aligned
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_queue = off;
    off += up(sizeof(unsigned) * 8);
    const size_t o_tiles = off;
    off += up(sizeof(int4) * (size_t)n_tiles);
    const size_t o_range = off;
    off += up(sizeof(int2) * (size_t)c->L);
    const size_t o_np = off;
    off += up(sizeof(long long) * (size_t)c->L);
    const size_t o_part = off;
    off += up(sizeof(double) * 6 * (size_t)n_tiles);
    const size_t o_stack = off;
    const int gdepth = std::max(gstack_depth(c), 1);
    const size_t per_wave = sizeof(int) * (size_t)gdepth * 64;
    const long long waves = off < kNoAllocBytes ? std::min<long long>((long long)((kNoAllocBytes - off) / per_wave),
                                                                     resident_waves(c))
                                                : 0;
    if (waves < 64)
        return fail(c, LT_EINVAL,
                    "workload too large for the no-allocation scratch (" + std::to_string(kNoAllocBytes >> 20) +
                        " MiB: work tiles, partial sums and stack overflow for at least 64 waves); use "
                        "lt_trace_adjoint");
    HIPCHK(c, hipSetDevice(c->device));
    unsigned char* base = c->noalloc;
    TraceArgs a = trace_args(c, cfg);
    a.g = d_dOdE;
    a.tiles = (const int4*)(base + o_tiles);
    a.n_tiles = (int)n_tiles;
    a.partials = (double*)(base + o_part);
    a.bin_hist = nullptr;
    a.gstack = (int*)(base + o_stack);
    a.gdepth = gdepth;
    a.gstack_waves = waves;
    a.queue = (unsigned*)(base + o_queue);
    for (int q = 0; q < 8; ++q) {
        const long long lo = n_tiles * q / a.n_queues, hi = n_tiles * (q + 1) / a.n_queues;
        a.q_first[q] = q < a.n_queues ? (int)lo : 0;
        a.q_len[q] = q < a.n_queues ? (int)(hi - lo) : 0;
    }
    int2* range = (int2*)(base + o_range);
    long long* npaths = (long long*)(base + o_np);
    hipStream_t st = c->stream;
    HIPCHK(c, launch_build_tiles(c->d_si, c->L, ppl, tp, (int)n_tiles, (int4*)(base + o_tiles), range, npaths, st));
    HIPCHK(c, launch_light_setup(d_params, c->d_si, c->d_sf, npaths, c->L, c->d_lights, c->d_flags, st));
    HIPCHK(c, launch_trace(true, false, a, c->tune.waves_per_block, c->tune.lds_depth, c->n_cu, st));
    HIPCHK(c, launch_grad_reduce(a.partials, range, c->L, d_grad, st));
    return LT_OK;
}

int lt_gradient_votes(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE,
                      int32_t light, int32_t param, double* d_vote, float* d_grad)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_dOdE || !d_grad || !d_vote) return fail(c, LT_EINVAL, "NULL device buffer");
    if ((uintptr_t)d_vote & 15) return fail(c, LT_EINVAL, "d_vote must be 16-byte aligned");
    if (light < 0 || light >= c->L) return fail(c, LT_EINVAL, "light out of range");
    if (param < 0 || param > 5) return fail(c, LT_EINVAL, "parameter out of range");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.g = d_dOdE;
    a.partials = c->d_partials;
    a.vote = d_vote;
    a.vote_light = light;
    a.vote_param = param;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess) e = launch_clear((long long*)d_vote, c->K, st);
        if (e == hipSuccess) e = timed_trace(c, true, graph, a, st);
        if (e == hipSuccess) e = launch_grad_reduce(c->d_partials, c->d_range, c->L, d_grad, st);
        return e;
    };
    return run_seq(c, graph,
                   make_key(c, 4, cfg, {d_params, d_dOdE, d_grad, d_vote, (const void*)(uintptr_t)(light * 8 + param)}),
                   body);
}

int lt_set_albedo_rgb(lt_ctx* c, const float* h_albedo)
{
    if (!c) return LT_EINVAL;
    if (!c->has_scene) return fail(c, LT_ESTATE, "no scene uploaded");
    if (!h_albedo) return fail(c, LT_EINVAL, "NULL albedo table");
    std::vector<float4> rr(c->n_patches);
    for (int q = 0; q < c->n_patches; ++q) {
        const float* a = h_albedo + 3 * (size_t)q;
        for (int ch = 0; ch < 3; ++ch)
            if (!(a[ch] >= 0.0f && a[ch] <= 1.0f)) return fail(c, LT_EINVAL, "albedo outside [0, 1]");
        rr[q] = make_float4(a[0], a[1], a[2], 0.f);
    }
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->rho_rgb, rr.data(), sizeof(float4) * c->n_patches, hipMemcpyHostToDevice));
    free_graphs(c);
    return LT_OK;
}

int lt_trace_forward_rgb(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, const float* d_colour,
                         int64_t* d_S, float* d_E)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_colour || !d_S || !d_E) return fail(c, LT_EINVAL, "NULL device buffer");
    if (cfg->flags & LT_FLAG_LINEAR) return fail(c, LT_EINVAL, "colour mode takes the box basis only");
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_E & 7) || ((uintptr_t)d_params & 3) || ((uintptr_t)d_colour & 3))
        return fail(c, LT_EINVAL, "d_S must be 16-byte and d_E 8-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.S = (long long*)d_S;
    a.rgb = 1;
    a.colour = d_colour;
    a.rho_rgb = c->rho_rgb;
    const long long n = 3 * c->K * c->n_layouts;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess) e = launch_clear(a.S, n, st);
        if (e == hipSuccess) e = timed_trace(c, false, graph, a, st);
        if (e == hipSuccess) e = launch_finalize(a.S, d_E, n, c->d_flags, st);
        return e;
    };
    return run_seq(c, graph, make_key(c, 5, cfg, {d_params, d_colour, d_S, d_E}), body);
}

int lt_trace_adjoint_rgb(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, const float* d_colour,
                         const float* d_dOdE, float* d_grad, float* d_grad_colour, float* d_bin_hist)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_colour || !d_dOdE || !d_grad || !d_grad_colour)
        return fail(c, LT_EINVAL, "NULL device buffer");
    if (cfg->flags & LT_FLAG_LINEAR) return fail(c, LT_EINVAL, "colour mode takes the box basis only");
    if (d_bin_hist && ((uintptr_t)d_bin_hist & 15)) return fail(c, LT_EINVAL, "d_bin_hist must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    const size_t need = (size_t)std::max(c->n_tiles, 1) * 3;
    if (c->partials_col_cap < need) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        free_graphs(c);
        hipFree(c->d_partials_col);
        c->d_partials_col = nullptr;
        c->partials_col_cap = 0;
        HIPCHK(c, hipMalloc(&c->d_partials_col, sizeof(double) * need));
        c->partials_col_cap = need;
    }
    TraceArgs a = trace_args(c, cfg);
    a.g = d_dOdE;
    a.partials = c->d_partials;
    a.bin_hist = d_bin_hist;
    a.rgb = 1;
    a.colour = d_colour;
    a.rho_rgb = c->rho_rgb;
    a.partials_col = c->d_partials_col;
    // two passes as the grey adjoint's (below 2^30 paths per layout)
    const bool two_pass = cfg->paths_per_layout < (1ll << 30) && rec_fits(c);
    if (two_pass) {
        rc = ensure_rec(c);
        if (rc) return rc;
        a.rec = c->d_rec;
        a.rec_stride = c->rec_paths;
        a.rec_base = c->d_rec_base;
    }
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess && d_bin_hist) e = launch_fill_f32(d_bin_hist, (long long)c->L * 1024, 0.0f, st);
        if (e == hipSuccess) e = timed_trace(c, true, graph, a, st);
        if (e == hipSuccess && two_pass) e = launch_rec_grad(a, c->d_partials, st);
        if (e == hipSuccess) e = launch_grad_reduce(c->d_partials, c->d_range, c->L, d_grad, st);
        if (e == hipSuccess) e = launch_grad_reduce_col(c->d_partials_col, c->d_range, c->L, d_grad_colour, st);
        return e;
    };
    return run_seq(c, graph, make_key(c, 6, cfg, {d_params, d_colour, d_dOdE, d_grad, d_grad_colour, d_bin_hist}),
                   body);
}

int lt_trace_tangent(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int32_t light, int32_t param,
                     int64_t* d_T, float* d_D)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_T || !d_D) return fail(c, LT_EINVAL, "NULL device buffer");
    if (cfg->flags & (LT_FLAG_PROPOSAL | LT_FLAG_LINEAR))
        return fail(c, LT_EINVAL, "the direct-differentiation map takes the plain emission and the box basis only");
    if (light < 0 || light >= c->L) return fail(c, LT_EINVAL, "light out of range");
    if (param < 0 || param > 5) return fail(c, LT_EINVAL, "parameter out of range");
    if (((uintptr_t)d_T & 15) || ((uintptr_t)d_D & 7)) return fail(c, LT_EINVAL, "d_T must be 16-byte and d_D 8-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.tangent = (long long*)d_T;
    a.tan_light = light;
    a.tan_param = param;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess) e = launch_clear(a.tangent, c->K, st);
        if (e == hipSuccess) e = timed_trace(c, false, graph, a, st);
        if (e == hipSuccess) e = launch_finalize(a.tangent, d_D, c->K, c->d_flags, st);
        return e;
    };
    return run_seq(c, graph,
                   make_key(c, 11, cfg, {d_params, d_T, d_D, (const void*)(uintptr_t)(light * 8 + param)}), body);
}

int lt_fd_map(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int32_t light, int32_t param, float h,
              int64_t* d_Sp, int64_t* d_Sm, float* d_F)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_Sp || !d_Sm || !d_F) return fail(c, LT_EINVAL, "NULL device buffer");
    if (cfg->flags & (LT_FLAG_PROPOSAL | LT_FLAG_LINEAR))
        return fail(c, LT_EINVAL, "the central-difference map takes the plain emission and the box basis only");
    if (light < 0 || light >= c->L) return fail(c, LT_EINVAL, "light out of range");
    if (param < 0 || param > 5) return fail(c, LT_EINVAL, "parameter out of range");
    if (!(h > 0.0f) || !__builtin_isfinite(h)) return fail(c, LT_EINVAL, "h must be positive and finite");
    if (((uintptr_t)d_Sp & 15) || ((uintptr_t)d_Sm & 15) || ((uintptr_t)d_params & 3))
        return fail(c, LT_EINVAL, "d_Sp and d_Sm must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    if (c->pfd_cap < c->L) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        free_graphs(c);
        hipFree(c->d_pfd);
        c->d_pfd = nullptr;
        c->pfd_cap = 0;
        HIPCHK(c, hipMalloc(&c->d_pfd, sizeof(float) * 12 * c->L + 16));
        c->pfd_cap = c->L;
    }
    float* pp = c->d_pfd;
    float* pm = c->d_pfd + 6 * c->pfd_cap;
    double* den = (double*)(c->d_pfd + 12 * c->pfd_cap);   // 48 L bytes in: 16-byte aligned
    int layout = 0;
    while (c->offs[layout + 1] <= light) ++layout;
    const long long n = c->K * c->n_layouts;
    const long long row = (long long)layout * c->K;
    TraceArgs ap = trace_args(c, cfg), am = trace_args(c, cfg);
    ap.S = (long long*)d_Sp;
    am.S = (long long*)d_Sm;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_fd_params(d_params, 6 * c->L, 6 * light + param, h, pp, pm, den, st);
        if (e == hipSuccess) e = launch_light_setup(pp, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess) e = launch_clear(ap.S, n, st);
        if (e == hipSuccess) e = timed_trace(c, false, graph, ap, st);
        if (e == hipSuccess) e = launch_light_setup(pm, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess) e = launch_clear(am.S, n, st);
        if (e == hipSuccess) e = timed_trace(c, false, graph, am, st);
        if (e == hipSuccess) e = launch_fd_diff(ap.S + row, am.S + row, c->K, den, d_F, st);
        return e;
    };
    return run_seq(c, graph,
                   make_key(c, 12, cfg, {d_params, d_Sp, d_Sm, d_F, (const void*)(uintptr_t)(light * 8 + param),
                                         (const void*)(uintptr_t)__builtin_bit_cast(uint32_t, h)}),
                   body);
}

int lt_trace_forward_rv(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int64_t* d_S, float* d_E)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_S || !d_E) return fail(c, LT_EINVAL, "NULL device buffer");
    if (cfg->flags & (LT_FLAG_PROPOSAL | LT_FLAG_LINEAR))
        return fail(c, LT_EINVAL, "rotation vectors take the plain emission and the box basis only");
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_E & 7) || ((uintptr_t)d_params & 3))
        return fail(c, LT_EINVAL, "d_S must be 16-byte and d_E 8-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.S = (long long*)d_S;
    const long long n = c->K * c->n_layouts;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st, 1);
        if (e == hipSuccess) e = launch_clear(a.S, n, st);
        if (e == hipSuccess) e = timed_trace(c, false, graph, a, st);
        if (e == hipSuccess) e = launch_finalize(a.S, d_E, n, c->d_flags, st);
        return e;
    };
    return run_seq(c, graph, make_key(c, 9, cfg, {d_params, d_S, d_E}), body);
}

int lt_trace_adjoint_rv(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE, float* d_grad)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_dOdE || !d_grad) return fail(c, LT_EINVAL, "NULL device buffer");
    if (cfg->flags & (LT_FLAG_PROPOSAL | LT_FLAG_LINEAR))
        return fail(c, LT_EINVAL, "rotation vectors take the plain emission and the box basis only");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    const size_t need = (size_t)std::max(c->n_tiles, 1) * 7;
    if (c->partials7_cap < need) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        free_graphs(c);
        hipFree(c->d_partials7);
        c->d_partials7 = nullptr;
        c->partials7_cap = 0;
        HIPCHK(c, hipMalloc(&c->d_partials7, sizeof(double) * need));
        c->partials7_cap = need;
    }
    TraceArgs a = trace_args(c, cfg);
    a.g = d_dOdE;
    a.partials = c->d_partials7;
    a.rotvec = 1;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st, 1);
        if (e == hipSuccess) e = timed_trace(c, true, graph, a, st);
        if (e == hipSuccess) e = launch_grad_reduce_rv(c->d_partials7, c->d_range, d_params, c->L, d_grad, st);
        return e;
    };
    return run_seq(c, graph, make_key(c, 10, cfg, {d_params, d_dOdE, d_grad}), body);
}

int lt_trace_adjoint_cone(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, const float* d_dOdE,
                          float* d_grad, float* d_grad_cone)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_dOdE || !d_grad || !d_grad_cone) return fail(c, LT_EINVAL, "NULL device buffer");
    if (cfg->flags & (LT_FLAG_PROPOSAL | LT_FLAG_LINEAR))
        return fail(c, LT_EINVAL, "cone-angle gradients take the plain emission and the box basis only");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    const size_t need = (size_t)std::max(c->n_tiles, 1) * 8;
    if (c->partials8_cap < need || c->cone_cap < c->L) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        free_graphs(c);
        if (c->partials8_cap < need) {
            hipFree(c->d_partials8);
            c->d_partials8 = nullptr;
            c->partials8_cap = 0;
            HIPCHK(c, hipMalloc(&c->d_partials8, sizeof(double) * need));
            c->partials8_cap = need;
        }
        if (c->cone_cap < c->L) {
            hipFree(c->d_cone);
            c->d_cone = nullptr;
            c->cone_cap = 0;
            HIPCHK(c, hipMalloc(&c->d_cone, sizeof(float) * 5 * c->L));
            c->cone_cap = c->L;
        }
    }
    TraceArgs a = trace_args(c, cfg);
    a.g = d_dOdE;
    a.partials = c->d_partials8;
    a.cone = c->d_cone;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e =
            launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st, 0, c->d_cone);
        if (e == hipSuccess) e = timed_trace(c, true, graph, a, st);
        if (e == hipSuccess)
            e = launch_grad_reduce_cone(c->d_partials8, c->d_range, c->L, d_grad, d_grad_cone, st);
        return e;
    };
    return run_seq(c, graph, make_key(c, 13, cfg, {d_params, d_dOdE, d_grad, d_grad_cone}), body);
}

int lt_set_glossy(lt_ctx* c, const float* h_glossy)
{
    if (!c) return LT_EINVAL;
    if (!c->has_scene) return fail(c, LT_ESTATE, "no scene uploaded");
    if (!h_glossy) return fail(c, LT_EINVAL, "NULL glossy table");
    std::vector<float2> gg(c->n_patches);
    for (int q = 0; q < c->n_patches; ++q) {
        const float rs = h_glossy[2 * (size_t)q], e = h_glossy[2 * (size_t)q + 1];
        if (!(rs >= 0.0f && rs <= 1.0f) || !(e >= 0.0f && e <= 1e4f))
            return fail(c, LT_EINVAL, "specular albedo outside [0, 1] or exponent outside [0, 1e4]");
        gg[q] = make_float2(rs, e);
    }
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->glossy, gg.data(), sizeof(float2) * c->n_patches, hipMemcpyHostToDevice));
    return LT_OK;
}

namespace {

int dir_check(lt_ctx* c, const lt_trace_cfg* cfg, int32_t order, int32_t samples)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (order < 0 || order > 3) return fail(c, LT_EINVAL, "hemispherical-harmonic order must be 0 to 3");
    if (samples < 1 || samples > 64) return fail(c, LT_EINVAL, "local samples per hit must be in [1, 64]");
    if (cfg->flags & LT_FLAG_LINEAR) return fail(c, LT_EINVAL, "directional texels take the box basis only");
    if (cfg->max_hits > 64) return fail(c, LT_EINVAL, "max_hits too large for the local-sample counters");
    return LT_OK;
}

}  // namespace

int lt_trace_forward_dir(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int32_t order, int32_t samples,
                         int64_t* d_S, float* d_E)
{
    int rc = dir_check(c, cfg, order, samples);
    if (rc) return rc;
    if (!d_params || !d_S || !d_E) return fail(c, LT_EINVAL, "NULL device buffer");
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_E & 7) || ((uintptr_t)d_params & 3))
        return fail(c, LT_EINVAL, "d_S must be 16-byte and d_E 8-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.S = (long long*)d_S;
    a.dir_order = order;
    a.dir_samples = samples;
    a.glossy = c->glossy;
    const long long n = (long long)(order + 1) * (order + 1) * c->K * c->n_layouts;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess) e = launch_clear(a.S, n, st);
        if (e == hipSuccess) e = timed_trace(c, false, graph, a, st);
        if (e == hipSuccess) e = launch_finalize(a.S, d_E, n, c->d_flags, st);
        return e;
    };
    return run_seq(c, graph, make_key(c, 7, cfg, {d_params, d_S, d_E, (const void*)(uintptr_t)(order * 256 + samples)}),
                   body);
}

int lt_trace_adjoint_dir(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int32_t order, int32_t samples,
                         const float* d_dOdE, float* d_grad, float* d_bin_hist)
{
    int rc = dir_check(c, cfg, order, samples);
    if (rc) return rc;
    if (!d_params || !d_dOdE || !d_grad) return fail(c, LT_EINVAL, "NULL device buffer");
    if (d_bin_hist && ((uintptr_t)d_bin_hist & 15)) return fail(c, LT_EINVAL, "d_bin_hist must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.g = d_dOdE;
    a.partials = c->d_partials;
    a.bin_hist = d_bin_hist;
    a.dir_order = order;
    a.dir_samples = samples;
    a.glossy = c->glossy;
    const bool graph = (cfg->flags & LT_FLAG_GRAPH) != 0;
    auto body = [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st);
        if (e == hipSuccess && d_bin_hist) e = launch_fill_f32(d_bin_hist, (long long)c->L * 1024, 0.0f, st);
        if (e == hipSuccess) e = timed_trace(c, true, graph, a, st);
        if (e == hipSuccess) e = launch_grad_reduce(c->d_partials, c->d_range, c->L, d_grad, st);
        return e;
    };
    return run_seq(c, graph,
                   make_key(c, 8, cfg, {d_params, d_dOdE, d_grad, d_bin_hist, (const void*)(uintptr_t)(order * 256 + samples)}),
                   body);
}

namespace {

int pt_check(lt_ctx* c, const lt_trace_cfg* cfg, int32_t samples_per_texel)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (cfg->flags != 0) return fail(c, LT_EINVAL, "the path tracer takes no flags");
    if (samples_per_texel < 1) return fail(c, LT_EINVAL, "samples_per_texel must be >= 1");
    if (c->K * (long long)samples_per_texel > 0xFFFFFFFFll)
        return fail(c, LT_EINVAL, "more than 2^32 samples per layout");
    for (int j = 0; j < c->n_layouts; ++j)
        if (c->offs[j + 1] - c->offs[j] > kPtMaxLights)
            return fail(c, LT_EINVAL, "the path tracer takes at most 256 luminaires per layout");
    return ensure_gstack(c, (long long)kPtBlocks * 4);
}

PtArgs pt_args(lt_ctx* c, const lt_trace_cfg* cfg, int32_t samples_per_texel, int j)
{
    PtArgs a;
    memset(&a, 0, sizeof(a));
    a.nodes = c->nodes;
    a.tris = c->tris;
    a.patches = c->patches;
    a.pbase = c->pbase;
    a.n_patches = c->n_patches;
    a.lights = c->d_lights + c->offs[j];
    a.nl = c->offs[j + 1] - c->offs[j];
    a.layout = j;
    a.K = c->K;
    a.M = samples_per_texel;
    a.max_hits = cfg->max_hits;
    a.key0 = (uint32_t)cfg->seed;
    a.key1 = (uint32_t)(cfg->seed >> 32);
    a.gstack = c->d_gstack;
    a.gdepth = std::max(gstack_depth(c), 1);
    a.max_steps = 2 * c->n_nodes + 16;
    a.flags = c->d_flags;
    return a;
}

}  // namespace

int lt_pt_forward(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int32_t samples_per_texel, int64_t* d_S,
                  float* d_E)
{
    if (!c) return LT_EINVAL;
    if (!d_params || !d_S || !d_E) return fail(c, LT_EINVAL, "NULL device buffer");
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_E & 7) || ((uintptr_t)d_params & 3))
        return fail(c, LT_EINVAL, "d_S must be 16-byte and d_E 8-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = pt_check(c, cfg, samples_per_texel);
    if (rc) return rc;
    const long long n = c->K * c->n_layouts;
    hipStream_t st = c->stream;
    HIPCHK(c, launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st));
    HIPCHK(c, launch_clear((long long*)d_S, n, st));
    for (int j = 0; j < c->n_layouts; ++j) {
        PtArgs a = pt_args(c, cfg, samples_per_texel, j);
        a.S = (long long*)d_S + (long long)j * c->K;
        HIPCHK(c, launch_pt(false, a, c->tune.lds_depth, st));
    }
    HIPCHK(c, launch_finalize((const long long*)d_S, d_E, n, c->d_flags, st));
    return LT_OK;
}

int lt_pt_adjoint(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int32_t samples_per_texel,
                  const float* d_dOdE, float* d_grad)
{
    if (!c) return LT_EINVAL;
    if (!d_params || !d_dOdE || !d_grad) return fail(c, LT_EINVAL, "NULL device buffer");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = pt_check(c, cfg, samples_per_texel);
    if (rc) return rc;
    const size_t need = (size_t)c->L * 6;
    if (c->ptgrad_cap < need) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        hipFree(c->d_ptgrad);
        c->d_ptgrad = nullptr;
        c->ptgrad_cap = 0;
        HIPCHK(c, hipMalloc(&c->d_ptgrad, sizeof(double) * need));
        c->ptgrad_cap = need;
    }
    hipStream_t st = c->stream;
    HIPCHK(c, launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, st));
    HIPCHK(c, launch_fill_f32((float*)c->d_ptgrad, (long long)need * 2, 0.0f, st));
    for (int j = 0; j < c->n_layouts; ++j) {
        PtArgs a = pt_args(c, cfg, samples_per_texel, j);
        a.g = d_dOdE + (long long)j * c->K;
        a.grad = c->d_ptgrad + 6 * (long long)c->offs[j];
        HIPCHK(c, launch_pt(true, a, c->tune.lds_depth, st));
    }
    HIPCHK(c, launch_f64_to_f32(c->d_ptgrad, d_grad, (long long)need, st));
    return LT_OK;
}

int lt_record_paths(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int32_t layout, int32_t light,
                    int64_t first, int64_t count, int32_t* d_prim, int32_t* d_texel, const float* d_dOdE,
                    float* d_contrib)
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_prim || !d_texel) return fail(c, LT_EINVAL, "NULL device buffer");
    if ((d_dOdE == nullptr) != (d_contrib == nullptr)) return fail(c, LT_EINVAL, "dOdE and contrib go together");
    if (layout < 0 || layout >= c->n_layouts) return fail(c, LT_EINVAL, "layout out of range");
    const int nl = c->offs[layout + 1] - c->offs[layout];
    if (light < 0 || light >= nl) return fail(c, LT_EINVAL, "light out of range");
    const long long np = paths_of_light(cfg->paths_per_layout, nl, light);
    if (first < 0 || count < 0 || first + count > np) return fail(c, LT_EINVAL, "path range out of range");
    if (count == 0) return LT_OK;
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, (long long)kRecordBlocks * 4);
    if (rc) return rc;
    RecordArgs r;
    memset(&r, 0, sizeof(r));
    r.nodes = c->nodes;
    r.tris = c->tris;
    r.patches = c->patches;
    r.lights = c->d_lights;
    r.gl = c->offs[layout] + light;
    r.layout = layout;
    r.max_hits = cfg->max_hits;
    r.K = c->K;
    r.stream_id = ((uint32_t)layout << 16) | (uint32_t)light;
    r.key0 = (uint32_t)cfg->seed;
    r.key1 = (uint32_t)(cfg->seed >> 32);
    r.first = first;
    r.count = count;
    r.prim = d_prim;
    r.texel = d_texel;
    r.g = d_dOdE;
    r.contrib = d_contrib;
    r.linear = (cfg->flags & LT_FLAG_LINEAR) ? 1 : 0;
    r.gstack = c->d_gstack;
    r.gdepth = std::max(gstack_depth(c), 1);
    r.max_steps = 2 * c->n_nodes + 16;
    r.flags = c->d_flags;
    if (cfg->flags & LT_FLAG_PROPOSAL) {
        r.prop_pdf = c->prop_pdf;
        r.prop_cdf = c->prop_cdf;
        r.prop_guide = c->prop_guide;
        r.alpha_plain = cfg->alpha_plain;
    }
    HIPCHK(c, launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, c->stream));
    HIPCHK(c, launch_record(r, c->tune.lds_depth, c->stream));
    return LT_OK;
}

int lt_trace_stats(lt_ctx* c, const lt_trace_cfg* cfg, const float* d_params, int64_t* d_S, int64_t h_counts[8])
{
    int rc = check_cfg(c, cfg);
    if (rc) return rc;
    if (!d_params || !d_S || !h_counts) return fail(c, LT_EINVAL, "NULL buffer");
    if ((uintptr_t)d_S & 15) return fail(c, LT_EINVAL, "d_S must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    rc = ensure_gstack(c, resident_waves(c));
    if (rc) return rc;
    TraceArgs a = trace_args(c, cfg);
    a.S = (long long*)d_S;
    HIPCHK(c, hipMemsetAsync(c->d_stats, 0, sizeof(unsigned long long) * 8, c->stream));
    HIPCHK(c, launch_light_setup(d_params, c->d_si, c->d_sf, c->d_npaths, c->L, c->d_lights, c->d_flags, c->stream));
    HIPCHK(c, launch_clear(a.S, c->K * c->n_layouts, c->stream));
    HIPCHK(c, launch_trace(false, true, a, c->tune.waves_per_block, c->tune.lds_depth, c->n_cu, c->stream));
    unsigned long long h[8];
    HIPCHK(c, hipMemcpyAsync(h, c->d_stats, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < 8; ++i) h_counts[i] = (int64_t)h[i];
    return LT_OK;
}

int lt_get_tuning(const lt_ctx* c, lt_tuning* out)
{
    if (!c || !out) return LT_EINVAL;
    *out = c->tune;
    return LT_OK;
}

int lt_set_tuning(lt_ctx* c, const lt_tuning* t)
{
    if (!c || !t) return LT_EINVAL;
    if (t->waves_per_block != 1 && t->waves_per_block != 2 && t->waves_per_block != 4)
        return fail(c, LT_EINVAL, "waves_per_block must be 1, 2 or 4");
    if (t->xcd_remap != 0 && t->xcd_remap != 1) return fail(c, LT_EINVAL, "xcd_remap must be 0 or 1");
    if (t->tile_paths < 0 || t->tile_paths % 64 != 0 || t->tile_paths > (1 << 24))
        return fail(c, LT_EINVAL, "tile_paths must be 0 or a positive multiple of 64");
    if (t->refill_threshold < 1 || t->refill_threshold > 64)
        return fail(c, LT_EINVAL, "refill_threshold must be in [1, 64]");
    if (t->lds_depth != 16 && t->lds_depth != 32) return fail(c, LT_EINVAL, "lds_depth must be 16 or 32");
    if (t->tri_share < 0 || t->tri_share > 8) return fail(c, LT_EINVAL, "tri_share must be in [0, 8]");
    free_graphs(c);
    c->tune = *t;
    c->tiles_tp = -1;   // recompute tiles at the next call
    return LT_OK;
}

int lt_bvh_copy(lt_ctx* c, void* h_nodes, int64_t nodes_bytes, void* h_tris, int64_t tris_bytes)
{
    if (!c) return LT_EINVAL;
    if (!c->nodes || !c->tris) return fail(c, LT_EINVAL, "no scene uploaded");
    if (!h_nodes || !h_tris) return fail(c, LT_EINVAL, "NULL host buffer");
    const int64_t nb = (int64_t)c->n_nodes * 16 * kNodeRows;
    const int64_t tb = (c->n_tris > 1 ? c->n_tris : 2) * 48;   // a single triangle fills both root slots
    if (nodes_bytes < nb || tris_bytes < tb) return fail(c, LT_EINVAL, "host buffer too small for the BVH");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(h_nodes, c->nodes, (size_t)nb, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(h_tris, c->tris, (size_t)tb, hipMemcpyDeviceToHost));
    return LT_OK;
}

int lt_info_get(const lt_ctx* c, lt_info* out)
{
    if (!c || !out) return LT_EINVAL;
    memset(out, 0, sizeof(*out));
    out->n_tris = c->n_tris;
    out->n_patches = c->n_patches;
    out->n_texels = c->K;
    out->bvh_nodes = c->n_nodes;
    out->bvh_depth = c->depth;
    out->device_bytes = (int64_t)c->n_nodes * 16 * kNodeRows + c->n_tris * 48 + (int64_t)c->n_patches * sizeof(DevPatch) +
                        c->K * 4 + (int64_t)c->gstack_cap * 4 + (int64_t)c->partials_cap * 8 +
                        (int64_t)c->rec_cap * 4;
    out->n_lights = c->L;
    out->n_layouts = c->n_layouts;
    return LT_OK;
}

int lt_proposal_set_table(lt_ctx* c, const float* d_pdf, const float* d_cdf)
{
    if (!c) return LT_EINVAL;
    if (!c->has_lights) return fail(c, LT_ESTATE, "no luminaires set");
    if (!d_pdf || !d_cdf) return fail(c, LT_EINVAL, "NULL device buffer");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n = sizeof(float) * 1024 * (size_t)c->L;
    HIPCHK(c, hipMemcpyAsync(c->prop_pdf, d_pdf, n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->prop_cdf, d_cdf, n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, launch_guide_build(c->prop_cdf, c->L, c->prop_guide, c->stream));
    c->has_proposal = true;
    return LT_OK;
}

int lt_proposal_get_table(lt_ctx* c, float* d_pdf, float* d_cdf)
{
    if (!c) return LT_EINVAL;
    if (!c->has_proposal) return fail(c, LT_ESTATE, "no emission proposal loaded");
    if (!d_pdf || !d_cdf) return fail(c, LT_EINVAL, "NULL device buffer");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n = sizeof(float) * 1024 * (size_t)c->L;
    HIPCHK(c, hipMemcpyAsync(d_pdf, c->prop_pdf, n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d_cdf, c->prop_cdf, n, hipMemcpyDeviceToDevice, c->stream));
    return LT_OK;
}

int lt_proposal_set_scale(lt_ctx* c, const float* d_inv_sigma)
{
    if (!c) return LT_EINVAL;
    if (!c->has_lights) return fail(c, LT_ESTATE, "no luminaires set");
    if (!d_inv_sigma) return fail(c, LT_EINVAL, "NULL device buffer");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(c->inv_sigma, d_inv_sigma, sizeof(float) * 6 * (size_t)c->L, hipMemcpyDeviceToDevice,
                             c->stream));
    return LT_OK;
}

int lt_proposal_mlp_infer(lt_ctx* c, const uint16_t* d_w_bf16, const float* d_x, float* d_logits)
{
    if (!c) return LT_EINVAL;
    if (!c->has_lights) return fail(c, LT_ESTATE, "no luminaires set");
    if (!d_w_bf16 || !d_x) return fail(c, LT_EINVAL, "NULL device buffer");
    if (((uintptr_t)d_w_bf16 & 7) || ((uintptr_t)d_x & 3)) return fail(c, LT_EINVAL, "misaligned buffer");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_mlp_infer(d_w_bf16, d_x, c->L, d_logits, c->prop_pdf, c->prop_cdf, c->stream));
    HIPCHK(c, launch_guide_build(c->prop_cdf, c->L, c->prop_guide, c->stream));
    c->has_proposal = true;
    return LT_OK;
}

int lt_proposal_mlp_train(lt_ctx* c, float* d_w, float* d_mw, float* d_vw, uint16_t* d_w_bf16, float* d_x,
                          float* d_mx, float* d_vx, const float* d_target, int32_t step, float lr, float* d_loss,
                          float* d_grad_out)
{
    if (!c) return LT_EINVAL;
    if (!c->has_lights) return fail(c, LT_ESTATE, "no luminaires set");
    if (!d_w || !d_mw || !d_vw || !d_w_bf16 || !d_x || !d_mx || !d_vx || !d_target)
        return fail(c, LT_EINVAL, "NULL device buffer");
    if (step < 1) return fail(c, LT_EINVAL, "step counts from 1");
    if (!(lr > 0.0f) || !isfinite(lr)) return fail(c, LT_EINVAL, "invalid learning rate");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t need = mlp_train_scratch_floats(c->L);
    if (need > c->mlp_scratch_cap) {
        hipFree(c->mlp_scratch);
        c->mlp_scratch = nullptr;
        c->mlp_scratch_cap = 0;
        HIPCHK(c, hipMalloc(&c->mlp_scratch, sizeof(float) * need));
        c->mlp_scratch_cap = need;
    }
    HIPCHK(c, launch_mlp_train(d_w, d_mw, d_vw, d_w_bf16, d_x, d_mx, d_vx, d_target, c->L, step, lr, c->mlp_scratch,
                               d_loss, d_grad_out, c->stream));
    return LT_OK;
}

int lt_proposal_set(lt_ctx* c, const float* d_w, const float* d_embed, const lt_proposal_cfg* cfg)
{
    if (!c) return LT_EINVAL;
    if (!c->has_lights) return fail(c, LT_ESTATE, "no luminaires set");
    if (!d_w || !d_embed || !cfg) return fail(c, LT_EINVAL, "NULL argument");
    for (int k = 0; k < 6; ++k)
        if (!isfinite(cfg->param_lo[k]) || !isfinite(cfg->param_hi[k]) || !(cfg->param_hi[k] > cfg->param_lo[k]))
            return fail(c, LT_EINVAL, "parameter box needs finite lo < hi");
    if (!(cfg->hist_decay >= 0.0f && cfg->hist_decay < 1.0f) || !(cfg->sigma_decay >= 0.0f && cfg->sigma_decay < 1.0f))
        return fail(c, LT_EINVAL, "decays must lie in [0, 1)");
    if (!(cfg->plain_floor >= 0.0f && cfg->plain_floor <= 1.0f)) return fail(c, LT_EINVAL, "plain_floor outside [0, 1]");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_net(c);
    const size_t L = (size_t)c->L, nw = kMlpWeights;
    HIPCHK(c, hipMalloc(&c->net_w, sizeof(float) * nw));
    HIPCHK(c, hipMalloc(&c->net_mw, sizeof(float) * nw));
    HIPCHK(c, hipMalloc(&c->net_vw, sizeof(float) * nw));
    HIPCHK(c, hipMalloc(&c->net_wb, sizeof(uint16_t) * nw));
    HIPCHK(c, hipMalloc(&c->net_x, sizeof(float) * L * kMlpIn));
    HIPCHK(c, hipMalloc(&c->net_mx, sizeof(float) * L * kMlpIn));
    HIPCHK(c, hipMalloc(&c->net_vx, sizeof(float) * L * kMlpIn));
    HIPCHK(c, hipMalloc(&c->net_havg, sizeof(double) * L * kMlpBins));
    HIPCHK(c, hipMalloc(&c->net_pmass, sizeof(double) * L * kMlpBins));
    HIPCHK(c, hipMalloc(&c->net_target, sizeof(float) * L * kMlpBins));
    HIPCHK(c, hipMalloc(&c->net_sig2, sizeof(float) * L * 6));
    HIPCHK(c, hipMemcpyAsync(c->net_w, d_w, sizeof(float) * nw, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->net_mw, 0, sizeof(float) * nw, c->stream));
    HIPCHK(c, hipMemsetAsync(c->net_vw, 0, sizeof(float) * nw, c->stream));
    HIPCHK(c, hipMemsetAsync(c->net_x, 0, sizeof(float) * L * kMlpIn, c->stream));
    HIPCHK(c, hipMemsetAsync(c->net_mx, 0, sizeof(float) * L * kMlpIn, c->stream));
    HIPCHK(c, hipMemsetAsync(c->net_vx, 0, sizeof(float) * L * kMlpIn, c->stream));
    HIPCHK(c, hipMemcpy2DAsync(c->net_x + kMlpParams, sizeof(float) * kMlpIn, d_embed, sizeof(float) * kMlpEmbed,
                               sizeof(float) * kMlpEmbed, L, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, launch_to_bf16(c->net_w, c->net_wb, (int)nw, c->stream));
    // the plain lobe's cell masses (the training target's floor)
    std::vector<float> lobe(L);
    for (size_t l = 0; l < L; ++l) lobe[l] = c->lights[l].lobe_n;
    float* d_lobe = nullptr;
    HIPCHK(c, hipMalloc(&d_lobe, sizeof(float) * L));
    HIPCHK(c, hipMemcpy(d_lobe, lobe.data(), sizeof(float) * L, hipMemcpyHostToDevice));
    hipError_t e = launch_plain_mass(d_lobe, c->L, c->net_pmass, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    hipFree(d_lobe);
    HIPCHK(c, e);
    c->net_cfg = *cfg;
    c->net_step = 0;
    c->net_havg_ok = false;
    c->net_sig2_ok = false;
    c->has_net = true;
    return LT_OK;
}

int lt_proposal_refresh(lt_ctx* c, const float* d_params)
{
    if (!c) return LT_EINVAL;
    if (!c->has_net) return fail(c, LT_ESTATE, "no proposal network (lt_proposal_set)");
    if (!d_params) return fail(c, LT_EINVAL, "NULL device buffer");
    HIPCHK(c, hipSetDevice(c->device));
    ParamBox box;
    for (int k = 0; k < 6; ++k) {
        box.lo[k] = c->net_cfg.param_lo[k];
        box.hi[k] = c->net_cfg.param_hi[k];
    }
    HIPCHK(c, launch_proposal_inputs(d_params, c->L, box, c->net_x, c->stream));
    HIPCHK(c, launch_mlp_infer(c->net_wb, c->net_x, c->L, nullptr, c->prop_pdf, c->prop_cdf, c->stream));
    HIPCHK(c, launch_guide_build(c->prop_cdf, c->L, c->prop_guide, c->stream));
    c->has_proposal = true;
    return LT_OK;
}

int lt_proposal_update_scale(lt_ctx* c, const float* d_grad, const float* h_mask)
{
    if (!c) return LT_EINVAL;
    if (!c->has_net) return fail(c, LT_ESTATE, "no proposal network (lt_proposal_set)");
    if (!d_grad) return fail(c, LT_EINVAL, "NULL device buffer");
    Param6 m;
    for (int k = 0; k < 6; ++k) {
        m.v[k] = h_mask ? h_mask[k] : 1.0f;
        if (!isfinite(m.v[k])) return fail(c, LT_EINVAL, "non-finite mask");
    }
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_proposal_scale(d_grad, c->L, c->net_sig2, c->net_sig2_ok ? 0 : 1, c->net_cfg.sigma_decay, m,
                                    c->inv_sigma, c->stream));
    c->net_sig2_ok = true;
    return LT_OK;
}

int lt_proposal_train_step(lt_ctx* c, const float* d_bin_hist, float lr, int32_t steps, float* d_loss,
                           float* d_target_out)
{
    if (!c) return LT_EINVAL;
    if (!c->has_net) return fail(c, LT_ESTATE, "no proposal network (lt_proposal_set)");
    if (!d_bin_hist) return fail(c, LT_EINVAL, "NULL device buffer");
    if (!(lr > 0.0f) || !isfinite(lr)) return fail(c, LT_EINVAL, "invalid learning rate");
    if (steps < 0 || steps > 1000) return fail(c, LT_EINVAL, "steps must be in [0, 1000]");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_proposal_target(d_bin_hist, c->L, c->net_havg, c->net_pmass, c->net_havg_ok ? 0 : 1,
                                     (double)c->net_cfg.hist_decay, (double)c->net_cfg.plain_floor, c->net_target,
                                     c->stream));
    c->net_havg_ok = true;
    if (d_target_out)
        HIPCHK(c, hipMemcpyAsync(d_target_out, c->net_target, sizeof(float) * 1024 * (size_t)c->L,
                                 hipMemcpyDeviceToDevice, c->stream));
    const size_t need = mlp_train_scratch_floats(c->L);
    if (need > c->mlp_scratch_cap) {
        hipFree(c->mlp_scratch);
        c->mlp_scratch = nullptr;
        c->mlp_scratch_cap = 0;
        HIPCHK(c, hipMalloc(&c->mlp_scratch, sizeof(float) * need));
        c->mlp_scratch_cap = need;
    }
    for (int s = 0; s < steps; ++s) {
        ++c->net_step;
        HIPCHK(c, launch_mlp_train(c->net_w, c->net_mw, c->net_vw, c->net_wb, c->net_x, c->net_mx, c->net_vx,
                                   c->net_target, c->L, c->net_step, lr, c->mlp_scratch, d_loss, nullptr, c->stream));
    }
    return LT_OK;
}

int lt_proposal_get_net(lt_ctx* c, float* d_w, float* d_x)
{
    if (!c) return LT_EINVAL;
    if (!c->has_net) return fail(c, LT_ESTATE, "no proposal network (lt_proposal_set)");
    HIPCHK(c, hipSetDevice(c->device));
    if (d_w)
        HIPCHK(c, hipMemcpyAsync(d_w, c->net_w, sizeof(float) * kMlpWeights, hipMemcpyDeviceToDevice, c->stream));
    if (d_x)
        HIPCHK(c, hipMemcpyAsync(d_x, c->net_x, sizeof(float) * kMlpIn * (size_t)c->L, hipMemcpyDeviceToDevice,
                                 c->stream));
    return LT_OK;
}

int lt_set_timing(lt_ctx* c, int enable)
{
    if (!c) return LT_EINVAL;
    c->timing = enable != 0;
    return LT_OK;
}

int lt_timing_read(lt_ctx* c, double* fwd_ms, int32_t* n_fwd, double* adj_ms, int32_t* n_adj)
{
    if (!c) return LT_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    double sums[2] = {0.0, 0.0};
    int counts[2] = {0, 0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>>* lists[2] = {&c->t_fwd, &c->t_adj};
    hipError_t err = hipSuccess;
    for (int k = 0; k < 2; ++k) {
        for (auto& pr : *lists[k]) {
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventSynchronize(pr.second);
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, pr.first, pr.second);
            sums[k] += ms;
            counts[k]++;
            hipEventDestroy(pr.first);
            hipEventDestroy(pr.second);
        }
        lists[k]->clear();
    }
    if (err != hipSuccess) return fail(c, LT_EHIP, std::string("timing events: ") + hipGetErrorString(err));
    if (fwd_ms) *fwd_ms = sums[0];
    if (n_fwd) *n_fwd = counts[0];
    if (adj_ms) *adj_ms = sums[1];
    if (n_adj) *n_adj = counts[1];
    return LT_OK;
}

namespace {

std::string tune_key(const lt_ctx* c, const lt_trace_cfg* cfg)
{
    char buf[256];
    hipDeviceProp_t prop;
    const char* arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    snprintf(buf, sizeof(buf), "v6 arch=%s tris=%lld texels=%lld lights=%d layouts=%d ppl=%lld hits=%d", arch,
             (long long)c->n_tris, (long long)c->K, c->L, c->n_layouts, (long long)cfg->paths_per_layout,
             cfg->max_hits);
    for (char* q = buf; *q; ++q)
        if (*q == '|' || *q == '\n') *q = '_';
    return buf;
}

bool tune_lookup(const char* path, const std::string& key, lt_tuning* t, float* ms)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        char* bar = strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        if (key != line) continue;
        lt_tuning x;
        memset(&x, 0, sizeof(x));
        float m = 0.f;
        if (sscanf(bar + 1, "%d %d %d %d %d %d %f", &x.waves_per_block, &x.xcd_remap, &x.tile_paths,
                   &x.refill_threshold, &x.lds_depth, &x.tri_share, &m) == 7) {
            *t = x;
            *ms = m;
            found = true;   // the last matching line wins
        }
    }
    fclose(f);
    return found;
}

}  // namespace

// Coordinate descent over the launch shape, timing forward + adjoint with
// HIP events on the context stream (one warm-up, best of two).
int lt_autotune(lt_ctx* c, const lt_trace_cfg* cfg_in, const float* d_params, int64_t* d_S, float* d_E,
                const float* d_dOdE, float* d_grad, const char* cache_path, float* h_best_ms)
{
    int rc = check_cfg(c, cfg_in);
    if (rc) return rc;
    if (!d_params || !d_S || !d_E || !d_dOdE || !d_grad) return fail(c, LT_EINVAL, "NULL device buffer");
    lt_trace_cfg cfg = *cfg_in;
    cfg.flags &= ~LT_FLAG_GRAPH;
    const std::string key = tune_key(c, &cfg);
    lt_tuning best_t;
    float best_ms = 0.f;
    if (cache_path && tune_lookup(cache_path, key, &best_t, &best_ms)) {
        rc = lt_set_tuning(c, &best_t);
        if (rc) return rc;
        if (h_best_ms) *h_best_ms = best_ms;
        return LT_OK;
    }
    HIPCHK(c, hipSetDevice(c->device));
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    const bool timing_was = c->timing;
    c->timing = false;
    auto measure = [&](const lt_tuning& t, float* out) -> int {
        int r = lt_set_tuning(c, &t);
        if (r) return r;
        float bestm = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHK(c, hipEventRecord(e0, c->stream));
            r = lt_trace_forward(c, &cfg, d_params, d_S, d_E);
            if (!r) r = lt_trace_adjoint(c, &cfg, d_params, d_dOdE, d_grad, nullptr);
            if (r) return r;
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) bestm = std::min(bestm, ms);
        }
        *out = bestm;
        return LT_OK;
    };
    const int auto_tp = effective_tile_paths(c, cfg.paths_per_layout);
    lt_tuning cur = c->tune;
    float cur_ms = 0.f;
    rc = measure(cur, &cur_ms);
    const int opts_wpb[] = {1, 2, 4};
    const int opts_lds[] = {16, 32};
    const int opts_thr[] = {4, 8, 16, 24, 32, 48};
    const int opts_xcd[] = {0, 1};
    const int opts_tri[] = {0, 2, 3, 4, 5, 6};
    for (int pass = 0; pass < 2 && !rc; ++pass) {
        for (int dim = 0; dim < 6 && !rc; ++dim) {
            std::vector<lt_tuning> cands;
            lt_tuning t = cur;
            if (dim == 0) for (int v : opts_wpb) { t.waves_per_block = v; cands.push_back(t); }
            if (dim == 1) for (int v : opts_lds) { t.lds_depth = v; cands.push_back(t); }
            if (dim == 2) for (int v : opts_thr) { t.refill_threshold = v; cands.push_back(t); }
            if (dim == 3) for (int v : opts_xcd) { t.xcd_remap = v; cands.push_back(t); }
            if (dim == 5) for (int v : opts_tri) { t.tri_share = v; cands.push_back(t); }
            if (dim == 4)
                for (int f : {-2, -1, 0, 1, 2}) {
                    long long tp = f >= 0 ? (long long)auto_tp << f : (long long)auto_tp >> (-f);
                    tp = std::max<long long>(64, std::min<long long>(1 << 16, (tp / 64) * 64));
                    t.tile_paths = (int)tp;
                    cands.push_back(t);
                }
            for (const lt_tuning& cand : cands) {
                if (!memcmp(&cand, &cur, sizeof(cand))) continue;
                float ms = 0.f;
                rc = measure(cand, &ms);
                if (rc) break;
                if (ms < cur_ms) {
                    cur = cand;
                    cur_ms = ms;
                }
            }
        }
    }
    c->timing = timing_was;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    rc = lt_set_tuning(c, &cur);
    if (rc) return rc;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s|%d %d %d %d %d %d %.3f\n", key.c_str(), cur.waves_per_block, cur.xcd_remap,
                    cur.tile_paths, cur.refill_threshold, cur.lds_depth, cur.tri_share, cur_ms);
            fclose(f);
        }
    }
    if (h_best_ms) *h_best_ms = cur_ms;
    return LT_OK;
}

}  // extern "C"
