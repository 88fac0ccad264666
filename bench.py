"""Benchmark: light paths/s (forward + adjoint) on one MI355X.

Headline workload: the procedural 80 x 60 x 3.2 m building floor (2M
triangles, 16M texels, 128 rectangular cos^n luminaires), 2^28 light paths
per step, 6 hits per path.  One step is the whole hot path: luminaire setup,
accumulator clear, primal light tracing, fixed-point to float, objective and
dO/dE, adjoint light tracing (its first-hit records, then the per-path
contributions and per-tile sums), per-light gradient reduction.  Inputs are
resident in HBM before the timed region.

The launch tuning comes from the autotuner (a matching entry of
paper_2310_02043_amd/tuning.cache is reused).  Prints one JSON line: metric,
value, the roofline of the dominant kernel, the CPU oracle timed on a bounded
sample of the same workload (all host cores and one core), and as extra keys
the office (200k triangles, 2^26 paths, 5 hits) throughput, its directional
texels, and the learned-proposal study: gradient error x time of the adjoint
pass against the plain tracer at the initial and at the converged
luminaires.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TUNING_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2310_02043_amd", "tuning.cache")
METRIC = "light paths/s (forward+adjoint); gradient-error×time vs plain tracer"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# one non-packed FP32 operation per lane per cycle: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (the rate the traversal's comparisons and min/max can reach)
UNPACKED_LANE_OPS_T = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic work per unit (see the design notes): one node visit = four box
# tests of 20 ops and a 64 B node (4-wide tree); one triangle test = 40 ops and
# a 48 B record; one hit = an 80 B patch record plus an 8 B atomic (forward) or
# a 4 B gather (adjoint).
BOXES_PER_NODE, OPS_PER_BOX, OPS_PER_TRI = 4, 20, 40
# the same work in VALU issue slots (an FMA is one slot): a box test is 6 FMA,
# 6 min/max and 2 compares; a triangle test's 40 operations have no FMA
SLOTS_PER_BOX, SLOTS_PER_TRI = 14, 40
NODE_BYTES, TRI_BYTES, PATCH_BYTES = 64, 48, 80
# Per-lane vector-memory requests (one 16 B row each): a node visit loads its
# four rows, a triangle test three, a hit the five rows of its patch record
# plus one atomic (forward) or one gather (adjoint).  A lane's request mostly
# falls in a cache line of its own, and the counters (TD busy ~100 %, one TD
# cycle per lane request) show the vector-memory path serving about one
# distinct line per CU per clock: 256 CUs x 2.4 GHz (lanes sharing a line in
# one instruction, at the top of the tree, can take the rate slightly above).
REQ_PER_NODE, REQ_PER_TRI, REQ_PER_HIT = 4, 3, 6
VMEM_REQ_PEAK_G = 256 * 2.4e9 / 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILES = {"building": os.path.join(ROOT, "profiles", "k_trace_building_2e28.traffic.json"),
                 "office": os.path.join(ROOT, "profiles", "k_trace_office_2e26.traffic.json")}


def measured_traffic(workload, kind, tuning=None, paths=None):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes (scaled by the copy-kernel calibration), or None if there are none
    for the workload or the kernel sources, the launch tuning or the path
    count differ from those the counters were taken with."""
    import hashlib
    try:
        d = json.load(open(TRAFFIC_FILES[workload]))
    except (KeyError, OSError, ValueError):
        return None
    h = hashlib.sha256()
    for s in d["sources"]:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    if h.hexdigest() != d["kernel_sources_sha256"]:
        return None
    if tuning is not None and d.get("tuning") != tuning:
        return None
    if paths is not None and d.get("paths_per_layout") != paths:
        return None
    k = d[kind]
    return int((k["fetch_kib"] * d["fetch_scale"] + k["write_kib"] * d["write_scale"]) * 1024)


def cpu_baseline(scene, lights, seed, ppl, B, target_seconds):
    """The oracle as it stands, on the host cores, on a bounded sample: the
    first m paths of every luminaire (same Phi_r), forward + objective +
    adjoint; paths/s over that sample.  Timed with all host threads (the
    oracle parallelises each luminaire's paths in chunks of 1024, so the
    sample gives every luminaire at least one chunk per thread) and with one
    thread on a smaller sample."""
    import oracle
    oracle.build(force=False)
    log("oracle BVH build ...")
    osc = oracle.OracleScene(scene, use_bvh=True)
    ol = oracle.OracleLights(lights)
    A = scene.texel_area()
    import lt_inputs as li
    Et = np.stack([li.painted_target(scene, 0.5, seed=j) for j in range(lights.n_layouts)])

    def run(m, threads):
        t0 = time.perf_counter()
        S, _ = oracle.forward(osc, ol, lights.params, seed, ppl, B, limit_per_light=m, n_threads=threads)
        t1 = time.perf_counter()
        _, g = oracle.objective(oracle.fixed_to_float(S), Et, A)
        t2 = time.perf_counter()
        oracle.adjoint(osc, ol, lights.params, seed, ppl, B, g, limit_per_light=m, n_threads=threads)
        t3 = time.perf_counter()
        return (t1 - t0) + (t3 - t2)

    nthr = oracle.num_threads()
    # one thread: grow the per-light sample until a run takes >= 1 s, then
    # time about a third of the budget
    m = 64
    dt = run(m, 1)
    while dt < 1.0 and m < (1 << 20):
        m *= 4
        dt = run(m, 1)
    m1 = int(max(64, min(1 << 20, m * (target_seconds / 3) / max(dt, 1e-3))))
    log(f"oracle, one thread: {m1} paths per luminaire ...")
    dt1 = run(m1, 1)
    rate1 = m1 * lights.n_lights / dt1
    # all threads: about the rest of the budget, at least one 1024-path chunk
    # per thread and luminaire
    mn = int(max(1024 * nthr, min(1 << 22, rate1 * nthr * (2 * target_seconds / 3) / lights.n_lights)))
    log(f"oracle, {nthr} threads: {mn} paths per luminaire ...")
    dtn = run(mn, nthr)
    n_n, n_1 = mn * lights.n_lights, m1 * lights.n_lights
    return {"value": n_n / dtn, "unit": "paths/s", "cores": nthr, "kind": "oracle",
            "sample": f"first {mn} paths of each of the {lights.n_lights} luminaires ({n_n} paths, {B} hits, "
                      f"forward+adjoint, {dtn:.1f} s on {nthr} threads)",
            "single_core": {"value": rate1, "unit": "paths/s", "cores": 1,
                            "sample": f"first {m1} paths of each luminaire ({n_1} paths, {dt1:.1f} s)"}}


def proposal_study(ctx, wl, N, at="initial", seeds=32, ref_runs=48, train_iters=30, alpha=0.2, train_every=4,
                   pt_seeds=16):
    """Gradient error x time of the adjoint pass, learned proposal vs plain.

    The luminaires sit at their perturbed initial parameters (at="initial")
    or at the converged ones (at="converged": the ground truth, where an Adam
    run ends), the target irradiance comes from the hidden ground-truth
    parameters, and the adjoint
    source g = dO/dE is fixed from a 2^28-path forward pass.  The reference
    gradient averages ref_runs plain adjoint passes of 2^28 paths.  The
    proposal is trained online on the adjoint pass's own direction histograms
    (train_iters passes of 2^24 paths) and then frozen; each estimator runs
    `seeds` independent N-path adjoint passes.  eps = |g_hat - g_ref| /
    |g_ref|; eps^2 * t is independent of N for an unbiased estimator, so the
    ratio learned / plain is the time ratio at equal relative error.  The
    learned form's time per gradient is its adjoint pass plus, amortised over
    `train_every` optimisation steps, the histogram it accumulates for
    training and the network's training + inference.  The same reference
    also scores object-space path tracing (next-event estimation, the
    comparison estimator) with as many samples per texel as fit the plain
    adjoint pass's time."""
    import torch
    from paper_2310_02043_amd.proposal import LearnedProposal
    lights, B = wl["lights"], wl["max_hits"]
    dev = "cuda:0"
    pt = torch.tensor(wl["params_target"], device=dev)
    p0 = torch.tensor(lights.params, device=dev) if at == "initial" else pt.clone()
    big = 1 << 28
    Et, _ = ctx.trace_forward(pt, ctx.cfg(0x7A11, big, B))
    Et = Et.clone()
    E0, _ = ctx.trace_forward(p0, ctx.cfg(0x7A12, big, B))
    _, g = ctx.objective(E0, Et)
    g = g.clone()
    ref = torch.zeros((lights.n_lights, 6), dtype=torch.float64, device=dev)
    for s in range(ref_runs):
        ref += ctx.trace_adjoint(p0, g, ctx.cfg(0x10000 + s, big, B)).double()
    ref /= ref_runs
    unit = ref.pow(2).mean(0).sqrt()      # per-parameter RMS: a unit-free second error norm

    def errs(gh):
        e = gh.double() - ref
        return float(e.norm() / ref.norm()), float((e / unit).norm() / (ref / unit).norm())

    lp = LearnedProposal(ctx, [0, 0, 2.5, -0.6, -0.6, 0], [30, 20, 3.0, 0.6, 0.6, 80], alpha_plain=alpha)
    lp.refresh(p0)
    losses = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for it in range(train_iters):
        gr = ctx.trace_adjoint(p0, g, ctx.cfg(0x20000 + it, 1 << 24, B, proposal=True, alpha_plain=alpha),
                               bin_hist=lp.hist)
        lp.update_scale(gr)
        ev0.record()     # proposal upkeep: 4 training steps + inference
        losses.append(lp.train(steps=4))
        lp.refresh(p0)
        ev1.record()
    torch.cuda.synchronize()
    upkeep_ms = ev0.elapsed_time(ev1)

    def timed(prop, hist, seed0, n):
        ctx.trace_adjoint(p0, g, ctx.cfg(1, N, B, proposal=prop, alpha_plain=alpha), bin_hist=hist)
        torch.cuda.synchronize()
        ctx.timing_read()
        ctx.set_timing(True)
        ee = [errs(ctx.trace_adjoint(p0, g, ctx.cfg(seed0 + s, N, B, proposal=prop, alpha_plain=alpha),
                                     bin_hist=hist)) for s in range(n)]
        torch.cuda.synchronize()
        ctx.set_timing(False)
        _, _, adj_ms, na = ctx.timing_read()
        return np.asarray(ee), adj_ms / max(na, 1)

    e_pl, t_pl = timed(False, None, 0x30000, seeds)
    e_le, t_le = timed(True, None, 0x40000, seeds)
    _, t_hist = timed(True, lp.hist, 0x50000, 4)
    t_learn = t_le + (max(t_hist - t_le, 0.0) + upkeep_ms) / train_every
    e2_pl, e2_le = (e_pl ** 2).mean(0), (e_le ** 2).mean(0)

    # object-space path tracing with next-event estimation (the comparison
    # estimator) against the same reference, at about the light tracer's time
    def pt_timed(M, seed0, n):
        cfg = ctx.cfg(seed0, N, B)
        ctx.pt_adjoint(p0, g, cfg, M)
        torch.cuda.synchronize()
        ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev_a.record()
        grads = [ctx.pt_adjoint(p0, g, ctx.cfg(seed0 + s, N, B), M).clone() for s in range(n)]
        ev_b.record()
        torch.cuda.synchronize()
        return grads, ev_a.elapsed_time(ev_b) / n

    rng = np.random.default_rng(0)
    bs = [(e_le[rng.integers(0, seeds, seeds), 0] ** 2).mean() / (e_pl[rng.integers(0, seeds, seeds), 0] ** 2).mean()
          for _ in range(2000)]
    ratio = e2_le[0] * t_learn / (e2_pl[0] * t_pl)
    res = {"workload": f"office, adjoint pass at the {'perturbed initial' if at == 'initial' else 'converged'} "
                       f"luminaires", "paths": N, "seeds": seeds,
           "alpha_plain": alpha, "reference": f"mean of {ref_runs} plain passes x 2^28 paths",
           "train_iters": train_iters, "train_paths": 1 << 24,
           "train_loss": [round(losses[0], 4), round(losses[-1], 4)], "train_every": train_every,
           "plain": {"adjoint_ms": round(t_pl, 3), "eps": round(float(e_pl[:, 0].mean()), 6),
                     "eps2": float(e2_pl[0]), "eps2_unit_norm": float(e2_pl[1])},
           "learned": {"adjoint_ms": round(t_le, 3), "adjoint_with_histogram_ms": round(t_hist, 3),
                       "proposal_upkeep_ms": round(upkeep_ms, 3), "ms_per_gradient": round(t_learn, 3),
                       "eps": round(float(e_le[:, 0].mean()), 6), "eps2": float(e2_le[0]),
                       "eps2_unit_norm": float(e2_le[1])},
           "variance_ratio": round(float(e2_le[0] / e2_pl[0]), 4),
           "variance_ratio_90ci": [round(float(np.percentile(bs, 5)), 4), round(float(np.percentile(bs, 95)), 4)],
           "eps2_t_ratio": round(float(ratio), 4),
           "eps2_t_ratio_unit_norm": round(float(e2_le[1] * t_learn / (e2_pl[1] * t_pl)), 4)}
    if pt_seeds <= 0:
        return res
    _, t_pt1 = pt_timed(1, 0x60000, 2)
    M_pt = max(1, int(round(t_pl / t_pt1)))
    g_pt, t_pt = pt_timed(M_pt, 0x70000, pt_seeds)
    e_pt = np.asarray([errs(x) for x in g_pt])
    e2_pt = (e_pt ** 2).mean(0)
    mean_pt = torch.stack([x.double() for x in g_pt]).mean(0)
    bias = float((mean_pt - ref).norm() / ref.norm())
    bias_se = float(math.sqrt(e2_pt[0] / pt_seeds))
    res["path_tracing"] = {"estimator": "object-space path tracing, next-event estimation, same texels",
                           "samples_per_texel": M_pt, "seeds": pt_seeds, "adjoint_ms": round(t_pt, 3),
                           "eps": round(float(e_pt[:, 0].mean()), 6), "eps2": float(e2_pt[0]),
                           "eps2_unit_norm": float(e2_pt[1]),
                           "mean_vs_reference": round(bias, 6), "mean_standard_error": round(bias_se, 6),
                           "eps2_t_ratio_vs_light_tracing": round(float(e2_pt[0] * t_pt / (e2_pl[0] * t_pl)), 3),
                           "eps2_t_ratio_vs_light_tracing_unit_norm":
                               round(float(e2_pt[1] * t_pt / (e2_pl[1] * t_pl)), 3)}
    return res


WORKLOADS = {
    "building": ("building_floor", "building floor 80x60x3.2 m"),
    "office": ("office", "procedural office 30x20x3 m"),
    "room_set": ("room_set", "room set (four 6x5x3 m rooms), 64 candidate layouts of 4-48 point/spot lights"),
}


def throughput(name, args, paths=0, steps=None, warmup=None):
    """Set up one workload, time forward + adjoint steps; returns (ctx, wl,
    buffers, result dict with value, ms per step, kernel times and the
    roofline of the dominant kernel)."""
    import torch
    import lt_inputs as li
    from paper_2310_02043_amd import Context
    gen, desc = WORKLOADS[name]
    wl = getattr(li, gen)()
    scene, lights = wl["scene"], wl["lights"]
    B, seed = wl["max_hits"], wl["seed"]
    N = paths if paths else wl["paths"]   # paths per layout
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    n_layouts = lights.n_layouts
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    if args.tuning:
        ctx.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
    log(name, "scene", ctx.info())
    dev = "cuda:0"
    p = torch.tensor(lights.params, device=dev)
    K = scene.n_texels
    Et = torch.tensor(np.stack([li.painted_target(scene, 0.5, seed=j) for j in range(n_layouts)]), device=dev)
    S = torch.empty((n_layouts, K), dtype=torch.int64, device=dev)
    E = torch.empty((n_layouts, K), dtype=torch.float32, device=dev)
    g = torch.empty((n_layouts, K), dtype=torch.float32, device=dev)
    O = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty((lights.n_lights, 6), dtype=torch.float32, device=dev)
    cfg = ctx.cfg(seed, N, B, graph=args.graph)
    if not args.tuning and not args.no_autotune:
        t0 = time.time()
        g.normal_()
        cache = args.tuning_cache if args.tuning_cache else None
        best = ctx.autotune(p, ctx.cfg(seed, N, B), S, E, g, grad, cache_path=cache)
        log(f"{name} autotune: {ctx.get_tuning().as_dict()} ({best:.1f} ms fwd+adj, {time.time() - t0:.1f} s)")

    def step():
        ctx.trace_forward(p, cfg, S=S, E=E)
        ctx.objective(E, Et, g=g, O=O)
        ctx.trace_adjoint(p, g, cfg, grad=grad)

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"{name} warmup {i + 1}/{warmup} done")
    ctx.sync()
    # algorithmic work of one pass (instrumented forward kernel, untimed)
    stats = ctx.trace_stats(p, cfg)
    log(f"{name} work per pass", stats)

    # kernel durations: HIP events recorded on the launch stream around each
    # trace kernel inside the timed region (direct launches); with graph
    # replay, the same number of steps is launched directly afterwards
    ctx.timing_read()
    ctx.set_timing(not args.graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flags = ctx.sync()
    ms_step = (t1 - t0) * 1000.0 / steps
    total_paths = N * n_layouts
    value = total_paths / (ms_step / 1000.0)
    if args.graph:
        ctx.set_timing(True)
        kcfg = ctx.cfg(seed, N, B)
        for i in range(steps):
            ctx.trace_forward(p, kcfg, S=S, E=E)
            ctx.objective(E, Et, g=g, O=O)
            ctx.trace_adjoint(p, g, kcfg, grad=grad)
        torch.cuda.synchronize()
    ctx.set_timing(False)
    fwd_ms, nf, adj_ms, na = ctx.timing_read()
    fwd_avg, adj_avg = fwd_ms / max(nf, 1), adj_ms / max(na, 1)
    log(f"{name} step {ms_step:.2f} ms  fwd kernel {fwd_avg:.2f} ms  adj kernel {adj_avg:.2f} ms  flags {flags}")

    dominant = "adjoint" if adj_avg >= fwd_avg else "forward"
    dur_s = max(fwd_avg, adj_avg) / 1000.0
    ops = BOXES_PER_NODE * OPS_PER_BOX * stats["nodes"] + OPS_PER_TRI * stats["tri_tests"]
    slots = BOXES_PER_NODE * SLOTS_PER_BOX * stats["nodes"] + SLOTS_PER_TRI * stats["tri_tests"]
    byt = NODE_BYTES * stats["nodes"] + TRI_BYTES * stats["tri_tests"] + \
        (PATCH_BYTES + (4 if dominant == "adjoint" else 8)) * stats["hits"]
    tflops = ops / dur_s / 1e12
    gbs = byt / dur_s / 1e9
    reqs = REQ_PER_NODE * stats["nodes"] + REQ_PER_TRI * stats["tri_tests"] + REQ_PER_HIT * stats["hits"]
    traffic = measured_traffic(name, dominant, ctx.get_tuning().as_dict(), N)
    # The traversal is bound on the chip's issue side, not by HBM (~10 % of
    # its peak): the committed profiles show wave-level VALU issue at ~100 %
    # of the wave64 rate and the vector-memory path (TA/TD) busy ~100 %, so
    # the headline roofline is the ALU one (algorithmic box and triangle
    # operations against the FP32 vector peak), with the per-lane request
    # rate of the vector-memory path beside it.
    roofline = {"bound": "alu", "achieved": round(tflops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tflops / FP32_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": f"k_trace ({dominant})", "kernel_ms": round(max(fwd_avg, adj_avg), 3),
                "unpacked_issue": {"peak": round(UNPACKED_LANE_OPS_T, 1), "unit": "Tslots/s",
                                   "achieved": round(slots / dur_s / 1e12, 3),
                                   "frac": round(slots / dur_s / 1e12 / UNPACKED_LANE_OPS_T, 4),
                                   "note": f"algorithmic VALU issue slots (box test {SLOTS_PER_BOX}, triangle "
                                           f"test {SLOTS_PER_TRI}; an FMA is one slot) against one non-packed "
                                           "FP32 slot per lane per cycle, 256 CU x 4 SIMD x 16 lanes x 2.4 GHz"},
                "vmem_requests": {"achieved": round(reqs / dur_s / 1e9, 1), "peak": round(VMEM_REQ_PEAK_G, 1),
                                  "unit": "G lane-requests/s", "frac": round(reqs / dur_s / 1e9 / VMEM_REQ_PEAK_G, 4),
                                  "per_launch": int(reqs),
                                  "note": f"per-lane 16 B loads: {REQ_PER_NODE} per node visit, {REQ_PER_TRI} per "
                                          f"triangle test, {REQ_PER_HIT} per hit; about one distinct cache line per CU per clock, "
                                          "256 CU x 2.4 GHz"},
                "ops_per_launch": int(ops),
                "hbm": {"achieved": None if traffic is None else round(traffic / dur_s / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": None if traffic is None else round(traffic / dur_s / 1e9 / HBM_PEAK_GBS, 4)},
                "cache_level": {"achieved": round(gbs, 1), "unit": "GB/s", "bytes_per_launch": int(byt),
                                "note": "node, triangle and patch bytes the traversal reads, served by L2 and "
                                        "the Infinity Cache"},
                "work_per_launch": stats}
    res = {"value": round(value, 1), "ms_per_step": round(ms_step, 3), "fwd_kernel_ms": round(fwd_avg, 3),
           "adj_kernel_ms": round(adj_avg, 3), "roofline": roofline,
           "config": {"workload": f"{desc}, {scene.n_tris} triangles, {K} texels, {lights.n_lights} luminaires, "
                                  f"{n_layouts} layout(s) x {N} paths, {B} hits",
                      "paths": total_paths, "paths_per_layout": N, "layouts": n_layouts, "max_hits": B,
                      "triangles": scene.n_tris, "texels": K, "luminaires": lights.n_lights,
                      "graph": bool(args.graph), "tuning": ctx.get_tuning().as_dict(),
                      "parallelism": "single GPU"}}
    bufs = dict(p=p, S=S, E=E, g=g, grad=grad, N=N, B=B, seed=seed)
    return ctx, wl, bufs, res


def kernel_extras(ctx, bufs):
    """Gradient-contribution map and direct-differentiation map of luminaire
    0's x coordinate, timed beside the plain passes."""
    import torch
    p, g, grad, N, B, seed = (bufs[k] for k in ("p", "g", "grad", "N", "B", "seed"))
    K = ctx.n_texels
    out = {}
    vote = torch.empty(K, dtype=torch.float64, device="cuda:0")
    vcfg = ctx.cfg(seed, N, B)
    ctx.gradient_votes(p, g, vcfg, 0, 0, vote=vote, grad=grad)
    torch.cuda.synchronize()
    ctx.timing_read()
    ctx.set_timing(True)
    for i in range(3):
        ctx.gradient_votes(p, g, vcfg, 0, 0, vote=vote, grad=grad)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    _, _, v_ms, nv = ctx.timing_read()
    out["gradient_votes"] = {"kernel_ms": round(v_ms / max(nv, 1), 3), "light": 0, "param": "x"}
    ctx.trace_tangent(p, vcfg, 0, 0)
    torch.cuda.synchronize()
    ctx.timing_read()
    ctx.set_timing(True)
    for i in range(3):
        ctx.trace_tangent(p, vcfg, 0, 0)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    t_ms, nt, _, _ = ctx.timing_read()
    out["direct_differentiation"] = {"kernel_ms": round(t_ms / max(nt, 1), 3), "light": 0, "param": "x"}
    log("extras", out)
    return out


def directional(ctx, scene, bufs, order=3, ns=4):
    """Directional texels at the paper's Table 1 order (3, 16 coefficients
    per texel), 4 local samples, glossy surfaces (rho_s 0.3, e 20)."""
    import torch
    p, N, B, seed = bufs["p"], bufs["N"], bufs["B"], bufs["seed"]
    nc = (order + 1) ** 2
    n_layouts, K = ctx.n_layouts, ctx.n_texels
    ctx.set_glossy(np.stack([np.full(scene.n_patches, 0.3), np.full(scene.n_patches, 20.0)], 1).astype(np.float32))
    Sd = torch.empty((n_layouts, nc, K), dtype=torch.int64, device="cuda:0")
    Ed = torch.empty((n_layouts, nc, K), dtype=torch.float32, device="cuda:0")
    gd = torch.randn((n_layouts, nc, K), device="cuda:0")
    gradd = torch.empty_like(bufs["grad"])
    vcfg = ctx.cfg(seed, N, B)
    ctx.trace_forward_dir(p, vcfg, order, ns, S=Sd, E=Ed)
    ctx.trace_adjoint_dir(p, gd, vcfg, order, ns, grad=gradd)
    torch.cuda.synchronize()
    ctx.timing_read()
    ctx.set_timing(True)
    for i in range(2):
        ctx.trace_forward_dir(p, vcfg, order, ns, S=Sd, E=Ed)
        ctx.trace_adjoint_dir(p, gd, vcfg, order, ns, grad=gradd)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    f_ms, nf, a_ms, na = ctx.timing_read()
    out = {"order": order, "local_samples": ns, "fwd_kernel_ms": round(f_ms / max(nf, 1), 3),
           "adj_kernel_ms": round(a_ms / max(na, 1), 3)}
    log("directional texels", out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="building")
    ap.add_argument("--paths", type=int, default=0, help="paths per layout (default: the workload's)")
    ap.add_argument("--graph", action="store_true", help="replay forward / adjoint as captured hipGraphs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch tuning instead of the autotuner's choice")
    ap.add_argument("--tuning-cache", type=str, default=TUNING_CACHE,
                    help="autotuner cache file (a matching entry is reused; new results are appended)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline line: no contribution / direct-differentiation maps, no office line, "
                         "no directional texels, no learned-proposal study")
    ap.add_argument("--no-proposal-study", action="store_true",
                    help="skip the learned-proposal gradient error x time comparison")
    ap.add_argument("--tuning", type=str, default="", help="k=v,... launch tuning override")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device 3 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {n * 4} bytes 3 times")
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of this "
              f"path is described in the design notes and not launched here.", file=sys.stderr)
        sys.exit(2)

    ctx, wl, bufs, head = throughput(args.workload, args, paths=args.paths)
    out = {
        "metric": METRIC + ("" if args.workload == "building" else f" [{args.workload}]"),
        "value": head["value"], "unit": "paths/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+i64", "data": "synthetic", "config": head["config"],
        "fwd_kernel_ms": head["fwd_kernel_ms"], "adj_kernel_ms": head["adj_kernel_ms"],
        "roofline": head["roofline"], "cpu_baseline": None,
    }
    if not args.no_extras:
        out.update(kernel_extras(ctx, bufs))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl["scene"], wl["lights"], bufs["seed"], bufs["N"], bufs["B"],
                                           args.cpu_seconds)
        log("cpu baseline", out["cpu_baseline"])
    if not args.no_extras:
        if args.workload == "office":
            octx, owl, obufs = ctx, wl, bufs
        else:
            del ctx, bufs
            octx, owl, obufs, office = throughput("office", args, steps=3, warmup=1)
            out["office"] = {"value": office["value"], "unit": "paths/s", "ms_per_step": office["ms_per_step"],
                             "fwd_kernel_ms": office["fwd_kernel_ms"], "adj_kernel_ms": office["adj_kernel_ms"],
                             "roofline_frac": office["roofline"]["frac"],
                             "traffic": office["roofline"]["traffic"], "workload": office["config"]["workload"]}
        out["directional"] = directional(octx, owl["scene"], obufs)
        if not args.no_proposal_study:
            log("learned proposal vs plain: gradient error x time ...")
            out["grad_error_time"] = proposal_study(octx, owl, obufs["N"], at="initial")
            log("proposal study (initial)", json.dumps(out["grad_error_time"]))
            out["grad_error_time_converged"] = proposal_study(octx, owl, obufs["N"], at="converged", pt_seeds=0)
            log("proposal study (converged)", json.dumps(out["grad_error_time_converged"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
