"""Learned emission proposal on the GPU (through the C ABI).

* MFMA inference of the proposal network vs the numpy oracle (bf16 rounding
  points mirrored);
* the training kernel's gradient vs the oracle's hand-derived backprop;
* sampling with a proposal table: texels, gradients and the adjoint histogram
  vs the CPU oracle given the same table;
* unbiasedness: mean gradient with a proposal equals the plain mean;
* online training from the tracer's own adjoint histograms lowers the loss.
"""
import math

import numpy as np
import pytest

import lt_inputs as li

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def office_ctx(torch, scene, lights):
    from paper_2310_02043_amd import Context
    ctx = Context(0)
    ctx.upload_scene(scene.verts, scene.tris, scene.tri_patch, scene.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    return ctx


def _weights(rng, scale=0.15):
    from oracle import proposal as op
    w = rng.normal(0, scale, op.N_WEIGHTS).astype(np.float32)
    return w


def _inputs(rng, L):
    from oracle import proposal as op
    x = np.zeros((L, op.IN), np.float32)
    x[:, :op.NPAR + op.NEMB] = rng.normal(0, 1, (L, op.NPAR + op.NEMB))
    return x


def _ctx_with_lights(torch, n):
    """Box room with n cos^n spots (the network's batch is one row per light)."""
    from lt_inputs.scenes import make_lights, SPOT
    from paper_2310_02043_amd import Context
    sc = li.box_room()["scene"]
    rng = np.random.default_rng(n)
    ps = [[rng.uniform(0.5, 3.5), rng.uniform(0.5, 2.5), rng.uniform(1.5, 2.4), rng.uniform(-0.3, 0.3),
           rng.uniform(-0.3, 0.3), rng.uniform(5, 20)] for _ in range(n)]
    lights = make_lights([SPOT] * n, rng.uniform(1, 6, n), [(0, 0)] * n, [0] * n, ps)
    ctx = Context(0)
    ctx.upload_scene(sc.verts, sc.tris, sc.tri_patch, sc.patches)
    ctx.set_lights(lights.static, lights.layout_offsets)
    return ctx


@pytest.mark.parametrize("L", [13, 16, 128])
def test_mlp_inference_matches_oracle(torch_dev, L):
    """MFMA inference (16-row blocks, so 13 is one partial block and 128 the
    building floor's eight) against the numpy network with the same bfloat16
    rounding points: logits within 1e-5 of the row's largest and cell
    probabilities within 1e-5 in L1, per light.  Where FP32 accumulation may
    legitimately round a hidden activation to the other bfloat16 neighbour
    (the exact value lies within the accumulation bound of a tie), every such
    rounding is admissible and the GPU must match one of them; a truncating
    conversion or a dropped tail row fails."""
    torch = torch_dev
    from oracle import proposal as op
    ctx = _ctx_with_lights(torch, L)
    rng = np.random.default_rng(L)
    w = _weights(rng)
    x = _inputs(rng, L)
    wb = torch.tensor(op.bf16_bits(w).view(np.int16), device="cuda")
    logits = torch.full((L, 1024), float("nan"), dtype=torch.float32, device="cuda")
    ctx.mlp_infer(wb, torch.tensor(x, device="cuda"), logits)
    pdf_d, cdf_d = ctx.proposal_get_table()
    torch.cuda.synchronize()
    z = logits.cpu().numpy().astype(np.float64)
    pdf = pdf_d.cpu().numpy().astype(np.float64)
    alts = op.infer_alternatives(w, x)
    checked, multi, worst_z, worst_p = 0, 0, 0.0, 0.0
    for r in range(L):
        assert alts[r] is not None, f"row {r}: too many admissible roundings"
        best = min(alts[r], key=lambda zp: np.abs(z[r] - zp[0]).max())
        ez = float(np.abs(z[r] - best[0]).max() / np.abs(best[0]).max())
        ep = float(np.abs(pdf[r] - best[1]).sum())
        worst_z, worst_p = max(worst_z, ez), max(worst_p, ep)
        checked += 1
        multi += len(alts[r]) > 1
        assert ez <= 1e-5 and ep <= 1e-5, (r, ez, ep, len(alts[r]))
    say(f"  L={L}: logits max rel err {worst_z:.2e}, pdf L1 {worst_p:.2e} "
        f"({multi} of {checked} rows with an ambiguous bf16 rounding)")
    cdf = cdf_d.cpu().numpy()
    assert np.all(cdf[:, -1] == 1.0) and np.all(np.diff(cdf, axis=1) >= 0)
    assert np.allclose(pdf.sum(1), 1.0, atol=1e-5)


def test_mlp_training_step_matches_oracle(torch_dev):
    torch = torch_dev
    from oracle import proposal as op
    c2 = li.office(target_tris=20_000, target_texels=200_000)
    ctx = office_ctx(torch, c2["scene"], c2["lights"])
    rng = np.random.default_rng(1)
    L = ctx.n_lights
    w = _weights(rng)
    x = _inputs(rng, L)
    t = rng.dirichlet(np.ones(1024) * 0.3, L).astype(np.float32)
    loss_ref, g_ref, gx_ref = op.loss_and_grad(w, x, t)
    d = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    wd, xd = d(w), d(x)
    mw, vw = torch.zeros_like(wd), torch.zeros_like(wd)
    mx, vx = torch.zeros_like(xd), torch.zeros_like(xd)
    wb = torch.zeros(op.N_WEIGHTS, dtype=torch.int16, device="cuda")
    loss = torch.zeros(1, device="cuda")
    gout = torch.zeros(op.N_WEIGHTS + L * op.IN, device="cuda")
    lr = 1e-3
    ctx.mlp_train(wd, mw, vw, wb, xd, mx, vx, d(t), 1, lr, loss=loss, grad_out=gout)
    torch.cuda.synchronize()
    g = gout.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g[:op.N_WEIGHTS] - g_ref) / np.linalg.norm(g_ref)
    relx = np.linalg.norm(g[op.N_WEIGHTS:].reshape(L, op.IN) - gx_ref) / np.linalg.norm(gx_ref)
    say(f"  loss {loss.item():.6f} vs {loss_ref:.6f}; grad rel-L2 {rel:.2e}, embedding grad {relx:.2e}")
    assert abs(loss.item() / loss_ref - 1) < 1e-5
    assert rel < 1e-4 and relx < 1e-4
    w_ref, _, _ = op.adam(w.astype(np.float64), 0.0, 0.0, g_ref, 1, lr)
    big = np.abs(g_ref) > 1e-4 * np.abs(g_ref).max()
    assert np.allclose(wd.cpu().numpy()[big], w_ref[big], atol=1e-6 + 1e-3 * lr)
    assert np.array_equal(wb.cpu().numpy().view(np.uint16), op.bf16_bits(wd.cpu().numpy()))


def test_proposal_train_step_matches_oracle(torch_dev, oracle_lib):
    """The context-held network (lt_proposal_set / refresh / update_scale /
    train_step): inputs normalised from the parameters, the training target
    from two successive histograms (running average, square root, plain-lobe
    floor; one light's row empty) within 1e-6 of the oracle's, one Adam step
    toward it equal to the oracle's backprop + Adam, and the histogram scale
    from two successive gradients driving an adjoint histogram equal to the
    oracle's."""
    torch = torch_dev
    from oracle import proposal as op
    c2 = li.office(target_tris=20_000, target_texels=200_000)
    sc, lights = c2["scene"], c2["lights"]
    ctx = office_ctx(torch, sc, lights)
    L = ctx.n_lights
    rng = np.random.default_rng(12)
    d = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    w = _weights(rng, 0.1)
    emb = rng.normal(0, 0.5, (L, 16)).astype(np.float32)
    lo = np.array([0, 0, 2.5, -0.6, -0.6, 0], np.float32)
    hi = np.array([30, 20, 3.0, 0.6, 0.6, 80], np.float32)
    decay, floor, sdecay, lr = 0.8, 0.3, 0.9, 1e-3
    ctx.proposal_set(d(w), d(emb), lo, hi, hist_decay=decay, plain_floor=floor, sigma_decay=sdecay)
    p = lights.params.astype(np.float32)
    ctx.proposal_refresh(d(p))
    w0, x0 = (t.cpu().numpy() for t in ctx.proposal_get_net())
    x_ref = np.zeros((L, 32), np.float32)
    x_ref[:, :6] = (np.float32(2.0) * (p - lo)) / (hi - lo) - np.float32(1.0)
    x_ref[:, 6:22] = emb
    assert np.array_equal(w0, w) and np.array_equal(x0, x_ref)
    pm = op.plain_cell_mass(lights.static["lobe_n"])
    h1 = rng.gamma(0.3, 1.0, (L, 1024)).astype(np.float32)
    h1[3] = 0.0
    h2 = rng.gamma(0.3, 1.0, (L, 1024)).astype(np.float32)
    loss = torch.zeros(1, device="cuda")
    tgt = torch.empty((L, 1024), device="cuda")
    ctx.proposal_train_step(d(h1), lr, 1, loss=loss, target_out=tgt)
    t1 = tgt.cpu().numpy()
    t1_ref, avg = op.training_target(h1, None, decay, pm, floor)
    e1 = np.abs(t1 - t1_ref).max() / t1_ref.max()
    w1 = ctx.proposal_get_net()[0].cpu().numpy()
    loss_ref, g_ref, _ = op.loss_and_grad(w, x_ref, t1)
    w1_ref, _, _ = op.adam(w.astype(np.float64), 0.0, 0.0, g_ref, 1, lr)
    big = np.abs(g_ref) > 1e-4 * np.abs(g_ref).max()
    say(f"  target rel err {e1:.2e}; loss {loss.item():.6f} vs {loss_ref:.6f}")
    assert e1 <= 1e-6 and np.allclose(t1.sum(1), 1.0, atol=1e-5)
    assert abs(loss.item() / loss_ref - 1) < 1e-5
    assert np.allclose(w1[big], w1_ref[big], atol=1e-6 + 1e-3 * lr)
    ctx.proposal_train_step(d(h2), lr, 0, target_out=tgt)
    t2_ref, _ = op.training_target(h2, avg, decay, pm, floor)
    e2 = np.abs(tgt.cpu().numpy() - t2_ref).max() / t2_ref.max()
    say(f"  second target (running average) rel err {e2:.2e}")
    assert e2 <= 1e-6
    # histogram units from two gradients, seen through the adjoint histogram
    mask = [1, 1, 0, 1, 1, 1]
    g1 = rng.normal(0, 3, (L, 6)).astype(np.float32)
    g2 = rng.normal(0, 3, (L, 6)).astype(np.float32)
    ctx.proposal_update_scale(d(g1), mask)
    ctx.proposal_update_scale(d(g2), mask)
    s2 = np.float32(sdecay) * (g1 * g1) + (np.float32(1.0) - np.float32(sdecay)) * (g2 * g2)
    inv_sigma = (np.float32(1.0) / np.sqrt(s2 + np.float32(1e-30))) * np.array(mask, np.float32)
    ctx.proposal_refresh(d(p))
    pdf, cdf = (t.cpu().numpy() for t in ctx.proposal_get_table())
    N, B, seed = 1 << 16, c2["max_hits"], 0x77
    cfg = ctx.cfg(seed, N, B, proposal=True, alpha_plain=0.2)
    prop = oracle_lib.Proposal(pdf, cdf, 0.2, inv_sigma=inv_sigma, with_hist=True)
    osc, ol = oracle_lib.OracleScene(sc, use_bvh=True), oracle_lib.OracleLights(lights)
    S_ref, _ = oracle_lib.forward(osc, ol, p, seed, N, B, proposal=prop)
    _, g_ref2 = oracle_lib.objective(oracle_lib.fixed_to_float(S_ref), li.painted_target(sc, 0.5)[None],
                                     sc.texel_area())
    prop.hist[:] = 0.0
    oracle_lib.adjoint(osc, ol, p, seed, N, B, g_ref2, proposal=prop)
    hist_d = torch.zeros((L, 1024), device="cuda")
    ctx.trace_adjoint(d(p), d(g_ref2), cfg, bin_hist=hist_d)
    torch.cuda.synchronize()
    herr = np.linalg.norm(hist_d.cpu().numpy() - prop.hist) / np.linalg.norm(prop.hist)
    say(f"  adjoint histogram with the context's scale: rel-L2 {herr:.2e}")
    assert herr <= 1e-4


def _table(rng, L, types):
    from oracle.proposal import cdf_table
    logits = rng.normal(0, 2.5, (L, 1024))
    p = np.exp(logits - logits.max(1, keepdims=True))
    p = (p / p.sum(1, keepdims=True)).astype(np.float32)
    return p, cdf_table(p)


def test_proposal_sampling_parity(torch_dev, oracle_lib):
    torch = torch_dev
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    ctx = office_ctx(torch, sc, lights)
    rng = np.random.default_rng(5)
    pdf, cdf = _table(rng, lights.n_lights, lights.static["type"])
    inv_sigma = rng.uniform(0.5, 2.0, (lights.n_lights, 6)).astype(np.float32)
    d = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    ctx.proposal_set_table(d(pdf), d(cdf))
    ctx.proposal_set_scale(d(inv_sigma))
    N, B, seed = 1 << 18, c2["max_hits"], 0x515
    cfg = ctx.cfg(seed, N, B, proposal=True, alpha_plain=0.2)
    p_d = d(lights.params)
    E_d, S_d = ctx.trace_forward(p_d, cfg)
    prop = oracle_lib.Proposal(pdf, cdf, 0.2, inv_sigma=inv_sigma, with_hist=True)
    osc, ol = oracle_lib.OracleScene(sc, use_bvh=True), oracle_lib.OracleLights(lights)
    S_ref, _ = oracle_lib.forward(osc, ol, lights.params, seed, N, B, proposal=prop)
    same = float((S_d.cpu().numpy() == S_ref).mean())
    say(f"  texels bit-identical {same * 100:.4f} %")
    E_ref = oracle_lib.fixed_to_float(S_ref)
    assert np.linalg.norm(E_d.cpu().numpy() - E_ref) / np.linalg.norm(E_ref) <= 1e-4
    _, g_ref = oracle_lib.objective(E_ref, li.painted_target(sc, 0.5)[None], sc.texel_area())
    grad_ref, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, N, B, g_ref, proposal=prop)
    hist_d = torch.zeros((lights.n_lights, 1024), device="cuda")
    grad_d = ctx.trace_adjoint(p_d, d(g_ref), cfg, bin_hist=hist_d)
    torch.cuda.synchronize()
    gg = grad_d.cpu().numpy()
    scale = np.maximum(np.abs(grad_ref), 1e-6 * np.abs(grad_ref).max())
    err = float(np.max(np.abs(gg - grad_ref) / scale))
    herr = np.linalg.norm(hist_d.cpu().numpy() - prop.hist) / np.linalg.norm(prop.hist)
    say(f"  gradient max rel err {err:.2e}; histogram rel-L2 {herr:.2e}")
    assert err <= 1e-3 and herr <= 1e-4


@pytest.mark.parametrize("basis", ["box", "linear"])
def test_proposal_mixed_light_types(torch_dev, oracle_lib, basis):
    """Box room with a point light, a cos^n spot, a rectangle and a
    soft-edged spot under a proposal table: the table applies to the spot and
    the rectangle only, on both sides; histogram rows of the others stay 0.
    With the box and the piecewise-linear texel basis."""
    from lt_inputs.scenes import make_lights, POINT, SPOT, RECT, SOFT
    torch = torch_dev
    sc = li.box_room()["scene"]
    lights = make_lights([POINT, SPOT, RECT, SOFT], [0.0, 3.0, 1.0, 0.0], [(0, 0), (0, 0), (0.5, 0.3), (0.3, 0.8)],
                         [0, 0, 0, 0], [[3.0, 2.0, 1.8, 0, 0, 30.0], [1.0, 1.0, 2.2, 0.1, 0.2, 50.0],
                                        [2.0, 1.5, 2.4, -0.2, 0.3, 70.0], [2.8, 0.9, 2.3, 0.25, -0.1, 40.0]])
    ctx = office_ctx(torch, sc, lights)
    rng = np.random.default_rng(8)
    pdf, cdf = _table(rng, lights.n_lights, lights.static["type"])
    inv_sigma = rng.uniform(0.5, 2.0, (lights.n_lights, 6)).astype(np.float32)
    d = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    ctx.proposal_set_table(d(pdf), d(cdf))
    ctx.proposal_set_scale(d(inv_sigma))
    N, B, seed = 1 << 18, 4, 0x5A5
    cfg = ctx.cfg(seed, N, B, proposal=True, alpha_plain=0.3, linear=basis == "linear")
    p_d = d(lights.params)
    E_d, S_d = ctx.trace_forward(p_d, cfg)
    prop = oracle_lib.Proposal(pdf, cdf, 0.3, inv_sigma=inv_sigma, with_hist=True)
    osc, ol = oracle_lib.OracleScene(sc, basis=basis), oracle_lib.OracleLights(lights)
    S_ref, _ = oracle_lib.forward(osc, ol, lights.params, seed, N, B, proposal=prop)
    same = float((S_d.cpu().numpy() == S_ref).mean())
    say(f"  texels bit-identical {same * 100:.4f} %")
    E_ref = oracle_lib.fixed_to_float(S_ref)
    assert np.linalg.norm(E_d.cpu().numpy() - E_ref) / np.linalg.norm(E_ref) <= 1e-4
    _, g_ref = oracle_lib.objective(E_ref, li.painted_target(sc, 2.0)[None], sc.texel_area())
    grad_ref, _ = oracle_lib.adjoint(osc, ol, lights.params, seed, N, B, g_ref, proposal=prop)
    hist_d = torch.zeros((lights.n_lights, 1024), device="cuda")
    grad_d = ctx.trace_adjoint(p_d, d(g_ref), cfg, bin_hist=hist_d)
    torch.cuda.synchronize()
    gg = grad_d.cpu().numpy()
    scale = np.maximum(np.abs(grad_ref), 1e-6 * np.abs(grad_ref).max())
    err = float(np.max(np.abs(gg - grad_ref) / scale))
    h = hist_d.cpu().numpy()
    herr = np.linalg.norm(h - prop.hist) / np.linalg.norm(prop.hist)
    say(f"  gradient max rel err {err:.2e}; histogram rel-L2 {herr:.2e}")
    assert err <= 1e-3 and herr <= 1e-4
    assert not h[0].any() and not h[3].any() and h[1].any() and h[2].any()


def test_proposal_unbiased_vs_plain(torch_dev):
    """Mean gradient over 16 seeds with a (deliberately poor) random proposal
    equals the plain tracer's mean within statistical error."""
    torch = torch_dev
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    ctx = office_ctx(torch, sc, lights)
    rng = np.random.default_rng(6)
    pdf, cdf = _table(rng, lights.n_lights, lights.static["type"])
    d = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    ctx.proposal_set_table(d(pdf), d(cdf))
    p_d = d(lights.params)
    N, B = 1 << 22, c2["max_hits"]
    Et = d(li.painted_target(sc, 0.5)[None])
    E_hi, _ = ctx.trace_forward(p_d, ctx.cfg(99, 1 << 26, B))
    _, g = ctx.objective(E_hi, Et)
    G = {False: [], True: []}
    for s in range(16):
        for prop in (False, True):
            cfg = ctx.cfg(1000 + s, N, B, proposal=prop, alpha_plain=0.2)
            G[prop].append(ctx.trace_adjoint(p_d, g, cfg).cpu().numpy().astype(np.float64))
    a, b = np.array(G[False]), np.array(G[True])
    diff = a.mean(0) - b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / 16 + b.var(0, ddof=1) / 16)
    z = np.abs(diff) / np.maximum(se, 1e-30)
    say("  max |z| plain vs proposal:", float(z.max()))
    assert z.max() < 5.0


def test_online_training_lowers_loss(torch_dev):
    torch = torch_dev
    from paper_2310_02043_amd.proposal import LearnedProposal
    c2 = li.office()
    sc, lights = c2["scene"], c2["lights"]
    ctx = office_ctx(torch, sc, lights)
    d = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    p_d = d(lights.params)
    lp = LearnedProposal(ctx, [0, 0, 2.5, -0.6, -0.6, 0], [30, 20, 3.0, 0.6, 0.6, 80])
    lp.refresh(p_d)
    Et = d(li.painted_target(sc, 0.5)[None])
    N, B = 1 << 22, c2["max_hits"]
    losses = []
    for it in range(12):
        cfg = ctx.cfg(2000 + it, N, B, proposal=True, alpha_plain=0.2)
        E, _ = ctx.trace_forward(p_d, cfg)
        _, g = ctx.objective(E, Et)
        grad = ctx.trace_adjoint(p_d, g, cfg, bin_hist=lp.hist)
        lp.update_scale(grad)
        losses.append(lp.train(steps=8))
        lp.refresh(p_d)
    say("  training loss", [round(x, 3) for x in losses])
    assert losses[-1] < losses[0]
    pdf, cdf = ctx.proposal_get_table()
    assert torch.isfinite(pdf).all() and torch.all(cdf[:, -1] == 1.0)
