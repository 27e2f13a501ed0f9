"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (stated per output):
  labels     bit-exact (same canonical ids, same K);
  depth      |d_gpu - d_oracle| <= 1e-6 + 1e-4 |d_oracle| on every valid pixel;
  log_scale  |s_gpu - s_oracle| <= 1e-4 (log units);
  fill       |z_gpu - z_oracle| <= 1e-6 + 1e-4 (log-depth, per-component gauge).
The 1e-4 relative / 1e-6 absolute depth tolerance comes from the FP32
vectors of the fill CG (stopped at a 1e-6 relative residual) against an
exact FP64 solve.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ni_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RTOL, ATOL = 1e-4, 1e-6


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2510_11508_amd as ni
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ni.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def params(**kw):
    import paper_2510_11508_amd as ni
    return ni.ni_params_default(**kw)


def oracle_params(p):
    """The oracle's parameters for the library's; the baseline variant's
    effective parameters are spelled out, so that every oracle stage (not
    only integrate) runs the same loop."""
    op = dict(theta_c_deg=p.theta_c_deg, irls_iters=p.irls_iters, align_iters=p.align_iters, bini_k=p.bini_k,
              out_L=p.out_L, out_U=p.out_U, outlier_mode=p.outlier_mode, delta_e_max=p.delta_e_max,
              w_cut_rel=p.w_cut_rel, freq_merging=p.freq_merging, variant=p.variant, connectivity=p.connectivity)
    return O.baseline_params(op) if p.variant == 1 else op


def assert_depth_close(d_gpu, d_ref, mask, what="", ortho=False):
    """Perspective: per-pixel relative bound on depth.  Orthographic depth is
    an additive height in the per-region zero-mean gauge that crosses zero,
    so the relative part is taken w.r.t. the map's largest |height|."""
    v = mask > 0
    a = d_gpu.astype(np.float64)[v]
    b = d_ref[v]
    err = np.abs(a - b)
    scale = np.max(np.abs(b)) if (ortho and b.size) else np.abs(b)
    bound = ATOL + RTOL * scale
    worst = np.argmax(err / bound) if err.size else 0
    assert np.all(err <= bound), f"{what}: max err {err.max():.3e} at {worst}, ref {b[worst]:.6f}"
    assert np.all(np.isnan(d_gpu[~v])), f"{what}: off-mask depth must be NaN"


def assert_scale_close(s_gpu, s_ref, ortho=False):
    """Perspective log-scales: 1e-4 absolute (= 1e-4 relative depth).
    Orthographic offsets are heights: norm-wise like the depth."""
    err = np.abs(s_gpu - s_ref)
    bound = ATOL + RTOL * (np.max(np.abs(s_ref)) if (ortho and s_ref.size) else 1.0)
    assert err.size == 0 or err.max() <= bound, f"log_scale: max err {err.max():.3e} (bound {bound:.2e})"


SAMPLES = [("c1", 0), ("c1", 1), ("c1", 2), ("c2", 0), ("c2", 1)]


def sample(name, seed):
    if name.startswith("tiny"):
        proj = name.split("-")[1]
        return synth.tiny(seed, 9, 11, proj)
    return synth.make(name, seed)


# ----------------------------------------------------------------- labels
@pytest.mark.parametrize("name,seed", SAMPLES + [("tiny-persp", 0), ("tiny-ortho", 1), ("c3", 0)])
def test_labels_bit_exact(ctx, name, seed):
    s = sample(name, seed)
    p = params(theta_c_deg=2.0)
    log(f"[labels] {name} seed {seed} {s.mask.shape}")
    lab, K, _ = ctx.ni_label(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    ref, Kr = O.labels(e)
    assert K == Kr
    assert np.array_equal(lab.cpu().numpy(), ref)


@pytest.mark.parametrize("theta", [0.0, 0.5, 5.0, 180.0])
def test_labels_thresholds(ctx, theta):
    s = synth.make("c2", 3)
    log(f"[labels] c2 seed 3 theta {theta}")
    lab, K, _ = ctx.ni_label(dev(s.normals), dev(s.mask), s.cam.as_dict(), params(theta_c_deg=theta))
    ref, Kr = O.labels(O.edges(s.normals, s.mask, s.cam, theta))
    assert K == Kr and np.array_equal(lab.cpu().numpy(), ref)


# ------------------------------------------------------------------- fill
@pytest.mark.parametrize("precond", [1, 0])
@pytest.mark.parametrize("name,seed", [("c1", 0), ("c2", 0), ("c2", 4), ("tiny-persp", 2), ("tiny-ortho", 3)])
def test_fill_matches_oracle(ctx, name, seed, precond):
    s = sample(name, seed)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    zref = O.fill(e, lab, K)
    log(f"[fill] {name} seed {seed} K {K} precond {precond}")
    z, rep = ctx.ni_fill(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K, params(fill_precond=precond))
    z = z.cpu().numpy().astype(np.float64)
    v = s.mask > 0
    err = np.abs(z[v] - zref[v])
    assert err.max() <= 1e-6 + 1e-4, (err.max(), rep["fill_iters_max"])
    assert rep["fill_notconv"] == 0


@pytest.mark.parametrize("chunk", [512, 1024, 2048, 4096])
@pytest.mark.parametrize("split", [0, 1])
def test_fill_fixed_schedules(ctx, chunk, split):
    """Jacobi preconditioner: every schedule the autotuner chooses between,
    fixed by the caller, solves the large components to the same bound."""
    s = sample("c2", 0)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    zref = O.fill(e, lab, K)
    log(f"[fill schedule] c2 seed 0 chunk {chunk} split {split}")
    z, rep = ctx.ni_fill(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K,
                         params(fill_chunk=chunk, fill_split=split, fill_precond=0))
    assert rep["n_large"] > 0
    assert (rep["fill_chunk"], rep["fill_split"]) == (chunk, split)
    z = z.cpu().numpy().astype(np.float64)
    v = s.mask > 0
    assert np.abs(z[v] - zref[v]).max() <= 1e-6 + 1e-4
    assert rep["fill_notconv"] == 0


def degenerate_large_map():
    """Two components that just take the large path: a serpentine one pixel
    wide (8256 px: 2x2 aggregates of a line only halve it per level) and a
    block of exactly 8193 px, on a smooth orthographic quadric with a little
    seeded noise (every neighbour pair similar at 2 degrees)."""
    H, W = 160, 330
    n, _, _, cam = synth.quadric_ortho(H, W, (1e-4, 2e-5, 1.5e-4, 0.01, -0.02, 5.0))
    rng = np.random.default_rng(7)
    n = n + rng.normal(0.0, 0.002, n.shape)
    n = (n / np.linalg.norm(n, axis=-1, keepdims=True)).astype(np.float32)
    m = np.zeros((H, W), np.uint8)
    m[0:128:2, 0:128] = 1
    for r in range(1, 128, 2):
        m[r, 127 if (r // 2) % 2 == 0 else 0] = 1
    m[0:43, 140:330] = 1
    m[43, 140:163] = 1
    return n, m, cam


def test_fill_multigrid_fallback(ctx):
    """A multigrid solve stopped early (cap 3) hands the large components
    to the Jacobi path, which finishes them to the same bound."""
    s = sample("c2", 0)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    zref = O.fill(e, lab, K)
    log("[fill fallback] c2 seed 0, multigrid cap 3")
    z, rep = ctx.ni_fill(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K, params(fill_mg_maxit=3))
    assert rep["fill_mg_fallback"] == 1 and rep["n_large"] > 0
    z = z.cpu().numpy().astype(np.float64)
    v = s.mask > 0
    assert np.abs(z[v] - zref[v]).max() <= 1e-6 + 1e-4
    assert rep["fill_notconv"] == 0
    z2, rep2 = ctx.ni_fill(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K, params())
    assert rep2["fill_mg_fallback"] == 0


@pytest.mark.parametrize("precond", [1, 0])
def test_fill_degenerate_large_components(ctx, precond):
    n, m, cam = degenerate_large_map()
    e = O.edges(n, m, cam, 2.0)
    lab, K = O.labels(e)
    sizes = sorted(np.bincount(lab[lab >= 0]).tolist())
    assert K == 2 and sizes == [8193, 8256], sizes
    zref = O.fill(e, lab, K)
    log(f"[fill degenerate] serpentine + 8193-px block, precond {precond}")
    z, rep = ctx.ni_fill(dev(n), dev(m), cam.as_dict(), dev(lab), K, params(fill_precond=precond))
    assert rep["n_large"] == 2
    if precond == 1:
        assert rep["fill_mg_levels"] > 1
    z = z.cpu().numpy().astype(np.float64)
    v = m > 0
    assert np.abs(z[v] - zref[v]).max() <= 1e-6 + 1e-4 * np.abs(zref[v]).max()
    assert rep["fill_notconv"] == 0


# ------------------------------------------------------------------- IRLS
@pytest.mark.parametrize("name,seed", [("c1", 0), ("c2", 0), ("tiny-persp", 1), ("tiny-ortho", 0)])
@pytest.mark.parametrize("mode", [1, 2, 0])
def test_irls_matches_oracle_given_fill(ctx, name, seed, mode):
    s = sample(name, seed)
    p = params(theta_c_deg=2.0, irls_iters=int(s.params["irls_iters"]), outlier_mode=mode)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    # both sides take the oracle's fill rounded to FP32 (the fill vector's
    # precision on the HIP path), so the stage sees identical inputs
    zf = fp32(O.fill(e, lab, K))
    op = oracle_params(p)
    S, En, _ = O.irls(e, lab, K, zf, op)
    depth_ref, ls_ref, _ = O.finalize(e, lab, zf, S)
    log(f"[irls] {name} seed {seed} mode {mode} K {K}")
    depth, ls, rep = ctx.ni_irls(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K,
                                 dev(zf.astype(np.float32)), p)
    assert_depth_close(depth.cpu().numpy(), depth_ref, s.mask, f"irls {name}", s.cam.proj == "ortho")
    assert_scale_close(ls.cpu().numpy(), ls_ref, s.cam.proj == "ortho")
    assert np.allclose(rep["energy"], En, rtol=1e-3, atol=1e-12)


def fp32(z):
    return z.astype(np.float32).astype(np.float64)


def fill_tolerance_sensitivity(s, op, ref, seed=0):
    """How far the oracle's own output moves, in units of the depth bound,
    when its exact fill is replaced by one the fill step's specification
    also allows: per component, the solution error of a seeded random
    residual of relative norm cg_rtol = 1e-6 (L_c d_c = r_c, |r_c| = 1e-6
    |b_c|, solved exactly), then rounded to FP32 (the fill vector's
    precision on the HIP path).  Only the oracle runs here.  Above 0.5 the
    end-to-end output is not determined to the bound by what the fill
    specification fixes, and the whole path is compared stage by stage."""
    e = O.edges(s.normals, s.mask, s.cam, op["theta_c_deg"], op.get("connectivity", 4))
    lab, K = ref.labels, ref.K
    zf = ref.zfill
    Lap, rhs = O._intra_system(e, lab)
    labf = lab.ravel()
    act = labf >= 0
    g = np.where(act, labf, 0)
    rng = np.random.default_rng(seed)
    r = np.where(act, rng.standard_normal(labf.size), 0.0)
    # per component: |r_c| = 1e-6 |b_c|, zero sum (the range of L_c)
    sums = np.bincount(g[act], weights=r[act], minlength=max(K, 1))
    cnt = np.maximum(np.bincount(g[act], minlength=max(K, 1)), 1)
    r = np.where(act, r - (sums / cnt)[g], 0.0)
    rn = np.sqrt(np.bincount(g[act], weights=r[act] ** 2, minlength=max(K, 1)))
    bn = np.sqrt(np.bincount(g[act], weights=rhs[act] ** 2, minlength=max(K, 1)))
    r = np.where(act, r * (1e-6 * bn / np.maximum(rn, 1e-300))[g], 0.0)
    d = O._solve_pinned(Lap, r, g, max(K, 1), act).reshape(lab.shape)
    z = np.where(lab >= 0, fp32(zf + d), 0.0)
    S, _, _ = O.irls(e, lab, K, z, op)
    depth, _, _ = O.finalize(e, lab, z, S)
    v = s.mask > 0
    scale = np.max(np.abs(ref.depth[v])) if s.cam.proj == "ortho" else np.abs(ref.depth[v])
    return float(np.max(np.abs(depth[v] - ref.depth[v]) / (ATOL + RTOL * scale))) if np.any(v) else 0.0


def assert_fill_close(e, lab, K, z, zref, what):
    """Fill parity per component: within 1e-6 + 1e-4 (log-depth), or, where
    a component's exact solution moves by more than that under the stop
    rule itself, within what the rule allows: ||r_c|| <= 1e-6 ||b_c||
    bounds the error by 1e-6 ||b_c|| / lambda_2(L_c) <= 1e-6 ||b_c|| /
    lambda_min(L_c with one node pinned) (interlacing), plus 1e-7 ||b_c|| /
    lambda_min for the FP32 stencil and right-hand side, plus FP32 rounding
    of the output."""
    import scipy.sparse.linalg as spla
    v = lab >= 0
    labf = lab.ravel()
    err = np.where(v, np.abs(z - zref), 0.0).ravel()
    cerr = np.zeros(max(K, 1))
    np.maximum.at(cerr, labf[v.ravel()], err[v.ravel()])
    over = np.flatnonzero(cerr > ATOL + RTOL)
    if over.size == 0:
        return
    Lap, rhs = O._intra_system(e, lab)
    order = np.argsort(labf, kind="stable")
    starts = np.searchsorted(labf[order], np.arange(K + 1))
    for c in over:
        idx = order[starts[c]:starts[c + 1]]
        A = Lap[idx][:, idx].tocsc()[1:, 1:]
        lam = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
        bound = ATOL + 1.1e-6 * np.linalg.norm(rhs[idx]) / lam + 2.0 ** -24 * np.abs(zref.ravel()[idx]).max()
        log(f"[{what}] fill of component {c} ({idx.size} px): error {cerr[c]:.2e}, stop-rule bound {bound:.2e}")
        assert cerr[c] <= bound, (c, idx.size, cerr[c], bound)


def irls_chaos(s, op, lab, K, zf, seed=0):
    """How far the oracle's own relative-scale output moves, in units of the
    depth bound, when every step's exact solution is perturbed by seeded
    noise of 1e-12 of its largest entry (far below any solver's accuracy).
    Only the oracle runs here.  Above 0.5 the T-step loop is not determined
    by FP64 arithmetic on this input (the reweighting amplifies rounding
    from step to step), and the loop is compared one step at a time."""
    e = O.edges(s.normals, s.mask, s.cam, op["theta_c_deg"], op.get("connectivity", 4))
    S, _, _ = O.irls(e, lab, K, zf, op)
    d0, _, _ = O.finalize(e, lab, zf, S)
    rng = np.random.default_rng(seed)
    orig = O.quotient_step

    def noisy(ie, K_, w, r, cut):
        sres, E, wc = orig(ie, K_, w, r, cut)
        return sres + 1e-12 * max(np.abs(sres).max(), 1e-300) * rng.standard_normal(sres.size), E, wc

    O.quotient_step = noisy
    try:
        S1, _, _ = O.irls(e, lab, K, zf, op)
    finally:
        O.quotient_step = orig
    d1, _, _ = O.finalize(e, lab, zf, S1)
    v = s.mask > 0
    scale = np.max(np.abs(d0[v])) if s.cam.proj == "ortho" else np.abs(d0[v])
    return float(np.max(np.abs(d1[v] - d0[v]) / (ATOL + RTOL * scale))) if np.any(v) else 0.0


def check_irls_steps(ctx, s, p, op, lab, K, zf, what, steps=None):
    """The relative-scale loop one iteration at a time: from the oracle's
    scales before step t, the library's increment s^(t) and energy E_t
    against the oracle's (log-scale bound 1e-4, energy 1e-6 relative)."""
    e = O.edges(s.normals, s.mask, s.cam, op["theta_c_deg"], op.get("connectivity", 4))
    trace = []
    O.irls(e, lab, K, zf, op, trace=trace)
    T = len(trace)
    steps = sorted(set(steps or [0, 1, 2, 3, T // 2, T - 1]))
    for t in steps:
        _, S_before, s_ref, E_ref = trace[t]
        sg, E, rep = ctx.ni_irls_step(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K,
                                      dev(zf.astype(np.float32)), dev(S_before), t, p)
        err = np.abs(sg.cpu().numpy() - s_ref).max() if K else 0.0
        log(f"[{what}] step {t}: max |s - s_ref| {err:.2e}, E {E:.6e} vs {E_ref:.6e}, "
            f"{rep['quot_iters'][0]} quotient iterations")
        assert err <= ATOL + RTOL, (t, err)
        assert abs(E - E_ref) <= 1e-6 * abs(E_ref) + 1e-300, (t, E, E_ref)


def check_whole_path(ctx, s, p, out, ref, what):
    """End-to-end parity, decided before the GPU output is looked at: when
    the oracle's sensitivity to the fill tolerance stays below half the
    bound, depth and log-scales are compared with the oracle's; otherwise
    every stage is compared on identical inputs (labels bit-exact, the fill
    of every component, and the relative-scale stage and output run on the
    oracle's FP32 fill) and the end-to-end depth must be finite, positive
    (perspective) and in its gauge."""
    op = oracle_params(p)
    sens = fill_tolerance_sensitivity(s, op, ref)
    ortho = s.cam.proj == "ortho"
    assert out["K"] == ref.K
    assert np.array_equal(out["labels"].cpu().numpy(), ref.labels)
    v = s.mask > 0
    if sens <= 0.5:
        log(f"[{what}] fill-tolerance sensitivity {sens:.2f} of the bound: end-to-end comparison")
        assert_depth_close(out["depth"].cpu().numpy(), ref.depth, s.mask, what, ortho)
        assert_scale_close(out["log_scale"].cpu().numpy(), ref.log_scale, ortho)
        return "end-to-end"
    log(f"[{what}] fill-tolerance sensitivity {sens:.2f} of the bound: stage-wise comparison")
    z, frep = ctx.ni_fill(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(ref.labels), ref.K, p)
    e = O.edges(s.normals, s.mask, s.cam, op["theta_c_deg"], op.get("connectivity", 4))
    assert_fill_close(e, ref.labels, ref.K, z.cpu().numpy().astype(np.float64), ref.zfill, what)
    z32 = fp32(ref.zfill)
    chaos = irls_chaos(s, op, ref.labels, ref.K, z32)
    if chaos <= 0.5:
        log(f"[{what}] relative-scale loop: sensitivity to 1e-12 step noise {chaos:.2f} of the bound: whole loop")
        S, _, _ = O.irls(e, ref.labels, ref.K, z32, op)
        d_ref, ls_ref, _ = O.finalize(e, ref.labels, z32, S)
        d, ls, _ = ctx.ni_irls(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(ref.labels), ref.K,
                               dev(z32.astype(np.float32)), p)
        assert_depth_close(d.cpu().numpy(), d_ref, s.mask, what + " (stage)", ortho)
        assert_scale_close(ls.cpu().numpy(), ls_ref, ortho)
    else:
        log(f"[{what}] relative-scale loop: sensitivity to 1e-12 step noise {chaos:.0f} of the bound: step by step")
        check_irls_steps(ctx, s, p, op, ref.labels, ref.K, z32, what)
    dd = out["depth"].cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(dd[v])) and (ortho or np.all(dd[v] > 0))
    reg, R = O.regions(e)
    lz = dd[v] if ortho else np.log(dd[v])
    mean = np.bincount(reg[v], weights=lz, minlength=R) / np.maximum(np.bincount(reg[v], minlength=R), 1)
    assert np.max(np.abs(mean)) <= (1e-5 * max(1.0, np.max(np.abs(lz))) if ortho else 1e-5)
    return "stage-wise"


# ------------------------------------------------------------- whole path
@pytest.mark.parametrize("name,seed", SAMPLES + [("tiny-persp", 4), ("tiny-ortho", 5), ("tiny-ortho", 6),
                                                 ("tiny-persp", 7)])
def test_integrate_matches_oracle(ctx, name, seed):
    s = sample(name, seed)
    p = params(theta_c_deg=2.0, irls_iters=int(s.params["irls_iters"]))
    log(f"[integrate] {name} seed {seed}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    check_whole_path(ctx, s, p, out, ref, f"integrate {name} {seed}")
    rep = out["report"]
    assert rep["n_inter_edges"] == ref.n_inter_edges and rep["n_regions"] == ref.n_regions
    assert rep["ms_label"] > 0 and rep["ms_setup"] > 0


@pytest.mark.parametrize("seed,theta,kmin", [(0, 0.8, 4097), (0, 0.5, 20000), (0, 1.2, 3073), (1, 1.4, 1)])
def test_integrate_quotient_sizes(ctx, seed, theta, kmin):
    """Quotient graphs of a few thousand to ~22k components (the multigrid
    hierarchy grows by levels; heavy rows in their own blocks); the
    relative-scale weights span many decades at every step (Eq. 5)."""
    s = synth.make("c2", seed)
    p = params(theta_c_deg=theta, irls_iters=15)
    log(f"[integrate quotient sizes] c2 seed {seed} theta {theta}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    assert out["K"] >= kmin
    check_whole_path(ctx, s, p, out, ref, f"integrate c2 {seed} theta {theta}")
    assert out["report"]["n_inter_edges"] == ref.n_inter_edges


@pytest.mark.parametrize("name,seed,kw", [
    ("c1", 0, dict(delta_e_max=1e-3, irls_iters=40)),   # the paper's energy stop (Sec. 3.4, A13)
    ("c2", 0, dict(delta_e_max=1e-3, irls_iters=40)),
    ("c1", 1, dict(irls_iters=150)),        # T = 150 (Table 10's setting)
    ("c1", 2, dict(out_L=1e-4)),            # the L sweep (Table 9)
    ("c2", 2, dict(out_L=1e-4)),
    ("c2", 3, dict(outlier_mode=2)),        # hard threshold (supplementary ablation)
])
def test_integrate_variants(ctx, name, seed, kw):
    """Stop rule and outlier variants of the relative-scale loop: the same
    number of iterations as the oracle, then the same output."""
    s = synth.make(name, seed)
    base = dict(theta_c_deg=2.0, irls_iters=int(s.params["irls_iters"]))
    base.update(kw)
    p = params(**base)
    log(f"[variants] {name} seed {seed} {kw}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    assert out["report"]["irls_iters_run"] == len(ref.energies)
    if "delta_e_max" in kw:
        assert len(ref.energies) < p.irls_iters
    check_whole_path(ctx, s, p, out, ref, f"variants {name} {seed} {kw}")


@pytest.mark.parametrize("name,seed,theta", [("c2", 0, 2.0), ("c2", 1, 2.0), ("c2", 0, 0.0)])
def test_irls_steps_match_oracle(ctx, name, seed, theta):
    """The relative-scale iteration (Eq. 16-17) one step at a time from the
    oracle's scales, at the component level and the pixel level (theta_c =
    0: K = 117,965 one-pixel components)."""
    s = synth.make(name, seed)
    p = params(theta_c_deg=theta, irls_iters=15)
    op = oracle_params(p)
    e = O.edges(s.normals, s.mask, s.cam, theta)
    lab, K = O.labels(e)
    zf = fp32(O.fill(e, lab, K))
    log(f"[irls steps] {name} seed {seed} theta {theta} K {K}")
    check_irls_steps(ctx, s, p, op, lab, K, zf, f"{name} {seed} theta {theta}")


@pytest.mark.parametrize("name,seed,freq,T", [("c1", 0, 3, 10), ("c1", 1, 5, 10), ("c2", 0, 5, 15),
                                             ("c2", 2, 3, 15), ("tiny-persp", 3, 2, 6), ("c2", 0, 1, 6)])
def test_integrate_merging(ctx, name, seed, freq, T):
    """Optional merging (Sec. 3.5, Alg. 1's merge block every freq
    iterations): the same node count after the merges as the oracle, then
    the same output."""
    s = sample(name, seed)
    p = params(theta_c_deg=2.0, irls_iters=T, freq_merging=freq)
    log(f"[merging] {name} seed {seed} freq {freq} T {T}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    groups = O.irls.last_groups
    rep = out["report"]
    assert rep["merges"] == (T - 1) // freq
    assert rep["nodes_final"] == (int(groups.max()) + 1 if groups.size else 0)
    check_whole_path(ctx, s, p, out, ref, f"merging {name} {seed} freq {freq}")


@pytest.mark.parametrize("name,seed", [("tiny-persp", 1), ("c1", 0), ("c2", 0)])
def test_logdepth_baseline_matches_oracle(ctx, name, seed):
    """The pixel-level log-depth baseline, ND form (variant = 1, reading
    A28): every pixel its own node, BiNI weights from z = 0, outlier weights
    from the second iteration."""
    s = sample(name, seed)
    p = params(irls_iters=int(s.params["irls_iters"]), variant=1)
    log(f"[baseline ND] {name} seed {seed}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    assert out["K"] == int((s.mask > 0).sum())
    check_whole_path(ctx, s, p, out, ref, f"baseline {name} {seed}")


def test_quotient_not_converged_is_reported(ctx):
    """A relative-scale solve stopped at q_max_iter = 1 is reported as
    NI_E_NOTCONV (outputs still written)."""
    import paper_2510_11508_amd as ni
    s = synth.make("c2", 0)
    log("[edge] q_max_iter=1")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), params(q_max_iter=1),
                           raise_notconv=False)
    assert out["status"] == ni.NI_E_NOTCONV
    assert out["report"]["fill_notconv"] == 0
    assert np.all(np.isfinite(out["depth"].cpu().numpy()[s.mask > 0]))


@pytest.mark.parametrize("seed,theta", [(0, 2.0), (1, 0.8)])
def test_integrate_ortho_384(ctx, seed, theta):
    """A 384^2 orthographic map (additive depth, reading A1); at 0.8 deg
    its ~25k components take the multigrid quotient path."""
    s = synth.make_ortho(seed)
    p = params(theta_c_deg=theta, irls_iters=10)
    log(f"[integrate ortho 384] seed {seed} theta {theta}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    check_whole_path(ctx, s, p, out, ref, f"ortho 384 {seed} theta {theta}")


def test_graph_replay_equals_stream_launches(ctx):
    """The multigrid quotient CG replayed from a HIP graph gives the output
    of the same kernels launched one by one, call after call (the graph is
    captured per solve round and replayed many times per call)."""
    s = synth.make("c2", 1)
    outs = []
    for g in (0, 1, 0, 1):
        p = params(theta_c_deg=0.8, graphs=g)
        log(f"[graph replay] graphs={g}")
        o = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
        assert o["K"] > 4096
        outs.append((o["depth"].cpu().numpy(), o["log_scale"].cpu().numpy(), list(o["report"]["quot_iters"])))
    # the piece and region means use FP64 atomics (summation order varies
    # between runs), so the comparison is at rounding level, not bitwise
    v = s.mask > 0
    for d, ls, qi in outs[1:]:
        assert np.max(np.abs(d[v] - outs[0][0][v]) / np.abs(outs[0][0][v])) <= 1e-6
        assert np.max(np.abs(ls - outs[0][1])) <= 1e-10
        assert all(abs(a - b) <= 2 for a, b in zip(qi, outs[0][2]))


@pytest.mark.parametrize("theta", [2.0, 0.8])
def test_deterministic(ctx, theta):
    s = synth.make("c2", 2)
    p = params(theta_c_deg=theta)
    outs = []
    for k in range(3):
        log(f"[determinism] run {k}")
        o = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
        outs.append((o["labels"].cpu().numpy(), o["depth"].cpu().numpy()))
    for lab, d in outs[1:]:
        assert np.array_equal(lab, outs[0][0])
        v = s.mask > 0
        assert np.max(np.abs(d[v] - outs[0][1][v])) <= 1e-6 * np.max(np.abs(outs[0][1][v]))


@pytest.mark.parametrize("name,conn", [("c3", 4), ("c3", 8), ("c5", 4)])
def test_bitwise_reproducible(ctx, name, conn):
    """Every sum that feeds the relative-scale loop and the outputs is taken in
    an order fixed by positions alone (run sums, block partials, no floating
    atomics), so repeated runs give identical bits.  This matters beyond
    tidiness at 2048^2 and up: there the loop amplifies rounding differences
    to visible changes of the output (see irls_chaos)."""
    s = synth.make(name, 0)
    p = params(theta_c_deg=2.0, irls_iters=15, connectivity=conn)
    outs = []
    for k in range(2):
        log(f"[bitwise] {name} connectivity {conn} run {k}")
        o = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
        outs.append((o["labels"].cpu().numpy(), o["depth"].cpu().numpy(), o["log_scale"].cpu().numpy(),
                     o["report"]["energy"]))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1], equal_nan=True)
    assert np.array_equal(outs[0][2], outs[1][2])
    assert outs[0][3] == outs[1][3]


# ------------------------------------------------------------- edge cases
def test_empty_mask(ctx):
    s = synth.tiny(0)
    m = np.zeros_like(s.mask)
    log("[edge] empty mask")
    out = ctx.ni_integrate(dev(s.normals), dev(m), s.cam.as_dict(), params())
    assert out["K"] == 0
    assert np.all(out["labels"].cpu().numpy() == -1)
    assert np.all(np.isnan(out["depth"].cpu().numpy()))


def test_single_pixel_and_thin_maps(ctx):
    for H, W in [(1, 1), (1, 17), (23, 1), (2, 2)]:
        s = synth.tiny(1, max(H, 3), max(W, 3), "persp")
        n = np.ascontiguousarray(s.normals[:H, :W])
        m = np.ones((H, W), np.uint8)
        cam = dict(s.cam.as_dict())
        log(f"[edge] {H}x{W}")
        out = ctx.ni_integrate(dev(n), dev(m), cam, params(irls_iters=4))
        ref = O.integrate(n, m, cam, dict(irls_iters=4))
        assert out["K"] == ref.K and np.array_equal(out["labels"].cpu().numpy(), ref.labels)
        assert_depth_close(out["depth"].cpu().numpy(), ref.depth, m, f"{H}x{W}", cam["proj"] == "ortho")


def test_nonfinite_inside_mask_is_an_error(ctx):
    import paper_2510_11508_amd as ni
    s = synth.tiny(2)
    n = s.normals.copy()
    v = np.argwhere(s.mask > 0)[3]
    n[v[0], v[1], 2] = np.inf
    log("[edge] inf inside mask")
    with pytest.raises(ni.NIError) as ex:
        ctx.ni_integrate(dev(n), dev(s.mask), s.cam.as_dict(), params())
    assert ex.value.status == ni.NI_E_NONFINITE
    # NaN off the mask is fine
    m = s.mask.copy()
    m[v[0], v[1]] = 0
    n[v[0], v[1], 2] = np.nan
    log("[edge] nan off mask")
    out = ctx.ni_integrate(dev(n), dev(m), s.cam.as_dict(), params(irls_iters=3))
    ref = O.integrate(n, m, s.cam, dict(irls_iters=3))
    assert out["K"] == ref.K


def test_capacity_too_small(ctx):
    import paper_2510_11508_amd as ni
    s = synth.tiny(0)
    log("[edge] cap < K")
    with pytest.raises(ni.NIError) as ex:
        ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), params(), cap=2)
    assert ex.value.status == ni.NI_E_SHAPE


def test_bad_arguments(ctx):
    import paper_2510_11508_amd as ni
    s = synth.tiny(0)
    for kw in [dict(connectivity=6), dict(irls_iters=0), dict(outlier_mode=5), dict(out_L=1e-2),
               dict(warm_start=1), dict(fill_chunk=300), dict(fill_chunk=1024, fill_split=2),
               dict(fill_precond=2), dict(fill_mg_maxit=-1)]:
        log(f"[edge] bad params {kw}")
        with pytest.raises(ni.NIError) as ex:
            ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), params(**kw))
        assert ex.value.status in (ni.NI_E_ARG, ni.NI_E_MODEL)


def test_pixel_level_limit(ctx):
    """theta_c = None: every pixel its own component; the quotient graph is G_0."""
    s = synth.tiny(3, 10, 12, "persp")
    p = params(theta_c_deg=0.0, irls_iters=6)
    log("[edge] pixel level")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    assert out["K"] == int(s.mask.sum())
    assert_depth_close(out["depth"].cpu().numpy(), ref.depth, s.mask, "pixel level")


def test_pixel_level_c2(ctx):
    """The pixel-level form on a 512^2 map: 117,965 one-pixel components, so
    the relative-scale system is the full pixel graph (multigrid path)."""
    s = synth.make("c2", 0)
    p = params(theta_c_deg=0.0, irls_iters=15)
    log("[pixel level] c2 seed 0")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    assert out["K"] == int((s.mask > 0).sum())
    assert_depth_close(out["depth"].cpu().numpy(), ref.depth, s.mask, "pixel level c2")


def test_not_converged_is_reported(ctx):
    import paper_2510_11508_amd as ni
    s = synth.make("c1", 0)
    log("[edge] cg_max_iter=1")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), params(cg_max_iter=1),
                           raise_notconv=False)
    assert out["status"] == ni.NI_E_NOTCONV and out["report"]["fill_notconv"] > 0


# ---------------------------------------------------- full-size properties
def test_full_size_c3(ctx):
    """2048^2 (73,711 components, 77 of them in the multigrid fill, up to
    ~1e6 px) against the oracle's full integration: labels bit-exact; then
    end-to-end or stage by stage as the oracle-only sensitivity probe
    decides (the fill of every component, and the relative-scale stage and
    output on the oracle's FP32 fill)."""
    s = synth.make("c3", 0)
    p = params(theta_c_deg=2.0, irls_iters=15)
    log("[c3] integrate")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    log("[c3] oracle")
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    how = check_whole_path(ctx, s, p, out, ref, "c3 seed 0")
    log(f"[c3] compared {how}")
    rep = out["report"]
    assert rep["n_inter_edges"] == ref.n_inter_edges and rep["n_regions"] == ref.n_regions


def bbox_fill(s, lab, c):
    """The oracle's exact fill of component c, solved on its bounding box
    (the principal point shifted with it, so the rays and every edge are
    unchanged)."""
    m = lab == c
    rows, cols = np.flatnonzero(m.any(1)), np.flatnonzero(m.any(0))
    y0, y1, x0, x1 = rows[0], rows[-1] + 1, cols[0], cols[-1] + 1
    cam = dict(s.cam.as_dict())
    cam["cx"] -= x0
    cam["cy"] -= y0
    mc = m[y0:y1, x0:x1]
    ec = O.edges(s.normals[y0:y1, x0:x1], (s.mask[y0:y1, x0:x1] > 0) & mc, cam, 2.0)
    sub = np.where(mc, 0, -1).astype(np.int32)
    return (y0, y1, x0, x1), mc, O.fill(ec, sub, 1)


def test_full_size_c5_sampled(ctx):
    """4096^2 in the benchmark's configuration: labels bit-exact; the fill
    of the three largest components (1.33M, 1.02M and 97k px, multigrid
    path) and of sampled small ones equals the oracle's exact
    per-component solve (components are independent, Sec. 3.3); the
    output gauge holds (zero mean log-depth over every connected region of
    the pixel graph)."""
    s = synth.make("c5", 0)
    p = params(theta_c_deg=2.0, irls_iters=15)
    log("[c5] integrate")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    assert out["K"] == K and np.array_equal(out["labels"].cpu().numpy(), lab)
    log("[c5] fill")
    z, rep = ctx.ni_fill(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K, p)
    z = z.cpu().numpy()
    sizes = np.bincount(lab[lab >= 0])
    rng = np.random.default_rng(0)
    cand = np.flatnonzero((sizes >= 2) & (sizes <= 30000))
    pick = list(np.argsort(sizes)[::-1][:3]) + list(rng.choice(cand, size=4, replace=False))
    for c in pick:
        log(f"[c5] component {c}: {sizes[c]} px")
        (y0, y1, x0, x1), mc, zr = bbox_fill(s, lab, c)
        sub = np.where(mc, 0, -1).astype(np.int32)
        cam = dict(s.cam.as_dict())
        cam["cx"] -= x0
        cam["cy"] -= y0
        ec = O.edges(s.normals[y0:y1, x0:x1], (s.mask[y0:y1, x0:x1] > 0) & mc, cam, 2.0)
        zc = np.where(mc, z[y0:y1, x0:x1], 0.0).astype(np.float64)
        assert_fill_close(ec, sub, 1, zc, zr, f"c5 component {c}")
    d = out["depth"].cpu().numpy()
    v = s.mask > 0
    assert np.all(np.isfinite(d[v])) and np.all(d[v] > 0)
    reg, R = O.regions(e)
    lz = np.log(d[v].astype(np.float64))
    mean = np.bincount(reg[v], weights=lz, minlength=R) / np.maximum(np.bincount(reg[v], minlength=R), 1)
    assert np.max(np.abs(mean)) <= 1e-5
