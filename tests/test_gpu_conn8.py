"""8-connectivity (the diagonal neighbours join the pixel graph; the reading
of Sec. 3.1 spelled out in the oracle's diagonal edge model) on the HIP
path against the FP64 oracle, through the C ABI.

Bars as for 4-connectivity: labels bit-exact; the fill per component
within 1e-6 + 1e-4 (log-depth) or the CG stop rule's own bound; depth
1e-6 + 1e-4 relative and log-scales 1e-4, end to end where the oracle's
sensitivity to the fill tolerance allows it, else stage by stage on
identical inputs.
"""
import numpy as np
import pytest

import synth
from oracle import ni_oracle as O
from test_gpu_parity import (assert_depth_close, assert_fill_close, assert_scale_close, check_irls_steps,
                             check_whole_path, dev, fp32, irls_chaos, log, oracle_params, params, sample)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_2510_11508_amd as ni
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ni.Context(0)
    yield c
    c.close()


def edges8(s, theta):
    return O.edges(s.normals, s.mask, s.cam, theta, connectivity=8)


@pytest.mark.parametrize("name,seed,theta", [("c1", 0, 2.0), ("c1", 1, 2.0), ("c2", 0, 2.0), ("c2", 3, 0.5),
                                             ("c2", 1, 180.0), ("c2", 2, 0.0), ("tiny-persp", 0, 2.0),
                                             ("tiny-ortho", 1, 2.0), ("c3", 0, 2.0)])
def test_labels8_bit_exact(ctx, name, seed, theta):
    s = sample(name, seed)
    log(f"[labels8] {name} seed {seed} theta {theta}")
    lab, K, _ = ctx.ni_label(dev(s.normals), dev(s.mask), s.cam.as_dict(), params(theta_c_deg=theta, connectivity=8))
    ref, Kr = O.labels(edges8(s, theta))
    assert K == Kr and np.array_equal(lab.cpu().numpy(), ref)
    if theta == 2.0:
        # the diagonals only ever join components
        _, K4 = O.labels(O.edges(s.normals, s.mask, s.cam, theta))
        assert K <= K4


@pytest.mark.parametrize("name,seed,warm", [("c1", 0, 0), ("c2", 0, 0), ("c2", 4, 0), ("tiny-persp", 2, 0),
                                            ("tiny-ortho", 3, 0), ("c2", 1, 1)])
def test_fill8_matches_oracle(ctx, name, seed, warm):
    s = sample(name, seed)
    e = edges8(s, 2.0)
    lab, K = O.labels(e)
    zref = O.fill(e, lab, K)
    log(f"[fill8] {name} seed {seed} K {K} warm {warm}")
    if warm:
        ctx.ni_unet_init(11)
    z, rep = ctx.ni_fill(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K,
                         params(connectivity=8, warm_start=warm))
    assert rep["fill_notconv"] == 0 and rep["n_small"] == 0
    assert rep["n_large"] == int(np.sum(np.bincount(lab[lab >= 0], minlength=K) >= 2))
    z = z.cpu().numpy().astype(np.float64)
    assert np.all(z[s.mask == 0] == 0)
    assert_fill_close(e, lab, K, z, zref, f"fill8 {name} {seed}")


@pytest.mark.parametrize("name,seed,mode", [("c1", 0, 1), ("c1", 1, 2), ("c1", 2, 0), ("c2", 0, 1),
                                            ("tiny-persp", 1, 1), ("tiny-ortho", 0, 1)])
def test_irls8_given_fill(ctx, name, seed, mode):
    """The relative-scale stage and output on the oracle's FP32 fill; the
    whole loop when the oracle itself is stable to 1e-12 step noise, else
    one step at a time."""
    s = sample(name, seed)
    p = params(theta_c_deg=2.0, irls_iters=int(s.params["irls_iters"]), outlier_mode=mode, connectivity=8)
    op = oracle_params(p)
    e = edges8(s, 2.0)
    lab, K = O.labels(e)
    zf = fp32(O.fill(e, lab, K))
    chaos = irls_chaos(s, op, lab, K, zf)
    log(f"[irls8] {name} seed {seed} mode {mode} K {K}: step-noise sensitivity {chaos:.2f}")
    if chaos > 0.5:
        check_irls_steps(ctx, s, p, op, lab, K, zf, f"irls8 {name} {seed}")
        return
    S, En, ie = O.irls(e, lab, K, zf, op)
    d_ref, ls_ref, _ = O.finalize(e, lab, zf, S)
    d, ls, rep = ctx.ni_irls(dev(s.normals), dev(s.mask), s.cam.as_dict(), dev(lab), K, dev(zf.astype(np.float32)),
                             p)
    ortho = s.cam.proj == "ortho"
    assert_depth_close(d.cpu().numpy(), d_ref, s.mask, f"irls8 {name}", ortho)
    assert_scale_close(ls.cpu().numpy(), ls_ref, ortho)
    assert np.allclose(rep["energy"], En, rtol=1e-3, atol=1e-12)
    assert rep["n_inter_edges"] == ie.a.size


@pytest.mark.parametrize("name,seed", [("c1", 0), ("c1", 1), ("c2", 0), ("c2", 1), ("tiny-persp", 4),
                                       ("tiny-ortho", 5), ("tiny-persp", 7)])
def test_integrate8_matches_oracle(ctx, name, seed):
    s = sample(name, seed)
    p = params(theta_c_deg=2.0, irls_iters=int(s.params["irls_iters"]), connectivity=8)
    log(f"[integrate8] {name} seed {seed}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    check_whole_path(ctx, s, p, out, ref, f"integrate8 {name} {seed}")
    rep = out["report"]
    assert rep["n_inter_edges"] == ref.n_inter_edges and rep["n_regions"] == ref.n_regions


@pytest.mark.parametrize("name,seed,freq,T", [("c1", 0, 3, 10), ("tiny-persp", 3, 2, 6), ("c2", 0, 5, 15)])
def test_merging8(ctx, name, seed, freq, T):
    s = sample(name, seed)
    p = params(theta_c_deg=2.0, irls_iters=T, freq_merging=freq, connectivity=8)
    log(f"[merging8] {name} seed {seed} freq {freq} T {T}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    groups = O.irls.last_groups
    rep = out["report"]
    assert rep["merges"] == (T - 1) // freq
    assert rep["nodes_final"] == (int(groups.max()) + 1 if groups.size else 0)
    check_whole_path(ctx, s, p, out, ref, f"merging8 {name} {seed}")


@pytest.mark.parametrize("name,seed", [("tiny-persp", 1), ("c1", 0)])
def test_logdepth_baseline8(ctx, name, seed):
    """The pixel-level log-depth baseline (variant = 1) on the 8-connected
    pixel graph."""
    s = sample(name, seed)
    p = params(irls_iters=int(s.params["irls_iters"]), variant=1, connectivity=8)
    log(f"[baseline8] {name} seed {seed}")
    out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
    assert out["K"] == int(np.sum(s.mask > 0))
    check_whole_path(ctx, s, p, out, ref, f"baseline8 {name} {seed}")


def test_irls8_steps_c2(ctx):
    """One step at a time on a 512^2 map (the component level)."""
    s = synth.make("c2", 0)
    p = params(theta_c_deg=2.0, irls_iters=15, connectivity=8)
    op = oracle_params(p)
    e = edges8(s, 2.0)
    lab, K = O.labels(e)
    zf = fp32(O.fill(e, lab, K))
    log(f"[irls8 steps] c2 seed 0 K {K}")
    check_irls_steps(ctx, s, p, op, lab, K, zf, "irls8 steps c2 0")


def test_edge_cases8(ctx):
    """Single pixel, one-pixel-wide strips (diagonal edges run off the map)
    and a checkerboard mask (connected only through the diagonals)."""
    import paper_2510_11508_amd as ni
    for H, W in [(1, 1), (1, 7), (7, 1), (2, 2)]:
        s = synth.tiny(3, H, W, "persp")
        p = params(connectivity=8, irls_iters=6)
        out = ctx.ni_integrate(dev(s.normals), dev(s.mask), s.cam.as_dict(), p)
        ref = O.integrate(s.normals, s.mask, s.cam, oracle_params(p))
        log(f"[edge8] {H}x{W}: K {out['K']}")
        assert out["K"] == ref.K
        assert_depth_close(out["depth"].cpu().numpy(), ref.depth, s.mask, f"edge8 {H}x{W}")
    s = synth.tiny(4, 12, 12, "persp")
    m = ((np.add.outer(np.arange(12), np.arange(12)) % 2) == 0).astype(np.uint8)
    p = params(theta_c_deg=180.0, connectivity=8, irls_iters=6)
    out = ctx.ni_integrate(dev(s.normals), dev(m), s.cam.as_dict(), p)
    ref = O.integrate(s.normals, m, s.cam, oracle_params(p))
    log(f"[edge8] checkerboard: K {out['K']} regions {out['report']['n_regions']}")
    assert out["K"] == ref.K and np.array_equal(out["labels"].cpu().numpy(), ref.labels)
    assert out["report"]["n_regions"] == ref.n_regions
    assert_depth_close(out["depth"].cpu().numpy(), ref.depth, m, "edge8 checkerboard")
    with pytest.raises(ni.NIError):
        ctx.ni_label(dev(s.normals), dev(s.mask), s.cam.as_dict(), params(connectivity=6))
