"""Pins of the FP64 oracle against values the paper prints, closed forms,
brute force on tiny maps and invariants (no GPU)."""
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import bruteforce as BF
from oracle import ni_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- Eq. 18 ----
def test_outlier_weight_printed_values():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "outlier_weight.txt"))
            if l.strip() and not l.startswith("#")]
    for chi, w, prec in rows:
        got = float(O.outlier_weight(float(chi), 1e-5, 1e-3, 1))
        assert abs(got - float(w)) <= float(prec), (chi, got, w)


def test_outlier_weight_matches_plotted_curve():
    # Suppl. Fig. 10 plots 1/(1+exp(2(2x+8))) for L=1e-5, U=1e-3
    x = np.linspace(-5.6, -1.6, 41)
    got = O.outlier_weight(10.0 ** x, 1e-5, 1e-3, 1)
    ref = 1.0 / (1.0 + np.exp(2.0 * (2.0 * x + 8.0)))
    assert np.max(np.abs(got - ref)) < 1e-12


def test_outlier_weight_limits_and_modes():
    assert O.outlier_weight(0.0) == 1.0                      # sigma(+inf)
    assert O.outlier_weight(1.0) < 1e-6                      # far outlier
    hard = O.outlier_weight(np.array([0.0, 9.99e-4, 1e-3, 0.5]), mode=2)
    assert list(hard) == [1.0, 1.0, 0.0, 0.0]
    assert np.all(O.outlier_weight(np.array([0.0, 1.0]), mode=0) == 1.0)
    # monotone decreasing in |chi|
    c = np.logspace(-8, 0, 200)
    assert np.all(np.diff(O.outlier_weight(c)) <= 0)


# ------------------------------------------------------ Eq. 3 closed forms ---
def test_plane_perspective_exact():
    """Tangent planes of a plane are the plane: Eq. 3 is exact for every edge."""
    n, m, z, cam = synth.plane_persp(24, 31, 40.0, [0.3, -0.2, -1.0], 2.5)
    e = O.edges(n, m, cam, 2.0)
    # the plane whose normal is the stored FP32 vector
    n64 = n[0, 0].astype(np.float64)
    tx, ty, _, _ = O.ray_tables(cam, *m.shape)
    lz = np.log(-1.0 / (n64[0] * tx[None, :] + n64[1] * ty[:, None] + n64[2]))
    assert e.valid_r[:, :-1].all() and e.valid_d[:-1, :].all()
    assert np.max(np.abs(e.omega_r[:, :-1] - (lz[:, :-1] - lz[:, 1:]))) < 1e-13
    assert np.max(np.abs(e.omega_d[:-1, :] - (lz[:-1, :] - lz[1:, :]))) < 1e-13
    r = O.integrate(n, m, cam, dict(irls_iters=3))
    assert r.K == 1
    ratio = np.log(r.depth) - lz
    assert np.ptp(ratio) < 1e-12


def test_quadric_orthographic_exact():
    """Orthographic reading (A1) is exact for quadratic height fields."""
    rng = np.random.default_rng(5)
    coef = rng.uniform(-0.02, 0.02, 6)
    n, m, z, cam = synth.quadric_ortho(17, 23, coef, pitch=0.7)
    e = O.edges(n.astype(np.float32), m, cam, 180.0)
    # FP32 input normals limit this to ~1e-7 relative
    err = np.max(np.abs(e.omega_r[:, :-1] - (z[:, :-1] - z[:, 1:])))
    assert err < 2e-7
    n64 = n  # FP64 normals through the same formula are exact to rounding
    nx, ny, nz = n64[..., 0], n64[..., 1], n64[..., 2]
    om = 0.7 * (nx[:, :-1] / (2 * nz[:, :-1]) + nx[:, 1:] / (2 * nz[:, 1:]))
    assert np.max(np.abs(om - (z[:, :-1] - z[:, 1:]))) < 1e-13
    r = O.integrate(n.astype(np.float32), m, cam, dict(theta_c_deg=180.0, irls_iters=2))
    assert r.K == 1
    d = r.depth - z
    assert np.ptp(d) < 1e-5


def test_sphere_second_order():
    """On a sphere the per-edge error of Eq. 3 falls ~8x per resolution
    doubling (third-order local error of the two-tangent-plane model).
    FP64 normals, edges away from the silhouette (incidence < 60 deg)."""
    errs = []
    for Wd in (32, 64, 128):
        n, m, z, cam = synth.sphere_persp(Wd, Wd, 1.2 * Wd, 1.0, 4.0)
        e = O.edges(n, m, cam, 0.0)
        lz = np.log(z)
        tx, ty, _, _ = O.ray_tables(cam, Wd, Wd)
        tau = np.stack(np.broadcast_arrays(tx[None, :], ty[:, None], 1.0), -1)
        cosi = -np.sum(n * tau, -1) / np.linalg.norm(tau, axis=-1)
        ok = (m > 0) & (cosi > 0.5)
        sel = e.valid_r[:, :-1] & ok[:, :-1] & ok[:, 1:]
        errs.append(np.max(np.abs(e.omega_r[:, :-1][sel] - (lz[:, :-1] - lz[:, 1:])[sel])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.0 < r1 < 10.0 and 6.0 < r2 < 10.0, errs


def test_omega_mirror_antisymmetry():
    """Mirroring the image swaps a and b of every horizontal edge: omega_{a->b} = -omega_{b->a}."""
    s = synth.tiny(3, 9, 12, "persp", noise=0.02)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    H, W = s.mask.shape
    nm = s.normals[:, ::-1].copy()
    nm[..., 0] *= -1
    cam = synth.Camera("persp", fx=s.cam.fx, fy=s.cam.fy, cx=(W - 1) - s.cam.cx, cy=s.cam.cy)
    em = O.edges(nm, s.mask[:, ::-1].copy(), cam, 2.0)
    assert np.array_equal(em.valid_r[:, :-1], e.valid_r[:, :-1][:, ::-1])
    sel = e.valid_r[:, :-1]
    assert np.max(np.abs(em.omega_r[:, :-1][:, ::-1][sel] + e.omega_r[:, :-1][sel])) < 1e-14
    assert np.array_equal(em.sim_r[:, :-1][:, ::-1], e.sim_r[:, :-1])


def test_global_sign_flip_invariance():
    s = synth.tiny(1, proj="persp")
    a = O.integrate(s.normals, s.mask, s.cam, s.params)
    b = O.integrate(-s.normals, s.mask, s.cam, s.params)
    assert np.array_equal(a.labels, b.labels)
    v = s.mask > 0
    assert np.max(np.abs(a.logz[v] - b.logz[v])) < 1e-12


def test_edges_match_bruteforce_pairs():
    for proj in ("persp", "ortho"):
        s = synth.tiny(2, proj=proj, noise=0.03)
        e = O.edges(s.normals, s.mask, s.cam, 2.0)
        valid, usable, similar, info = BF.model(s.normals, s.mask, s.cam.as_dict(), 2.0)
        H, W = s.mask.shape
        ur = np.zeros((H, W), bool); ud = np.zeros((H, W), bool)
        for (a, b) in usable:
            (ur if a[1] == b[1] else ud)[a[1], a[0]] = True
        assert np.array_equal(ur, e.valid_r) and np.array_equal(ud, e.valid_d)
        for (a, b), (om, g2a, g2b) in info.items():
            if a[1] == b[1]:
                assert abs(e.omega_r[a[1], a[0]] - om) < 1e-13
                assert abs(e.g2_h[a[1], a[0]] - g2a) <= 1e-12 * g2a
                assert abs(e.g2_h[b[1], b[0]] - g2b) <= 1e-12 * g2b
            else:
                assert abs(e.omega_d[a[1], a[0]] - om) < 1e-13
                assert abs(e.g2_v[a[1], a[0]] - g2a) <= 1e-12 * g2a


# ---------------------------------------------------------------- labels ----
@pytest.mark.parametrize("seed", range(6))
def test_labels_match_transitive_closure(seed):
    proj = "persp" if seed % 2 else "ortho"
    s = synth.tiny(seed, proj=proj)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    valid, usable, similar, info = BF.model(s.normals, s.mask, s.cam.as_dict(), 2.0)
    ref, Kr = BF.closure_labels(*s.mask.shape, valid, similar)
    assert K == Kr and np.array_equal(lab, ref)


def test_labels_theta_180_is_mask_connectivity():
    s = synth.tiny(4, 12, 12, "persp", noise=0.0, step=0.0)
    e = O.edges(s.normals, s.mask, s.cam, 180.0)
    assert e.valid_r[:, :-1][(s.mask[:, :-1] > 0) & (s.mask[:, 1:] > 0)].all()
    lab, K = O.labels(e)
    ref, nref = ndimage.label(s.mask, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    assert K == nref and np.array_equal(lab, ref - 1)


def test_labels_pixel_level_limit():
    """theta_c = None: every pixel is its own component and Q = G_0."""
    s = synth.tiny(0)
    e = O.edges(s.normals, s.mask, s.cam, 0.0)
    lab, K = O.labels(e)
    v = s.mask > 0
    assert K == v.sum()
    assert np.array_equal(lab[v], np.arange(K))
    assert np.all(O.fill(e, lab, K)[v] == 0.0)
    ie = O.inter_edges(e, lab)
    assert ie.a.size == e.valid_r.sum() + e.valid_d.sum()


# ------------------------------------------------------------------ fill ----
@pytest.mark.parametrize("seed", range(4))
def test_fill_matches_dense_rows(seed):
    proj = "persp" if seed % 2 == 0 else "ortho"
    s = synth.tiny(seed, proj=proj, noise=0.02)
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    z = O.fill(e, lab, K)
    valid, usable, similar, info = BF.model(s.normals, s.mask, s.cam.as_dict(), 2.0)
    zr = BF.fill_rows(s.normals, s.mask, s.cam.as_dict(), lab, info)
    v = s.mask > 0
    assert np.max(np.abs(z[v] - zr[v])) < 1e-10
    for c in range(K):
        assert abs(z[lab == c].mean()) < 1e-12


# ------------------------------------------------------------------ IRLS ----
@pytest.mark.parametrize("seed,mode", [(0, 1), (1, 1), (2, 2), (3, 0), (5, 1)])
def test_irls_matches_dense_rows(seed, mode):
    proj = "persp" if seed % 2 == 0 else "ortho"
    s = synth.tiny(seed, proj=proj, noise=0.01)
    p = dict(O.DEFAULT_PARAMS)
    p.update(irls_iters=6, outlier_mode=mode, bini_k=2.0)
    if proj == "ortho":
        p["bini_k"] = 50.0     # make the BiNI factor bite at pixel-unit depths
    e = O.edges(s.normals, s.mask, s.cam, 2.0)
    lab, K = O.labels(e)
    zf = O.fill(e, lab, K)
    S, En, _ = O.irls(e, lab, K, zf, p)
    valid, usable, similar, info = BF.model(s.normals, s.mask, s.cam.as_dict(), 2.0)
    Sr, Er = BF.irls_rows(s.normals, s.mask, s.cam.as_dict(), lab, K, zf, usable, info, p)
    assert np.max(np.abs(S - Sr)) < 1e-8
    assert np.allclose(En, Er, rtol=1e-8, atol=1e-14)


def _exact_logz(s, ref, p):
    """Log-depth from the brute-force uncut solve of Eq. 16-17 (every row
    with a non-zero weight kept), on the oracle's labels and fill, shifted to
    zero mean on each connected region of the mask (scipy.ndimage.label;
    every edge of these maps is usable, which the test asserts)."""
    S, _ = BF.irls_exact(s.normals, s.mask, s.cam.as_dict(), ref.labels, ref.K, ref.zfill, p)
    v = ref.labels >= 0
    z = np.where(v, ref.zfill + S[np.maximum(ref.labels, 0)], 0.0)
    reg, R = ndimage.label(v)
    for r in range(1, R + 1):
        z[reg == r] -= z[reg == r].mean()
    return z, v


def _depth_err(s, z, v, ref_logz):
    """max violation of |d - d_ref| <= 1e-6 + 1e-4 |d_ref| (perspective depth)
    or the norm-wise 1e-4 max|h_ref| bound (orthographic heights cross zero)."""
    if s.cam.proj == "persp":
        d, dr = np.exp(z[v]), np.exp(ref_logz[v])
        return float(np.max(np.abs(d - dr) / (1e-6 + 1e-4 * np.abs(dr))))
    return float(np.max(np.abs(z[v] - ref_logz[v])) / (1e-4 * np.max(np.abs(ref_logz[v]))))


@pytest.mark.parametrize("name,seed", [("c1", 0), ("c1", 1), ("c1", 2), ("c2", 0)])
def test_irls_equals_uncut_exact_solve(name, seed):
    """Eq. 17 solved with no relative weight cut (only rows whose weight is
    exactly zero are dropped) by the brute-force directed-row formulation
    gives the oracle's output (cut at 1e-12 of the largest weight, A16)
    within the depth parity bound."""
    s = synth.make(name, seed)
    p = dict(O.DEFAULT_PARAMS, irls_iters=synth.CONFIGS[name]["T"])
    ref = O.integrate(s.normals, s.mask, s.cam, p)
    e = O.edges(s.normals, s.mask, s.cam, p["theta_c_deg"])
    v = s.mask > 0
    assert np.array_equal(e.valid_r[:, :-1], v[:, :-1] & v[:, 1:])
    assert np.array_equal(e.valid_d[:-1, :], v[:-1, :] & v[1:, :])
    z, v = _exact_logz(s, ref, p)
    assert _depth_err(s, z, v, ref.logz) <= 1.0


@pytest.mark.parametrize("name,seed", [("c1", 0), ("c2", 0)])
def test_coarse_cut_reading_fails_exact_pin(name, seed):
    """The pin above is sharp: a cut at 1e-4 of the largest weight (which
    drops links that Eq. 17 keeps) misses the uncut solution by far more
    than the parity bound."""
    s = synth.make(name, seed)
    p = dict(O.DEFAULT_PARAMS, irls_iters=synth.CONFIGS[name]["T"])
    ref = O.integrate(s.normals, s.mask, s.cam, p)
    z, v = _exact_logz(s, ref, p)
    coarse = O.integrate(s.normals, s.mask, s.cam, dict(p, w_cut_rel=1e-4))
    assert _depth_err(s, z, v, coarse.logz) > 20.0


# -------------------------------------------------------------- finalize ----
@pytest.mark.parametrize("name,seed", [("c1", 1), ("c2", 0), ("tiny", 3)])
def test_finalize_gauge_and_scales(name, seed):
    """The output gauge (A15) characterised without the oracle's own code:
    log-depth = fill + S_pi + one constant per connected region of G_0, with
    zero pixel mean on every region; log_scale_c = log-depth - fill on the
    pixels of c; depth = exp(log-depth) (perspective) or the height itself
    (orthographic); NaN off the mask.  Regions come from scipy.ndimage.label
    where every edge of the mask is usable."""
    s = synth.tiny(seed, proj="persp", H=12, W=13) if name == "tiny" else synth.make(name, seed)
    p = dict(O.DEFAULT_PARAMS, irls_iters=synth.CONFIGS[name]["T"] if name in synth.CONFIGS else 6)
    e = O.edges(s.normals, s.mask, s.cam, p["theta_c_deg"])
    lab, K = O.labels(e)
    zf = O.fill(e, lab, K)
    S, _, _ = O.irls(e, lab, K, zf, p)
    depth, log_scale, logz = O.finalize(e, lab, zf, S)
    v = lab >= 0
    assert np.all(np.isnan(depth[~v]))
    reg, R = ndimage.label(v)
    # G_0 regions: the same partition as the mask's 4-connected regions here
    ours, R2 = O.regions(e)
    assert R2 == R
    for r in range(1, R + 1):
        m = reg == r
        assert np.unique(ours[m]).size == 1
        # one constant shift per region, and zero mean
        shift = logz[m] - (zf[m] + S[lab[m]])
        assert np.ptp(shift) < 1e-12
        assert abs(logz[m].mean()) < 1e-12
    # log-scale = log-depth - fill on every pixel of the component
    assert np.max(np.abs(logz[v] - zf[v] - log_scale[lab[v]])) < 1e-12
    if s.cam.proj == "persp":
        assert np.allclose(depth[v], np.exp(logz[v]), rtol=1e-15, atol=0)
    else:
        assert np.array_equal(depth[v], logz[v])
    # gauge invariance: a constant added to S on a whole region changes nothing
    rng = np.random.default_rng(seed)
    comp_reg = np.zeros(K, np.int64)
    comp_reg[lab[v]] = reg[v]
    S2 = S + rng.normal(0, 0.5, R + 1)[comp_reg]
    d2, ls2, z2 = O.finalize(e, lab, zf, S2)
    assert np.max(np.abs(z2[v] - logz[v])) < 1e-12
    assert np.max(np.abs(ls2 - log_scale)) < 1e-12


def test_alignment_restitches_cut_plane():
    """Uniform-weight iterations re-stitch a plane cut into artificial components."""
    n, m, z, cam = synth.plane_persp(16, 20, 30.0, [0.2, 0.1, -1.0], 3.0)
    n64 = n[0, 0].astype(np.float64)
    tx, ty, _, _ = O.ray_tables(cam, *m.shape)
    z = -1.0 / (n64[0] * tx[None, :] + n64[1] * ty[:, None] + n64[2])
    lab = np.zeros(m.shape, np.int32)
    lab[:8, 10:] = 1
    lab[8:, :10] = 2
    lab[8:, 10:] = 3
    r = O.integrate(n, m, cam, dict(irls_iters=2), labels_in=lab)
    assert np.ptp(np.log(r.depth) - np.log(z)) < 1e-12


def test_component_offset_invariance():
    """Per-component log offsets added to the fill do not change the output."""
    s = synth.tiny(1, proj="persp")
    p = dict(s.params)
    a = O.integrate(s.normals, s.mask, s.cam, p)
    rng = np.random.default_rng(0)
    off = rng.normal(0, 0.3, a.K)
    zf = np.where(a.labels >= 0, a.zfill + off[np.maximum(a.labels, 0)], 0.0)
    b = O.integrate(s.normals, s.mask, s.cam, p, zfill_in=zf)
    v = s.mask > 0
    assert np.max(np.abs(a.logz[v] - b.logz[v])) < 1e-9


def test_nonfinite_raises():
    s = synth.tiny(0)
    n = s.normals.copy()
    v = np.argwhere(s.mask > 0)[0]
    n[v[0], v[1], 1] = np.nan
    with pytest.raises(O.NonFiniteInput):
        O.edges(n, s.mask, s.cam, 2.0)
    m = s.mask.copy()
    m[v[0], v[1]] = 0
    O.edges(n, m, s.cam, 2.0)   # NaN off the mask is ignored


def test_generator_deterministic():
    a = synth.make("c1", 3)
    b = synth.make("c1", 3)
    assert np.array_equal(a.normals, b.normals) and np.array_equal(a.mask, b.mask)
    c = synth.make("c1", 4)
    assert not np.array_equal(a.normals, c.normals)


# --------------------------------------------------------------- merging ----
def _region_gauge(z, v, conn=4):
    from scipy import ndimage
    reg, R = ndimage.label(v, structure=np.ones((3, 3)) if conn == 8 else None)
    z = z.copy()
    for r in range(1, R + 1):
        z[reg == r] -= z[reg == r].mean()
    return z


@pytest.mark.parametrize("which,seed,freq,T", [("tiny", 1, 3, 10), ("tiny", 2, 2, 6), ("tiny", 4, 5, 8),
                                               ("c1", 0, 5, 8), ("c1", 1, 3, 10), ("c1", 2, 4, 9)])
def test_merging_equals_bruteforce(which, seed, freq, T):
    """Optional merging (Sec. 3.5 (i)-(iii), Alg. 1): the oracle's grouped
    form (one scale per original component, nodes regrouped) equals a
    brute force that rewrites pixel labels and carries the log-depth itself
    through every merge."""
    s = synth.tiny(seed, 12, 14, "persp") if which == "tiny" else synth.make(which, seed)
    p = dict(O.DEFAULT_PARAMS, irls_iters=T, freq_merging=freq)
    e = O.edges(s.normals, s.mask, s.cam, p["theta_c_deg"])
    lab, K = O.labels(e)
    zf = O.fill(e, lab, K)
    S, En, _ = O.irls(e, lab, K, zf, p)
    v = lab >= 0
    zo = np.where(v, zf + S[np.maximum(lab, 0)], 0.0)
    zb, Eb = BF.irls_merging(s.normals, s.mask, s.cam.as_dict(), lab, K, zf, p)
    assert np.max(np.abs(_region_gauge(zo, v) - _region_gauge(zb, v))[v]) < 1e-9
    assert np.allclose(En, Eb, rtol=1e-8, atol=1e-14)


def test_merge_selection_and_halving():
    """One merge on c1 after two reweighted steps: every group's selected
    edge has the smallest |residual| among its live edges (on the 2^-40
    grid, ties to the smaller code), and every new group holds at least two
    old ones unless
    the old one had no live edge, so the node count at least halves."""
    s = synth.make("c1", 3)
    p = dict(O.DEFAULT_PARAMS, irls_iters=4)
    e = O.edges(s.normals, s.mask, s.cam, p["theta_c_deg"])
    lab, K = O.labels(e)
    zf = O.fill(e, lab, K)
    S, _, ie = O.irls(e, lab, K, zf, p)
    z = np.where(lab >= 0, zf + S[np.maximum(lab, 0)], 0.0).ravel()
    r = z[ie.a] - z[ie.b] - ie.omega
    grp0 = np.arange(K)
    new = O.merge_groups(ie, r, grp0)
    code = ie.code
    for g in range(K):
        inc = np.flatnonzero((ie.c == g) | (ie.d == g))
        if inc.size == 0:
            continue
        best = inc[np.lexsort((code[inc], np.floor(np.abs(r[inc]) * 2.0 ** 40)))[0]]
        other = ie.d[best] if ie.c[best] == g else ie.c[best]
        assert new[g] == new[other]
    sizes = np.bincount(new)
    has_edge = np.zeros(K, bool)
    has_edge[ie.c] = True
    has_edge[ie.d] = True
    for h in range(sizes.size):
        members = np.flatnonzero(new == h)
        assert members.size >= 2 or not has_edge[members[0]]
    assert sizes.size <= (K + 1) // 2 + np.sum(~has_edge)


def test_merging_after_the_last_step_changes_nothing():
    """A merge frequency beyond T leaves the loop without merging; a merge
    that would fall after the last iteration is not taken."""
    s = synth.make("c1", 0)
    base = dict(O.DEFAULT_PARAMS, irls_iters=7)
    e = O.edges(s.normals, s.mask, s.cam, base["theta_c_deg"])
    lab, K = O.labels(e)
    zf = O.fill(e, lab, K)
    S0, E0, _ = O.irls(e, lab, K, zf, base)
    for f in (7, 50):
        S1, E1, _ = O.irls(e, lab, K, zf, dict(base, freq_merging=f))
        assert np.array_equal(S0, S1) and E0 == E1


# ------------------------------------------------- pixel-level baseline ----
@pytest.mark.parametrize("which,seed", [("tiny", 1), ("tiny", 2), ("tiny", 3), ("c1", 0)])
def test_logdepth_baseline_equals_direct_solve(which, seed):
    """The pixel-level log-depth baseline (ND form, reading A28) run through
    the oracle's relative-scale loop (every pixel a node, increments) equals
    a brute force that solves each iteration for the log-depth itself."""
    s = synth.tiny(seed, 12, 14, "persp") if which == "tiny" else synth.make(which, seed)
    p = dict(O.DEFAULT_PARAMS, irls_iters=8, variant=1)
    ref = O.integrate(s.normals, s.mask, s.cam, p)
    zb, Eb = BF.logdepth_irls(s.normals, s.mask, s.cam.as_dict(), p)
    v = s.mask > 0
    assert ref.K == int(v.sum())
    # two exact FP64 solves of the same pixel-level systems (weights spanning
    # many decades on c1) agree to ~1e-9 of the unit-scale log-depth
    assert np.max(np.abs(ref.logz[v] - _region_gauge(zb, v)[v])) < 1e-8
    assert np.allclose(ref.energies, Eb, rtol=1e-9, atol=1e-14)


# --------------------------------------------------------- 8-connectivity ----
def _dir_of(a, b):
    du, dv = b[0] - a[0], b[1] - a[1]
    return {(1, 0): 0, (0, 1): 1, (1, 1): 2, (-1, 1): 3}[(du, dv)]


@pytest.mark.parametrize("proj", ["persp", "ortho"])
def test_edges8_match_bruteforce_pairs(proj):
    """Diagonal edges (reading A29): usability, omega and gamma^2 of every
    pair equal the scalar two-tangent-planes model with the midpoint ray and
    f^2 = fx fy."""
    s = synth.tiny(2, 11, 13, proj=proj, noise=0.03)
    e = O.edges(s.normals, s.mask, s.cam, 2.0, connectivity=8)
    valid, usable, similar, info = BF.model(s.normals, s.mask, s.cam.as_dict(), 2.0, connectivity=8)
    H, W = s.mask.shape
    dirs = e.directions()
    flags = [np.zeros((H, W), bool) for _ in range(4)]
    simf = [np.zeros((H, W), bool) for _ in range(4)]
    for (a, b) in usable:
        flags[_dir_of(a, b)][a[1], a[0]] = True
    for (a, b) in similar:
        simf[_dir_of(a, b)][a[1], a[0]] = True
    for k, du, dv, use, sim, om, g2 in dirs:
        assert np.array_equal(flags[k], use), k
        assert np.array_equal(simf[k], sim), k
    for (a, b), (om, g2a, g2b) in info.items():
        k, _, _, _, _, omk, g2k = dirs[_dir_of(a, b)]
        assert abs(omk[a[1], a[0]] - om) < 1e-13
        assert abs(g2k[a[1], a[0]] - g2a) <= 1e-12 * g2a
        assert abs(g2k[b[1], b[0]] - g2b) <= 1e-12 * g2b


def test_diagonal_omega_exact_on_planes_and_quadrics():
    """The diagonal model of continuity is exact where the axis one is: a
    perspective plane, and (orthographic) any quadratic height field."""
    n, m, z, cam = synth.plane_persp(16, 20, 30.0, [0.2, 0.1, -1.0], 3.0)
    e = O.edges(n, m, cam, 2.0, connectivity=8)
    lz = np.log(z)
    assert e.valid_dr[:-1, :-1].all() and e.valid_dl[:-1, 1:].all()
    assert np.max(np.abs(e.omega_dr[:-1, :-1] - (lz[:-1, :-1] - lz[1:, 1:]))) < 1e-6
    assert np.max(np.abs(e.omega_dl[:-1, 1:] - (lz[:-1, 1:] - lz[1:, :-1]))) < 1e-6
    n, m, z, cam = synth.quadric_ortho(14, 17, (0.01, -0.02, 0.015, 0.1, -0.2, 3.0))
    e = O.edges(n.astype(np.float64), m, cam, 2.0, connectivity=8)
    assert np.max(np.abs(e.omega_dr[:-1, :-1] - (z[:-1, :-1] - z[1:, 1:]))) < 1e-12
    assert np.max(np.abs(e.omega_dl[:-1, 1:] - (z[:-1, 1:] - z[1:, :-1]))) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_labels8_match_transitive_closure(seed):
    proj = "persp" if seed % 2 else "ortho"
    s = synth.tiny(seed, proj=proj)
    e = O.edges(s.normals, s.mask, s.cam, 2.0, connectivity=8)
    lab, K = O.labels(e)
    valid, usable, similar, info = BF.model(s.normals, s.mask, s.cam.as_dict(), 2.0, connectivity=8)
    ref, Kr = BF.closure_labels(*s.mask.shape, valid, similar)
    assert K == Kr and np.array_equal(lab, ref)


def test_labels8_theta_180_is_mask_8_connectivity():
    s = synth.tiny(4, 12, 12, "persp", noise=0.0, step=0.0)
    e = O.edges(s.normals, s.mask, s.cam, 180.0, connectivity=8)
    lab, K = O.labels(e)
    ref, nref = ndimage.label(s.mask, structure=np.ones((3, 3)))
    assert K == nref and np.array_equal(lab, ref - 1)


@pytest.mark.parametrize("seed", range(3))
def test_fill8_matches_dense_rows(seed):
    proj = "persp" if seed % 2 == 0 else "ortho"
    s = synth.tiny(seed, proj=proj, noise=0.02)
    e = O.edges(s.normals, s.mask, s.cam, 2.0, connectivity=8)
    lab, K = O.labels(e)
    z = O.fill(e, lab, K)
    valid, usable, similar, info = BF.model(s.normals, s.mask, s.cam.as_dict(), 2.0, connectivity=8)
    zr = BF.fill_rows(s.normals, s.mask, s.cam.as_dict(), lab, info)
    v = s.mask > 0
    assert np.max(np.abs(z[v] - zr[v])) < 1e-10


@pytest.mark.parametrize("seed,mode", [(0, 1), (1, 1), (2, 2)])
def test_irls8_matches_dense_rows(seed, mode):
    proj = "persp" if seed % 2 == 0 else "ortho"
    s = synth.tiny(seed, proj=proj, noise=0.01)
    p = dict(O.DEFAULT_PARAMS, irls_iters=6, outlier_mode=mode, connectivity=8)
    if proj == "ortho":
        p["bini_k"] = 50.0
    e = O.edges(s.normals, s.mask, s.cam, 2.0, connectivity=8)
    lab, K = O.labels(e)
    zf = O.fill(e, lab, K)
    S, En, _ = O.irls(e, lab, K, zf, p)
    valid, usable, similar, info = BF.model(s.normals, s.mask, s.cam.as_dict(), 2.0, connectivity=8)
    Sr, Er = BF.irls_rows(s.normals, s.mask, s.cam.as_dict(), lab, K, zf, usable, info, p)
    assert np.max(np.abs(S - Sr)) < 1e-8
    assert np.allclose(En, Er, rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("which,seed,freq", [("tiny", 1, 3), ("c1", 0, 4)])
def test_merging8_equals_bruteforce(which, seed, freq):
    s = synth.tiny(seed, 12, 14, "persp") if which == "tiny" else synth.make(which, seed)
    p = dict(O.DEFAULT_PARAMS, irls_iters=9, freq_merging=freq, connectivity=8)
    e = O.edges(s.normals, s.mask, s.cam, p["theta_c_deg"], connectivity=8)
    lab, K = O.labels(e)
    zf = O.fill(e, lab, K)
    S, En, _ = O.irls(e, lab, K, zf, p)
    v = lab >= 0
    zo = np.where(v, zf + S[np.maximum(lab, 0)], 0.0)
    zb, Eb = BF.irls_merging(s.normals, s.mask, s.cam.as_dict(), lab, K, zf, p)
    assert np.max(np.abs(_region_gauge(zo, v, 8) - _region_gauge(zb, v, 8))[v]) < 1e-9
    assert np.allclose(En, Eb, rtol=1e-8, atol=1e-14)


def test_baseline8_equals_direct_solve():
    s = synth.tiny(2, 12, 14, "persp")
    p = dict(O.DEFAULT_PARAMS, irls_iters=6, variant=1, connectivity=8)
    ref = O.integrate(s.normals, s.mask, s.cam, p)
    zb, Eb = BF.logdepth_irls(s.normals, s.mask, s.cam.as_dict(), p)
    v = s.mask > 0
    assert np.max(np.abs(ref.logz[v] - _region_gauge(zb, v, p.get("connectivity", 4))[v])) < 1e-8
    assert np.allclose(ref.energies, Eb, rtol=1e-9, atol=1e-14)
