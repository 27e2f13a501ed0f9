"""FP64 CPU oracle of component-based normal integration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may call it.  It shares no code with the HIP library.

It follows the method of "Towards Fast and Scalable Normal Integration using
Continuous Components" (Milano et al., WACV 2026) step by step, with every
linear system solved *exactly* (sparse direct factorisation of the
gauge-fixed system) instead of by conjugate gradients:

  edges()     model of continuity on log-depth (Sec. 3.1, Eq. 1) with the
              central-camera coefficient of Eq. 3, the per-row factor
              gamma = f n_a.tau_a (Eq. 7), and the normal-similarity test of
              Sec. 3.3 (theta_ab < theta_c);
  labels()    continuous components = connected components over similar
              edges (Sec. 3.3), canonicalised to the minimum raster index;
  fill()      per-component weighted least squares on the intra-component
              edges with BiNI weights at z=0 (Sec. 3.3, Eq. 14-15);
  irls()      relative-scale optimisation on the inter-component edges
              (Sec. 3.4, Eq. 11-12 and 16-19; Alg. 1's main loop);
  finalize()  log-depth = fill + scale, one gauge per connected region.

Where the paper is silent or ambiguous (orthographic analogue of Eq. 3,
gauge choices, the weight cut, threshold strictness, ...) the reading taken
is stated where it is applied and tagged A1..A26.
Every function here is pinned by tests/test_oracle_pins.py (printed values,
closed forms, brute force on tiny maps, invariants).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import connected_components

# Method parameters.  Values in brackets are the paper's (Sec. 3.4, Sec. 4).
DEFAULT_PARAMS = dict(
    theta_c_deg=2.0,      # similarity threshold [2.0 deg on large maps]; <= 0: pixel level
    irls_iters=15,        # T [15 on large maps]
    align_iters=2,        # uniform-weight iterations t <= 1 [2]
    bini_k=2.0,           # sigmoid sharpness k of Eq. 5 (value not given; A5)
    out_L=1e-5,           # Eq. 18 lower threshold [1e-5]
    out_U=1e-3,           # Eq. 18 upper threshold [1e-3]
    outlier_mode=1,       # 0 off, 1 soft (Eq. 18), 2 hard (Suppl. ablation)
    delta_e_max=0.0,      # relative-energy stop; 0 runs exactly T iterations (A13)
    w_cut_rel=1e-12,      # quotient edges below this fraction of the max weight are cut (A16)
    freq_merging=0,       # optional merging (Sec. 3.5) after every freq-th iteration; 0 off [5]
    variant=0,            # 0 the component method; 1 the pixel-level log-depth baseline, ND form (A28)
    connectivity=4,       # 4 or 8 neighbours (A21, A29) [8]
)


class NonFiniteInput(ValueError):
    pass


@dataclass
class Edges:
    H: int
    W: int
    proj: str
    valid: np.ndarray       # bool [H, W]      pixel is a graph node
    valid_r: np.ndarray     # bool [H, W]      edge (u,v)-(u+1,v) usable
    valid_d: np.ndarray     # bool [H, W]      edge (u,v)-(u,v+1) usable
    sim_r: np.ndarray       # bool [H, W]      ... and normals similar
    sim_d: np.ndarray
    omega_r: np.ndarray     # f64 [H, W]       omega_{b->a} for b = right neighbour
    omega_d: np.ndarray     # f64 [H, W]       omega_{b->a} for b = lower neighbour
    g2_h: np.ndarray        # f64 [H, W]       gamma^2 of horizontal rows ending at the pixel
    g2_v: np.ndarray        # f64 [H, W]       gamma^2 of vertical rows ending at the pixel
    # 8-connectivity (A29): edge (u,v)-(u+1,v+1) ("dr") and (u,v)-(u-1,v+1)
    # ("dl"); all False / 0 with 4-connectivity
    valid_dr: np.ndarray = None
    valid_dl: np.ndarray = None
    sim_dr: np.ndarray = None
    sim_dl: np.ndarray = None
    omega_dr: np.ndarray = None
    omega_dl: np.ndarray = None
    g2_x: np.ndarray = None  # f64 [H, W]       gamma^2 of diagonal rows ending at the pixel
    conn: int = 4

    def directions(self):
        """(dir, du, dv, usable, similar, omega, gamma^2 per pixel) of every
        edge direction owned by the upper / left end: 0 right, 1 down, and
        with 8-connectivity 2 down-right, 3 down-left."""
        out = [(0, 1, 0, self.valid_r, self.sim_r, self.omega_r, self.g2_h),
               (1, 0, 1, self.valid_d, self.sim_d, self.omega_d, self.g2_v)]
        if self.conn == 8:
            out += [(2, 1, 1, self.valid_dr, self.sim_dr, self.omega_dr, self.g2_x),
                    (3, -1, 1, self.valid_dl, self.sim_dl, self.omega_dl, self.g2_x)]
        return out


def ray_tables(cam, H, W):
    """Ray direction tables tau(u, v) = ((u-cx)/fx, (v-cy)/fy, 1) at pixel
    centres and at the midpoints between horizontal / vertical neighbours
    (the interpolating subpixel m of Eq. 3, read as the midpoint: A2)."""
    u = np.arange(W, dtype=np.float64)
    v = np.arange(H, dtype=np.float64)
    tx = (u - cam.cx) / cam.fx
    ty = (v - cam.cy) / cam.fy
    txm = ((u + 0.5) - cam.cx) / cam.fx
    tym = ((v + 0.5) - cam.cy) / cam.fy
    return tx, ty, txm, tym


def _cam_get(cam, k):
    return cam[k] if isinstance(cam, dict) else getattr(cam, k)


class _Cam:
    def __init__(self, cam):
        self.proj = _cam_get(cam, "proj")
        if self.proj not in ("ortho", "persp"):
            raise ValueError("camera projection must be 'ortho' or 'persp'")
        self.fx = float(_cam_get(cam, "fx"))
        self.fy = float(_cam_get(cam, "fy"))
        self.cx = float(_cam_get(cam, "cx"))
        self.cy = float(_cam_get(cam, "cy"))
        self.pixel_pitch = float(_cam_get(cam, "pixel_pitch"))


def edges(normals, mask, cam, theta_c_deg, connectivity=4) -> Edges:
    """Per-edge quantities of the model of continuity (Sec. 3.1).

    Perspective (Eq. 3): with the four dot products d_aa = n_a.tau_a,
    d_am = n_a.tau_m, d_bb = n_b.tau_b, d_bm = n_b.tau_m,
        omega_{b->a} = log( (d_am / d_aa) * (d_bb / d_bm) ),
    the log-depth difference of two tangent planes that meet on the ray of the
    midpoint m.  The edge is usable iff each tangent plane meets that ray in
    front of the camera: d_aa, d_am non-zero of one sign and d_bb, d_bm
    non-zero of one sign (A18).  gamma_{b->a} = f n_a.tau_a (Eq. 7) with f = fx
    for horizontal and fy for vertical rows (A4).

    Orthographic (A1): additive depth, the same two-tangent-plane construction
    with parallel rays:
        omega_{b->a} = s ( (n_ax du + n_ay dv)/(2 n_az) + (n_bx du + n_by dv)/(2 n_bz) ),
    (du, dv) = b - a, s = pixel pitch; usable iff n_az, n_bz are non-zero;
    gamma = n_z.

    Similarity (Sec. 3.3): theta_ab < theta_c  <=>  n_a.n_b > cos(theta_c)
    (A19), evaluated in FP64 from the FP32 inputs as
    (n_ax n_bx + n_ay n_by) + n_az n_bz.  theta_c <= 0 marks no edge similar
    (every pixel its own component, "theta_c = None").
    """
    cam = _Cam(cam)
    n = np.asarray(normals)
    if n.dtype not in (np.float32, np.float64) or n.ndim != 3 or n.shape[2] != 3:
        raise TypeError("normals must be float32 (or float64) [H, W, 3]")
    H, W, _ = n.shape
    valid = np.asarray(mask) != 0
    if not np.all(np.isfinite(n[valid])):
        raise NonFiniteInput("non-finite normal inside the mask")
    nx = n[..., 0].astype(np.float64)
    ny = n[..., 1].astype(np.float64)
    nz = n[..., 2].astype(np.float64)
    nx = np.where(valid, nx, 0.0)
    ny = np.where(valid, ny, 0.0)
    nz = np.where(valid, nz, 0.0)

    vr = np.zeros((H, W), bool)
    vd = np.zeros((H, W), bool)
    vr[:, :-1] = valid[:, :-1] & valid[:, 1:]
    vd[:-1, :] = valid[:-1, :] & valid[1:, :]
    om_r = np.zeros((H, W))
    om_d = np.zeros((H, W))

    if cam.proj == "persp":
        tx, ty, txm, tym = ray_tables(cam, H, W)
        TX, TY = tx[None, :], ty[:, None]
        nt = (nx * TX + ny * TY) + nz                      # n_a . tau_a
        # horizontal edges: midpoint ray (txm[u], ty[v], 1)
        dam = (nx[:, :-1] * txm[None, :-1] + ny[:, :-1] * TY) + nz[:, :-1]
        dbm = (nx[:, 1:] * txm[None, :-1] + ny[:, 1:] * TY) + nz[:, 1:]
        daa, dbb = nt[:, :-1], nt[:, 1:]
        ok = (daa != 0) & (dam != 0) & (dbb != 0) & (dbm != 0) \
            & ((daa > 0) == (dam > 0)) & ((dbb > 0) == (dbm > 0))
        vr[:, :-1] &= ok
        with np.errstate(divide="ignore", invalid="ignore"):
            om_r[:, :-1] = np.where(vr[:, :-1], np.log((dam / daa) * (dbb / dbm)), 0.0)
        # vertical edges: midpoint ray (tx[u], tym[v], 1)
        dam = (nx[:-1, :] * TX + ny[:-1, :] * tym[:-1, None]) + nz[:-1, :]
        dbm = (nx[1:, :] * TX + ny[1:, :] * tym[:-1, None]) + nz[1:, :]
        daa, dbb = nt[:-1, :], nt[1:, :]
        ok = (daa != 0) & (dam != 0) & (dbb != 0) & (dbm != 0) \
            & ((daa > 0) == (dam > 0)) & ((dbb > 0) == (dbm > 0))
        vd[:-1, :] &= ok
        with np.errstate(divide="ignore", invalid="ignore"):
            om_d[:-1, :] = np.where(vd[:-1, :], np.log((dam / daa) * (dbb / dbm)), 0.0)
        g2h = (cam.fx * nt) ** 2
        g2v = (cam.fy * nt) ** 2
    else:
        s = cam.pixel_pitch
        okz = nz != 0
        vr[:, :-1] &= okz[:, :-1] & okz[:, 1:]
        vd[:-1, :] &= okz[:-1, :] & okz[1:, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            om_r[:, :-1] = np.where(vr[:, :-1], s * (nx[:, :-1] / (2.0 * nz[:, :-1])
                                                     + nx[:, 1:] / (2.0 * nz[:, 1:])), 0.0)
            om_d[:-1, :] = np.where(vd[:-1, :], s * (ny[:-1, :] / (2.0 * nz[:-1, :])
                                                     + ny[1:, :] / (2.0 * nz[1:, :])), 0.0)
        g2h = nz ** 2
        g2v = nz ** 2

    sr = np.zeros((H, W), bool)
    sd = np.zeros((H, W), bool)
    if theta_c_deg > 0:
        cth = math.cos(theta_c_deg * math.pi / 180.0)
        dot_r = (nx[:, :-1] * nx[:, 1:] + ny[:, :-1] * ny[:, 1:]) + nz[:, :-1] * nz[:, 1:]
        dot_d = (nx[:-1, :] * nx[1:, :] + ny[:-1, :] * ny[1:, :]) + nz[:-1, :] * nz[1:, :]
        sr[:, :-1] = vr[:, :-1] & (dot_r > cth)
        sd[:-1, :] = vd[:-1, :] & (dot_d > cth)
    g2h = np.where(valid, g2h, 0.0)
    g2v = np.where(valid, g2v, 0.0)
    e = Edges(H, W, cam.proj, valid, vr, vd, sr, sd, om_r, om_d, g2h, g2v)
    z = np.zeros((H, W), bool)
    e.valid_dr, e.valid_dl, e.sim_dr, e.sim_dl = z, z.copy(), z.copy(), z.copy()
    e.omega_dr, e.omega_dl, e.g2_x = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W))
    if connectivity == 8:
        _diagonal_edges(e, nx, ny, nz, cam, theta_c_deg)
    elif connectivity != 4:
        raise ValueError("connectivity must be 4 or 8")
    return e


def _diagonal_edges(e: Edges, nx, ny, nz, cam, theta_c_deg):
    """Diagonal edges of 8-connectivity (reading A29): the same model of
    continuity with the interpolating subpixel at the midpoint of the two
    pixel centres (A2), i.e. the ray (u + 1/2, v + 1/2) for a = (u, v) and
    b = (u+1, v+1), and (u - 1/2, v + 1/2) for b = (u-1, v+1); gamma =
    f n_a.tau_a with f^2 = fx fy (the geometric mean of the two focal
    lengths, A4's choice for each axis); orthographic: A1 with (du, dv) =
    (+-1, 1) and gamma = n_z.  Similarity and usability as for the axis
    edges."""
    H, W = e.H, e.W
    valid = e.valid
    vdr = np.zeros((H, W), bool)
    vdl = np.zeros((H, W), bool)
    vdr[:-1, :-1] = valid[:-1, :-1] & valid[1:, 1:]
    vdl[:-1, 1:] = valid[:-1, 1:] & valid[1:, :-1]
    om_dr = np.zeros((H, W))
    om_dl = np.zeros((H, W))
    if cam.proj == "persp":
        tx, ty, txm, tym = ray_tables(cam, H, W)
        TX, TY = tx[None, :], ty[:, None]
        nt = (nx * TX + ny * TY) + nz
        # down-right: a = [:-1, :-1], b = [1:, 1:], midpoint ray (txm[u], tym[v])
        dam = (nx[:-1, :-1] * txm[None, :-1] + ny[:-1, :-1] * tym[:-1, None]) + nz[:-1, :-1]
        dbm = (nx[1:, 1:] * txm[None, :-1] + ny[1:, 1:] * tym[:-1, None]) + nz[1:, 1:]
        daa, dbb = nt[:-1, :-1], nt[1:, 1:]
        ok = (daa != 0) & (dam != 0) & (dbb != 0) & (dbm != 0) \
            & ((daa > 0) == (dam > 0)) & ((dbb > 0) == (dbm > 0))
        vdr[:-1, :-1] &= ok
        with np.errstate(divide="ignore", invalid="ignore"):
            om_dr[:-1, :-1] = np.where(vdr[:-1, :-1], np.log((dam / daa) * (dbb / dbm)), 0.0)
        # down-left: a = [:-1, 1:] (u >= 1), b = [1:, :-1], midpoint ray (txm[u-1], tym[v])
        dam = (nx[:-1, 1:] * txm[None, :-1] + ny[:-1, 1:] * tym[:-1, None]) + nz[:-1, 1:]
        dbm = (nx[1:, :-1] * txm[None, :-1] + ny[1:, :-1] * tym[:-1, None]) + nz[1:, :-1]
        daa, dbb = nt[:-1, 1:], nt[1:, :-1]
        ok = (daa != 0) & (dam != 0) & (dbb != 0) & (dbm != 0) \
            & ((daa > 0) == (dam > 0)) & ((dbb > 0) == (dbm > 0))
        vdl[:-1, 1:] &= ok
        with np.errstate(divide="ignore", invalid="ignore"):
            om_dl[:-1, 1:] = np.where(vdl[:-1, 1:], np.log((dam / daa) * (dbb / dbm)), 0.0)
        g2x = (cam.fx * cam.fy) * nt ** 2
    else:
        s = cam.pixel_pitch
        okz = nz != 0
        vdr[:-1, :-1] &= okz[:-1, :-1] & okz[1:, 1:]
        vdl[:-1, 1:] &= okz[:-1, 1:] & okz[1:, :-1]
        with np.errstate(divide="ignore", invalid="ignore"):
            om_dr[:-1, :-1] = np.where(vdr[:-1, :-1], s * ((nx[:-1, :-1] + ny[:-1, :-1]) / (2.0 * nz[:-1, :-1])
                                                         + (nx[1:, 1:] + ny[1:, 1:]) / (2.0 * nz[1:, 1:])), 0.0)
            om_dl[:-1, 1:] = np.where(vdl[:-1, 1:], s * ((-nx[:-1, 1:] + ny[:-1, 1:]) / (2.0 * nz[:-1, 1:])
                                                       + (-nx[1:, :-1] + ny[1:, :-1]) / (2.0 * nz[1:, :-1])), 0.0)
        g2x = nz ** 2
    sdr = np.zeros((H, W), bool)
    sdl = np.zeros((H, W), bool)
    if theta_c_deg > 0:
        cth = math.cos(theta_c_deg * math.pi / 180.0)
        dot_dr = (nx[:-1, :-1] * nx[1:, 1:] + ny[:-1, :-1] * ny[1:, 1:]) + nz[:-1, :-1] * nz[1:, 1:]
        dot_dl = (nx[:-1, 1:] * nx[1:, :-1] + ny[:-1, 1:] * ny[1:, :-1]) + nz[:-1, 1:] * nz[1:, :-1]
        sdr[:-1, :-1] = vdr[:-1, :-1] & (dot_dr > cth)
        sdl[:-1, 1:] = vdl[:-1, 1:] & (dot_dl > cth)
    e.valid_dr, e.valid_dl, e.sim_dr, e.sim_dl = vdr, vdl, sdr, sdl
    e.omega_dr, e.omega_dl = om_dr, om_dl
    e.g2_x = np.where(valid, g2x, 0.0)
    e.conn = 8


def _grid_graph(e: Edges, masks):
    """Sparse adjacency over the H*W raster indices; masks[k] flags the
    edges of direction k (0 right, 1 down, 2 down-right, 3 down-left) at
    their upper / left end."""
    H, W = e.H, e.W
    idx = np.arange(H * W).reshape(H, W)
    step = {0: 1, 1: W, 2: W + 1, 3: W - 1}
    a = np.concatenate([idx[m] for m in masks])
    b = np.concatenate([idx[m] + step[k] for k, m in enumerate(masks)])
    G = sp.coo_matrix((np.ones(a.size), (a, b)), shape=(H * W, H * W))
    return G


def canonical_components(e: Edges, masks):
    """Connected components of the valid pixels over the given edges (one
    mask per direction), numbered by ascending minimum raster index (A20);
    -1 off the mask."""
    H, W = e.H, e.W
    N = H * W
    ncomp, lab = connected_components(_grid_graph(e, masks), directed=False)
    valid = e.valid.ravel()
    roots = np.full(ncomp, N, dtype=np.int64)
    pix = np.arange(N)
    np.minimum.at(roots, lab[valid], pix[valid])
    used = roots < N
    order = np.argsort(roots[used], kind="stable")
    remap = np.full(ncomp, -1, dtype=np.int64)
    remap[np.flatnonzero(used)[order]] = np.arange(order.size)
    out = np.where(valid, remap[lab], -1).astype(np.int32)
    return out.reshape(H, W), int(order.size)


def labels(e: Edges):
    """Continuous components (Sec. 3.3): connected components of the
    subgraph of G_0 keeping only edges with theta_ab < theta_c."""
    return canonical_components(e, [d[4] for d in e.directions()])


def regions(e: Edges):
    """Connected regions of G_0 itself (all usable edges)."""
    return canonical_components(e, [d[3] for d in e.directions()])


def _intra_system(e: Edges, lab):
    """Normal equations A_c^T W_c A_c z = A_c^T W_c b_c of Eq. 14-15 for all
    components at once (block diagonal).  Rows: both directed rows of every
    usable edge with both ends in one component (A8, A9), weighted by
    W = gamma^2 * sigma_k(0) = gamma^2 / 2 (a single reweighting pass from
    z = 0: A7).  Per undirected edge the two rows fold into
    w = (gamma^2_{b->a} + gamma^2_{a->b}) / 2 times (z_a - z_b - omega_{b->a})^2."""
    H, W = e.H, e.W
    N = H * W
    idx = np.arange(N).reshape(H, W)
    labf = lab.ravel()
    step = {0: 1, 1: W, 2: W + 1, 3: W - 1}
    aa, bb, ww, oo = [], [], [], []
    for k, du, dv, usable, _, omega, g2 in e.directions():
        ai = idx[usable]
        bi = ai + step[k]
        inside = labf[ai] == labf[bi]
        ai, bi = ai[inside], bi[inside]
        g2f = g2.ravel()
        aa.append(ai)
        bb.append(bi)
        ww.append(0.5 * g2f[ai] + 0.5 * g2f[bi])
        oo.append(omega[usable][inside])
    a = np.concatenate(aa)
    b = np.concatenate(bb)
    w = np.concatenate(ww)
    om = np.concatenate(oo)
    Lap = sp.coo_matrix((np.concatenate([w, w, -w, -w]),
                         (np.concatenate([a, b, a, b]), np.concatenate([a, b, b, a]))),
                        shape=(N, N)).tocsr()
    rhs = np.zeros(N)
    np.add.at(rhs, a, w * om)
    np.add.at(rhs, b, -w * om)
    return Lap, rhs


def _solve_pinned(Lap, rhs, groups, ngroups, active):
    """Exact solution of a block-diagonal graph-Laplacian system with one
    block per group: pin the minimum index of each group to zero, factorise
    the remaining SPD system, then shift each group to zero mean (A15).
    Nodes with active=False (e.g. off the mask) get 0."""
    n = Lap.shape[0]
    x = np.zeros(n)
    nodes = np.flatnonzero(active)
    if nodes.size == 0:
        return x
    g = groups[nodes]
    first = np.full(ngroups, n, dtype=np.int64)
    np.minimum.at(first, g, nodes)
    keep = np.ones(n, bool)
    keep[first[first < n]] = False
    keep &= active
    kidx = np.flatnonzero(keep)
    if kidx.size:
        A = Lap[kidx][:, kidx].tocsc()
        x[kidx] = spla.spsolve(A, rhs[kidx]) if kidx.size > 1 else rhs[kidx] / A.toarray()[0, 0]
    sums = np.zeros(ngroups)
    cnt = np.zeros(ngroups)
    np.add.at(sums, g, x[nodes])
    np.add.at(cnt, g, 1.0)
    x[nodes] -= sums[g] / cnt[g]
    return x


def fill(e: Edges, lab, K):
    """Fill every component (Sec. 3.3, Eq. 15): exact solution of the
    component's weighted normal equations, gauge = zero mean per component
    (the minimum-norm solution that CG from z = 0 converges to; A15)."""
    Lap, rhs = _intra_system(e, lab)
    labf = lab.ravel()
    active = labf >= 0
    z = _solve_pinned(Lap, rhs, np.where(active, labf, 0), max(K, 1), active)
    return z.reshape(e.H, e.W)


@dataclass
class InterEdges:
    a: np.ndarray       # raster index of the upper / left pixel
    b: np.ndarray       # raster index of the other end
    dir: np.ndarray     # 0 right (b = a+1), 1 down (a+W), 2 down-right (a+W+1), 3 down-left (a+W-1)
    omega: np.ndarray   # omega_{b->a}
    c: np.ndarray       # pi(a)
    d: np.ndarray       # pi(b)

    @property
    def code(self):
        """Edge code 4 a + dir (the order of the merge tie-break, A27)."""
        return 4 * self.a + self.dir


def inter_edges(e: Edges, lab) -> InterEdges:
    """E_inter (Eq. 9): usable edges whose ends lie in different components."""
    H, W = e.H, e.W
    idx = np.arange(H * W).reshape(H, W)
    labf = lab.ravel()
    step = {0: 1, 1: W, 2: W + 1, 3: W - 1}
    aa, dd, oo = [], [], []
    for k, du, dv, usable, _, omega, g2 in e.directions():
        ai = idx[usable]
        x = labf[ai] != labf[ai + step[k]]
        aa.append(ai[x])
        dd.append(np.full(int(x.sum()), k, dtype=np.int64))
        oo.append(omega[usable][x])
    a = np.concatenate(aa)
    dirs = np.concatenate(dd)
    b = a + np.array([1, W, W + 1, W - 1], dtype=np.int64)[dirs]
    om = np.concatenate(oo)
    return InterEdges(a, b, dirs, om, labf[a].astype(np.int64), labf[b].astype(np.int64))


def sigmoid(x, k=1.0):
    """sigma_k(x) = 1 / (1 + exp(-k x)) (Eq. 5); exp overflow gives 0."""
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-k * np.asarray(x, dtype=np.float64)))


def outlier_weight(chi_abs, L=1e-5, U=1e-3, mode=1):
    """W^out of Eq. 18 (mode 1): sigma_1( 4/(lL - lU) * (2 log10|chi| - (lL + lU)) )
    with lX = log10(X); |chi| = 0 maps to 1 (A12).  Mode 2 is the hard
    threshold of the supplementary ablation (0 if |chi| >= U else 1); mode 0
    disables the reweighting."""
    chi_abs = np.abs(np.asarray(chi_abs, dtype=np.float64))
    if mode == 0:
        return np.ones_like(chi_abs)
    if mode == 2:
        return (chi_abs < U).astype(np.float64)
    lL, lU = math.log10(L), math.log10(U)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        x = np.log10(chi_abs)
        arg = 4.0 / (lL - lU) * (2.0 * x - (lL + lU))
        out = 1.0 / (1.0 + np.exp(-arg))
    return np.where(chi_abs == 0, 1.0, out)


def edge_weights(e: Edges, ie: InterEdges, z, t, params):
    """Per undirected inter edge, w_e = W_{b->a} + W_{a->b} (A9) and the
    residual r_e = z_a - z_b - omega_{b->a} at the current log-depth (A11).

    t < align_iters: every directed row weighs 1 (Alg. 1's alignment phase).
    Otherwise (Eq. 5-7, 18-19), for the row ending at pixel a with the other
    end b and the pixel -b opposite b across a:
        W_{b->a} = g^2 sigma_k( g^2 ((z_{-b} - z_a)^2 - (z_b - z_a)^2) ) W^out(|r_e|)
    with g^2 = gamma^2_{b->a}; a missing (unusable) edge (a, -b) contributes
    (z_{-b} - z_a) = 0 (A6)."""
    H, W = e.H, e.W
    zf = z.ravel()
    r = zf[ie.a] - zf[ie.b] - ie.omega
    if t < params["align_iters"]:
        return np.full(r.size, 2.0), r
    k = params["bini_k"]
    dirs = e.directions()
    usable = np.stack([d[3].ravel() for d in dirs] + [np.zeros(H * W, bool)] * (4 - len(dirs)))
    g2 = np.stack([d[6].ravel() for d in dirs] + [np.zeros(H * W)] * (4 - len(dirs)))
    step = np.array([1, W, W + 1, W - 1], dtype=np.int64)[ie.dir]
    ua, va = ie.a % W, ie.a // W
    # row b -> a: opposite pixel -b = a - step, edge (a - step, a) of the same direction
    has_ma = np.select([ie.dir == 0, ie.dir == 1, ie.dir == 2], [ua > 0, va > 0, (ua > 0) & (va > 0)],
                       (ua < W - 1) & (va > 0))
    ma = np.where(has_ma, ie.a - step, 0)
    ok_ma = has_ma & usable[ie.dir, ma]
    dm = np.where(ok_ma, zf[ma] - zf[ie.a], 0.0)
    dp = zf[ie.b] - zf[ie.a]
    g2a = g2[ie.dir, ie.a]
    Wba = g2a * sigmoid(g2a * (dm * dm - dp * dp), k)
    # row a -> b: opposite pixel -a = b + step, edge (b, b + step)
    ok_pb = usable[ie.dir, ie.b]
    pb = np.where(ok_pb, ie.b + step, 0)
    dm2 = np.where(ok_pb, zf[pb] - zf[ie.b], 0.0)
    dp2 = zf[ie.a] - zf[ie.b]
    g2b = g2[ie.dir, ie.b]
    Wab = g2b * sigmoid(g2b * (dm2 * dm2 - dp2 * dp2), k)
    wout = outlier_weight(r, params["out_L"], params["out_U"], params["outlier_mode"])
    if t < params.get("out_from", 0):
        wout = np.ones_like(wout)
    return (Wba + Wab) * wout, r


def quotient_step(ie: InterEdges, K, w, r, w_cut_rel):
    """One relative-scale solve (Eq. 16-17) on the quotient graph (Eq. 10).

    Minimises sum_e w_e (r_e + s_c - s_d)^2 over s (c = pi(a), d = pi(b)).
    Edges lighter than w_cut_rel * max_e w_e are dropped (A16); the remaining
    weighted quotient graph splits into pieces, each solved exactly with zero
    (unweighted) mean of s over its components (A15).  Returns (s, E_t, w).
    """
    w = np.array(w, dtype=np.float64)
    if w.size:
        wmax = w.max()
        w[w < w_cut_rel * wmax] = 0.0
    c, d = ie.c, ie.d
    Q = sp.coo_matrix((np.concatenate([w, w, -w, -w]),
                       (np.concatenate([c, d, c, d]), np.concatenate([c, d, d, c]))),
                      shape=(K, K)).tocsr()
    rhs = np.zeros(K)
    np.add.at(rhs, c, -w * r)
    np.add.at(rhs, d, w * r)
    pos = w > 0
    G = sp.coo_matrix((np.ones(int(pos.sum())), (c[pos], d[pos])), shape=(K, K))
    npieces, piece = connected_components(G, directed=False)
    s = _solve_pinned(Q, rhs, piece, npieces, np.ones(K, bool))
    res = r + s[c] - s[d]
    E = float(np.sum(w * res * res))
    return s, E, w


def merge_groups(ie: InterEdges, r, grp):
    """Optional merging (Sec. 3.5, steps (i)-(iii); Alg. 1's merge block).

    grp maps every original component to its current group (a node of the
    quotient graph Q_m).  (i) Every group selects, among the inter edges
    incident to it (edges whose ends lie in different groups), the one
    with the smallest residual magnitude |chi| = |r_e| at the current
    log-depth.  Magnitudes are compared on a grid of 2^-40 (~9.1e-13 in
    log-depth units), and equal grid values go to the smaller edge code
    4 a + dir (dir 0 right, 1 down, 2 down-right, 3 down-left; reading A27):
    after the uniform-weight
    alignment every bridge of the quotient graph has a residual that is
    zero in exact arithmetic, so FP64 rounding alone would otherwise decide
    between them.  (ii) The selected edges form a subgraph of Q_m
    over all its nodes; (iii) its connected components are the new groups,
    numbered by the smallest original component they contain.  Returns
    the new map of original components to groups."""
    gc, gd = grp[ie.c], grp[ie.d]
    live = gc != gd
    Kg = int(grp.max()) + 1 if grp.size else 0
    code = ie.code
    best = np.full(Kg, -1, dtype=np.int64)
    idx = np.flatnonzero(live)
    # smallest |r| on the 2^-40 grid, then smallest code, per group end
    mag = np.floor(np.abs(r[idx]) * 2.0 ** 40)
    order = idx[np.lexsort((code[idx], mag))]
    for e in order:                      # first hit per group wins
        for g in (gc[e], gd[e]):
            if best[g] < 0:
                best[g] = e
    sel = best[best >= 0]
    G = sp.coo_matrix((np.ones(sel.size), (gc[sel], gd[sel])), shape=(Kg, Kg))
    _, comp = connected_components(G, directed=False)
    # canonical numbering: by the smallest original component in the group
    first = np.full(Kg, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(first, comp[grp], np.arange(grp.size))
    used = np.flatnonzero(first < np.iinfo(np.int64).max)
    rank = np.empty(comp.max() + 1 if comp.size else 0, dtype=np.int64)
    rank[used[np.argsort(first[used], kind="stable")]] = np.arange(used.size)
    return rank[comp[grp]]


def irls(e: Edges, lab, K, zfill, params=None, S0=None, t0=0, trace=None):
    """Relative-scale optimisation (Sec. 3.4; Alg. 1's loop).

    z^(t) = zfill + S_pi; each iteration solves for one increment per node
    of the current quotient graph with the weights of iteration t, then
    adds it to every component of the node (Eq. 12).  Stops after T
    iterations, or earlier when delta_e_max > 0 and |E_t - E_{t-1}| /
    E_{t-1} < delta_e_max with both t-1, t past the alignment phase (A13).

    With freq_merging = f > 0, after every iteration t with (t + 1) % f == 0
    the nodes are merged (merge_groups, Sec. 3.5) on the residuals at the
    updated log-depth; the merged node's components keep their scales (the
    log-depth does not change at a merge) and move together from then on,
    and edges inside a merged node leave the optimisation.  S stays one
    value per original component.

    S0 / t0 resume the loop at iteration t0 from the scales S0 (a test hook:
    one step at a time, without merging); trace, when a list, receives (t,
    S before step t, s^(t) per original component, E_t) for every
    iteration run.  irls.last_groups holds the final node of every
    component."""
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    ie = inter_edges(e, lab)
    S = np.zeros(K) if S0 is None else np.array(S0, dtype=np.float64)
    labf = lab.ravel()
    valid = labf >= 0
    energies = []
    margin = np.inf
    grp = np.arange(K, dtype=np.int64)
    freq = int(p.get("freq_merging", 0))
    for t in range(int(t0), int(p["irls_iters"])):
        z = np.where(valid, zfill.ravel() + S[np.where(valid, labf, 0)], 0.0)
        w, r = edge_weights(e, ie, z, t, p)
        live = grp[ie.c] != grp[ie.d]
        w = np.where(live, w, 0.0)
        if w.size and p["w_cut_rel"] > 0 and w.max() > 0:
            pos = w[w > 0]
            margin = min(margin, float(np.min(np.abs(np.log10(pos / (p["w_cut_rel"] * w.max()))))))
        Kg = int(grp.max()) + 1 if K else 0
        ieg = InterEdges(ie.a, ie.b, ie.dir, ie.omega, grp[ie.c], grp[ie.d])
        sg, E, _ = quotient_step(ieg, Kg, w, r, p["w_cut_rel"])
        s = sg[grp] if K else sg
        if trace is not None:
            trace.append((t, S.copy(), s.copy(), E))
        S += s
        energies.append(E)
        if freq > 0 and (t + 1) % freq == 0 and t + 1 < int(p["irls_iters"]):
            z = np.where(valid, zfill.ravel() + S[np.where(valid, labf, 0)], 0.0)
            r_now = z[ie.a] - z[ie.b] - ie.omega
            grp = merge_groups(ie, r_now, grp)
        if p["delta_e_max"] > 0 and t >= p["align_iters"] + 1 and len(energies) >= 2:
            Ep = energies[-2]
            if Ep == 0.0 or abs(E - Ep) / Ep < p["delta_e_max"]:
                break
    irls.last_cut_margin = margin
    irls.last_groups = grp
    return S, energies, ie


def finalize(e: Edges, lab, zfill, S):
    """Output gauge: log-depth z = zfill + S_pi shifted to zero pixel mean over
    every connected region of G_0 (A15); depth = exp(z) in perspective and
    z itself (additive model) in orthographic mode.  Returns
    (depth f64 [H, W] with NaN off the mask, log_scale f64 [K], z)."""
    reg, R = regions(e)
    labf = lab.ravel()
    regf = reg.ravel()
    valid = labf >= 0
    z = np.where(valid, zfill.ravel() + S[np.where(valid, labf, 0)], 0.0)
    sums = np.zeros(max(R, 1))
    cnt = np.zeros(max(R, 1))
    np.add.at(sums, regf[valid], z[valid])
    np.add.at(cnt, regf[valid], 1.0)
    shift = sums / np.maximum(cnt, 1.0)
    z = np.where(valid, z - shift[np.where(valid, regf, 0)], np.nan)
    K = S.size
    comp_region = np.zeros(K, dtype=np.int64)
    comp_region[labf[valid]] = regf[valid]
    log_scale = S - shift[comp_region] if K else S
    depth = np.exp(z) if e.proj == "persp" else z
    return depth.reshape(e.H, e.W), log_scale, z.reshape(e.H, e.W)


@dataclass
class Result:
    depth: np.ndarray
    labels: np.ndarray
    log_scale: np.ndarray
    K: int
    zfill: np.ndarray
    logz: np.ndarray
    energies: list
    n_inter_edges: int
    n_regions: int
    extra: dict = field(default_factory=dict)


def baseline_params(p):
    """The pixel-level log-depth baseline without discontinuity term (the ND
    form of the method the paper compares with, Sec. 4, Table 1; reading
    A28), as parameters of the same loop: every pixel its own node (no
    continuous components, so every fill is 0 and z starts at 0); no
    alignment phase, so the first iteration weighs each row by the BiNI
    weight at z = 0, gamma^2 sigma_k(0) = gamma^2 / 2 (Eq. 5-7); the outlier
    weights of Eq. 18 from the second iteration on (at z = 0 no residual
    carries information).  Each iteration then solves the full pixel system
    for the new log-depth, which is what solving for the increment of every
    pixel's log-depth amounts to."""
    q = dict(p)
    q.update(theta_c_deg=0.0, align_iters=0, out_from=1, freq_merging=0)
    return q


def integrate(normals, mask, cam, params=None, labels_in=None, zfill_in=None) -> Result:
    """The whole path: edges -> components -> fill -> relative scales -> output.

    labels_in / zfill_in inject a partition or a fill (test hooks that mirror
    the HIP library's staged entry points).  variant = 1 runs the pixel-level
    baseline instead (baseline_params)."""
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    if p.get("variant", 0) == 1:
        p = baseline_params(p)
    e = edges(normals, mask, cam, p["theta_c_deg"], p.get("connectivity", 4))
    if labels_in is None:
        lab, K = labels(e)
    else:
        lab = np.asarray(labels_in, dtype=np.int32)
        K = int(lab.max()) + 1 if lab.size and lab.max() >= 0 else 0
    zf = fill(e, lab, K) if zfill_in is None else np.where(lab >= 0, np.asarray(zfill_in, np.float64), 0.0)
    S, energies, ie = irls(e, lab, K, zf, p)
    depth, log_scale, logz = finalize(e, lab, zf, S)
    _, R = regions(e)
    # smallest |log10(w_e / (w_cut_rel * max w))| over all iterations: how
    # close any cut decision came to flipping (a diagnostic, not a result)
    return Result(depth, lab, log_scale, K, zf, logz, energies, int(ie.a.size), R,
                  extra=dict(cut_margin=irls.last_cut_margin))
