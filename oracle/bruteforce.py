"""Brute-force references for tiny maps (<= ~12x12), used to pin the oracle.

TEST INFRASTRUCTURE ONLY.  Written independently of ni_oracle.py: scalar
Python loops over pixels and edges, explicit stacked *directed rows* exactly
as the paper writes the systems (A_c, b_c, W_c of Eq. 14 and the quotient
A_m, b_m, W_m of Eq. 16), dense minimum-norm least squares, and transitive
closure for connectivity.  Different formulation, different code: a wrong
sign, index or transposition in the oracle's vectorised Laplacian assembly
shows up as a mismatch here.
"""
from __future__ import annotations

import math

import numpy as np


def _tau(cam, u, v):
    if cam["proj"] == "persp":
        return np.array([(u - cam["cx"]) / cam["fx"], (v - cam["cy"]) / cam["fy"], 1.0])
    return np.array([0.0, 0.0, 1.0])


def pair_model(n, cam, a, b):
    """(usable, omega_{b->a}, gamma2_{b->a}, gamma2_{a->b}) of one neighbour
    pair a=(u,v), b=(u',v') from the two-tangent-planes construction; the
    focal factor of gamma is fx along a row, fy along a column and
    sqrt(fx fy) along a diagonal."""
    (ua, va), (ub, vb) = a, b
    na = n[va, ua].astype(np.float64)
    nb = n[vb, ub].astype(np.float64)
    horiz = va == vb
    vert = ua == ub
    if cam["proj"] == "persp":
        ta = _tau(cam, ua, va)
        tb = _tau(cam, ub, vb)
        tm = _tau(cam, 0.5 * (ua + ub), 0.5 * (va + vb))
        daa, dam, dbb, dbm = na @ ta, na @ tm, nb @ tb, nb @ tm
        if min(abs(daa), abs(dam), abs(dbb), abs(dbm)) == 0:
            return False, 0.0, 0.0, 0.0
        if (daa > 0) != (dam > 0) or (dbb > 0) != (dbm > 0):
            return False, 0.0, 0.0, 0.0
        # z_m from a's tangent plane equals z_m from b's: z_a daa/dam = z_b dbb/dbm
        om = math.log(dam / daa) - math.log(dbm / dbb)
        f2 = cam["fx"] ** 2 if horiz else cam["fy"] ** 2 if vert else cam["fx"] * cam["fy"]
        return True, om, f2 * daa ** 2, f2 * dbb ** 2
    if na[2] == 0 or nb[2] == 0:
        return False, 0.0, 0.0, 0.0
    s = cam["pixel_pitch"]
    du, dv = ub - ua, vb - va
    # tangent plane at a reaches the midpoint column at z_a - s (na_x du/2 + na_y dv/2)/na_z
    zm_from_a = -s * (na[0] * du / 2 + na[1] * dv / 2) / na[2]
    zm_from_b = s * (nb[0] * du / 2 + nb[1] * dv / 2) / nb[2]
    return True, zm_from_b - zm_from_a, na[2] ** 2, nb[2] ** 2


def neighbour_pairs(H, W, connectivity=4):
    for v in range(H):
        for u in range(W):
            if u + 1 < W:
                yield (u, v), (u + 1, v)
            if v + 1 < H:
                yield (u, v), (u, v + 1)
            if connectivity == 8 and v + 1 < H:
                if u + 1 < W:
                    yield (u, v), (u + 1, v + 1)
                if u >= 1:
                    yield (u, v), (u - 1, v + 1)


def closure_labels(H, W, valid, linked):
    """Labels by transitive closure of the boolean adjacency (Warshall);
    label = rank of the component's smallest raster index."""
    N = H * W
    R = np.eye(N, dtype=bool)
    for (a, b) in linked:
        ia, ib = a[1] * W + a[0], b[1] * W + b[0]
        R[ia, ib] = R[ib, ia] = True
    for k in range(N):
        R |= R[:, k:k + 1] & R[k:k + 1, :]
    lab = -np.ones(N, dtype=np.int64)
    roots = []
    for p in range(N):
        if valid.ravel()[p]:
            root = int(np.flatnonzero(R[p] & valid.ravel())[0])
            roots.append(root)
            lab[p] = root
    uniq = sorted(set(roots))
    rank = {r: i for i, r in enumerate(uniq)}
    out = np.array([rank[x] if x >= 0 else -1 for x in lab]).reshape(H, W)
    return out, len(uniq)


def model(normals, mask, cam, theta_c_deg, connectivity=4):
    H, W, _ = normals.shape
    valid = np.asarray(mask) != 0
    usable, similar = [], []
    info = {}
    for a, b in neighbour_pairs(H, W, connectivity):
        if not (valid[a[1], a[0]] and valid[b[1], b[0]]):
            continue
        ok, om, g2a, g2b = pair_model(normals, cam, a, b)
        if not ok:
            continue
        usable.append((a, b))
        info[(a, b)] = (om, g2a, g2b)
        na = normals[a[1], a[0]].astype(np.float64)
        nb = normals[b[1], b[0]].astype(np.float64)
        if theta_c_deg > 0:
            ang = math.degrees(math.acos(max(-1.0, min(1.0, float(na @ nb)))))
            if ang < theta_c_deg:
                similar.append((a, b))
    return valid, usable, similar, info


def fill_rows(normals, mask, cam, lab, info):
    """Eq. 14-15 per component with explicit rows: for every usable edge
    inside a component, rows b->a (+1 at a, -1 at b, rhs omega_{b->a}) and
    a->b (+1 at b, -1 at a, rhs -omega_{b->a}), weights gamma^2/2.  Dense
    minimum-norm weighted least squares (zero mean per component)."""
    H, W = lab.shape
    z = np.zeros((H, W))
    for c in range(int(lab.max()) + 1 if lab.max() >= 0 else 0):
        pix = [(u, v) for v in range(H) for u in range(W) if lab[v, u] == c]
        col = {p: i for i, p in enumerate(pix)}
        rows, rhs, wts = [], [], []
        for (a, b), (om, g2a, g2b) in info.items():
            if a in col and b in col:
                r1 = np.zeros(len(pix)); r1[col[a]] = 1; r1[col[b]] = -1
                rows.append(r1); rhs.append(om); wts.append(0.5 * g2a)
                rows.append(-r1); rhs.append(-om); wts.append(0.5 * g2b)
        if not rows:
            continue
        sw = np.sqrt(np.array(wts))
        A = np.array(rows) * sw[:, None]
        x = np.linalg.lstsq(A, np.array(rhs) * sw, rcond=None)[0]
        x -= x.mean()
        for p, i in col.items():
            z[p[1], p[0]] = x[i]
    return z


def _sig(x, k):
    if -k * x > 700:
        return 0.0
    return 1.0 / (1.0 + math.exp(-k * x))


def _wout(chi, L, U, mode):
    chi = abs(chi)
    if mode == 0:
        return 1.0
    if mode == 2:
        return 1.0 if chi < U else 0.0
    if chi == 0:
        return 1.0
    lL, lU = math.log10(L), math.log10(U)
    arg = 4.0 / (lL - lU) * (2.0 * math.log10(chi) - (lL + lU))
    if -arg > 700:
        return 0.0
    return 1.0 / (1.0 + math.exp(-arg))


def irls_rows(normals, mask, cam, lab, K, zfill, usable, info, params):
    """Alg. 1's relative-scale loop with explicit inter-component rows.

    Row b->a of inter edge (a, b): +1 at pi(a), -1 at pi(b),
    rhs omega_{b->a} - (z_a - z_b) (Eq. 16); its weight is 1 in the
    alignment iterations and gamma_{b->a}^2 sigma_k(gamma^2 ((z_{-b}-z_a)^2 -
    (z_b-z_a)^2)) W^out otherwise, with -b the pixel across a from b.
    No relative weight cut: a row is dropped only when its weight is exactly
    zero (FP64 underflow).  Returns (S, energies)."""
    H, W = lab.shape
    usable_set = set(usable)
    inter = [(a, b) for (a, b) in usable if lab[a[1], a[0]] != lab[b[1], b[0]]]
    return _irls_loop(lab, K, zfill, inter, lambda a, b: info[(a, b)],
                      lambda p, q: (p, q) in usable_set or (q, p) in usable_set, params)


def irls_exact(normals, mask, cam, lab, K, zfill, params):
    """The same loop on a map of any size: the inter-component pairs are
    found from the labels and only their pair models (and those of the
    pairs across each end) are evaluated, one scalar pair at a time."""
    lab = np.asarray(lab)
    H, W = lab.shape
    valid = np.asarray(mask) != 0
    cache = {}

    def pm(a, b):
        if (a, b) not in cache:
            ok = valid[a[1], a[0]] and valid[b[1], b[0]]
            cache[(a, b)] = pair_model(normals, cam, a, b) if ok else (False, 0.0, 0.0, 0.0)
        return cache[(a, b)]

    inter = []
    vs, us = np.nonzero((lab[:, :-1] != lab[:, 1:]) & valid[:, :-1] & valid[:, 1:])
    for v, u in zip(vs.tolist(), us.tolist()):
        if pm((u, v), (u + 1, v))[0]:
            inter.append(((u, v), (u + 1, v)))
    vs, us = np.nonzero((lab[:-1, :] != lab[1:, :]) & valid[:-1, :] & valid[1:, :])
    for v, u in zip(vs.tolist(), us.tolist()):
        if pm((u, v), (u, v + 1))[0]:
            inter.append(((u, v), (u, v + 1)))

    def info(a, b):
        return pm(a, b)[1:]

    def edge_ok(p, q):
        if (p[1], p[0]) > (q[1], q[0]):
            p, q = q, p
        return pm(p, q)[0]

    return _irls_loop(lab, K, zfill, inter, info, edge_ok, params)


def _solve_pieces(N, rhs, K, rows_c, rows_d, keep):
    """Minimum-norm solution of the normal equations N s = rhs of a graph
    Laplacian: connected pieces over the kept rows by a breadth-first walk,
    one node pinned per piece, a dense solve of the rest, zero mean per piece."""
    adj = [[] for _ in range(K)]
    for c, d, k in zip(rows_c, rows_d, keep):
        if k:
            adj[c].append(d)
            adj[d].append(c)
    seen = np.zeros(K, bool)
    s = np.zeros(K)
    Nd = N.tocsr()
    for root in range(K):
        if seen[root]:
            continue
        piece, stack = [], [root]
        seen[root] = True
        while stack:
            x = stack.pop()
            piece.append(x)
            for y in adj[x]:
                if not seen[y]:
                    seen[y] = True
                    stack.append(y)
        piece.sort()
        if len(piece) < 2:
            continue
        free = piece[1:]
        M = Nd[free][:, free].toarray()
        s[free] = np.linalg.solve(M, rhs[free])
        s[piece] -= s[piece].mean()
    return s


def _irls_loop(lab, K, zfill, inter, info, edge_ok, params):
    import scipy.sparse as sp
    H, W = lab.shape
    S = np.zeros(K)
    energies = []
    k = params["bini_k"]

    def zval(p):
        return zfill[p[1], p[0]] + S[lab[p[1], p[0]]]

    cidx = np.array([lab[a[1], a[0]] for (a, b) in inter], dtype=np.int64)
    didx = np.array([lab[b[1], b[0]] for (a, b) in inter], dtype=np.int64)
    n = len(inter)
    # stacked directed rows: 2i = row b->a (+1 at pi(a)), 2i+1 = row a->b (+1 at pi(b))
    ridx = np.repeat(np.arange(2 * n), 2)
    cols = np.empty(4 * n, dtype=np.int64)
    vals = np.empty(4 * n)
    cols[0::4], vals[0::4] = cidx, 1.0
    cols[1::4], vals[1::4] = didx, -1.0
    cols[2::4], vals[2::4] = didx, 1.0
    cols[3::4], vals[3::4] = cidx, -1.0
    A = sp.csr_matrix((vals, (ridx, cols)), shape=(2 * n, max(K, 1)))
    for t in range(params["irls_iters"]):
        if n == 0:
            energies.append(0.0)
            continue
        wts = np.empty(2 * n)
        rhs = np.empty(2 * n)
        for i, (a, b) in enumerate(inter):
            om, g2a, g2b = info(a, b)
            za, zb = zval(a), zval(b)
            chi = za - zb - om
            if t < params["align_iters"]:
                wba = wab = 1.0
            else:
                d = (b[0] - a[0], b[1] - a[1])
                mb = (a[0] - d[0], a[1] - d[1])          # across a from b
                ma = (b[0] + d[0], b[1] + d[1])          # across b from a
                dm = (zval(mb) - za) if (0 <= mb[0] < W and 0 <= mb[1] < H and edge_ok(mb, a)) else 0.0
                dm2 = (zval(ma) - zb) if (0 <= ma[0] < W and 0 <= ma[1] < H and edge_ok(b, ma)) else 0.0
                wo = _wout(chi, params["out_L"], params["out_U"], params["outlier_mode"])
                wba = g2a * _sig(g2a * (dm * dm - (zb - za) ** 2), k) * wo
                wab = g2b * _sig(g2b * (dm2 * dm2 - (za - zb) ** 2), k) * wo
            wts[2 * i], rhs[2 * i] = wba, om - (za - zb)
            wts[2 * i + 1], rhs[2 * i + 1] = wab, -om - (zb - za)
        keep = (wts[0::2] + wts[1::2]) > 0
        Wd = sp.diags(wts)
        N = (A.T @ Wd @ A)
        s = _solve_pieces(N, A.T @ (wts * rhs), K, cidx, didx, keep)
        res = A @ s - rhs
        energies.append(float(np.sum(wts * res * res)))
        S = S + s
    return S, energies


def irls_merging(normals, mask, cam, lab, K, zfill, params):
    """Alg. 1's loop with the optional merging of Sec. 3.5, written
    independently of the oracle: the state is the current log-depth of
    every pixel and the current (merged) label of every pixel; every step
    rebuilds the inter-component rows from the current labels, solves them
    per connected piece, and adds each component's increment to its pixels;
    every freq_merging-th step each current component picks its boundary
    edge of smallest |z_a - z_b - omega| counted in units of 2^-40 (equal
    counts: smaller code 4 a + dir, dir 0 right, 1 down, 2 down-right, 3
    down-left, a the raster index of the upper / left pixel), and
    the components joined by picked edges are relabelled as one (pixel
    labels rewritten through a plain union-find).  Returns the final
    log-depth [H, W] (0 off the labels) and the energies."""
    import scipy.sparse as sp
    lab = np.asarray(lab)
    H, W = lab.shape
    valid = np.asarray(mask) != 0
    cache = {}

    def pm(a, b):
        if (a, b) not in cache:
            ok = valid[a[1], a[0]] and valid[b[1], b[0]]
            cache[(a, b)] = pair_model(normals, cam, a, b) if ok else (False, 0.0, 0.0, 0.0)
        return cache[(a, b)]

    pairs = []
    for v in range(H):
        for u in range(W):
            if lab[v, u] < 0:
                continue
            dirs = ((1, 0), (0, 1), (1, 1), (-1, 1)) if params.get("connectivity", 4) == 8 else ((1, 0), (0, 1))
            for k, (du, dv) in enumerate(dirs):
                b = (u + du, v + dv)
                if 0 <= b[0] < W and b[1] < H and lab[b[1], b[0]] >= 0 and pm((u, v), b)[0]:
                    pairs.append(((u, v), b, 4 * (v * W + u) + k))
    usable = set((a, b) for a, b, _ in pairs)

    def edge_ok(p, q):
        return (p, q) in usable or (q, p) in usable

    z = np.where(lab >= 0, np.asarray(zfill, dtype=np.float64), 0.0)
    cl = lab.copy()
    k = params["bini_k"]
    freq = int(params.get("freq_merging", 0))
    T = int(params["irls_iters"])
    energies = []
    for t in range(T):
        inter = [(a, b, code) for (a, b, code) in pairs if cl[a[1], a[0]] != cl[b[1], b[0]]]
        Kc = int(cl.max()) + 1
        n = len(inter)
        if n:
            cidx = np.array([cl[a[1], a[0]] for a, b, _ in inter])
            didx = np.array([cl[b[1], b[0]] for a, b, _ in inter])
            ridx = np.repeat(np.arange(2 * n), 2)
            cols = np.empty(4 * n, dtype=np.int64)
            vals = np.empty(4 * n)
            cols[0::4], vals[0::4] = cidx, 1.0
            cols[1::4], vals[1::4] = didx, -1.0
            cols[2::4], vals[2::4] = didx, 1.0
            cols[3::4], vals[3::4] = cidx, -1.0
            A = sp.csr_matrix((vals, (ridx, cols)), shape=(2 * n, Kc))
            wts = np.empty(2 * n)
            rhs = np.empty(2 * n)
            for i, (a, b, _) in enumerate(inter):
                _, om, g2a, g2b = pm(a, b)
                za, zb = z[a[1], a[0]], z[b[1], b[0]]
                chi = za - zb - om
                if t < params["align_iters"]:
                    wba = wab = 1.0
                else:
                    d = (b[0] - a[0], b[1] - a[1])
                    mb = (a[0] - d[0], a[1] - d[1])
                    ma = (b[0] + d[0], b[1] + d[1])
                    dm = (z[mb[1], mb[0]] - za) if (0 <= mb[0] < W and 0 <= mb[1] < H and edge_ok(mb, a)) else 0.0
                    dm2 = (z[ma[1], ma[0]] - zb) if (0 <= ma[0] < W and 0 <= ma[1] < H and edge_ok(b, ma)) else 0.0
                    wo = _wout(chi, params["out_L"], params["out_U"], params["outlier_mode"])
                    wba = g2a * _sig(g2a * (dm * dm - (zb - za) ** 2), k) * wo
                    wab = g2b * _sig(g2b * (dm2 * dm2 - (za - zb) ** 2), k) * wo
                wts[2 * i], rhs[2 * i] = wba, om - (za - zb)
                wts[2 * i + 1], rhs[2 * i + 1] = wab, -om - (zb - za)
            keep = (wts[0::2] + wts[1::2]) > 0
            N = A.T @ sp.diags(wts) @ A
            s = _solve_pieces(N, A.T @ (wts * rhs), Kc, cidx, didx, keep)
            energies.append(float(np.sum(wts * (A @ s - rhs) ** 2)))
            z = np.where(cl >= 0, z + s[np.maximum(cl, 0)], 0.0)
        else:
            energies.append(0.0)
        if freq > 0 and (t + 1) % freq == 0 and t + 1 < T and n:
            pick = {}
            for a, b, code in inter:
                mag = math.floor(abs(z[a[1], a[0]] - z[b[1], b[0]] - pm(a, b)[1]) * 2.0 ** 40)
                for c in (cl[a[1], a[0]], cl[b[1], b[0]]):
                    if c not in pick or (mag, code) < pick[c][0]:
                        pick[c] = ((mag, code), cl[a[1], a[0]], cl[b[1], b[0]])
            parent = list(range(Kc))

            def find(x):
                while parent[x] != x:
                    parent[x] = parent[parent[x]]
                    x = parent[x]
                return x

            for _, c, d in pick.values():
                rc, rd = find(c), find(d)
                if rc != rd:
                    parent[max(rc, rd)] = min(rc, rd)
            roots = sorted(set(find(c) for c in range(Kc)))
            newid = {r: i for i, r in enumerate(roots)}
            cl = np.where(cl >= 0, np.vectorize(lambda c: newid[find(int(c))])(np.maximum(cl, 0)), -1)
    return z, energies


def logdepth_irls(normals, mask, cam, params):
    """The pixel-level log-depth baseline (ND form), written directly: the
    unknown is the log-depth of every pixel, z = 0 to start; iteration t
    minimises sum over both directed rows of every usable pixel pair of
    W_{b->a} (z_a - z_b - omega_{b->a})^2 with W_{b->a} = g^2 sigma_k(g^2
    ((z_{-b} - z_a)^2 - (z_b - z_a)^2)) at the previous z, times the outlier
    weight of the previous residual from the second iteration on; the new z
    is the minimum-norm solution per connected piece.  Returns (z [H, W],
    energies)."""
    import scipy.sparse as sp
    mask = np.asarray(mask)
    H, W = mask.shape
    valid = mask != 0
    cache = {}

    def pm(a, b):
        if (a, b) not in cache:
            ok = valid[a[1], a[0]] and valid[b[1], b[0]]
            cache[(a, b)] = pair_model(normals, cam, a, b) if ok else (False, 0.0, 0.0, 0.0)
        return cache[(a, b)]

    pix = {}
    for v in range(H):
        for u in range(W):
            if valid[v, u]:
                pix[(u, v)] = len(pix)
    pairs = []
    for (u, v) in pix:
        dirs = ((1, 0), (0, 1), (1, 1), (-1, 1)) if params.get("connectivity", 4) == 8 else ((1, 0), (0, 1))
        for (du, dv) in dirs:
            b = (u + du, v + dv)
            if b in pix and pm((u, v), b)[0]:
                pairs.append(((u, v), b))
    usable = set(pairs)

    def edge_ok(p, q):
        return (p, q) in usable or (q, p) in usable

    n, N = len(pairs), len(pix)
    ci = np.array([pix[a] for a, _ in pairs], dtype=np.int64)
    di = np.array([pix[b] for _, b in pairs], dtype=np.int64)
    ridx = np.repeat(np.arange(2 * n), 2)
    cols = np.empty(4 * n, dtype=np.int64)
    vals = np.empty(4 * n)
    cols[0::4], vals[0::4] = ci, 1.0
    cols[1::4], vals[1::4] = di, -1.0
    cols[2::4], vals[2::4] = di, 1.0
    cols[3::4], vals[3::4] = ci, -1.0
    A = sp.csr_matrix((vals, (ridx, cols)), shape=(2 * n, max(N, 1)))
    z = np.zeros(N)
    k = params["bini_k"]
    energies = []

    def zv(p):
        return z[pix[p]]

    for t in range(int(params["irls_iters"])):
        if n == 0:
            energies.append(0.0)
            continue
        wts = np.empty(2 * n)
        rhs = np.empty(2 * n)
        for i, (a, b) in enumerate(pairs):
            _, om, g2a, g2b = pm(a, b)
            za, zb = zv(a), zv(b)
            d = (b[0] - a[0], b[1] - a[1])
            mb = (a[0] - d[0], a[1] - d[1])
            ma = (b[0] + d[0], b[1] + d[1])
            dm = (zv(mb) - za) if (mb in pix and edge_ok(mb, a)) else 0.0
            dm2 = (zv(ma) - zb) if (ma in pix and edge_ok(b, ma)) else 0.0
            wo = _wout(za - zb - om, params["out_L"], params["out_U"], params["outlier_mode"]) if t >= 1 else 1.0
            wts[2 * i] = g2a * _sig(g2a * (dm * dm - (zb - za) ** 2), k) * wo
            wts[2 * i + 1] = g2b * _sig(g2b * (dm2 * dm2 - (za - zb) ** 2), k) * wo
            rhs[2 * i], rhs[2 * i + 1] = om, -om
        keep = (wts[0::2] + wts[1::2]) > 0
        Nm = A.T @ sp.diags(wts) @ A
        znew = _solve_pieces(Nm, A.T @ (wts * rhs), N, ci, di, keep)
        energies.append(float(np.sum(wts * (A @ znew - rhs) ** 2)))
        z = znew
    out = np.zeros((H, W))
    for (u, v), i in pix.items():
        out[v, u] = z[i]
    return out, energies
