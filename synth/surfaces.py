"""Seeded synthetic normal maps shaped like the paper's workloads.

This module only *draws inputs*: analytic depth fields (plane + Gaussian
bumps + line/circle depth steps), masks, cameras, and the normals obtained
from central differences of the 3-D point map.  It contains none of the
integration method's arithmetic (no edge models, weights or solves), so
both the FP64 oracle and the HIP path can consume its output.

Normal orientation: every normal faces the camera (n . tau < 0, with
tau = ((u-cx)/fx, (v-cy)/fy, 1) in perspective and tau = (0, 0, 1) in
orthographic mode).  Pixel (u, v) = (column, row) has its centre at the
integer coordinates; the raster index is v*W + u.

Workload shapes (pixel counts, focal lengths, numbers of steps and bumps)
follow the resolutions the paper reports for its object-level and
large-scale maps (Sec. 4, Fig. 5); the concrete recipes are:

  c1  64x64 orthographic, tilted plane + 2 bumps + a circular step, disk mask
  c2  512x512 perspective f=600, 5 steps, 6 bumps, ~45 % blob mask
  c3  2048x2048 perspective f=2400, 40 steps, 60 bumps, ~70 % blob mask
  c5  4096x4096 perspective f=4800, 150 steps, 240 bumps, ~72 % blob mask
  patch  256x256 crops of c3-style scenes (training data for the warm start)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage


@dataclass
class Camera:
    proj: str  # "ortho" or "persp"
    fx: float = 1.0
    fy: float = 1.0
    cx: float = 0.0
    cy: float = 0.0
    pixel_pitch: float = 1.0

    def as_dict(self):
        return dict(proj=self.proj, fx=self.fx, fy=self.fy, cx=self.cx,
                    cy=self.cy, pixel_pitch=self.pixel_pitch)


@dataclass
class Sample:
    normals: np.ndarray          # float32 [H, W, 3]
    mask: np.ndarray             # uint8 [H, W]
    depth_gt: np.ndarray         # float64 [H, W] (ground-truth depth)
    cam: Camera
    params: dict = field(default_factory=dict)   # method parameters of this workload
    name: str = ""


CONFIGS = {
    "c1": dict(H=64, W=64, proj="ortho", T=10),
    "c2": dict(H=512, W=512, proj="persp", f=600.0, steps=5, bumps=6,
               coverage=0.45, noise=0.005, T=15),
    "c3": dict(H=2048, W=2048, proj="persp", f=2400.0, steps=40, bumps=60,
               coverage=0.70, noise=0.005, T=15),
    "c5": dict(H=4096, W=4096, proj="persp", f=4800.0, steps=150, bumps=240,
               coverage=0.72, noise=0.01, T=15),
}


# ----------------------------------------------------------------------------
# analytic depth fields
# ----------------------------------------------------------------------------
class _Scene:
    """Analytic depth z(u, v) defined on the whole real plane."""

    def __init__(self):
        self.base = None          # callable(u, v) -> z
        self.bumps = []           # (A, uc, vc, sigma)
        self.lines = []           # (delta, u0, v0, cos, sin)
        self.circles = []         # (delta, uc, vc, r)
        self.zmin = None

    def __call__(self, u, v):
        z = self.base(u, v)
        for A, uc, vc, s in self.bumps:
            z = z + A * np.exp(-((u - uc) ** 2 + (v - vc) ** 2) / (2.0 * s * s))
        for d, u0, v0, c, s in self.lines:
            z = z + d * (((u - u0) * c + (v - v0) * s) > 0.0)
        for d, uc, vc, r in self.circles:
            z = z + d * (((u - uc) ** 2 + (v - vc) ** 2) < r * r)
        if self.zmin is not None:
            z = np.maximum(z, self.zmin)
        return z

    def grid(self, u0, v0, H, W, du=0.0, dv=0.0):
        """z at (u0 + j + du, v0 + i + dv) for i < H, j < W, evaluating each
        bump and circle only inside its support window (6 sigma / radius)
        and every half-plane step through one row-wise prefix sum."""
        u = u0 + np.arange(W, dtype=np.float64) + du
        v = v0 + np.arange(H, dtype=np.float64) + dv
        z = self.base(u[None, :], v[:, None]) + np.zeros((H, W))
        for A, uc, vc, sg in self.bumps:
            rad = 6.0 * sg
            j0, j1 = np.searchsorted(u, uc - rad), np.searchsorted(u, uc + rad, side="right")
            i0, i1 = np.searchsorted(v, vc - rad), np.searchsorted(v, vc + rad, side="right")
            if j0 < j1 and i0 < i1:
                gu = np.exp(-((u[j0:j1] - uc) ** 2) / (2.0 * sg * sg))
                gv = np.exp(-((v[i0:i1] - vc) ** 2) / (2.0 * sg * sg))
                z[i0:i1, j0:j1] += A * gv[:, None] * gu[None, :]
        if self.lines:
            diff = np.zeros((H, W + 1))
            for d, lu, lv, c, sn in self.lines:
                # (u - lu) c + (v - lv) sn > 0, solved for u row by row
                if c == 0.0:
                    on = ((v - lv) * sn) > 0.0
                    diff[on, 0] += d
                    diff[on, W] -= d
                    continue
                thr = lu - (v - lv) * sn / c
                if c > 0:
                    k = np.clip(np.searchsorted(u, thr, side="right"), 0, W)
                    diff[np.arange(H), k] += d
                    diff[:, W] -= d
                else:
                    k = np.clip(np.searchsorted(u, thr, side="left"), 0, W)
                    diff[:, 0] += d
                    diff[np.arange(H), k] -= d
            z += np.cumsum(diff, axis=1)[:, :W]
        for d, uc, vc, r in self.circles:
            j0, j1 = np.searchsorted(u, uc - r), np.searchsorted(u, uc + r, side="right")
            i0, i1 = np.searchsorted(v, vc - r), np.searchsorted(v, vc + r, side="right")
            if j0 < j1 and i0 < i1:
                inside = ((u[None, j0:j1] - uc) ** 2 + (v[i0:i1, None] - vc) ** 2) < r * r
                z[i0:i1, j0:j1] += d * inside
        if self.zmin is not None:
            z = np.maximum(z, self.zmin)
        return z


def _blob_mask(rng, H, W, coverage):
    """Gaussian-smoothed white noise (correlation length W/16) thresholded at
    the coverage quantile.  The field is drawn on a grid 8x coarser and
    bilinearly upsampled, which keeps 4096^2 masks cheap."""
    f = 8
    h, w = max(H // f, 4), max(W // f, 4)
    noise = rng.standard_normal((h, w))
    sm = ndimage.gaussian_filter(noise, sigma=max(W / 16.0 / f, 1.0), mode="wrap")
    up = ndimage.zoom(sm, (H / h, W / w), order=1, mode="grid-wrap", grid_mode=True)
    up = up[:H, :W]
    thr = np.quantile(up, 1.0 - coverage)
    return (up > thr).astype(np.uint8)


def _ortho_normals(z_fn, H, W, pitch):
    u = np.arange(W, dtype=np.float64)[None, :]
    v = np.arange(H, dtype=np.float64)[:, None]
    zu = (z_fn(u + 1, v) - z_fn(u - 1, v)) / (2.0 * pitch)
    zv = (z_fn(u, v + 1) - z_fn(u, v - 1)) / (2.0 * pitch)
    n = np.stack([zu, zv, -np.ones_like(zu)], axis=-1)  # faces the camera (n_z < 0)
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


def _persp_points(z_fn, u, v, cam):
    z = z_fn(u, v)
    return np.stack([z * (u - cam.cx) / cam.fx, z * (v - cam.cy) / cam.fy, z], axis=-1)


def _persp_normals(z_fn, H, W, cam, u0=0, v0=0):
    u = np.arange(u0, u0 + W, dtype=np.float64)[None, :] + np.zeros((H, 1))
    v = np.arange(v0, v0 + H, dtype=np.float64)[:, None] + np.zeros((1, W))
    if isinstance(z_fn, _Scene):
        def pts(a, b):
            z = z_fn.grid(u0, v0, H, W, a, b)
            return np.stack([z * (u + a - cam.cx) / cam.fx, z * (v + b - cam.cy) / cam.fy, z], axis=-1)
        du = pts(1.0, 0.0) - pts(-1.0, 0.0)
        dv = pts(0.0, 1.0) - pts(0.0, -1.0)
    else:
        du = _persp_points(z_fn, u + 1, v, cam) - _persp_points(z_fn, u - 1, v, cam)
        dv = _persp_points(z_fn, u, v + 1, cam) - _persp_points(z_fn, u, v - 1, cam)
    n = np.cross(du, dv)
    tau = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones_like(u)], axis=-1)
    s = np.sign(np.sum(n * tau, axis=-1, keepdims=True))
    s[s == 0] = 1.0
    n = -s * n
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


def _add_noise(rng, n, sigma):
    if sigma > 0:
        n = n + rng.normal(0.0, sigma, size=n.shape)
        n = n / np.linalg.norm(n, axis=-1, keepdims=True)
    return n


def _uniform_in_mask(rng, mask, k):
    idx = np.flatnonzero(mask)
    pick = rng.choice(idx, size=k, replace=True)
    W = mask.shape[1]
    return (pick % W).astype(np.float64) + rng.uniform(-0.5, 0.5, k), \
           (pick // W).astype(np.float64) + rng.uniform(-0.5, 0.5, k)


# ----------------------------------------------------------------------------
# configuration c1: 64x64 orthographic
# ----------------------------------------------------------------------------
def make_c1(seed: int, noise: float = 0.01) -> Sample:
    rng = np.random.default_rng([1, seed])
    H = W = 64
    cx = cy = (W - 1) / 2.0
    uu = np.arange(W)[None, :]
    vv = np.arange(H)[:, None]
    mask = (((uu - cx) ** 2 + (vv - cy) ** 2) <= 30.0 ** 2).astype(np.uint8)
    sc = _Scene()
    phi = rng.uniform(0, 2 * math.pi)
    g = math.tan(math.radians(10.0))
    sc.base = lambda u, v: 10.0 + g * (math.cos(phi) * (u - cx) + math.sin(phi) * (v - cy))
    bu, bv = _uniform_in_mask(rng, mask, 2)
    sc.bumps = [(0.3, bu[i], bv[i], 8.0) for i in range(2)]
    rr = 18.0 * math.sqrt(rng.uniform())
    aa = rng.uniform(0, 2 * math.pi)
    sc.circles = [(0.2, cx + rr * math.cos(aa), cy + rr * math.sin(aa), 12.0)]
    n = _ortho_normals(sc, H, W, 1.0)
    n = _add_noise(rng, n, noise)
    u = np.arange(W, dtype=np.float64)[None, :] + np.zeros((H, 1))
    v = np.arange(H, dtype=np.float64)[:, None] + np.zeros((1, W))
    z = sc(u, v)
    cam = Camera("ortho", pixel_pitch=1.0)
    return Sample(n.astype(np.float32), mask, z, cam,
                  params=dict(theta_c_deg=2.0, irls_iters=10), name=f"c1/s{seed}")


def make_ortho(seed: int, H: int = 384, W: int = 384, noise: float = 0.01) -> Sample:
    """A larger orthographic map in the style of c1: tilted plane, Gaussian
    bumps and circular steps over a blob mask (55%), pixel pitch 1."""
    rng = np.random.default_rng([7, seed])
    mask = _blob_mask(rng, H, W, 0.55)
    sc = _Scene()
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    phi = rng.uniform(0, 2 * math.pi)
    g = math.tan(math.radians(10.0))
    sc.base = lambda u, v: 10.0 + g * (math.cos(phi) * (u - cx) + math.sin(phi) * (v - cy))
    bu, bv = _uniform_in_mask(rng, mask, 8)
    sc.bumps = [(rng.uniform(0.5, 3.0) * rng.choice([-1.0, 1.0]), bu[i], bv[i], rng.uniform(6.0, 30.0))
                for i in range(8)]
    cu, cv = _uniform_in_mask(rng, mask, 4)
    sc.circles = [(rng.uniform(0.2, 1.0), cu[i], cv[i], rng.uniform(10.0, 60.0)) for i in range(4)]
    n = _ortho_normals(sc, H, W, 1.0)
    n = _add_noise(rng, n, noise)
    z = sc.grid(0, 0, H, W)
    cam = Camera("ortho", pixel_pitch=1.0)
    return Sample(n.astype(np.float32), mask, z, cam,
                  params=dict(theta_c_deg=2.0, irls_iters=10), name=f"ortho{H}/s{seed}")


# ----------------------------------------------------------------------------
# perspective configurations
# ----------------------------------------------------------------------------
def _persp_scene(rng, H, W, n_steps, n_bumps, mask, bump_sigma=(4.0, 64.0)):
    sc = _Scene()
    cxi, cyi = (W - 1) / 2.0, (H - 1) / 2.0
    phi = rng.uniform(0, 2 * math.pi)
    R = 0.5 * math.hypot(W, H)
    c, s = math.cos(phi), math.sin(phi)
    # 1/z affine in (u, v): a plane in 3-D spanning depth 2 .. 3 over the image
    sc.base = lambda u, v: 1.0 / (0.5 + (1.0 / 3.0 - 0.5) * 0.5 * (1.0 + ((u - cxi) * c + (v - cyi) * s) / R))
    bu, bv = _uniform_in_mask(rng, mask, n_bumps)
    lo, hi = math.log(bump_sigma[0]), math.log(bump_sigma[1])
    for i in range(n_bumps):
        A = rng.uniform(0.02, 0.1) * rng.choice([-1.0, 1.0])
        sig = math.exp(rng.uniform(lo, hi))
        sc.bumps.append((A, bu[i], bv[i], sig))
    rlo, rhi = math.log(W / 64.0), math.log(W / 4.0)
    for _ in range(n_steps):
        d = rng.uniform(0.05, 0.3) * rng.choice([-1.0, 1.0])
        if rng.uniform() < 0.5:
            a = rng.uniform(0, 2 * math.pi)
            sc.lines.append((d, rng.uniform(0, W), rng.uniform(0, H), math.cos(a), math.sin(a)))
        else:
            sc.circles.append((d, rng.uniform(0, W), rng.uniform(0, H), math.exp(rng.uniform(rlo, rhi))))
    sc.zmin = 1.0
    return sc


def make_persp(name: str, seed: int) -> Sample:
    cfg = CONFIGS[name]
    H, W, f = cfg["H"], cfg["W"], cfg["f"]
    rng = np.random.default_rng([int(name[1:]), seed])
    mask = _blob_mask(rng, H, W, cfg["coverage"])
    sc = _persp_scene(rng, H, W, cfg["steps"], cfg["bumps"], mask)
    cam = Camera("persp", fx=f, fy=f, cx=(W - 1) / 2.0, cy=(H - 1) / 2.0)
    n = _persp_normals(sc, H, W, cam)
    n = _add_noise(rng, n, cfg["noise"])
    z = sc.grid(0, 0, H, W)
    return Sample(n.astype(np.float32), mask, z, cam,
                  params=dict(theta_c_deg=2.0, irls_iters=cfg["T"]), name=f"{name}/s{seed}")


def make_patch(seed: int, size: int = 256) -> Sample:
    """A size x size crop of a c3-style scene (f=2400 on a 2048^2 sensor).

    The crop keeps the full sensor's intrinsics by shifting the principal
    point, so the rays are those of the crop's pixels in the big image."""
    cfg = CONFIGS["c3"]
    Hf, Wf, f = cfg["H"], cfg["W"], cfg["f"]
    rng = np.random.default_rng([7, seed])
    u0 = int(rng.integers(0, Wf - size))
    v0 = int(rng.integers(0, Hf - size))
    # scene parameters are drawn for the full sensor; bump centres uniform in it
    full = np.ones((8, 8), np.uint8)
    sc = _persp_scene(rng, Hf, Wf, cfg["steps"], cfg["bumps"], full)
    # rescale bump centres from the 8x8 proxy grid to the sensor
    sc.bumps = [(A, uc * Wf / 8.0, vc * Hf / 8.0, s) for (A, uc, vc, s) in sc.bumps]
    cov = rng.uniform(0.5, 1.0)
    mask = _blob_mask(rng, size, size, cov)
    cam_full = Camera("persp", fx=f, fy=f, cx=(Wf - 1) / 2.0, cy=(Hf - 1) / 2.0)
    n = _persp_normals(sc, size, size, cam_full, u0=u0, v0=v0)
    n = _add_noise(rng, n, cfg["noise"])
    cam = Camera("persp", fx=f, fy=f, cx=(Wf - 1) / 2.0 - u0, cy=(Hf - 1) / 2.0 - v0)
    z = sc.grid(u0, v0, size, size)
    return Sample(n.astype(np.float32), mask, z, cam,
                  params=dict(theta_c_deg=2.0, irls_iters=15), name=f"patch/s{seed}")


def make(name: str, seed: int = 0) -> Sample:
    if name == "c1":
        return make_c1(seed)
    if name in ("c2", "c3", "c5"):
        return make_persp(name, seed)
    if name == "patch":
        return make_patch(seed)
    raise ValueError(f"unknown workload {name!r}")


# ----------------------------------------------------------------------------
# closed-form surfaces used to pin the oracle
# ----------------------------------------------------------------------------
def plane_persp(H, W, f, normal, dist, seed_noise=None):
    """Constant-normal plane {X : n.X = -dist} seen by a pinhole camera.

    Every pixel sees the same normal; depth along the ray is
    z = -dist / (n . tau)."""
    cam = Camera("persp", fx=f, fy=f, cx=(W - 1) / 2.0, cy=(H - 1) / 2.0)
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    u = np.arange(W, dtype=np.float64)[None, :] + np.zeros((H, 1))
    v = np.arange(H, dtype=np.float64)[:, None] + np.zeros((1, W))
    ntau = n[0] * (u - cam.cx) / f + n[1] * (v - cam.cy) / f + n[2]
    z = -dist / ntau
    nm = np.broadcast_to(n, (H, W, 3)).astype(np.float32).copy()
    return nm, np.ones((H, W), np.uint8), z, cam


def quadric_ortho(H, W, coef, pitch=1.0):
    """z = a u^2 + b u v + c v^2 + d u + e v + g (u, v in pitch units) with
    normals from central differences, which are exact for quadratics."""
    a, b, c, d, e, g = coef

    def zf(u, v):
        x, y = u * pitch, v * pitch
        return a * x * x + b * x * y + c * y * y + d * x + e * y + g

    n = _ortho_normals(zf, H, W, pitch)
    u = np.arange(W, dtype=np.float64)[None, :] + np.zeros((H, 1))
    v = np.arange(H, dtype=np.float64)[:, None] + np.zeros((1, W))
    return n, np.ones((H, W), np.uint8), zf(u, v), Camera("ortho", pixel_pitch=pitch)


def sphere_persp(H, W, f, radius, centre_depth):
    """Sphere of the given radius centred on the optical axis, with exact
    normals (X - C)/r evaluated on the ray intersections; mask = hit pixels."""
    cam = Camera("persp", fx=f, fy=f, cx=(W - 1) / 2.0, cy=(H - 1) / 2.0)
    u = np.arange(W, dtype=np.float64)[None, :] + np.zeros((H, 1))
    v = np.arange(H, dtype=np.float64)[:, None] + np.zeros((1, W))
    tau = np.stack([(u - cam.cx) / f, (v - cam.cy) / f, np.ones_like(u)], -1)
    C = np.array([0.0, 0.0, centre_depth])
    # |z tau - C|^2 = r^2 -> (tau.tau) z^2 - 2 (tau.C) z + C.C - r^2 = 0
    A = np.sum(tau * tau, -1)
    B = -2.0 * tau @ C
    Cc = C @ C - radius * radius
    disc = B * B - 4 * A * Cc
    hit = disc > 0
    z = np.where(hit, (-B - np.sqrt(np.maximum(disc, 0))) / (2 * A), np.nan)
    P = z[..., None] * tau
    n = (P - C) / radius
    n = np.where(hit[..., None], n, np.array([0.0, 0.0, -1.0]))
    return n, hit.astype(np.uint8), z, cam


def tiny(seed: int, H: int = 9, W: int = 11, proj: str = "persp", noise: float = 0.01,
         step: float = 0.25) -> Sample:
    """A small piecewise-smooth map (plane + one bump + one circular step,
    a random mask with holes) for brute-force comparisons."""
    rng = np.random.default_rng([99, seed])
    sc = _Scene()
    gu, gv = rng.uniform(-0.05, 0.05, 2)
    z0 = 2.5
    sc.base = lambda u, v: z0 + gu * u + gv * v
    sc.bumps = [(rng.uniform(0.05, 0.15) * rng.choice([-1, 1]), rng.uniform(0, W),
                 rng.uniform(0, H), rng.uniform(1.5, 3.0))]
    sc.circles = [(step, rng.uniform(0, W), rng.uniform(0, H), rng.uniform(2.0, 4.0))]
    mask = (rng.uniform(size=(H, W)) > 0.12).astype(np.uint8)
    if proj == "persp":
        f = 12.0
        cam = Camera("persp", fx=f, fy=f * 1.1, cx=(W - 1) / 2.0 + 0.3, cy=(H - 1) / 2.0 - 0.2)
        n = _persp_normals(sc, H, W, cam)
    else:
        cam = Camera("ortho", pixel_pitch=0.5)
        n = _ortho_normals(sc, H, W, 0.5)
    n = _add_noise(rng, n, noise)
    u = np.arange(W, dtype=np.float64)[None, :] + np.zeros((H, 1))
    v = np.arange(H, dtype=np.float64)[:, None] + np.zeros((1, W))
    return Sample(n.astype(np.float32), mask, sc(u, v), cam,
                  params=dict(theta_c_deg=2.0, irls_iters=6), name=f"tiny/{proj}/s{seed}")
