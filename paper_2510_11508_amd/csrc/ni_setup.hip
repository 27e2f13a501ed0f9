// Edge setup (model of continuity, Sec. 3.1 / Eq. 3 and Eq. 7) and
// union-find connected components on the pixel grid (Sec. 3.3).
#include "ni_common.h"

namespace {

// FP64 arithmetic whose rounding must match the FP64 reference bit for bit:
// explicit round-to-nearest intrinsics, never contracted into FMAs.
__device__ __forceinline__ double mul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double add(double a, double b) { return __dadd_rn(a, b); }
// (nx*tx + ny*ty) + nz  -- n . tau with tau_z = 1
__device__ __forceinline__ double ndot(double nx, double ny, double nz, double tx, double ty) {
  return add(add(mul(nx, tx), mul(ny, ty)), nz);
}
__device__ __forceinline__ bool same_sign_nz(double a, double b) {
  return a != 0.0 && b != 0.0 && ((a > 0.0) == (b > 0.0));
}

// Model of continuity of one edge a -> b = a + (du, dv) of direction d
// (0 right, 1 down, 2 down-right, 3 down-left), in FP64 from the FP32
// normals.  Perspective (Eq. 3): the four dots d_aa = n_a.tau_a, d_am =
// n_a.tau_m, d_bb = n_b.tau_b, d_bm = n_b.tau_m, m the midpoint of the two
// pixel centres (for a diagonal the ray (u +- 1/2, v + 1/2)); the edge is
// usable iff (d_aa, d_am) and (d_bb, d_bm) are non-zero pairs of one sign,
// and omega = log((d_am/d_aa)*(d_bb/d_bm)).  Orthographic: usable iff n_az,
// n_bz != 0, omega = s*(n_a.(du,dv)/(2 n_az) + n_b.(du,dv)/(2 n_bz)).  On
// return *ta = d_aa and *tb = d_bb (n_az, n_bz orthographic): gamma = f * ta
// of the row ending at a (Eq. 7).
struct RayTabs {
  const double *tx, *ty, *txm, *tym;
};

__device__ __forceinline__ bool edge_model(const float* __restrict__ nrm, long long p, long long q, int u, int v,
                                           int d, int persp, double pitch, const RayTabs& T, double* om,
                                           double* ta, double* tb) {
  const double nax = nrm[3 * p], nay = nrm[3 * p + 1], naz = nrm[3 * p + 2];
  const double nbx = nrm[3 * q], nby = nrm[3 * q + 1], nbz = nrm[3 * q + 2];
  const int du = d == 1 ? 0 : d == 3 ? -1 : 1, dv = d == 0 ? 0 : 1;
  if (persp) {
    const double ub = T.tx[u + du], vb = T.ty[v + dv];
    const double um = du == 0 ? T.tx[u] : T.txm[du > 0 ? u : u - 1];
    const double vm = dv == 0 ? T.ty[v] : T.tym[v];
    const double daa = ndot(nax, nay, naz, T.tx[u], T.ty[v]);
    const double dam = ndot(nax, nay, naz, um, vm);
    const double dbb = ndot(nbx, nby, nbz, ub, vb);
    const double dbm = ndot(nbx, nby, nbz, um, vm);
    *ta = daa;
    *tb = dbb;
    if (!(same_sign_nz(daa, dam) && same_sign_nz(dbb, dbm))) return false;
    *om = log((dam / daa) * (dbb / dbm));
  } else {
    *ta = naz;
    *tb = nbz;
    if (!(naz != 0.0 && nbz != 0.0)) return false;
    // n . (du, dv) of each end
    const double ca = d == 0 ? nax : d == 1 ? nay : d == 2 ? nax + nay : -nax + nay;
    const double cb = d == 0 ? nbx : d == 1 ? nby : d == 2 ? nbx + nby : -nbx + nby;
    *om = pitch * (ca / (2.0 * naz) + cb / (2.0 * nbz));
  }
  return true;
}

__device__ __forceinline__ bool similar(const float* __restrict__ nrm, long long p, long long q, double cth) {
  const double nax = nrm[3 * p], nay = nrm[3 * p + 1], naz = nrm[3 * p + 2];
  const double nbx = nrm[3 * q], nby = nrm[3 * q + 1], nbz = nrm[3 * q + 2];
  return add(add(mul(nax, nbx), mul(nay, nby)), mul(naz, nbz)) > cth;
}

// One thread per pixel a; it owns the edges to its right and lower
// neighbours b (and with eb2 given, 8-connectivity, to its lower-right and
// lower-left ones).  Writes:
//   ebits[a]  EB_VALID | usable/similar bits of its axis edges
//   eb2[a]    usable/similar bits of its diagonal edges (if eb2)
//   om_*      omega_{b->a} (FP32, the fill's stencil precision), 0 where
//             unusable; om_r / om_d / om_dr / om_dl may be null
//   nt[a]     n_a . tau_a (perspective) or n_az (orthographic), FP32
// Similar iff usable and (n_ax n_bx + n_ay n_by) + n_az n_bz > cos(theta_c).
__global__ void __launch_bounds__(256) k_setup(
    const float* __restrict__ nrm, const uint8_t* __restrict__ mask, int H, int W, int persp,
    double pitch, RayTabs T, double cth, int use_sim,
    uint8_t* __restrict__ ebits, float* __restrict__ om_r, float* __restrict__ om_d,
    float* __restrict__ nt, int* __restrict__ err, uint8_t* __restrict__ eb2, float* __restrict__ om_dr,
    float* __restrict__ om_dl) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)H * W) return;
  const int u = (int)(p % W), v = (int)(p / W);
  uint8_t eb = 0, e2 = 0;
  float o[4] = {0.f, 0.f, 0.f, 0.f}, ntp = 0.f;
  if (mask[p]) {
    const float ax = nrm[3 * p], ay = nrm[3 * p + 1], az = nrm[3 * p + 2];
    if (!(isfinite(ax) && isfinite(ay) && isfinite(az))) atomicOr(err, 1);
    ntp = (float)(persp ? ndot((double)ax, (double)ay, (double)az, T.tx[u], T.ty[v]) : (double)az);
    eb = EB_VALID;
    const int nd = eb2 ? 4 : 2;
    for (int d = 0; d < nd; ++d) {
      const bool inside = d == 0 ? u + 1 < W : d == 1 ? v + 1 < H : d == 2 ? (u + 1 < W && v + 1 < H)
                                                                          : (u >= 1 && v + 1 < H);
      if (!inside) continue;
      const long long q = p + (d == 0 ? 1 : d == 1 ? W : d == 2 ? W + 1 : W - 1);
      double om, ta, tb;
      if (!mask[q] || !edge_model(nrm, p, q, u, v, d, persp, pitch, T, &om, &ta, &tb)) continue;
      o[d] = (float)om;
      const bool sim = use_sim && similar(nrm, p, q, cth);
      if (d == 0) eb |= EB_VR | (sim ? EB_SR : 0);
      if (d == 1) eb |= EB_VD | (sim ? EB_SD : 0);
      if (d == 2) e2 |= EB2_VDR | (sim ? EB2_SDR : 0);
      if (d == 3) e2 |= EB2_VDL | (sim ? EB2_SDL : 0);
    }
  }
  ebits[p] = eb;
  if (om_r) om_r[p] = o[0];
  if (om_d) om_d[p] = o[1];
  nt[p] = ntp;
  if (eb2) {
    eb2[p] = e2;
    if (om_dr) om_dr[p] = o[2];
    if (om_dl) om_dl[p] = o[3];
  }
}

// FP64 model of every inter-component edge (code = 4 a + direction):
// omega and the two gamma factors, for the relative-scale weights and
// residuals, which are computed in FP64 throughout
__global__ void __launch_bounds__(256) k_inter_geom(const uint32_t* __restrict__ eidx, int E, int W,
                                                    const float* __restrict__ nrm, int persp, double pitch,
                                                    RayTabs T, double* __restrict__ eom, double* __restrict__ eta,
                                                    double* __restrict__ etb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  const uint32_t code = eidx[i];
  const long long p = code >> 2;
  const int d = (int)(code & 3u);
  const int u = (int)(p % W), v = (int)(p / W);
  double om = 0.0, ta = 0.0, tb = 0.0;
  (void)edge_model(nrm, p, p + ni::dir_step(d, W), u, v, d, persp, pitch, T, &om, &ta, &tb);
  eom[i] = om;
  eta[i] = ta;
  etb[i] = tb;
}

__global__ void k_set_i32(int* __restrict__ a, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ray tables tau = ((u - cx)/fx, (v - cy)/fy) at pixel centres and at the
// midpoints u + 1/2, v + 1/2, in FP64 on the device (the same correctly
// rounded subtraction and division as the host's tables)
__global__ void k_ray_tables(int H, int W, double cx, double cy, double fx, double fy, double* __restrict__ t) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < W) {
    t[i] = ((double)i - cx) / fx;
    t[W + H + i] = (((double)i + 0.5) - cx) / fx;
  } else if (i < W + H) {
    const int v = i - W;
    t[W + v] = ((double)v - cy) / fy;
    t[2 * W + H + v] = (((double)v + 0.5) - cy) / fy;
  }
}

// ------------------------------------------------------------ union-find
// parent[x] <= x always holds, so the root of every tree is its smallest
// index and the final labelling is canonical whatever the order of unions.

__device__ __forceinline__ int uf_find(int* parent, int x) {
  int cur = parent[x];
  if (cur != x) {
    int prev = x, nxt;
    while (cur > (nxt = parent[cur])) {
      parent[prev] = nxt;  // path halving; any ancestor is a valid parent
      prev = cur;
      cur = nxt;
    }
  }
  return cur;
}

// hook the larger root under the smaller one; a failed CAS returns the
// root's new (smaller) parent and the walk resumes from there
__device__ __forceinline__ void uf_union(int* parent, int a, int b) {
  int ra = uf_find(parent, a), rb = uf_find(parent, b);
  while (ra != rb) {
    if (ra < rb) {
      int old = atomicCAS(&parent[rb], rb, ra);
      if (old == rb) break;
      rb = old;
    } else {
      int old = atomicCAS(&parent[ra], ra, rb);
      if (old == ra) break;
      ra = old;
    }
  }
}

__global__ void k_uf_init(const uint8_t* __restrict__ ebits, int P, int* __restrict__ parent) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) parent[p] = (ebits[p] & EB_VALID) ? p : -1;
}

// unions over the grid edges flagged by (bit_r, bit_d) in ebits and, with
// eb2 given, (bit_dr, bit_dl) in eb2
__global__ void k_uf_union_grid(const uint8_t* __restrict__ ebits, int P, int W, uint8_t bit_r,
                                uint8_t bit_d, const uint8_t* __restrict__ eb2, uint8_t bit_dr, uint8_t bit_dl,
                                int* parent) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  uint8_t e = ebits[p];
  if (e & bit_r) uf_union(parent, p, p + 1);
  if (e & bit_d) uf_union(parent, p, p + W);
  if (eb2) {
    const uint8_t f = eb2[p];
    if (f & bit_dr) uf_union(parent, p, p + W + 1);
    if (f & bit_dl) uf_union(parent, p, p + W - 1);
  }
}

// union over an explicit edge list (a[i], b[i]) where keep[i] != 0 (keep may be null)
__global__ void k_uf_union_list(const int* __restrict__ a, const int* __restrict__ b,
                                const double* __restrict__ keep, int n, int* parent) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (keep && !(keep[i] > 0.0)) return;
  uf_union(parent, a[i], b[i]);
}

__global__ void k_uf_flatten(int* parent, int P, int* __restrict__ root_flag) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int r = -1;
  if (parent[p] >= 0) {
    r = p;
    while (parent[r] != r) r = parent[r];
  }
  if (r >= 0) parent[p] = r;  // a root is a valid parent for concurrent walkers
  if (root_flag) root_flag[p] = (r == p) ? 1 : 0;
}

__global__ void k_uf_label(const int* __restrict__ parent, const int* __restrict__ cid, int P,
                           int* __restrict__ label) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) label[p] = parent[p] >= 0 ? cid[parent[p]] : -1;
}

__global__ void k_iota(int* a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

}  // namespace

namespace nil {

hipError_t launch_setup(const float* nrm, const uint8_t* mask, int H, int W, int persp, double pitch,
                        const double* tables, double cth, int use_sim, uint8_t* ebits, float* om_r,
                        float* om_d, float* nt, int* err, hipStream_t st, uint8_t* eb2, float* om_dr,
                        float* om_dl) {
  long long P = (long long)H * W;
  const double* tx = tables;
  const double* ty = tables + W;
  const double* txm = tables + W + H;
  const double* tym = tables + 2 * W + H;
  k_setup<<<ni::ceil_div(P, 256), 256, 0, st>>>(nrm, mask, H, W, persp, pitch, RayTabs{tx, ty, txm, tym}, cth,
                                                use_sim, ebits, om_r, om_d, nt, err, eb2, om_dr, om_dl);
  return hipGetLastError();
}

hipError_t set_i32(int* a, int n, int v, hipStream_t st) {
  if (n > 0) k_set_i32<<<ni::ceil_div(n, 256), 256, 0, st>>>(a, n, v);
  return hipGetLastError();
}

hipError_t ray_tables(int H, int W, double cx, double cy, double fx, double fy, double* t, hipStream_t st) {
  k_ray_tables<<<ni::ceil_div(W + H, 256), 256, 0, st>>>(H, W, cx, cy, fx, fy, t);
  return hipGetLastError();
}

hipError_t launch_inter_geom(const uint32_t* eidx, int E, int H, int W, const float* nrm, int persp, double pitch,
                             const double* tables, double* eom, double* eta, double* etb, hipStream_t st) {
  if (E <= 0) return hipSuccess;
  const RayTabs T{tables, tables + W, tables + W + H, tables + 2 * W + H};
  k_inter_geom<<<ni::ceil_div(E, 256), 256, 0, st>>>(eidx, E, W, nrm, persp, pitch, T, eom, eta, etb);
  return hipGetLastError();
}

// connected components of the valid pixels over the edges flagged by
// (bit_r, bit_d) and, with eb2 given (8-connectivity), (bit_dr, bit_dl).
// parent[P] ends flattened (root = min index, -1 invalid); flag/cid are
// scratch of P ints; label (optional) gets compact ids in ascending-root
// order; *count_dev gets the number of components.
hipError_t grid_components(const uint8_t* ebits, int H, int W, uint8_t bit_r, uint8_t bit_d,
                           int* parent, int* flag, int* cid, int* label, int* count_dev,
                           int* scan_tmp, hipStream_t st, const uint8_t* eb2, uint8_t bit_dr, uint8_t bit_dl) {
  int P = H * W;
  int nb = ni::ceil_div(P, 256);
  k_uf_init<<<nb, 256, 0, st>>>(ebits, P, parent);
  k_uf_union_grid<<<nb, 256, 0, st>>>(ebits, P, W, bit_r, bit_d, eb2, bit_dr, bit_dl, parent);
  k_uf_flatten<<<nb, 256, 0, st>>>(parent, P, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_i32(flag, cid, P, count_dev, scan_tmp, st);
  if (e != hipSuccess) return e;
  if (label) k_uf_label<<<nb, 256, 0, st>>>(parent, cid, P, label);
  return hipGetLastError();
}

// connected components of n nodes over the listed edges with keep > 0;
// parent[n] ends flattened (root = min index)
hipError_t list_components(int n, const int* a, const int* b, const double* keep, int m, int* parent,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_iota<<<ni::ceil_div(n, 256), 256, 0, st>>>(parent, n);
  if (m > 0) k_uf_union_list<<<ni::ceil_div(m, 256), 256, 0, st>>>(a, b, keep, m, parent);
  k_uf_flatten<<<ni::ceil_div(n, 256), 256, 0, st>>>(parent, n, nullptr);
  return hipGetLastError();
}

}  // namespace nil
