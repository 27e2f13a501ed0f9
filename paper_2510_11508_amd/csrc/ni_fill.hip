// Component fill (Sec. 3.3, Eq. 14-15): segments, matrix-free assembly and
// batched Jacobi-preconditioned CG, one independent system per component.
//
// Layout: the valid pixels are stored component-major ("compact" order):
// component c owns the index range [comp_off[c], comp_off[c+1]) and inside
// it the pixels keep raster order.  Hence the right neighbour of compact
// pixel i, when it lies in the same component, is i+1 and the left one is
// i-1; the lower / upper neighbours are i + off_d and i - off_u with
// 1 <= off <= W, packed in one 32-bit word (0 = no intra-component edge).
//
// System per component: L_c z = b_c with
//   L_c = sum over intra edges (a,b) of w_ab (e_a - e_b)(e_a - e_b)^T,
//   b_c = sum over intra edges of w_ab omega_{b->a} (e_a - e_b),
//   w_ab = (gamma^2_{b->a} + gamma^2_{a->b}) / 2     (BiNI weight at z = 0),
// which are the normal equations A_c^T W_c A_c z = A_c^T W_c b_c of Eq. 15
// with both directed rows of every edge.  Vectors are FP32, the stencil is
// evaluated in difference form sum_b w_ab (p_a - p_b), and every dot
// product / norm is accumulated in FP64.
#include "ni_common.h"

namespace {

constexpr uint32_t OFF_MASK = 0xFFFFu;

__global__ void k_valid_flags(const int* __restrict__ label, int P, int* __restrict__ flag) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) flag[p] = label[p] >= 0 ? 1 : 0;
}

__global__ void k_compact_valid(const int* __restrict__ label, const int* __restrict__ vpos, int P,
                                uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int c = label[p];
  if (c >= 0) {
    key[vpos[p]] = (uint32_t)c;
    val[vpos[p]] = (uint32_t)p;
  }
}

// caller-supplied labels: id in [0, K) exactly on the valid pixels, -1 elsewhere
__global__ void k_check_labels(const int* __restrict__ label, const uint8_t* __restrict__ ebits, int P, int K,
                               int* __restrict__ bad) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int l = label[p];
  bool valid = ebits[p] & EB_VALID;
  if (valid ? (l < 0 || l >= K) : (l != -1)) atomicOr(bad, 1);
}

// after sorting: every id 0..K-1 present (consecutive keys, first 0, last K-1)
__global__ void k_check_ids(const uint32_t* __restrict__ skey, int N, int K, int* __restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint32_t k = skey[i];
  bool ok = (i == 0) ? (k == 0u) : (k - skey[i - 1] <= 1u);
  if (i == N - 1) ok = ok && (k == (uint32_t)(K - 1));
  if (!ok) atomicOr(bad, 2);
}

// comp_off[c] = first compact index of component c; pos[p] = compact index
__global__ void k_segments(const uint32_t* __restrict__ skey, const uint32_t* __restrict__ spix, int N,
                           int K, int* __restrict__ comp_off, int* __restrict__ pos) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint32_t c = skey[i];
  if (i == 0 || skey[i - 1] != c) comp_off[c] = i;
  if (i == N - 1) comp_off[K] = N;
  pos[spix[i]] = i;
}

// Intra-component weights, packed neighbour offsets, rhs and inverse
// diagonal, computed in FP64 and stored FP32.  gamma^2 = (f n.tau)^2 in
// perspective (f = fx for horizontal, fy for vertical rows), n_z^2 in
// orthographic mode; g2f = (fx^2, fy^2) or (1, 1).
__global__ void k_assemble(const uint32_t* __restrict__ cpix, int N, int W, int P,
                           const int* __restrict__ label, const uint8_t* __restrict__ ebits,
                           const float* __restrict__ nt, const float* __restrict__ om_r,
                           const float* __restrict__ om_d, const int* __restrict__ pos, double g2fx,
                           double g2fy, float4* __restrict__ cst,
                           float* __restrict__ rhs, float* __restrict__ dinv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int p = (int)cpix[i];
  const int c = label[p];
  const int u = p % W;
  const uint8_t e = ebits[p];
  const double tp = nt[p];
  const double t2 = tp * tp;
  double wr = 0, wl = 0, wd = 0, wu = 0, b = 0;
  uint32_t ou = 0, od = 0;
  if ((e & EB_VR) && label[p + 1] == c) {
    double tq = nt[p + 1];
    wr = 0.5 * g2fx * t2 + 0.5 * g2fx * (tq * tq);
    b += wr * (double)om_r[p];
  }
  if (u > 0 && (ebits[p - 1] & EB_VR) && label[p - 1] == c) {
    double tq = nt[p - 1];
    wl = 0.5 * g2fx * (tq * tq) + 0.5 * g2fx * t2;
    b -= wl * (double)om_r[p - 1];
  }
  if ((e & EB_VD) && label[p + W] == c) {
    double tq = nt[p + W];
    wd = 0.5 * g2fy * t2 + 0.5 * g2fy * (tq * tq);
    b += wd * (double)om_d[p];
    od = (uint32_t)(pos[p + W] - i);
  }
  if (p >= W && (ebits[p - W] & EB_VD) && label[p - W] == c) {
    double tq = nt[p - W];
    wu = 0.5 * g2fy * (tq * tq) + 0.5 * g2fy * t2;
    b -= wu * (double)om_d[p - W];
    ou = (uint32_t)(i - pos[p - W]);
  }
  // weights are rounded to FP32 first so that the stored matrix is exactly
  // symmetric (w_l of pixel i is bitwise the w_r of pixel i-1)
  const float fr = (float)wr, fl = (float)wl, fd = (float)wd, fu = (float)wu;
  cst[i] = make_float4(fr, fd, fu, __uint_as_float(ou | (od << 16)));
  rhs[i] = (float)b;
  double dg = (double)fr + (double)fl + (double)fd + (double)fu;
  dinv[i] = dg > 0 ? (float)(1.0 / dg) : 0.f;
}

// size tiers: 1: 2..256 px (one wave), 2: ..2048 (256 threads), 3: ..8192
// (1024 threads), 4: larger (grid-wide chunks); singletons need no solve
__device__ __forceinline__ int size_tier(int n) {
  return n <= 1 ? 0 : n <= 256 ? 1 : n <= 2048 ? 2 : n <= 8192 ? 3 : 4;
}

// tier 1..4 as size_tier; tier 5: every component of two or more pixels
__global__ void k_tier_flags(const int* __restrict__ comp_off, int K, int tier, int* __restrict__ flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  const int t = size_tier(comp_off[c + 1] - comp_off[c]);
  flag[c] = (tier == 5 ? t >= 1 : t == tier) ? 1 : 0;
}

__global__ void k_tier_list(const int* __restrict__ flag, const int* __restrict__ pos, int K, int* __restrict__ list) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K && flag[c]) list[pos[c]] = c;
}

__device__ __forceinline__ int chunk_len(int n, int chunk, int maxch, int nt) {
  int nch = min(max(ni::ceil_div(n, chunk), 1), maxch);
  return ni::ceil_div(ni::ceil_div(n, nch), nt) * nt;
}

__global__ void k_chunk_counts(const int* __restrict__ comp_off, int K, int chunk, int maxch, int nt,
                               int* __restrict__ nchunk) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  int n = comp_off[c + 1] - comp_off[c];
  nchunk[c] = size_tier(n) == 4 ? ni::ceil_div(n, chunk_len(n, chunk, maxch, nt)) : 0;
}

__global__ void k_chunk_table(const int* __restrict__ comp_off, const int* __restrict__ nchunk,
                              const int* __restrict__ cbase, int K, int chunk, int maxch, int nt,
                              int* __restrict__ chunk_comp, int* __restrict__ chunk_start,
                              int* __restrict__ chunk_end) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K || nchunk[c] == 0) return;
  const int lo = comp_off[c], hi = comp_off[c + 1];
  const int len = chunk_len(hi - lo, chunk, maxch, nt);
  for (int j = 0; j < nchunk[c]; ++j) {
    chunk_comp[cbase[c] + j] = c;
    chunk_start[cbase[c] + j] = lo + j * len;
    chunk_end[cbase[c] + j] = min(lo + (j + 1) * len, hi);
  }
}

// x0: gathered learned start (grid, may be null -> 0)
__global__ void k_gather_x0(const uint32_t* __restrict__ cpix, int N, const float* __restrict__ x0g,
                            float* __restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) x[i] = x0g ? x0g[cpix[i]] : 0.f;
}

// ------------------------------------------------------- stencil helpers
struct Stencil {
  float wr, wl, wd, wu;
  int od, ou;
};

__device__ __forceinline__ Stencil load_stencil(const float4* __restrict__ cst, int i, int lo) {
  Stencil s;
  const float4 v = cst[i];
  s.wr = v.x;
  s.wl = i > lo ? cst[i - 1].x : 0.f;
  s.wd = v.y;
  s.wu = v.z;
  uint32_t o = __float_as_uint(v.w);
  s.ou = (int)(o & OFF_MASK);
  s.od = (int)(o >> 16);
  return s;
}

// ============================================================ small path
// One workgroup solves one component of n <= NT*PPT pixels with every
// vector in registers and the search direction shared through LDS; no
// global traffic inside the iteration loop.
template <int NT, int PPT>
__global__ void __launch_bounds__(NT) k_fill_small(
    const int* __restrict__ list, const int* __restrict__ comp_off, const float4* __restrict__ cst,
    const float* __restrict__ rhs, const float* __restrict__ dinv, const float* __restrict__ x0,
    const uint32_t* __restrict__ cpix, float* __restrict__ zgrid, double rtol, int maxit, int warm,
    int* __restrict__ iters, double* __restrict__ relres, int* __restrict__ stats) {
  constexpr int CAP = NT * PPT;
  constexpr int NW = NT / 64;
  __shared__ float sp[CAP];
  __shared__ double red[2][3 * NW];
  const int c = list[blockIdx.x];
  const int lo = comp_off[c];
  const int n = comp_off[c + 1] - lo;
  float wr[PPT], wl[PPT], wd[PPT], wu[PPT], di[PPT], x[PPT], r[PPT], pv[PPT];
  int od[PPT], ou[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int j = threadIdx.x + k * NT;
    if (j < n) {
      Stencil s = load_stencil(cst, lo + j, lo);
      wr[k] = s.wr; wl[k] = s.wl; wd[k] = s.wd; wu[k] = s.wu; od[k] = s.od; ou[k] = s.ou;
      di[k] = dinv[lo + j];
      r[k] = rhs[lo + j];
      x[k] = warm ? x0[lo + j] : 0.f;
    } else {
      wr[k] = wl[k] = wd[k] = wu[k] = 0.f;
      od[k] = ou[k] = 0;
      di[k] = 0.f; r[k] = 0.f; x[k] = 0.f;
    }
    pv[k] = 0.f;
  }
  auto spmv = [&](int k, float pj, int j) -> float {
    float q = 0.f;
    if (wr[k] != 0.f) q += wr[k] * (pj - sp[j + 1]);
    if (wl[k] != 0.f) q += wl[k] * (pj - sp[j - 1]);
    if (wd[k] != 0.f) q += wd[k] * (pj - sp[j + od[k]]);
    if (wu[k] != 0.f) q += wu[k] * (pj - sp[j - ou[k]]);
    return q;
  };
  // ||b||^2
  double v1[1] = {0.0};
#pragma unroll
  for (int k = 0; k < PPT; ++k) v1[0] += (double)r[k] * r[k];
  ni::block_sum<1>(v1, red[0]);
  const double bb = v1[0];
  int fallback = 0;
  if (warm) {
    // centre the start on the component (only differences matter) and
    // form r0 = b - L x0; restart from zero if the start is worse than 0
    double vm[1] = {0.0};
#pragma unroll
    for (int k = 0; k < PPT; ++k) vm[0] += x[k];
    ni::block_sum<1>(vm, red[1]);
    const float mean = (float)(vm[0] / n);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int j = threadIdx.x + k * NT;
      if (j < n) { x[k] -= mean; sp[j] = x[k]; }
    }
    __syncthreads();
    double v2[1] = {0.0};
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int j = threadIdx.x + k * NT;
      if (j < n) r[k] -= spmv(k, x[k], j);
      v2[0] += (double)r[k] * r[k];
    }
    ni::block_sum<1>(v2, red[0]);
    if (!(v2[0] < bb)) {
      fallback = 1;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int j = threadIdx.x + k * NT;
        x[k] = 0.f;
        r[k] = j < n ? rhs[lo + j] : 0.f;
      }
    }
    __syncthreads();
  }
  const double tol2 = rtol * rtol * bb;
  double vz[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    vz[0] += (double)r[k] * r[k];
    vz[1] += (double)r[k] * (di[k] * r[k]);
  }
  ni::block_sum<2>(vz, red[1]);
  double rr = vz[0], rho = vz[1];
  int it = 0;
  float beta = 0.f;
  if (bb > 0.0) {
    while (rr > tol2 && it < maxit) {
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int j = threadIdx.x + k * NT;
        pv[k] = di[k] * r[k] + beta * pv[k];
        if (j < n) sp[j] = pv[k];
      }
      __syncthreads();
      float q[PPT];
      double vq[1] = {0.0};
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int j = threadIdx.x + k * NT;
        q[k] = j < n ? spmv(k, pv[k], j) : 0.f;
        vq[0] += (double)pv[k] * q[k];
      }
      ni::block_sum<1>(vq, red[0]);
      const float alpha = (float)(rho / vq[0]);
      double vr[2] = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        x[k] += alpha * pv[k];
        r[k] -= alpha * q[k];
        vr[0] += (double)r[k] * r[k];
        vr[1] += (double)r[k] * (di[k] * r[k]);
      }
      ni::block_sum<2>(vr, red[1]);
      rr = vr[0];
      beta = (float)(vr[1] / rho);
      rho = vr[1];
      ++it;
    }
  } else {
#pragma unroll
    for (int k = 0; k < PPT; ++k) x[k] = 0.f;
  }
  // zero mean per component (A15), scatter to the grid
  double vm[1] = {0.0};
#pragma unroll
  for (int k = 0; k < PPT; ++k) vm[0] += x[k];
  ni::block_sum<1>(vm, red[0]);
  const double mean = vm[0] / n;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int j = threadIdx.x + k * NT;
    if (j < n) zgrid[cpix[lo + j]] = (float)((double)x[k] - mean);
  }
  if (threadIdx.x == 0) {
    iters[c] = it;
    relres[c] = bb > 0 ? sqrt(rr / bb) : 0.0;
    if (it >= maxit && rr > tol2) atomicAdd(&stats[0], 1);
    if (fallback) atomicAdd(&stats[1], 1);
  }
}

// ============================================================ large path
// Components above the LDS capacity are cut into chunks of LCH pixels and
// all of them advance together through Jacobi-preconditioned CG, two
// kernel launches per iteration:
//   A_i: beta_i = rho_i / rho_{i-1}; p_i = D^-1 r_i + beta_i p_{i-1};
//        q_i = L p_i (the neighbours' p_i are recomputed from their r_i and
//        p_{i-1}); partial (p_i, q_i)
//   B_i: alpha_i = rho_i / (p_i, q_i); x += alpha_i p_i; r -= alpha_i q_i;
//        partials rho_{i+1} = (r, D^-1 r) and ||r||^2
// The stencil is evaluated in difference form sum_b w_ab (p_a - p_b), which
// keeps the FP32 vectors accurate; every dot product is an FP64 sum.  Each
// launch writes per-chunk FP64 partials [rho, rr, pq, bb] into one of two
// slots, and every workgroup of a component sums the previous launch's slot
// itself, in chunk order: the scalars are bitwise identical across the
// component's workgroups and across runs, and no atomic or in-kernel fence
// is needed for them because the launch boundary orders global memory.
// chunks: up to 256 per component, at least 512 pixels each, a multiple
// of the workgroup size long (so mid-size problems still fill the GPU while
// the per-workgroup partial sums stay short)
constexpr int LNT = 256, LCH = 512, LMAXCH = 512;
constexpr int LU = 4;  // pixels per thread whose loads are issued together

struct LargeState {
  const int* comp_off;
  const int* cbase;       // first chunk of each component
  const int* nchunk;      // chunks per component
  const int* chunk_comp;
  const int* chunk_start;
  const int* chunk_end;
  double* part;           // [2][nchunks][4] = (rho, rr, pq, bb) by launch parity
  double* gam;            // [2][K] rho_i by iteration parity
  double* tol2;           // [K]
  double* rr;             // [K] last ||r||^2
  double* bb;             // [K] ||b||^2
  int* iters;             // [K]
  int* active;            // [2] components still iterating, by iteration parity
  int* stats;             // [0] not converged, [1] warm fallbacks
  const float4* cst;  // per pixel (w_right, w_down, w_up, packed offsets)
  const float *rhs, *dinv;
  float *x, *p, *r0, *r1, *w0, *w1, *s0, *s1;  // r0 = r, w0 = q, s0/s1 = p by parity
  int nchunks;
  double rtol;
  int maxit;
};

// component sums of the previous launch's partials (slot), fixed order
__device__ __forceinline__ void comp_partials(const LargeState& S, int c, int slot, double (&v)[4], double* red) {
  const int base = S.cbase[c], nch = S.nchunk[c];
  const double* pp = S.part + (size_t)slot * S.nchunks * 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = 0.0;
  for (int j = threadIdx.x; j < nch; j += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += pp[(size_t)(base + j) * 4 + k];
  }
  ni::block_sum<4>(v, red);
}

// write this chunk's partials: fields in `mask` from v, the others copied
// from the previous slot (so every slot always holds the latest values)
__device__ __forceinline__ void put_partials(const LargeState& S, int ch, int wslot, const double* v, int mask) {
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    const size_t dst = ((size_t)wslot * S.nchunks + ch) * 4 + k;
    const size_t src = ((size_t)(wslot ^ 1) * S.nchunks + ch) * 4 + k;
    // select without indexing v by the thread (that would put v in scratch)
    const double vk = k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3];
    S.part[dst] = ((mask >> k) & 1) ? vk : S.part[src];
  }
}

// init A: r = b - L x for the start x (0 or learned); partials -> slot 0
__global__ void __launch_bounds__(LNT) k_lg_init_a(LargeState S) {
  __shared__ double red[4 * (LNT / 64)];
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int clo = S.comp_off[c], hi = S.comp_off[c + 1];
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = lo + threadIdx.x; i < S.chunk_end[ch]; i += LNT) {
    Stencil s = load_stencil(S.cst, i, clo);
    const float xi = S.x[i];
    float q = 0.f;
    if (s.wr != 0.f) q += s.wr * (xi - S.x[i + 1]);
    if (s.wl != 0.f) q += s.wl * (xi - S.x[i - 1]);
    if (s.wd != 0.f) q += s.wd * (xi - S.x[i + s.od]);
    if (s.wu != 0.f) q += s.wu * (xi - S.x[i - s.ou]);
    const float b = S.rhs[i];
    const float ri = b - q;
    S.r0[i] = ri;
    v[0] += (double)ri * (S.dinv[i] * ri);
    v[1] += (double)ri * ri;
    v[2] += (double)b * b;
  }
  ni::block_sum<3>(v, red);
  if (threadIdx.x < 4) {
    const double vv[4] = {v[0], v[1], 0.0, v[2]};
    S.part[(size_t)ch * 4 + threadIdx.x] = vv[threadIdx.x];
  }
}

// init B: a start no better than zero (||r|| >= ||b||) is dropped (x = 0,
// r = b); p_{-1} = 0; partials -> slot 1, read by launch A_0
__global__ void __launch_bounds__(LNT) k_lg_init_b(LargeState S, int warm) {
  __shared__ double red[8 * (LNT / 64)];
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int hi = S.comp_off[c + 1];
  double t[4];
  comp_partials(S, c, 0, t, red);
  const bool reset = warm && !(t[1] < t[3]);
  double v[2] = {0.0, 0.0};
  for (int i = lo + threadIdx.x; i < S.chunk_end[ch]; i += LNT) {
    S.s1[i] = 0.f;
    if (reset) {
      const float b = S.rhs[i];
      S.x[i] = 0.f;
      S.r0[i] = b;
      v[0] += (double)b * (S.dinv[i] * b);
      v[1] += (double)b * b;
    }
  }
  if (reset) ni::block_sum<2>(v, red + 4 * (LNT / 64));
  if (threadIdx.x < 4) {
    const size_t src = (size_t)ch * 4 + threadIdx.x;
    const size_t dst = ((size_t)S.nchunks + ch) * 4 + threadIdx.x;
    double val = S.part[src];
    if (reset && threadIdx.x < 2) val = v[threadIdx.x];
    S.part[dst] = val;
  }
  if (threadIdx.x == 0 && ch == S.cbase[c]) {
    S.bb[c] = t[3];
    S.tol2[c] = S.rtol * S.rtol * t[3];
    S.iters[c] = 0;
    if (reset) atomicAdd(&S.stats[1], 1);
  }
}

// A_i: launch 2i, writes slot 0, reads slot 1
__global__ void __launch_bounds__(LNT) k_lg_a(LargeState S, int it, int K) {
  __shared__ double red[8 * (LNT / 64)];
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int clo = S.comp_off[c], hi = S.comp_off[c + 1];
  double g[4];
  comp_partials(S, c, 1, g, red);
  const double rho = g[0], rri = g[1];
  const bool conv = (S.bb[c] == 0.0) || (rri <= S.tol2[c]);
  if (conv || it >= S.maxit) {
    put_partials(S, ch, 0, g, 0);
    if (threadIdx.x == 0 && ch == S.cbase[c]) {
      S.rr[c] = rri;
      if (!conv && it == S.maxit) atomicAdd(&S.stats[0], 1);
    }
    return;
  }
  const double beta = it == 0 ? 0.0 : rho / S.gam[(size_t)((it - 1) & 1) * K + c];
  if (threadIdx.x == 0 && ch == S.cbase[c]) S.gam[(size_t)(it & 1) * K + c] = rho;
  const float bt = (float)beta;
  const float* pold = (it & 1) ? S.s0 : S.s1;  // p_{i-1}
  float* pnew = (it & 1) ? S.s1 : S.s0;        // p_i
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int end = S.chunk_end[ch];
  auto P = [&](int j) { return S.dinv[j] * S.r0[j] + bt * pold[j]; };
  // LU pixels per thread and round, every load issued before any use; a
  // missing neighbour (weight 0) reads the pixel itself
  for (int i0 = lo + threadIdx.x; i0 < end; i0 += LNT * LU) {
    int ix[LU];
    Stencil st[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      ix[u] = i0 + u * LNT < end ? i0 + u * LNT : lo;
      st[u] = load_stencil(S.cst, ix[u], clo);
    }
    float pc[LU], pr[LU], pl[LU], pd[LU], pu[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int i = ix[u];
      pc[u] = P(i);
      pr[u] = P(st[u].wr != 0.f ? i + 1 : i);
      pl[u] = P(st[u].wl != 0.f ? i - 1 : i);
      pd[u] = P(st[u].wd != 0.f ? i + st[u].od : i);
      pu[u] = P(st[u].wu != 0.f ? i - st[u].ou : i);
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      if (i0 + u * LNT < end) {
        const int i = ix[u];
        float q = 0.f;
        q += st[u].wr * (pc[u] - pr[u]);
        q += st[u].wl * (pc[u] - pl[u]);
        q += st[u].wd * (pc[u] - pd[u]);
        q += st[u].wu * (pc[u] - pu[u]);
        pnew[i] = pc[u];
        S.w0[i] = q;
        v[2] += (double)pc[u] * q;
      }
    }
  }
  ni::block_sum<4>(v, red + 4 * (LNT / 64));
  put_partials(S, ch, 0, v, 4);
}

// Three-launch form of the same iteration (chosen by the autotuner where it
// is faster, on the largest maps): P_i materialises p_i, then Q_i applies
// the stencil to p_i alone, so a neighbour costs one load instead of three
// at the price of one more launch and 4 more bytes per pixel.
// P_i: p_i = D^-1 r + beta p_{i-1}, elementwise (reads slot 1)
__global__ void __launch_bounds__(LNT) k_lg_p(LargeState S, int it, int K) {
  __shared__ double red[8 * (LNT / 64)];
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  double g[4];
  comp_partials(S, c, 1, g, red);
  const double rho = g[0], rri = g[1];
  const bool conv = (S.bb[c] == 0.0) || (rri <= S.tol2[c]);
  if (conv || it >= S.maxit) return;
  const double beta = it == 0 ? 0.0 : rho / S.gam[(size_t)((it - 1) & 1) * K + c];
  if (threadIdx.x == 0 && ch == S.cbase[c]) S.gam[(size_t)(it & 1) * K + c] = rho;
  const float bt = (float)beta;
  const float* pold = (it & 1) ? S.s0 : S.s1;
  float* pnew = (it & 1) ? S.s1 : S.s0;
  const int end = S.chunk_end[ch];
  for (int i0 = lo + threadIdx.x; i0 < end; i0 += LNT * LU) {
    float d[LU], r[LU], po[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int i = i0 + u * LNT < end ? i0 + u * LNT : lo;
      d[u] = S.dinv[i];
      r[u] = S.r0[i];
      po[u] = pold[i];
    }
#pragma unroll
    for (int u = 0; u < LU; ++u)
      if (i0 + u * LNT < end) pnew[i0 + u * LNT] = d[u] * r[u] + bt * po[u];
  }
}

// Q_i: q = L p_i and (p, q) -> slot 0 (reads slot 1 for the convergence test)
__global__ void __launch_bounds__(LNT) k_lg_q(LargeState S, int it, int K) {
  __shared__ double red[8 * (LNT / 64)];
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int clo = S.comp_off[c];
  double g[4];
  comp_partials(S, c, 1, g, red);
  const double rri = g[1];
  const bool conv = (S.bb[c] == 0.0) || (rri <= S.tol2[c]);
  if (conv || it >= S.maxit) {
    put_partials(S, ch, 0, g, 0);
    if (threadIdx.x == 0 && ch == S.cbase[c]) {
      S.rr[c] = rri;
      if (!conv && it == S.maxit) atomicAdd(&S.stats[0], 1);
    }
    return;
  }
  const float* pp = (it & 1) ? S.s1 : S.s0;  // p_i
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int end = S.chunk_end[ch];
  for (int i0 = lo + threadIdx.x; i0 < end; i0 += LNT * LU) {
    int ix[LU];
    Stencil st[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      ix[u] = i0 + u * LNT < end ? i0 + u * LNT : lo;
      st[u] = load_stencil(S.cst, ix[u], clo);
    }
    float pc[LU], pr[LU], pl[LU], pd[LU], pu[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int i = ix[u];
      pc[u] = pp[i];
      pr[u] = pp[st[u].wr != 0.f ? i + 1 : i];
      pl[u] = pp[st[u].wl != 0.f ? i - 1 : i];
      pd[u] = pp[st[u].wd != 0.f ? i + st[u].od : i];
      pu[u] = pp[st[u].wu != 0.f ? i - st[u].ou : i];
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      if (i0 + u * LNT < end) {
        float q = 0.f;
        q += st[u].wr * (pc[u] - pr[u]);
        q += st[u].wl * (pc[u] - pl[u]);
        q += st[u].wd * (pc[u] - pd[u]);
        q += st[u].wu * (pc[u] - pu[u]);
        S.w0[ix[u]] = q;
        v[2] += (double)pc[u] * q;
      }
    }
  }
  ni::block_sum<4>(v, red + 4 * (LNT / 64));
  put_partials(S, ch, 0, v, 4);
}

// B_i: launch 2i+1, writes slot 1, reads slot 0
__global__ void __launch_bounds__(LNT) k_lg_b(LargeState S, int it, int K) {
  __shared__ double red[8 * (LNT / 64)];
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int hi = S.comp_off[c + 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) S.active[(it + 1) & 1] = 0;  // read by the host already
  double g[4];
  comp_partials(S, c, 0, g, red);
  const double rho = g[0], rri = g[1], pq = g[2];
  const bool conv = (S.bb[c] == 0.0) || (rri <= S.tol2[c]);
  if (conv || it >= S.maxit) {
    put_partials(S, ch, 1, g, 0);
    return;
  }
  if (threadIdx.x == 0 && ch == S.cbase[c]) {
    S.iters[c] = it + 1;
    atomicAdd(&S.active[it & 1], 1);
  }
  const float alpha = (float)(rho / pq);
  const float* pcur = (it & 1) ? S.s1 : S.s0;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int end = S.chunk_end[ch];
  for (int i0 = lo + threadIdx.x; i0 < end; i0 += LNT * LU) {
    float r[LU], w[LU], x[LU], pp[LU], d[LU];
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int i = i0 + u * LNT < end ? i0 + u * LNT : lo;
      r[u] = S.r0[i];
      w[u] = S.w0[i];
      x[u] = S.x[i];
      pp[u] = pcur[i];
      d[u] = S.dinv[i];
    }
#pragma unroll
    for (int u = 0; u < LU; ++u) {
      const int i = i0 + u * LNT;
      if (i < end) {
        const float ri = r[u] - alpha * w[u];
        S.x[i] = x[u] + alpha * pp[u];
        S.r0[i] = ri;
        v[0] += (double)ri * (d[u] * ri);
        v[1] += (double)ri * ri;
      }
    }
  }
  ni::block_sum<4>(v, red + 4 * (LNT / 64));
  put_partials(S, ch, 1, v, 3);
  if (threadIdx.x == 0 && ch == S.cbase[c]) S.rr[c] = rri;
}

// zero mean per component, scatter to the grid
__global__ void __launch_bounds__(LNT) k_lg_sum(LargeState S, int slot) {
  __shared__ double red[4 * (LNT / 64)];
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int hi = S.comp_off[c + 1];
  double v[1] = {0.0};
  for (int i = lo + threadIdx.x; i < S.chunk_end[ch]; i += LNT) {
    v[0] += S.x[i];
  }
  ni::block_sum<1>(v, red);
  if (threadIdx.x == 0) S.part[((size_t)slot * S.nchunks + ch) * 4] = v[0];
}

__global__ void __launch_bounds__(LNT) k_lg_center(LargeState S, int slot, float* __restrict__ out,
                                                   const uint32_t* __restrict__ cpix) {
  __shared__ double red[4 * (LNT / 64)];
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int clo = S.comp_off[c], hi = S.comp_off[c + 1];
  const int base = S.cbase[c], nch = S.nchunk[c];
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < nch; j += blockDim.x) v[0] += S.part[((size_t)slot * S.nchunks + base + j) * 4];
  ni::block_sum<1>(v, red);
  const double mean = v[0] / (double)(hi - clo);
  for (int i = lo + threadIdx.x; i < S.chunk_end[ch]; i += LNT) {
    if (out) out[cpix[i]] = (float)((double)S.x[i] - mean);
    else S.x[i] = (float)((double)S.x[i] - mean);
  }
}

// ====================================================== multigrid path
// The large components' systems as one weighted graph Laplacian for the
// multigrid PCG: level-0 nodes are the compacted pixels (a node of a small
// component has an empty row and takes no part), entries in FP64 from the
// same FP32 weights as the stencil, pairs (i < j) for the right and down
// edges, the pixel coordinates and component of every node.
__device__ __forceinline__ bool is_large(const uint32_t* skey, const int* comp_off, int i, int cap, int& k) {
  k = (int)skey[i];
  return comp_off[k + 1] - comp_off[k] > cap;
}

__global__ void k_mg_count(int N, const float4* __restrict__ cst, const uint32_t* __restrict__ skey,
                           const int* __restrict__ comp_off, int cap, int* __restrict__ deg, int* __restrict__ npair) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int k;
  int d = 0, pr = 0;
  if (is_large(skey, comp_off, i, cap, k)) {
    const Stencil s = load_stencil(cst, i, comp_off[k]);
    d = (s.wr != 0.f) + (s.wl != 0.f) + (s.wd != 0.f) + (s.wu != 0.f);
    pr = (s.wr != 0.f) + (s.wd != 0.f);
  }
  deg[i] = d;
  npair[i] = pr;
}

__global__ void k_mg_build(int N, int W, const float4* __restrict__ cst, const float* __restrict__ rhs,
                           const float* __restrict__ x32, const uint32_t* __restrict__ cpix,
                           const uint32_t* __restrict__ skey, const int* __restrict__ comp_off, int cap,
                           const int* __restrict__ row_off, const int* __restrict__ pair_off, int* __restrict__ col,
                           double* __restrict__ w, double* __restrict__ diag, int* __restrict__ plo,
                           int* __restrict__ phi, double* __restrict__ pw, int* __restrict__ gy, int* __restrict__ gx,
                           int* __restrict__ gc, double* __restrict__ b64, double* __restrict__ x64) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int k;
  const int p = (int)cpix[i];
  gy[i] = p / W;
  gx[i] = p % W;
  if (!is_large(skey, comp_off, i, cap, k)) {
    diag[i] = 0.0;
    gc[i] = -1;
    b64[i] = 0.0;
    x64[i] = 0.0;
    return;
  }
  const Stencil s = load_stencil(cst, i, comp_off[k]);
  int j = row_off[i];
  double dg = 0.0;
  auto put = [&](int c, float v) {
    col[j] = c;
    w[j] = (double)v;
    dg += (double)v;
    ++j;
  };
  if (s.wl != 0.f) put(i - 1, s.wl);
  if (s.wu != 0.f) put(i - s.ou, s.wu);
  if (s.wd != 0.f) put(i + s.od, s.wd);
  if (s.wr != 0.f) put(i + 1, s.wr);
  diag[i] = dg;
  int q = pair_off[i];
  if (s.wr != 0.f) {
    plo[q] = i;
    phi[q] = i + 1;
    pw[q] = (double)s.wr;
    ++q;
  }
  if (s.wd != 0.f) {
    plo[q] = i;
    phi[q] = i + s.od;
    pw[q] = (double)s.wd;
  }
  gc[i] = k;
  b64[i] = (double)rhs[i];
  x64[i] = (double)x32[i];
}

__global__ void k_mg_out(int N, const uint32_t* __restrict__ skey, const int* __restrict__ comp_off, int cap,
                         const double* __restrict__ x64, float* __restrict__ x32) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int k;
  if (i < N && is_large(skey, comp_off, i, cap, k)) x32[i] = (float)x64[i];
}

__global__ void k_zero_grid(float* z, int P) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) z[p] = 0.f;
}

// ===================================================== 8-connectivity
// The level-0 system of every component of two or more pixels, assembled
// straight from the edge bits in FP64 (a pixel row holds up to eight
// neighbours, beyond the packed four-neighbour stencil) and solved by the
// multigrid PCG.  Neighbour slot k of pixel p: k < 4 the edge of direction
// k that p owns, k >= 4 the edge of direction k - 4 that ends at p.
struct Om4 {
  const float* o[4];  // omega_{b->a} per direction at the owner a
};

__device__ __forceinline__ bool nb8(const uint8_t* __restrict__ eb, const uint8_t* __restrict__ eb2, int p, int W,
                                    int k, int& owner, int& other, int& d) {
  d = k & 3;
  const int step = ni::dir_step(d, W);
  if (k < 4) {
    owner = p;
    other = p + step;
    return ni::dir_usable(eb, eb2, p, d);
  }
  owner = p - step;
  other = p;
  return ni::has_back(p, d, W) && ni::dir_usable(eb, eb2, owner, d);
}

// w = (gamma^2_{b->a} + gamma^2_{a->b}) / 2 with gamma^2 = f^2 t^2, in a
// fixed rounding order so that both ends of an edge compute the same bits
__device__ __forceinline__ double edge_w(double ta, double tb, double g2f) {
  return __dadd_rn(__dmul_rn(__dmul_rn(0.5, g2f), __dmul_rn(ta, ta)),
                   __dmul_rn(__dmul_rn(0.5, g2f), __dmul_rn(tb, tb)));
}

__global__ void k_fill8_count(int N, int W, const uint32_t* __restrict__ cpix, const int* __restrict__ label,
                              const uint8_t* __restrict__ eb, const uint8_t* __restrict__ eb2, int* __restrict__ deg,
                              int* __restrict__ npair) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int p = (int)cpix[i];
  const int c = label[p];
  int dg = 0, pr = 0;
  for (int k = 0; k < 8; ++k) {
    int a, b, d;
    if (nb8(eb, eb2, p, W, k, a, b, d) && label[k < 4 ? b : a] == c) {
      ++dg;
      pr += k < 4;
    }
  }
  deg[i] = dg;
  npair[i] = pr;
}

__global__ void k_fill8_build(int N, int W, const uint32_t* __restrict__ cpix, const uint32_t* __restrict__ skey,
                              const int* __restrict__ comp_off, const int* __restrict__ label,
                              const uint8_t* __restrict__ eb, const uint8_t* __restrict__ eb2,
                              const float* __restrict__ nt, Om4 om, const int* __restrict__ pos, double g2fx,
                              double g2fy, double g2fd, const int* __restrict__ row_off,
                              const int* __restrict__ pair_off, const float* __restrict__ x32, int* __restrict__ col,
                              double* __restrict__ w, double* __restrict__ diag, int* __restrict__ plo,
                              int* __restrict__ phi, double* __restrict__ pw, int* __restrict__ gy,
                              int* __restrict__ gx, int* __restrict__ gc, double* __restrict__ b64,
                              double* __restrict__ x64) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int p = (int)cpix[i];
  const int c = label[p];
  const int k0 = (int)skey[i];
  gy[i] = p / W;
  gx[i] = p % W;
  gc[i] = comp_off[k0 + 1] - comp_off[k0] >= 2 ? k0 : -1;
  int j = row_off[i], q = pair_off[i];
  double dg = 0.0, b = 0.0;
  for (int k = 0; k < 8; ++k) {
    int a, o, d;
    if (!nb8(eb, eb2, p, W, k, a, o, d)) continue;
    const int nbr = k < 4 ? o : a;
    if (label[nbr] != c) continue;
    const double g2f = d == 0 ? g2fx : d == 1 ? g2fy : g2fd;
    const double wv = edge_w((double)nt[a], (double)nt[o], g2f);
    const double omv = (double)om.o[d][a];
    col[j] = pos[nbr];
    w[j] = wv;
    ++j;
    dg += wv;
    if (k < 4) {
      b += wv * omv;
      plo[q] = i;
      phi[q] = pos[nbr];
      pw[q] = wv;
      ++q;
    } else {
      b -= wv * omv;
    }
  }
  diag[i] = dg;
  b64[i] = b;
  x64[i] = (double)x32[i];
}

// zero mean per component (the gauge of Eq. 15), scattered to the grid;
// a singleton's log-depth is 0
__global__ void k_fill8_out(int N, const uint32_t* __restrict__ cpix, const uint32_t* __restrict__ skey,
                            const int* __restrict__ comp_off, const double* __restrict__ x64,
                            const double* __restrict__ csum, float* __restrict__ z) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int k = (int)skey[i];
  const int n = comp_off[k + 1] - comp_off[k];
  z[cpix[i]] = n >= 2 ? (float)(x64[i] - csum[k] / (double)n) : 0.f;
}

}  // namespace

namespace nil {

int fill_small_cap() { return 8192; }
int fill_chunk() { return LCH; }

hipError_t check_labels(const int* label, const uint8_t* ebits, int P, int K, int* bad, hipStream_t st) {
  k_check_labels<<<ni::ceil_div(P, 256), 256, 0, st>>>(label, ebits, P, K, bad);
  return hipGetLastError();
}

hipError_t check_ids(const uint32_t* skey, int N, int K, int* bad, hipStream_t st) {
  if (N > 0) k_check_ids<<<ni::ceil_div(N, 256), 256, 0, st>>>(skey, N, K, bad);
  return hipGetLastError();
}

hipError_t fill_segments(const int* label, int P, int K, int* flag, int* vpos, int* n_dev,
                         uint32_t* key, uint32_t* val, uint32_t* skey, uint32_t* spix, uint32_t* ktmp,
                         uint32_t* vtmp, int N, int* comp_off, int* pos, int* scan_tmp, hipStream_t st,
                         int phase) {
  int nb = ni::ceil_div(P, 256);
  if (phase == 0) {
    k_valid_flags<<<nb, 256, 0, st>>>(label, P, flag);
    hipError_t e = scan_exclusive_i32(flag, vpos, P, n_dev, scan_tmp, st);
    if (e != hipSuccess) return e;
    k_compact_valid<<<nb, 256, 0, st>>>(label, vpos, P, key, val);
    return hipGetLastError();
  }
  int bits = 0;
  while ((1ll << bits) < (long long)K) ++bits;
  hipError_t e = radix_sort_pairs(key, val, skey, spix, ktmp, vtmp, N, bits, scan_tmp, st);
  if (e != hipSuccess) return e;
  if (N > 0) k_segments<<<ni::ceil_div(N, 256), 256, 0, st>>>(skey, spix, N, K, comp_off, pos);
  return hipGetLastError();
}

hipError_t fill_assemble(const uint32_t* cpix, int N, int W, int P, const int* label,
                         const uint8_t* ebits, const float* nt, const float* om_r, const float* om_d,
                         const int* pos, double g2fx, double g2fy, float4* cst, float* rhs, float* dinv,
                         hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_assemble<<<ni::ceil_div(N, 256), 256, 0, st>>>(cpix, N, W, P, label, ebits, nt, om_r, om_d, pos, g2fx,
                                                   g2fy, cst, rhs, dinv);
  return hipGetLastError();
}

// list of the components of one size tier (ascending id); count -> *count_dev
hipError_t fill_tier_list(const int* comp_off, int K, int tier, int* flag, int* pos, int* list, int* count_dev,
                          int* scan_tmp, hipStream_t st) {
  if (K <= 0) return hipMemsetAsync(count_dev, 0, sizeof(int), st);
  int nb = ni::ceil_div(K, 256);
  k_tier_flags<<<nb, 256, 0, st>>>(comp_off, K, tier, flag);
  hipError_t e = scan_exclusive_i32(flag, pos, K, count_dev, scan_tmp, st);
  if (e != hipSuccess) return e;
  k_tier_list<<<nb, 256, 0, st>>>(flag, pos, K, list);
  return hipGetLastError();
}

// chunk table of the large components; total chunks -> *count_dev
hipError_t fill_chunks(const int* comp_off, int K, int chunk, int* nchunk, int* cbase, int* count_dev, int* scan_tmp,
                       hipStream_t st) {
  if (K <= 0) return hipMemsetAsync(count_dev, 0, sizeof(int), st);
  k_chunk_counts<<<ni::ceil_div(K, 256), 256, 0, st>>>(comp_off, K, chunk > 0 ? chunk : LCH, LMAXCH, LNT, nchunk);
  return scan_exclusive_i32(nchunk, cbase, K, count_dev, scan_tmp, st);
}

hipError_t fill_chunk_table(const int* comp_off, const int* nchunk, const int* cbase, int K, int chunk, int* chunk_comp,
                            int* chunk_start, int* chunk_end, hipStream_t st) {
  if (K <= 0) return hipSuccess;
  k_chunk_table<<<ni::ceil_div(K, 256), 256, 0, st>>>(comp_off, nchunk, cbase, K, chunk > 0 ? chunk : LCH, LMAXCH,
                                                      LNT, chunk_comp,
                                                      chunk_start, chunk_end);
  return hipGetLastError();
}

hipError_t fill_zero_grid(float* z, int P, hipStream_t st) {
  k_zero_grid<<<ni::ceil_div(P, 256), 256, 0, st>>>(z, P);
  return hipGetLastError();
}

hipError_t fill_gather_x0(const uint32_t* cpix, int N, const float* x0g, float* x, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_gather_x0<<<ni::ceil_div(N, 256), 256, 0, st>>>(cpix, N, x0g, x);
  return hipGetLastError();
}

hipError_t fill_small(int tier, const int* list, int n, const int* comp_off, const float4* cst, const float* rhs,
                      const float* dinv,
                      const float* x0, const uint32_t* cpix, float* zgrid, double rtol, int maxit, int warm,
                      int* iters, double* relres, int* stats, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (tier == 1)
    k_fill_small<64, 4><<<n, 64, 0, st>>>(list, comp_off, cst, rhs, dinv, x0, cpix, zgrid, rtol,
                                          maxit, warm, iters, relres, stats);
  else if (tier == 2)
    k_fill_small<256, 8><<<n, 256, 0, st>>>(list, comp_off, cst, rhs, dinv, x0, cpix, zgrid, rtol,
                                            maxit, warm, iters, relres, stats);
  else
    k_fill_small<1024, 8><<<n, 1024, 0, st>>>(list, comp_off, cst, rhs, dinv, x0, cpix, zgrid,
                                              rtol, maxit, warm, iters, relres, stats);
  return hipGetLastError();
}

static LargeState to_state(const LargeArgs& a) {
  LargeState S;
  S.comp_off = a.comp_off; S.cbase = a.cbase; S.nchunk = a.nchunk; S.chunk_comp = a.chunk_comp;
  S.chunk_start = a.chunk_start; S.chunk_end = a.chunk_end; S.part = a.part; S.gam = a.gam; S.tol2 = a.tol2;
  S.rr = a.rr; S.bb = a.bb; S.iters = a.iters; S.active = a.active; S.stats = a.stats;
  S.cst = a.cst; S.rhs = a.rhs; S.dinv = a.dinv;
  S.x = a.x; S.p = a.p; S.r0 = a.r0; S.r1 = a.r1; S.w0 = a.w0; S.w1 = a.w1; S.s0 = a.s0; S.s1 = a.s1;
  S.nchunks = a.nchunks; S.rtol = a.rtol; S.maxit = a.maxit;
  return S;
}

hipError_t large_init(const LargeArgs& a, int warm, hipStream_t st) {
  LargeState S = to_state(a);
  if (warm) {
    // centre the learned start on each component: only differences matter
    k_lg_sum<<<a.nchunks, LNT, 0, st>>>(S, 0);
    k_lg_center<<<a.nchunks, LNT, 0, st>>>(S, 0, nullptr, nullptr);
  }
  k_lg_init_a<<<a.nchunks, LNT, 0, st>>>(S);
  k_lg_init_b<<<a.nchunks, LNT, 0, st>>>(S, warm);
  return hipGetLastError();
}

// one CG iteration = launches A_it and B_it
hipError_t large_iter(const LargeArgs& a, int it, hipStream_t st) {
  LargeState S = to_state(a);
  if (a.split) {
    k_lg_p<<<a.nchunks, LNT, 0, st>>>(S, it, a.K);
    k_lg_q<<<a.nchunks, LNT, 0, st>>>(S, it, a.K);
  } else {
    k_lg_a<<<a.nchunks, LNT, 0, st>>>(S, it, a.K);
  }
  k_lg_b<<<a.nchunks, LNT, 0, st>>>(S, it, a.K);
  return hipGetLastError();
}

hipError_t mg_count(int N, const float4* cst, const uint32_t* skey, const int* comp_off, int* deg, int* npair,
                    hipStream_t st) {
  if (N > 0) k_mg_count<<<ni::ceil_div(N, 256), 256, 0, st>>>(N, cst, skey, comp_off, fill_small_cap(), deg, npair);
  return hipGetLastError();
}

hipError_t mg_build(int N, int W, const float4* cst, const float* rhs, const float* x32, const uint32_t* cpix,
                    const uint32_t* skey, const int* comp_off, const int* row_off, const int* pair_off, int* col,
                    double* w, double* diag, int* plo, int* phi, double* pw, int* gy, int* gx, int* gc, double* b64,
                    double* x64, hipStream_t st) {
  if (N > 0)
    k_mg_build<<<ni::ceil_div(N, 256), 256, 0, st>>>(N, W, cst, rhs, x32, cpix, skey, comp_off, fill_small_cap(),
                                                     row_off, pair_off, col, w, diag, plo, phi, pw, gy, gx, gc, b64,
                                                     x64);
  return hipGetLastError();
}

hipError_t mg_out(int N, const uint32_t* skey, const int* comp_off, const double* x64, float* x32, hipStream_t st) {
  if (N > 0) k_mg_out<<<ni::ceil_div(N, 256), 256, 0, st>>>(N, skey, comp_off, fill_small_cap(), x64, x32);
  return hipGetLastError();
}

// zero mean per large component of the start (a learned start: only
// differences matter)
hipError_t large_center(const LargeArgs& a, hipStream_t st) {
  LargeState S = to_state(a);
  k_lg_sum<<<a.nchunks, LNT, 0, st>>>(S, 0);
  k_lg_center<<<a.nchunks, LNT, 0, st>>>(S, 0, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t large_finish(const LargeArgs& a, const uint32_t* cpix, float* zgrid, hipStream_t st) {
  LargeState S = to_state(a);
  k_lg_sum<<<a.nchunks, LNT, 0, st>>>(S, 0);
  k_lg_center<<<a.nchunks, LNT, 0, st>>>(S, 0, zgrid, cpix);
  return hipGetLastError();
}

hipError_t fill8_count(int N, int W, const uint32_t* cpix, const uint32_t* skey, const int* comp_off,
                       const int* label, const uint8_t* eb, const uint8_t* eb2, int* deg, int* npair,
                       hipStream_t st) {
  (void)skey;
  (void)comp_off;
  if (N > 0) k_fill8_count<<<ni::ceil_div(N, 256), 256, 0, st>>>(N, W, cpix, label, eb, eb2, deg, npair);
  return hipGetLastError();
}

hipError_t fill8_build(int N, int W, const uint32_t* cpix, const uint32_t* skey, const int* comp_off,
                       const int* label, const uint8_t* eb, const uint8_t* eb2, const float* nt,
                       const float* const* om, const int* pos, double g2fx, double g2fy, double g2fd,
                       const int* row_off, const int* pair_off, const float* x32, int* col, double* w, double* diag,
                       int* plo, int* phi, double* pw, int* gy, int* gx, int* gc, double* b64, double* x64,
                       hipStream_t st) {
  const Om4 o{{om[0], om[1], om[2], om[3]}};
  if (N > 0)
    k_fill8_build<<<ni::ceil_div(N, 256), 256, 0, st>>>(N, W, cpix, skey, comp_off, label, eb, eb2, nt, o, pos, g2fx,
                                                        g2fy, g2fd, row_off, pair_off, x32, col, w, diag, plo, phi,
                                                        pw, gy, gx, gc, b64, x64);
  return hipGetLastError();
}

// per-component sums of the solution (run_sums over the component-major
// order), then the centred output
hipError_t fill8_out(int N, int K, const uint32_t* cpix, const uint32_t* skey, const int* comp_off,
                     const double* x64, double* csum, void* rtmp, float* z, hipStream_t st) {
  if (N <= 0 || K <= 0) return hipSuccess;
  hipError_t e = run_sums(skey, x64, N, csum, rtmp, st);
  if (e != hipSuccess) return e;
  k_fill8_out<<<ni::ceil_div(N, 256), 256, 0, st>>>(N, cpix, skey, comp_off, x64, csum, z);
  return hipGetLastError();
}

}  // namespace nil
