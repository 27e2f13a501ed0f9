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
                           double g2fy, float* __restrict__ cwr, float* __restrict__ cwd,
                           float* __restrict__ cwu, uint32_t* __restrict__ coff,
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
  cwr[i] = fr;
  cwd[i] = fd;
  cwu[i] = fu;
  coff[i] = ou | (od << 16);
  rhs[i] = (float)b;
  double dg = (double)fr + (double)fl + (double)fd + (double)fu;
  dinv[i] = dg > 0 ? (float)(1.0 / dg) : 0.f;
}

// n_c = comp_off[c+1] - comp_off[c]; flags: 1 small (2..cap), 2 large (> cap)
__global__ void k_classify(const int* __restrict__ comp_off, int K, int cap, int* __restrict__ fsmall,
                           int* __restrict__ flarge, int* __restrict__ nchunk, int chunk) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  int n = comp_off[c + 1] - comp_off[c];
  fsmall[c] = (n >= 2 && n <= cap) ? 1 : 0;
  flarge[c] = n > cap ? 1 : 0;
  nchunk[c] = n > cap ? ni::ceil_div(n, chunk) : 0;
}

__global__ void k_make_lists(const int* __restrict__ fsmall, const int* __restrict__ flarge,
                             const int* __restrict__ spos, const int* __restrict__ lpos,
                             const int* __restrict__ nchunk, const int* __restrict__ cbase,
                             const int* __restrict__ comp_off, int K, int chunk,
                             int* __restrict__ small_list, int* __restrict__ large_list,
                             int* __restrict__ chunk_comp, int* __restrict__ chunk_start) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  if (fsmall[c]) small_list[spos[c]] = c;
  if (flarge[c]) {
    large_list[lpos[c]] = c;
    for (int j = 0; j < nchunk[c]; ++j) {
      chunk_comp[cbase[c] + j] = c;
      chunk_start[cbase[c] + j] = comp_off[c] + j * chunk;
    }
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

__device__ __forceinline__ Stencil load_stencil(const float* __restrict__ cwr, const float* __restrict__ cwd,
                                                const float* __restrict__ cwu,
                                                const uint32_t* __restrict__ coff, int i, int lo) {
  Stencil s;
  s.wr = cwr[i];
  s.wl = i > lo ? cwr[i - 1] : 0.f;
  s.wd = cwd[i];
  s.wu = cwu[i];
  uint32_t o = coff[i];
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
    const int* __restrict__ list, const int* __restrict__ comp_off, const float* __restrict__ cwr,
    const float* __restrict__ cwd, const float* __restrict__ cwu, const uint32_t* __restrict__ coff,
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
      Stencil s = load_stencil(cwr, cwd, cwu, coff, lo + j, lo);
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
// Components above the LDS capacity are cut into chunks of CH pixels; a
// workgroup handles one chunk per phase.  Per-component scalars come from a
// deterministic two-level reduction: every chunk writes its FP64 partials,
// the last chunk to arrive (atomic counter) sums them in chunk order.
constexpr int LNT = 256, LPPT = 8, LCH = LNT * LPPT;

struct LargeState {
  // per component
  const int* comp_off;
  const int* cbase;     // first chunk of the component
  const int* nchunk;
  int* cnt;             // arrival counters (reset by the last arriver)
  double* part;         // [nchunks_total * 4]
  double* rho;
  double* bb;
  double* tol2;
  double* alpha;
  double* beta;
  double* rr;
  int* done;
  int* iters;
  int* active;          // number of components not yet converged
  int* stats;           // [0] not converged, [1] warm fallbacks
  // per chunk
  const int* chunk_comp;
  const int* chunk_start;
  // per compact pixel
  const float *cwr, *cwd, *cwu, *rhs, *dinv;
  const uint32_t* coff;
  float *x, *r, *z, *p0, *p1, *q;
  double rtol;
  int maxit;
};

// sums NV partials of component c in chunk order with the whole block;
// called by the block that arrived last; result in every thread
template <int NV>
__device__ __forceinline__ void reduce_parts(const LargeState& S, int c, double (&v)[NV], double* scratch) {
  const int base = S.cbase[c], nch = S.nchunk[c];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int j = threadIdx.x; j < nch; j += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += S.part[(size_t)(base + j) * 4 + k];
  }
  ni::block_sum<NV>(v, scratch);
}

// write partials, count arrival; returns true in every thread of the last block
template <int NV>
__device__ __forceinline__ bool arrive(const LargeState& S, int c, int ch, const double (&v)[NV], int* flag) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) S.part[(size_t)ch * 4 + k] = v[k];
    __threadfence();
    int old = atomicAdd(&S.cnt[c], 1);
    *flag = (old == S.nchunk[c] - 1);
  }
  __syncthreads();
  bool last = *flag;
  if (last) __threadfence();
  return last;
}

// phase 0 (warm start only): mean of x0 per component
__global__ void __launch_bounds__(LNT) k_large_mean(LargeState S, float* x, int apply_mean) {
  __shared__ double red[4 * (LNT / 64)];
  __shared__ int flag;
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int hi = S.comp_off[c + 1];
  double v[1] = {0.0};
  for (int k = 0; k < LPPT; ++k) {
    int i = lo + threadIdx.x + k * LNT;
    if (i < hi) v[0] += x[i];
  }
  ni::block_sum<1>(v, red);
  if (arrive<1>(S, c, ch, v, &flag)) {
    double t[1];
    reduce_parts<1>(S, c, t, red + 2 * (LNT / 64));
    if (threadIdx.x == 0) {
      S.alpha[c] = t[0] / (double)(hi - S.comp_off[c]);  // alpha[] doubles as scratch here
      S.cnt[c] = 0;
    }
  }
}

__global__ void __launch_bounds__(LNT) k_large_center(LargeState S, float* x) {
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int hi = S.comp_off[c + 1];
  const float m = (float)S.alpha[c];
  for (int k = 0; k < LPPT; ++k) {
    int i = lo + threadIdx.x + k * LNT;
    if (i < hi) x[i] -= m;
  }
}

// init: r = b - L x, z = D^-1 r, p_old = 0; partials rr, rz, bb.
// With check_warm, only decides per component whether the start is kept
// (rr < bb) and otherwise zeroes x.
__global__ void __launch_bounds__(LNT) k_large_init(LargeState S, int check_warm) {
  __shared__ double red[6 * (LNT / 64)];
  __shared__ int flag;
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int clo = S.comp_off[c], hi = S.comp_off[c + 1];
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < LPPT; ++k) {
    int i = lo + threadIdx.x + k * LNT;
    if (i >= hi) continue;
    Stencil s = load_stencil(S.cwr, S.cwd, S.cwu, S.coff, i, clo);
    float xi = S.x[i];
    float q = 0.f;
    if (s.wr != 0.f) q += s.wr * (xi - S.x[i + 1]);
    if (s.wl != 0.f) q += s.wl * (xi - S.x[i - 1]);
    if (s.wd != 0.f) q += s.wd * (xi - S.x[i + s.od]);
    if (s.wu != 0.f) q += s.wu * (xi - S.x[i - s.ou]);
    float b = S.rhs[i];
    float ri = b - q;
    float zi = S.dinv[i] * ri;
    if (!check_warm) {
      S.r[i] = ri;
      S.z[i] = zi;
      S.p0[i] = 0.f;
      S.p1[i] = 0.f;
    }
    v[0] += (double)ri * ri;
    v[1] += (double)ri * zi;
    v[2] += (double)b * b;
  }
  ni::block_sum<3>(v, red);
  if (arrive<3>(S, c, ch, v, &flag)) {
    double t[3];
    reduce_parts<3>(S, c, t, red + 3 * (LNT / 64));
    if (threadIdx.x == 0) {
      S.cnt[c] = 0;
      if (check_warm) {
        S.beta[c] = (t[0] < t[2]) ? 1.0 : 0.0;  // keep the start?
        if (!(t[0] < t[2])) atomicAdd(&S.stats[1], 1);
      } else {
        S.bb[c] = t[2];
        S.tol2[c] = S.rtol * S.rtol * t[2];
        S.rho[c] = t[1];
        S.rr[c] = t[0];
        S.beta[c] = 0.0;
        S.iters[c] = 0;
        int d = (t[2] == 0.0) || (t[0] <= S.tol2[c]);
        S.done[c] = d;
        if (!d) atomicAdd(S.active, 1);
      }
    }
  }
}

__global__ void __launch_bounds__(LNT) k_large_reset(LargeState S) {
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int hi = S.comp_off[c + 1];
  if (S.beta[c] != 0.0) return;
  for (int k = 0; k < LPPT; ++k) {
    int i = lo + threadIdx.x + k * LNT;
    if (i < hi) S.x[i] = 0.f;
  }
}

// Phase A: p_new = z + beta p_old (also at the neighbours, recomputed),
// q = L p_new, partial p.q; the last chunk sets alpha = rho / p.q.
__device__ __forceinline__ void phase_a(const LargeState& S, int ch, const float* __restrict__ pold,
                                        float* __restrict__ pnew, double* red, int* flag) {
  const int c = S.chunk_comp[ch];
  if (S.done[c]) return;
  const int lo = S.chunk_start[ch], clo = S.comp_off[c], hi = S.comp_off[c + 1];
  const float beta = (float)S.beta[c];
  double v[1] = {0.0};
  for (int k = 0; k < LPPT; ++k) {
    int i = lo + threadIdx.x + k * LNT;
    if (i >= hi) continue;
    Stencil s = load_stencil(S.cwr, S.cwd, S.cwu, S.coff, i, clo);
    const float pi = S.z[i] + beta * pold[i];
    float q = 0.f;
    if (s.wr != 0.f) q += s.wr * (pi - (S.z[i + 1] + beta * pold[i + 1]));
    if (s.wl != 0.f) q += s.wl * (pi - (S.z[i - 1] + beta * pold[i - 1]));
    if (s.wd != 0.f) q += s.wd * (pi - (S.z[i + s.od] + beta * pold[i + s.od]));
    if (s.wu != 0.f) q += s.wu * (pi - (S.z[i - s.ou] + beta * pold[i - s.ou]));
    pnew[i] = pi;
    S.q[i] = q;
    v[0] += (double)pi * q;
  }
  ni::block_sum<1>(v, red);
  if (arrive<1>(S, c, ch, v, flag)) {
    double t[1];
    reduce_parts<1>(S, c, t, red + 4 * (LNT / 64));
    if (threadIdx.x == 0) {
      S.alpha[c] = S.rho[c] / t[0];
      S.cnt[c] = 0;
    }
  }
}

// Phase B: x += alpha p, r -= alpha q, z = D^-1 r; partials rr, rz; the
// last chunk sets beta = rz_new / rz and retires converged components.
__device__ __forceinline__ void phase_b(const LargeState& S, int ch, const float* __restrict__ pnew,
                                        double* red, int* flag) {
  const int c = S.chunk_comp[ch];
  if (S.done[c]) return;
  const int lo = S.chunk_start[ch], hi = S.comp_off[c + 1];
  const float alpha = (float)S.alpha[c];
  double v[2] = {0.0, 0.0};
  for (int k = 0; k < LPPT; ++k) {
    int i = lo + threadIdx.x + k * LNT;
    if (i >= hi) continue;
    float xi = S.x[i] + alpha * pnew[i];
    float ri = S.r[i] - alpha * S.q[i];
    float zi = S.dinv[i] * ri;
    S.x[i] = xi;
    S.r[i] = ri;
    S.z[i] = zi;
    v[0] += (double)ri * ri;
    v[1] += (double)ri * zi;
  }
  ni::block_sum<2>(v, red);
  if (arrive<2>(S, c, ch, v, flag)) {
    double t[2];
    reduce_parts<2>(S, c, t, red + 4 * (LNT / 64));
    if (threadIdx.x == 0) {
      S.cnt[c] = 0;
      int it = S.iters[c] + 1;
      S.iters[c] = it;
      S.beta[c] = t[1] / S.rho[c];
      S.rho[c] = t[1];
      S.rr[c] = t[0];
      if (t[0] <= S.tol2[c] || it >= S.maxit) {
        S.done[c] = 1;
        atomicSub(S.active, 1);
        if (t[0] > S.tol2[c]) atomicAdd(&S.stats[0], 1);
      }
    }
  }
}

__global__ void __launch_bounds__(LNT) k_large_a(LargeState S, int parity) {
  __shared__ double red[6 * (LNT / 64)];
  __shared__ int flag;
  phase_a(S, blockIdx.x, parity ? S.p1 : S.p0, parity ? S.p0 : S.p1, red, &flag);
}

__global__ void __launch_bounds__(LNT) k_large_b(LargeState S, int parity) {
  __shared__ double red[6 * (LNT / 64)];
  __shared__ int flag;
  phase_b(S, blockIdx.x, parity ? S.p0 : S.p1, red, &flag);
}

// One persistent, cooperatively launched grid runs every CG iteration of
// every large component: the workgroups stride over the chunks of the
// components still active, with a grid barrier after each phase.
__global__ void __launch_bounds__(LNT) k_large_persistent(LargeState S, int nchunks, unsigned* bar) {
  __shared__ double red[6 * (LNT / 64)];
  __shared__ int flag;
  const unsigned nb = gridDim.x;
  for (int it = 0;; ++it) {
    // every block reads the same counter between two barriers: uniform exit
    if (__hip_atomic_load(S.active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0) break;
    const int par = it & 1;
    const float* pold = par ? S.p1 : S.p0;
    float* pnew = par ? S.p0 : S.p1;
    for (int ch = blockIdx.x; ch < nchunks; ch += nb) phase_a(S, ch, pold, pnew, red, &flag);
    ni::grid_barrier(bar, nb);
    for (int ch = blockIdx.x; ch < nchunks; ch += nb) phase_b(S, ch, pnew, red, &flag);
    ni::grid_barrier(bar, nb);
  }
}

// zero mean per component and scatter to the grid (two kernels)
__global__ void __launch_bounds__(LNT) k_large_out(LargeState S, const uint32_t* __restrict__ cpix,
                                                   float* __restrict__ zgrid) {
  const int ch = blockIdx.x, c = S.chunk_comp[ch], lo = S.chunk_start[ch];
  const int hi = S.comp_off[c + 1];
  const double m = S.alpha[c];
  for (int k = 0; k < LPPT; ++k) {
    int i = lo + threadIdx.x + k * LNT;
    if (i < hi) zgrid[cpix[i]] = (float)((double)S.x[i] - m);
  }
}

__global__ void k_zero_grid(float* z, int P) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) z[p] = 0.f;
}

}  // namespace

namespace nil {

// capacity of the LDS-resident path
constexpr int SMALL_NT = 256, SMALL_PPT = 8, SMALL_CAP = SMALL_NT * SMALL_PPT;
constexpr int TINY_NT = 64, TINY_PPT = 4, TINY_CAP = TINY_NT * TINY_PPT;

int fill_small_cap() { return SMALL_CAP; }

hipError_t check_labels(const int* label, const uint8_t* ebits, int P, int K, int* bad, hipStream_t st) {
  k_check_labels<<<ni::ceil_div(P, 256), 256, 0, st>>>(label, ebits, P, K, bad);
  return hipGetLastError();
}

hipError_t check_ids(const uint32_t* skey, int N, int K, int* bad, hipStream_t st) {
  if (N > 0) k_check_ids<<<ni::ceil_div(N, 256), 256, 0, st>>>(skey, N, K, bad);
  return hipGetLastError();
}
int fill_chunk() { return LCH; }

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
                         const int* pos, double g2fx, double g2fy, float* cwr, float* cwd, float* cwu,
                         uint32_t* coff, float* rhs, float* dinv, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  k_assemble<<<ni::ceil_div(N, 256), 256, 0, st>>>(cpix, N, W, P, label, ebits, nt, om_r, om_d, pos, g2fx,
                                                   g2fy, cwr, cwd, cwu, coff, rhs, dinv);
  return hipGetLastError();
}

// builds small / large component lists and the chunk table; counts land in
// counts_dev[0] = n_small, [1] = n_large, [2] = n_chunks (device)
hipError_t fill_classify(const int* comp_off, int K, int* fsmall, int* flarge, int* nchunk, int* spos,
                         int* lpos, int* cbase, int* counts_dev, int* scan_tmp, hipStream_t st) {
  if (K <= 0) return hipMemsetAsync(counts_dev, 0, 3 * sizeof(int), st);
  k_classify<<<ni::ceil_div(K, 256), 256, 0, st>>>(comp_off, K, SMALL_CAP, fsmall, flarge, nchunk, LCH);
  hipError_t e = scan_exclusive_i32(fsmall, spos, K, counts_dev + 0, scan_tmp, st);
  if (e != hipSuccess) return e;
  e = scan_exclusive_i32(flarge, lpos, K, counts_dev + 1, scan_tmp, st);
  if (e != hipSuccess) return e;
  return scan_exclusive_i32(nchunk, cbase, K, counts_dev + 2, scan_tmp, st);
}

hipError_t fill_lists(const int* fsmall, const int* flarge, const int* spos, const int* lpos,
                      const int* nchunk, const int* cbase, const int* comp_off, int K, int* small_list,
                      int* large_list, int* chunk_comp, int* chunk_start, hipStream_t st) {
  if (K <= 0) return hipSuccess;
  k_make_lists<<<ni::ceil_div(K, 256), 256, 0, st>>>(fsmall, flarge, spos, lpos, nchunk, cbase, comp_off, K,
                                                     LCH, small_list, large_list, chunk_comp, chunk_start);
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

hipError_t fill_small(const int* list, int n_small, const int* comp_off, const float* cwr, const float* cwd,
                      const float* cwu, const uint32_t* coff, const float* rhs, const float* dinv,
                      const float* x0, const uint32_t* cpix, float* zgrid, double rtol, int maxit, int warm,
                      int* iters, double* relres, int* stats, hipStream_t st) {
  if (n_small <= 0) return hipSuccess;
  k_fill_small<SMALL_NT, SMALL_PPT><<<n_small, SMALL_NT, 0, st>>>(
      list, comp_off, cwr, cwd, cwu, coff, rhs, dinv, x0, cpix, zgrid, rtol, maxit, warm, iters, relres, stats);
  return hipGetLastError();
}

struct LargeArgs {
  const int *comp_off, *cbase, *nchunk, *chunk_comp, *chunk_start;
  int* cnt;
  double *part, *rho, *bb, *tol2, *alpha, *beta, *rr;
  int *done, *iters, *active, *stats;
  const float *cwr, *cwd, *cwu, *rhs, *dinv;
  const uint32_t* coff;
  float *x, *r, *z, *p0, *p1, *q;
  double rtol;
  int maxit;
};

static LargeState to_state(const LargeArgs& a) {
  LargeState S;
  S.comp_off = a.comp_off; S.cbase = a.cbase; S.nchunk = a.nchunk; S.cnt = a.cnt; S.part = a.part;
  S.rho = a.rho; S.bb = a.bb; S.tol2 = a.tol2; S.alpha = a.alpha; S.beta = a.beta; S.rr = a.rr;
  S.done = a.done; S.iters = a.iters; S.active = a.active; S.stats = a.stats;
  S.chunk_comp = a.chunk_comp; S.chunk_start = a.chunk_start;
  S.cwr = a.cwr; S.cwd = a.cwd; S.cwu = a.cwu; S.rhs = a.rhs; S.dinv = a.dinv; S.coff = a.coff;
  S.x = a.x; S.r = a.r; S.z = a.z; S.p0 = a.p0; S.p1 = a.p1; S.q = a.q;
  S.rtol = a.rtol; S.maxit = a.maxit;
  return S;
}

hipError_t large_init(const LargeArgs& a, int nchunks, int warm, hipStream_t st) {
  LargeState S = to_state(a);
  if (warm) {
    k_large_mean<<<nchunks, LNT, 0, st>>>(S, S.x, 1);
    k_large_center<<<nchunks, LNT, 0, st>>>(S, S.x);
    k_large_init<<<nchunks, LNT, 0, st>>>(S, 1);
    k_large_reset<<<nchunks, LNT, 0, st>>>(S);
  }
  k_large_init<<<nchunks, LNT, 0, st>>>(S, 0);
  return hipGetLastError();
}

hipError_t large_step(const LargeArgs& a, int nchunks, int parity, hipStream_t st) {
  LargeState S = to_state(a);
  k_large_a<<<nchunks, LNT, 0, st>>>(S, parity);
  k_large_b<<<nchunks, LNT, 0, st>>>(S, parity);
  return hipGetLastError();
}

int large_persistent_blocks(int device) {
  int per_cu = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_large_persistent, LNT, 0) != hipSuccess)
    return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return per_cu * ncu;
}

hipError_t large_persistent(const LargeArgs& a, int nchunks, int nblocks, unsigned* bar, hipStream_t st) {
  LargeState S = to_state(a);
  void* args[] = {(void*)&S, (void*)&nchunks, (void*)&bar};
  return hipLaunchCooperativeKernel((const void*)k_large_persistent, dim3(nblocks), dim3(LNT), args, 0, st);
}

hipError_t large_finish(const LargeArgs& a, int nchunks, const uint32_t* cpix, float* zgrid, hipStream_t st) {
  LargeState S = to_state(a);
  k_large_mean<<<nchunks, LNT, 0, st>>>(S, S.x, 0);
  k_large_out<<<nchunks, LNT, 0, st>>>(S, cpix, zgrid);
  return hipGetLastError();
}

}  // namespace nil
