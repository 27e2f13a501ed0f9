// Relative-scale optimisation on the quotient graph (Sec. 3.4, Eq. 10-12,
// 16-19; the main loop of Alg. 1 without merging).
//
// Structure (built once per partition): the inter-component edges E_inter
// sorted by their component pair (lo, hi), lo < hi; the distinct pairs;
// and a K-row CSR of the quotient Laplacian whose entries point at pairs.
// Per iteration t (all FP64):
//   r_e   = z_a - z_b - omega_{b->a}, z = zfill + S_pi          (Eq. 11)
//   w_e   = W_{b->a} + W_{a->b}: 2 in the alignment iterations, else
//           gamma^2 sigma_k(gamma^2 ((z_{-b}-z_a)^2 - (z_b-z_a)^2)) W^out
//           per directed row                                   (Eq. 5-7, 18-19)
//   edges lighter than w_cut_rel * max_e w_e are dropped;
//   quotient Laplacian sum_e w_e (e_lo - e_hi)(e_lo - e_hi)^T, rhs
//   -sum_e w_e rho_e (e_lo - e_hi) with rho_e the residual oriented lo->hi;
//   s = PCG solution, shifted to zero mean on every connected piece;
//   E_t = sum_e w_e (rho_e + s_lo - s_hi)^2; S += s            (Eq. 12, 17)
#include "ni_common.h"

namespace {

__global__ void k_inter_flags(const int* __restrict__ label, const uint8_t* __restrict__ ebits, int P, int W,
                              int* __restrict__ flag) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  uint8_t e = ebits[p];
  int c = label[p];
  flag[2 * p] = ((e & EB_VR) && label[p + 1] != c) ? 1 : 0;
  flag[2 * p + 1] = ((e & EB_VD) && label[p + W] != c) ? 1 : 0;
}

__global__ void k_inter_compact(const int* __restrict__ flag, const int* __restrict__ epos, int P2,
                                uint32_t* __restrict__ eidx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P2 && flag[i]) eidx[epos[i]] = (uint32_t)i;
}

__device__ __forceinline__ void edge_ends(uint32_t code, int W, int& a, int& b, bool& horiz) {
  a = (int)(code >> 1);
  horiz = (code & 1u) == 0u;
  b = horiz ? a + 1 : a + W;
}

// key = max(pi(a), pi(b)) (which = 1) or min (which = 0)
__global__ void k_edge_keys(const uint32_t* __restrict__ eidx, int E, int W, const int* __restrict__ label,
                            int which, uint32_t* __restrict__ key) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  int a, b;
  bool h;
  edge_ends(eidx[i], W, a, b, h);
  int c = label[a], d = label[b];
  key[i] = (uint32_t)(which ? max(c, d) : min(c, d));
}

__global__ void k_pair_flags(const uint32_t* __restrict__ eidx, int E, int W, const int* __restrict__ label,
                             int* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  int a, b, a0, b0;
  bool h;
  edge_ends(eidx[i], W, a, b, h);
  int f = 1;
  if (i > 0) {
    edge_ends(eidx[i - 1], W, a0, b0, h);
    int c = label[a], d = label[b], c0 = label[a0], d0 = label[b0];
    f = (min(c, d) != min(c0, d0) || max(c, d) != max(c0, d0)) ? 1 : 0;
  }
  flag[i] = f;
}

__global__ void k_pair_build(const uint32_t* __restrict__ eidx, const int* __restrict__ flag,
                             const int* __restrict__ ppos, int E, int W, const int* __restrict__ label,
                             int* __restrict__ pair_start, int* __restrict__ pair_lo, int* __restrict__ pair_hi,
                             int npairs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  if (flag[i]) {
    int a, b;
    bool h;
    edge_ends(eidx[i], W, a, b, h);
    int c = label[a], d = label[b];
    int pid = ppos[i];
    pair_start[pid] = i;
    pair_lo[pid] = min(c, d);
    pair_hi[pid] = max(c, d);
  }
  if (i == E - 1) pair_start[npairs] = E;
}

// CSR entry e in [0, 2P): pair e>>1, row = lo (e even) or hi (e odd)
__global__ void k_entry_keys(const int* __restrict__ pair_lo, const int* __restrict__ pair_hi, int P2, int by_row,
                             const uint32_t* __restrict__ ent, uint32_t* __restrict__ key) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P2) return;
  uint32_t e = ent ? ent[i] : (uint32_t)i;
  int pid = (int)(e >> 1);
  bool odd = e & 1u;
  int row = odd ? pair_hi[pid] : pair_lo[pid];
  int col = odd ? pair_lo[pid] : pair_hi[pid];
  key[i] = (uint32_t)(by_row ? row : col);
}

__global__ void k_row_count(const int* __restrict__ pair_lo, const int* __restrict__ pair_hi, int P,
                            int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  atomicAdd(&cnt[pair_lo[i]], 1);
  atomicAdd(&cnt[pair_hi[i]], 1);
}

__global__ void k_fill_i32(int* a, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_iota_u32(uint32_t* a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (uint32_t)i;
}

__global__ void k_fill_f64(double* a, int n, double v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ---------------------------------------------------------- per iteration
struct EdgeParams {
  int W, align, outlier_mode, t;
  double g2fx, g2fy, k, lL, lU, U;
};

__device__ __forceinline__ double sigmoid_k(double x, double k) { return 1.0 / (1.0 + exp(-k * x)); }

__device__ __forceinline__ double outlier_w(double chi, const EdgeParams& q) {
  chi = fabs(chi);
  if (q.outlier_mode == 0) return 1.0;
  if (q.outlier_mode == 2) return chi < q.U ? 1.0 : 0.0;
  if (chi == 0.0) return 1.0;
  double arg = 4.0 / (q.lL - q.lU) * (2.0 * log10(chi) - (q.lL + q.lU));
  return 1.0 / (1.0 + exp(-arg));
}

__global__ void __launch_bounds__(256) k_irls_edges(
    const uint32_t* __restrict__ eidx, int E, const int* __restrict__ label, const uint8_t* __restrict__ ebits,
    const float* __restrict__ nt, const float* __restrict__ om_r, const float* __restrict__ om_d,
    const float* __restrict__ zfill, const double* __restrict__ S, EdgeParams q, double* __restrict__ ew,
    double* __restrict__ erho, unsigned long long* __restrict__ wmax_bits) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double w = 0.0;
  if (i < E) {
    int a, b;
    bool h;
    edge_ends(eidx[i], q.W, a, b, h);
    const int c = label[a], d = label[b];
    const double za = (double)zfill[a] + S[c];
    const double zb = (double)zfill[b] + S[d];
    const double om = h ? (double)om_r[a] : (double)om_d[a];
    const double r = za - zb - om;
    if (q.t < q.align) {
      w = 2.0;
    } else {
      const int step = h ? 1 : q.W;
      const uint8_t bit = h ? EB_VR : EB_VD;
      const double g2f = h ? q.g2fx : q.g2fy;
      // row b -> a, opposite pixel a - step
      const bool has_ma = h ? (a % q.W) > 0 : a >= q.W;
      double dm = 0.0;
      if (has_ma && (ebits[a - step] & bit)) {
        int m = a - step;
        dm = ((double)zfill[m] + S[label[m]]) - za;
      }
      const double dp = zb - za;
      const double ta = nt[a];
      const double g2a = g2f * (ta * ta);
      const double wba = g2a * sigmoid_k(g2a * (dm * dm - dp * dp), q.k);
      // row a -> b, opposite pixel b + step
      double dm2 = 0.0;
      if (ebits[b] & bit) {
        int m = b + step;
        dm2 = ((double)zfill[m] + S[label[m]]) - zb;
      }
      const double dp2 = za - zb;
      const double tb = nt[b];
      const double g2b = g2f * (tb * tb);
      const double wab = g2b * sigmoid_k(g2b * (dm2 * dm2 - dp2 * dp2), q.k);
      w = (wba + wab) * outlier_w(r, q);
    }
    ew[i] = w;
    erho[i] = (c < d) ? r : -r;
  }
  // block max, one atomic per block (non-negative doubles order like their bits)
  __shared__ double bm[4];
  double m = w;
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) bm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = bm[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) mm = fmax(mm, bm[k]);
    atomicMax(wmax_bits, (unsigned long long)__double_as_longlong(mm));
  }
}

// per pair: apply the cut, sum weights and weighted residuals in edge order
__global__ void k_irls_pairs(const int* __restrict__ pair_start, int P, double* __restrict__ ew,
                             const double* __restrict__ erho, const unsigned long long* __restrict__ wmax_bits,
                             double cut_rel, double* __restrict__ pW, double* __restrict__ pB) {
  int pid = blockIdx.x * blockDim.x + threadIdx.x;
  if (pid >= P) return;
  const double cut = cut_rel * __longlong_as_double((long long)*wmax_bits);
  double Wp = 0.0, Bp = 0.0;
  for (int i = pair_start[pid]; i < pair_start[pid + 1]; ++i) {
    double w = ew[i];
    if (w < cut) {
      w = 0.0;
      ew[i] = 0.0;
    }
    Wp += w;
    Bp += w * erho[i];
  }
  pW[pid] = Wp;
  pB[pid] = Bp;
}

__global__ void k_irls_nodes(const int* __restrict__ row_off, const uint32_t* __restrict__ ent, int K,
                             const double* __restrict__ pW, const double* __restrict__ pB,
                             double* __restrict__ diag, double* __restrict__ rhs, double* __restrict__ babs) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  double dg = 0.0, b = 0.0, ba = 0.0;
  for (int j = row_off[c]; j < row_off[c + 1]; ++j) {
    uint32_t e = ent[j];
    int pid = (int)(e >> 1);
    dg += pW[pid];
    double v = (e & 1u) ? pB[pid] : -pB[pid];  // row = hi: +B, row = lo: -B
    b += v;
    ba += fabs(v);
  }
  diag[c] = dg;
  rhs[c] = b;
  babs[c] = ba;
}

// ------------------------------------------------------ quotient PCG (FP64)
// Matrix per iteration: qcol/qw = neighbour id and pair weight of every CSR
// entry, diag = row sum (pure graph Laplacian), applied in difference form
// q_c = sum_d w_cd (p_c - p_d).  Jacobi preconditioner; rows with diag = 0
// (components whose every quotient edge was cut) keep s = 0.
__global__ void k_q_matrix(const int* __restrict__ row_off, const uint32_t* __restrict__ ent,
                           const int* __restrict__ pair_lo, const int* __restrict__ pair_hi,
                           const double* __restrict__ pW, int nnz, int* __restrict__ qcol, double* __restrict__ qw) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nnz) return;
  uint32_t e = ent[j];
  int pid = (int)(e >> 1);
  qcol[j] = (e & 1u) ? pair_lo[pid] : pair_hi[pid];
  qw[j] = pW[pid];
}

struct QMat {
  const int* row_off;
  const int* qcol;
  const double* qw;
  const double* diag;
  const double* rhs;
  const double* babs;
  const int* heavy;   // rows with more than QHEAVY entries (one wavefront each)
  int nheavy;
  int K;
};

// rows with more entries than this are multiplied by a whole wavefront;
// the others by one thread each (quotient degrees are very uneven: a large
// component can border thousands of others while most border four)
constexpr int QHEAVY = 32;

__global__ void k_heavy_flags(const int* __restrict__ row_off, int K, int* __restrict__ flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K) flag[c] = (row_off[c + 1] - row_off[c]) > QHEAVY ? 1 : 0;
}

__global__ void k_heavy_list(const int* __restrict__ flag, const int* __restrict__ pos, int K, int* __restrict__ list) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K && flag[c]) list[pos[c]] = c;
}

// One workgroup of QWG threads owns every row (K <= QCAP): the search
// direction and the product L p live in LDS, so an iteration costs a few
// workgroup barriers and no global synchronisation.  The product is formed
// one row per wavefront (lanes stride over the row's entries): quotient
// rows are very uneven, a large component can border thousands of others.
constexpr int QWG = 1024, QR = 8, QCAP = QWG * QR, QNW = QWG / 64;

__global__ void __launch_bounds__(QWG) k_qcg_wg(QMat M, double* __restrict__ s, double* __restrict__ rv,
                                                double rtol, int maxit, int* __restrict__ iters_out) {
  __shared__ double pl[QCAP];
  __shared__ double ql[QCAP];
  __shared__ double red[2][3 * QNW];
  const int K = M.K;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v3[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < QR; ++k) {
    const int c = threadIdx.x + k * QWG;
    if (c < K) {
      const double b = M.rhs[c], dg = M.diag[c];
      const double z = dg > 0 ? b / dg : 0.0;
      s[c] = 0.0;
      rv[c] = b;
      pl[c] = z;
      v3[0] += b * b;
      v3[1] += b * z;
      v3[2] += M.babs[c] * M.babs[c];
    }
  }
  ni::block_sum<3>(v3, red[0]);
  double rr = v3[0], rho = v3[1];
  const double tol2 = rtol * rtol * v3[2];
  int it = 0;
  while (rr > tol2 && it < maxit) {
    double v1[1] = {0.0};
#pragma unroll
    for (int k = 0; k < QR; ++k) {
      const int c = threadIdx.x + k * QWG;
      if (c < K) {
        const int j0 = M.row_off[c], j1 = M.row_off[c + 1];
        if (j1 - j0 <= QHEAVY) {
          const double pc = pl[c];
          double acc = 0.0;
          for (int j = j0; j < j1; ++j) acc += M.qw[j] * (pc - pl[M.qcol[j]]);
          ql[c] = acc;
          v1[0] += pc * acc;
        }
      }
    }
    for (int h = wid; h < M.nheavy; h += QNW) {
      const int c = M.heavy[h];
      const double pc = pl[c];
      double acc = 0.0;
      for (int j = M.row_off[c] + lane; j < M.row_off[c + 1]; j += 64) acc += M.qw[j] * (pc - pl[M.qcol[j]]);
      acc = ni::wave_sum(acc);
      if (lane == 0) {
        ql[c] = acc;
        v1[0] += pc * acc;
      }
    }
    ni::block_sum<1>(v1, red[1]);
    const double alpha = rho / v1[0];
    double v2[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < QR; ++k) {
      const int c = threadIdx.x + k * QWG;
      if (c < K) {
        const double dg = M.diag[c];
        s[c] += alpha * pl[c];
        const double r = rv[c] - alpha * ql[c];
        rv[c] = r;
        const double z = dg > 0 ? r / dg : 0.0;
        v2[0] += r * r;
        v2[1] += r * z;
      }
    }
    ni::block_sum<2>(v2, red[0]);
    const double beta = v2[1] / rho;
    rr = v2[0];
    rho = v2[1];
#pragma unroll
    for (int k = 0; k < QR; ++k) {
      const int c = threadIdx.x + k * QWG;
      if (c < K) {
        const double dg = M.diag[c];
        pl[c] = (dg > 0 ? rv[c] / dg : 0.0) + beta * pl[c];
      }
    }
    __syncthreads();
    ++it;
  }
  if (threadIdx.x == 0) *iters_out = it;
}

// Larger quotient systems: Jacobi PCG with two launches per iteration over
// blocks of QB rows (one row per wavefront in the product).  Every block
// re-sums all blocks' FP64 partials of the previous launch in block order
// (deterministic, no atomics, no in-kernel fences); partial fields are
// (rho, rr, pq, bscale^2) and each launch copies the fields it does not own.
constexpr int QNT = 256, QB = 256;

struct QIter {
  QMat M;
  double *s, *p0, *p1, *r, *q;
  double* part;   // [2][nblk][4]
  double* sc;     // [2] rho by iteration parity
  int* flag;      // [2] still iterating, by iteration parity
  int nblk;
  double rtol;
  int maxit;
  int* iters_out;
};

__device__ __forceinline__ void q_partials(const QIter& Q, int slot, double (&v)[4], double* red) {
  const double* pp = Q.part + (size_t)slot * Q.nblk * 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = 0.0;
  for (int j = threadIdx.x; j < Q.nblk; j += blockDim.x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += pp[(size_t)j * 4 + k];
  }
  ni::block_sum<4>(v, red);
}

__device__ __forceinline__ void q_put(const QIter& Q, int wslot, const double* v, int mask) {
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    const size_t dst = ((size_t)wslot * Q.nblk + blockIdx.x) * 4 + k;
    const size_t src = ((size_t)(wslot ^ 1) * Q.nblk + blockIdx.x) * 4 + k;
    Q.part[dst] = ((mask >> k) & 1) ? v[k] : Q.part[src];
  }
}

// s = 0, r = b, p_{-1} = 0; partials (rho, rr, 0, bscale^2) -> slot 1
__global__ void __launch_bounds__(QNT) k_qcg_init(QIter Q) {
  __shared__ double red[4 * (QNT / 64)];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int c = blockIdx.x * QB + threadIdx.x;
  if (c < Q.M.K) {
    const double b = Q.M.rhs[c], dg = Q.M.diag[c];
    Q.s[c] = 0.0;
    Q.r[c] = b;
    Q.p1[c] = 0.0;
    v[0] = dg > 0 ? b * b / dg : 0.0;
    v[1] = b * b;
    v[3] = Q.M.babs[c] * Q.M.babs[c];
  }
  ni::block_sum<4>(v, red);
  if (threadIdx.x < 4) Q.part[((size_t)Q.nblk + blockIdx.x) * 4 + threadIdx.x] = v[threadIdx.x];
}

// A_i: p_i = D^-1 r + beta p_{i-1} (neighbours recomputed), q = L p_i, (p, q)
__global__ void __launch_bounds__(QNT) k_qcg_a(QIter Q, int it) {
  __shared__ double red[8 * (QNT / 64)];
  double g[4];
  q_partials(Q, 1, g, red);
  const bool done = !(g[1] > Q.rtol * Q.rtol * g[3]) || it >= Q.maxit;
  if (done) {
    q_put(Q, 0, g, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Q.flag[it & 1] = 0;
      if (*Q.iters_out < 0) *Q.iters_out = it;
    }
    return;
  }
  const double beta = it == 0 ? 0.0 : g[0] / Q.sc[(it - 1) & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Q.sc[it & 1] = g[0];
    Q.flag[it & 1] = 1;
  }
  const double* pold = (it & 1) ? Q.p0 : Q.p1;
  double* pnew = (it & 1) ? Q.p1 : Q.p0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  {
    // light rows of this block's range: one thread each
    const int c = blockIdx.x * QB + threadIdx.x;
    if (c < Q.M.K) {
      const int j0 = Q.M.row_off[c], j1 = Q.M.row_off[c + 1];
      if (j1 - j0 <= QHEAVY) {
        const double dc = Q.M.diag[c];
        const double pc = (dc > 0 ? Q.r[c] / dc : 0.0) + beta * pold[c];
        double acc = 0.0;
        for (int j = j0; j < j1; ++j) {
          const int d = Q.M.qcol[j];
          const double dd = Q.M.diag[d];
          const double pd = (dd > 0 ? Q.r[d] / dd : 0.0) + beta * pold[d];
          acc += Q.M.qw[j] * (pc - pd);
        }
        pnew[c] = pc;
        Q.q[c] = acc;
        v[2] += pc * acc;
      }
    }
  }
  // heavy rows, dealt round-robin to the blocks: one wavefront each
  for (int h = blockIdx.x * (QNT / 64) + wid; h < Q.M.nheavy; h += gridDim.x * (QNT / 64)) {
    const int c = Q.M.heavy[h];
    const double dc = Q.M.diag[c];
    const double pc = (dc > 0 ? Q.r[c] / dc : 0.0) + beta * pold[c];
    double acc = 0.0;
    for (int j = Q.M.row_off[c] + lane; j < Q.M.row_off[c + 1]; j += 64) {
      const int d = Q.M.qcol[j];
      const double dd = Q.M.diag[d];
      const double pd = (dd > 0 ? Q.r[d] / dd : 0.0) + beta * pold[d];
      acc += Q.M.qw[j] * (pc - pd);
    }
    acc = ni::wave_sum(acc);
    if (lane == 0) {
      pnew[c] = pc;
      Q.q[c] = acc;
      v[2] += pc * acc;
    }
  }
  ni::block_sum<4>(v, red + 4 * (QNT / 64));
  q_put(Q, 0, v, 4);
}

// B_i: alpha = rho / (p, q); s += alpha p; r -= alpha q; (r, D^-1 r), ||r||^2
__global__ void __launch_bounds__(QNT) k_qcg_b(QIter Q, int it) {
  __shared__ double red[8 * (QNT / 64)];
  double g[4];
  q_partials(Q, 0, g, red);
  const bool done = !(g[1] > Q.rtol * Q.rtol * g[3]) || it >= Q.maxit;
  if (done) {
    q_put(Q, 1, g, 0);
    return;
  }
  const double alpha = g[0] / g[2];
  const double* pcur = (it & 1) ? Q.p1 : Q.p0;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const int c = blockIdx.x * QB + threadIdx.x;
  if (c < Q.M.K) {
    const double dg = Q.M.diag[c];
    Q.s[c] += alpha * pcur[c];
    const double r = Q.r[c] - alpha * Q.q[c];
    Q.r[c] = r;
    v[0] = dg > 0 ? r * r / dg : 0.0;
    v[1] = r * r;
  }
  ni::block_sum<4>(v, red + 4 * (QNT / 64));
  q_put(Q, 1, v, 3);
}

// piece gauge: zero mean of s over every connected piece (root = parent)
__global__ void k_piece_acc(const int* __restrict__ parent, const double* __restrict__ s, int K,
                            double* __restrict__ psum, int* __restrict__ pcnt) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  int r = parent[c];
  atomicAdd(&psum[r], s[c]);
  atomicAdd(&pcnt[r], 1);
}

__global__ void k_piece_apply(const int* __restrict__ parent, double* __restrict__ s, int K,
                              const double* __restrict__ psum, const int* __restrict__ pcnt,
                              double* __restrict__ S) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  int r = parent[c];
  double sc = s[c] - psum[r] / (double)pcnt[r];
  s[c] = sc;
  S[c] += sc;
}

// per pair energy contribution; block partials
__global__ void __launch_bounds__(256) k_irls_energy(const int* __restrict__ pair_start, const int* __restrict__ pair_lo,
                                                     const int* __restrict__ pair_hi, int P,
                                                     const double* __restrict__ ew, const double* __restrict__ erho,
                                                     const double* __restrict__ s, double* __restrict__ bpart) {
  __shared__ double red[4];
  int pid = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (pid < P) {
    const double ds = s[pair_lo[pid]] - s[pair_hi[pid]];
    for (int i = pair_start[pid]; i < pair_start[pid + 1]; ++i) {
      double x = erho[i] + ds;
      e += ew[i] * x * x;
    }
  }
  double v[1] = {e};
  ni::block_sum<1>(v, red);
  if (threadIdx.x == 0) bpart[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(256) k_sum_parts(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[4];
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) v[0] += part[i];
  ni::block_sum<1>(v, red);
  if (threadIdx.x == 0) *out = v[0];
}

}  // namespace

namespace nil {

// rows of the quotient CSR with more than QHEAVY entries; count -> *count_dev
hipError_t quot_heavy_rows(const int* row_off, int K, int* flag, int* pos, int* list, int* count_dev, int* scan_tmp,
                           hipStream_t st) {
  if (K <= 0) return hipMemsetAsync(count_dev, 0, sizeof(int), st);
  k_heavy_flags<<<ni::ceil_div(K, 256), 256, 0, st>>>(row_off, K, flag);
  hipError_t e = scan_exclusive_i32(flag, pos, K, count_dev, scan_tmp, st);
  if (e != hipSuccess) return e;
  k_heavy_list<<<ni::ceil_div(K, 256), 256, 0, st>>>(flag, pos, K, list);
  return hipGetLastError();
}

hipError_t list_components(int n, const int* a, const int* b, const double* keep, int m, int* parent,
                           hipStream_t st);

hipError_t quot_inter_edges(const int* label, const uint8_t* ebits, int P, int W, int* flag, int* epos,
                            int* count_dev, uint32_t* eidx_raw, int* scan_tmp, hipStream_t st, int phase) {
  if (phase == 0) {
    k_inter_flags<<<ni::ceil_div(P, 256), 256, 0, st>>>(label, ebits, P, W, flag);
    return scan_exclusive_i32(flag, epos, 2 * P, count_dev, scan_tmp, st);
  }
  k_inter_compact<<<ni::ceil_div(2 * (long long)P, 256), 256, 0, st>>>(flag, epos, 2 * P, eidx_raw);
  return hipGetLastError();
}

// sort edges by (lo, hi), find pairs; pair count -> count_dev
hipError_t quot_sort_edges(uint32_t* eidx_raw, int E, int W, int K, const int* label, uint32_t* keys,
                           uint32_t* eidx, uint32_t* ktmp, uint32_t* vtmp, uint32_t* kout2, int* flag, int* ppos,
                           int* count_dev, int* scan_tmp, hipStream_t st) {
  if (E <= 0) return hipMemsetAsync(count_dev, 0, sizeof(int), st);
  int bits = 0;
  while ((1ll << bits) < (long long)K) ++bits;
  int nb = ni::ceil_div(E, 256);
  // pass 1: by hi, into eidx
  k_edge_keys<<<nb, 256, 0, st>>>(eidx_raw, E, W, label, 1, keys);
  hipError_t e = radix_sort_pairs(keys, eidx_raw, kout2, eidx, ktmp, vtmp, E, bits, scan_tmp, st);
  if (e != hipSuccess) return e;
  // pass 2: stable by lo, back into eidx_raw then copy order into eidx
  k_edge_keys<<<nb, 256, 0, st>>>(eidx, E, W, label, 0, keys);
  e = radix_sort_pairs(keys, eidx, kout2, eidx_raw, ktmp, vtmp, E, bits, scan_tmp, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(eidx, eidx_raw, sizeof(uint32_t) * E, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  k_pair_flags<<<nb, 256, 0, st>>>(eidx, E, W, label, flag);
  return scan_exclusive_i32(flag, ppos, E, count_dev, scan_tmp, st);
}

hipError_t quot_pairs(const uint32_t* eidx, const int* flag, const int* ppos, int E, int W, const int* label,
                      int npairs, int* pair_start, int* pair_lo, int* pair_hi, hipStream_t st) {
  if (E <= 0) return hipSuccess;
  k_pair_build<<<ni::ceil_div(E, 256), 256, 0, st>>>(eidx, flag, ppos, E, W, label, pair_start, pair_lo, pair_hi,
                                                     npairs);
  return hipGetLastError();
}

// CSR over K rows; entries sorted by (row, col): ent[j] = 2*pid + (row == hi)
hipError_t quot_csr(const int* pair_lo, const int* pair_hi, int P, int K, uint32_t* keys, uint32_t* ent,
                    uint32_t* ktmp, uint32_t* vtmp, uint32_t* kout2, uint32_t* ent_tmp, int* cnt, int* row_off,
                    int* scan_tmp, hipStream_t st) {
  hipError_t e;
  if (K <= 0) return hipSuccess;
  k_fill_i32<<<ni::ceil_div(K, 256), 256, 0, st>>>(cnt, K, 0);
  if (P > 0) {
    int bits = 0;
    while ((1ll << bits) < (long long)K) ++bits;
    int P2 = 2 * P;
    int nb = ni::ceil_div(P2, 256);
    k_iota_u32<<<nb, 256, 0, st>>>(ent_tmp, P2);
    // pass 1: by column, pass 2 (stable): by row
    k_entry_keys<<<nb, 256, 0, st>>>(pair_lo, pair_hi, P2, 0, nullptr, keys);
    e = radix_sort_pairs(keys, ent_tmp, kout2, ent, ktmp, vtmp, P2, bits, scan_tmp, st);
    if (e != hipSuccess) return e;
    k_entry_keys<<<nb, 256, 0, st>>>(pair_lo, pair_hi, P2, 1, ent, keys);
    e = radix_sort_pairs(keys, ent, kout2, ent_tmp, ktmp, vtmp, P2, bits, scan_tmp, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(ent, ent_tmp, sizeof(uint32_t) * P2, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    k_row_count<<<ni::ceil_div(P, 256), 256, 0, st>>>(pair_lo, pair_hi, P, cnt);
  }
  e = scan_exclusive_i32(cnt, row_off, K, row_off + K, scan_tmp, st);
  return e;
}



hipError_t irls_iteration(const IrlsArgs& a, int t, hipStream_t st) {
  hipError_t e;
  EdgeParams q;
  q.W = a.W;
  q.align = a.align;
  q.outlier_mode = a.outlier_mode;
  q.t = t;
  q.g2fx = a.g2fx;
  q.g2fy = a.g2fy;
  q.k = a.k;
  q.lL = log10(a.L);
  q.lU = log10(a.U);
  q.U = a.U;
  if (a.K <= 0) return hipSuccess;
  if (a.E > 0) {
    e = hipMemsetAsync(a.wmax, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    k_irls_edges<<<ni::ceil_div(a.E, 256), 256, 0, st>>>(a.eidx, a.E, a.label, a.ebits, a.nt, a.om_r, a.om_d,
                                                        a.zfill, a.S, q, a.ew, a.erho, a.wmax);
    k_irls_pairs<<<ni::ceil_div(a.P, 256), 256, 0, st>>>(a.pair_start, a.P, a.ew, a.erho, a.wmax, a.cut_rel, a.pW,
                                                        a.pB);
  }
  k_irls_nodes<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.row_off, a.ent, a.K, a.pW, a.pB, a.diag, a.rhs, a.babs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // pieces of the weighted quotient graph
  e = list_components(a.K, a.pair_lo, a.pair_hi, a.pW, a.P, a.parent, st);
  if (e != hipSuccess) return e;
  // quotient PCG
  if (a.nnz > 0) k_q_matrix<<<ni::ceil_div(a.nnz, 256), 256, 0, st>>>(a.row_off, a.ent, a.pair_lo, a.pair_hi, a.pW,
                                                                       a.nnz, a.qcol, a.qw);
  QMat M;
  M.row_off = a.row_off; M.qcol = a.qcol; M.qw = a.qw; M.diag = a.diag; M.rhs = a.rhs; M.babs = a.babs; M.K = a.K;
  M.heavy = a.heavy; M.nheavy = a.nheavy;
  if (a.K <= QCAP) {
    k_qcg_wg<<<1, QWG, 0, st>>>(M, a.s, a.r, a.q_rtol, a.q_maxit, a.qiters_out + t);
    e = hipGetLastError();
  } else {
    QIter Q;
    Q.M = M; Q.s = a.s; Q.p0 = a.p0; Q.p1 = a.p1; Q.r = a.r; Q.q = a.q;
    Q.part = a.part; Q.sc = a.sc; Q.flag = a.qflag; Q.nblk = ni::ceil_div(a.K, QB); Q.rtol = a.q_rtol;
    Q.maxit = a.q_maxit; Q.iters_out = a.qiters_out + t;
    k_fill_i32<<<1, 1, 0, st>>>(Q.iters_out, 1, -1);
    k_qcg_init<<<Q.nblk, QNT, 0, st>>>(Q);
    e = hipGetLastError();
    // two launches per iteration; the host polls the "still iterating" flag in batches
    const int batch = 32;
    for (int it = 0; e == hipSuccess && it <= a.q_maxit + 1; it += batch) {
      for (int k = 0; k < batch; ++k) {
        k_qcg_a<<<Q.nblk, QNT, 0, st>>>(Q, it + k);
        k_qcg_b<<<Q.nblk, QNT, 0, st>>>(Q, it + k);
      }
      e = hipGetLastError();
      if (e != hipSuccess) break;
      e = hipMemcpyAsync(a.host_flag, Q.flag + ((it + batch - 1) & 1), sizeof(int), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (*a.host_flag == 0) break;
    }
  }
  if (e != hipSuccess) return e;
  // piece gauge and accumulate S
  k_fill_f64<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.psum, a.K, 0.0);
  k_fill_i32<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.pcnt, a.K, 0);
  k_piece_acc<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.parent, a.s, a.K, a.psum, a.pcnt);
  k_piece_apply<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.parent, a.s, a.K, a.psum, a.pcnt, a.S);
  // energy
  if (a.P > 0) {
    int nb = ni::ceil_div(a.P, 256);
    k_irls_energy<<<nb, 256, 0, st>>>(a.pair_start, a.pair_lo, a.pair_hi, a.P, a.ew, a.erho, a.s, a.epart);
    k_sum_parts<<<1, 256, 0, st>>>(a.epart, nb, a.energy_out + t);
  } else {
    k_fill_f64<<<1, 1, 0, st>>>(a.energy_out + t, 1, 0.0);
  }
  return hipGetLastError();
}

}  // namespace nil
