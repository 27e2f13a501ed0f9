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

// quotient rows with more entries than QELL are "heavy" (see the row classes below)
constexpr int QELL = 8, QBIG = 512;

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
  if (c >= K || row_off[c + 1] - row_off[c] > QELL) return;  // long rows: k_irls_nodes_heavy
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

// the same for the rows with more than QELL entries, one wavefront each
__global__ void k_irls_nodes_heavy(const int* __restrict__ row_off, const uint32_t* __restrict__ ent,
                                   const int* __restrict__ heavy, int nheavy, const double* __restrict__ pW,
                                   const double* __restrict__ pB, double* __restrict__ diag,
                                   double* __restrict__ rhs, double* __restrict__ babs) {
  const int h = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (h >= nheavy) return;
  const int c = heavy[h];
  double dg = 0.0, b = 0.0, ba = 0.0;
  for (int j = row_off[c] + lane; j < row_off[c + 1]; j += 64) {
    uint32_t e = ent[j];
    int pid = (int)(e >> 1);
    dg += pW[pid];
    double v = (e & 1u) ? pB[pid] : -pB[pid];
    b += v;
    ba += fabs(v);
  }
  dg = ni::wave_sum(dg);
  b = ni::wave_sum(b);
  ba = ni::wave_sum(ba);
  if (lane == 0) {
    diag[c] = dg;
    rhs[c] = b;
    babs[c] = ba;
  }
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

// Row classes of the quotient matrix.  Most rows have at most QELL entries
// (a component borders a handful of others); they are also stored in an
// ELL layout ecol/ew [QELL][K] (padding: column = the row, weight 0) so that
// a thread loads all its entries with coalesced, independent loads.  Rows
// with more entries ("heavy") are listed big first (> QBIG entries: one
// workgroup each) then mid (one wavefront each); a large component can
// border a thousand others.
constexpr int QUNR = 8;  // entries per lane loaded ahead in a heavy row

struct QMat {
  const int* row_off;
  const int* qcol;
  const double* qw;
  const int* ecol;
  const double* ew;
  const double* diag;
  const double* rhs;
  const double* babs;
  const int* heavy;  // nbig big rows, then the mid rows
  int nheavy, nbig;
  int K;
};

__global__ void k_heavy_flags(const int* __restrict__ row_off, int K, int lo, int hi, int* __restrict__ flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K) {
    const int n = row_off[c + 1] - row_off[c];
    flag[c] = (n > lo && n <= hi) ? 1 : 0;
  }
}

__global__ void k_heavy_list(const int* __restrict__ flag, const int* __restrict__ pos, int K, int base,
                             int* __restrict__ list) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K && flag[c]) list[base + pos[c]] = c;
}

// ELL copy of the rows with at most QELL entries (heavy rows: padding only)
__global__ void k_q_ell(const int* __restrict__ row_off, const int* __restrict__ qcol, const double* __restrict__ qw,
                        int K, int* __restrict__ ecol, double* __restrict__ ew) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  const int j0 = row_off[c], n = row_off[c + 1] - j0;
  const bool light = n <= QELL;
#pragma unroll
  for (int k = 0; k < QELL; ++k) {
    const bool use = light && k < n;
    ecol[(size_t)k * K + c] = use ? qcol[j0 + k] : c;
    ew[(size_t)k * K + c] = use ? qw[j0 + k] : 0.0;
  }
}

// sum over the ELL entries of row c of q (X_c - X_d), X = one LDS vector
__device__ __forceinline__ double ell_lds(const QMat& M, int c, const double* __restrict__ xl, double xc) {
  int d[QELL];
  double q[QELL];
#pragma unroll
  for (int k = 0; k < QELL; ++k) {
    d[k] = M.ecol[(size_t)k * M.K + c];
    q[k] = M.ew[(size_t)k * M.K + c];
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < QELL; ++k) acc += q[k] * (xc - xl[d[k]]);
  return acc;
}

// Quotient systems are solved by Jacobi-preconditioned CG in the
// single-reduction form of Chronopoulos and Gear.  With u = D^-1 r and
// w = L u carried along, an iteration needs the three sums (r,u), (w,u) and
// (r,r) of the same vectors, so one reduction instead of two:
//   p_i = u_i + b_i p_{i-1},   h_i = w_i + b_i h_{i-1}        (h_i = L p_i)
//   s  += a_i p_i,   r_{i+1} = r_i - a_i h_i,   u_{i+1} = D^-1 r_{i+1},   w_{i+1} = L u_{i+1}
//   g_{i+1} = (r_{i+1}, u_{i+1}),   d_{i+1} = (w_{i+1}, u_{i+1})
//   b_{i+1} = g_{i+1} / g_i,   a_{i+1} = g_{i+1} / (d_{i+1} - b_{i+1} g_{i+1} / a_i)
// from s = 0, r_0 = b, b_0 = 0, a_0 = g_0 / d_0.  In exact arithmetic these
// are the iterates of standard PCG.  The products are applied in difference
// form (L v)_c = sum_d w_cd (v_c - v_d); rows whose every quotient edge was
// cut (diag = 0) keep s = 0.  Iteration stops at ||r|| <= rtol ||b_abs||,
// b_abs = the row-wise sums of |w_e r_e| (a scale of the right-hand side
// that does not cancel).
//
// One workgroup of QWG threads owns every row (K <= QCAP): u and L u live
// in LDS, and an iteration costs one block reduction and two or three
// barriers.  QR rows per thread; r, p, h, 1/diag of the rows stay in
// registers (with more rows per thread they would spill), the solution
// accumulates in place in s (each thread its own rows).
constexpr int QWG = 1024, QNW = QWG / 64, QR = 4, QCAP = QWG * QR;

__global__ void __launch_bounds__(QWG) k_qcg_wg(QMat M, double* __restrict__ s, double rtol, int maxit,
                                                int* __restrict__ iters_out) {
  __shared__ double ul[QCAP];  // u = D^-1 r of every row
  __shared__ double wl[QCAP];  // L u of every row
  __shared__ double red0[QNW];
  __shared__ double red[3 * QNW];
  const int K = M.K;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double r[QR], p[QR], h[QR], di[QR];
  int lmask = 0;  // bit k: row k of this thread is light
  double v0[1] = {0.0};
#pragma unroll
  for (int k = 0; k < QR; ++k) {
    const int c = threadIdx.x + k * QWG;
    r[k] = p[k] = h[k] = di[k] = 0.0;
    if (c < K) {
      if (M.row_off[c + 1] - M.row_off[c] <= QELL) lmask |= 1 << k;
      const double dg = M.diag[c];
      di[k] = dg > 0 ? 1.0 / dg : 0.0;
      r[k] = M.rhs[c];
      ul[c] = r[k] * di[k];
      s[c] = 0.0;
      v0[0] += M.babs[c] * M.babs[c];
    }
  }
  ni::block_sum<1>(v0, red0);  // its barrier also publishes ul
  const double tol2 = rtol * rtol * v0[0];
  double gam_old = 1.0, alp_old = 1.0;
  int it = 0;
  for (;;) {
    // one row at a time: the loads of all rows at once would not fit in registers
#pragma unroll 1
    for (int k = 0; k < QR; ++k) {
      const int c = threadIdx.x + k * QWG;
      if (c < K && ((lmask >> k) & 1)) wl[c] = ell_lds(M, c, ul, ul[c]);
    }
    for (int hh = wid; hh < M.nheavy; hh += QNW) {
      const int c = M.heavy[hh];
      const double uc = ul[c];
      const int j1 = M.row_off[c + 1];
      double acc = 0.0;
      for (int base = M.row_off[c]; base < j1; base += 64 * QUNR) {
        int d[QUNR];
        double q[QUNR];
#pragma unroll
        for (int u = 0; u < QUNR; ++u) {
          const int j = base + u * 64 + lane;
          d[u] = j < j1 ? M.qcol[j] : c;
          q[u] = j < j1 ? M.qw[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < QUNR; ++u) acc += q[u] * (uc - ul[d[u]]);
      }
      acc = ni::wave_sum(acc);
      if (lane == 0) wl[c] = acc;
    }
    if (M.nheavy > 0) __syncthreads();
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < QR; ++k) {
      const int c = threadIdx.x + k * QWG;
      if (c < K) {
        const double uc = r[k] * di[k];
        v[0] += r[k] * uc;
        v[1] += wl[c] * uc;
        v[2] += r[k] * r[k];
      }
    }
    ni::block_sum<3>(v, red);
    if (!(v[2] > tol2) || it >= maxit) break;
    const double gam = v[0], del = v[1];
    const double beta = it == 0 ? 0.0 : gam / gam_old;
    const double alpha = it == 0 ? gam / del : gam / (del - beta * gam / alp_old);
    gam_old = gam;
    alp_old = alpha;
#pragma unroll
    for (int k = 0; k < QR; ++k) {
      const int c = threadIdx.x + k * QWG;
      if (c < K) {
        p[k] = r[k] * di[k] + beta * p[k];
        h[k] = wl[c] + beta * h[k];
        s[c] += alpha * p[k];
        r[k] -= alpha * h[k];
        ul[c] = r[k] * di[k];
      }
    }
    __syncthreads();  // u complete before the next product; red and wl free again
    ++it;
  }
  if (threadIdx.x == 0) *iters_out = it;
}

// The same iteration for K <= QR3 * QWG with the matrix staged once per
// solve, so that the loop touches no global memory: rows of at most QRE
// entries keep them in registers (column indices packed two per register),
// longer rows are listed in LDS with their entries (summed by the thread
// that owns the row, or by a wavefront with lanes strided over the entries
// above QMID entries), and the solution stays in registers until the end.
// If the long rows do not fit (more than QHROWS rows, QHCAP entries or
// QBROWS wavefront rows), each thread sums its own long rows from global
// memory.
constexpr int QR3 = 3, QRE = 4, QHCAP = 8192, QHROWS = 1536, QMID = 32, QBROWS = 256;
__global__ void __launch_bounds__(QWG) k_qcg_wgr(QMat M, double* __restrict__ s, double rtol, int maxit,
                                                 int* __restrict__ iters_out) {
  __shared__ double ul[QR3 * QWG];
  __shared__ double wl[QR3 * QWG];
  __shared__ double hw[QHCAP];
  __shared__ uint16_t hc[QHCAP];
  __shared__ int hoff[QHROWS + 1];
  __shared__ int hrow[QHROWS];
  __shared__ int blist[QBROWS];
  __shared__ double red0[QNW];
  __shared__ double red[3 * QNW];
  __shared__ int nlong_s, nbig_s;
  const int K = M.K;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nt = blockDim.x, nw = nt >> 6;  // a multiple of 64 with QR3 * nt >= K
  if (threadIdx.x == 0) {
    nlong_s = 0;
    nbig_s = 0;
  }
  __syncthreads();
  // rows of this thread: entries in registers, or listed as long
  uint32_t lc[QR3][QRE / 2];
  double lw[QR3][QRE];
  double r[QR3], p[QR3], h[QR3], di[QR3], sx[QR3];
  int smask = 0;  // bit k: row k is short (entries in registers)
  int lmask = 0;  // bit k: row k is long
  int tmask = 0;  // bit k: row k is long and summed by this thread
  int bmask = 0;  // bit k: row k is summed by a wavefront (its (w, u) term too)
  int lidx[QR3];  // list index of a long row
  double v0[1] = {0.0};
#pragma unroll
  for (int k = 0; k < QR3; ++k) {
    const int c = threadIdx.x + k * nt;
    r[k] = p[k] = h[k] = di[k] = sx[k] = 0.0;
    lidx[k] = 0;
    int j0 = 0, n = 0;
    if (c < K) {
      j0 = M.row_off[c];
      n = M.row_off[c + 1] - j0;
      if (n <= QRE) {
        smask |= 1 << k;
      } else {
        lmask |= 1 << k;
        const int idx = atomicAdd(&nlong_s, 1);
        lidx[k] = idx;
        if (idx < QHROWS) {
          hrow[idx] = c;
          hoff[idx] = n;  // the length for now; offsets below
          if (n > QMID) {
            const int b = atomicAdd(&nbig_s, 1);
            if (b < QBROWS) blist[b] = idx;
            bmask |= 1 << k;
          } else {
            tmask |= 1 << k;
          }
        }
      }
    }
    const bool sh = (smask >> k) & 1;
#pragma unroll
    for (int e = 0; e < QRE; e += 2) {
      const uint32_t c0 = sh && e < n ? (uint32_t)M.qcol[j0 + e] : (uint32_t)max(c, 0);
      const uint32_t c1 = sh && e + 1 < n ? (uint32_t)M.qcol[j0 + e + 1] : (uint32_t)max(c, 0);
      lc[k][e / 2] = c0 | (c1 << 16);
      lw[k][e] = sh && e < n ? M.qw[j0 + e] : 0.0;
      lw[k][e + 1] = sh && e + 1 < n ? M.qw[j0 + e + 1] : 0.0;
    }
    if (c < K) {
      const double dg = M.diag[c];
      di[k] = dg > 0 ? 1.0 / dg : 0.0;
      r[k] = M.rhs[c];
      ul[c] = r[k] * di[k];
      v0[0] += M.babs[c] * M.babs[c];
    }
  }
  __syncthreads();
  const int nlong = nlong_s;
  // offsets of the listed rows (one wavefront, 64 rows at a time)
  if (wid == 0 && nlong <= QHROWS) {
    int base = 0;
    for (int h0 = 0; h0 < nlong; h0 += 64) {
      const int hh = h0 + lane;
      const int len = hh < nlong ? hoff[hh] : 0;
      int inc = len;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
      }
      if (hh < nlong) hoff[hh] = base + inc - len;
      base += __shfl(inc, 63, 64);
    }
    if (lane == 0) hoff[nlong] = base;
  }
  __syncthreads();
  const int nbig = nbig_s;
  const bool hl = nlong <= QHROWS && nbig <= QBROWS && hoff[nlong] <= QHCAP;
  if (!hl) bmask = 0;
  if (hl) {
    for (int hh = wid; hh < nlong; hh += nw) {
      const int c = hrow[hh], j0 = M.row_off[c], o = hoff[hh], n = hoff[hh + 1] - o;
      for (int j = lane; j < n; j += 64) {
        hc[o + j] = (uint16_t)M.qcol[j0 + j];
        hw[o + j] = M.qw[j0 + j];
      }
    }
  }
  ni::block_sum<1>(v0, red0);  // its barrier also publishes ul and the LDS rows
  const double tol2 = rtol * rtol * v0[0];
  double gam_old = 1.0, alp_old = 1.0;
  int it = 0;
  for (;;) {
    double vbig = 0.0;
#pragma unroll
    for (int k = 0; k < QR3; ++k) {
      const int c = threadIdx.x + k * nt;
      if ((smask >> k) & 1) {
        const double uc = ul[c];
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < QRE; ++e) {
          const int d = (int)((lc[k][e / 2] >> (16 * (e & 1))) & 0xFFFFu);
          acc += lw[k][e] * (uc - ul[d]);
        }
        wl[c] = acc;
      }
    }
    if (hl) {
#pragma unroll
      for (int k = 0; k < QR3; ++k) {
        if ((tmask >> k) & 1) {
          const int c = threadIdx.x + k * nt;
          const double uc = ul[c];
          double acc = 0.0;
          for (int j = hoff[lidx[k]]; j < hoff[lidx[k] + 1]; ++j) acc += hw[j] * (uc - ul[hc[j]]);
          wl[c] = acc;
        }
      }
      for (int bb = wid; bb < nbig; bb += nw) {
        const int hh = blist[bb];
        const int c = hrow[hh];
        const double uc = ul[c];
        double acc = 0.0;
        for (int j = hoff[hh] + lane; j < hoff[hh + 1]; j += 64) acc += hw[j] * (uc - ul[hc[j]]);
        acc = ni::wave_sum(acc);
        if (lane == 0) {
          wl[c] = acc;
          vbig += acc * uc;
        }
      }
    } else {
#pragma unroll 1
      for (int k = 0; k < QR3; ++k) {
        const int c = threadIdx.x + k * nt;
        if ((lmask >> k) & 1) {
          const double uc = ul[c];
          double acc = 0.0;
          for (int j = M.row_off[c]; j < M.row_off[c + 1]; ++j) acc += M.qw[j] * (uc - ul[M.qcol[j]]);
          wl[c] = acc;
        }
      }
    }
    // no barrier here: every row's (w, u) term is added by the thread that
    // formed w (the reduction's barrier then publishes wl for the update)
    double v[3] = {0.0, vbig, 0.0};
#pragma unroll
    for (int k = 0; k < QR3; ++k) {
      const int c = threadIdx.x + k * nt;
      if (c < K) {
        const double uc = r[k] * di[k];
        v[0] += r[k] * uc;
        if (!((bmask >> k) & 1)) v[1] += wl[c] * uc;
        v[2] += r[k] * r[k];
      }
    }
    ni::block_sum<3>(v, red);
    if (!(v[2] > tol2) || it >= maxit) break;
    const double gam = v[0], del = v[1];
    const double beta = it == 0 ? 0.0 : gam / gam_old;
    const double alpha = it == 0 ? gam / del : gam / (del - beta * gam / alp_old);
    gam_old = gam;
    alp_old = alpha;
#pragma unroll
    for (int k = 0; k < QR3; ++k) {
      const int c = threadIdx.x + k * nt;
      if (c < K) {
        p[k] = r[k] * di[k] + beta * p[k];
        h[k] = wl[c] + beta * h[k];
        sx[k] += alpha * p[k];
        r[k] -= alpha * h[k];
        ul[c] = r[k] * di[k];
      }
    }
    __syncthreads();  // u complete before the next product; red and wl free again
    ++it;
  }
#pragma unroll
  for (int k = 0; k < QR3; ++k) {
    const int c = threadIdx.x + k * nt;
    if (c < K) s[c] = sx[k];
  }
  if (threadIdx.x == 0) *iters_out = it;
}

// Larger quotient systems: the same iteration, one launch per iteration.
// Blocks [0, nblk) own QB consecutive rows each (light rows through the ELL
// copy); the next nbig blocks form L u for one big row each, all QNT
// threads striding over its entries; the last blocks give one mid row to
// each wavefront.
//
// Per row and parity slot one 32-byte record {r, w, h, 1/diag}: launch i
// reads r_i, w_i, h_{i-1} from slot i&1 and writes r_{i+1}, w_{i+1}, h_i to
// the other slot, so a neighbour costs one record load, and the neighbours'
// u_{i+1} are recomputed from their slot-i values (no block waits for
// another).  Every block re-sums all blocks' FP64 partials (g, d, rr, |b|^2)
// of the previous launch in block order (deterministic, no atomics, no
// in-kernel fences); the gathers that do not depend on a_i, b_i are issued
// first, so the two latencies overlap.
constexpr int QNT = 256, QB = 256, QNWB = QNT / 64;

struct QIter {
  QMat M;
  double *x, *p;
  double4* st;     // [2][K] records {r, w, h, 1/diag}
  double* part;    // [2][nparts][4]: g, d, rr, |b|^2
  double* sc;      // [2][2]: g_i, a_i by iteration parity
  int* flag;       // [2] still iterating, by iteration parity
  int nblk, nparts;
  double rtol;
  int maxit;
  int* iters_out;
};

__host__ __device__ inline int q_nparts(int nblk, int nbig, int nmid) { return nblk + nbig + (nmid + QNWB - 1) / QNWB; }

// terms q (X_e - X_d), X = r, w, h scaled by 1/diag, over entries
// [j0 + t0, j1) with stride `stride`; QUNR entries are loaded before use
__device__ __forceinline__ void row_terms(const QMat& M, const double4* __restrict__ sA, int e, int j0, int j1,
                                          int t0, int stride, double Re, double We, double He, double& sR,
                                          double& sW, double& sH) {
  sR = sW = sH = 0.0;
  for (int base = j0 + t0; base < j1; base += stride * QUNR) {
    int d[QUNR];
    double q[QUNR];
#pragma unroll
    for (int u = 0; u < QUNR; ++u) {
      const int j = base + u * stride;
      d[u] = j < j1 ? M.qcol[j] : e;
      q[u] = j < j1 ? M.qw[j] : 0.0;
    }
    double4 n[QUNR];
#pragma unroll
    for (int u = 0; u < QUNR; ++u) n[u] = sA[d[u]];
#pragma unroll
    for (int u = 0; u < QUNR; ++u) {
      sR += q[u] * (Re - n[u].x * n[u].w);
      sW += q[u] * (We - n[u].y * n[u].w);
      sH += q[u] * (He - n[u].z * n[u].w);
    }
  }
}

// s = 0, p = 0, slot 0 = {b, L D^-1 b, 0, 1/diag}; partials -> slot 0.
// Same block layout as the iteration.
__global__ void __launch_bounds__(QNT) k_qcg_init(QIter Q) {
  __shared__ double red[4 * QNWB];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int big0 = Q.nblk, mid0 = Q.nblk + Q.M.nbig;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (blockIdx.x < big0) {
    const int c = blockIdx.x * QB + threadIdx.x;
    if (c < Q.M.K) {
      const double dg = Q.M.diag[c];
      const double dc = dg > 0 ? 1.0 / dg : 0.0;
      const double b = Q.M.rhs[c], uc = b * dc;
      Q.x[c] = 0.0;
      Q.p[c] = 0.0;
      const int j0 = Q.M.row_off[c], j1 = Q.M.row_off[c + 1];
      if (j1 - j0 <= QELL) {
        double acc = 0.0;
        for (int j = j0; j < j1; ++j) {
          const int d = Q.M.qcol[j];
          const double dd = Q.M.diag[d];
          acc += Q.M.qw[j] * (uc - (dd > 0 ? Q.M.rhs[d] / dd : 0.0));
        }
        v[1] = acc * uc;
        Q.st[c] = make_double4(b, acc, 0.0, dc);
      } else {  // w of a heavy row is stored by the block or wavefront that forms it
        double* rec = reinterpret_cast<double*>(Q.st + c);
        rec[0] = b;
        rec[2] = 0.0;
        rec[3] = dc;
      }
      v[0] = b * uc;
      v[2] = b * b;
      v[3] = Q.M.babs[c] * Q.M.babs[c];
    }
  } else {
    // heavy row: a whole block (big) or one wavefront (mid)
    const bool big = blockIdx.x < mid0;
    const int hi = big ? blockIdx.x - big0 : Q.M.nbig + (blockIdx.x - mid0) * QNWB + wid;
    const bool have = big || hi < Q.M.nheavy;
    double acc = 0.0, ue = 0.0;
    int e = 0;
    if (have) {
      e = Q.M.heavy[hi];
      const double de = Q.M.diag[e];
      ue = de > 0 ? Q.M.rhs[e] / de : 0.0;
      const int t0 = big ? threadIdx.x : lane, stride = big ? QNT : 64;
      for (int j = Q.M.row_off[e] + t0; j < Q.M.row_off[e + 1]; j += stride) {
        const int d = Q.M.qcol[j];
        const double dd = Q.M.diag[d];
        acc += Q.M.qw[j] * (ue - (dd > 0 ? Q.M.rhs[d] / dd : 0.0));
      }
    }
    if (big) {
      double a1[1] = {acc};
      ni::block_sum<1>(a1, red);
      acc = a1[0];
      __syncthreads();
    } else {
      acc = ni::wave_sum(acc);
    }
    const bool writer = have && (big ? threadIdx.x == 0 : lane == 0);
    if (writer) {
      reinterpret_cast<double*>(Q.st + e)[1] = acc;
      v[1] = acc * ue;
    }
  }
  ni::block_sum<4>(v, red);
  if (threadIdx.x < 4) Q.part[(size_t)blockIdx.x * 4 + threadIdx.x] = v[threadIdx.x];
}

__global__ void __launch_bounds__(QNT) k_qcg_it(QIter Q, int it) {
  __shared__ double red[4 * QNWB];
  __shared__ double gsh[4];
  const int A = it & 1;
  const double4* sA = Q.st + (size_t)A * Q.M.K;
  double4* sB = Q.st + (size_t)(A ^ 1) * Q.M.K;
  const double* pin = Q.part + (size_t)A * Q.nparts * 4;
  double* pout = Q.part + (size_t)(A ^ 1) * Q.nparts * 4;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int big0 = Q.nblk, mid0 = Q.nblk + Q.M.nbig;
  const int kind = blockIdx.x < big0 ? 0 : (blockIdx.x < mid0 ? 1 : 2);  // rows / big row / mid rows
  // 1. gathers that do not depend on a_i, b_i
  int c = -1;
  if (kind == 0) {
    c = blockIdx.x * QB + threadIdx.x;
    if (c >= Q.M.K) c = -1;
  } else if (kind == 1) {
    c = Q.M.heavy[blockIdx.x - big0];
  } else {
    const int hi = Q.M.nbig + (blockIdx.x - mid0) * QNWB + wid;
    c = hi < Q.M.nheavy ? Q.M.heavy[hi] : -1;
  }
  bool light = false;
  double4 s4 = make_double4(0.0, 0.0, 0.0, 0.0);
  double aR = 0.0, aW = 0.0, aH = 0.0;
  if (c >= 0) {
    s4 = sA[c];
    const double Rc = s4.x * s4.w, Wc = s4.y * s4.w, Hc = s4.z * s4.w;
    const int j0 = Q.M.row_off[c], j1 = Q.M.row_off[c + 1];
    if (kind == 0) {
      light = j1 - j0 <= QELL;
      int d[QELL];
      double q[QELL];
#pragma unroll
      for (int k = 0; k < QELL; ++k) {
        d[k] = Q.M.ecol[(size_t)k * Q.M.K + c];
        q[k] = Q.M.ew[(size_t)k * Q.M.K + c];
      }
      double4 n[QELL];
#pragma unroll
      for (int k = 0; k < QELL; ++k) n[k] = sA[d[k]];
#pragma unroll
      for (int k = 0; k < QELL; ++k) {
        aR += q[k] * (Rc - n[k].x * n[k].w);
        aW += q[k] * (Wc - n[k].y * n[k].w);
        aH += q[k] * (Hc - n[k].z * n[k].w);
      }
    } else if (kind == 1) {
      row_terms(Q.M, sA, c, j0, j1, threadIdx.x, QNT, Rc, Wc, Hc, aR, aW, aH);
    } else {
      row_terms(Q.M, sA, c, j0, j1, lane, 64, Rc, Wc, Hc, aR, aW, aH);
    }
  }
  // 2. partials of the previous launch, summed by the first wavefront
  if (wid == 0) {
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = lane; j < Q.nparts; j += 64) {
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] += pin[(size_t)j * 4 + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = ni::wave_sum(g[k]);
    if (lane < 4) gsh[lane] = g[lane];
  }
  if (kind == 1) {
    double t3[3] = {aR, aW, aH};
    ni::block_sum<3>(t3, red);
    aR = t3[0];
    aW = t3[1];
    aH = t3[2];
  } else if (kind == 2) {
    aR = ni::wave_sum(aR);
    aW = ni::wave_sum(aW);
    aH = ni::wave_sum(aH);
  }
  __syncthreads();  // gsh ready; red free again
  const double gam = gsh[0], del = gsh[1], rr = gsh[2], bs = gsh[3];
  const bool done = !(rr > Q.rtol * Q.rtol * bs) || it >= Q.maxit;
  if (done) {
    if (threadIdx.x < 4) pout[(size_t)blockIdx.x * 4 + threadIdx.x] = pin[(size_t)blockIdx.x * 4 + threadIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Q.flag[it & 1] = 0;
      if (*Q.iters_out < 0) *Q.iters_out = it;
    }
    return;
  }
  double beta = 0.0, alpha = gam / del;
  if (it > 0) {
    const double gp = Q.sc[((it - 1) & 1) * 2], ap = Q.sc[((it - 1) & 1) * 2 + 1];
    beta = gam / gp;
    alpha = gam / (del - beta * gam / ap);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Q.sc[(it & 1) * 2] = gam;
    Q.sc[(it & 1) * 2 + 1] = alpha;
    Q.flag[it & 1] = 1;
  }
  // 3. updates: row blocks own r, h, p, x of their rows (and w of the light
  // ones); the block or wavefront of a heavy row stores its w
  double v[3] = {0.0, 0.0, 0.0};
  const double dc = s4.w;
  const double hn = s4.y + beta * s4.z;
  const double rn = s4.x - alpha * hn;
  const double un = rn * dc;
  const double wn = aR - alpha * (aW + beta * aH);
  if (kind == 0) {
    if (c >= 0) {
      const double pn = s4.x * dc + beta * Q.p[c];
      Q.x[c] += alpha * pn;
      Q.p[c] = pn;
      v[0] = rn * un;
      v[2] = rn * rn;
      if (light) {
        sB[c] = make_double4(rn, wn, hn, dc);
        v[1] = wn * un;
      } else {
        double* rec = reinterpret_cast<double*>(sB + c);
        rec[0] = rn;
        rec[2] = hn;
        rec[3] = dc;
      }
    }
  } else if (c >= 0 && (kind == 1 ? threadIdx.x == 0 : lane == 0)) {
    reinterpret_cast<double*>(sB + c)[1] = wn;
    v[1] = wn * un;
  }
  ni::block_sum<3>(v, red);
  if (threadIdx.x < 3) pout[(size_t)blockIdx.x * 4 + threadIdx.x] = v[threadIdx.x];
  if (threadIdx.x == 3) pout[(size_t)blockIdx.x * 4 + 3] = pin[(size_t)blockIdx.x * 4 + 3];
}

// piece gauge: zero mean of s over every connected piece (root = parent)
__global__ void k_piece_acc(const int* __restrict__ parent, const double* __restrict__ s, int K,
                            double* __restrict__ psum, int* __restrict__ pcnt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool v = c < K;
  ni::acc_by_key<int>(v, v ? parent[c] : 0, v ? s[c] : 0.0, 1, psum, pcnt);
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

// rows of the quotient CSR with more than QELL entries: the big ones
// (> QBIG entries) first, then the mid ones; counts -> count_dev[0..1]
hipError_t quot_heavy_rows(const int* row_off, int K, int* flag, int* pos, int* list, int* count_dev, int* scan_tmp,
                           hipStream_t st) {
  if (K <= 0) return hipMemsetAsync(count_dev, 0, 2 * sizeof(int), st);
  const int nb = ni::ceil_div(K, 256);
  k_heavy_flags<<<nb, 256, 0, st>>>(row_off, K, QBIG, 1 << 30, flag);
  hipError_t e = scan_exclusive_i32(flag, pos, K, count_dev, scan_tmp, st);
  if (e != hipSuccess) return e;
  k_heavy_list<<<nb, 256, 0, st>>>(flag, pos, K, 0, list);
  int nbig = 0;
  e = hipMemcpyAsync(&nbig, count_dev, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  k_heavy_flags<<<nb, 256, 0, st>>>(row_off, K, QELL, QBIG, flag);
  e = scan_exclusive_i32(flag, pos, K, count_dev + 1, scan_tmp, st);
  if (e != hipSuccess) return e;
  k_heavy_list<<<nb, 256, 0, st>>>(flag, pos, K, nbig, list);
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
  if (a.nheavy > 0)
    k_irls_nodes_heavy<<<ni::ceil_div(a.nheavy, 4), 256, 0, st>>>(a.row_off, a.ent, a.heavy, a.nheavy, a.pW, a.pB,
                                                                   a.diag, a.rhs, a.babs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // pieces of the weighted quotient graph
  e = list_components(a.K, a.pair_lo, a.pair_hi, a.pW, a.P, a.parent, st);
  if (e != hipSuccess) return e;
  // quotient PCG
  if (a.nnz > 0) k_q_matrix<<<ni::ceil_div(a.nnz, 256), 256, 0, st>>>(a.row_off, a.ent, a.pair_lo, a.pair_hi, a.pW,
                                                                       a.nnz, a.qcol, a.qw);
  if (a.K > 0) k_q_ell<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.row_off, a.qcol, a.qw, a.K, a.ell_col, a.ell_w);
  QMat M;
  M.row_off = a.row_off; M.qcol = a.qcol; M.qw = a.qw; M.ecol = a.ell_col; M.ew = a.ell_w;
  M.diag = a.diag; M.rhs = a.rhs; M.babs = a.babs; M.K = a.K;
  M.heavy = a.heavy; M.nheavy = a.nheavy; M.nbig = a.nbig;
  if (a.K <= QR3 * QWG) {
    // as few wavefronts as hold QR3 rows per thread (cheaper barriers)
    const int nt = std::max(64, ni::ceil_div(ni::ceil_div(a.K, QR3), 64) * 64);
    k_qcg_wgr<<<1, nt, 0, st>>>(M, a.s, a.q_rtol, a.q_maxit, a.qiters_out + t);
    e = hipGetLastError();
  } else if (a.K <= QCAP) {
    k_qcg_wg<<<1, QWG, 0, st>>>(M, a.s, a.q_rtol, a.q_maxit, a.qiters_out + t);
    e = hipGetLastError();
  } else if (a.amg) {
    // multigrid-preconditioned CG on a hierarchy built from this step's
    // weights (the cut set and the weights change from step to step)
    e = hipGetLastError();
    // the uniform-weight steps (t < align) share one matrix: the hierarchy of
    // step 0 serves them all
    const bool same_as_previous = t > 0 && t < a.align;
    if (e == hipSuccess && !same_as_previous)
      e = amg_build(a.amg, a.K, a.P, a.row_off, a.qcol, a.qw, a.diag, a.pair_lo, a.pair_hi, a.pW, st);
    if (e == hipSuccess) e = amg_update(a.amg, a.qw, a.diag, a.pW, st);
    if (e == hipSuccess)
      e = amg_solve(a.amg, a.rhs, a.babs, a.s, a.q_rtol, a.q_maxit, a.qiters_out + t, a.host_flag, a.graphs != 0, st);
  } else {
    QIter Q;
    Q.M = M; Q.x = a.s; Q.p = a.pv; Q.st = reinterpret_cast<double4*>(a.qst);
    Q.part = a.part; Q.sc = a.sc; Q.flag = a.qflag; Q.nblk = ni::ceil_div(a.K, QB);
    Q.nparts = q_nparts(Q.nblk, a.nbig, a.nheavy - a.nbig); Q.rtol = a.q_rtol;
    Q.maxit = a.q_maxit; Q.iters_out = a.qiters_out + t;
    k_fill_i32<<<1, 1, 0, st>>>(Q.iters_out, 1, -1);
    k_qcg_init<<<Q.nparts, QNT, 0, st>>>(Q);
    e = hipGetLastError();
    // one launch per iteration; the host polls the "still iterating" flag in batches
    const int batch = 32;
    for (int it = 0; e == hipSuccess && it <= a.q_maxit + 1; it += batch) {
      for (int k = 0; k < batch; ++k) k_qcg_it<<<Q.nparts, QNT, 0, st>>>(Q, it + k);
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
