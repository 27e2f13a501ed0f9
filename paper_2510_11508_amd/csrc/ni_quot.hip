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
struct QState {
  const int* row_off;
  const uint32_t* ent;
  const int* pair_lo;
  const int* pair_hi;
  const double* pW;
  const double* diag;
  const double* rhs;
  const double* babs;
  double *s, *r, *z, *p0, *p1, *q, *part;
  int K;
  double rtol;
  int maxit;
  int* iters_out;
};

// grid-wide sum of NV per-block values, same result and order in every block
template <int NV>
__device__ __forceinline__ void grid_sum(const QState& Q, double (&v)[NV], double* red, unsigned* bar,
                                         int slot) {
  ni::block_sum<NV>(v, red);
  const unsigned nb = gridDim.x;
  if (nb == 1) return;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) Q.part[(size_t)slot * 4 * nb + blockIdx.x * 4 + k] = v[k];
  }
  ni::grid_barrier(bar, nb);
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (unsigned j = threadIdx.x; j < nb; j += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += Q.part[(size_t)slot * 4 * nb + j * 4 + k];
  }
  ni::block_sum<NV>(v, red + 8 * (blockDim.x >> 6));
}

__device__ __forceinline__ int nbr_of(const QState& Q, uint32_t e, int row) {
  int pid = (int)(e >> 1);
  return (e & 1u) ? Q.pair_lo[pid] : Q.pair_hi[pid];
}

__global__ void __launch_bounds__(256) k_qcg(QState Q, unsigned* bar) {
  __shared__ double red[16 * 4];
  const int K = Q.K;
  const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gsz = gridDim.x * blockDim.x;
  double v3[3] = {0.0, 0.0, 0.0};
  for (int c = gtid; c < K; c += gsz) {
    double b = Q.rhs[c];
    double dg = Q.diag[c];
    double zc = dg > 0 ? b / dg : 0.0;
    Q.s[c] = 0.0;
    Q.r[c] = b;
    Q.z[c] = zc;
    Q.p0[c] = 0.0;
    v3[0] += b * b;
    v3[1] += b * zc;
    v3[2] += Q.babs[c] * Q.babs[c];
  }
  grid_sum<3>(Q, v3, red, bar, 0);
  double rr = v3[0], rho = v3[1];
  const double tol2 = Q.rtol * Q.rtol * v3[2];
  double beta = 0.0;
  int it = 0;
  while (rr > tol2 && it < Q.maxit) {
    const double* pold = (it & 1) ? Q.p1 : Q.p0;
    double* pnew = (it & 1) ? Q.p0 : Q.p1;
    double v1[1] = {0.0};
    for (int c = gtid; c < K; c += gsz) {
      double pc = Q.z[c] + beta * pold[c];
      double qc = 0.0;
      for (int j = Q.row_off[c]; j < Q.row_off[c + 1]; ++j) {
        uint32_t e = Q.ent[j];
        int d = nbr_of(Q, e, c);
        double pd = Q.z[d] + beta * pold[d];
        qc += Q.pW[e >> 1] * (pc - pd);
      }
      pnew[c] = pc;
      Q.q[c] = qc;
      v1[0] += pc * qc;
    }
    grid_sum<1>(Q, v1, red, bar, 1);
    const double alpha = rho / v1[0];
    double v2[2] = {0.0, 0.0};
    for (int c = gtid; c < K; c += gsz) {
      double dg = Q.diag[c];
      Q.s[c] += alpha * pnew[c];
      double rc = Q.r[c] - alpha * Q.q[c];
      double zc = dg > 0 ? rc / dg : 0.0;
      Q.r[c] = rc;
      Q.z[c] = zc;
      v2[0] += rc * rc;
      v2[1] += rc * zc;
    }
    grid_sum<2>(Q, v2, red, bar, 2);
    rr = v2[0];
    beta = v2[1] / rho;
    rho = v2[1];
    ++it;
  }
  if (gtid == 0) *Q.iters_out = it;
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

struct IrlsArgs {
  const uint32_t* eidx;
  int E, P, K, W;
  const int* label;
  const uint8_t* ebits;
  const float *nt, *om_r, *om_d, *zfill;
  const int *pair_start, *pair_lo, *pair_hi, *row_off;
  const uint32_t* ent;
  double *S, *ew, *erho, *pW, *pB, *diag, *rhs, *babs;
  double *s, *r, *z, *p0, *p1, *q, *part, *psum;
  int *pcnt, *parent;
  unsigned long long* wmax;
  unsigned* bar;
  double* energy_out;  // [t]
  int* qiters_out;     // [t]
  double* epart;
  double g2fx, g2fy, k, L, U, cut_rel, q_rtol;
  int align, outlier_mode, q_maxit, qblocks;
};

int qcg_max_blocks(int device) {
  int per_cu = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_qcg, 256, 0) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 1;
  return per_cu * ncu;
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
  // PCG
  QState Q;
  Q.row_off = a.row_off; Q.ent = a.ent; Q.pair_lo = a.pair_lo; Q.pair_hi = a.pair_hi;
  Q.pW = a.pW; Q.diag = a.diag; Q.rhs = a.rhs; Q.babs = a.babs;
  Q.s = a.s; Q.r = a.r; Q.z = a.z; Q.p0 = a.p0; Q.p1 = a.p1; Q.q = a.q; Q.part = a.part;
  Q.K = a.K; Q.rtol = a.q_rtol; Q.maxit = a.q_maxit; Q.iters_out = a.qiters_out + t;
  unsigned* bar = a.bar;
  if (a.qblocks <= 1) {
    k_qcg<<<1, 256, 0, st>>>(Q, bar);
    e = hipGetLastError();
  } else {
    void* args[] = {(void*)&Q, (void*)&bar};
    e = hipLaunchCooperativeKernel((const void*)k_qcg, dim3(a.qblocks), dim3(256), args, 0, st);
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
