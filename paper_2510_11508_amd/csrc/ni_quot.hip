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
//   edges lighter than w_cut_rel * max_e w_e are dropped (only weights
//   at the edge of FP64 underflow with the default 1e-12);
//   quotient Laplacian sum_e w_e (e_lo - e_hi)(e_lo - e_hi)^T, rhs
//   -sum_e w_e rho_e (e_lo - e_hi) with rho_e the residual oriented lo->hi;
//   s = solution by multigrid PCG plus one refinement round on the
//   flow-form residual, shifted to zero mean on every connected piece;
//   E_t = sum_e w_e (rho_e + s_lo - s_hi)^2; S += s            (Eq. 12, 17)
#include "ni_common.h"

namespace {

// quotient rows with more entries than QELL are "heavy" (see the row classes below)
constexpr int QELL = 8, QBIG = 512;

// flag[nd p + d]: the usable edge of direction d owned by p joins two
// nodes (nd = 2 directions, or 4 with the diagonals: eb2 non-null)
__global__ void k_inter_flags(const int* __restrict__ label, const uint8_t* __restrict__ ebits,
                              const uint8_t* __restrict__ eb2, int P, int W, int* __restrict__ flag) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int c = label[p];
  const int nd = eb2 ? 4 : 2;
  for (int d = 0; d < nd; ++d)
    flag[nd * p + d] = (ni::dir_usable(ebits, eb2, p, d) && label[p + ni::dir_step(d, W)] != c) ? 1 : 0;
}

// edge codes 4 a + d in ascending order
__global__ void k_inter_compact(const int* __restrict__ flag, const int* __restrict__ epos, long long n, int nd,
                                uint32_t* __restrict__ eidx) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) eidx[epos[i]] = (uint32_t)(4 * (i / nd) + i % nd);
}

__device__ __forceinline__ void edge_ends(uint32_t code, int W, int& a, int& b, int& d) {
  a = (int)(code >> 2);
  d = (int)(code & 3u);
  b = a + ni::dir_step(d, W);
}

// key = max(pi(a), pi(b)) (which = 1) or min (which = 0)
__global__ void k_edge_keys(const uint32_t* __restrict__ eidx, int E, int W, const int* __restrict__ label,
                            int which, uint32_t* __restrict__ key) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  int a, b, h;
  edge_ends(eidx[i], W, a, b, h);
  int c = label[a], d = label[b];
  key[i] = (uint32_t)(which ? max(c, d) : min(c, d));
}

__global__ void k_pair_flags(const uint32_t* __restrict__ eidx, int E, int W, const int* __restrict__ label,
                             int* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  int a, b, a0, b0, h;
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
    int a, b, h;
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

__global__ void k_fill_u64(unsigned long long* a, int n, unsigned long long v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_u32(unsigned* a, int n, unsigned v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_f64(double* a, int n, double v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ---------------------------------------------------------- per iteration
struct EdgeParams {
  int W, align, outlier_mode, t, out_from;
  double g2fx, g2fy, g2fd, k, lL, lU, U;  // f^2 of the right, down and diagonal rows
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
    const uint32_t* __restrict__ eidx, int E, const int* __restrict__ label, const int* __restrict__ glabel,
    const uint8_t* __restrict__ ebits, const uint8_t* __restrict__ eb2, const double* __restrict__ eom,
    const double* __restrict__ eta, const double* __restrict__ etb, const float* __restrict__ zfill,
    const double* __restrict__ S, EdgeParams q, double* __restrict__ ew, double* __restrict__ erho, unsigned long long* __restrict__ wmax_bits) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double w = 0.0;
  if (i < E) {
    int a, b, dir;
    edge_ends(eidx[i], q.W, a, b, dir);
    const int c = label[a], d = label[b];
    const double za = (double)zfill[a] + S[c];
    const double zb = (double)zfill[b] + S[d];
    const double om = eom[i];
    const double r = za - zb - om;
    if (q.t < q.align) {
      w = 2.0;
    } else {
      const int step = ni::dir_step(dir, q.W);
      const double g2f = dir == 0 ? q.g2fx : dir == 1 ? q.g2fy : q.g2fd;
      // row b -> a, opposite pixel a - step (a missing or unusable edge
      // there contributes no difference)
      double dm = 0.0;
      if (ni::has_back(a, dir, q.W) && ni::dir_usable(ebits, eb2, a - step, dir)) {
        int m = a - step;
        dm = ((double)zfill[m] + S[label[m]]) - za;
      }
      const double dp = zb - za;
      const double ta = eta[i];
      const double g2a = g2f * (ta * ta);
      const double wba = g2a * sigmoid_k(g2a * (dm * dm - dp * dp), q.k);
      // row a -> b, opposite pixel b + step
      double dm2 = 0.0;
      if (ni::dir_usable(ebits, eb2, b, dir)) {
        int m = b + step;
        dm2 = ((double)zfill[m] + S[label[m]]) - zb;
      }
      const double dp2 = za - zb;
      const double tb = etb[i];
      const double g2b = g2f * (tb * tb);
      const double wab = g2b * sigmoid_k(g2b * (dm2 * dm2 - dp2 * dp2), q.k);
      w = (wba + wab) * (q.t >= q.out_from ? outlier_w(r, q) : 1.0);
    }
    ew[i] = w;
    erho[i] = (glabel[a] < glabel[b]) ? r : -r;  // oriented lo -> hi of the node pair
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
    b += (e & 1u) ? pB[pid] : -pB[pid];  // row = hi: +B, row = lo: -B
    ba += fabs(pB[pid]);
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
    b += (e & 1u) ? pB[pid] : -pB[pid];
    ba += fabs(pB[pid]);
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

// ------------------------------------------------ quotient matrix (FP64)
// Matrix per iteration: qcol/qw = neighbour id and pair weight of every CSR
// entry, diag = row sum (pure graph Laplacian), applied in difference form
// q_c = sum_d w_cd (p_c - p_d).  Rows with diag = 0 (components whose every
// quotient edge was cut) keep s = 0.
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

// Rows with more than QELL entries ("heavy": a large component can border a
// thousand others) are listed, those above QBIG first; the node and
// residual kernels give each of them a wavefront.
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

// Residual of the relative-scale normal equations in flow form.  Pair p
// (lo, hi) carries the flow f_p = B_p + W_p (s_lo - s_hi), the derivative
// of its energy term W_p (rho_p + s_lo - s_hi)^2 / 2 summed over its edges
// (B_p = sum of w_e rho_e); the residual of row c is the sum of -f_p over
// the pairs where c is lo and +f_p where c is hi.  Each pair's flow is
// formed once (one fused multiply-add) and enters both of its rows with
// opposite signs, so summed over any set of rows the inner pairs cancel
// exactly and only the flows across its boundary remain.  The usual form
// b_c - (L s)_c rounds every row at the scale of its heaviest entries,
// which hides the flows through links many orders of magnitude lighter;
// those alone fix the offset of a piece that hangs by such links.
__device__ __forceinline__ double pair_flow(const double* __restrict__ pW, const double* __restrict__ pB,
                                            const int* __restrict__ plo, const int* __restrict__ phi,
                                            const double* __restrict__ s, int pid) {
  return __fma_rn(pW[pid], s[plo[pid]] - s[phi[pid]], pB[pid]);
}

__global__ void k_flow_resid(const int* __restrict__ row_off, const uint32_t* __restrict__ ent, int K,
                             const double* __restrict__ pW, const double* __restrict__ pB,
                             const int* __restrict__ plo, const int* __restrict__ phi,
                             const double* __restrict__ s, double* __restrict__ r) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K || row_off[c + 1] - row_off[c] > QELL) return;  // long rows: k_flow_resid_heavy
  double acc = 0.0;
  for (int j = row_off[c]; j < row_off[c + 1]; ++j) {
    const uint32_t e = ent[j];
    const double f = pair_flow(pW, pB, plo, phi, s, (int)(e >> 1));
    acc += (e & 1u) ? f : -f;
  }
  r[c] = acc;
}

// the same for the rows with more than QELL entries, one wavefront each
// (lane partials summed by a fixed butterfly)
__global__ void k_flow_resid_heavy(const int* __restrict__ row_off, const uint32_t* __restrict__ ent,
                                   const int* __restrict__ heavy, int nheavy, const double* __restrict__ pW,
                                   const double* __restrict__ pB, const int* __restrict__ plo,
                                   const int* __restrict__ phi, const double* __restrict__ s, double* __restrict__ r) {
  const int h = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (h >= nheavy) return;
  const int c = heavy[h];
  double acc = 0.0;
  for (int j = row_off[c] + lane; j < row_off[c + 1]; j += 64) {
    const uint32_t e = ent[j];
    const double f = pair_flow(pW, pB, plo, phi, s, (int)(e >> 1));
    acc += (e & 1u) ? f : -f;
  }
  acc = ni::wave_sum(acc);
  if (lane == 0) r[c] = acc;
}

__global__ void k_add_f64(double* __restrict__ a, const double* __restrict__ b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += b[i];
}

// Piece sums: the nodes sorted by their piece's root (a stable sort, so
// each piece is one run in node order) and summed per run by run_sums, in
// an order that does not depend on scheduling.  g[i] = v of the i-th node
// in that order (v null: 1, the piece sizes).
__global__ void k_piece_gather(const uint32_t* __restrict__ node, const double* __restrict__ v, int K,
                               double* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) g[i] = v ? v[node[i]] : 1.0;
}

// v -= its mean over the piece (the piece gauge of s; for a right-hand side
// of the singular Laplacian only rounding is removed)
__global__ void k_piece_center(const int* __restrict__ parent, double* __restrict__ v, int K,
                               const double* __restrict__ psum, const double* __restrict__ pcnt) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  const int r = parent[c];
  v[c] -= psum[r] / pcnt[r];
}

// S_c += s of the node that holds component c (Eq. 12; every component of a
// merged node moves with it)
__global__ void k_scale_add(const double* __restrict__ s, const int* __restrict__ grp, int K0,
                            double* __restrict__ S) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K0) S[c] += s[grp ? grp[c] : c];
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

// ------------------------------------------------------------ merging
// Optional merging (Sec. 3.5 (i)-(iii)).  Every node picks the live inter
// edge incident to it with the smallest |residual| at the current
// log-depth, compared on a 2^-40 grid, equal values to the smaller edge
// code; the nodes joined by picked edges become one.  The key of an edge
// is floor(|r| 2^40) (|r| < 2^23 holds for any log-depth residual).
__device__ __forceinline__ unsigned long long merge_key(const uint32_t* eidx, const int* label, const float* zfill,
                                                         const double* S, const double* eom, int W, int i) {
  int a, b, h;
  edge_ends(eidx[i], W, a, b, h);
  const double r = ((double)zfill[a] + S[label[a]]) - ((double)zfill[b] + S[label[b]]) - eom[i];
  return (unsigned long long)floor(fabs(r) * 1099511627776.0);  // 2^40
}

__global__ void k_merge_min(const uint32_t* __restrict__ eidx, int E, int W, const int* __restrict__ label,
                            const int* __restrict__ glabel, const float* __restrict__ zfill,
                            const double* __restrict__ S, const double* __restrict__ eom,
                            unsigned long long* __restrict__ gkey) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  const unsigned long long k = merge_key(eidx, label, zfill, S, eom, W, i);
  int a, b, h;
  edge_ends(eidx[i], W, a, b, h);
  atomicMin(&gkey[glabel[a]], k);
  atomicMin(&gkey[glabel[b]], k);
}

__global__ void k_merge_code(const uint32_t* __restrict__ eidx, int E, int W, const int* __restrict__ label,
                             const int* __restrict__ glabel, const float* __restrict__ zfill,
                             const double* __restrict__ S, const double* __restrict__ eom,
                             const unsigned long long* __restrict__ gkey, unsigned* __restrict__ gcode) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  const unsigned long long k = merge_key(eidx, label, zfill, S, eom, W, i);
  int a, b, h;
  edge_ends(eidx[i], W, a, b, h);
  const int ga = glabel[a], gb = glabel[b];
  if (gkey[ga] == k) atomicMin(&gcode[ga], eidx[i]);
  if (gkey[gb] == k) atomicMin(&gcode[gb], eidx[i]);
}

// the picked edge of node g as a pair (g, other end), or (g, g)
__global__ void k_merge_pairs(const unsigned* __restrict__ gcode, int Kg, int W, const int* __restrict__ glabel,
                              int* __restrict__ pa, int* __restrict__ pb, double* __restrict__ pkeep) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= Kg) return;
  const unsigned code = gcode[g];
  int o = g;
  if (code != 0xffffffffu) {
    int a, b, h;
    edge_ends(code, W, a, b, h);
    o = glabel[a] == g ? glabel[b] : glabel[a];
  }
  pa[g] = g;
  pb[g] = o;
  pkeep[g] = o != g ? 1.0 : 0.0;
}

__global__ void k_root_flags(const int* __restrict__ parent, int n, int* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = parent[i] == i ? 1 : 0;
}

// new node of every component and of every pixel
__global__ void k_merge_relabel(int* __restrict__ grp, int K0, const int* __restrict__ parent,
                                const int* __restrict__ rank) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K0) grp[c] = rank[parent[grp[c]]];
}

__global__ void k_merge_pixels(const int* __restrict__ label, const int* __restrict__ grp, int P,
                               int* __restrict__ glabel) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) {
    const int c = label[p];
    glabel[p] = c >= 0 ? grp[c] : -1;
  }
}

__global__ void k_iota_i32(int* a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
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

hipError_t quot_inter_edges(const int* label, const uint8_t* ebits, const uint8_t* eb2, int P, int W, int* flag,
                            int* epos, int* count_dev, uint32_t* eidx_raw, int* scan_tmp, hipStream_t st, int phase) {
  const int nd = eb2 ? 4 : 2;
  if (phase == 0) {
    k_inter_flags<<<ni::ceil_div(P, 256), 256, 0, st>>>(label, ebits, eb2, P, W, flag);
    return scan_exclusive_i32(flag, epos, nd * P, count_dev, scan_tmp, st);
  }
  k_inter_compact<<<ni::ceil_div((long long)nd * P, 256), 256, 0, st>>>(flag, epos, (long long)nd * P, nd, eidx_raw);
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



// One merge of the quotient nodes (Sec. 3.5): a.glabel / a.K describe the
// current nodes, grp maps components to them; on return grp and glabel_out
// hold the merged nodes and *kg_out their number (device count in cnt).
hipError_t merge_nodes(const IrlsArgs& a, int* grp, int* glabel_out, int P, unsigned long long* gkey, unsigned* gcode,
                       int* pa, int* pb, double* pkeep, int* parent, int* flag, int* rank, int* cnt, int* scan_tmp,
                       hipStream_t st) {
  const int Kg = a.K;
  if (Kg <= 0) return hipSuccess;
  hipError_t e;
  k_fill_u64<<<ni::ceil_div(Kg, 256), 256, 0, st>>>(gkey, Kg, ~0ull);
  k_fill_u32<<<ni::ceil_div(Kg, 256), 256, 0, st>>>(gcode, Kg, 0xffffffffu);
  if (a.E > 0) {
    k_merge_min<<<ni::ceil_div(a.E, 256), 256, 0, st>>>(a.eidx, a.E, a.W, a.label, a.glabel, a.zfill, a.S, a.eom, gkey);
    k_merge_code<<<ni::ceil_div(a.E, 256), 256, 0, st>>>(a.eidx, a.E, a.W, a.label, a.glabel, a.zfill, a.S, a.eom,
                                                         gkey, gcode);
  }
  k_merge_pairs<<<ni::ceil_div(Kg, 256), 256, 0, st>>>(gcode, Kg, a.W, a.glabel, pa, pb, pkeep);
  e = list_components(Kg, pa, pb, pkeep, Kg, parent, st);
  if (e != hipSuccess) return e;
  // roots are the smallest node of each merged set, and node order follows
  // the smallest original component, so ranking the roots numbers the new
  // nodes by their smallest component
  k_root_flags<<<ni::ceil_div(Kg, 256), 256, 0, st>>>(parent, Kg, flag);
  e = scan_exclusive_i32(flag, rank, Kg, cnt, scan_tmp, st);
  if (e != hipSuccess) return e;
  k_merge_relabel<<<ni::ceil_div(a.K0, 256), 256, 0, st>>>(grp, a.K0, parent, rank);
  k_merge_pixels<<<ni::ceil_div(P, 256), 256, 0, st>>>(a.label, grp, P, glabel_out);
  return hipGetLastError();
}

hipError_t identity_groups(int* grp, int K0, hipStream_t st) {
  if (K0 > 0) k_iota_i32<<<ni::ceil_div(K0, 256), 256, 0, st>>>(grp, K0);
  return hipGetLastError();
}

hipError_t irls_iteration(const IrlsArgs& a, int t, hipStream_t st) {
  hipError_t e;
  EdgeParams q;
  q.W = a.W;
  q.align = a.align;
  q.out_from = a.out_from;
  q.outlier_mode = a.outlier_mode;
  q.t = t;
  q.g2fx = a.g2fx;
  q.g2fy = a.g2fy;
  q.g2fd = a.g2fd;
  q.k = a.k;
  q.lL = log10(a.L);
  q.lU = log10(a.U);
  q.U = a.U;
  if (a.K <= 0) return hipSuccess;
  if (a.E > 0) {
    e = hipMemsetAsync(a.wmax, 0, sizeof(unsigned long long), st);
    if (e != hipSuccess) return e;
    k_irls_edges<<<ni::ceil_div(a.E, 256), 256, 0, st>>>(a.eidx, a.E, a.label, a.glabel, a.ebits, a.eb2, a.eom, a.eta,
                                                        a.etb, a.zfill, a.S, q, a.ew, a.erho, a.wmax);
    k_irls_pairs<<<ni::ceil_div(a.P, 256), 256, 0, st>>>(a.pair_start, a.P, a.ew, a.erho, a.wmax, a.cut_rel, a.pW,
                                                        a.pB);
  }
  k_irls_nodes<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.row_off, a.ent, a.K, a.pW, a.pB, a.diag, a.rhs, a.babs);
  if (a.nheavy > 0)
    k_irls_nodes_heavy<<<ni::ceil_div(a.nheavy, 4), 256, 0, st>>>(a.row_off, a.ent, a.heavy, a.nheavy, a.pW, a.pB,
                                                                   a.diag, a.rhs, a.babs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // pieces of the weighted quotient graph, and the nodes in piece order
  e = list_components(a.K, a.pair_lo, a.pair_hi, a.pW, a.P, a.parent, st);
  if (e != hipSuccess) return e;
  {
    int bits = 1;
    while ((1ll << bits) < (long long)a.K) ++bits;
    k_iota_u32<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.pnode_in, a.K);
    e = radix_sort_pairs(reinterpret_cast<const uint32_t*>(a.parent), a.pnode_in, a.pkey, a.pnode, a.pk_tmp,
                         a.pv_tmp, a.K, bits, a.pscan, st);
    if (e != hipSuccess) return e;
  }
  auto piece_sums = [&](const double* v, double* out) {
    k_piece_gather<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.pnode, v, a.K, a.pval);
    return run_sums(a.pkey, a.pval, a.K, out, a.prun, st);
  };
  e = piece_sums(nullptr, a.pcnt);
  if (e != hipSuccess) return e;
  // a right-hand side of a singular system is consistent in exact
  // arithmetic (zero sum over every piece); rounding is taken out before
  // each solve round, so that the round's relative tolerance can be met
  auto center = [&](double* v) {
    hipError_t ce = piece_sums(v, a.psum);
    k_piece_center<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.parent, v, a.K, a.psum, a.pcnt);
    return ce;
  };
  e = center(a.rhs);
  if (e != hipSuccess) return e;
  // quotient solve: multigrid-preconditioned CG on a hierarchy built from
  // this step's weights (the cut set and the weights change from step to
  // step; the uniform-weight steps t < align share one matrix and the
  // hierarchy of step 0)
  if (a.nnz > 0) k_q_matrix<<<ni::ceil_div(a.nnz, 256), 256, 0, st>>>(a.row_off, a.ent, a.pair_lo, a.pair_hi, a.pW,
                                                                       a.nnz, a.qcol, a.qw);
  e = hipGetLastError();
  const bool same_as_previous = t > 0 && t < a.align && !a.fresh;
  if (e == hipSuccess && !same_as_previous)
    e = amg_build(a.amg, a.K, a.P, a.row_off, a.qcol, a.qw, a.diag, a.pair_lo, a.pair_hi, a.pW, st);
  if (e == hipSuccess) e = amg_update(a.amg, a.qw, a.diag, a.pW, st);
  // first solve: s from zero to ||r|| <= q_rtol ||b_abs|| (b_abs = row sums of
  // |B_p|, a scale of the right-hand side that does not cancel)
  if (e == hipSuccess)
    e = amg_solve(a.amg, a.rhs, a.babs, nullptr, 0.0, a.s, a.q_rtol, a.q_maxit, a.qiters_out + t, a.host_flag,
                  a.graphs != 0, st, a.hints);
  // second solve (refinement): the residual of s in flow form, then the
  // correction d from zero to ||r_d|| <= max(q_rtol2 ||b - L s||, 1e-13
  // ||b_abs||), s += d.  The recursive residual of the first solve carries rounding
  // at the scale of the heaviest rows; the flow-form residual restores what
  // the light links say, and the correction solve, whose right-hand side
  // is small, resolves it.  The floor is the rounding level of the
  // right-hand side itself.
  if (e == hipSuccess) {
    k_flow_resid<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.row_off, a.ent, a.K, a.pW, a.pB, a.pair_lo, a.pair_hi,
                                                         a.s, a.t0);
    if (a.nheavy > 0)
      k_flow_resid_heavy<<<ni::ceil_div(a.nheavy, 4), 256, 0, st>>>(a.row_off, a.ent, a.heavy, a.nheavy, a.pW, a.pB,
                                                                    a.pair_lo, a.pair_hi, a.s, a.t0);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = center(a.t0);
  if (e == hipSuccess)
    e = amg_solve(a.amg, a.t0, a.t0, a.babs, 1e-13, a.t1, a.q_rtol2, a.q_maxit, a.qiters2_out + t, a.host_flag,
                  a.graphs != 0, st, a.hints ? a.hints + 1 : nullptr);
  if (e == hipSuccess) {
    k_add_f64<<<ni::ceil_div(a.K, 256), 256, 0, st>>>(a.s, a.t1, a.K);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  // piece gauge and accumulate S
  e = center(a.s);
  if (e != hipSuccess) return e;
  k_scale_add<<<ni::ceil_div(a.K0, 256), 256, 0, st>>>(a.s, a.grp, a.K0, a.S);
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
