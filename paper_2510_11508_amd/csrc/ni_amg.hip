// Aggregation multigrid preconditioner for the quotient relative-scale
// systems (Sec. 3.4, Eq. 16-17) of large component graphs.
//
// The quotient Laplacian of a large map is badly conditioned: after the
// weight cut it splits into many pieces, and regions where every pixel is
// its own component form grid-like sub-graphs.  Jacobi PCG then needs
// thousands of iterations per IRLS step.  Here the CG is preconditioned by
// one V-cycle of an aggregation hierarchy:
//
//   aggregation   pairwise handshakes (each free node proposes its strongest
//                 free neighbour among its strong entries, those within a
//                 factor ATHETA of the row's heaviest; equal weights
//                 ordered by a hash of the edge; mutual proposals pair up;
//                 three rounds), then every node left over joins the
//                 aggregate of its strongest aggregated strong neighbour,
//                 or stays alone; nodes without a weighted edge take no
//                 part.  Aggregate ids follow the smallest
//                 member, so the hierarchy is deterministic.
//   coarse graph  Galerkin product with piecewise-constant prolongation: a
//                 coarse pair's weight is the sum of the fine pair weights
//                 between the two aggregates (again a weighted graph
//                 Laplacian), summed in a fixed order.
//   cycle         V(1,1) with damped Jacobi (omega = 2/3) on every level
//                 and an exact solve on the coarsest (<= AMAXC nodes): one
//                 node per connected piece is pinned to zero and the
//                 remaining SPD matrix is inverted once per IRLS step.
//
// The pre- and post-smoothers are the same and restriction is the
// transpose of prolongation, so the cycle is a symmetric positive operator
// and plain PCG applies.  The hierarchy is rebuilt from every IRLS step's
// weights: a hierarchy kept from one step loses most of its effect a few
// steps later, once the weight cut has moved.
//
// All reductions are block partials summed in block order by a one-block
// kernel, so results are reproducible run to run.
#include <vector>

#include "ni_common.h"

namespace {

constexpr int ANT = 256;      // threads per block, one row per thread
constexpr int AH = 16;        // rows with more entries are heavy: one block each
constexpr int AMAXC = 128;    // largest coarsest level solved exactly (its matrix fits in LDS)
constexpr int AMAXL = 24;     // levels at most
constexpr double AOMEGA = 2.0 / 3.0;

// scalars of the PCG, one double each
enum { S_RHO = 0, S_RHOP, S_BETA, S_ALPHA, S_RR, S_BS, S_PQ, S_RH0, S_RH1, S_FL, S_N };

// device view of one level
struct ALev {
  int n, nblk, nheavy;
  const int* row_off;  // [n+1]
  const int* col;      // neighbour of every entry
  const double* w;     // weight of every entry
  const double* diag;  // row sums
  const int* heavy;    // rows with more than AH entries
  const int* cid;      // node -> node of the next level (-1: none); null on the coarsest
  const int* ccol;     // entry -> node of the next level of its neighbour (cid of col); null on the coarsest
  double *b, *x, *r, *y;
};

__device__ __forceinline__ bool is_done(const int* done) { return *reinterpret_cast<const volatile int*>(done) != 0; }

// row index handled by this thread: regular blocks skip heavy rows; heavy
// blocks (index >= nblk) take one heavy row with all threads
struct RowSel {
  int c;      // row, or -1
  bool big;   // block-wide row
};

__device__ __forceinline__ RowSel row_sel(const ALev& L) {
  RowSel s;
  if ((int)blockIdx.x < L.nblk) {
    const int c = blockIdx.x * ANT + threadIdx.x;
    s.big = false;
    s.c = (c < L.n && L.row_off[c + 1] - L.row_off[c] <= AH) ? c : -1;
  } else {
    s.big = true;
    s.c = L.heavy[blockIdx.x - L.nblk];
  }
  return s;
}

// sum over the entries j of row c of w_j * (vc - val(col_j, j)); a heavy
// row is split over the block's threads (then summed by the caller).
// Entries past the row's end enter as w = 0 with val(c, -1).
template <class V>
__device__ __forceinline__ double row_diff_sum(const ALev& L, const RowSel& s, double vc, V val) {
  const int j0 = L.row_off[s.c], j1 = L.row_off[s.c + 1];
  const int t0 = s.big ? threadIdx.x : 0, st = s.big ? ANT : 1;
  double acc = 0.0;
  for (int base = j0 + t0; base < j1; base += 8 * st) {
    int d[8], e[8];
    double q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = base + u * st;
      d[u] = j < j1 ? L.col[j] : s.c;
      e[u] = j < j1 ? j : -1;
      q[u] = j < j1 ? L.w[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += q[u] * (vc - val(d[u], e[u]));
  }
  return acc;
}

template <int NV>
__device__ __forceinline__ void put_parts(double (&v)[NV], double* red, double* parts, int stride) {
  ni::block_sum<NV>(v, red);
  if (threadIdx.x < NV) parts[(size_t)threadIdx.x * stride + blockIdx.x] = v[threadIdx.x];
}

// ------------------------------------------------------------------ cycle
// The cycle and CG kernels are instantiated twice, FILL = 1 for the fill
// of the large components and 0 for the relative-scale systems: the same
// code under two names, so that kernel traces separate the two solves.
// pre-smoothing from zero and the residual: r = b - A x with x = w D^-1 b
// (x itself is recomputed where it is needed)
template <int FILL>
__global__ void __launch_bounds__(ANT) k_cy_down(ALev L, const int* done) {
  if (is_done(done)) return;
  __shared__ double red[ANT / 64];
  const RowSel s = row_sel(L);
  const double* b = L.b;
  const double* dg = L.diag;
  auto xv = [&](int d, int) { const double e = dg[d]; return e > 0 ? AOMEGA * b[d] / e : 0.0; };
  double acc = 0.0;
  if (s.c >= 0) acc = row_diff_sum(L, s, xv(s.c, -1), xv);
  if (s.big) {
    double t[1] = {acc};
    ni::block_sum<1>(t, red);
    acc = t[0];
  }
  if (s.c >= 0 && (!s.big || threadIdx.x == 0)) L.r[s.c] = b[s.c] - acc;
}

// restriction b' = P^T r: each coarse node sums its members' residuals
// (aggregates with more than AH members are summed by a whole block)
template <int FILL>
__global__ void __launch_bounds__(ANT) k_cy_restrict(int n, int nblk, const int* __restrict__ mem_off,
                                                     const int* __restrict__ mem, const int* __restrict__ mheavy,
                                                     const double* __restrict__ r, double* __restrict__ bc,
                                                     const int* done) {
  if (is_done(done)) return;
  __shared__ double red[ANT / 64];
  int C;
  bool big;
  if ((int)blockIdx.x < nblk) {
    C = blockIdx.x * ANT + threadIdx.x;
    big = false;
    if (C >= n || mem_off[C + 1] - mem_off[C] > AH) C = -1;
  } else {
    C = mheavy[blockIdx.x - nblk];
    big = true;
  }
  double acc = 0.0;
  if (C >= 0) {
    const int i0 = mem_off[C], i1 = mem_off[C + 1];
    for (int i = i0 + (big ? threadIdx.x : 0); i < i1; i += big ? ANT : 1) acc += r[mem[i]];
  }
  if (big) {
    double t[1] = {acc};
    ni::block_sum<1>(t, red);
    acc = t[0];
  }
  if (C >= 0 && (!big || threadIdx.x == 0)) bc[C] = acc;
}

// exact coarsest solve y = A^+ b with the pinned inverse: one block of
// CO_NT threads, CO_P per output (strided over the inverse's rows, then
// summed over those lanes in a fixed order)
constexpr int CO_P = 8, CO_NT = AMAXC * CO_P;
template <int FILL>
__global__ void __launch_bounds__(CO_NT) k_cy_coarsest(int n, const double* __restrict__ ainv,
                                                       const uint8_t* __restrict__ pin, const double* __restrict__ b,
                                                       double* __restrict__ y, const int* done) {
  if (is_done(done)) return;
  __shared__ double bl[AMAXC];
  for (int i = threadIdx.x; i < n; i += blockDim.x) bl[i] = pin[i] ? 0.0 : b[i];
  __syncthreads();
  const int c = threadIdx.x / CO_P, part = threadIdx.x % CO_P;
  double acc = 0.0;
  if (c < n)
    for (int j = part; j < n; j += CO_P) acc += ainv[(size_t)j * n + c] * bl[j];  // symmetric: column c = row c
#pragma unroll
  for (int o = 1; o < CO_P; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (c < n && part == 0) y[c] = acc;
}

// block partials of (b, y) on a level whose cycle is the exact solve alone
// (a hierarchy of one level); heavy blocks write zero partials
template <int FILL>
__global__ void __launch_bounds__(ANT) k_cy_dot(ALev L, double* __restrict__ parts, int pstride, const int* done) {
  if (is_done(done)) return;
  __shared__ double red[ANT / 64];
  const int c = blockIdx.x * ANT + threadIdx.x;
  double v[1] = {0.0};
  if ((int)blockIdx.x < L.nblk && c < L.n) v[0] = L.b[c] * L.y[c];
  put_parts<1>(v, red, parts, pstride);
}

// prolongation and post-smoothing: x = w D^-1 b + corr P y',
// y = x + w D^-1 (b - A x) (yn = null: no coarser level, the two Jacobi
// sweeps only).  corr > 1 over-corrects: piecewise-constant prolongation
// over 4:1 aggregates undershoots smooth errors, and a constant factor
// below 2 keeps the cycle symmetric positive definite.  On the finest level
// the block partials of (b, y) are written to parts.
template <int FILL>
__global__ void __launch_bounds__(ANT) k_cy_up(ALev L, const double* __restrict__ yn, double* __restrict__ parts,
                                               int pstride, double corr, const int* done) {
  if (is_done(done)) return;
  __shared__ double red[ANT / 64];
  const RowSel s = row_sel(L);
  const double* b = L.b;
  const double* dg = L.diag;
  const int* cid = L.cid;
  const int* ccol = L.ccol;
  // the own row's value; a neighbour's takes its coarse node from the
  // entry (ccol), which saves a dependent load of cid
  auto xown = [&](int d) {
    const double e = dg[d];
    double v = e > 0 ? AOMEGA * b[d] / e : 0.0;
    if (yn) {
      const int k = cid[d];
      if (k >= 0) v += corr * yn[k];
    }
    return v;
  };
  double acc = 0.0, xc = 0.0;
  if (s.c >= 0) {
    xc = xown(s.c);
    auto xv = [&](int d, int j) {
      if (j < 0) return xc;
      const double e = dg[d];
      double v = e > 0 ? AOMEGA * b[d] / e : 0.0;
      if (yn) {
        const int k = ccol[j];
        if (k >= 0) v += corr * yn[k];
      }
      return v;
    };
    acc = row_diff_sum(L, s, xc, xv);
  }
  if (s.big) {
    double t[1] = {acc};
    ni::block_sum<1>(t, red);
    acc = t[0];
  }
  double v[1] = {0.0};
  if (s.c >= 0 && (!s.big || threadIdx.x == 0)) {
    const double e = L.diag[s.c];
    const double yc = e > 0 ? xc + AOMEGA * (L.b[s.c] - acc) / e : 0.0;
    L.y[s.c] = yc;
    v[0] = L.b[s.c] * yc;
  }
  if (parts) {
    __syncthreads();
    put_parts<1>(v, red, parts, pstride);
  }
}

// ------------------------------------------------------------------ tail
// The coarse end of the cycle in one workgroup.  Below a few thousand
// nodes a level's kernels are bound by their chain of dependent global
// loads (offsets, entries, gathered neighbour values: ~6-10 us each, three
// kernels per level).  From level t0 on, every level (the coarsest
// included) is copied into LDS at the start of one kernel, and the down
// sweep, the restrictions, the exact coarsest solve and the up sweep run
// there between barriers.  Rows of at most AH entries are summed in the
// order of the per-level kernels; longer rows by a wavefront (lanes
// strided over the entries, then the butterfly) instead of a block, and
// aggregates of any size in member order.  The prolongation is a scatter:
// each coarse node adds its correction to the x of its members.
constexpr int TNT = 1024;              // threads of the tail workgroup
constexpr int TMAXL = 10;              // tail levels at most
constexpr int TAIL_LDS = 152 * 1024;   // bytes of LDS the tail may use
static_assert(AMAXC * CO_P == TNT, "the coarsest solve takes CO_P threads per node");
static_assert(TAIL_LDS <= 10 * 16 * TNT, "the image is copied with ten 16-byte loads per thread");
static_assert(sizeof(uint4) == 16, "16-byte copies");

// one tail level: sizes and byte offsets of its arrays in LDS (this table
// heads the image), then the global sources of the packed arrays
struct TOff {
  int n, nnz, nh, nmem;  // rows, entries, rows with more than AH entries, members (finer rows with a node here)
  int o_ro, o_col, o_w, o_dg, o_b, o_x, o_y, o_mo, o_mem, o_hv;
};
struct TLev : TOff {
  const int *row_off, *col, *mem_off, *mem, *heavy;
  const double *w, *diag;
};
constexpr int TTAB = (TMAXL * (int)sizeof(TOff) + 15) & ~15;  // bytes of the table
// The LDS arena: the level table, the per-step arrays of every level
// (16-bit row offsets, columns and member lists, FP64 weights and row
// sums, pinned flags), all packed once per solve into a global image of
// the same layout and copied in with one 16-byte load per thread and
// chunk; then the vectors of the cycle (b, x, y), which the kernel writes
// before it reads them.
struct TailPlan {
  int nl;             // tail levels, the coarsest included (at least 2)
  int o_pin;          // pinned flags of the coarsest
  int img_bytes;      // bytes of the packed image (a multiple of 16)
  double corr;        // coarse-correction factor
  const double* bin;  // b of the first tail level (written by the restriction above it)
  double* yout;       // its y (read by the up sweep above it)
  const double* ainv;
  const uint8_t* pin;
  unsigned char* img;
  TLev lv[TMAXL];
};
// the tail kernel's arguments: the image and what the first level needs
// before the image has landed
struct TailHead {
  int nl, o_pin, img_bytes, n0, o_b0, o_x0;
  double corr;
  const double *bin, *diag0, *ainv;
  double* yout;
  const unsigned char* img;
};

// pack the per-step arrays of tail level blockIdx.y into the image
__global__ void k_tail_pack(TailPlan T) {
  const int k = blockIdx.y;
  const TLev& L = T.lv[k];
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x, st = gridDim.x * blockDim.x;
  unsigned char* im = T.img;
  if (k + 1 < T.nl) {
    uint16_t* ro = reinterpret_cast<uint16_t*>(im + L.o_ro);
    for (int i = i0; i <= L.n; i += st) ro[i] = (uint16_t)L.row_off[i];
    uint16_t* cl = reinterpret_cast<uint16_t*>(im + L.o_col);
    double* w = reinterpret_cast<double*>(im + L.o_w);
    for (int i = i0; i < L.nnz; i += st) {
      cl[i] = (uint16_t)L.col[i];
      w[i] = L.w[i];
    }
    double* dg = reinterpret_cast<double*>(im + L.o_dg);
    for (int i = i0; i < L.n; i += st) dg[i] = L.diag[i];
    uint16_t* hv = reinterpret_cast<uint16_t*>(im + L.o_hv);
    for (int i = i0; i < L.nh; i += st) hv[i] = (uint16_t)L.heavy[i];
  } else {
    for (int i = i0; i < L.n; i += st) im[T.o_pin + i] = T.pin[i];
  }
  if (k > 0) {
    uint16_t* mo = reinterpret_cast<uint16_t*>(im + L.o_mo);
    for (int i = i0; i <= L.n; i += st) mo[i] = (uint16_t)L.mem_off[i];
    uint16_t* mem = reinterpret_cast<uint16_t*>(im + L.o_mem);
    for (int i = i0; i < L.nmem; i += st) mem[i] = (uint16_t)L.mem[i];
  }
}

// LDS loops of the tail.  Sum over the entries j0 <= j < j1 of
// w_j (xc - x[col_j]), in entry order (the order of row_diff_sum on a
// regular row).  A plain loop: in a synthetic one-workgroup phase of 889
// rows it took 1.1 us against 1.8 us for eight predicated loads per step;
// in the tail itself the two are within the noise.
__device__ __forceinline__ double lds_row_sum(const uint16_t* cl, const double* w, const double* x, int j0, int j1,
                                              double xc) {
  double acc = 0.0;
  for (int j = j0; j < j1; ++j) acc += w[j] * (xc - x[cl[j]]);
  return acc;
}

// The member loops keep eight independent loads in flight per step:
// indices past the end are clamped to the last element (in bounds, its
// term discarded), so the loads need no branches.
// sum of v[mem[i]] over i0 <= i < i1, in order
__device__ __forceinline__ double lds_gather_sum(const uint16_t* mem, const double* v, int i0, int i1) {
  double s = 0.0;
  for (int base = i0; base < i1; base += 8) {
    double q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = v[mem[min(base + u, i1 - 1)]];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (base + u < i1) s += q[u];
  }
  return s;
}

// v[mem[i]] += a for i0 <= i < i1 (members are distinct)
__device__ __forceinline__ void lds_scatter_add(const uint16_t* mem, double* v, int i0, int i1, double a) {
  for (int base = i0; base < i1; base += 8) {
    int m[8];
    double q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) m[u] = mem[min(base + u, i1 - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = v[m[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (base + u < i1) v[m[u]] = q[u] + a;
  }
}

template <int FILL>
__global__ void __launch_bounds__(TNT) k_cy_tail(TailHead T, const int* done) {
  if (is_done(done)) return;
  __shared__ __align__(16) unsigned char sm[TAIL_LDS];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int NW = TNT / 64;
  auto u16 = [&](int o) { return reinterpret_cast<uint16_t*>(sm + o); };
  auto f64 = [&](int o) { return reinterpret_cast<double*>(sm + o); };
  const int nl = T.nl;
  const uint8_t* pin = sm + T.o_pin;
  const TOff* lv = reinterpret_cast<const TOff*>(sm);
  // ---- the image, all loads in flight at once; b and x = w D^-1 b of
  // the first level (its row sums taken from global memory)
  {
    const uint4* src = reinterpret_cast<const uint4*>(T.img);
    uint4* dst = reinterpret_cast<uint4*>(sm);
    const int nv = T.img_bytes / 16;
    const uint4 z = make_uint4(0, 0, 0, 0);
    uint4 v0 = z, v1 = z, v2 = z, v3 = z, v4 = z, v5 = z, v6 = z, v7 = z, v8 = z, v9 = z;
#define TAIL_LD(u) if (tid + (u) * TNT < nv) v##u = src[tid + (u) * TNT];
#define TAIL_ST(u) if (tid + (u) * TNT < nv) dst[tid + (u) * TNT] = v##u;
    TAIL_LD(0) TAIL_LD(1) TAIL_LD(2) TAIL_LD(3) TAIL_LD(4) TAIL_LD(5) TAIL_LD(6) TAIL_LD(7) TAIL_LD(8) TAIL_LD(9)
    double *b = f64(T.o_b0), *x = f64(T.o_x0);
    for (int i = tid; i < T.n0; i += TNT) {
      const double bi = T.bin[i], e = T.diag0[i];
      b[i] = bi;
      x[i] = e > 0 ? AOMEGA * bi / e : 0.0;
    }
    TAIL_ST(0) TAIL_ST(1) TAIL_ST(2) TAIL_ST(3) TAIL_ST(4) TAIL_ST(5) TAIL_ST(6) TAIL_ST(7) TAIL_ST(8) TAIL_ST(9)
#undef TAIL_LD
#undef TAIL_ST
  }
  __syncthreads();
  // ---- down: residual r = b - A x (into y), restriction to the next level
  for (int k = 0; k + 1 < nl; ++k) {
    const TOff L = lv[k];
    const uint16_t *ro = u16(L.o_ro), *cl = u16(L.o_col), *hv = u16(L.o_hv);
    const double *w = f64(L.o_w), *b = f64(L.o_b), *x = f64(L.o_x);
    double* r = f64(L.o_y);
    for (int c = tid; c < L.n; c += TNT) {
      const int j0 = ro[c], j1 = ro[c + 1];
      if (j1 - j0 > AH) continue;
      r[c] = j1 > j0 ? b[c] - lds_row_sum(cl, w, x, j0, j1, x[c]) : b[c] - 0.0;
    }
    for (int h = wid; h < L.nh; h += NW) {
      const int c = hv[h], j0 = ro[c], j1 = ro[c + 1];
      const double xc = x[c];
      double acc = 0.0;
      for (int j = j0 + lane; j < j1; j += 64) acc += w[j] * (xc - x[cl[j]]);
      acc = ni::wave_sum(acc);
      if (lane == 0) r[c] = b[c] - acc;
    }
    __syncthreads();
    const TOff C = lv[k + 1];
    const bool coarsest = k + 2 == nl;
    const uint16_t *mo = u16(C.o_mo), *mem = u16(C.o_mem);
    double* bc = f64(C.o_b);
    for (int c = tid; c < C.n; c += TNT) {
      const double s = lds_gather_sum(mem, r, mo[c], mo[c + 1]);
      if (coarsest) {
        bc[c] = pin[c] ? 0.0 : s;
      } else {
        bc[c] = s;
        const double e = f64(C.o_dg)[c];
        f64(C.o_x)[c] = e > 0 ? AOMEGA * s / e : 0.0;
      }
    }
    __syncthreads();
  }
  // ---- exact coarsest solve (CO_P threads per node, as k_cy_coarsest),
  // prolonged into the x of the level above
  {
    const TOff C = lv[nl - 1];
    const int n = C.n;
    const double* bc = f64(C.o_b);
    const int c = tid / CO_P, part = tid % CO_P;
    double acc = 0.0;
    if (c < n)
      for (int j = part; j < n; j += CO_P) acc += T.ainv[(size_t)j * n + c] * bc[j];
#pragma unroll
    for (int o = 1; o < CO_P; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (c < n && part == 0) {
      const uint16_t *mo = u16(C.o_mo), *mem = u16(C.o_mem);
      double* xf = f64(lv[nl - 2].o_x);
      lds_scatter_add(mem, xf, mo[c], mo[c + 1], T.corr * acc);
    }
    __syncthreads();
  }
  // ---- up: y = x + w D^-1 (b - A x), prolonged into the level above (or
  // written out on the first tail level)
  for (int k = nl - 2; k >= 0; --k) {
    const TOff L = lv[k];
    const uint16_t *ro = u16(L.o_ro), *cl = u16(L.o_col), *hv = u16(L.o_hv);
    const double *w = f64(L.o_w), *b = f64(L.o_b), *x = f64(L.o_x), *dg = f64(L.o_dg);
    const uint16_t *mo = k > 0 ? u16(L.o_mo) : nullptr, *mem = k > 0 ? u16(L.o_mem) : nullptr;
    double* xf = k > 0 ? f64(lv[k - 1].o_x) : nullptr;
    for (int c = tid; c < L.n; c += TNT) {
      const int j0 = ro[c], j1 = ro[c + 1];
      if (j1 - j0 > AH) continue;
      const double xc = x[c];
      const double acc = j1 > j0 ? lds_row_sum(cl, w, x, j0, j1, xc) : 0.0;
      const double e = dg[c];
      const double yc = e > 0 ? xc + AOMEGA * (b[c] - acc) / e : 0.0;
      if (k == 0) {
        T.yout[c] = yc;
      } else {
        lds_scatter_add(mem, xf, mo[c], mo[c + 1], T.corr * yc);
      }
    }
    for (int h = wid; h < L.nh; h += NW) {
      const int c = hv[h], j0 = ro[c], j1 = ro[c + 1];
      const double xc = x[c];
      double acc = 0.0;
      for (int j = j0 + lane; j < j1; j += 64) acc += w[j] * (xc - x[cl[j]]);
      acc = ni::wave_sum(acc);
      const double e = dg[c];
      const double yc = e > 0 ? xc + AOMEGA * (b[c] - acc) / e : 0.0;
      if (k == 0) {
        if (lane == 0) T.yout[c] = yc;
      } else {
        for (int i = mo[c] + lane; i < mo[c + 1]; i += 64) xf[mem[i]] += T.corr * yc;
      }
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------------- PCG
// x = 0, r = b, p = q = 0; partials of (r, r), |scale|^2 and |floor|^2
__global__ void __launch_bounds__(ANT) k_cg_init(int n, const double* __restrict__ rhs, const double* __restrict__ scale,
                                                 const double* __restrict__ floorv, double floor_ratio,
                                                 double* __restrict__ x, double* __restrict__ r, double* __restrict__ p,
                                                 double* __restrict__ q, double* __restrict__ sc,
                                                 double* __restrict__ parts, int pstride) {
  __shared__ double red[3 * (ANT / 64)];
  const int c = blockIdx.x * ANT + threadIdx.x;
  if (c == 0) sc[S_FL] = floor_ratio;
  double v[3] = {0.0, 0.0, 0.0};
  if (c < n) {
    const double b = rhs[c];
    x[c] = 0.0;
    r[c] = b;
    p[c] = 0.0;
    q[c] = 0.0;
    v[0] = b * b;
    v[1] = scale[c] * scale[c];
    v[2] = floorv ? floorv[c] * floorv[c] : 0.0;
  }
  put_parts<3>(v, red, parts, pstride);
}

// p = z + beta p, q = A z + beta q (= A p), block partials of (p, q)
template <int FILL>
__global__ void __launch_bounds__(ANT) k_cg_pq(ALev L, double* __restrict__ p, double* __restrict__ q,
                                               const double* __restrict__ sc, double* __restrict__ parts,
                                               int pstride, const int* done) {
  if (is_done(done)) return;
  __shared__ double red[ANT / 64];
  const RowSel s = row_sel(L);
  const double* z = L.y;
  auto zv = [&](int d, int) { return z[d]; };
  double acc = 0.0;
  if (s.c >= 0) acc = row_diff_sum(L, s, z[s.c], zv);
  if (s.big) {
    double t[1] = {acc};
    ni::block_sum<1>(t, red);
    acc = t[0];
  }
  double v[1] = {0.0};
  if (s.c >= 0 && (!s.big || threadIdx.x == 0)) {
    const double beta = sc[S_BETA];
    const double pn = z[s.c] + beta * p[s.c];
    const double qn = acc + beta * q[s.c];
    p[s.c] = pn;
    q[s.c] = qn;
    v[0] = pn * qn;
  }
  __syncthreads();
  put_parts<1>(v, red, parts, pstride);
}

// x += alpha p, r -= alpha q, block partials of (r, r)
__global__ void __launch_bounds__(ANT) k_cg_xr(int n, double* __restrict__ x, double* __restrict__ r,
                                               const double* __restrict__ p, const double* __restrict__ q,
                                               const double* __restrict__ sc, double* __restrict__ parts,
                                               const int* done) {
  if (is_done(done)) return;
  __shared__ double red[ANT / 64];
  const int c = blockIdx.x * ANT + threadIdx.x;
  double v[1] = {0.0};
  if (c < n) {
    const double a = sc[S_ALPHA];
    x[c] += a * p[c];
    const double rn = r[c] - a * q[c];
    r[c] = rn;
    v[0] = rn * rn;
  }
  put_parts<1>(v, red, parts, gridDim.x);
}

// one-block scalar steps; partial arrays are summed in block order
__device__ __forceinline__ double sum_parts(const double* parts, int n, double* red) {
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += blockDim.x) v[0] += parts[i];
  ni::block_sum<1>(v, red);
  return v[0];
}

// mode 0 (after init): rr and |b|^2 from nrr partials at parts and
// parts + pstride.  mode 1 (after the cycle): rho from np partials at
// parts; rr of the last update from nrr partials at parts + pstride (none
// before the first update); convergence test, beta.  mode 2 (after (p, q)):
// alpha.
constexpr int SC_NT = 1024;  // threads of the one-block scalar kernel (a short chain of loads each)
template <int FILL>
__global__ void __launch_bounds__(SC_NT) k_cg_scal(int mode, const double* __restrict__ parts, int np, int pstride,
                                                   int nrr, double* __restrict__ sc, int* __restrict__ done,
                                                   int* it_ctr, double rtol, int maxit, int* __restrict__ iters_out,
                                                   int* __restrict__ flag) {
  __shared__ double red[SC_NT / 64];
  if (mode != 0 && is_done(done)) return;
  if (mode == 0) {
    const double rr = sum_parts(parts, nrr, red);
    __syncthreads();
    const double bs = sum_parts(parts + pstride, nrr, red);
    __syncthreads();
    const double fs = sum_parts(parts + 2 * (size_t)pstride, nrr, red);
    if (threadIdx.x == 0) {
      sc[S_RR] = rr;
      // stop at ||r|| <= max(rtol |scale|, floor_rel |floor|): the floor
      // enters as an equivalent scale (floor_rel / rtol, set by k_cg_init)
      sc[S_BS] = fmax(bs, fs * sc[S_FL] * sc[S_FL]);
      sc[S_RHOP] = 1.0;
      *done = 0;
      *it_ctr = 0;
      *flag = 1;
    }
  } else if (mode == 1) {
    const int it = *it_ctr;
    const double rho = sum_parts(parts, np, red);
    double rr = 0.0;
    if (it > 0) {
      __syncthreads();
      rr = sum_parts(parts + pstride, nrr, red);
    }
    if (threadIdx.x == 0) {
      if (it > 0) sc[S_RR] = rr;
      if (!(sc[S_RR] > rtol * rtol * sc[S_BS]) || it >= maxit) {
        *done = 1;
        *flag = 0;
        *iters_out = it;
      } else {
        sc[S_BETA] = it == 0 ? 0.0 : rho / sc[S_RHOP];
        sc[S_RHO] = rho;
        sc[S_RHOP] = rho;
        *it_ctr = it + 1;
      }
    }
  } else {
    const double pq = sum_parts(parts, np, red);
    if (threadIdx.x == 0) {
      sc[S_PQ] = pq;
      sc[S_ALPHA] = pq != 0.0 ? sc[S_RHO] / pq : 0.0;
    }
  }
}

// Fused forms of the scalar steps (stream launches; the iteration index `it`
// comes from the host).  Every block sums the same partials in the same
// order, so all blocks take the same decisions and scalars without a
// one-block kernel between the launches.  rho of iteration it is kept in
// slot S_RH0 + (it & 1): blocks read the previous iteration's slot while
// block 0 writes the current one.  Partials: rho at parts (from the
// finest k_cy_up), (r, r) at parts + pstride, (p, q) at parts + 2 pstride.
__global__ void __launch_bounds__(ANT) k_cg_pq_f(ALev L, double* __restrict__ p, double* __restrict__ q,
                                                 double* __restrict__ sc, double* __restrict__ parts, int pstride,
                                                 int np, int nrr, int it, double rtol, int maxit,
                                                 int* __restrict__ done, int* __restrict__ flag,
                                                 int* __restrict__ iters_out) {
  if (is_done(done)) return;
  __shared__ double red[ANT / 64];
  const double rho = sum_parts(parts, np, red);
  __syncthreads();
  const double rr = it > 0 ? sum_parts(parts + pstride, nrr, red) : sc[S_RR];
  if (!(rr > rtol * rtol * sc[S_BS]) || it >= maxit) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *done = 1;
      *flag = 0;
      *iters_out = it;
    }
    return;
  }
  const double beta = it == 0 ? 0.0 : rho / sc[S_RH0 + ((it - 1) & 1)];
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[S_RH0 + (it & 1)] = rho;
  const RowSel s = row_sel(L);
  const double* z = L.y;
  auto zv = [&](int d, int) { return z[d]; };
  double acc = 0.0;
  if (s.c >= 0) acc = row_diff_sum(L, s, z[s.c], zv);
  __syncthreads();  // red is reused below
  if (s.big) {
    double t[1] = {acc};
    ni::block_sum<1>(t, red);
    acc = t[0];
  }
  double v[1] = {0.0};
  if (s.c >= 0 && (!s.big || threadIdx.x == 0)) {
    const double pn = z[s.c] + beta * p[s.c];
    const double qn = acc + beta * q[s.c];
    p[s.c] = pn;
    q[s.c] = qn;
    v[0] = pn * qn;
  }
  __syncthreads();
  put_parts<1>(v, red, parts + 2 * (size_t)pstride, pstride);
}

__global__ void __launch_bounds__(ANT) k_cg_xr_f(int n, double* __restrict__ x, double* __restrict__ r,
                                                 const double* __restrict__ p, const double* __restrict__ q,
                                                 const double* __restrict__ sc, double* __restrict__ parts,
                                                 int pstride, int np, int it, const int* done) {
  if (is_done(done)) return;
  __shared__ double red[ANT / 64];
  const double pq = sum_parts(parts + 2 * (size_t)pstride, np, red);
  const double a = pq != 0.0 ? sc[S_RH0 + (it & 1)] / pq : 0.0;
  const int c = blockIdx.x * ANT + threadIdx.x;
  double v[1] = {0.0};
  if (c < n) {
    x[c] += a * p[c];
    const double rn = r[c] - a * q[c];
    r[c] = rn;
    v[0] = rn * rn;
  }
  __syncthreads();  // red is reused below
  put_parts<1>(v, red, parts + pstride, pstride);
}

// ------------------------------------------------------------------ setup
__global__ void k_am_fill(int* a, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// a node takes part when it has an edge of positive weight (row sum > 0);
// nodes with more than AH entries start as aggregates of their own (their
// neighbours may attach to them; scanning their rows would be slow)
__global__ void k_am_active(int n, const int* __restrict__ row_off, const double* __restrict__ diag,
                            int* __restrict__ agg, uint8_t* __restrict__ act) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const bool a = diag[c] > 0.0;
  act[c] = a ? 1 : 0;
  agg[c] = (a && row_off[c + 1] - row_off[c] > AH) ? c : -1;
}

// A symmetric hash of an edge, used to break ties between equal weights.
// (With ties broken by the smaller index, the uniform weights of a pixel
// grid make every node propose to the same side and no proposal is ever
// mutual; a hash of the edge pairs them up like a random matching.)
__device__ __forceinline__ uint32_t edge_hash(int c, int d) {
  uint64_t k = ((uint64_t)(uint32_t)min(c, d) << 32) | (uint32_t)max(c, d);
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return (uint32_t)k;
}

// Strength of connection: an entry (c, d) is strong for c when its weight
// is at least ATHETA times the heaviest entry of row c.  Aggregates grow
// along strong entries only.  The relative-scale weights span many orders
// of magnitude (the BiNI sigmoid of Eq. 5 decays exponentially across a
// depth step), and a node whose strong neighbours are already taken must
// not pair up over a link a million times weaker: the aggregate's constant
// vector would then not be a near-null vector of its rows, and the cycle
// would lose the pieces that hang by weak links.
constexpr double ATHETA = 0.1;

// strongest strong neighbour with agg == -1 (want_free) or agg >= 0; ties
// -> larger edge hash, then smaller index
__device__ __forceinline__ int strongest(int c, const int* row_off, const int* col, const double* w, const int* agg,
                                         const uint8_t* act, bool want_free) {
  double rmax = 0.0;
  for (int j = row_off[c]; j < row_off[c + 1]; ++j)
    if (col[j] != c && act[col[j]]) rmax = fmax(rmax, w[j]);
  const double floor_w = ATHETA * rmax;
  int best = -1;
  double bw = 0.0;
  uint32_t bh = 0;
  for (int j = row_off[c]; j < row_off[c + 1]; ++j) {
    const int d = col[j];
    const double v = w[j];
    if (v <= 0.0 || v < floor_w || d == c || !act[d] || ((agg[d] < 0) != want_free)) continue;
    const uint32_t h = edge_hash(c, d);
    if (v > bw || (v == bw && (h > bh || (h == bh && d < best)))) {
      bw = v;
      bh = h;
      best = d;
    }
  }
  return best;
}

__global__ void k_am_pick(int n, const int* __restrict__ row_off, const int* __restrict__ col,
                          const double* __restrict__ w, const int* __restrict__ agg, const uint8_t* __restrict__ act,
                          int* __restrict__ best) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  best[c] = (act[c] && agg[c] < 0) ? strongest(c, row_off, col, w, agg, act, true) : -1;
}

__global__ void k_am_match(int n, const int* __restrict__ best, int* __restrict__ agg) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int b = best[c];
  if (agg[c] < 0 && b >= 0 && best[b] == c) agg[c] = min(c, b);
}

// leftover active nodes join their strongest aggregated neighbour's
// aggregate, or stay alone; leaders (agg == self) are flagged
__global__ void k_am_attach(int n, const int* __restrict__ row_off, const int* __restrict__ col,
                            const double* __restrict__ w, const int* __restrict__ agg,
                            const uint8_t* __restrict__ act, int* __restrict__ agg2, int* __restrict__ lead) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int a = agg[c];
  if (act[c] && a < 0) {
    const int d = strongest(c, row_off, col, w, agg, act, false);
    a = d >= 0 ? agg[d] : c;
  }
  if (!act[c]) a = -1;
  agg2[c] = a;
  lead[c] = (a == c) ? 1 : 0;
}

__global__ void k_am_cid(int n, const int* __restrict__ agg2, const int* __restrict__ pos, int* __restrict__ cid,
                         int* __restrict__ flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int a = agg2[c];
  cid[c] = a >= 0 ? pos[a] : -1;
  flag[c] = a >= 0 ? 1 : 0;
}

// coarse node of every entry's neighbour
__global__ void k_am_ccol(int ne, const int* __restrict__ col, const int* __restrict__ cid, int* __restrict__ ccol) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < ne) ccol[j] = cid[col[j]];
}

// compact (key, value) of the flagged entries
__global__ void k_am_compact(int n, const int* __restrict__ flag, const int* __restrict__ pos,
                             const int* __restrict__ key, uint32_t* __restrict__ ko, uint32_t* __restrict__ vo) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) {
    ko[pos[i]] = (uint32_t)key[i];
    vo[pos[i]] = (uint32_t)i;
  }
}

// offsets of runs of a sorted key array: off[k] = first index of key k
// (every key 0..nk-1 present), off[nk] = m
__global__ void k_am_offsets(int m, const uint32_t* __restrict__ keys, int nk, int* __restrict__ off) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  if (i == 0 || keys[i] != keys[i - 1]) off[keys[i]] = i;
  if (i == m - 1) off[nk] = m;
}

// offsets when some keys may be absent: counts per key (then scanned)
__global__ void k_am_count(int m, const uint32_t* __restrict__ keys, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) atomicAdd(&cnt[keys[i]], 1);
}

__global__ void k_am_u32(const uint32_t* __restrict__ a, int n, int* __restrict__ o) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = (int)a[i];
}

// coarse pair keys of the fine pairs whose ends lie in two different aggregates
__global__ void k_am_pflag(int np, const int* __restrict__ plo, const int* __restrict__ phi,
                           const int* __restrict__ cid, int* __restrict__ flag) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int a = cid[plo[p]], b = cid[phi[p]];
  flag[p] = (a >= 0 && b >= 0 && a != b) ? 1 : 0;
}

__global__ void k_am_pcompact(int np, const int* __restrict__ flag, const int* __restrict__ pos,
                              const int* __restrict__ plo, const int* __restrict__ phi, const int* __restrict__ cid,
                              uint32_t* __restrict__ klo, uint32_t* __restrict__ khi, uint32_t* __restrict__ fp,
                              uint32_t* __restrict__ idx) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np || !flag[p]) return;
  const int a = cid[plo[p]], b = cid[phi[p]];
  const int i = pos[p];
  klo[i] = (uint32_t)min(a, b);
  khi[i] = (uint32_t)max(a, b);
  fp[i] = (uint32_t)p;
  idx[i] = (uint32_t)i;
}

__global__ void k_am_gather(int m, const uint32_t* __restrict__ a, const uint32_t* __restrict__ idx,
                            uint32_t* __restrict__ o) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) o[i] = a[idx[i]];
}

// runs of equal (lo, hi) in sorted order -> coarse pairs
__global__ void k_am_runs(int m, const uint32_t* __restrict__ ord, const uint32_t* __restrict__ klo,
                          const uint32_t* __restrict__ khi, int* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t k = ord[i];
  flag[i] = (i == 0 || klo[k] != klo[ord[i - 1]] || khi[k] != khi[ord[i - 1]]) ? 1 : 0;
}

__global__ void k_am_pairs_out(int m, const uint32_t* __restrict__ ord, const uint32_t* __restrict__ klo,
                               const uint32_t* __restrict__ khi, const int* __restrict__ flag,
                               const int* __restrict__ pos, const uint32_t* __restrict__ fsrc, int* __restrict__ plo,
                               int* __restrict__ phi, int* __restrict__ gal_off, int* __restrict__ gal_src,
                               int npn) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t k = ord[i];
  gal_src[i] = (int)fsrc[k];
  if (flag[i]) {
    const int q = pos[i];
    plo[q] = (int)klo[k];
    phi[q] = (int)khi[k];
    gal_off[q] = i;
  }
  if (i == m - 1) gal_off[npn] = m;
}

// CSR entries of a pair list: entry e = 2 p + side; row = side ? hi : lo
__global__ void k_am_ekeys(int np, const int* __restrict__ plo, const int* __restrict__ phi,
                           uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * np) return;
  key[e] = (uint32_t)((e & 1) ? phi[e >> 1] : plo[e >> 1]);
  val[e] = (uint32_t)e;
}

__global__ void k_am_ecol(int ne, const uint32_t* __restrict__ ent, const int* __restrict__ plo,
                          const int* __restrict__ phi, int* __restrict__ ento, int* __restrict__ col) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ne) return;
  const int e = (int)ent[j];
  ento[j] = e;
  col[j] = (e & 1) ? plo[e >> 1] : phi[e >> 1];
}

__global__ void k_am_heavy_flag(int n, const int* __restrict__ off, int* __restrict__ flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) flag[c] = off[c + 1] - off[c] > AH ? 1 : 0;
}

__global__ void k_am_list(int n, const int* __restrict__ flag, const int* __restrict__ pos, int* __restrict__ list) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && flag[c]) list[pos[c]] = c;
}

// ------------------------------------------------------- per-step values
// coarse pair weight = sum of its fine pairs' weights (fixed order)
__global__ void k_am_gal(int np, const int* __restrict__ gal_off, const int* __restrict__ gal_src,
                         const double* __restrict__ pwf, double* __restrict__ pw) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  double s = 0.0;
  for (int i = gal_off[q]; i < gal_off[q + 1]; ++i) s += pwf[gal_src[i]];
  pw[q] = s;
}

__global__ void k_am_ew(int ne, const int* __restrict__ ent, const double* __restrict__ pw, double* __restrict__ w) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < ne) w[j] = pw[ent[j] >> 1];
}

__global__ void k_am_diag(int n, const int* __restrict__ row_off, const double* __restrict__ w,
                          double* __restrict__ diag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double s = 0.0;
  for (int j = row_off[c]; j < row_off[c + 1]; ++j) s += w[j];
  diag[c] = s;
}

// Coarsest level (n <= AMAXC): dense Laplacian in LDS, pieces by label
// propagation, the smallest node of every piece (and every node without
// edges) pinned, then an in-place Gauss-Jordan inverse of the SPD rest;
// the inverse goes to A.
__global__ void __launch_bounds__(1024) k_am_invert(int n, const int* __restrict__ row_off, const int* __restrict__ col,
                                                    const double* __restrict__ w, const double* __restrict__ diag,
                                                    double* __restrict__ A, uint8_t* __restrict__ pin) {
  __shared__ double M[AMAXC * AMAXC];
  __shared__ int lab[AMAXC];
  __shared__ uint8_t pn[AMAXC];
  __shared__ int changed;
  __shared__ double colk[AMAXC];
  __shared__ double rowk[AMAXC];
  const int T = blockDim.x;
  for (int i = threadIdx.x; i < n * n; i += T) M[i] = 0.0;
  for (int c = threadIdx.x; c < n; c += T) lab[c] = c;
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += T) {
    M[c * n + c] = diag[c];
    for (int j = row_off[c]; j < row_off[c + 1]; ++j)
      if (w[j] > 0.0) M[c * n + col[j]] -= w[j];
  }
  // pieces: minimum label over edges of positive weight, until stable
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += T) {
      int m = lab[c];
      for (int j = row_off[c]; j < row_off[c + 1]; ++j)
        if (w[j] > 0.0) m = min(m, lab[col[j]]);
      if (m < lab[c]) {
        atomicMin(&lab[c], m);
        changed = 1;
      }
    }
    __syncthreads();
    if (!changed) break;
  }
  for (int c = threadIdx.x; c < n; c += T) {
    pn[c] = (lab[c] == c || !(diag[c] > 0.0)) ? 1 : 0;
    pin[c] = pn[c];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n * n; i += T) {
    const int r = i / n, c = i % n;
    if (pn[r] || pn[c]) M[i] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    for (int i = threadIdx.x; i < n; i += T) {
      colk[i] = M[i * n + k];
      rowk[i] = M[k * n + i];
    }
    __syncthreads();
    const double piv = 1.0 / colk[k];
    for (int idx = threadIdx.x; idx < n * n; idx += T) {
      const int i = idx / n, j = idx % n;
      double v;
      if (i == k) v = (j == k) ? piv : rowk[j] * piv;
      else if (j == k) v = -colk[i] * piv;
      else v = M[idx] - colk[i] * rowk[j] * piv;
      M[idx] = v;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n * n; i += T) A[i] = M[i];
}

// ------------------------------------------- geometric aggregation (fill)
// Pixel graphs carry coordinates: a node of level l stands for the pixels
// of one component inside a 2^l x 2^l block.  Its aggregate on level l+1 is
// the set of nodes of the same component in the same 2x2 block of level-l
// cells (at most four).  Keys: the cell of the aggregate ((y>>1) << bx |
// x>>1, bx bits for x>>1 on this level) and the component.
__global__ void k_gm_keys(int n, const double* __restrict__ diag, const int* __restrict__ gy,
                          const int* __restrict__ gx, const int* __restrict__ gc, int bx, int* __restrict__ kcell,
                          uint32_t* __restrict__ kcomp, int* __restrict__ flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const bool a = diag[c] > 0.0 && gc[c] >= 0;
  flag[c] = a ? 1 : 0;
  kcell[c] = ((gy[c] >> 1) << bx) | (gx[c] >> 1);
  kcomp[c] = a ? (uint32_t)gc[c] : 0u;
}

// first position of every run of equal keys (runs sorted by key, members by
// node index: the first member is the smallest)
__global__ void k_gm_starts(int m, const int* __restrict__ rflag, const int* __restrict__ rpos, int* __restrict__ rs) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m && rflag[j]) rs[rpos[j]] = j;
}

// every member joins the aggregate led by its run's smallest node
__global__ void k_gm_agg(int m, const uint32_t* __restrict__ node, const int* __restrict__ rflag,
                         const int* __restrict__ rpos, const int* __restrict__ rs, int* __restrict__ agg2,
                         int* __restrict__ lead) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int run = rpos[j] - 1 + rflag[j];
  const int ld = (int)node[rs[run]];
  const int me = (int)node[j];
  agg2[me] = ld;
  lead[me] = ld == me ? 1 : 0;
}

// coordinates of the coarse nodes from their leaders
__global__ void k_gm_coarse(int n, const int* __restrict__ agg2, const int* __restrict__ pos,
                            const int* __restrict__ gy, const int* __restrict__ gx, const int* __restrict__ gc,
                            int* __restrict__ cy, int* __restrict__ cx, int* __restrict__ cc) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || agg2[c] != c) return;
  const int k = pos[c];
  cy[k] = gy[c] >> 1;
  cx[k] = gx[c] >> 1;
  cc[k] = gc[c];
}

// ------------------------------------------------- batched fill PCG
// Many independent component systems on one level-0 graph (block
// diagonal); one global alpha and beta, and a stop when every component
// meets its own test ||r_c|| <= rtol ||b_c||.  comp[c] < 0: a node of no
// system (its row is empty and its right-hand side zero).

// r = b - A x for the start x; p = q = 0; per component |r|^2 and |b|^2
__global__ void __launch_bounds__(ANT) k_fs_init(ALev L, const int* __restrict__ comp, const double* __restrict__ x,
                                                 const double* __restrict__ b, double* __restrict__ r,
                                                 double* __restrict__ p, double* __restrict__ q,
                                                 double* __restrict__ vr, double* __restrict__ vb) {
  const int c = blockIdx.x * ANT + threadIdx.x;
  if (c >= L.n) return;
  const int k = comp[c];
  double rv = 0.0, bv = 0.0;
  {
    const double xc = x[c];
    double acc = 0.0;
    for (int j = L.row_off[c]; j < L.row_off[c + 1]; ++j) acc += L.w[j] * (xc - x[L.col[j]]);
    bv = b[c];
    rv = bv - acc;
    r[c] = rv;
    p[c] = 0.0;
    q[c] = 0.0;
  }
  vr[c] = k >= 0 ? rv * rv : 0.0;
  vb[c] = k >= 0 ? bv * bv : 0.0;
}

// one block: a learned start no better than zero is dropped (flag per
// component; its |r|^2 becomes |b|^2); iteration counts start at -1
__global__ void __launch_bounds__(ANT) k_fs_scal0(const int* __restrict__ list, int nl, double* __restrict__ rrc,
                                                  const double* __restrict__ bbc, int* __restrict__ reset, int warm,
                                                  int* __restrict__ iters, int* __restrict__ stats,
                                                  double* __restrict__ sc, int* __restrict__ done,
                                                  int* __restrict__ itc, int* __restrict__ flag,
                                                  int* __restrict__ frozen, double* __restrict__ rzc,
                                                  double* __restrict__ pqc, int* __restrict__ open) {
  if (threadIdx.x == 0) *open = 0;
  for (int i = threadIdx.x; i < nl; i += blockDim.x) {
    const int c = list[i];
    frozen[c] = 0;
    rzc[c] = 0.0;
    pqc[c] = 0.0;
    const bool rs = warm && !(rrc[c] < bbc[c]);
    reset[c] = rs ? 1 : 0;
    if (rs) {
      rrc[c] = bbc[c];
      atomicAdd(&stats[1], 1);
    }
    iters[c] = -1;
  }
  if (threadIdx.x == 0) {
    sc[S_RHOP] = 1.0;
    *done = 0;
    *itc = 0;
    *flag = 1;
  }
}

__global__ void k_fs_reset(int n, const int* __restrict__ comp, const int* __restrict__ reset,
                           const double* __restrict__ b, double* __restrict__ x, double* __restrict__ r) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int k = comp[c];
  if (k >= 0 && reset[k]) {
    x[c] = 0.0;
    r[c] = b[c];
  }
}

// x += alpha_c p, r -= alpha_c q on the open components' rows; r^2 per node
// (summed per component by run_sums).  The per-component sums of the batch
// (r^2, b^2, r z, p q) go through run_sums rather than atomics: their
// order, and so the iteration, is then the same on every run.
__global__ void __launch_bounds__(ANT) k_fs_xr(int n, const int* __restrict__ comp, double* __restrict__ x,
                                               double* __restrict__ r, const double* __restrict__ p,
                                               const double* __restrict__ q, const double* __restrict__ alpha,
                                               const int* __restrict__ frozen, double* __restrict__ vr,
                                               const int* done) {
  if (is_done(done)) return;
  const int c = blockIdx.x * ANT + threadIdx.x;
  if (c >= n) return;
  const int key = comp[c];
  double v = 0.0;
  if (key >= 0 && !frozen[key]) {
    const double a = alpha[key];
    x[c] += a * p[c];
    const double rv = r[c] - a * q[c];
    r[c] = rv;
    v = rv * rv;
  }
  vr[c] = v;
}

// r z per node of an open component (summed per component by run_sums)
__global__ void __launch_bounds__(ANT) k_fs_rz(int n, const int* __restrict__ comp, const double* __restrict__ r,
                                               const double* __restrict__ z, const int* __restrict__ frozen,
                                               double* __restrict__ vz, const int* done) {
  if (is_done(done)) return;
  const int c = blockIdx.x * ANT + threadIdx.x;
  if (c >= n) return;
  const int key = comp[c];
  vz[c] = (key >= 0 && !frozen[key]) ? r[c] * z[c] : 0.0;
}

// Per listed component, after the cycle: the test on the residual of the
// last update (the start's before the first); a component that passes
// records the iteration and is frozen (its x and r stay as they are); one
// still open at maxit is counted in stats[0] and frozen; otherwise beta_c
// = rho_c / rho_c(previous) and the component counts as open.
__global__ void __launch_bounds__(ANT) k_fs_scal1(const int* __restrict__ list, int nl, double* __restrict__ rrc,
                                               double* __restrict__ rr, const double* __restrict__ bbc,
                                               double* __restrict__ rzc, double* __restrict__ rhop,
                                               double* __restrict__ beta, int* __restrict__ frozen,
                                               int* __restrict__ iters, int* __restrict__ stats,
                                               const int* __restrict__ itc, double rtol, int maxit,
                                               int* __restrict__ open, const int* done) {
  if (is_done(done)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl) return;
  const int c = list[i];
  if (frozen[c]) return;
  const int it = *itc;
  const double v = rrc[c];
  rr[c] = v;
  const double rho = rzc[c];
  if (!(v > rtol * rtol * bbc[c])) {
    if (iters[c] < 0) iters[c] = it;
    frozen[c] = 1;
    return;
  }
  if (it >= maxit || !(rho > 0.0)) {  // cap reached, or a breakdown
    iters[c] = it;
    atomicAdd(&stats[0], 1);
    frozen[c] = 1;
    return;
  }
  beta[c] = it == 0 ? 0.0 : rho / rhop[c];
  rhop[c] = rho;
  atomicAdd(open, 1);
}

// p = z + beta_c p, q = A z + beta_c q (= A p) and p q per node, on the
// open components' rows (level 0 has no heavy rows)
__global__ void __launch_bounds__(ANT) k_fs_pq(ALev L, const int* __restrict__ comp, const int* __restrict__ frozen,
                                               const double* __restrict__ beta, double* __restrict__ p,
                                               double* __restrict__ q, double* __restrict__ vpq, const int* done) {
  if (is_done(done)) return;
  const int c = blockIdx.x * ANT + threadIdx.x;
  if (c >= L.n) return;
  const int k = comp[c];
  const bool act = k >= 0 && !frozen[k];
  double v = 0.0;
  if (act) {
    const double* z = L.y;
    const double zc = z[c];
    double acc = 0.0;
    for (int j = L.row_off[c]; j < L.row_off[c + 1]; ++j) acc += L.w[j] * (zc - z[L.col[j]]);
    const double b = beta[k];
    const double pn = zc + b * p[c];
    const double qn = acc + b * q[c];
    p[c] = pn;
    q[c] = qn;
    v = pn * qn;
  }
  vpq[c] = v;
}

// alpha_c = rho_c / (p, q)_c per open component; block 0 then ends the
// solve when no component is open, else advances the iteration counter
__global__ void __launch_bounds__(ANT) k_fs_alpha(const int* __restrict__ list, int nl, const int* __restrict__ frozen,
                                                  const double* __restrict__ rhop, double* __restrict__ pqc,
                                                  double* __restrict__ alpha, int* __restrict__ open,
                                                  int* __restrict__ itc, int* __restrict__ done,
                                                  int* __restrict__ flag) {
  if (is_done(done)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nl) {
    const int c = list[i];
    if (!frozen[c]) {
      const double pq = pqc[c];
      alpha[c] = pq > 0.0 ? rhop[c] / pq : 0.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (*open == 0) {
      *done = 1;
      *flag = 0;
    } else {
      *itc = *itc + 1;
    }
    *open = 0;
  }
}

// ------------------------------------------------------------ host side
struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
};

template <class T>
T* grow(DBuf& b, size_t count, hipError_t& err) {
  const size_t bytes = ((std::max<size_t>(count, 1) * sizeof(T)) + 255) & ~size_t(255);
  if (b.cap < bytes) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      err = e;
      return nullptr;
    }
    b.cap = bytes;
  }
  return static_cast<T*>(b.p);
}

inline int nb256(long long n) { return (int)std::max<long long>((n + 255) / 256, 1); }

}  // namespace

namespace nil {

struct AmgLevel {
  int n = 0, np = 0, nheavy = 0, nmheavy = 0;
  int nmem = 0;  // levels >= 1: finer nodes that belong to a node of this level
  // levels >= 1: members of every node, Galerkin lists (fine pairs per pair)
  DBuf mem_off_b, mem_b, mheavy_b, gal_off_b, gal_src_b;
  // map of this level's nodes to the next level, and of its entries'
  // neighbours
  DBuf cid_b, ccol_b;
  // pairs and CSR (level 0: views of the quotient arrays)
  DBuf plo_b, phi_b, row_off_b, ent_b, col_b, heavy_b;
  // per step
  DBuf pw_b, w_b, diag_b;
  // cycle vectors
  DBuf bv_b, x_b, r_b, y_b;
  // pixel coordinates and component of every node (geometric aggregation)
  DBuf gy_b, gx_b, gc_b;
  const int *gy = nullptr, *gx = nullptr, *gc = nullptr;
  const int *row_off = nullptr, *col = nullptr, *ent = nullptr, *plo = nullptr, *phi = nullptr;
  const double *w = nullptr, *diag = nullptr, *pw = nullptr;
  const int *mem_off = nullptr, *mem = nullptr, *mheavy = nullptr, *gal_off = nullptr, *gal_src = nullptr;
  const int* heavy = nullptr;
  int* cid = nullptr;
  const int* ccol = nullptr;
  double *bv = nullptr, *x = nullptr, *r = nullptr, *y = nullptr;
};

constexpr int NSCR = 16;

struct Amg {
  std::vector<AmgLevel*> lv;
  int nlev = 0;        // levels in use (0 .. nlev-1); the last is the coarsest
  bool dense = false;  // coarsest solved exactly
  double corr = 1.0;   // coarse-correction factor
  DBuf s[NSCR];
  DBuf scan, ainv, pin, p, q, r, parts, sc, ctr, rrc, rst, fs_c, fs_frozen, fs_v, fs_rt, timg;
  // host readbacks of the build: a pinned landing area, and the counts
  // that only the solve needs (heavy rows and aggregates per level),
  // gathered in device slots and read once at the end of the build
  int* hpin = nullptr;
  DBuf cnts;
  std::vector<int*> pend;
  hipStream_t cap = nullptr;  // capture stream of the iteration graph
  ~Amg() {
    if (cap) (void)hipStreamDestroy(cap);
    if (hpin) (void)hipHostFree(hpin);
    for (AmgLevel* L : lv) {
      DBuf* b[] = {&L->mem_off_b, &L->mem_b, &L->mheavy_b, &L->gal_off_b, &L->gal_src_b, &L->cid_b, &L->ccol_b, &L->plo_b,
                   &L->phi_b, &L->row_off_b, &L->ent_b, &L->col_b, &L->heavy_b, &L->pw_b, &L->w_b, &L->diag_b,
                   &L->bv_b, &L->x_b, &L->r_b, &L->y_b, &L->gy_b, &L->gx_b, &L->gc_b};
      for (DBuf* d : b)
        if (d->p) (void)hipFree(d->p);
      delete L;
    }
    for (DBuf& d : s)
      if (d.p) (void)hipFree(d.p);
    DBuf* own[] = {&scan, &ainv, &pin, &p, &q, &r, &parts, &sc, &ctr, &rrc, &rst, &cnts, &fs_c, &fs_frozen, &fs_v, &fs_rt, &timg};
    for (DBuf* d : own)
      if (d->p) (void)hipFree(d->p);
  }
};

Amg* amg_new() { return new Amg(); }
void amg_free(Amg* a) { delete a; }
int amg_levels(const Amg* a) { return a ? a->nlev : 0; }
static int tail_start(const Amg* A, long long* img_bytes);

// Algorithmic HBM bytes of one batched-fill PCG iteration on this
// hierarchy (values FP64, indices int32; neighbour re-reads are cache hits
// and not counted).  Per level l with n rows and e entries, above the
// tail: down reads row_off, col, w, b, diag and writes r (28 n + 12 e);
// restrict reads mem_off, mem, r and writes b' (12 n + 12 n'); up reads
// row_off, col, ccol, w, b, diag, cid, y' and writes y (32 n + 16 e +
// 8 n').  The tail reads its packed image, the inverse of the coarsest
// and b, diag of its first level and writes y there (image + 8 n_c^2 +
// 24 n).  Without a tail the coarsest reads the inverse and two vectors
// (8 n^2 + 16 n).  Level 0 also, per node: comp read and one per-node term
// written by each of the three per-component kernels (12 n each), the
// three run sums reading key and term (36 n); on the rows of a system:
// r z reads r, z (16 n_sys), (p, q) reads row_off, z, p, q and the
// entries and writes p, q (44 n_sys + 12 e), the update reads x, r, p, q
// and writes x, r (48 n_sys): 72 n + 12 e + 108 n_sys.
double amg_fill_bytes(const Amg* A, long long n_sys) {
  if (!A || A->nlev <= 0) return 0.0;
  double by = 0.0;
  long long img = 0;
  const int t0 = tail_start(A, &img);
  for (int l = 0; l < A->nlev; ++l) {
    const AmgLevel* L = A->lv[l];
    const double n = L->n, e = 2.0 * L->np;
    if (l == t0) {
      const double nc = A->lv[A->nlev - 1]->n;
      by += (double)img + 8.0 * nc * nc + 24.0 * n;
      break;
    }
    if (l == A->nlev - 1) {
      by += A->dense ? 8.0 * n * n + 16.0 * n : 60.0 * n + 24.0 * e;
      break;
    }
    const double nc = A->lv[l + 1]->n;
    by += 28.0 * n + 12.0 * e + 12.0 * n + 12.0 * nc + 32.0 * n + 16.0 * e + 8.0 * nc;
  }
  const AmgLevel* L0 = A->lv[0];
  by += 72.0 * L0->n + 12.0 * 2.0 * L0->np + 108.0 * (double)n_sys;
  return by;
}

void amg_set_corr(Amg* a, double corr) {
  if (a) a->corr = corr;
}

#define AMG_TRY(x)                      \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

constexpr int NCNT = 2 * AMAXL + 2;  // deferred count slots

static hipError_t read_int(Amg* A, const int* dev, int* host, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(A->hpin + NCNT, dev, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) *host = A->hpin[NCNT];
  return e;
}

// a device slot whose value lands in *dest at the end of the build
static int* defer_count(Amg* A, int* dest) {
  A->pend.push_back(dest);
  return static_cast<int*>(A->cnts.p) + (A->pend.size() - 1);
}

static hipError_t flush_counts(Amg* A, hipStream_t st) {
  if (A->pend.empty()) return hipSuccess;
  const size_t n = A->pend.size();
  AMG_TRY(hipMemcpyAsync(A->hpin, A->cnts.p, n * sizeof(int), hipMemcpyDeviceToHost, st));
  AMG_TRY(hipStreamSynchronize(st));
  for (size_t k = 0; k < n; ++k) *A->pend[k] = A->hpin[k];
  A->pend.clear();
  return hipSuccess;
}

static int bits_for(int n) {
  int b = 0;
  while ((1ll << b) < (long long)n) ++b;
  return b;
}


// rows (or members) with more than AH entries of an offset array
static hipError_t heavy_list(Amg* A, int n, const int* off, DBuf& out, int* count, const int*& view,
                             hipStream_t st) {
  hipError_t err = hipSuccess;
  int* flag = grow<int>(A->s[14], n, err);
  int* pos = grow<int>(A->s[15], n + 1, err);
  int* list = grow<int>(out, n, err);
  int* scan = grow<int>(A->scan, scan_tmp_ints(n + 1), err);
  AMG_TRY(err);
  k_am_heavy_flag<<<nb256(n), 256, 0, st>>>(n, off, flag);
  AMG_TRY(scan_exclusive_i32(flag, pos, n, defer_count(A, count), scan, st));
  k_am_list<<<nb256(n), 256, 0, st>>>(n, flag, pos, list);
  view = list;
  return hipGetLastError();
}

// CSR (row_off, ent, col) of a level's pair list, and its heavy rows
static hipError_t build_csr(Amg* A, AmgLevel* L, hipStream_t st) {
  hipError_t err = hipSuccess;
  const int n = L->n, np = L->np, ne = 2 * np;
  int* row_off = grow<int>(L->row_off_b, n + 1, err);
  int* ent = grow<int>(L->ent_b, ne, err);
  int* col = grow<int>(L->col_b, ne, err);
  uint32_t* k0 = grow<uint32_t>(A->s[0], ne, err);
  uint32_t* v0 = grow<uint32_t>(A->s[1], ne, err);
  uint32_t* k1 = grow<uint32_t>(A->s[2], ne, err);
  uint32_t* v1 = grow<uint32_t>(A->s[3], ne, err);
  uint32_t* kt = grow<uint32_t>(A->s[4], ne, err);
  uint32_t* vt = grow<uint32_t>(A->s[5], ne, err);
  int* cnt = grow<int>(A->s[6], n + 1, err);
  int* scan = grow<int>(A->scan, std::max(radix_tmp_ints(std::max(ne, 1)), scan_tmp_ints(n + 1)), err);
  AMG_TRY(err);
  k_am_fill<<<nb256(n + 1), 256, 0, st>>>(cnt, n + 1, 0);
  if (ne > 0) {
    k_am_ekeys<<<nb256(ne), 256, 0, st>>>(np, L->plo, L->phi, k0, v0);
    AMG_TRY(radix_sort_pairs(k0, v0, k1, v1, kt, vt, ne, bits_for(n), scan, st));
    k_am_ecol<<<nb256(ne), 256, 0, st>>>(ne, v1, L->plo, L->phi, ent, col);
    k_am_count<<<nb256(ne), 256, 0, st>>>(ne, k1, cnt);
  }
  AMG_TRY(scan_exclusive_i32(cnt, row_off, n + 1, nullptr, scan, st));
  L->row_off = row_off;
  L->ent = ent;
  L->col = col;
  return heavy_list(A, n, row_off, L->heavy_b, &L->nheavy, L->heavy, st);
}

// per-step values of a coarse level from the finer level's pair weights
static void level_values(AmgLevel* L, const double* pwf, hipStream_t st) {
  hipError_t err = hipSuccess;
  double* pw = grow<double>(L->pw_b, L->np, err);
  double* w = grow<double>(L->w_b, 2 * (size_t)L->np, err);
  double* diag = grow<double>(L->diag_b, L->n, err);
  if (err != hipSuccess) return;
  if (L->np > 0) {
    k_am_gal<<<nb256(L->np), 256, 0, st>>>(L->np, L->gal_off, L->gal_src, pwf, pw);
    k_am_ew<<<nb256(2 * (long long)L->np), 256, 0, st>>>(2 * L->np, L->ent, pw, w);
  }
  k_am_diag<<<nb256(L->n), 256, 0, st>>>(L->n, L->row_off, w, diag);
  L->pw = pw;
  L->w = w;
  L->diag = diag;
}

// 2x2-block aggregation of a pixel-graph level: every active node (row
// sum > 0) is sorted on (component, aggregate cell) with its index as the
// value (stable sorts keep equal keys in index order), and joins the
// aggregate led by the first node of its run.  Inactive nodes: agg2 = -1.
// (a level-l coordinate is the level-0 one shifted right by l, so x >> 1 is
// at most (gw - 1) >> (l + 1): the key takes bx + by bits)
static hipError_t geo_aggregate(Amg* A, const AmgLevel* F, int l, int gw, int gh, int ncomp, int* agg2, int* lead,
                                hipStream_t st) {
  const int bx = bits_for(((gw - 1) >> (l + 1)) + 1), by = bits_for(((gh - 1) >> (l + 1)) + 1);
  hipError_t err = hipSuccess;
  const int n = F->n;
  int* kcell = grow<int>(A->s[14], n, err);
  uint32_t* kcomp = grow<uint32_t>(A->s[15], n, err);
  int* flag = grow<int>(A->s[13], n, err);
  int* fpos = grow<int>(A->s[11], n + 1, err);
  uint32_t* ko = grow<uint32_t>(A->s[0], n, err);
  uint32_t* vo = grow<uint32_t>(A->s[1], n, err);
  uint32_t* k1 = grow<uint32_t>(A->s[2], n, err);
  uint32_t* v1 = grow<uint32_t>(A->s[3], n, err);
  uint32_t* tk = grow<uint32_t>(A->s[4], n, err);
  uint32_t* tv = grow<uint32_t>(A->s[5], n, err);
  uint32_t* k2 = grow<uint32_t>(A->s[6], n, err);
  uint32_t* k3 = grow<uint32_t>(A->s[7], n, err);
  uint32_t* v3 = grow<uint32_t>(A->s[8], n, err);
  int* rflag = grow<int>(A->s[12], n, err);
  int* scan = grow<int>(A->scan, std::max(radix_tmp_ints(std::max(n, 1)), scan_tmp_ints(n + 1)), err);
  int* tot = grow<int>(A->ctr, 8, err);
  AMG_TRY(err);
  k_am_fill<<<nb256(n), 256, 0, st>>>(agg2, n, -1);
  k_am_fill<<<nb256(n), 256, 0, st>>>(lead, n, 0);
  k_gm_keys<<<nb256(n), 256, 0, st>>>(n, F->diag, F->gy, F->gx, F->gc, bx, kcell, kcomp, flag);
  AMG_TRY(scan_exclusive_i32(flag, fpos, n, tot, scan, st));
  int m = 0;
  AMG_TRY(read_int(A, tot, &m, st));
  if (m <= 0) return hipGetLastError();
  k_am_compact<<<nb256(n), 256, 0, st>>>(n, flag, fpos, kcell, ko, vo);
  AMG_TRY(radix_sort_pairs(ko, vo, k1, v1, tk, tv, m, std::max(bx + by, 1), scan, st));
  k_am_gather<<<nb256(m), 256, 0, st>>>(m, kcomp, v1, k2);
  AMG_TRY(radix_sort_pairs(k2, v1, k3, v3, tk, tv, m, std::max(bits_for(ncomp), 1), scan, st));
  k_am_runs<<<nb256(m), 256, 0, st>>>(m, v3, kcomp, reinterpret_cast<const uint32_t*>(kcell), rflag);
  int* rpos = reinterpret_cast<int*>(ko);
  int* rs = reinterpret_cast<int*>(vo);
  AMG_TRY(scan_exclusive_i32(rflag, rpos, m, nullptr, scan, st));
  k_gm_starts<<<nb256(m), 256, 0, st>>>(m, rflag, rpos, rs);
  k_gm_agg<<<nb256(m), 256, 0, st>>>(m, v3, rflag, rpos, rs, agg2, lead);
  return hipGetLastError();
}

// Build the hierarchy from the quotient graph of this step: K nodes, P
// pairs (pair_lo < pair_hi, weights pW), CSR row_off / qcol / qw, row sums
// diag.
hipError_t amg_build(Amg* A, int K, int P, const int* row_off, const int* qcol, const double* qw,
                     const double* diag, const int* pair_lo, const int* pair_hi, const double* pW, hipStream_t st,
                     const int* gy, const int* gx, const int* gc, int ncomp, int gw, int gh) {
  const bool geo = gy && gx && gc;
  hipError_t err = hipSuccess;
  if (A->lv.empty()) A->lv.push_back(new AmgLevel());
  AmgLevel* L0 = A->lv[0];
  L0->n = K;
  L0->np = P;
  L0->row_off = row_off;
  L0->col = qcol;
  L0->w = qw;
  L0->diag = diag;
  L0->plo = pair_lo;
  L0->phi = pair_hi;
  L0->pw = pW;
  L0->gy = geo ? gy : nullptr;
  L0->gx = geo ? gx : nullptr;
  L0->gc = geo ? gc : nullptr;
  // every scratch array at its largest size up front: nothing is freed and
  // reallocated while kernels that use it may still be queued
  {
    const size_t big = (size_t)std::max(2 * (size_t)P, (size_t)K) + 2;
    for (int i = 0; i < NSCR; ++i) grow<uint32_t>(A->s[i], big, err);
    grow<int>(A->scan, std::max(radix_tmp_ints((int)big), scan_tmp_ints((int)big)), err);
    grow<int>(A->ctr, 8, err);
    grow<int>(A->cnts, NCNT, err);
    AMG_TRY(err);
    if (!A->hpin) AMG_TRY(hipHostMalloc(reinterpret_cast<void**>(&A->hpin), (NCNT + 4) * sizeof(int)));
    A->pend.clear();
  }
  AMG_TRY(heavy_list(A, K, row_off, L0->heavy_b, &L0->nheavy, L0->heavy, st));
  int* tot = static_cast<int*>(A->ctr.p);
  int l = 0;
  A->dense = false;
  for (;;) {
    AmgLevel* F = A->lv[l];
    const int n = F->n;
    if (n <= AMAXC) {
      A->dense = true;
      break;
    }
    if (l + 1 >= AMAXL) break;
    // ---- aggregation of level l
    int* agg = grow<int>(A->s[7], n, err);
    int* best = grow<int>(A->s[8], n, err);
    int* agg2 = grow<int>(A->s[9], n, err);
    int* lead = grow<int>(A->s[10], n, err);
    int* pos = grow<int>(A->s[11], n + 1, err);
    uint8_t* act = grow<uint8_t>(A->s[12], n, err);
    int* cid = grow<int>(F->cid_b, n, err);
    int* flag = grow<int>(A->s[13], n, err);
    int* scan = grow<int>(A->scan, std::max(radix_tmp_ints(std::max(std::max(2 * F->np, n), 1)),
                                            scan_tmp_ints(std::max(F->np, n) + 1)), err);
    AMG_TRY(err);
    if (geo) {
      AMG_TRY(geo_aggregate(A, F, l, gw, gh, ncomp, agg2, lead, st));
    } else {
      k_am_active<<<nb256(n), 256, 0, st>>>(n, F->row_off, F->diag, agg, act);
      for (int round = 0; round < 3; ++round) {
        k_am_pick<<<nb256(n), 256, 0, st>>>(n, F->row_off, F->col, F->w, agg, act, best);
        k_am_match<<<nb256(n), 256, 0, st>>>(n, best, agg);
      }
      k_am_attach<<<nb256(n), 256, 0, st>>>(n, F->row_off, F->col, F->w, agg, act, agg2, lead);
    }
    AMG_TRY(scan_exclusive_i32(lead, pos, n, tot, scan, st));
    int nc = 0;
    AMG_TRY(read_int(A, tot, &nc, st));
    if (nc <= 0 || nc > (int)(0.9 * n)) break;  // no edges left, or coarsening stalled
    k_am_cid<<<nb256(n), 256, 0, st>>>(n, agg2, pos, cid, flag);
    F->cid = cid;
    {
      const int ne = 2 * F->np;
      int* ccol = grow<int>(F->ccol_b, ne, err);
      AMG_TRY(err);
      if (ne > 0) k_am_ccol<<<nb256(ne), 256, 0, st>>>(ne, F->col, cid, ccol);
      F->ccol = ccol;
    }
    if (l + 1 >= (int)A->lv.size()) A->lv.push_back(new AmgLevel());
    AmgLevel* C = A->lv[l + 1];
    C->n = nc;
    if (geo) {
      int* cy = grow<int>(C->gy_b, nc, err);
      int* cx = grow<int>(C->gx_b, nc, err);
      int* cc = grow<int>(C->gc_b, nc, err);
      AMG_TRY(err);
      k_gm_coarse<<<nb256(n), 256, 0, st>>>(n, agg2, pos, F->gy, F->gx, F->gc, cy, cx, cc);
      C->gy = cy;
      C->gx = cx;
      C->gc = cc;
    } else {
      C->gy = C->gx = C->gc = nullptr;
    }
    // ---- members of every coarse node: the fine nodes sorted on cid
    {
      int* fpos = grow<int>(A->s[11], n + 1, err);
      uint32_t* ko = grow<uint32_t>(A->s[0], n, err);
      uint32_t* vo = grow<uint32_t>(A->s[1], n, err);
      uint32_t* ks = grow<uint32_t>(A->s[2], n, err);
      uint32_t* vs = grow<uint32_t>(A->s[3], n, err);
      uint32_t* kt = grow<uint32_t>(A->s[4], n, err);
      uint32_t* vt = grow<uint32_t>(A->s[5], n, err);
      int* mem_off = grow<int>(C->mem_off_b, nc + 1, err);
      int* mem = grow<int>(C->mem_b, n, err);
      AMG_TRY(err);
      AMG_TRY(scan_exclusive_i32(flag, fpos, n, tot, scan, st));
      int m = 0;
      AMG_TRY(read_int(A, tot, &m, st));
      C->nmem = m;
      k_am_compact<<<nb256(n), 256, 0, st>>>(n, flag, fpos, cid, ko, vo);
      AMG_TRY(radix_sort_pairs(ko, vo, ks, vs, kt, vt, m, bits_for(nc), scan, st));
      k_am_u32<<<nb256(m), 256, 0, st>>>(vs, m, mem);
      k_am_offsets<<<nb256(m), 256, 0, st>>>(m, ks, nc, mem_off);
      C->mem_off = mem_off;
      C->mem = mem;
      // aggregates with more than AH members: a block each in the restriction
      int* hf = grow<int>(A->s[14], nc, err);
      int* hp = grow<int>(A->s[15], nc + 1, err);
      int* hl = grow<int>(C->mheavy_b, nc, err);
      AMG_TRY(err);
      k_am_heavy_flag<<<nb256(nc), 256, 0, st>>>(nc, mem_off, hf);
      AMG_TRY(scan_exclusive_i32(hf, hp, nc, defer_count(A, &C->nmheavy), scan, st));
      k_am_list<<<nb256(nc), 256, 0, st>>>(nc, hf, hp, hl);
      C->mheavy = hl;
    }
    // ---- coarse pairs: fine pairs between two aggregates, grouped by (lo, hi)
    {
      const int npf = F->np;
      int* pflag = grow<int>(A->s[13], std::max(npf, n), err);
      int* ppos = grow<int>(A->s[11], npf + 1, err);
      uint32_t* klo = grow<uint32_t>(A->s[0], npf, err);
      uint32_t* khi = grow<uint32_t>(A->s[1], npf, err);
      uint32_t* fp = grow<uint32_t>(A->s[2], npf, err);
      uint32_t* idx = grow<uint32_t>(A->s[3], npf, err);
      uint32_t* k1 = grow<uint32_t>(A->s[4], npf, err);
      uint32_t* o1 = grow<uint32_t>(A->s[5], npf, err);
      uint32_t* k2 = grow<uint32_t>(A->s[6], npf, err);
      uint32_t* k3 = grow<uint32_t>(A->s[7], npf, err);  // agg no longer needed
      uint32_t* ord = grow<uint32_t>(A->s[8], npf, err);
      uint32_t* tk = grow<uint32_t>(A->s[9], npf, err);
      uint32_t* tv = grow<uint32_t>(A->s[10], npf, err);
      int* rflag = grow<int>(A->s[12], npf, err);
      int* rpos = grow<int>(A->s[14], npf + 1, err);
      AMG_TRY(err);
      int mp = 0;
      if (npf > 0) {
        k_am_pflag<<<nb256(npf), 256, 0, st>>>(npf, F->plo, F->phi, cid, pflag);
        AMG_TRY(scan_exclusive_i32(pflag, ppos, npf, tot, scan, st));
        AMG_TRY(read_int(A, tot, &mp, st));
      }
      int npc = 0;
      if (mp > 0) {
        k_am_pcompact<<<nb256(npf), 256, 0, st>>>(npf, pflag, ppos, F->plo, F->phi, cid, klo, khi, fp, idx);
        const int bc = bits_for(nc);
        AMG_TRY(radix_sort_pairs(khi, idx, k1, o1, tk, tv, mp, bc, scan, st));   // by hi
        k_am_gather<<<nb256(mp), 256, 0, st>>>(mp, klo, o1, k2);                 // lo in that order
        AMG_TRY(radix_sort_pairs(k2, o1, k3, ord, tk, tv, mp, bc, scan, st));     // stably by lo
        k_am_runs<<<nb256(mp), 256, 0, st>>>(mp, ord, klo, khi, rflag);
        AMG_TRY(scan_exclusive_i32(rflag, rpos, mp, tot, scan, st));
        AMG_TRY(read_int(A, tot, &npc, st));
      }
      int* plo = grow<int>(C->plo_b, npc, err);
      int* phi = grow<int>(C->phi_b, npc, err);
      int* gal_off = grow<int>(C->gal_off_b, npc + 1, err);
      int* gal_src = grow<int>(C->gal_src_b, mp, err);
      AMG_TRY(err);
      if (mp > 0)
        k_am_pairs_out<<<nb256(mp), 256, 0, st>>>(mp, ord, klo, khi, rflag, rpos, fp, plo, phi, gal_off, gal_src,
                                                  npc);
      else
        k_am_fill<<<1, 1, 0, st>>>(gal_off, 1, 0);
      C->np = npc;
      C->plo = plo;
      C->phi = phi;
      C->gal_off = gal_off;
      C->gal_src = gal_src;
    }
    AMG_TRY(build_csr(A, C, st));
    // this step's weights on the new level (the next aggregation uses them)
    level_values(C, F->pw, st);
    AMG_TRY(hipGetLastError());
    ++l;
  }
  A->nlev = l + 1;
  AmgLevel* Lc = A->lv[l];
  Lc->cid = nullptr;
  Lc->ccol = nullptr;
  AMG_TRY(flush_counts(A, st));
  // cycle vectors
  for (int k = 0; k < A->nlev; ++k) {
    AmgLevel* L = A->lv[k];
    L->bv = grow<double>(L->bv_b, L->n, err);
    L->x = grow<double>(L->x_b, L->n, err);
    L->r = grow<double>(L->r_b, L->n, err);
    L->y = grow<double>(L->y_b, L->n, err);
  }
  AMG_TRY(err);
  return hipGetLastError();
}

// per IRLS step: the finest level's values (quotient CSR weights and row
// sums, pair weights) and the Galerkin sums of every coarser level; the
// coarsest pinned inverse
hipError_t amg_update(Amg* A, const double* qw, const double* diag, const double* pW, hipStream_t st) {
  if (A->nlev <= 0) return hipErrorInvalidValue;
  AmgLevel* L0 = A->lv[0];
  L0->w = qw;
  L0->diag = diag;
  L0->pw = pW;
  for (int k = 1; k < A->nlev; ++k) level_values(A->lv[k], A->lv[k - 1]->pw, st);
  AmgLevel* Lc = A->lv[A->nlev - 1];
  if (A->dense && Lc->n > 0) {
    hipError_t err = hipSuccess;
    double* ainv = grow<double>(A->ainv, (size_t)Lc->n * Lc->n, err);
    uint8_t* pin = grow<uint8_t>(A->pin, Lc->n, err);
    AMG_TRY(err);
    k_am_invert<<<1, 1024, 0, st>>>(Lc->n, Lc->row_off, Lc->col, Lc->w, Lc->diag, ainv, pin);
  }
  return hipGetLastError();
}

static ALev view(const AmgLevel* L, double* b) {
  ALev v;
  v.n = L->n;
  v.nblk = nb256(L->n);
  v.nheavy = L->nheavy;
  v.row_off = L->row_off;
  v.col = L->col;
  v.w = L->w;
  v.diag = L->diag;
  v.heavy = L->heavy;
  v.cid = L->cid;
  v.ccol = L->ccol;
  v.b = b;
  v.x = L->x;
  v.r = L->r;
  v.y = L->y;
  return v;
}

// The LDS layout of the tail from level t0 on (the packed per-step arrays
// first, then the cycle vectors); its size in bytes, or -1 when a level is
// too large for 16-bit indices.  *img_bytes: the packed part.
static long long tail_layout(const Amg* A, int t0, TailPlan* T, long long* img_bytes) {
  long long off = TTAB;
  auto take = [&](long long bytes) {
    const long long o = off;
    off += (bytes + 15) & ~15ll;
    return (int)o;
  };
  const int nl = A->nlev - t0;
  TLev v[TMAXL] = {};
  for (int k = 0; k < nl; ++k) {
    const AmgLevel* L = A->lv[t0 + k];
    const long long n = L->n, nnz = 2ll * L->np;
    if (n >= 65535 || nnz >= 65535 || L->nmem >= 65535) return -1;
    TLev& t = v[k];
    t.n = L->n;
    t.nnz = (int)nnz;
    t.nh = L->nheavy;
    t.nmem = k > 0 ? L->nmem : 0;
    if (k + 1 < nl) {
      t.o_ro = take(2 * (n + 1));
      t.o_col = take(2 * nnz);
      t.o_w = take(8 * nnz);
      t.o_dg = take(8 * n);
      t.o_hv = take(2ll * L->nheavy);
    }
    if (k > 0) {
      t.o_mo = take(2 * (n + 1));
      t.o_mem = take(2ll * L->nmem);
    }
    t.row_off = L->row_off;
    t.col = L->col;
    t.mem_off = L->mem_off;
    t.mem = L->mem;
    t.heavy = L->heavy;
    t.w = L->w;
    t.diag = L->diag;
  }
  const int o_pin = take(A->lv[A->nlev - 1]->n);
  *img_bytes = off;
  for (int k = 0; k < nl; ++k) {
    const long long n = v[k].n;
    v[k].o_b = take(8 * n);
    if (k + 1 < nl) {
      v[k].o_x = take(8 * n);
      v[k].o_y = take(8 * n);
    }
  }
  if (T) {
    for (int k = 0; k < nl; ++k) T->lv[k] = v[k];
    T->o_pin = o_pin;
  }
  return off;
}

// The tail for this hierarchy: the first tail level is the largest that
// still fits in TAIL_LDS (and is not the finest).  Packs the image (img:
// at least TAIL_LDS bytes) on st.  Returns t0, or -1 for no tail (no
// exact coarsest, or not even one smoothed level fits).
static int tail_start(const Amg* A, long long* img_bytes) {
  if (!A->dense || A->nlev < 3) return -1;
  int t0 = -1;
  long long ib = 0;
  for (int t = A->nlev - 2; t >= 1 && A->nlev - t <= TMAXL; --t) {
    const long long by = tail_layout(A, t, nullptr, &ib);
    if (by < 0 || by > TAIL_LDS) break;
    t0 = t;
    *img_bytes = ib;
  }
  return t0;
}

static int plan_tail(const Amg* A, const std::vector<ALev>& V, unsigned char* img, TailPlan& T, hipStream_t st) {
  long long ib = 0;
  const int t0 = img ? tail_start(A, &ib) : -1;
  if (t0 < 0) return -1;
  tail_layout(A, t0, &T, &ib);
  T.nl = A->nlev - t0;
  T.img_bytes = (int)ib;
  T.corr = A->corr;
  T.bin = V[t0].b;
  T.yout = V[t0].y;
  T.ainv = static_cast<const double*>(A->ainv.p);
  T.pin = static_cast<const uint8_t*>(A->pin.p);
  T.img = img;
  TOff tab[TMAXL] = {};
  int most = 0;
  for (int k = 0; k < T.nl; ++k) {
    tab[k] = T.lv[k];
    most = std::max(most, std::max(T.lv[k].n + 1, std::max(T.lv[k].nnz, T.lv[k].nmem)));
  }
  // a pageable source: the copy is staged when it is enqueued
  if (hipMemcpyAsync(img, tab, sizeof(tab), hipMemcpyHostToDevice, st) != hipSuccess) return -1;
  k_tail_pack<<<dim3(std::min(nb256(most), 64), T.nl), 256, 0, st>>>(T);
  return hipGetLastError() == hipSuccess ? t0 : -1;
}

// one V-cycle on V[0].b -> V[0].y; the finest level writes the block
// partials of (b, y) to parts.  With t0 >= 1 the levels from t0 on run in
// the tail kernel (plan T).
template <int FILL>
static void launch_cycle(const Amg* A, const std::vector<ALev>& V, double* parts, int pstride, const int* done,
                         hipStream_t q_, int t0, const TailPlan& T) {
  if (t0 >= 1) {
    for (int l = 0; l < t0; ++l) {
      const ALev& L = V[l];
      k_cy_down<FILL><<<L.nblk + L.nheavy, ANT, 0, q_>>>(L, done);
      const AmgLevel* C = A->lv[l + 1];
      k_cy_restrict<FILL><<<nb256(C->n) + C->nmheavy, ANT, 0, q_>>>(C->n, nb256(C->n), C->mem_off, C->mem,
                                                                    C->mheavy, L.r, V[l + 1].b, done);
    }
    TailHead h;
    h.nl = T.nl;
    h.o_pin = T.o_pin;
    h.img_bytes = T.img_bytes;
    h.n0 = T.lv[0].n;
    h.o_b0 = T.lv[0].o_b;
    h.o_x0 = T.lv[0].o_x;
    h.corr = T.corr;
    h.bin = T.bin;
    h.diag0 = T.lv[0].diag;
    h.ainv = T.ainv;
    h.yout = T.yout;
    h.img = T.img;
    k_cy_tail<FILL><<<1, TNT, 0, q_>>>(h, done);
    for (int l = t0 - 1; l >= 0; --l) {
      const ALev& L = V[l];
      k_cy_up<FILL><<<L.nblk + L.nheavy, ANT, 0, q_>>>(L, V[l + 1].y, l == 0 ? parts : nullptr, pstride, A->corr,
                                                       done);
    }
    return;
  }
  for (int l = 0; l + 1 < A->nlev; ++l) {
    const ALev& L = V[l];
    k_cy_down<FILL><<<L.nblk + L.nheavy, ANT, 0, q_>>>(L, done);
    const AmgLevel* C = A->lv[l + 1];
    k_cy_restrict<FILL><<<nb256(C->n) + C->nmheavy, ANT, 0, q_>>>(C->n, nb256(C->n), C->mem_off, C->mem, C->mheavy, L.r,
                                                            V[l + 1].b, done);
  }
  const ALev& Lc = V[A->nlev - 1];
  if (A->dense) {
    k_cy_coarsest<FILL><<<1, CO_NT, 0, q_>>>(Lc.n, static_cast<const double*>(A->ainv.p),
                                       static_cast<const uint8_t*>(A->pin.p), Lc.b, Lc.y, done);
    if (A->nlev == 1 && parts) k_cy_dot<FILL><<<Lc.nblk + Lc.nheavy, ANT, 0, q_>>>(Lc, parts, pstride, done);
  } else {  // no exact coarsest: smoothing only
    k_cy_up<FILL><<<Lc.nblk + Lc.nheavy, ANT, 0, q_>>>(Lc, nullptr, A->nlev == 1 ? parts : nullptr, pstride, A->corr,
                                                 done);
  }
  for (int l = A->nlev - 2; l >= 0; --l) {
    const ALev& L = V[l];
    k_cy_up<FILL><<<L.nblk + L.nheavy, ANT, 0, q_>>>(L, V[l + 1].y, l == 0 ? parts : nullptr, pstride, A->corr, done);
  }
}

// PCG on the finest level, preconditioned by one V-cycle.  rhs / babs as
// in the Jacobi solver; the solution goes to s.  Iterations -> *iters_out
// (device).  The host polls the "still iterating" flag every `batch`
// iterations.
hipError_t amg_solve(Amg* A, const double* rhs, const double* scale, const double* floorv, double floor_rel,
                     double* s, double rtol, int maxit, int* iters_out, int* host_flag, bool graph, hipStream_t st,
                     int* hint) {
  hipError_t err = hipSuccess;
  AmgLevel* L0 = A->lv[0];
  const int n = L0->n;
  const int nblk = nb256(n);
  double* p = grow<double>(A->p, n, err);
  double* q = grow<double>(A->q, n, err);
  double* r = grow<double>(A->r, n, err);
  const int pstride = nblk + L0->nheavy;
  double* parts = grow<double>(A->parts, 3 * (size_t)pstride, err);
  double* sc = grow<double>(A->sc, S_N, err);
  int* ctr = grow<int>(A->ctr, 8, err);  // [0] done, [1] iteration, [2] flag
  unsigned char* timg = grow<unsigned char>(A->timg, TAIL_LDS, err);
  AMG_TRY(err);
  int* done = ctr;
  int* itc = ctr + 1;
  int* flag = ctr + 2;
  const double ratio = (floorv && rtol > 0) ? floor_rel / rtol : 0.0;
  k_cg_init<<<nblk, ANT, 0, st>>>(n, rhs, scale, floorv, ratio, s, r, p, q, sc, parts, pstride);
  k_cg_scal<0><<<1, SC_NT, 0, st>>>(0, parts, nblk, pstride, nblk, sc, done, itc, rtol, maxit, iters_out, flag);
  std::vector<ALev> V(A->nlev);
  for (int k = 0; k < A->nlev; ++k) V[k] = view(A->lv[k], k == 0 ? r : A->lv[k]->bv);
  TailPlan tp{};
  const int t0 = plan_tail(A, V, timg, tp, st);
  // one PCG iteration: V-cycle on r -> z (= y of level 0), then the CG
  // update; every kernel returns at once after convergence
  auto iteration = [&](hipStream_t q_) {
    launch_cycle<0>(A, V, parts, pstride, done, q_, t0, tp);
    // rho = (r, z) -> beta; convergence on ||r||
    k_cg_scal<0><<<1, SC_NT, 0, q_>>>(1, parts, pstride, pstride, nblk, sc, done, itc, rtol, maxit, iters_out, flag);
    k_cg_pq<0><<<V[0].nblk + V[0].nheavy, ANT, 0, q_>>>(V[0], p, q, sc, parts, pstride, done);
    k_cg_scal<0><<<1, SC_NT, 0, q_>>>(2, parts, pstride, pstride, nblk, sc, done, itc, rtol, maxit, iters_out, flag);
    k_cg_xr<<<nblk, ANT, 0, q_>>>(n, s, r, p, q, sc, parts + pstride, done);
  };
  // optionally the iteration's ~3 launches per level are captured once per
  // solve into a graph (on a private stream: the caller's may be the legacy
  // default stream, which cannot be captured) and replayed on the caller's
  // stream.  On gfx950 this did not shorten an iteration (the time between
  // dependent kernels is spent on the device, not in the launch calls).
  hipGraphExec_t ge = nullptr;
  if (graph) {
    if (!A->cap) AMG_TRY(hipStreamCreateWithFlags(&A->cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    AMG_TRY(hipStreamBeginCapture(A->cap, hipStreamCaptureModeThreadLocal));
    iteration(A->cap);
    hipError_t ce = hipStreamEndCapture(A->cap, &g);
    if (ce == hipSuccess) ce = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    AMG_TRY(ce);
  }
  struct ExecGuard {
    hipGraphExec_t e;
    ~ExecGuard() {
      if (e) (void)hipGraphExecDestroy(e);
    }
  } guard{ge};
  // stream launches: the scalar steps fused into the (p, q) and (x, r)
  // kernels (the captured graph keeps the separate one-block kernels).
  // Every block re-reads every block's partials, so this pays only while
  // the partials are few: beyond FUSE_MAX the one-block kernels stay.
  constexpr int FUSE_MAX = 1024;
  const bool fuse = pstride <= FUSE_MAX;
  auto fused = [&](int it) {
    launch_cycle<0>(A, V, parts, pstride, done, st, t0, tp);
    k_cg_pq_f<<<V[0].nblk + V[0].nheavy, ANT, 0, st>>>(V[0], p, q, sc, parts, pstride, pstride, nblk, it, rtol,
                                                      maxit, done, flag, iters_out);
    k_cg_xr_f<<<nblk, ANT, 0, st>>>(n, s, r, p, q, sc, parts, pstride, pstride, it, done);
  };
  // The host launches a batch of iterations, then reads the flag; the
  // iterations launched after convergence return at once but still cost a
  // dispatch each.  With a hint (the iteration count of the previous
  // solve of this kind) the first batch stops just short of it and the
  // next ones are short; without one, or past the hint, batches of 8.
  int* hp = A->hpin + NCNT + 1;  // [0] flag, [1] iterations
  const int expect = hint ? *hint : 0;
  int batch = expect > 0 ? std::max(expect - 1, 1) : 8;
  for (int it = 0; it <= maxit + 1;) {
    for (int k = 0; k < batch; ++k) {
      if (ge) AMG_TRY(hipGraphLaunch(ge, st));
      else if (fuse) fused(it + k);
      else iteration(st);
    }
    it += batch;
    AMG_TRY(hipGetLastError());
    AMG_TRY(hipMemcpyAsync(hp, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    AMG_TRY(hipMemcpyAsync(hp + 1, iters_out, sizeof(int), hipMemcpyDeviceToHost, st));
    AMG_TRY(hipStreamSynchronize(st));
    if (hp[0] == 0) break;
    batch = (expect > 0 && it <= expect + 4) ? 2 : 8;
  }
  *host_flag = hp[0];
  if (hint) *hint = hp[1];
  return hipSuccess;
}

hipError_t amg_fill_solve(Amg* A, const int* comp, const uint32_t* rkey, const int* list, int nl, int K,
                          const double* b, double* x,
                          double rtol, int maxit, int warm, double* rr, double* bb, int* iters, int* stats,
                          int* host_flag, int* its, hipStream_t st) {
  *its = 0;
  if (A->nlev <= 0 || nl <= 0) return hipSuccess;
  hipError_t err = hipSuccess;
  AmgLevel* L0 = A->lv[0];
  if (L0->nheavy != 0) return hipErrorInvalidValue;  // pixel rows have at most four entries
  const int n = L0->n;
  const int nblk = nb256(n);
  double* p = grow<double>(A->p, n, err);
  double* q = grow<double>(A->q, n, err);
  double* r = grow<double>(A->r, n, err);
  double* sc = grow<double>(A->sc, S_N, err);
  int* ctr = grow<int>(A->ctr, 8, err);  // [0] done, [1] iteration, [2] flag, [3] open components
  const size_t K1 = (size_t)std::max(K, 1);
  double* rrc = grow<double>(A->rrc, K1, err);
  int* rst = grow<int>(A->rst, K1, err);
  // per-component PCG state: rho, (p, q), previous rho, beta, alpha
  double* cs = grow<double>(A->fs_c, 5 * K1, err);
  int* frozen = grow<int>(A->fs_frozen, K1, err);
  // per-node terms of the per-component sums, and the run-sum scratch
  double* vn = grow<double>(A->fs_v, 2 * (size_t)n, err);
  void* rtmp = grow<uint8_t>(A->fs_rt, run_sums_tmp_bytes(n), err);
  unsigned char* timg = grow<unsigned char>(A->timg, TAIL_LDS, err);
  AMG_TRY(err);
  double *rzc = cs, *pqc = cs + K1, *rhop = cs + 2 * K1, *beta = cs + 3 * K1, *alpha = cs + 4 * K1;
  int* done = ctr;
  int* itc = ctr + 1;
  int* flag = ctr + 2;
  int* open = ctr + 3;
  std::vector<ALev> V(A->nlev);
  for (int k = 0; k < A->nlev; ++k) V[k] = view(A->lv[k], k == 0 ? r : A->lv[k]->bv);
  TailPlan tp{};
  const int t0 = plan_tail(A, V, timg, tp, st);
  // components without a node on this level keep zero sums
  AMG_TRY(hipMemsetAsync(rrc, 0, sizeof(double) * K1, st));
  AMG_TRY(hipMemsetAsync(bb, 0, sizeof(double) * K1, st));
  k_fs_init<<<nblk, ANT, 0, st>>>(V[0], comp, x, b, r, p, q, vn, vn + n);
  AMG_TRY(run_sums(rkey, vn, n, rrc, rtmp, st, 1));
  AMG_TRY(run_sums(rkey, vn + n, n, bb, rtmp, st, 1));
  k_fs_scal0<<<1, ANT, 0, st>>>(list, nl, rrc, bb, rst, warm, iters, stats, sc, done, itc, flag, frozen, rzc, pqc,
                                open);
  if (warm) k_fs_reset<<<nblk, ANT, 0, st>>>(n, comp, rst, b, x, r);
  AMG_TRY(hipGetLastError());
  // every component runs its own PCG (its own rho, beta, alpha) through the
  // shared V-cycle, which never couples two components; a component stops
  // (is frozen) at its first pass of the test
  const int nbl = nb256(nl);
  const int batch = 8;
  for (int it = 0; it <= maxit + 1; it += batch) {
    for (int k = 0; k < batch; ++k) {
      launch_cycle<1>(A, V, nullptr, 0, done, st, t0, tp);
      k_fs_rz<<<nblk, ANT, 0, st>>>(n, comp, r, V[0].y, frozen, vn, done);
      AMG_TRY(run_sums(rkey, vn, n, rzc, rtmp, st, 1));
      k_fs_scal1<<<nbl, ANT, 0, st>>>(list, nl, rrc, rr, bb, rzc, rhop, beta, frozen, iters, stats, itc, rtol, maxit,
                                      open, done);
      k_fs_pq<<<nblk, ANT, 0, st>>>(V[0], comp, frozen, beta, p, q, vn, done);
      AMG_TRY(run_sums(rkey, vn, n, pqc, rtmp, st, 1));
      k_fs_alpha<<<nbl, ANT, 0, st>>>(list, nl, frozen, rhop, pqc, alpha, open, itc, done, flag);
      k_fs_xr<<<nblk, ANT, 0, st>>>(n, comp, x, r, p, q, alpha, frozen, vn, done);
      AMG_TRY(run_sums(rkey, vn, n, rrc, rtmp, st, 1));
    }
    AMG_TRY(hipGetLastError());
    AMG_TRY(hipMemcpyAsync(host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    AMG_TRY(hipStreamSynchronize(st));
    if (*host_flag == 0) break;
  }
  AMG_TRY(hipMemcpyAsync(host_flag, itc, sizeof(int), hipMemcpyDeviceToHost, st));
  AMG_TRY(hipStreamSynchronize(st));
  *its = *host_flag;
  return hipSuccess;
}

}  // namespace nil
