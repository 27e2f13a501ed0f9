// Internal helpers shared by the HIP kernels of libni (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define NI_WAVE 64

// per-pixel edge bits written by the setup kernel
enum : uint8_t {
  EB_VR = 1,    // edge to the right neighbour usable
  EB_VD = 2,    // edge to the lower neighbour usable
  EB_SR = 4,    // ... and normals similar (theta < theta_c)
  EB_SD = 8,
  EB_VALID = 128
};

// diagonal edge bits of 8-connectivity, a second byte per pixel
enum : uint8_t {
  EB2_VDR = 1,  // edge to the lower-right neighbour usable
  EB2_VDL = 2,  // edge to the lower-left neighbour usable
  EB2_SDR = 4,  // ... and normals similar
  EB2_SDL = 8
};

namespace ni {

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
  // fixed butterfly order: every lane ends with the same, deterministic sum
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, NI_WAVE);
  return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, NI_WAVE);
  return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, NI_WAVE);
  return v;
}

// Block-wide sum of NV doubles; every thread receives the totals.  `scratch`
// must hold NV * (blockDim/64) doubles and must not be reused by the caller
// until a later __syncthreads(); the sum order is fixed (deterministic).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) scratch[k * nw + wid] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += scratch[k * nw + w];
    v[k] = s;
  }
}

__host__ __device__ inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Edge directions, each edge owned by its upper end (in a row: the left
// one): 0 right, 1 down, 2 down-right, 3 down-left (8-connectivity only).
// An edge's code is 4 a + dir, a its owner pixel.
__device__ __forceinline__ int dir_step(int d, int W) { return d == 0 ? 1 : d == 1 ? W : d == 2 ? W + 1 : W - 1; }

// usable edge of direction d at owner p; eb2 is null under 4-connectivity
__device__ __forceinline__ bool dir_usable(const uint8_t* eb, const uint8_t* eb2, int p, int d) {
  if (d < 2) return (eb[p] & (d == 0 ? EB_VR : EB_VD)) != 0;
  return eb2 && (eb2[p] & (d == 2 ? EB2_VDR : EB2_VDL)) != 0;
}

// the pixel a - step(d) lies on the grid (the owner of the edge of
// direction d that ends at a)
__device__ __forceinline__ bool has_back(int a, int d, int W) {
  const int u = a % W;
  if (d == 0) return u > 0;
  if (a < W) return false;
  return d == 1 || (d == 2 ? u > 0 : u < W - 1);
}

}  // namespace ni

// ------------------------------------------------------------- host launchers
// Each .hip file exposes plain host functions that enqueue its kernels on a
// stream; they return the HIP error of the launch.
namespace nil {

hipError_t scan_exclusive_i32(const int* in, int* out, int n, int* total_dev,
                              int* tmp, hipStream_t st);
size_t scan_tmp_ints(int n);

// stable LSD radix sort of (key, val) by the low `bits` bits of key.  The
// result lands in (k_out, v_out); (k_tmp, v_tmp) are scratch of length n.
hipError_t radix_sort_pairs(const uint32_t* k_in, const uint32_t* v_in, uint32_t* k_out,
                            uint32_t* v_out, uint32_t* k_tmp, uint32_t* v_tmp, int n,
                            int bits, int* scan_tmp, hipStream_t st);
size_t radix_tmp_ints(int n);

// out[k] = sum of v[i] over every run of equal consecutive keys k = key[i]
// (each key one run), summed in an order fixed by the positions alone
// (reproducible run to run).  tmp: run_sums_tmp_bytes(n) of device memory.
// tag 1 marks the batched fill's calls in kernel traces.
hipError_t run_sums(const uint32_t* key, const double* v, int n, double* out, void* tmp, hipStream_t st,
                    int tag = 0);
size_t run_sums_tmp_bytes(int n);

// arguments of the batched CG of the large fill components (ni_fill.hip)
struct LargeArgs {
  const int *comp_off, *cbase, *nchunk, *chunk_comp, *chunk_start, *chunk_end;
  double *part, *gam, *tol2, *rr, *bb;
  int *iters, *active, *stats;
  const float4* cst;  // per pixel (w_right, w_down, w_up, packed offsets)
  const float *rhs, *dinv;
  float *x, *p, *r0, *r1, *w0, *w1, *s0, *s1;
  int nchunks, K;
  double rtol;
  int maxit;
  int split;  // 0: two launches per CG iteration; 1: three (p materialised)
};

// aggregation multigrid for the quotient systems (ni_amg.hip)
struct Amg;
Amg* amg_new();
void amg_free(Amg*);
int amg_levels(const Amg*);
// gy / gx / gc (optional): pixel coordinates and component of every node;
// when given, aggregates are 2x2 blocks of one component (pixel graphs),
// otherwise pairwise handshakes (general graphs).  gc < ncomp, gx < gw,
// gy < gh.
hipError_t amg_build(Amg*, int K, int P, const int* row_off, const int* qcol, const double* qw, const double* diag,
                     const int* pair_lo, const int* pair_hi, const double* pW, hipStream_t st,
                     const int* gy = nullptr, const int* gx = nullptr, const int* gc = nullptr, int ncomp = 0,
                     int gw = 32768, int gh = 32768);
// algorithmic HBM bytes of one batched-fill PCG iteration (n_sys: rows that
// belong to a system)
double amg_fill_bytes(const Amg*, long long n_sys);
// coarse-correction factor of the cycle (1 unless set)
void amg_set_corr(Amg*, double corr);
// Batched PCG of independent component systems on level 0 (block
// diagonal), each component with its own scalars: comp[node] (-1: no
// system), rkey[node] the component of every node (equal keys contiguous),
// list[nl] the components; x holds the start (warm != 0: a start no better
// than zero is dropped per component) and receives the solution.  Per
// component: rr = |r|^2 at the end, bb = |b|^2, iters = iterations to
// ||r_c|| <= rtol ||b_c||; stats[0] counts components that hit maxit,
// stats[1] dropped starts.  *its = iterations run.
hipError_t amg_fill_solve(Amg*, const int* comp, const uint32_t* rkey, const int* list, int nl, int K,
                          const double* b, double* x,
                          double rtol, int maxit, int warm, double* rr, double* bb, int* iters, int* stats,
                          int* host_flag, int* its, hipStream_t st);
hipError_t amg_update(Amg*, const double* qw, const double* diag, const double* pW, hipStream_t st);
// PCG preconditioned by one V-cycle: s from zero until ||r|| <= max(rtol
// ||scale||, floor_rel ||floorv||) (floorv may be null).  hint (host, may
// be null): the expected iteration count in, the count run out.
hipError_t amg_solve(Amg*, const double* rhs, const double* scale, const double* floorv, double floor_rel, double* s,
                     double rtol, int maxit, int* iters_out, int* host_flag, bool graph, hipStream_t st,
                     int* hint = nullptr);

// arguments of one relative-scale iteration (ni_quot.hip)
struct IrlsArgs {
  const uint32_t* eidx;
  int E, P, K, W;
  const int* label;   // component of every pixel (indexes S)
  const int* glabel;  // quotient node of every pixel (the component, or its merged node)
  const int* grp;     // node of every component (null: the identity)
  int K0;             // components (K = quotient nodes)
  int fresh = 0;      // 1: the node structure changed since the last step
  const uint8_t* ebits;
  const uint8_t* eb2 = nullptr;   // diagonal edge bits (8-connectivity), else null
  const double *eom, *eta, *etb;  // FP64 omega and gamma factors per inter edge
  const float* zfill;
  const int *pair_start, *pair_lo, *pair_hi, *row_off;
  const uint32_t* ent;
  double *S, *ew, *erho, *pW, *pB, *diag, *rhs, *babs;
  double *s, *psum, *pcnt;  // piece sums and sizes
  int* parent;
  // the nodes sorted by piece (keys, nodes, sort scratch, gathered values,
  // run-sum scratch)
  uint32_t *pkey, *pnode, *pnode_in, *pk_tmp, *pv_tmp;
  int* pscan;
  double* pval;
  void* prun;
  unsigned long long* wmax;
  double* energy_out;  // [t]
  int* qiters_out;     // [t] iterations of the first solve round
  int* qiters2_out;    // [t] iterations of the refinement round
  double* epart;
  double g2fx, g2fy, g2fd, k, L, U, cut_rel, q_rtol;
  double q_rtol2 = 1e-5;  // relative target of the refinement round  // g2f*: f^2 per right, down, diagonal row
  int align, outlier_mode, q_maxit, nnz;
  int out_from;  // first iteration with outlier weights (the baseline: 1)
  int* qcol;
  double *qw, *t0, *t1;  // t0: flow-form residual, t1: correction [K]
  int* host_flag;
  const int* heavy;
  int nheavy, nbig;
  Amg* amg;   // multigrid of the quotient solve
  int* hints = nullptr;  // host [2]: iterations of the last first / refinement round (poll batching)
  int graphs; // replay the multigrid iteration from a HIP graph
};
// scratch of the output stage (ni_final.hip): g holds max(N, 2K) doubles,
// k0..v2 K keys / values each, scan radix_tmp_ints(K) ints, rtmp
// run_sums_tmp_bytes(max(N, K)) bytes
struct FinalScratch {
  double* g;
  uint32_t *k0, *v0, *k1, *v1, *k2, *v2;
  int* scan;
  void* rtmp;
};

hipError_t merge_nodes(const IrlsArgs& a, int* grp, int* glabel_out, int P, unsigned long long* gkey, unsigned* gcode,
                       int* pa, int* pb, double* pkeep, int* parent, int* flag, int* rank, int* cnt, int* scan_tmp,
                       hipStream_t st);
hipError_t identity_groups(int* grp, int K0, hipStream_t st);

}  // namespace nil
