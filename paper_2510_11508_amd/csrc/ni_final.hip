// Output stage: log-depth z = zfill + S_pi, shifted to zero pixel mean over
// every connected region of the full pixel graph G_0 (the gauge the method
// leaves free: depth is recovered up to one scale per region, Sec. 3.1);
// depth = exp(z) in perspective and z in orthographic mode.
#include "ni_common.h"

namespace {

// FP64 sum of each component's filled log-depth over the component-major
// pixel order: a block whose pixels all belong to one component (the
// common case inside large components) adds one partial; others add per
// wavefront
__global__ void __launch_bounds__(1024) k_comp_sums(const int* __restrict__ label, const uint32_t* __restrict__ cpix,
                                                    int N, const float* __restrict__ zfill, double* __restrict__ csum,
                                                    int* __restrict__ ccnt) {
  __shared__ double red[2 * (1024 / 64)];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool v = i < N;
  const uint32_t p = v ? cpix[i] : 0u;
  ni::acc_by_key_block<int>(v, v ? label[p] : 0, v ? (double)zfill[p] : 0.0, 1, csum, ccnt, red);
}

__global__ void k_comp_region(const int* __restrict__ comp_off, const uint32_t* __restrict__ cpix,
                              const int* __restrict__ parent, const int* __restrict__ cid, int K,
                              int* __restrict__ comp_rid) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K) comp_rid[c] = cid[parent[cpix[comp_off[c]]]];
}

__global__ void k_zero_sums(double* csum, int* cnt, int K) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) {
    csum[i] = 0.0;
    cnt[i] = 0;
  }
}

__global__ void k_region_zero(double* rsum, double* rcnt, int R) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R) {
    rsum[i] = 0.0;
    rcnt[i] = 0.0;
  }
}

__global__ void k_region_acc(const int* __restrict__ comp_off, const double* __restrict__ csum,
                             const double* __restrict__ S, const int* __restrict__ comp_rid, int K,
                             double* __restrict__ rsum, double* __restrict__ rcnt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool v = c < K;
  const double n = v ? (double)(comp_off[c + 1] - comp_off[c]) : 0.0;
  ni::acc_by_key<double>(v, v ? comp_rid[c] : 0, v ? csum[c] + n * S[c] : 0.0, n, rsum, rcnt);
}

__global__ void k_final_out(const int* __restrict__ label, const float* __restrict__ zfill,
                            const double* __restrict__ S, const int* __restrict__ parent,
                            const int* __restrict__ cid, const double* __restrict__ rsum,
                            const double* __restrict__ rcnt, int P, int persp, float* __restrict__ depth) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int c = label[p];
  float out = __builtin_nanf("");
  if (c >= 0) {
    int rid = cid[parent[p]];
    double z = (double)zfill[p] + S[c] - rsum[rid] / rcnt[rid];
    out = persp ? (float)exp(z) : (float)z;
  }
  depth[p] = out;
}

__global__ void k_final_scale(const double* __restrict__ S, const int* __restrict__ comp_rid,
                              const double* __restrict__ rsum, const double* __restrict__ rcnt, int K,
                              double* __restrict__ log_scale) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K) log_scale[c] = S[c] - rsum[comp_rid[c]] / rcnt[comp_rid[c]];
}

}  // namespace

namespace nil {

hipError_t final_outputs(const int* label, const float* zfill, const double* S, const int* comp_off,
                         const uint32_t* cpix, const int* parent, const int* cid, int K, int N, int R, int P, int persp,
                         double* csum, int* comp_rid, double* rsum, double* rcnt, float* depth, double* log_scale,
                         hipStream_t st) {
  if (K > 0) {
    // csum and its count scratch (comp_rid, overwritten below) start at zero
    k_zero_sums<<<ni::ceil_div(K, 256), 256, 0, st>>>(csum, comp_rid, K);
    k_comp_sums<<<ni::ceil_div(N, 1024), 1024, 0, st>>>(label, cpix, N, zfill, csum, comp_rid);
    k_comp_region<<<ni::ceil_div(K, 256), 256, 0, st>>>(comp_off, cpix, parent, cid, K, comp_rid);
  }
  if (R > 0) k_region_zero<<<ni::ceil_div(R, 256), 256, 0, st>>>(rsum, rcnt, R);
  if (K > 0) k_region_acc<<<ni::ceil_div(K, 256), 256, 0, st>>>(comp_off, csum, S, comp_rid, K, rsum, rcnt);
  k_final_out<<<ni::ceil_div(P, 256), 256, 0, st>>>(label, zfill, S, parent, cid, rsum, rcnt, P, persp, depth);
  if (K > 0 && log_scale)
    k_final_scale<<<ni::ceil_div(K, 256), 256, 0, st>>>(S, comp_rid, rsum, rcnt, K, log_scale);
  return hipGetLastError();
}

}  // namespace nil
