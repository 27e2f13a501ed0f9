// Output stage: log-depth z = zfill + S_pi, shifted to zero pixel mean over
// every connected region of the full pixel graph G_0 (the gauge the method
// leaves free: depth is recovered up to one scale per region, Sec. 3.1);
// depth = exp(z) in perspective and z in orthographic mode.
#include <algorithm>

#include "ni_common.h"

namespace {

// the filled log-depth in component-major order (summed per component by
// run_sums, in a fixed order)
__global__ void k_comp_vals(const uint32_t* __restrict__ cpix, int N, const float* __restrict__ zfill,
                            double* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) g[i] = (double)zfill[cpix[i]];
}

// the components sorted by region: region id and component index, for the
// stable sort
__global__ void k_region_keys(const int* __restrict__ comp_rid, int K, uint32_t* __restrict__ key,
                              uint32_t* __restrict__ idx) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K) {
    key[c] = (uint32_t)comp_rid[c];
    idx[c] = (uint32_t)c;
  }
}

// per component in region order: csum + n S (the region's sum of z) and n
__global__ void k_region_vals(const uint32_t* __restrict__ order, const int* __restrict__ comp_off,
                              const double* __restrict__ csum, const double* __restrict__ S, int K,
                              double* __restrict__ gz, double* __restrict__ gn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const int c = (int)order[i];
  const double n = (double)(comp_off[c + 1] - comp_off[c]);
  gz[i] = csum[c] + n * S[c];
  gn[i] = n;
}

__global__ void k_comp_region(const int* __restrict__ comp_off, const uint32_t* __restrict__ cpix,
                              const int* __restrict__ parent, const int* __restrict__ cid, int K,
                              int* __restrict__ comp_rid) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < K) comp_rid[c] = cid[parent[cpix[comp_off[c]]]];
}

__global__ void k_region_zero(double* rsum, double* rcnt, int R) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R) {
    rsum[i] = 0.0;
    rcnt[i] = 0.0;
  }
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

// Every sum goes through run_sums (per component over the component-major
// order; per region over the components sorted by region), so the outputs
// are the same on every run.
hipError_t final_outputs(const int* label, const float* zfill, const double* S, const int* comp_off,
                         const uint32_t* cpix, const uint32_t* ckey, const int* parent, const int* cid, int K, int N,
                         int R, int P, int persp, double* csum, int* comp_rid, double* rsum, double* rcnt,
                         float* depth, double* log_scale, const FinalScratch& w, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (R > 0) k_region_zero<<<ni::ceil_div(R, 256), 256, 0, st>>>(rsum, rcnt, R);
  if (K > 0 && N > 0) {
    k_comp_vals<<<ni::ceil_div(N, 256), 256, 0, st>>>(cpix, N, zfill, w.g);
    e = run_sums(ckey, w.g, N, csum, w.rtmp, st);
    if (e != hipSuccess) return e;
    k_comp_region<<<ni::ceil_div(K, 256), 256, 0, st>>>(comp_off, cpix, parent, cid, K, comp_rid);
    k_region_keys<<<ni::ceil_div(K, 256), 256, 0, st>>>(comp_rid, K, w.k0, w.v0);
    int bits = 1;
    while ((1ll << bits) < (long long)std::max(R, 1)) ++bits;
    e = radix_sort_pairs(w.k0, w.v0, w.k1, w.v1, w.k2, w.v2, K, bits, w.scan, st);
    if (e != hipSuccess) return e;
    k_region_vals<<<ni::ceil_div(K, 256), 256, 0, st>>>(w.v1, comp_off, csum, S, K, w.g, w.g + K);
    e = run_sums(w.k1, w.g, K, rsum, w.rtmp, st);
    if (e == hipSuccess) e = run_sums(w.k1, w.g + K, K, rcnt, w.rtmp, st);
    if (e != hipSuccess) return e;
  }
  k_final_out<<<ni::ceil_div(P, 256), 256, 0, st>>>(label, zfill, S, parent, cid, rsum, rcnt, P, persp, depth);
  if (K > 0 && log_scale)
    k_final_scale<<<ni::ceil_div(K, 256), 256, 0, st>>>(S, comp_rid, rsum, rcnt, K, log_scale);
  return hipGetLastError();
}

}  // namespace nil
