// Device-wide exclusive scan (int32) and stable LSD radix sort of
// (uint32 key, uint32 value) pairs.  Both are deterministic: the scan is an
// integer scan and the sort ranks equal digits by their input order using
// wavefront ballots, so the output never depends on scheduling.
#include <algorithm>

#include "ni_common.h"

namespace {

constexpr int SC_NT = 256, SC_PPT = 8, SC_TILE = SC_NT * SC_PPT;

__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// exclusive scan of one value per thread across the block; returns the
// exclusive prefix, *total gets the block total (all threads)
__device__ __forceinline__ int block_excl_scan(int x, int* lds_w, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int inc = wave_incl_scan(x);
  if (lane == 63) lds_w[wid] = inc;
  __syncthreads();
  int woff = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    int s = lds_w[w];
    if (w < wid) woff += s;
    tot += s;
  }
  *total = tot;
  __syncthreads();
  return woff + inc - x;
}

__global__ void __launch_bounds__(SC_NT) k_scan_reduce(const int* __restrict__ in, int n,
                                                       int* __restrict__ bsum) {
  __shared__ int lds[SC_NT / 64];
  long long base = (long long)blockIdx.x * SC_TILE;
  int s = 0;
#pragma unroll
  for (int k = 0; k < SC_PPT; ++k) {
    long long i = base + k * SC_NT + threadIdx.x;
    if (i < n) s += in[i];
  }
  int tot;
  block_excl_scan(s, lds, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of a tile, offset by boff[block] (or 0)
__global__ void __launch_bounds__(SC_NT) k_scan_tile(const int* __restrict__ in, int* __restrict__ out,
                                                     int n, const int* __restrict__ boff,
                                                     int* __restrict__ total_dev) {
  __shared__ int tile[SC_TILE];
  __shared__ int lds[SC_NT / 64];
  long long base = (long long)blockIdx.x * SC_TILE;
#pragma unroll
  for (int k = 0; k < SC_PPT; ++k) {
    long long i = base + k * SC_NT + threadIdx.x;
    tile[k * SC_NT + threadIdx.x] = i < n ? in[i] : 0;
  }
  __syncthreads();
  int loc[SC_PPT];
  int s = 0;
#pragma unroll
  for (int k = 0; k < SC_PPT; ++k) {
    loc[k] = s;
    s += tile[threadIdx.x * SC_PPT + k];
  }
  int tot;
  int ex = block_excl_scan(s, lds, &tot);
  int off = (boff ? boff[blockIdx.x] : 0) + ex;
#pragma unroll
  for (int k = 0; k < SC_PPT; ++k) tile[threadIdx.x * SC_PPT + k] = off + loc[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SC_PPT; ++k) {
    long long i = base + k * SC_NT + threadIdx.x;
    if (i < n) out[i] = tile[k * SC_NT + threadIdx.x];
  }
  if (total_dev && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    *total_dev = (boff ? boff[blockIdx.x] : 0) + tot;
}

// ------------------------------------------------------------------ radix
constexpr int RS_NT = 256, RS_PPT = 8, RS_TILE = RS_NT * RS_PPT, RS_NW = RS_NT / 64;

__global__ void __launch_bounds__(RS_NT) k_rs_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                   int* __restrict__ hist, int nblk) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  long long base = (long long)blockIdx.x * RS_TILE;
#pragma unroll
  for (int r = 0; r < RS_PPT; ++r) {
    long long i = base + r * RS_NT + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(RS_NT) k_rs_scatter(const uint32_t* __restrict__ kin,
                                                      const uint32_t* __restrict__ vin, int n, int shift,
                                                      const int* __restrict__ off, int nblk,
                                                      uint32_t* __restrict__ kout,
                                                      uint32_t* __restrict__ vout) {
  __shared__ int wcnt[RS_NW][256];
  __shared__ int running[256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int w = 0; w < RS_NW; ++w) wcnt[w][threadIdx.x] = 0;
  running[threadIdx.x] = off[threadIdx.x * nblk + blockIdx.x];
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  long long base = (long long)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_PPT; ++r) {
    long long i = base + r * RS_NT + threadIdx.x;
    bool valid = i < n;
    uint32_t key = valid ? kin[i] : 0u;
    uint32_t val = valid ? vin[i] : 0u;
    int d = (key >> shift) & 255;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1;
      unsigned long long bal = __ballot(valid && bit);
      peers &= bit ? bal : ~bal;
    }
    int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[wid][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = running[d] + rank;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < RS_NW; ++w) {
      add += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    running[threadIdx.x] += add;
    __syncthreads();
  }
}

// ------------------------------------------------------------ small sort
// Up to SB_N pairs in one workgroup: a bitonic sort of (masked key,
// position) composites, which are distinct, so the result is the stable
// order of the radix passes below, in one launch instead of four per pass.
// Element i = t + k * SB_NT is held in register k of thread t.  A
// compare-exchange partner at distance j is in the same thread for
// j >= SB_NT, in the same wavefront for j < 64 (exchanged by shuffles) and
// in another wavefront otherwise (exchanged through LDS, between barriers).
constexpr int SB_N = 4096, SB_NT = 1024, SB_E = SB_N / SB_NT;

// the element kept at position i of the pair (i, i ^ j) inside a bitonic
// block of size kk: the smaller on the ascending side
__device__ __forceinline__ unsigned long long sb_keep(unsigned long long mine, unsigned long long other, int i, int j,
                                                      int kk) {
  const bool asc = (i & kk) == 0;
  const bool low = (i & j) == 0;
  const unsigned long long lo = mine < other ? mine : other, hi = mine < other ? other : mine;
  return (asc == low) ? lo : hi;
}

__global__ void __launch_bounds__(SB_NT) k_sort_small(const uint32_t* __restrict__ kin,
                                                      const uint32_t* __restrict__ vin, int n, uint32_t mask,
                                                      uint32_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  __shared__ unsigned long long sh[SB_N];
  const int t = threadIdx.x;
  int m = 1;
  while (m < n) m <<= 1;
  const int E = m > SB_NT ? m / SB_NT : 1;  // registers that hold elements below m
  unsigned long long a[SB_E];
#pragma unroll
  for (int k = 0; k < SB_E; ++k) {
    const int i = t + k * SB_NT;
    a[k] = i < n ? (((unsigned long long)(kin[i] & mask) << 32) | (unsigned long long)i) : ~0ull;
  }
  for (int kk = 2; kk <= m; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j >= SB_NT) {
        // partners in the same thread: registers k and k ^ (j / SB_NT)
        auto cx = [&](unsigned long long& x, unsigned long long& y, int k, int k2) {
          const unsigned long long u = x, v = y;
          x = sb_keep(u, v, t + k * SB_NT, j, kk);
          y = sb_keep(v, u, t + k2 * SB_NT, j, kk);
        };
        static_assert(SB_E == 4, "register pairs below are written for four elements per thread");
        if (j == SB_NT) {
          cx(a[0], a[1], 0, 1);
          if (E > 2) cx(a[2], a[3], 2, 3);
        } else {
          cx(a[0], a[2], 0, 2);
          cx(a[1], a[3], 1, 3);
        }
      } else if (j < 64) {
#pragma unroll
        for (int k = 0; k < SB_E; ++k) {
          if (k < E) {
            const unsigned long long o = __shfl_xor(a[k], j, 64);
            a[k] = sb_keep(a[k], o, t + k * SB_NT, j, kk);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < SB_E; ++k)
          if (k < E) sh[t + k * SB_NT] = a[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SB_E; ++k) {
          const int i = t + k * SB_NT;
          if (k < E) a[k] = sb_keep(a[k], sh[i ^ j], i, j, kk);
        }
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int k = 0; k < SB_E; ++k) {
    const int i = t + k * SB_NT;
    if (i < n) {
      const uint32_t pos = (uint32_t)(a[k] & 0xffffffffull);
      kout[i] = kin[pos];
      vout[i] = vin[pos];
    }
  }
}

// ------------------------------------------------------------- run sums
// out[k] = the sum of v over every run of equal keys (runs are maximal
// stretches of equal consecutive keys), in an order fixed by the element
// positions alone: 8 consecutive elements per thread in order, then a
// fixed pairwise tree over the block's threads, then over the blocks.  A
// record describes a stretch of elements: one key (single), or its first
// and last runs (multi), whose inner runs are complete and already written.
constexpr int RU_NT = 256, RU_PPT = 8, RU_TILE = RU_NT * RU_PPT, RU_TOP = 1024;

struct RunRec {
  uint32_t hk, tk;  // keys of the first and last runs (single: equal)
  double hs, ts;    // their partial sums
  int kind;         // 0 empty, 1 single, 2 multi
};

// A's stretch directly followed by B's; runs completed by the merge are
// written to out
__device__ __forceinline__ RunRec rr_merge(const RunRec& A, const RunRec& B, double* out) {
  if (A.kind == 0) return B;
  if (B.kind == 0) return A;
  RunRec R;
  if (A.kind == 1 && B.kind == 1) {
    if (A.hk == B.hk) {
      R = A;
      R.hs = A.hs + B.hs;
      R.ts = R.hs;
      return R;
    }
    R.kind = 2;
    R.hk = A.hk;
    R.hs = A.hs;
    R.tk = B.hk;
    R.ts = B.hs;
    return R;
  }
  if (A.kind == 1) {  // B multi
    R = B;
    if (A.hk == B.hk) {
      R.hs = A.hs + B.hs;
    } else {
      out[B.hk] = B.hs;
      R.hk = A.hk;
      R.hs = A.hs;
    }
    return R;
  }
  if (B.kind == 1) {  // A multi
    R = A;
    if (A.tk == B.hk) {
      R.ts = A.ts + B.hs;
    } else {
      out[A.tk] = A.ts;
      R.tk = B.hk;
      R.ts = B.hs;
    }
    return R;
  }
  if (A.tk == B.hk) {
    out[A.tk] = A.ts + B.hs;
  } else {
    out[A.tk] = A.ts;
    out[B.hk] = B.hs;
  }
  R.kind = 2;
  R.hk = A.hk;
  R.hs = A.hs;
  R.tk = B.tk;
  R.ts = B.ts;
  return R;
}

// fixed pairwise tree over the block's records in LDS; the result in rec[0]
__device__ __forceinline__ void rr_tree(RunRec* rec, double* out) {
  for (int s = 1; s < (int)blockDim.x; s <<= 1) {
    __syncthreads();
    const int t = threadIdx.x;
    if ((t & (2 * s - 1)) == 0 && t + s < (int)blockDim.x) rec[t] = rr_merge(rec[t], rec[t + s], out);
  }
  __syncthreads();
}

// TAG only names the caller in kernel traces (1: the batched fill)
template <int TAG>
__global__ void __launch_bounds__(RU_NT) k_runsum_tile(const uint32_t* __restrict__ key, const double* __restrict__ v,
                                                       int n, double* __restrict__ out, RunRec* __restrict__ brec) {
  __shared__ RunRec rec[RU_NT];
  const long long base = (long long)blockIdx.x * RU_TILE + (long long)threadIdx.x * RU_PPT;
  RunRec R;
  R.kind = 0;
  for (int j = 0; j < RU_PPT; ++j) {
    const long long i = base + j;
    if (i >= n) break;
    RunRec e;
    e.kind = 1;
    e.hk = e.tk = key[i];
    e.hs = e.ts = v[i];
    R = rr_merge(R, e, out);
  }
  rec[threadIdx.x] = R;
  rr_tree(rec, out);
  if (threadIdx.x == 0) brec[blockIdx.x] = rec[0];
}

// one block of RU_TOP threads over the tile records; the first and last
// runs of the whole array are complete at the end
template <int TAG>
__global__ void __launch_bounds__(RU_TOP) k_runsum_top(const RunRec* __restrict__ brec, int nb,
                                                       double* __restrict__ out) {
  __shared__ RunRec rec[RU_TOP];
  const int per = (nb + RU_TOP - 1) / RU_TOP;
  RunRec R;
  R.kind = 0;
  for (int j = 0; j < per; ++j) {
    const int b = threadIdx.x * per + j;
    if (b >= nb) break;
    R = rr_merge(R, brec[b], out);
  }
  rec[threadIdx.x] = R;
  rr_tree(rec, out);
  if (threadIdx.x == 0) {
    const RunRec& F = rec[0];
    if (F.kind >= 1) out[F.hk] = F.hs;
    if (F.kind == 2) out[F.tk] = F.ts;
  }
}

}  // namespace

namespace nil {

size_t scan_tmp_ints(int n) {
  size_t s = 0;
  while (n > SC_TILE) {
    int nb = ni::ceil_div(n, SC_TILE);
    s += 2 * (size_t)nb;
    n = nb;
  }
  return s + 4;
}

hipError_t scan_exclusive_i32(const int* in, int* out, int n, int* total_dev, int* tmp,
                              hipStream_t st) {
  if (n <= 0) {
    if (total_dev) return hipMemsetAsync(total_dev, 0, sizeof(int), st);
    return hipSuccess;
  }
  if (n <= SC_TILE) {
    k_scan_tile<<<1, SC_NT, 0, st>>>(in, out, n, nullptr, total_dev);
    return hipGetLastError();
  }
  int nb = ni::ceil_div(n, SC_TILE);
  int* bsum = tmp;
  int* boff = tmp + nb;
  k_scan_reduce<<<nb, SC_NT, 0, st>>>(in, n, bsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_i32(bsum, boff, nb, nullptr, tmp + 2 * nb, st);
  if (e != hipSuccess) return e;
  k_scan_tile<<<nb, SC_NT, 0, st>>>(in, out, n, boff, total_dev);
  return hipGetLastError();
}

size_t radix_tmp_ints(int n) {
  int nblk = ni::ceil_div(n > 0 ? n : 1, RS_TILE);
  return 2 * (size_t)256 * nblk + scan_tmp_ints(256 * nblk);
}

hipError_t radix_sort_pairs(const uint32_t* k_in, const uint32_t* v_in, uint32_t* k_out,
                            uint32_t* v_out, uint32_t* k_tmp, uint32_t* v_tmp, int n, int bits,
                            int* scan_tmp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int passes = bits <= 0 ? 1 : (bits + 7) / 8;
  const void* outs[2] = {k_out, v_out};
  const void* ins[2] = {k_in, v_in};
  bool apart = true;
  for (const void* o : outs)
    for (const void* i : ins) apart = apart && o != i;
  if (n <= SB_N && apart) {
    // the same order as the passes below: stable on the low 8 * passes bits
    const uint32_t mask = passes >= 4 ? 0xffffffffu : ((1u << (8 * passes)) - 1u);
    k_sort_small<<<1, SB_NT, 0, st>>>(k_in, v_in, n, mask, k_out, v_out);
    return hipGetLastError();
  }
  int nblk = ni::ceil_div(n, RS_TILE);
  int* hist = scan_tmp;
  int* off = scan_tmp + 256 * nblk;
  int* stmp = scan_tmp + 2 * 256 * nblk;
  const uint32_t* ks = k_in;
  const uint32_t* vs = v_in;
  for (int p = 0; p < passes; ++p) {
    // the last pass writes the output buffers
    bool to_out = ((passes - 1 - p) % 2) == 0;
    uint32_t* kd = to_out ? k_out : k_tmp;
    uint32_t* vd = to_out ? v_out : v_tmp;
    k_rs_hist<<<nblk, RS_NT, 0, st>>>(ks, n, 8 * p, hist, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive_i32(hist, off, 256 * nblk, nullptr, stmp, st);
    if (e != hipSuccess) return e;
    k_rs_scatter<<<nblk, RS_NT, 0, st>>>(ks, vs, n, 8 * p, off, nblk, kd, vd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ks = kd;
    vs = vd;
  }
  return hipSuccess;
}

size_t run_sums_tmp_bytes(int n) { return sizeof(RunRec) * (size_t)std::max(ni::ceil_div(n, RU_TILE), 1); }

hipError_t run_sums(const uint32_t* key, const double* v, int n, double* out, void* tmp, hipStream_t st, int tag) {
  if (n <= 0) return hipSuccess;
  const int nb = ni::ceil_div(n, RU_TILE);
  RunRec* brec = static_cast<RunRec*>(tmp);
  if (tag == 1) {
    k_runsum_tile<1><<<nb, RU_NT, 0, st>>>(key, v, n, out, brec);
    k_runsum_top<1><<<1, RU_TOP, 0, st>>>(brec, nb, out);
  } else {
    k_runsum_tile<0><<<nb, RU_NT, 0, st>>>(key, v, n, out, brec);
    k_runsum_top<0><<<1, RU_TOP, 0, st>>>(brec, nb, out);
  }
  return hipGetLastError();
}

}  // namespace nil
