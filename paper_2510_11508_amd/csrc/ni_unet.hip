// Learned warm start for the component fill: a small U-Net that maps
// (normal, mask, ray direction) to a log-depth estimate, trained on the
// fills the plain method produces, so that CG can start closer to the
// solution.  Everything runs in the kernels below:
//   - 3x3 convolutions as implicit GEMMs on BF16 MFMA (v_mfma_f32_16x16x32_bf16,
//     FP32 accumulation), NHWC activations with channel counts padded to
//     multiples of 8; one kernel serves the forward pass and the
//     data-gradient pass (flipped / transposed weights), a second MFMA
//     kernel computes weight gradients;
//   - 2x2 max-pool, nearest 2x upsampling into concatenation buffers,
//     ReLU, a 1x1 FP32 head, the per-component centred MSE loss and Adam.
// Architecture (channels): enc 16-16 | 32-32 | 64-64 | 128-128, dec
// (128+64)-64-64 | (64+32)-32-32 | (32+16)-16-16, head 16->1.
#include <math.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/ni.h"
#include "ni_common.h"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __bf16 bf16;

namespace {

constexpr int NCONV = 14;
constexpr int CIN_PAD0 = 8;  // input features: n(3), mask, tau_x, tau_y, 0, 0

struct ConvSpec {
  int cin_real, cin, cout;  // cin = padded input channels (multiple of 8)
};
constexpr ConvSpec SPECS[NCONV] = {
    {6, 8, 16},      {16, 16, 16},   // e0a e0b
    {16, 16, 32},    {32, 32, 32},   // e1a e1b
    {32, 32, 64},    {64, 64, 64},   // e2a e2b
    {64, 64, 128},   {128, 128, 128},  // e3a e3b
    {192, 192, 64},  {64, 64, 64},   // d2a d2b
    {96, 96, 32},    {32, 32, 32},   // d1a d1b
    {48, 48, 16},    {16, 16, 16},   // d0a d0b
};
constexpr int HEAD_C = 16;

__host__ __device__ inline int kpad_of(int cin) { return ((9 * cin + 31) / 32) * 32; }

// ---------------------------------------------------------------- kernels
__global__ void k_features(const float* __restrict__ nrm, const uint8_t* __restrict__ mask, int H, int W, int Hp,
                           int Wp, int persp, double fx, double fy, double cx, double cy, bf16* __restrict__ x) {
  // padded grid Hp x Wp; pixels outside the map get all-zero features
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Hp * Wp) return;
  int u = p % Wp, v = p / Wp;
  float f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (u < W && v < H) {
    long long q = (long long)v * W + u;
    if (mask[q]) {
      f[0] = nrm[3 * q];
      f[1] = nrm[3 * q + 1];
      f[2] = nrm[3 * q + 2];
      f[3] = 1.f;
    }
    if (persp) {
      f[4] = (float)(((double)u - cx) / fx);
      f[5] = (float)(((double)v - cy) / fy);
    }
  }
  bf16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = (bf16)f[k];
  *(bf16x8*)(x + (size_t)p * 8) = o;
}

// features from an FP32 [B][H][W][6] tensor (test hook)
__global__ void k_features_raw(const float* __restrict__ f6, long long P, bf16* __restrict__ x) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  bf16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = (bf16)(k < 6 ? f6[p * 6 + k] : 0.f);
  *(bf16x8*)(x + (size_t)p * 8) = o;
}

// Implicit-GEMM 3x3 convolution, zero padding 1:
//   out[p][co] = act( bias[co] + sum_{tap, ci} in[p + off(tap)][ci] * Wt[co][tap*cin + ci] )
// M = pixels (16 per wavefront), N = cout in tiles of 16 (at most 8 tiles
// per workgroup; blockIdx.y selects the 128-channel slice), K = 9*cin
// padded to a multiple of 32.  Lane l supplies A[m = l%16][k = 8(l/16)..+7]
// as one 16-byte load of 8 consecutive channels of one tap, and B[k][n] as
// one 16-byte load of the co-major weight row.
__global__ void __launch_bounds__(256) k_conv(const bf16* __restrict__ in, int in_stride, int in_off, int cin,
                                              const bf16* __restrict__ wt, int kpad,
                                              const float* __restrict__ bias, bf16* __restrict__ out,
                                              int out_stride, int out_off, int cout, int relu, int B, int H,
                                              int W) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long P = (long long)B * H * W;
  const long long p0 = ((long long)blockIdx.x * 4 + wave) * 16;
  if (p0 >= P) return;
  const int m = lane & 15, kq = lane >> 4;
  const long long p = p0 + m;
  const bool pv = p < P;
  int b = 0, y = 0, x = 0;
  if (pv) {
    x = (int)(p % W);
    long long t = p / W;
    y = (int)(t % H);
    b = (int)(t / H);
  }
  const int n0 = blockIdx.y * 128;
  const int nt = min(cout - n0, 128) >> 4;
  f32x4 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int K = 9 * cin;
  for (int k0 = 0; k0 < kpad; k0 += 32) {
    const int kk = k0 + 8 * kq;
    bf16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (bf16)0.f;
    if (pv && kk < K) {
      const int tap = kk / cin, ci = kk - tap * cin;
      const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        a = *(const bf16x8*)(in + (((long long)b * H + yy) * W + xx) * in_stride + in_off + ci);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t < nt) {
        const bf16x8 bw = *(const bf16x8*)(wt + (size_t)(n0 + t * 16 + m) * kpad + kk);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (t < nt) {
      const int co = n0 + t * 16 + m;
      const float bs = bias ? bias[co] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long q = p0 + 4 * kq + i;
        if (q < P) {
          float v = acc[t][i] + bs;
          if (relu) v = fmaxf(v, 0.f);
          out[q * out_stride + out_off + co] = (bf16)v;
        }
      }
    }
  }
}

// Weight gradient: dWt[co][k] += sum_p g[p][co] * im2col(in)[p][k], as the
// MFMA product C[co][k] = sum_p A[co][p] B[p][k] over a slab of pixels;
// one wavefront per 16x16 (co, k) tile, FP32 atomics across slabs.
constexpr int WG_SLAB = 2048;
__global__ void __launch_bounds__(256) k_wgrad(const bf16* __restrict__ in, int in_stride, int in_off, int cin,
                                               const bf16* __restrict__ g, int cout, float* __restrict__ dwt,
                                               int kpad, int B, int H, int W) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ktile = blockIdx.x * 4 + wave;
  if (ktile * 16 >= kpad) return;
  const int co0 = blockIdx.y * 16;
  const long long P = (long long)B * H * W;
  const long long s0 = (long long)blockIdx.z * WG_SLAB;
  const int m = lane & 15, kq = lane >> 4;
  const int K = 9 * cin;
  const int kcol = ktile * 16 + m;  // this lane's k for the B operand
  int tap = 0, ci = 0, dy = 0, dx = 0;
  const bool kvalid = kcol < K;
  if (kvalid) {
    tap = kcol / cin;
    ci = kcol - tap * cin;
    dy = tap / 3 - 1;
    dx = tap % 3 - 1;
  }
  f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (long long pb = s0; pb < s0 + WG_SLAB && pb < P; pb += 32) {
    bf16x8 a, bb;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const long long p = pb + 8 * kq + j;
      float av = 0.f, bv = 0.f;
      if (p < P) {
        av = (float)g[p * cout + co0 + m];
        if (kvalid) {
          const int x = (int)(p % W);
          const long long t = p / W;
          const int y = (int)(t % H), b = (int)(t / H);
          const int yy = y + dy, xx = x + dx;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            bv = (float)in[(((long long)b * H + yy) * W + xx) * in_stride + in_off + ci];
        }
      }
      a[j] = (bf16)av;
      bb[j] = (bf16)bv;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int co = co0 + 4 * kq + i;
    const int k = ktile * 16 + m;
    atomicAdd(&dwt[(size_t)co * kpad + k], acc[i]);
  }
}

// db[co] += sum_p g[p][co]
__global__ void __launch_bounds__(256) k_bias_grad(const bf16* __restrict__ g, long long P, int cout,
                                                   float* __restrict__ db) {
  // thread = channel (cout <= 256) of a pixel slab
  const int co = threadIdx.x;
  if (co >= cout) return;
  float s = 0.f;
  const long long p0 = (long long)blockIdx.x * 256;
  for (long long p = p0; p < p0 + 256 && p < P; ++p) s += (float)g[p * cout + co];
  atomicAdd(&db[co], s);
}

// g = dy * (y > 0) (ReLU backward); dy and y read at (stride, off), g contiguous
__global__ void k_relu_bwd(const bf16* __restrict__ dy, int dy_stride, int dy_off, const bf16* __restrict__ y,
                           int y_stride, int y_off, long long P, int C, bf16* __restrict__ g) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * C) return;
  long long p = i / C;
  int c = (int)(i - p * C);
  g[i] = ((float)y[p * y_stride + y_off + c] > 0.f) ? dy[p * dy_stride + dy_off + c] : (bf16)0.f;
}

// 2x2 max pool (H, W even); idx[q][c] = argmax position (0..3)
__global__ void k_pool(const bf16* __restrict__ in, int in_stride, int in_off, int C, int B, int H, int W,
                       bf16* __restrict__ out, uint8_t* __restrict__ idx) {
  const int Ho = H / 2, Wo = W / 2;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * Ho * Wo * C) return;
  const int c = (int)(i % C);
  long long q = i / C;
  const int xo = (int)(q % Wo);
  long long t = q / Wo;
  const int yo = (int)(t % Ho), b = (int)(t / Ho);
  float best = -INFINITY;
  int arg = 0;
  for (int k = 0; k < 4; ++k) {
    const int yy = 2 * yo + (k >> 1), xx = 2 * xo + (k & 1);
    const float v = (float)in[(((long long)b * H + yy) * W + xx) * in_stride + in_off + c];
    if (v > best) {
      best = v;
      arg = k;
    }
  }
  out[q * C + c] = (bf16)best;
  idx[q * C + c] = (uint8_t)arg;
}

// routes the pooled gradient to the argmax and ADDS it into dx (strided)
__global__ void k_pool_bwd(const bf16* __restrict__ dy, const uint8_t* __restrict__ idx, int C, int B, int H, int W,
                           bf16* __restrict__ dx, int dx_stride, int dx_off) {
  const int Ho = H / 2, Wo = W / 2;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * Ho * Wo * C) return;
  const int c = (int)(i % C);
  long long q = i / C;
  const int xo = (int)(q % Wo);
  long long t = q / Wo;
  const int yo = (int)(t % Ho), b = (int)(t / Ho);
  const int k = idx[i];
  const int yy = 2 * yo + (k >> 1), xx = 2 * xo + (k & 1);
  bf16* d = dx + (((long long)b * H + yy) * W + xx) * dx_stride + dx_off + c;
  *d = (bf16)((float)*d + (float)dy[i]);
}

// nearest 2x upsampling of a coarse [B][H/2][W/2][C] tensor into channels
// [0, C) of a fine buffer with the given stride
__global__ void k_upsample(const bf16* __restrict__ in, int C, int B, int H, int W, bf16* __restrict__ out,
                           int out_stride) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * H * W * C) return;
  const int c = (int)(i % C);
  long long p = i / C;
  const int x = (int)(p % W);
  long long t = p / W;
  const int y = (int)(t % H), b = (int)(t / H);
  out[p * out_stride + c] = in[(((long long)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c];
}

// backward of the upsampling: sum of the 2x2 fine gradients (channels [0, C))
__global__ void k_upsample_bwd(const bf16* __restrict__ dfine, int fstride, int C, int B, int H, int W,
                               bf16* __restrict__ dcoarse) {
  const int Ho = H / 2, Wo = W / 2;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * Ho * Wo * C) return;
  const int c = (int)(i % C);
  long long q = i / C;
  const int xo = (int)(q % Wo);
  long long t = q / Wo;
  const int yo = (int)(t % Ho), b = (int)(t / Ho);
  float s = 0.f;
  for (int k = 0; k < 4; ++k) {
    const int yy = 2 * yo + (k >> 1), xx = 2 * xo + (k & 1);
    s += (float)dfine[(((long long)b * H + yy) * W + xx) * fstride + c];
  }
  dcoarse[i] = (bf16)s;
}

// 1x1 head: out[p] = sum_c w[c] a[p][c] + b (FP32)
__global__ void k_head(const bf16* __restrict__ a, long long P, const float* __restrict__ w,
                       const float* __restrict__ bias, float* __restrict__ out) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const bf16x8* ap = (const bf16x8*)(a + p * HEAD_C);
  const bf16x8 a0 = ap[0], a1 = ap[1];
  float s = *bias;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += w[c] * (float)a0[c] + w[8 + c] * (float)a1[c];
  out[p] = s;
}

__global__ void __launch_bounds__(256) k_head_bwd(const float* __restrict__ dout, const bf16* __restrict__ a,
                                                  long long P, const float* __restrict__ w, bf16* __restrict__ da,
                                                  float* __restrict__ dw) {
  __shared__ float red[HEAD_C + 1][4];
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float d = p < P ? dout[p] : 0.f;
  float gw[HEAD_C + 1];
#pragma unroll
  for (int c = 0; c < HEAD_C; ++c) {
    const float av = p < P ? (float)a[p * HEAD_C + c] : 0.f;
    gw[c] = d * av;
    if (p < P) da[p * HEAD_C + c] = (bf16)(d * w[c]);
  }
  gw[HEAD_C] = d;
#pragma unroll
  for (int c = 0; c <= HEAD_C; ++c) {
    float v = ni::wave_sum_f(gw[c]);
    if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x <= HEAD_C) {
    float s = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
    atomicAdd(&dw[threadIdx.x], s);
  }
}

// per-component centred MSE: e = pred - target; L = sum (e - mean_c e)^2 / n_valid
__global__ void k_loss_sums(const float* __restrict__ pred, const float* __restrict__ tgt,
                            const int* __restrict__ lab, long long P, int ncomp, float* __restrict__ csum,
                            float* __restrict__ ccnt, int* __restrict__ nvalid) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int c = lab[p];
  if (c < 0 || c >= ncomp) return;  // ids outside [0, ncomp) are ignored
  atomicAdd(nvalid, 1);
  atomicAdd(&csum[c], pred[p] - tgt[p]);
  atomicAdd(&ccnt[c], 1.f);
}

__global__ void __launch_bounds__(256) k_loss_grad(const float* __restrict__ pred, const float* __restrict__ tgt,
                                                   const int* __restrict__ lab, long long P, int ncomp,
                                                   const float* __restrict__ csum, const float* __restrict__ ccnt,
                                                   const int* __restrict__ nvalid, float* __restrict__ dout,
                                                   double* __restrict__ loss) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  const float inv_n = *nvalid > 0 ? 1.f / (float)*nvalid : 0.f;
  if (p < P) {
    const int c = lab[p];
    float g = 0.f;
    if (c >= 0 && c < ncomp) {
      const float e = pred[p] - tgt[p] - csum[c] / ccnt[c];
      g = 2.f * e * inv_n;
      l = (double)e * e * inv_n;
    }
    dout[p] = g;
  }
  double v[1] = {l};
  __shared__ double red[4];
  ni::block_sum<1>(v, red);
  if (threadIdx.x == 0) atomicAdd(loss, v[0]);
}

// Adam on the FP32 master parameters; conv weight gradients arrive in the
// padded co-major layout dWt[co][tap*cin + ci] and are mapped here
struct ParamMap {
  int off_w[NCONV], off_b[NCONV], off_gw[NCONV], off_gb[NCONV];
  int off_hw, off_hb, off_ghw, off_ghb;
  int n;
};

__global__ void k_adam(float* __restrict__ prm, float* __restrict__ mom1, float* __restrict__ mom2,
                       const float* __restrict__ grad, const int* __restrict__ gidx, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[gidx[i]];
  const float m = b1 * mom1[i] + (1.f - b1) * g;
  const float v = b2 * mom2[i] + (1.f - b2) * g * g;
  mom1[i] = m;
  mom2[i] = v;
  prm[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// master W[tap][ci][co] (real cin) -> forward Wt[co][tap*cin_pad + ci] and
// data-gradient Wb[ci][(8-tap)*cout + co], both BF16, zero padded
__global__ void k_pack(const float* __restrict__ w, int cin_real, int cin, int cout, bf16* __restrict__ wt, int kpad,
                       bf16* __restrict__ wb, int kpad_b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cout * kpad) {
    const int co = i / kpad, k = i - co * kpad;
    float v = 0.f;
    if (k < 9 * cin) {
      const int tap = k / cin, ci = k - tap * cin;
      if (ci < cin_real) v = w[((size_t)tap * cin_real + ci) * cout + co];
    }
    wt[i] = (bf16)v;
  }
  if (wb && i < cin * kpad_b) {
    const int ci = i / kpad_b, k = i - ci * kpad_b;
    float v = 0.f;
    if (k < 9 * cout && ci < cin_real) {
      const int tapf = k / cout, co = k - tapf * cout;
      v = w[((size_t)(8 - tapf) * cin_real + ci) * cout + co];
    }
    wb[i] = (bf16)v;
  }
}

__global__ void k_zero_f32(float* a, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.f;
}

__global__ void k_zero_bf16(bf16* a, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (bf16)0.f;
}

__global__ void k_gather_grad(const float* __restrict__ g, const int* __restrict__ gidx, int n,
                              float* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = g[gidx[i]];
}

__global__ void k_crop(const float* __restrict__ in, int Wp, int H, int W, float* __restrict__ out) {
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (long long)H * W) return;
  out[p] = in[(p / W) * Wp + p % W];
}

inline int nblk(long long n, int b = 256) { return (int)((n + b - 1) / b); }

}  // namespace

// ================================================================== model
namespace nil {

struct Act {
  bf16* p = nullptr;
  int stride = 0, off = 0;
};

struct UnetModel {
  // master FP32 parameters (device) and Adam state
  float* prm = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* grad = nullptr;  // gradients in kernel layout (padded dWt, db, head)
  int* gidx = nullptr;    // master index -> gradient index
  int nprm = 0, ngrad = 0, step = 0;
  ParamMap map;
  bf16* wt[NCONV] = {};
  bf16* wb[NCONV] = {};
  int kpad[NCONV], kpad_b[NCONV];
  // activations for the current (B, H, W)
  int B = 0, H = 0, W = 0;
  std::vector<void*> act_bufs;
  bf16 *x = nullptr, *e0a, *cat0, *p0, *e1a, *cat1, *p1, *e2a, *cat2, *p2, *e3a, *e3b, *d2a, *d2b, *d1a, *d1b, *d0a,
       *d0b;
  uint8_t *i0, *i1, *i2;
  float* out = nullptr;
  // gradient buffers
  bf16 *g_a = nullptr, *g_b = nullptr, *g_cat0, *g_cat1, *g_cat2, *g_c;
  float* dout = nullptr;
  float *csum = nullptr, *ccnt = nullptr;
  int ccap = 0;
  double* loss = nullptr;
  void* pad_in = nullptr;
  size_t pad_cap = 0;
};

static void free_acts(UnetModel* M) {
  for (void* p : M->act_bufs) (void)hipFree(p);
  M->act_bufs.clear();
  M->B = M->H = M->W = 0;
}

static hipError_t alloc_acts(UnetModel* M, int B, int H, int W) {
  if (M->B == B && M->H == H && M->W == W) return hipSuccess;
  free_acts(M);
  const long long P0 = (long long)B * H * W, P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
  auto a = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) return nullptr;
    M->act_bufs.push_back(p);
    return p;
  };
  const size_t e = sizeof(bf16);
  M->x = (bf16*)a(P0 * 8 * e);
  M->e0a = (bf16*)a(P0 * 16 * e);
  M->cat0 = (bf16*)a(P0 * 48 * e);
  M->p0 = (bf16*)a(P1 * 16 * e);
  M->i0 = (uint8_t*)a(P1 * 16);
  M->e1a = (bf16*)a(P1 * 32 * e);
  M->cat1 = (bf16*)a(P1 * 96 * e);
  M->p1 = (bf16*)a(P2 * 32 * e);
  M->i1 = (uint8_t*)a(P2 * 32);
  M->e2a = (bf16*)a(P2 * 64 * e);
  M->cat2 = (bf16*)a(P2 * 192 * e);
  M->p2 = (bf16*)a(P3 * 64 * e);
  M->i2 = (uint8_t*)a(P3 * 64);
  M->e3a = (bf16*)a(P3 * 128 * e);
  M->e3b = (bf16*)a(P3 * 128 * e);
  M->d2a = (bf16*)a(P2 * 64 * e);
  M->d2b = (bf16*)a(P2 * 64 * e);
  M->d1a = (bf16*)a(P1 * 32 * e);
  M->d1b = (bf16*)a(P1 * 32 * e);
  M->d0a = (bf16*)a(P0 * 16 * e);
  M->d0b = (bf16*)a(P0 * 16 * e);
  M->out = (float*)a(P0 * sizeof(float));
  // gradient scratch: the largest per-layer tensor is P0 * 48 channels
  M->g_a = (bf16*)a(P0 * 48 * e);
  M->g_b = (bf16*)a(P0 * 48 * e);
  M->g_c = (bf16*)a(P0 * 48 * e);
  M->g_cat0 = (bf16*)a(P0 * 48 * e);
  M->g_cat1 = (bf16*)a(P1 * 96 * e);
  M->g_cat2 = (bf16*)a(P2 * 192 * e);
  M->dout = (float*)a(P0 * sizeof(float));
  for (void* p : M->act_bufs)
    if (!p) {
      free_acts(M);
      return hipErrorOutOfMemory;
    }
  M->B = B;
  M->H = H;
  M->W = W;
  return hipSuccess;
}

static void conv(const UnetModel* M, int l, const bf16* in, int in_stride, int in_off, bf16* out, int out_stride,
                 int out_off, int B, int H, int W, hipStream_t st) {
  const ConvSpec& s = SPECS[l];
  const long long P = (long long)B * H * W;
  dim3 grid(nblk(P, 64), (s.cout + 127) / 128);
  k_conv<<<grid, 256, 0, st>>>(in, in_stride, in_off, s.cin, M->wt[l], M->kpad[l], M->prm + M->map.off_b[l], out,
                               out_stride, out_off, s.cout, 1, B, H, W);
}

// forward pass on M->x (features, B x H x W, H and W multiples of 8)
static hipError_t forward(UnetModel* M, hipStream_t st) {
  const int B = M->B, H = M->H, W = M->W;
  const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
  const long long P0 = (long long)B * H * W;
  conv(M, 0, M->x, 8, 0, M->e0a, 16, 0, B, H, W, st);
  conv(M, 1, M->e0a, 16, 0, M->cat0, 48, 32, B, H, W, st);
  k_pool<<<nblk(P0 / 4 * 16), 256, 0, st>>>(M->cat0, 48, 32, 16, B, H, W, M->p0, M->i0);
  conv(M, 2, M->p0, 16, 0, M->e1a, 32, 0, B, H1, W1, st);
  conv(M, 3, M->e1a, 32, 0, M->cat1, 96, 64, B, H1, W1, st);
  k_pool<<<nblk(P0 / 16 * 32), 256, 0, st>>>(M->cat1, 96, 64, 32, B, H1, W1, M->p1, M->i1);
  conv(M, 4, M->p1, 32, 0, M->e2a, 64, 0, B, H2, W2, st);
  conv(M, 5, M->e2a, 64, 0, M->cat2, 192, 128, B, H2, W2, st);
  k_pool<<<nblk(P0 / 64 * 64), 256, 0, st>>>(M->cat2, 192, 128, 64, B, H2, W2, M->p2, M->i2);
  conv(M, 6, M->p2, 64, 0, M->e3a, 128, 0, B, H3, W3, st);
  conv(M, 7, M->e3a, 128, 0, M->e3b, 128, 0, B, H3, W3, st);
  k_upsample<<<nblk(P0 / 16 * 128), 256, 0, st>>>(M->e3b, 128, B, H2, W2, M->cat2, 192);
  conv(M, 8, M->cat2, 192, 0, M->d2a, 64, 0, B, H2, W2, st);
  conv(M, 9, M->d2a, 64, 0, M->d2b, 64, 0, B, H2, W2, st);
  k_upsample<<<nblk(P0 / 4 * 64), 256, 0, st>>>(M->d2b, 64, B, H1, W1, M->cat1, 96);
  conv(M, 10, M->cat1, 96, 0, M->d1a, 32, 0, B, H1, W1, st);
  conv(M, 11, M->d1a, 32, 0, M->d1b, 32, 0, B, H1, W1, st);
  k_upsample<<<nblk(P0 * 32), 256, 0, st>>>(M->d1b, 32, B, H, W, M->cat0, 48);
  conv(M, 12, M->cat0, 48, 0, M->d0a, 16, 0, B, H, W, st);
  conv(M, 13, M->d0a, 16, 0, M->d0b, 16, 0, B, H, W, st);
  k_head<<<nblk(P0), 256, 0, st>>>(M->d0b, P0, M->prm + M->map.off_hw, M->prm + M->map.off_hb, M->out);
  return hipGetLastError();
}

// One conv layer's backward.  dy = dL/d(output activation) at (dy_stride,
// dy_off); y = the stored output activation at (y_stride, y_off); `in` the
// layer input.  Accumulates the weight and bias gradients and, if asked,
// writes dL/d(input) contiguous [P][cin] into din (din_stride = cin) or
// into a wider buffer with din_stride.
struct LayerIO {
  const bf16* in;
  int in_stride, in_off;
  const bf16* y;
  int y_stride, y_off;
};

static void conv_bwd(UnetModel* M, int l, const LayerIO& io, const bf16* dy, int dy_stride, int dy_off, bf16* gpre,
                     bf16* din, int din_stride, int B, int H, int W, hipStream_t st) {
  const ConvSpec& s = SPECS[l];
  const long long P = (long long)B * H * W;
  k_relu_bwd<<<nblk(P * s.cout), 256, 0, st>>>(dy, dy_stride, dy_off, io.y, io.y_stride, io.y_off, P, s.cout, gpre);
  dim3 g((M->kpad[l] / 16 + 3) / 4, s.cout / 16, (unsigned)((P + WG_SLAB - 1) / WG_SLAB));
  k_wgrad<<<g, 256, 0, st>>>(io.in, io.in_stride, io.in_off, s.cin, gpre, s.cout, M->grad + M->map.off_gw[l],
                             M->kpad[l], B, H, W);
  k_bias_grad<<<nblk(P, 256), 256, 0, st>>>(gpre, P, s.cout, M->grad + M->map.off_gb[l]);
  if (din) {
    dim3 grid(nblk(P, 64), (s.cin + 127) / 128);
    k_conv<<<grid, 256, 0, st>>>(gpre, s.cout, 0, s.cout, M->wb[l], M->kpad_b[l], nullptr, din, din_stride, 0, s.cin,
                                 0, B, H, W);
  }
}

// backward from M->dout (dL/d out, FP32 [P]); accumulates into M->grad
static hipError_t backward(UnetModel* M, hipStream_t st) {
  const int B = M->B, H = M->H, W = M->W;
  const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
  const long long P0 = (long long)B * H * W, P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
  bf16 *ga = M->g_a, *gb = M->g_b, *gc = M->g_c;
  k_head_bwd<<<nblk(P0), 256, 0, st>>>(M->dout, M->d0b, P0, M->prm + M->map.off_hw, ga, M->grad + M->map.off_ghw);
  // level 0 decoder
  conv_bwd(M, 13, {M->d0a, 16, 0, M->d0b, 16, 0}, ga, 16, 0, gc, gb, 16, B, H, W, st);
  conv_bwd(M, 12, {M->cat0, 48, 0, M->d0a, 16, 0}, gb, 16, 0, gc, M->g_cat0, 48, B, H, W, st);
  k_upsample_bwd<<<nblk(P1 * 32), 256, 0, st>>>(M->g_cat0, 48, 32, B, H, W, ga);
  // level 1 decoder
  conv_bwd(M, 11, {M->d1a, 32, 0, M->d1b, 32, 0}, ga, 32, 0, gc, gb, 32, B, H1, W1, st);
  conv_bwd(M, 10, {M->cat1, 96, 0, M->d1a, 32, 0}, gb, 32, 0, gc, M->g_cat1, 96, B, H1, W1, st);
  k_upsample_bwd<<<nblk(P2 * 64), 256, 0, st>>>(M->g_cat1, 96, 64, B, H1, W1, ga);
  // level 2 decoder
  conv_bwd(M, 9, {M->d2a, 64, 0, M->d2b, 64, 0}, ga, 64, 0, gc, gb, 64, B, H2, W2, st);
  conv_bwd(M, 8, {M->cat2, 192, 0, M->d2a, 64, 0}, gb, 64, 0, gc, M->g_cat2, 192, B, H2, W2, st);
  k_upsample_bwd<<<nblk(P3 * 128), 256, 0, st>>>(M->g_cat2, 192, 128, B, H2, W2, ga);
  // bottom
  conv_bwd(M, 7, {M->e3a, 128, 0, M->e3b, 128, 0}, ga, 128, 0, gc, gb, 128, B, H3, W3, st);
  conv_bwd(M, 6, {M->p2, 64, 0, M->e3a, 128, 0}, gb, 128, 0, gc, ga, 64, B, H3, W3, st);
  // e2b feeds the pool and the skip: its gradient = g_cat2[:, 128:192] + pool_bwd
  k_pool_bwd<<<nblk(P3 * 64), 256, 0, st>>>(ga, M->i2, 64, B, H2, W2, M->g_cat2, 192, 128);
  conv_bwd(M, 5, {M->e2a, 64, 0, M->cat2, 192, 128}, M->g_cat2, 192, 128, gc, gb, 64, B, H2, W2, st);
  conv_bwd(M, 4, {M->p1, 32, 0, M->e2a, 64, 0}, gb, 64, 0, gc, ga, 32, B, H2, W2, st);
  k_pool_bwd<<<nblk(P2 * 32), 256, 0, st>>>(ga, M->i1, 32, B, H1, W1, M->g_cat1, 96, 64);
  conv_bwd(M, 3, {M->e1a, 32, 0, M->cat1, 96, 64}, M->g_cat1, 96, 64, gc, gb, 32, B, H1, W1, st);
  conv_bwd(M, 2, {M->p0, 16, 0, M->e1a, 32, 0}, gb, 32, 0, gc, ga, 16, B, H1, W1, st);
  k_pool_bwd<<<nblk(P1 * 16), 256, 0, st>>>(ga, M->i0, 16, B, H, W, M->g_cat0, 48, 32);
  conv_bwd(M, 1, {M->e0a, 16, 0, M->cat0, 48, 32}, M->g_cat0, 48, 32, gc, gb, 16, B, H, W, st);
  conv_bwd(M, 0, {M->x, 8, 0, M->e0a, 16, 0}, gb, 16, 0, gc, nullptr, 0, B, H, W, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------- setup
static int build_map(ParamMap& mp, std::vector<int>& gidx, int* kp, int* kpb) {
  int n = 0, g = 0;
  for (int l = 0; l < NCONV; ++l) {
    const ConvSpec& s = SPECS[l];
    kp[l] = kpad_of(s.cin);
    kpb[l] = kpad_of(s.cout);
    mp.off_w[l] = n;
    n += 9 * s.cin_real * s.cout;
    mp.off_b[l] = n;
    n += s.cout;
  }
  mp.off_hw = n;
  n += HEAD_C;
  mp.off_hb = n;
  n += 1;
  mp.n = n;
  for (int l = 0; l < NCONV; ++l) {
    mp.off_gw[l] = g;
    g += SPECS[l].cout * kp[l];
    mp.off_gb[l] = g;
    g += SPECS[l].cout;
  }
  mp.off_ghw = g;
  g += HEAD_C;
  mp.off_ghb = g;
  g += 1;
  gidx.assign(n, 0);
  for (int l = 0; l < NCONV; ++l) {
    const ConvSpec& s = SPECS[l];
    for (int tap = 0; tap < 9; ++tap)
      for (int ci = 0; ci < s.cin_real; ++ci)
        for (int co = 0; co < s.cout; ++co)
          gidx[mp.off_w[l] + (tap * s.cin_real + ci) * s.cout + co] = mp.off_gw[l] + co * kp[l] + tap * s.cin + ci;
    for (int co = 0; co < s.cout; ++co) gidx[mp.off_b[l] + co] = mp.off_gb[l] + co;
  }
  for (int c = 0; c < HEAD_C; ++c) gidx[mp.off_hw + c] = mp.off_ghw + c;
  gidx[mp.off_hb] = mp.off_ghb;
  return g;
}

static hipError_t pack(UnetModel* M, hipStream_t st) {
  for (int l = 0; l < NCONV; ++l) {
    const ConvSpec& s = SPECS[l];
    const int n = std::max(s.cout * M->kpad[l], s.cin * M->kpad_b[l]);
    k_pack<<<nblk(n), 256, 0, st>>>(M->prm + M->map.off_w[l], s.cin_real, s.cin, s.cout, M->wt[l], M->kpad[l],
                                   l == 0 ? nullptr : M->wb[l], M->kpad_b[l]);
  }
  return hipGetLastError();
}

void unet_free(UnetModel* M) {
  if (!M) return;
  free_acts(M);
  for (void* p : {(void*)M->prm, (void*)M->m1, (void*)M->m2, (void*)M->grad, (void*)M->gidx, (void*)M->csum,
                  (void*)M->ccnt, (void*)M->loss, M->pad_in})
    if (p) (void)hipFree(p);
  for (int l = 0; l < NCONV; ++l) {
    if (M->wt[l]) (void)hipFree(M->wt[l]);
    if (M->wb[l]) (void)hipFree(M->wb[l]);
  }
  delete M;
}

// allocates a model with the given FP32 master parameters (host)
static int make_model(UnetModel** out, const float* host_prm, std::string* err) {
  UnetModel* M = new (std::nothrow) UnetModel();
  if (!M) return 0;
  std::vector<int> gidx;
  M->ngrad = build_map(M->map, gidx, M->kpad, M->kpad_b);
  M->nprm = M->map.n;
  bool ok = hipMalloc(&M->prm, M->nprm * sizeof(float)) == hipSuccess &&
            hipMalloc(&M->m1, M->nprm * sizeof(float)) == hipSuccess &&
            hipMalloc(&M->m2, M->nprm * sizeof(float)) == hipSuccess &&
            hipMalloc(&M->grad, M->ngrad * sizeof(float)) == hipSuccess &&
            hipMalloc(&M->gidx, M->nprm * sizeof(int)) == hipSuccess &&
            hipMalloc(&M->loss, 2 * sizeof(double)) == hipSuccess;
  for (int l = 0; ok && l < NCONV; ++l) {
    ok = hipMalloc(&M->wt[l], (size_t)SPECS[l].cout * M->kpad[l] * sizeof(bf16)) == hipSuccess &&
         hipMalloc(&M->wb[l], (size_t)SPECS[l].cin * M->kpad_b[l] * sizeof(bf16)) == hipSuccess;
  }
  ok = ok && hipMemcpy(M->prm, host_prm, M->nprm * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(M->m1, 0, M->nprm * sizeof(float)) == hipSuccess &&
       hipMemset(M->m2, 0, M->nprm * sizeof(float)) == hipSuccess &&
       hipMemcpy(M->gidx, gidx.data(), M->nprm * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
       pack(M, nullptr) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    *err = "device allocation for the U-Net failed";
    unet_free(M);
    return 0;
  }
  *out = M;
  return 1;
}

int unet_param_count() {
  ParamMap mp;
  std::vector<int> g;
  int kp[NCONV], kpb[NCONV];
  build_map(mp, g, kp, kpb);
  return mp.n;
}

// He-normal initialisation from a 64-bit seed (counter-based Box-Muller)
void unet_init_params(uint64_t seed, float* out) {
  ParamMap mp;
  std::vector<int> g;
  int kp[NCONV], kpb[NCONV];
  build_map(mp, g, kp, kpb);
  uint64_t st = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  auto next = [&]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto normal = [&]() {
    double u1 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double u2 = ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  };
  for (int l = 0; l < NCONV; ++l) {
    const ConvSpec& s = SPECS[l];
    const double sd = sqrt(2.0 / (9.0 * s.cin_real));
    for (int i = 0; i < 9 * s.cin_real * s.cout; ++i) out[mp.off_w[l] + i] = (float)(sd * normal());
    for (int i = 0; i < s.cout; ++i) out[mp.off_b[l] + i] = 0.f;
  }
  for (int c = 0; c < HEAD_C; ++c) out[mp.off_hw + c] = (float)(sqrt(1.0 / HEAD_C) * normal());
  out[mp.off_hb] = 0.f;
}

// blob: "NIUNET01", int32 count, FP32 parameters
static const char MAGIC[8] = {'N', 'I', 'U', 'N', 'E', 'T', '0', '1'};
size_t unet_blob_size() { return 8 + 4 + (size_t)unet_param_count() * 4; }

int unet_load(UnetModel** out, const void* blob, size_t nbytes, std::string* err) {
  *out = nullptr;
  const int n = unet_param_count();
  if (nbytes != unet_blob_size() || memcmp(blob, MAGIC, 8) != 0) {
    *err = "weight blob has the wrong size or magic (expected NIUNET01)";
    return 0;
  }
  int32_t cnt;
  memcpy(&cnt, (const char*)blob + 8, 4);
  if (cnt != n) {
    *err = "weight blob parameter count mismatch";
    return 0;
  }
  std::vector<float> h(n);
  memcpy(h.data(), (const char*)blob + 12, (size_t)n * 4);
  for (float v : h)
    if (!std::isfinite(v)) {
      *err = "weight blob holds non-finite parameters";
      return 0;
    }
  return make_model(out, h.data(), err);
}

int unet_new(UnetModel** out, uint64_t seed, std::string* err) {
  std::vector<float> h(unet_param_count());
  unet_init_params(seed, h.data());
  return make_model(out, h.data(), err);
}

hipError_t unet_save(UnetModel* M, void* blob) {
  memcpy(blob, MAGIC, 8);
  int32_t n = M->nprm;
  memcpy((char*)blob + 8, &n, 4);
  return hipMemcpy((char*)blob + 12, M->prm, (size_t)n * 4, hipMemcpyDeviceToHost);
}

size_t unet_workspace_bytes(int H, int W) { return 256; }

// log-depth estimate for a whole map (padded to multiples of 8); out [H][W]
hipError_t unet_predict(UnetModel* M, const float* normals, const uint8_t* mask, int H, int W, const ni_camera* cam,
                        float* out, void* ws, size_t wsb, hipStream_t st) {
  const int Hp = (H + 7) / 8 * 8, Wp = (W + 7) / 8 * 8;
  hipError_t e = alloc_acts(M, 1, Hp, Wp);
  if (e != hipSuccess) return e;
  k_features<<<nblk((long long)Hp * Wp), 256, 0, st>>>(normals, mask, H, W, Hp, Wp, cam->proj == NI_PERSP, cam->fx,
                                                      cam->fy, cam->cx, cam->cy, M->x);
  e = forward(M, st);
  if (e != hipSuccess) return e;
  k_crop<<<nblk((long long)H * W), 256, 0, st>>>(M->out, Wp, H, W, out);
  return hipGetLastError();
}

// forward on FP32 features [B][H][W][6] (H, W multiples of 8): out [B][H][W]
hipError_t unet_forward_raw(UnetModel* M, const float* f6, int B, int H, int W, float* out, hipStream_t st) {
  hipError_t e = alloc_acts(M, B, H, W);
  if (e != hipSuccess) return e;
  const long long P = (long long)B * H * W;
  k_features_raw<<<nblk(P), 256, 0, st>>>(f6, P, M->x);
  e = forward(M, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(out, M->out, P * sizeof(float), hipMemcpyDeviceToDevice, st);
}

// gradient of sum(dout * out) w.r.t. the master parameters, after
// unet_forward_raw on the same shape; grad_out [n] FP32 device
static hipError_t grads(UnetModel* M, hipStream_t st) {
  const long long P = (long long)M->B * M->H * M->W;
  k_zero_f32<<<nblk(M->ngrad), 256, 0, st>>>(M->grad, M->ngrad);
  k_zero_bf16<<<nblk(P * 48), 256, 0, st>>>(M->g_cat0, P * 48);
  k_zero_bf16<<<nblk(P / 4 * 96), 256, 0, st>>>(M->g_cat1, P / 4 * 96);
  k_zero_bf16<<<nblk(P / 16 * 192), 256, 0, st>>>(M->g_cat2, P / 16 * 192);
  return backward(M, st);
}

hipError_t unet_backward_raw(UnetModel* M, const float* dout, float* grad_out, hipStream_t st) {
  const long long P = (long long)M->B * M->H * M->W;
  hipError_t e = hipMemcpyAsync(M->dout, dout, P * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  e = grads(M, st);
  if (e != hipSuccess) return e;
  k_gather_grad<<<nblk(M->nprm), 256, 0, st>>>(M->grad, M->gidx, M->nprm, grad_out);
  return hipGetLastError();
}

int unet_nprm(const UnetModel* M) { return M->nprm; }

hipError_t unet_get_params(UnetModel* M, float* host) {
  return hipMemcpy(host, M->prm, (size_t)M->nprm * 4, hipMemcpyDeviceToHost);
}

hipError_t unet_set_params(UnetModel* M, const float* host, hipStream_t st) {
  hipError_t e = hipMemcpy(M->prm, host, (size_t)M->nprm * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return pack(M, st);
}

// One Adam step on a batch of B patches of S x S pixels (S multiple of 8):
// normals [B][S][S][3], mask [B][S][S], per-patch cameras (host), target
// log-depth [B][S][S], labels [B][S][S] with ids unique across the batch
// (0 .. ncomp-1, -1 off the mask).  Loss = sum over valid pixels of
// (e - mean_c e)^2 / n_valid with e = prediction - target: the prediction
// is only asked to be right up to one offset per component.
hipError_t unet_train_step(UnetModel* M, const float* normals, const uint8_t* mask, const ni_camera* cams,
                           const float* target, const int* labels, int ncomp, int B, int S, float lr, double* loss,
                           hipStream_t st) {
  hipError_t e = alloc_acts(M, B, S, S);
  if (e != hipSuccess) return e;
  const long long PS = (long long)S * S, P = PS * B;
  for (int b = 0; b < B; ++b)
    k_features<<<nblk(PS), 256, 0, st>>>(normals + b * PS * 3, mask + b * PS, S, S, S, S, cams[b].proj == NI_PERSP,
                                         cams[b].fx, cams[b].fy, cams[b].cx, cams[b].cy, M->x + b * PS * 8);
  e = forward(M, st);
  if (e != hipSuccess) return e;
  if (ncomp > M->ccap) {
    if (M->csum) (void)hipFree(M->csum);
    if (M->ccnt) (void)hipFree(M->ccnt);
    M->csum = M->ccnt = nullptr;
    M->ccap = 0;
    if (hipMalloc(&M->csum, (size_t)ncomp * 4) != hipSuccess || hipMalloc(&M->ccnt, (size_t)ncomp * 4) != hipSuccess)
      return hipErrorOutOfMemory;
    M->ccap = ncomp;
  }
  k_zero_f32<<<nblk(ncomp), 256, 0, st>>>(M->csum, ncomp);
  k_zero_f32<<<nblk(ncomp), 256, 0, st>>>(M->ccnt, ncomp);
  // loss accumulator (double) and valid-pixel counter (int) share one buffer
  e = hipMemsetAsync(M->loss, 0, 2 * sizeof(double), st);
  if (e != hipSuccess) return e;
  int* nvalid = (int*)(M->loss + 1);
  k_loss_sums<<<nblk(P), 256, 0, st>>>(M->out, target, labels, P, ncomp, M->csum, M->ccnt, nvalid);
  k_loss_grad<<<nblk(P), 256, 0, st>>>(M->out, target, labels, P, ncomp, M->csum, M->ccnt, nvalid, M->dout,
                                      M->loss);
  e = grads(M, st);
  if (e != hipSuccess) return e;
  M->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)M->step), c2 = 1.f - powf(b2, (float)M->step);
  k_adam<<<nblk(M->nprm), 256, 0, st>>>(M->prm, M->m1, M->m2, M->grad, M->gidx, M->nprm, lr, b1, b2, 1e-8f, c1, c2);
  e = pack(M, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(loss, M->loss, sizeof(double), hipMemcpyDeviceToHost, st);
}

}  // namespace nil
