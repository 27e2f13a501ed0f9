/*
 * ni.h -- C ABI of the MI355X (gfx950) library for component-based normal
 * integration ("Towards Fast and Scalable Normal Integration using
 * Continuous Components", Milano et al., WACV 2026).
 *
 * Problem (Sec. 3.1): given a normal map n(u, v), a validity mask and the
 * camera intrinsics, recover log-depth z~ = log z such that neighbouring
 * pixels satisfy the model of continuity z~_a - z~_b = omega_{b->a}
 * (Eq. 1, with omega from Eq. 3).  The method (Sec. 3.2-3.4, Alg. 1):
 *   (a) label continuous components: connected components over 4-neighbour
 *       edges whose normals differ by less than theta_c (Sec. 3.3);
 *   (b) fill every component independently: weighted least squares on its
 *       intra-component edges, solved by preconditioned CG (Eq. 14-15);
 *   (c) relative-scale IRLS: one additive log-scale per component from the
 *       inter-component edges, with BiNI and outlier weights (Eq. 16-19).
 *
 * Conventions used by every entry point:
 *   - pixel (u, v) = (column, row), centre at integer coordinates; raster
 *     index p = v*W + u; arrays are row-major [H][W] (normals [H][W][3]).
 *   - perspective rays tau(u, v) = ((u - cx)/fx, (v - cy)/fy, 1).
 *   - orthographic mode (not in the paper): additive depth, the same
 *     two-tangent-planes construction with parallel rays; depth is in the
 *     unit of pixel_pitch and the per-component unknown is an offset.
 *   - every device pointer must be a device (hipMalloc / torch CUDA) buffer
 *     on the context's device; every host pointer a plain host buffer.  The
 *     caller owns all of them; the library never frees a caller pointer.
 *   - calls are stream-ordered on the context's stream (ni_set_stream) and
 *     blocking: they return after the results are written.
 *   - nothing throws across the ABI; every call returns ni_status and, on
 *     error, ni_last_error(ctx) holds a message.  One context per thread;
 *     contexts are independent.
 */
#ifndef NI_H
#define NI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NI_ABI_VERSION 3
#define NI_MAX_IRLS 256

typedef enum {
  NI_OK = 0,
  NI_E_ARG = 1,       /* bad argument (null pointer, bad enum, bad size)      */
  NI_E_SHAPE = 2,     /* output capacity too small (*K is still written)     */
  NI_E_NONFINITE = 3, /* NaN/Inf normal inside the mask                        */
  NI_E_NOMEM = 4,     /* device allocation failed                              */
  NI_E_DEVICE = 5,    /* HIP runtime error                                     */
  NI_E_NOTCONV = 6,   /* a CG solve hit its iteration cap (results written)   */
  NI_E_MODEL = 7      /* bad warm-start weight blob / no model loaded          */
} ni_status;

typedef enum { NI_ORTHO = 0, NI_PERSP = 1 } ni_proj;

typedef struct {
  int32_t proj;        /* ni_proj                                            */
  double fx, fy;       /* focal lengths in pixels (perspective)              */
  double cx, cy;       /* principal point in pixels (perspective)            */
  double pixel_pitch;  /* orthographic: metric size of one pixel             */
} ni_camera;

typedef struct {
  double theta_c_deg;   /* similarity threshold theta_c (Sec. 3.3); <= 0 means
                           every pixel is its own component (theta_c = None)  */
  int32_t connectivity; /* 4, or 8: the diagonal neighbours join the pixel
                           graph too, each diagonal edge modelled with its
                           subpixel at the midpoint of the two pixel centres
                           and f^2 = fx * fy (Sec. 3.1 names 4- and
                           8-connectivity); edge codes are 4 a + direction  */
  int32_t irls_iters;   /* T: relative-scale iterations (1..NI_MAX_IRLS)      */
  int32_t align_iters;  /* leading uniform-weight iterations (Alg. 1: 2)      */
  double bini_k;        /* sharpness k of the BiNI sigmoid (Eq. 5)            */
  double out_L, out_U;  /* outlier thresholds of Eq. 18 (1e-5, 1e-3)          */
  int32_t outlier_mode; /* 0 off, 1 soft (Eq. 18), 2 hard threshold at U      */
  double delta_e_max;   /* relative-energy stop; 0 = run exactly T iterations */
  double w_cut_rel;     /* quotient edges lighter than w_cut_rel * max weight
                           are dropped before each relative-scale solve
                           (1e-12: only weights at the edge of underflow;
                           Eq. 17 keeps every positive weight)              */
  double cg_rtol;       /* fill CG: stop at ||r_c|| <= cg_rtol * ||b_c||      */
  int32_t cg_max_iter;  /* fill CG iteration cap per component                */
  double q_rtol;        /* quotient solve, two rounds of multigrid PCG: the
                           first stops at ||r|| <= q_rtol ||b_abs|| (b_abs =
                           row sums of the pair terms' magnitudes), the
                           second solves for the correction from the
                           flow-form residual b - L s to q_rtol_refine of
                           that residual (at least 1e-13 ||b_abs||)         */
  int32_t q_max_iter;   /* iteration cap of each round; reaching it makes the
                           call return NI_E_NOTCONV (outputs still written) */
  int32_t warm_start;   /* 0 zero start; 1 learned start (needs ni_unet_load) */
  int32_t graphs;       /* 1: the multigrid quotient CG replays each iteration's
                           launches from a HIP graph; 0: plain stream launches
                           (same kernels, same results) */
  int32_t fill_chunk;   /* large-path schedule: 0 autotunes it per map size
                           class; 512, 1024, 2048 or 4096 fixes the shortest
                           chunk (px) per block ...                          */
  int32_t fill_split;   /* ... and, with fill_chunk set, 1 materialises p
                           (three launches per CG iteration), 0 recomputes it
                           (two launches)                                    */
  int32_t fill_precond; /* preconditioner of the large components' CG:
                           1 multigrid (aggregates of 2x2 pixel blocks per
                           component, V(1,1) cycle), 0 Jacobi (the chunked
                           schedule above)                                   */
  int32_t fill_mg_maxit; /* iteration cap of the multigrid fill solve before
                            the large components fall back to the Jacobi
                            path (0: 2000)                                   */
  int32_t freq_merging; /* optional merging (Sec. 3.5, Alg. 1): after every
                           freq_merging-th relative-scale iteration each
                           quotient node joins the neighbour across its
                           edge of smallest |residual| (on a 2^-40 grid,
                           ties to the smaller edge code) and the joined
                           nodes move as one from then on; 0 = off        */
  int32_t variant;      /* 0: the component method (Alg. 1); 1: the
                           pixel-level log-depth baseline the paper compares
                           with, without its discontinuity term (ND, Sec. 4,
                           Table 1): every pixel its own node, no alignment
                           phase (the first iteration weighs each row by
                           the BiNI weight at z = 0), outlier weights from
                           the second iteration, no merging; theta_c,
                           align_iters and freq_merging are ignored      */
  double q_rtol_refine; /* relative target of the quotient solve's second
                           (refinement) round, see q_rtol                  */
} ni_params;

typedef struct {
  int32_t K;             /* number of continuous components                   */
  int32_t n_valid;       /* pixels inside the mask                            */
  int32_t n_regions;     /* connected regions of the full pixel graph G_0     */
  int32_t n_inter_edges; /* |E_inter|                                         */
  int32_t n_pairs;       /* distinct neighbouring component pairs             */
  int32_t irls_iters_run;
  int32_t n_small, n_large;      /* components solved in LDS / grid-wide      */
  int32_t fill_iters_max;        /* largest CG iteration count of a component */
  int32_t fill_notconv;          /* components that hit cg_max_iter           */
  int64_t fill_px_iters;         /* sum over components of n_c * iters_c      */
  int64_t fill_large_px_iters;   /* same, grid-wide components only           */
  int32_t fill_large_launches;   /* CG iteration launches of the large path   */
  int32_t warm_fallbacks;        /* components whose learned start was reset */
  double fill_max_relres;        /* max_c ||r_c|| / ||b_c|| (recursive)       */
  int32_t quot_iters[NI_MAX_IRLS]; /* both quotient solve rounds together */
  double energy[NI_MAX_IRLS];    /* E_t of Alg. 1 per iteration               */
  float ms_setup, ms_label, ms_segments, ms_assemble, ms_warm,
        ms_fill_small, ms_fill_large, ms_irls, ms_finalize, ms_total;
  float ms_large_kernel;  /* the large-path CG iteration launches alone
                             (HIP events around each batch of launches)    */
  int32_t fill_chunk;     /* autotuned schedule of the large path: shortest */
  int32_t fill_split;     /* chunk (px), and 1 if p is materialised (three
                             launches per iteration) instead of recomputed */
  int32_t fill_mg_levels; /* levels of the fill multigrid (0: Jacobi path)  */
  float ms_fill_mg_build; /* its level-0 system and hierarchy build         */
  double fill_mg_bytes;   /* algorithmic HBM bytes of one of its PCG
                             iterations (every level; FP64 values)         */
  int32_t fill_mg_fallback; /* 1: the multigrid solve did not converge
                               within fill_mg_maxit iterations and the
                               large components were solved again with
                               the Jacobi path                             */
  int64_t fill_large_px;  /* pixels of the components on the large path    */
  int32_t merges;         /* merge steps taken (freq_merging > 0)          */
  int32_t nodes_final;    /* quotient nodes after the last merge (K if none) */
  int32_t quot_iters_refine[NI_MAX_IRLS]; /* of quot_iters: the refinement
                                             round's iterations           */
} ni_report;

typedef struct ni_ctx ni_ctx;

/* Defaults: theta_c 2 deg, T 15, 2 alignment iterations, k 2, L 1e-5,
 * U 1e-3, soft outliers, delta_e_max 0, w_cut_rel 1e-12, cg_rtol 1e-6,
 * cg_max_iter 50000, q_rtol 1e-5, q_max_iter 20000, zero start, no
 * graphs, autotuned fill schedule, multigrid fill preconditioner, no
 * merging.
 * Returns NI_E_ARG on a null pointer. */
ni_status ni_params_default(ni_params* p);

/* Create a context on HIP device `device`; it owns a device workspace that
 * grows on demand and is freed by ni_destroy, and a second stream (default
 * priority) on which the small components are filled while the large ones
 * are solved on the caller's stream; every call joins it before it
 * returns.  *out is set to NULL on error. */
ni_status ni_create(ni_ctx** out, int device);
ni_status ni_destroy(ni_ctx* ctx);

/* Stream for all later work (a hipStream_t, e.g. torch's
 * torch.cuda.current_stream().cuda_stream); NULL selects the null stream. */
ni_status ni_set_stream(ni_ctx* ctx, void* hip_stream);

/* Whole path (Alg. 1): components, fill, relative scales (with optional
 * merging when params->freq_merging > 0).
 *   normals   device f32 [H][W][3], read only; NaN/Inf allowed off the mask
 *   mask      device u8  [H][W]; non-zero = valid pixel
 *   depth     device f32 [H][W] out: exp(z~) (perspective) or z~ (ortho),
 *             gauge: zero mean log-depth over every connected region of
 *             the pixel graph; NaN off the mask
 *   labels    device i32 [H][W] out: component id, ids numbered by
 *             ascending smallest raster index; -1 off the mask
 *   log_scale device f64 [cap] out: per-component log-scale s~_c in the
 *             same gauge as depth
 *   K         host out: number of components; if K > cap the call stops
 *             with NI_E_SHAPE after labelling (call again with cap >= K)
 *   rep       host out, may be NULL
 * H, W in [1, 32767], H*W <= 2^28. */
ni_status ni_integrate(ni_ctx* ctx, const float* normals, const uint8_t* mask,
                       int32_t H, int32_t W, const ni_camera* cam,
                       const ni_params* params, float* depth, int32_t* labels,
                       double* log_scale, int64_t cap, int32_t* K,
                       ni_report* rep);

/* Stage (a) alone: component labels (Sec. 3.3), same layout as above. */
ni_status ni_label(ni_ctx* ctx, const float* normals, const uint8_t* mask,
                   int32_t H, int32_t W, const ni_camera* cam,
                   const ni_params* params, int32_t* labels, int32_t* K,
                   ni_report* rep);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): stage (a)
 * as ni_label, with no allocation of any kind.  Its scratch (edge arrays,
 * union-find, counters; 28 MiB) is a static device array of the library,
 * one copy per GPU, held until the process ends; its address is looked up
 * when a context is created on the device.  Maps are limited to H, W <=
 * 4096 and H*W <= 2^20 (NI_E_SHAPE beyond).  The call clears what must
 * start at zero, writes labels / *K exactly as ni_label does, and blocks
 * for *K.  All calls on one GPU share the array: calls that overlap in
 * time on one GPU (several threads or streams) race and must not be
 * issued. */
ni_status ni_label_noalloc(ni_ctx* ctx, const float* normals, const uint8_t* mask,
                           int32_t H, int32_t W, const ni_camera* cam,
                           const ni_params* params, int32_t* labels, int32_t* K);

/* Stage (b) from given labels (Eq. 14-15): labels device i32 [H][W] in
 * (ids 0..K-1 on valid pixels, each component 4-connected through usable
 * edges, -1 off the mask); zfill device f32 [H][W] out: filled log-depth
 * (ortho: depth), zero mean per component, 0 off the mask. */
ni_status ni_fill(ni_ctx* ctx, const float* normals, const uint8_t* mask,
                  int32_t H, int32_t W, const ni_camera* cam,
                  const ni_params* params, const int32_t* labels, int32_t K,
                  float* zfill, ni_report* rep);

/* Stage (c) and output from given labels and fill (Eq. 16-19, Alg. 1):
 * zfill device f32 [H][W] in; depth / log_scale out as in ni_integrate
 * (cap >= K required). */
ni_status ni_irls(ni_ctx* ctx, const float* normals, const uint8_t* mask,
                  int32_t H, int32_t W, const ni_camera* cam,
                  const ni_params* params, const int32_t* labels, int32_t K,
                  const float* zfill, float* depth, double* log_scale,
                  int64_t cap, ni_report* rep);

/* One relative-scale iteration t (Sec. 3.4, Eq. 16-17; Alg. 1's loop
 * body) from given scales, a test hook that injects the oracle's state:
 * labels / zfill as for ni_irls; S_in device f64 [K] the scales before the
 * step; the weights of iteration t (uniform when t < align_iters) are
 * formed at z = zfill + S_in, the system is solved as in ni_integrate,
 * and the increment s^(t) (zero mean on every connected piece of the
 * weighted quotient graph) goes to s_out device f64 [K]; *energy (host)
 * gets E_t.  NI_E_NOTCONV if a solve round stopped at q_max_iter. */
ni_status ni_irls_step(ni_ctx* ctx, const float* normals, const uint8_t* mask,
                       int32_t H, int32_t W, const ni_camera* cam,
                       const ni_params* params, const int32_t* labels, int32_t K,
                       const float* zfill, const double* S_in, int32_t t,
                       double* s_out, double* energy, ni_report* rep);

/* ---------------------------------------------------------------------
 * Learned warm start (not in the paper): a 4-level U-Net (16-32-64-128
 * channels, 3x3 convolutions, BF16 activations and weights, FP32
 * accumulation on MFMA) maps (normal, mask, ray direction) to a log-depth
 * estimate; with params->warm_start = 1 the fill CG of every component
 * starts from it (centred per component; a start no better than zero is
 * dropped).  Weight blob format: "NIUNET01", int32 n, n FP32 parameters.
 * All model calls use the context's device and stream.
 * ------------------------------------------------------------------- */
int32_t ni_unet_param_count(void);
size_t ni_unet_blob_size(void);
/* fresh model, He-normal initialisation from a 64-bit seed */
ni_status ni_unet_init(ni_ctx* ctx, uint64_t seed);
/* load / save a weight blob (host memory of ni_unet_blob_size() bytes) */
ni_status ni_unet_load(ni_ctx* ctx, const void* blob, size_t nbytes);
ni_status ni_unet_save(ni_ctx* ctx, void* blob, size_t nbytes);
/* FP32 master parameters, host arrays of ni_unet_param_count() floats */
ni_status ni_unet_get_params(ni_ctx* ctx, float* host, int32_t n);
ni_status ni_unet_set_params(ni_ctx* ctx, const float* host, int32_t n);
/* log-depth estimate of a whole map: normals / mask as in ni_integrate,
 * out device f32 [H][W] */
ni_status ni_unet_predict(ni_ctx* ctx, const float* normals, const uint8_t* mask, int32_t H, int32_t W,
                          const ni_camera* cam, float* out);
/* forward on raw features: feat device f32 [B][H][W][6] (n, mask, tau_x,
 * tau_y), H and W multiples of 8; out device f32 [B][H][W] */
ni_status ni_unet_forward(ni_ctx* ctx, const float* feat, int32_t B, int32_t H, int32_t W, float* out);
/* after ni_unet_forward: gradient of sum(dout * out) w.r.t. the master
 * parameters; dout device f32 [B][H][W], grad device f32 [param_count] */
ni_status ni_unet_backward(ni_ctx* ctx, const float* dout, float* grad);
/* one Adam step (lr, beta 0.9 / 0.999) on B patches of S x S (S multiple
 * of 8): normals device f32 [B][S][S][3], mask device u8 [B][S][S], cams
 * host [B], target device f32 [B][S][S] (fill log-depth), labels device
 * i32 [B][S][S] with component ids unique across the batch in [0, ncomp)
 * (-1 off the mask); loss host out: per-component centred MSE */
ni_status ni_unet_train_step(ni_ctx* ctx, const float* normals, const uint8_t* mask, const ni_camera* cams,
                             const float* target, const int32_t* labels, int32_t ncomp, int32_t B, int32_t S,
                             float lr, double* loss);

const char* ni_status_str(ni_status s);
const char* ni_last_error(const ni_ctx* ctx);
int32_t ni_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NI_H */
