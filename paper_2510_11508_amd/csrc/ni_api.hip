// C ABI of libni: argument validation, workspace, stage orchestration.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ni.h"
#include "ni_common.h"

namespace nil {
// ni_setup.hip
hipError_t launch_setup(const float*, const uint8_t*, int, int, int, double, const double*, double, int,
                        uint8_t*, float*, float*, float*, int*, hipStream_t, uint8_t*, float*, float*);
hipError_t launch_inter_geom(const uint32_t*, int, int, int, const float*, int, double, const double*, double*,
                             double*, double*, hipStream_t);
hipError_t set_i32(int*, int, int, hipStream_t);
hipError_t ray_tables(int, int, double, double, double, double, double*, hipStream_t);
hipError_t grid_components(const uint8_t*, int, int, uint8_t, uint8_t, int*, int*, int*, int*, int*, int*,
                           hipStream_t, const uint8_t*, uint8_t, uint8_t);
// ni_fill.hip
int fill_small_cap();
int fill_chunk();
hipError_t check_labels(const int*, const uint8_t*, int, int, int*, hipStream_t);
hipError_t check_ids(const uint32_t*, int, int, int*, hipStream_t);
hipError_t fill_segments(const int*, int, int, int*, int*, int*, uint32_t*, uint32_t*, uint32_t*, uint32_t*,
                         uint32_t*, uint32_t*, int, int*, int*, int*, hipStream_t, int);
hipError_t fill_assemble(const uint32_t*, int, int, int, const int*, const uint8_t*, const float*, const float*,
                         const float*, const int*, double, double, float4*, float*, float*, hipStream_t);
hipError_t fill_tier_list(const int*, int, int, int*, int*, int*, int*, int*, hipStream_t);
hipError_t fill_chunks(const int*, int, int, int*, int*, int*, int*, hipStream_t);
hipError_t fill_chunk_table(const int*, const int*, const int*, int, int, int*, int*, int*, hipStream_t);
hipError_t fill_zero_grid(float*, int, hipStream_t);
hipError_t fill_gather_x0(const uint32_t*, int, const float*, float*, hipStream_t);
hipError_t fill_small(int, const int*, int, const int*, const float4*, const float*, const float*, const float*,
                      const uint32_t*, float*, double, int, int, int*, double*, int*, hipStream_t);

hipError_t large_init(const LargeArgs&, int, hipStream_t);
hipError_t large_iter(const LargeArgs&, int, hipStream_t);
hipError_t large_finish(const LargeArgs&, const uint32_t*, float*, hipStream_t);
hipError_t large_center(const LargeArgs&, hipStream_t);
hipError_t mg_count(int, const float4*, const uint32_t*, const int*, int*, int*, hipStream_t);
hipError_t mg_build(int, int, const float4*, const float*, const float*, const uint32_t*, const uint32_t*, const int*,
                    const int*, const int*, int*, double*, double*, int*, int*, double*, int*, int*, int*, double*,
                    double*, hipStream_t);
hipError_t mg_out(int, const uint32_t*, const int*, const double*, float*, hipStream_t);
hipError_t fill8_count(int, int, const uint32_t*, const uint32_t*, const int*, const int*, const uint8_t*,
                       const uint8_t*, int*, int*, hipStream_t);
hipError_t fill8_build(int, int, const uint32_t*, const uint32_t*, const int*, const int*, const uint8_t*,
                       const uint8_t*, const float*, const float* const*, const int*, double, double, double,
                       const int*, const int*, const float*, int*, double*, double*, int*, int*, double*, int*, int*,
                       int*, double*, double*, hipStream_t);
hipError_t fill8_out(int, int, const uint32_t*, const uint32_t*, const int*, const double*, double*, void*, float*,
                     hipStream_t);
// ni_quot.hip
hipError_t quot_inter_edges(const int*, const uint8_t*, const uint8_t*, int, int, int*, int*, int*, uint32_t*, int*,
                            hipStream_t, int);
hipError_t quot_sort_edges(uint32_t*, int, int, int, const int*, uint32_t*, uint32_t*, uint32_t*, uint32_t*,
                           uint32_t*, int*, int*, int*, int*, hipStream_t);
hipError_t quot_pairs(const uint32_t*, const int*, const int*, int, int, const int*, int, int*, int*, int*,
                      hipStream_t);
hipError_t quot_csr(const int*, const int*, int, int, uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint32_t*,
                    uint32_t*, int*, int*, int*, hipStream_t);
hipError_t quot_heavy_rows(const int*, int, int*, int*, int*, int*, int*, hipStream_t);

hipError_t irls_iteration(const IrlsArgs&, int, hipStream_t);
// ni_final.hip
hipError_t final_outputs(const int*, const float*, const double*, const int*, const uint32_t*, const uint32_t*,
                         const int*, const int*, int, int, int, int, int, double*, int*, double*, double*, float*,
                         double*, const FinalScratch&, hipStream_t);
// ni_unet.hip
hipError_t unet_predict(struct UnetModel*, const float*, const uint8_t*, int, int, const ni_camera*, float*,
                        void*, size_t, hipStream_t);
size_t unet_workspace_bytes(int, int);
int unet_load(struct UnetModel**, const void*, size_t, std::string*);
int unet_new(struct UnetModel**, uint64_t, std::string*);
void unet_free(struct UnetModel*);
int unet_param_count();
size_t unet_blob_size();
hipError_t unet_save(struct UnetModel*, void*);
hipError_t unet_get_params(struct UnetModel*, float*);
hipError_t unet_set_params(struct UnetModel*, const float*, hipStream_t);
hipError_t unet_forward_raw(struct UnetModel*, const float*, int, int, int, float*, hipStream_t);
hipError_t unet_backward_raw(struct UnetModel*, const float*, float*, hipStream_t);
hipError_t unet_train_step(struct UnetModel*, const float*, const uint8_t*, const ni_camera*, const float*,
                           const int*, int, int, int, float, double*, hipStream_t);
}  // namespace nil

namespace {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Fail {
  ni_status s;
};

}  // namespace

// Scratch of the allocation-free labelling entry point (ni_label_noalloc):
// one copy of this array per GPU, held until the process ends.  In host
// code its name is only a stand-in: the device address comes from
// hipGetSymbolAddress, looked up once per device when a context is
// created on it, and only that address is passed to kernels and copies.
constexpr int NOALLOC_MAX_SIDE = 4096;
constexpr long long NOALLOC_MAX_PX = 1ll << 20;
constexpr size_t NOALLOC_BYTES = (size_t)28 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_scratch_mu;
void* g_scratch[NOALLOC_MAX_DEV] = {};

// the device address of `scratch` on the current device (looked up once)
hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
  if (!g_scratch[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return hipSuccess;
}
}  // namespace

struct ni_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;  // small-component tiers, concurrent with the large solve
  std::string err;
  std::vector<Buf*> bufs;
  // grid
  Buf ebits, om_r, om_d, nt, parent, flag, scanv, pos, zgrid, tab, xwarm;
  Buf eb2, om_dr, om_dl;  // diagonal edges (8-connectivity)
  // compact / sort
  Buf key, val, skey, spix, ktmp, vtmp, kout2, cst, rhs, dinv, x, r, z, p0, p1, q, w0, w1, s0, s1;
  // components
  Buf comp_off, fsmall, flarge, nchunk, spos, lpos, cbase, small_list, large_list, cnt, done, iters, active,
      rho, bb, tol2, beta, rr, relres, S, qs, diag, qrhs, babs, psum, pcnt, qparent, csum, comp_rid;
  // the quotient nodes sorted by piece
  Buf pkey, pnode, pnode_in, pk_tmp, pv_tmp, pscan, pval, prun, fg, fv2;
  // chunks
  Buf chunk_comp, chunk_start, part;
  // edges / pairs
  Buf eidx_raw, eidx, ew, erho, pflag, ppos, pair_start, pair_lo, pair_hi, pW, pB, ent, ent_tmp, rowcnt,
      row_off, epart, rsum, rcnt, qcol, qw, qt0, qt1, eom, eta, etb;
  // merging
  Buf mgrp, mglab, mkey, mcode, mpa, mpb, mkeep, mrank;
  // fill multigrid: level-0 system of the large components
  Buf mg_deg, mg_pc, mg_row, mg_poff, mg_col, mg_w, mg_diag, mg_plo, mg_phi, mg_pw, mg_gy, mg_gx, mg_gc, mg_b, mg_x;
  // scratch
  Buf scan_tmp, misc, unet_ws;
  int* host = nullptr;  // pinned readback area (64 ints)
  hipEvent_t ev[16] = {};
  struct nil::UnetModel* unet = nullptr;
  void* noalloc = nullptr;       // device address of `scratch` on this device
  nil::Amg* amg = nullptr;       // quotient systems
  nil::Amg* amg_fill = nullptr;  // fill of the large components
  // autotuned schedule of the large fill path: shortest chunk per block,
  // and the map size class it was tuned for
  int fill_chunk = 0, fill_split = 0, fill_chunk_key = -1;
  float tune_ms[8] = {};


  ni_ctx() {
    Buf* all[] = {&ebits, &om_r, &om_d, &nt, &eb2, &om_dr, &om_dl, &parent, &flag, &scanv, &pos, &zgrid, &tab, &xwarm, &key, &val,
                  &skey, &spix, &ktmp, &vtmp, &kout2, &cst, &rhs, &dinv, &x, &r, &z, &p0,
                  &p1, &q, &w0, &w1, &s0, &s1, &comp_off, &fsmall, &flarge, &nchunk, &spos, &lpos, &cbase, &small_list, &large_list,
                  &cnt, &done, &iters, &active, &rho, &bb, &tol2, &beta, &rr, &relres, &S, &qs,
                  &diag, &qrhs, &babs, &psum, &pcnt, &qparent, &csum, &comp_rid, &pkey, &pnode, &pnode_in,
                  &pk_tmp, &pv_tmp, &pscan, &pval, &prun, &fg, &fv2,
                  &chunk_comp, &chunk_start, &part, &eidx_raw, &eidx, &ew, &erho, &pflag, &ppos, &pair_start,
                  &pair_lo, &pair_hi, &pW, &pB, &ent, &ent_tmp, &rowcnt, &row_off, &epart, &rsum,
                  &rcnt, &qcol, &qw, &qt0, &qt1, &eom, &eta, &etb, &mgrp, &mglab, &mkey, &mcode, &mpa,
                  &mpb, &mkeep, &mrank, &mg_deg, &mg_pc, &mg_row,
                  &mg_poff, &mg_col, &mg_w, &mg_diag, &mg_plo, &mg_phi, &mg_pw, &mg_gy, &mg_gx, &mg_gc, &mg_b,
                  &mg_x, &scan_tmp, &misc, &unet_ws};
    bufs.assign(std::begin(all), std::end(all));
  }
};

namespace {

// misc device area layout (ints unless stated)
enum {
  M_COUNT = 0,    // [0..7] counters written by scans
  M_ERR = 8,      // non-finite flag
  M_STATS = 12,   // [12..15] fill stats
  M_ACTIVE = 16,  // 2 ints (fill: components still iterating, by launch parity)
  M_QFLAG = 24,   // 2 ints (quotient: still iterating, by launch parity)
  M_WMAX = 32,    // u64 (8-byte aligned)
  M_ENERGY = 64,  // NI_MAX_IRLS doubles (8-byte aligned)
  M_QITERS = 64 + 2 * NI_MAX_IRLS,   // quotient iterations, first round
  M_QITERS2 = 64 + 3 * NI_MAX_IRLS,  // quotient iterations, refinement round
  M_TOTAL = 64 + 4 * NI_MAX_IRLS
};

void check(ni_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();
    throw Fail{e == hipErrorOutOfMemory ? NI_E_NOMEM : NI_E_DEVICE};
  }
}

template <class T>
T* ensure(ni_ctx* c, Buf& b, size_t count) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  bytes = (bytes + 255) & ~size_t(255);
  if (b.cap < bytes) {
    // grow by a quarter at least, so that sizes creeping up from call to
    // call do not reallocate every time
    const size_t want = (std::max(bytes, b.cap + b.cap / 4) + 255) & ~size_t(255);
    if (b.p) check(c, hipFree(b.p), "hipFree");
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
      b.p = nullptr;
      check(c, e, "hipMalloc");
    }
    b.cap = want;
  }
  return (T*)b.p;
}

template <class T>
T* ptr(Buf& b) {
  return (T*)b.p;
}

int* misc(ni_ctx* c) { return ptr<int>(c->misc); }

void readback(ni_ctx* c, const void* dev, size_t bytes, void* host) {
  check(c, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream), "readback");
  check(c, hipStreamSynchronize(c->stream), "stream sync");
}

float ev_ms(ni_ctx* c, int a, int b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) return 0.f;
  return ms;
}

void mark(ni_ctx* c, int i) { check(c, hipEventRecord(c->ev[i], c->stream), "event"); }

struct Problem {
  const float* normals;
  const uint8_t* mask;
  int H, W, P;
  ni_camera cam;
  ni_params prm;
};

ni_status validate(ni_ctx* c, const float* normals, const uint8_t* mask, int32_t H, int32_t W,
                   const ni_camera* cam, const ni_params* prm, Problem* pb) {
  if (!c) return NI_E_ARG;
  c->err.clear();
  auto bad = [&](const char* m) {
    c->err = m;
    return NI_E_ARG;
  };
  if (!normals || !mask || !cam || !prm) return bad("null input pointer");
  if (H < 1 || W < 1 || H > 32767 || W > 32767 || (long long)H * W > (1ll << 28)) return bad("H, W out of range");
  if (cam->proj != NI_ORTHO && cam->proj != NI_PERSP) return bad("camera proj must be NI_ORTHO or NI_PERSP");
  if (cam->proj == NI_PERSP && !(cam->fx > 0 && cam->fy > 0 && isfinite(cam->cx) && isfinite(cam->cy)))
    return bad("perspective camera needs fx, fy > 0 and finite cx, cy");
  if (cam->proj == NI_ORTHO && !(cam->pixel_pitch > 0)) return bad("orthographic camera needs pixel_pitch > 0");
  if (prm->connectivity != 4 && prm->connectivity != 8) return bad("connectivity must be 4 or 8");
  if (prm->irls_iters < 1 || prm->irls_iters > NI_MAX_IRLS) return bad("irls_iters out of range");
  if (prm->align_iters < 0) return bad("align_iters < 0");
  if (!(prm->cg_rtol > 0) || prm->cg_max_iter < 1 || !(prm->q_rtol > 0) || prm->q_max_iter < 1 ||
      !(prm->q_rtol_refine > 0 && prm->q_rtol_refine < 1))
    return bad("bad CG tolerance / iteration cap");
  if (!(prm->out_L > 0 && prm->out_U > prm->out_L)) return bad("need 0 < out_L < out_U");
  if (prm->outlier_mode < 0 || prm->outlier_mode > 2) return bad("outlier_mode must be 0, 1 or 2");
  if (!(prm->w_cut_rel >= 0 && prm->w_cut_rel < 1)) return bad("w_cut_rel must be in [0, 1)");
  if (prm->freq_merging < 0) return bad("freq_merging must be >= 0");
  if (prm->variant != 0 && prm->variant != 1) return bad("variant must be 0 or 1");
  if (!(prm->bini_k > 0)) return bad("bini_k must be > 0");
  if (prm->fill_chunk != 0 && prm->fill_chunk != 512 && prm->fill_chunk != 1024 && prm->fill_chunk != 2048 &&
      prm->fill_chunk != 4096)
    return bad("fill_chunk must be 0, 512, 1024, 2048 or 4096");
  if (prm->fill_split != 0 && prm->fill_split != 1) return bad("fill_split must be 0 or 1");
  if (prm->fill_precond != 0 && prm->fill_precond != 1) return bad("fill_precond must be 0 or 1");
  if (prm->fill_mg_maxit < 0) return bad("fill_mg_maxit must be >= 0");
  if (prm->warm_start && !c->unet) {
    c->err = "warm_start needs a model (ni_unet_load)";
    return NI_E_MODEL;
  }
  pb->normals = normals;
  pb->mask = mask;
  pb->H = H;
  pb->W = W;
  pb->P = H * W;
  pb->cam = *cam;
  pb->prm = *prm;
  if (prm->variant == 1) {
    // the pixel-level log-depth baseline (ND form): every pixel its own
    // node, no alignment phase, no merging; outlier weights from the second
    // iteration (set where the step parameters are formed)
    pb->prm.theta_c_deg = 0.0;
    pb->prm.align_iters = 0;
    pb->prm.freq_merging = 0;
  }
  return NI_OK;
}

void ensure_misc(ni_ctx* c) {
  if (!c->misc.p) {
    ensure<int>(c, c->misc, M_TOTAL);
    check(c, hipMemsetAsync(c->misc.p, 0, M_TOTAL * sizeof(int), c->stream), "memset");
  }
}

void ensure_scan(ni_ctx* c, size_t n) {
  size_t a = nil::scan_tmp_ints((int)std::min<size_t>(n, 1u << 30));
  size_t b = nil::radix_tmp_ints((int)std::min<size_t>(n, 1u << 30));
  ensure<int>(c, c->scan_tmp, std::max(a, b));
}

// edge directions per pixel: 2 (right, down), or 4 with the diagonals
size_t ndirs(const Problem& pb) { return pb.prm.connectivity == 8 ? 4 : 2; }

// diagonal edge bits (null under 4-connectivity)
uint8_t* eb2(ni_ctx* c, const Problem& pb) { return pb.prm.connectivity == 8 ? ptr<uint8_t>(c->eb2) : nullptr; }

// ----------------------------------------------------------------- stages
void stage_setup(ni_ctx* c, const Problem& pb) {
  const int H = pb.H, W = pb.W, P = pb.P;
  ensure_misc(c);
  ensure<uint8_t>(c, c->ebits, P);
  ensure<float>(c, c->om_r, P);
  ensure<float>(c, c->om_d, P);
  ensure<float>(c, c->nt, P);
  ensure<int>(c, c->parent, P);
  const size_t nd = ndirs(pb);
  ensure<int>(c, c->flag, nd * P);
  ensure<int>(c, c->scanv, nd * P);
  ensure<int>(c, c->pos, P);
  ensure<float>(c, c->zgrid, P);
  ensure_scan(c, nd * P);
  if (nd == 4) {
    ensure<uint8_t>(c, c->eb2, P);
    ensure<float>(c, c->om_dr, P);
    ensure<float>(c, c->om_dl, P);
  }
  // ray tables in FP64 on the host: tau = ((u - cx)/fx, (v - cy)/fy, 1) at
  // pixel centres and at the midpoints u + 1/2, v + 1/2
  std::vector<double> t(2 * (size_t)W + 2 * (size_t)H, 0.0);
  if (pb.cam.proj == NI_PERSP) {
    for (int u = 0; u < W; ++u) {
      t[u] = ((double)u - pb.cam.cx) / pb.cam.fx;
      t[W + H + u] = (((double)u + 0.5) - pb.cam.cx) / pb.cam.fx;
    }
    for (int v = 0; v < H; ++v) {
      t[W + v] = ((double)v - pb.cam.cy) / pb.cam.fy;
      t[2 * W + H + v] = (((double)v + 0.5) - pb.cam.cy) / pb.cam.fy;
    }
  }
  double* tab = ensure<double>(c, c->tab, t.size());
  check(c, hipMemcpyAsync(tab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, c->stream), "H2D");
  check(c, hipStreamSynchronize(c->stream), "sync");  // t is pageable and goes out of scope
  const double th = pb.prm.theta_c_deg;
  const int use_sim = th > 0 ? 1 : 0;
  const double cth = use_sim ? cos(th * M_PI / 180.0) : 2.0;
  check(c, hipMemsetAsync(misc(c) + M_ERR, 0, sizeof(int), c->stream), "memset");
  check(c,
        nil::launch_setup(pb.normals, pb.mask, H, W, pb.cam.proj == NI_PERSP, pb.cam.pixel_pitch, tab, cth, use_sim,
                          ptr<uint8_t>(c->ebits), ptr<float>(c->om_r), ptr<float>(c->om_d), ptr<float>(c->nt),
                          misc(c) + M_ERR, c->stream, eb2(c, pb), nd == 4 ? ptr<float>(c->om_dr) : nullptr,
                          nd == 4 ? ptr<float>(c->om_dl) : nullptr),
        "setup");
}

// components over similar edges -> labels; returns K
int stage_label(ni_ctx* c, const Problem& pb, int32_t* labels) {
  check(c,
        nil::grid_components(ptr<uint8_t>(c->ebits), pb.H, pb.W, EB_SR, EB_SD, ptr<int>(c->parent),
                             ptr<int>(c->flag), ptr<int>(c->scanv), labels, misc(c) + M_COUNT,
                             ptr<int>(c->scan_tmp), c->stream, eb2(c, pb), EB2_SDR, EB2_SDL),
        "label");
  readback(c, misc(c), 16 * sizeof(int), c->host);
  if (c->host[M_ERR]) {
    c->err = "non-finite normal inside the mask";
    throw Fail{NI_E_NONFINITE};
  }
  return c->host[M_COUNT];
}

struct Seg {
  int N = 0, K = 0;
};

}  // namespace

// The segments stage needs the valid count before the compact buffers can be
// sized, so it is split around one readback.
namespace {

Seg build_segments(ni_ctx* c, const Problem& pb, const int32_t* labels, int K, bool user_labels) {
  const int P = pb.P;
  Seg sg;
  sg.K = K;
  int* cntd = misc(c) + M_COUNT;
  int* bad = misc(c) + M_ERR + 1;
  if (user_labels) {
    check(c, hipMemsetAsync(bad, 0, sizeof(int), c->stream), "memset");
    check(c, nil::check_labels(labels, ptr<uint8_t>(c->ebits), P, K, bad, c->stream), "check labels");
    readback(c, bad, sizeof(int), c->host);
    if (c->host[0]) {
      c->err = "labels must hold ids in [0, K) on the valid pixels and -1 elsewhere";
      throw Fail{NI_E_ARG};
    }
  }
  // valid count first (flags + scan), then size the compact buffers
  ensure<uint32_t>(c, c->key, P);
  ensure<uint32_t>(c, c->val, P);
  check(c,
        nil::fill_segments(labels, P, K, ptr<int>(c->flag), ptr<int>(c->scanv), cntd, ptr<uint32_t>(c->key),
                           ptr<uint32_t>(c->val), nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr,
                           ptr<int>(c->scan_tmp), c->stream, 0),
        "segments/compact");
  readback(c, cntd, sizeof(int), c->host);
  const int N = c->host[0];
  sg.N = N;
  ensure<uint32_t>(c, c->skey, N);
  ensure<uint32_t>(c, c->spix, N);
  ensure<uint32_t>(c, c->ktmp, N);
  ensure<uint32_t>(c, c->vtmp, N);
  ensure<int>(c, c->comp_off, (size_t)K + 1);
  ensure_scan(c, std::max<size_t>(ndirs(pb) * P, N));
  check(c,
        nil::fill_segments(labels, P, K, nullptr, nullptr, nullptr, ptr<uint32_t>(c->key), ptr<uint32_t>(c->val),
                           ptr<uint32_t>(c->skey), ptr<uint32_t>(c->spix), ptr<uint32_t>(c->ktmp),
                           ptr<uint32_t>(c->vtmp), N, ptr<int>(c->comp_off), ptr<int>(c->pos),
                           ptr<int>(c->scan_tmp), c->stream, 1),
        "segments/sort");
  if (N == 0 && K >= 0) check(c, hipMemsetAsync(ptr<int>(c->comp_off), 0, sizeof(int) * (K + 1), c->stream), "memset");
  if (user_labels) {
    check(c, nil::check_ids(ptr<uint32_t>(c->skey), N, K, bad, c->stream), "check ids");
    readback(c, bad, sizeof(int), c->host);
    if (c->host[0] || (N == 0 && K != 0)) {
      c->err = "every component id 0..K-1 must label at least one valid pixel";
      throw Fail{NI_E_ARG};
    }
  }
  return sg;
}

// Fill under 8-connectivity: every component of two or more pixels in one
// multigrid-preconditioned CG over their block-diagonal system, assembled
// in FP64 from the edge bits; zero mean per component.
void stage_fill8(ni_ctx* c, const Problem& pb, const int32_t* labels, const Seg& sg, float* zout, ni_report* rep) {
  const int P = pb.P, W = pb.W, N = sg.N, K = sg.K;
  const bool persp = pb.cam.proj == NI_PERSP;
  const size_t K1 = (size_t)K + 1;
  const uint32_t* cpix = ptr<uint32_t>(c->spix);
  const uint32_t* skey = ptr<uint32_t>(c->skey);
  const int* comp_off = ptr<int>(c->comp_off);
  int* iters = ensure<int>(c, c->iters, K1);
  double* rr = ensure<double>(c, c->rr, K1);
  double* bb = ensure<double>(c, c->bb, K1);
  int* list = ensure<int>(c, c->small_list, K1);
  int* tflag = ensure<int>(c, c->fsmall, K1);
  int* tpos = ensure<int>(c, c->spos, K1);
  float* x = ensure<float>(c, c->x, N);
  int* cntd = misc(c) + M_COUNT;
  int* stats = misc(c) + M_STATS;
  mark(c, 3);
  check(c, nil::fill_zero_grid(zout, P, c->stream), "zero");
  check(c, hipMemsetAsync(iters, 0, K1 * sizeof(int), c->stream), "memset");
  check(c, hipMemsetAsync(rr, 0, K1 * sizeof(double), c->stream), "memset");
  check(c, hipMemsetAsync(stats, 0, 4 * sizeof(int), c->stream), "memset");
  check(c, nil::fill_tier_list(comp_off, K, 5, tflag, tpos, list, cntd, ptr<int>(c->scan_tmp), c->stream), "list");
  readback(c, cntd, sizeof(int), c->host);
  const int nl = c->host[0];
  const int warm = pb.prm.warm_start ? 1 : 0;
  mark(c, 4);
  const float* xw = nullptr;
  if (warm) {
    float* xg = ensure<float>(c, c->xwarm, P);
    size_t wsb = nil::unet_workspace_bytes(pb.H, pb.W);
    void* ws = ensure<uint8_t>(c, c->unet_ws, wsb);
    check(c, nil::unet_predict(c->unet, pb.normals, pb.mask, pb.H, pb.W, &pb.cam, xg, ws, wsb, c->stream), "unet");
    xw = xg;
  }
  check(c, nil::fill_gather_x0(cpix, N, xw, x, c->stream), "gather");
  mark(c, 5);
  int its = 0, levels = 0;
  double mg_bytes = 0.0;
  if (nl > 0) {
    int* deg = ensure<int>(c, c->mg_deg, N);
    int* npair = ensure<int>(c, c->mg_pc, N);
    int* row_off = ensure<int>(c, c->mg_row, (size_t)N + 1);
    int* poff = ensure<int>(c, c->mg_poff, (size_t)N + 1);
    check(c, nil::fill8_count(N, W, cpix, skey, comp_off, labels, ptr<uint8_t>(c->ebits), eb2(c, pb), deg, npair,
                              c->stream),
          "count");
    check(c, nil::scan_exclusive_i32(deg, row_off, N, row_off + N, ptr<int>(c->scan_tmp), c->stream), "scan");
    check(c, nil::scan_exclusive_i32(npair, poff, N, poff + N, ptr<int>(c->scan_tmp), c->stream), "scan");
    readback(c, row_off + N, sizeof(int), c->host);
    const int nnz = c->host[0];
    readback(c, poff + N, sizeof(int), c->host);
    const int npr = c->host[0];
    if (nnz != 2 * npr) {
      c->err = "fill: inconsistent 8-connected level-0 graph";
      throw Fail{NI_E_DEVICE};
    }
    int* col = ensure<int>(c, c->mg_col, nnz);
    double* w = ensure<double>(c, c->mg_w, nnz);
    double* dg = ensure<double>(c, c->mg_diag, N);
    int* plo = ensure<int>(c, c->mg_plo, npr);
    int* phi = ensure<int>(c, c->mg_phi, npr);
    double* pw = ensure<double>(c, c->mg_pw, npr);
    int* gy = ensure<int>(c, c->mg_gy, N);
    int* gx = ensure<int>(c, c->mg_gx, N);
    int* gc = ensure<int>(c, c->mg_gc, N);
    double* b64 = ensure<double>(c, c->mg_b, N);
    double* x64 = ensure<double>(c, c->mg_x, N);
    const float* om[4] = {ptr<float>(c->om_r), ptr<float>(c->om_d), ptr<float>(c->om_dr), ptr<float>(c->om_dl)};
    const double g2fx = persp ? pb.cam.fx * pb.cam.fx : 1.0;
    const double g2fy = persp ? pb.cam.fy * pb.cam.fy : 1.0;
    const double g2fd = persp ? pb.cam.fx * pb.cam.fy : 1.0;
    check(c,
          nil::fill8_build(N, W, cpix, skey, comp_off, labels, ptr<uint8_t>(c->ebits), eb2(c, pb), ptr<float>(c->nt),
                           om, ptr<int>(c->pos), g2fx, g2fy, g2fd, row_off, poff, x, col, w, dg, plo, phi, pw, gy, gx,
                           gc, b64, x64, c->stream),
          "assemble");
    if (!c->amg_fill) c->amg_fill = nil::amg_new();
    check(c, nil::amg_build(c->amg_fill, N, npr, row_off, col, w, dg, plo, phi, pw, c->stream, gy, gx, gc, K, W,
                            pb.H),
          "mg hierarchy");
    nil::amg_set_corr(c->amg_fill, 1.8);
    check(c, nil::amg_update(c->amg_fill, w, dg, pw, c->stream), "mg values");
    mark(c, 12);
    check(c,
          nil::amg_fill_solve(c->amg_fill, gc, skey, list, nl, K, b64, x64, pb.prm.cg_rtol, pb.prm.cg_max_iter, warm, rr,
                              bb, iters, stats, c->host, &its, c->stream),
          "mg solve");
    mark(c, 13);
    double* csum = ensure<double>(c, c->csum, K1);
    void* rtmp = ensure<uint8_t>(c, c->prun, nil::run_sums_tmp_bytes(N));
    check(c, nil::fill8_out(N, K, cpix, skey, comp_off, x64, csum, rtmp, zout, c->stream), "out");
    levels = nil::amg_levels(c->amg_fill);
  } else {
    mark(c, 12);
    mark(c, 13);
  }
  mark(c, 15);
  readback(c, stats, 4 * sizeof(int), c->host);
  const int notconv = c->host[0], fallbacks = c->host[1];
  if (rep) {
    std::vector<int> it(K), off(K1);
    std::vector<double> hrr(K), hbb(K);
    if (K > 0) {
      check(c, hipMemcpyAsync(it.data(), iters, K * sizeof(int), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipMemcpyAsync(off.data(), comp_off, K1 * sizeof(int), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipMemcpyAsync(hrr.data(), rr, K * sizeof(double), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipMemcpyAsync(hbb.data(), bb, K * sizeof(double), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipStreamSynchronize(c->stream), "sync");
    }
    long long pxit = 0, nsys = 0;
    int itmax = 0;
    double rmax = 0.0;
    for (int k = 0; k < K; ++k) {
      const int n = off[k + 1] - off[k];
      if (n < 2) continue;
      nsys += n;
      pxit += (long long)n * it[k];
      itmax = std::max(itmax, it[k]);
      rmax = std::max(rmax, hbb[k] > 0 ? sqrt(hrr[k] / hbb[k]) : 0.0);
    }
    if (nl > 0) mg_bytes = nil::amg_fill_bytes(c->amg_fill, nsys);
    rep->fill_large_px = nsys;
    rep->fill_px_iters = pxit;
    rep->fill_large_px_iters = pxit;
    rep->fill_iters_max = itmax;
    rep->fill_max_relres = rmax;
    rep->n_small = 0;
    rep->n_large = nl;
    rep->fill_notconv = notconv;
    rep->fill_large_launches = its;
    rep->warm_fallbacks = fallbacks;
    rep->ms_assemble = ev_ms(c, 5, 12);
    rep->ms_warm = ev_ms(c, 4, 5);
    rep->ms_fill_small = 0.f;
    rep->ms_fill_large = ev_ms(c, 12, 15);
    rep->ms_large_kernel = ev_ms(c, 12, 13);
    rep->fill_chunk = 0;
    rep->fill_split = 0;
    rep->fill_mg_levels = levels;
    rep->ms_fill_mg_build = ev_ms(c, 5, 12);
    rep->fill_mg_bytes = mg_bytes;
    rep->fill_mg_fallback = 0;
  }
  if (notconv > 0) {
    c->err = std::to_string(notconv) + " component(s) hit cg_max_iter";
    throw Fail{NI_E_NOTCONV};
  }
}

void stage_fill(ni_ctx* c, const Problem& pb, const int32_t* labels, const Seg& sg, float* zout,
                ni_report* rep) {
  if (pb.prm.connectivity == 8) {
    stage_fill8(c, pb, labels, sg, zout, rep);
    return;
  }
  const int P = pb.P, W = pb.W, N = sg.N, K = sg.K;
  const bool persp = pb.cam.proj == NI_PERSP;
  const double g2fx = persp ? pb.cam.fx * pb.cam.fx : 1.0;
  const double g2fy = persp ? pb.cam.fy * pb.cam.fy : 1.0;
  float4* cst = ensure<float4>(c, c->cst, N);  // stencil: w_right, w_down, w_up, packed offsets
  float* rhs = ensure<float>(c, c->rhs, N);
  float* dinv = ensure<float>(c, c->dinv, N);
  float* x = ensure<float>(c, c->x, N);
  const uint32_t* cpix = ptr<uint32_t>(c->spix);
  const int* comp_off = ptr<int>(c->comp_off);
  mark(c, 3);
  check(c,
        nil::fill_assemble(cpix, N, W, P, labels, ptr<uint8_t>(c->ebits), ptr<float>(c->nt), ptr<float>(c->om_r),
                           ptr<float>(c->om_d), ptr<int>(c->pos), g2fx, g2fy, cst, rhs, dinv, c->stream),
        "assemble");
  size_t K1 = (size_t)K + 1;
  int* tflag = ensure<int>(c, c->fsmall, K1);
  int* tpos = ensure<int>(c, c->spos, K1);
  int* lists = ensure<int>(c, c->small_list, 4 * K1);
  int* nchunk = ensure<int>(c, c->nchunk, K1);
  int* cbase = ensure<int>(c, c->cbase, K1);
  int* iters = ensure<int>(c, c->iters, K1);
  double* relres = ensure<double>(c, c->relres, K1);
  int* cntd = misc(c) + M_COUNT;
  for (int t = 1; t <= 4; ++t)
    check(c, nil::fill_tier_list(comp_off, K, t, tflag, tpos, lists + (t - 1) * K1, cntd + (t - 1),
                                 ptr<int>(c->scan_tmp), c->stream),
          "tier lists");
  readback(c, cntd, 4 * sizeof(int), c->host);
  int ntier[4] = {c->host[0], c->host[1], c->host[2], c->host[3]};
  const int n_large = ntier[3];
  double* rr = ensure<double>(c, c->rr, K1);
  double* bb = ensure<double>(c, c->bb, K1);
  // chunk table of the large components for chunk length `len`
  int n_chunks = 0;
  int *chunk_comp = nullptr, *chunk_start = nullptr, *chunk_end = nullptr;
  auto chunks = [&](int len) {
    check(c, nil::fill_chunks(comp_off, K, len, nchunk, cbase, cntd + 4, ptr<int>(c->scan_tmp), c->stream),
          "chunks");
    readback(c, cntd + 4, sizeof(int), c->host);
    n_chunks = c->host[0];
    chunk_comp = ensure<int>(c, c->chunk_comp, n_chunks);
    chunk_start = ensure<int>(c, c->chunk_start, n_chunks);
    chunk_end = ensure<int>(c, c->large_list, n_chunks);
    check(c, nil::fill_chunk_table(comp_off, nchunk, cbase, K, len, chunk_comp, chunk_start, chunk_end, c->stream),
          "chunk table");
  };
  auto large_args = [&]() {
    nil::LargeArgs a;
    a.comp_off = comp_off; a.cbase = cbase; a.nchunk = nchunk; a.chunk_comp = chunk_comp;
    a.chunk_start = chunk_start; a.chunk_end = chunk_end;
    a.part = ensure<double>(c, c->part, 2 * 4 * (size_t)n_chunks);
    a.gam = ensure<double>(c, c->rho, 2 * K1);
    a.tol2 = ensure<double>(c, c->tol2, K1);
    a.rr = rr; a.bb = bb; a.iters = iters;
    a.active = misc(c) + M_ACTIVE; a.stats = misc(c) + M_STATS;
    a.cst = cst; a.rhs = rhs; a.dinv = dinv;
    a.x = x;
    a.p = ensure<float>(c, c->p0, N);
    a.r0 = ensure<float>(c, c->r, N);
    a.r1 = ensure<float>(c, c->z, N);
    a.w0 = ensure<float>(c, c->w0, N);
    a.w1 = ensure<float>(c, c->w1, N);
    a.s0 = ensure<float>(c, c->s0, N);
    a.s1 = ensure<float>(c, c->s1, N);
    a.nchunks = n_chunks; a.K = K; a.rtol = pb.prm.cg_rtol; a.maxit = pb.prm.cg_max_iter;
    a.split = c->fill_split;
    return a;
  };
  // Autotuner: the first time a map of this size class reaches the large
  // path, every candidate schedule (chunk length x two- or three-launch
  // iteration) runs a few CG iterations from a zero start and the fastest
  // per iteration is kept for the context.  The probe's vectors are reset
  // before the real solve.
  int key = 0;
  while ((1ll << key) < (long long)N) ++key;
  const bool mg = n_large > 0 && pb.prm.fill_precond == 1;
  if (mg) {
    // the multigrid path does not use the chunked schedule (the chunk table
    // only serves the final centring)
  } else if (n_large > 0 && pb.prm.fill_chunk > 0) {
    // a fixed schedule; the next autotuned call tunes afresh
    c->fill_chunk = pb.prm.fill_chunk;
    c->fill_split = pb.prm.fill_split;
    c->fill_chunk_key = -1;
  } else if (n_large > 0 && c->fill_chunk_key != key) {
    const int cand[4] = {512, 1024, 2048, 4096};
    const int probe = 8;
    float best = 1e30f;
    int pick = cand[2], pick_split = 0;
    for (int k = 0; k < 8; ++k) {
      chunks(cand[k & 3]);
      c->fill_split = k >> 2;
      nil::LargeArgs a = large_args();
      check(c, nil::fill_gather_x0(cpix, N, nullptr, x, c->stream), "gather");
      check(c, hipMemsetAsync(a.active, 0, 2 * sizeof(int), c->stream), "memset");
      check(c, nil::large_init(a, 0, c->stream), "large init");
      mark(c, 12);
      for (int it = 0; it < probe; ++it) check(c, nil::large_iter(a, it, c->stream), "large iter");
      mark(c, 13);
      check(c, hipStreamSynchronize(c->stream), "sync");
      const float ms = ev_ms(c, 12, 13);
      c->tune_ms[k] = ms;
      if (ms < best) {
        best = ms;
        pick = cand[k & 3];
        pick_split = k >> 2;
      }
    }
    c->fill_chunk = pick;
    c->fill_split = pick_split;
    c->fill_chunk_key = key;
  }
  chunks(c->fill_chunk);
  check(c, hipMemsetAsync(iters, 0, K1 * sizeof(int), c->stream), "memset");
  check(c, hipMemsetAsync(relres, 0, K1 * sizeof(double), c->stream), "memset");
  check(c, hipMemsetAsync(misc(c) + M_STATS, 0, 4 * sizeof(int), c->stream), "memset");
  check(c, nil::fill_zero_grid(zout, P, c->stream), "zero");
  const int warm = pb.prm.warm_start ? 1 : 0;
  mark(c, 4);
  const float* xw = nullptr;
  if (warm) {
    float* xg = ensure<float>(c, c->xwarm, P);
    size_t wsb = nil::unet_workspace_bytes(pb.H, pb.W);
    void* ws = ensure<uint8_t>(c, c->unet_ws, wsb);
    check(c, nil::unet_predict(c->unet, pb.normals, pb.mask, pb.H, pb.W, &pb.cam, xg, ws, wsb, c->stream), "unet");
    xw = xg;
  }
  check(c, nil::fill_gather_x0(cpix, N, xw, x, c->stream), "gather");
  // the small components run on a side stream while the large ones are
  // solved here: they touch disjoint pixels, components and counters
  // (the large solve counts into M_STATS + 2 .. 3); joined before the end
  mark(c, 5);
  check(c, hipStreamWaitEvent(c->side, c->ev[5], 0), "fork");
  for (int t = 1; t <= 3; ++t)
    check(c, nil::fill_small(t, lists + (t - 1) * K1, ntier[t - 1], comp_off, cst, rhs, dinv, x,
                             cpix, zout, pb.prm.cg_rtol, pb.prm.cg_max_iter, warm, iters, relres, misc(c) + M_STATS,
                             c->side),
          "fill small");
  check(c, hipEventRecord(c->ev[6], c->side), "event");
  int launches = 0, mg_levels = 0, mg_fallback = 0;
  bool jacobi = n_large > 0 && !mg;
  // iteration cap of the multigrid solve (it needs tens); a stall beyond it
  // falls back to the Jacobi path with the caller's cap
  const int mg_maxit = std::min(pb.prm.cg_max_iter, pb.prm.fill_mg_maxit > 0 ? pb.prm.fill_mg_maxit : 2000);
  float large_kernel_ms = 0.f, mg_build_ms = 0.f;
  double mg_bytes = 0.0;
  if (mg) {
    // one multigrid-preconditioned CG over all large components together
    nil::LargeArgs a = large_args();
    if (warm) check(c, nil::large_center(a, c->stream), "centre start");
    mark(c, 14);
    int* deg = ensure<int>(c, c->mg_deg, N);
    int* npair = ensure<int>(c, c->mg_pc, N);
    int* row_off = ensure<int>(c, c->mg_row, (size_t)N + 1);
    int* poff = ensure<int>(c, c->mg_poff, (size_t)N + 1);
    check(c, nil::mg_count(N, cst, ptr<uint32_t>(c->skey), comp_off, deg, npair, c->stream), "mg count");
    check(c, nil::scan_exclusive_i32(deg, row_off, N, row_off + N, ptr<int>(c->scan_tmp), c->stream), "scan");
    check(c, nil::scan_exclusive_i32(npair, poff, N, poff + N, ptr<int>(c->scan_tmp), c->stream), "scan");
    readback(c, row_off + N, sizeof(int), c->host);
    const int nnz = c->host[0];
    readback(c, poff + N, sizeof(int), c->host);
    const int npr = c->host[0];
    if (nnz != 2 * npr) {
      c->err = "fill multigrid: inconsistent level-0 graph";
      throw Fail{NI_E_DEVICE};
    }
    int* col = ensure<int>(c, c->mg_col, nnz);
    double* w = ensure<double>(c, c->mg_w, nnz);
    double* dg = ensure<double>(c, c->mg_diag, N);
    int* plo = ensure<int>(c, c->mg_plo, npr);
    int* phi = ensure<int>(c, c->mg_phi, npr);
    double* pw = ensure<double>(c, c->mg_pw, npr);
    int* gy = ensure<int>(c, c->mg_gy, N);
    int* gx = ensure<int>(c, c->mg_gx, N);
    int* gc = ensure<int>(c, c->mg_gc, N);
    double* b64 = ensure<double>(c, c->mg_b, N);
    double* x64 = ensure<double>(c, c->mg_x, N);
    check(c,
          nil::mg_build(N, W, cst, rhs, x, cpix, ptr<uint32_t>(c->skey), comp_off, row_off, poff, col, w, dg, plo,
                        phi, pw, gy, gx, gc, b64, x64, c->stream),
          "mg build");
    if (!c->amg_fill) c->amg_fill = nil::amg_new();
    check(c, nil::amg_build(c->amg_fill, N, npr, row_off, col, w, dg, plo, phi, pw, c->stream, gy, gx, gc, K, W,
                            pb.H),
          "mg hierarchy");
    nil::amg_set_corr(c->amg_fill, 1.8);
    check(c, nil::amg_update(c->amg_fill, w, dg, pw, c->stream), "mg values");
    mark(c, 12);
    int its = 0;
    check(c,
          nil::amg_fill_solve(c->amg_fill, gc, ptr<uint32_t>(c->skey), lists + 3 * K1, n_large, K, b64, x64, pb.prm.cg_rtol, mg_maxit,
                              warm, rr, bb, iters, misc(c) + M_STATS + 2, c->host, &its, c->stream),
          "mg solve");
    mark(c, 13);
    readback(c, misc(c) + M_STATS + 2, sizeof(int), c->host);
    launches = its;
    large_kernel_ms = ev_ms(c, 12, 13);
    mg_build_ms = ev_ms(c, 14, 12);
    mg_levels = nil::amg_levels(c->amg_fill);
    if (c->host[0] > 0 && mg_maxit < pb.prm.cg_max_iter) {
      // the multigrid solve stalled: solve the large components again with
      // the Jacobi preconditioner, from the same start
      check(c, hipStreamWaitEvent(c->stream, c->ev[6], 0), "join");  // the small tiers read x
      check(c, hipMemsetAsync(misc(c) + M_STATS + 2, 0, 2 * sizeof(int), c->stream), "memset");
      check(c, nil::fill_gather_x0(cpix, N, xw, x, c->stream), "gather");
      mg_fallback = 1;
      jacobi = true;
      launches = 0;
    } else {
      check(c, nil::mg_out(N, ptr<uint32_t>(c->skey), comp_off, x64, x, c->stream), "mg out");
      check(c, nil::large_finish(a, cpix, zout, c->stream), "large finish");
    }
  }
  if (jacobi) {
    nil::LargeArgs a = large_args();
    check(c, hipMemsetAsync(a.active, 0, 2 * sizeof(int), c->stream), "memset");
    check(c, nil::large_init(a, warm, c->stream), "large init");
    // one launch per CG iteration; the host reads the count of components
    // still iterating once per batch.  Events bracket each batch of launches
    // (not the readbacks) for the kernel-time report.
    const int batch = 16;
    float kms = 0.f;
    for (int it = 0; it <= pb.prm.cg_max_iter + 1; it += batch) {
      mark(c, 12);
      for (int k = 0; k < batch; ++k) check(c, nil::large_iter(a, it + k, c->stream), "large iter");
      mark(c, 13);
      launches += batch;
      readback(c, a.active + ((it + batch - 1) & 1), sizeof(int), c->host);
      kms += ev_ms(c, 12, 13);
      if (c->host[0] <= 0) break;
    }
    large_kernel_ms = kms;
    check(c, nil::large_finish(a, cpix, zout, c->stream), "large finish");
  }
  check(c, hipEventRecord(c->ev[15], c->stream), "event");  // end of the large solve
  check(c, hipStreamWaitEvent(c->stream, c->ev[6], 0), "join");
  mark(c, 7);
  readback(c, misc(c) + M_STATS, 4 * sizeof(int), c->host);
  const int notconv = c->host[0] + c->host[2], fallbacks = c->host[1] + c->host[3];
  if (rep) {
    std::vector<int> it(K), off(K1);
    std::vector<double> rel(K), hrr(K), hbb(K);
    if (K > 0) {
      check(c, hipMemcpyAsync(it.data(), iters, K * sizeof(int), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipMemcpyAsync(off.data(), comp_off, K1 * sizeof(int), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipMemcpyAsync(rel.data(), relres, K * sizeof(double), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipMemcpyAsync(hrr.data(), rr, K * sizeof(double), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipMemcpyAsync(hbb.data(), bb, K * sizeof(double), hipMemcpyDeviceToHost, c->stream), "D2H");
      check(c, hipStreamSynchronize(c->stream), "sync");
      const int cap = nil::fill_small_cap();
      long long pxit = 0, lpxit = 0;
      int itmax = 0;
      double rmax = 0;
      for (int k = 0; k < K; ++k) {
        int n = off[k + 1] - off[k];
        pxit += (long long)n * it[k];
        if (n > cap) {
          lpxit += (long long)n * it[k];
          rel[k] = hbb[k] > 0 ? sqrt(hrr[k] / hbb[k]) : 0.0;
        }
        itmax = std::max(itmax, it[k]);
        rmax = std::max(rmax, rel[k]);
      }
      long long nsys = 0;
      for (int k = 0; k < K; ++k)
        if (off[k + 1] - off[k] > cap) nsys += off[k + 1] - off[k];
      if (mg) mg_bytes = nil::amg_fill_bytes(c->amg_fill, nsys);
      rep->fill_large_px = nsys;
      rep->fill_px_iters = pxit;
      rep->fill_large_px_iters = lpxit;
      rep->fill_iters_max = itmax;
      rep->fill_max_relres = rmax;
    }
    rep->n_small = ntier[0] + ntier[1] + ntier[2];
    rep->n_large = n_large;
    rep->fill_notconv = notconv;
    rep->fill_large_launches = launches;
    rep->warm_fallbacks = fallbacks;
    rep->ms_assemble = ev_ms(c, 3, 4);
    rep->ms_warm = ev_ms(c, 4, 5);
    rep->ms_fill_small = ev_ms(c, 5, 6);
    rep->ms_fill_large = ev_ms(c, 5, 15);
    rep->ms_large_kernel = large_kernel_ms;
    rep->fill_chunk = n_large > 0 && !mg ? c->fill_chunk : 0;
    rep->fill_split = n_large > 0 && !mg ? c->fill_split : 0;
    rep->fill_mg_levels = mg_levels;
    rep->ms_fill_mg_build = mg_build_ms;
    rep->fill_mg_bytes = mg_bytes;
    rep->fill_mg_fallback = mg_fallback;
  }
  if (notconv > 0) {
    c->err = std::to_string(notconv) + " component(s) hit cg_max_iter";
    throw Fail{NI_E_NOTCONV};
  }
}

// One step only (test hook): with step_S non-null the scales start from
// step_S, iteration step_t alone runs, and its increment s^(t) and energy go
// to step_s / *step_e instead of the outputs.
struct StepHook {
  const double* S = nullptr;
  int t = 0;
  double* s = nullptr;
  double* e = nullptr;
};

void stage_irls(ni_ctx* c, const Problem& pb, const int32_t* labels, const Seg& sg, const float* zfill,
                float* depth, double* log_scale, ni_report* rep, const StepHook& hook = StepHook()) {
  const int P = pb.P, W = pb.W, K = sg.K;
  const bool persp = pb.cam.proj == NI_PERSP;
  int* cntd = misc(c) + M_COUNT;
  mark(c, 8);
  size_t K1 = (size_t)K + 1;
  nil::IrlsArgs a;
  if (!c->amg) c->amg = nil::amg_new();
  a.amg = c->amg;
  a.graphs = pb.prm.graphs ? 1 : 0;
  a.W = W; a.label = labels; a.K0 = K; a.grp = nullptr; a.ebits = ptr<uint8_t>(c->ebits); a.eb2 = eb2(c, pb);
  a.zfill = zfill;
  a.S = ensure<double>(c, c->S, K1);
  a.psum = ensure<double>(c, c->psum, K1);
  a.pcnt = ensure<double>(c, c->pcnt, K1);
  a.pkey = ensure<uint32_t>(c, c->pkey, K1);
  a.pnode = ensure<uint32_t>(c, c->pnode, K1);
  a.pnode_in = ensure<uint32_t>(c, c->pnode_in, K1);
  a.pk_tmp = ensure<uint32_t>(c, c->pk_tmp, K1);
  a.pv_tmp = ensure<uint32_t>(c, c->pv_tmp, K1);
  a.pscan = ensure<int>(c, c->pscan, nil::radix_tmp_ints((int)K1));
  a.pval = ensure<double>(c, c->pval, K1);
  a.prun = ensure<uint8_t>(c, c->prun, nil::run_sums_tmp_bytes((int)K1));
  a.parent = ensure<int>(c, c->qparent, K1);
  a.wmax = (unsigned long long*)(misc(c) + M_WMAX);
  a.energy_out = (double*)(misc(c) + M_ENERGY);
  a.qiters_out = misc(c) + M_QITERS;
  a.qiters2_out = misc(c) + M_QITERS2;
  a.g2fx = persp ? pb.cam.fx * pb.cam.fx : 1.0;
  a.g2fy = persp ? pb.cam.fy * pb.cam.fy : 1.0;
  a.g2fd = persp ? pb.cam.fx * pb.cam.fy : 1.0;
  a.k = pb.prm.bini_k; a.L = pb.prm.out_L; a.U = pb.prm.out_U; a.cut_rel = pb.prm.w_cut_rel;
  a.q_rtol = pb.prm.q_rtol; a.q_rtol2 = pb.prm.q_rtol_refine; a.align = pb.prm.align_iters; a.outlier_mode = pb.prm.outlier_mode;
  a.out_from = pb.prm.variant == 1 ? 1 : 0;
  a.q_maxit = pb.prm.q_max_iter;
  a.host_flag = c->host + 32;
  int hints[2] = {0, 0};
  a.hints = hints;
  // The quotient structure of a node labelling (the components, or merged
  // nodes after a merge): inter edges, sorted pairs, CSR, heavy rows and the
  // FP64 edge geometry.  A rebuild after a merge only shrinks every size,
  // so no buffer in use is reallocated.
  auto build = [&](const int* gl, int Kg) {
    // inter-component edges
    check(c, nil::quot_inter_edges(gl, ptr<uint8_t>(c->ebits), eb2(c, pb), P, W, ptr<int>(c->flag),
                                   ptr<int>(c->scanv), cntd, nullptr, ptr<int>(c->scan_tmp), c->stream, 0),
          "inter edges");
    readback(c, cntd, sizeof(int), c->host);
    const int E = c->host[0];
    uint32_t* eidx_raw = ensure<uint32_t>(c, c->eidx_raw, E);
    uint32_t* eidx = ensure<uint32_t>(c, c->eidx, E);
    check(c, nil::quot_inter_edges(gl, ptr<uint8_t>(c->ebits), eb2(c, pb), P, W, ptr<int>(c->flag),
                                   ptr<int>(c->scanv), cntd, eidx_raw, ptr<int>(c->scan_tmp), c->stream, 1),
          "inter compact");
    size_t srt = std::max<size_t>(E, 1);
    uint32_t* keys = ensure<uint32_t>(c, c->key, std::max<size_t>(srt, P));
    uint32_t* ktmp = ensure<uint32_t>(c, c->ktmp, srt);
    uint32_t* vtmp = ensure<uint32_t>(c, c->vtmp, srt);
    uint32_t* kout2 = ensure<uint32_t>(c, c->kout2, srt);
    int* pflag = ensure<int>(c, c->pflag, srt);
    int* ppos = ensure<int>(c, c->ppos, srt);
    ensure_scan(c, std::max<size_t>(ndirs(pb) * P, srt));
    check(c, nil::quot_sort_edges(eidx_raw, E, W, Kg, gl, keys, eidx, ktmp, vtmp, kout2, pflag, ppos, cntd,
                                  ptr<int>(c->scan_tmp), c->stream),
          "sort edges");
    readback(c, cntd, sizeof(int), c->host);
    const int Pp = c->host[0];
    int* pair_start = ensure<int>(c, c->pair_start, (size_t)Pp + 1);
    int* pair_lo = ensure<int>(c, c->pair_lo, Pp);
    int* pair_hi = ensure<int>(c, c->pair_hi, Pp);
    check(c, nil::quot_pairs(eidx, pflag, ppos, E, W, gl, Pp, pair_start, pair_lo, pair_hi, c->stream), "pairs");
    size_t P2 = std::max<size_t>(2 * (size_t)Pp, 1);
    uint32_t* ent = ensure<uint32_t>(c, c->ent, P2);
    uint32_t* ent_tmp = ensure<uint32_t>(c, c->ent_tmp, P2);
    keys = ensure<uint32_t>(c, c->key, std::max<size_t>({srt, (size_t)P, P2}));
    ktmp = ensure<uint32_t>(c, c->ktmp, std::max(srt, P2));
    vtmp = ensure<uint32_t>(c, c->vtmp, std::max(srt, P2));
    kout2 = ensure<uint32_t>(c, c->kout2, std::max(srt, P2));
    ensure_scan(c, std::max<size_t>({ndirs(pb) * P, srt, P2}));
    const size_t Kg1 = (size_t)Kg + 1;
    int* rowcnt = ensure<int>(c, c->rowcnt, Kg1);
    int* row_off = ensure<int>(c, c->row_off, Kg1);
    check(c, nil::quot_csr(pair_lo, pair_hi, Pp, Kg, keys, ent, ktmp, vtmp, kout2, ent_tmp, rowcnt, row_off,
                           ptr<int>(c->scan_tmp), c->stream),
          "csr");
    // rows multiplied by a whole wavefront
    int* heavy = ensure<int>(c, c->lpos, Kg1);
    check(c, nil::quot_heavy_rows(row_off, Kg, ptr<int>(c->flag), ptr<int>(c->scanv), heavy, cntd + 2,
                                  ptr<int>(c->scan_tmp), c->stream),
          "heavy rows");
    readback(c, cntd + 2, 2 * sizeof(int), c->host);
    a.heavy = heavy;
    a.nbig = c->host[0];
    a.nheavy = c->host[0] + c->host[1];
    a.glabel = gl;
    a.eidx = eidx; a.E = E; a.P = Pp; a.K = Kg;
    a.pair_start = pair_start; a.pair_lo = pair_lo; a.pair_hi = pair_hi; a.row_off = row_off; a.ent = ent;
    double* eom = ensure<double>(c, c->eom, srt);
    double* eta = ensure<double>(c, c->eta, srt);
    double* etb = ensure<double>(c, c->etb, srt);
    check(c, nil::launch_inter_geom(eidx, E, pb.H, W, pb.normals, persp ? 1 : 0, pb.cam.pixel_pitch,
                                    ptr<double>(c->tab), eom, eta, etb, c->stream),
          "inter-edge geometry");
    a.eom = eom; a.eta = eta; a.etb = etb;
    a.ew = ensure<double>(c, c->ew, srt);
    a.erho = ensure<double>(c, c->erho, srt);
    a.pW = ensure<double>(c, c->pW, std::max(Pp, 1));
    a.pB = ensure<double>(c, c->pB, std::max(Pp, 1));
    a.diag = ensure<double>(c, c->diag, Kg1);
    a.rhs = ensure<double>(c, c->qrhs, Kg1);
    a.babs = ensure<double>(c, c->babs, Kg1);
    a.s = ensure<double>(c, c->qs, Kg1);
    a.epart = ensure<double>(c, c->epart, (size_t)ni::ceil_div(std::max(Pp, 1), 256));
    a.nnz = 2 * Pp;
    a.qcol = ensure<int>(c, c->qcol, std::max(a.nnz, 1));
    a.qw = ensure<double>(c, c->qw, std::max(a.nnz, 1));
    a.t0 = ensure<double>(c, c->qt0, Kg1);
    a.t1 = ensure<double>(c, c->qt1, Kg1);
  };
  build(labels, K);
  const int E = a.E, Pp = a.P;
  check(c, hipMemsetAsync(a.S, 0, K1 * sizeof(double), c->stream), "memset");
  if (hook.S) {
    if (K > 0)
      check(c, hipMemcpyAsync(a.S, hook.S, K * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "copy S");
    check(c, nil::irls_iteration(a, hook.t, c->stream), "irls");
    if (K > 0) check(c, hipMemcpyAsync(hook.s, a.s, K * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "copy s");
    check(c, hipMemcpyAsync(hook.e, a.energy_out + hook.t, sizeof(double), hipMemcpyDeviceToHost, c->stream), "D2H");
    int qa = 0, qb = 0;
    check(c, hipMemcpyAsync(&qa, a.qiters_out + hook.t, sizeof(int), hipMemcpyDeviceToHost, c->stream), "D2H");
    check(c, hipMemcpyAsync(&qb, a.qiters2_out + hook.t, sizeof(int), hipMemcpyDeviceToHost, c->stream), "D2H");
    check(c, hipStreamSynchronize(c->stream), "sync");
    if (rep) {
      rep->irls_iters_run = 1;
      rep->energy[0] = *hook.e;
      rep->quot_iters[0] = qa + qb;
      rep->quot_iters_refine[0] = qb;
      rep->n_inter_edges = E;
      rep->n_pairs = Pp;
    }
    if (qa >= pb.prm.q_max_iter || qb >= pb.prm.q_max_iter) {
      c->err = "relative-scale solve stopped at q_max_iter";
      throw Fail{NI_E_NOTCONV};
    }
    return;
  }
  const int T = pb.prm.irls_iters;
  const int freq = pb.prm.freq_merging;
  int ran = 0, merges = 0;
  std::vector<double> en(NI_MAX_IRLS, 0.0);
  int* grp = nullptr;
  int* gl = nullptr;
  if (freq > 0 && freq < T && K > 0) {
    grp = ensure<int>(c, c->mgrp, K1);
    gl = ensure<int>(c, c->mglab, (size_t)P);
    ensure<unsigned long long>(c, c->mkey, K1);
    ensure<unsigned>(c, c->mcode, K1);
    ensure<int>(c, c->mpa, K1);
    ensure<int>(c, c->mpb, K1);
    ensure<double>(c, c->mkeep, K1);
    ensure<int>(c, c->mrank, K1);
    ensure_scan(c, K1);
    check(c, nil::identity_groups(grp, K, c->stream), "groups");
  }
  for (int t = 0; t < T; ++t) {
    check(c, nil::irls_iteration(a, t, c->stream), "irls");
    a.fresh = 0;
    ran = t + 1;
    if (grp && (t + 1) % freq == 0 && t + 1 < T) {
      // optional merging (Sec. 3.5): new nodes from the residuals at the
      // updated log-depth, then the quotient structure of the new nodes (a
      // single node left: the merge is a no-op)
      if (a.K > 1) {
        a.grp = grp;
        check(c,
              nil::merge_nodes(a, grp, gl, P, ptr<unsigned long long>(c->mkey), ptr<unsigned>(c->mcode),
                               ptr<int>(c->mpa), ptr<int>(c->mpb), ptr<double>(c->mkeep), ptr<int>(c->qparent),
                               ptr<int>(c->flag), ptr<int>(c->mrank), cntd + 4, ptr<int>(c->scan_tmp), c->stream),
              "merge");
        readback(c, cntd + 4, sizeof(int), c->host);
        build(gl, c->host[0]);
        a.fresh = 1;  // the next step cannot reuse the previous hierarchy
      }
      ++merges;
    }
    if (pb.prm.delta_e_max > 0 && t >= pb.prm.align_iters + 1) {
      readback(c, a.energy_out, sizeof(double) * (t + 1), en.data());
      double Ep = en[t - 1], Et = en[t];
      if (Ep == 0.0 || fabs(Et - Ep) / Ep < pb.prm.delta_e_max) break;
    }
  }
  mark(c, 9);
  // a quotient solve round that stopped at its cap leaves the scales
  // unconverged: the outputs are still written, and the call reports it
  std::vector<int> qi(NI_MAX_IRLS, 0), qi2(NI_MAX_IRLS, 0);
  check(c, hipMemcpyAsync(qi.data(), a.qiters_out, sizeof(int) * NI_MAX_IRLS, hipMemcpyDeviceToHost, c->stream),
        "D2H");
  check(c, hipMemcpyAsync(qi2.data(), a.qiters2_out, sizeof(int) * NI_MAX_IRLS, hipMemcpyDeviceToHost, c->stream),
        "D2H");
  check(c, hipStreamSynchronize(c->stream), "sync");
  int capped = -1;
  for (int t = 0; t < ran && capped < 0; ++t)
    if (qi[t] >= pb.prm.q_max_iter || qi2[t] >= pb.prm.q_max_iter) capped = t;
  // regions of G_0 and outputs
  check(c,
        nil::grid_components(ptr<uint8_t>(c->ebits), pb.H, W, EB_VR, EB_VD, ptr<int>(c->parent), ptr<int>(c->flag),
                             ptr<int>(c->scanv), nullptr, cntd + 1, ptr<int>(c->scan_tmp), c->stream, eb2(c, pb),
                             EB2_VDR, EB2_VDL),
        "regions");
  readback(c, cntd + 1, sizeof(int), c->host);
  const int R = c->host[0];
  double* csum = ensure<double>(c, c->csum, K1);
  int* comp_rid = ensure<int>(c, c->comp_rid, K1);
  double* rsum = ensure<double>(c, c->rsum, std::max(R, 1));
  double* rcnt = ensure<double>(c, c->rcnt, std::max(R, 1));
  nil::FinalScratch fw;
  fw.g = ensure<double>(c, c->fg, std::max<size_t>(sg.N, 2 * K1));
  fw.k0 = ensure<uint32_t>(c, c->pkey, K1);
  fw.v0 = ensure<uint32_t>(c, c->pnode, K1);
  fw.k1 = ensure<uint32_t>(c, c->pnode_in, K1);
  fw.v1 = ensure<uint32_t>(c, c->pk_tmp, K1);
  fw.k2 = ensure<uint32_t>(c, c->pv_tmp, K1);
  fw.v2 = ensure<uint32_t>(c, c->fv2, K1);
  fw.scan = ensure<int>(c, c->pscan, nil::radix_tmp_ints((int)K1));
  fw.rtmp = ensure<uint8_t>(c, c->prun, nil::run_sums_tmp_bytes((int)std::max<size_t>(sg.N, K1)));
  check(c, nil::final_outputs(labels, zfill, a.S, ptr<int>(c->comp_off), ptr<uint32_t>(c->spix),
                              ptr<uint32_t>(c->skey), ptr<int>(c->parent), ptr<int>(c->scanv), K, sg.N, R, P,
                              persp ? 1 : 0, csum, comp_rid, rsum, rcnt, depth, log_scale, fw, c->stream),
        "finalize");
  mark(c, 10);
  check(c, hipStreamSynchronize(c->stream), "sync");
  if (rep) {
    rep->n_regions = R;
    rep->n_inter_edges = E;
    rep->n_pairs = Pp;
    rep->irls_iters_run = ran;
    rep->merges = merges;
    rep->nodes_final = a.K;
    check(c, hipMemcpy(en.data(), a.energy_out, sizeof(double) * NI_MAX_IRLS, hipMemcpyDeviceToHost), "D2H");
    for (int t = 0; t < NI_MAX_IRLS; ++t) {
      rep->energy[t] = t < ran ? en[t] : 0.0;
      rep->quot_iters[t] = t < ran ? qi[t] + qi2[t] : 0;
      rep->quot_iters_refine[t] = t < ran ? qi2[t] : 0;
    }
    rep->ms_irls = ev_ms(c, 8, 9);
    rep->ms_finalize = ev_ms(c, 9, 10);
  }
  if (capped >= 0) {
    c->err = "relative-scale solve of iteration " + std::to_string(capped) + " stopped at q_max_iter";
    throw Fail{NI_E_NOTCONV};
  }
}

template <class F>
ni_status guarded(ni_ctx* c, F&& f) {
  try {
    f();
    return NI_OK;
  } catch (const Fail& e) {
    return e.s;
  } catch (...) {
    c->err = "internal error";
    return NI_E_DEVICE;
  }
}

void begin(ni_ctx* c, ni_report* rep) {
  check(c, hipSetDevice(c->device), "hipSetDevice");
  if (rep) memset(rep, 0, sizeof(*rep));
  mark(c, 0);
}

}  // namespace

// ===================================================================== ABI
extern "C" {

int32_t ni_abi_version(void) { return NI_ABI_VERSION; }

ni_status ni_params_default(ni_params* p) {
  if (!p) return NI_E_ARG;
  memset(p, 0, sizeof(*p));
  p->theta_c_deg = 2.0;
  p->connectivity = 4;
  p->irls_iters = 15;
  p->align_iters = 2;
  p->bini_k = 2.0;
  p->out_L = 1e-5;
  p->out_U = 1e-3;
  p->outlier_mode = 1;
  p->delta_e_max = 0.0;
  p->w_cut_rel = 1e-12;
  p->cg_rtol = 1e-6;
  p->cg_max_iter = 50000;
  p->q_rtol = 1e-5;
  p->q_rtol_refine = 1e-5;
  p->q_max_iter = 20000;
  p->warm_start = 0;
  p->graphs = 0;
  p->fill_chunk = 0;
  p->freq_merging = 0;
  p->variant = 0;
  p->fill_split = 0;
  p->fill_precond = 1;
  p->fill_mg_maxit = 0;
  return NI_OK;
}

ni_status ni_create(ni_ctx** out, int device) {
  if (!out) return NI_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NI_E_DEVICE;
  ni_ctx* c = new (std::nothrow) ni_ctx();
  if (!c) return NI_E_NOMEM;
  c->device = device;
  ni_status s = guarded(c, [&] {
    check(c, hipSetDevice(device), "hipSetDevice");
    check(c, hipHostMalloc((void**)&c->host, 64 * sizeof(int), hipHostMallocDefault), "hipHostMalloc");
    for (auto& e : c->ev) check(c, hipEventCreate(&e), "hipEventCreate");
    check(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "hipStreamCreate");
    check(c, scratch_address(device, &c->noalloc), "hipGetSymbolAddress(scratch)");
  });
  if (s != NI_OK) {
    ni_destroy(c);
    return s;
  }
  *out = c;
  return NI_OK;
}

ni_status ni_destroy(ni_ctx* c) {
  if (!c) return NI_E_ARG;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  for (Buf* b : c->bufs)
    if (b->p) (void)hipFree(b->p);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->host) (void)hipHostFree(c->host);
  if (c->unet) nil::unet_free(c->unet);
  if (c->amg) nil::amg_free(c->amg);
  if (c->amg_fill) nil::amg_free(c->amg_fill);
  delete c;
  return NI_OK;
}

ni_status ni_set_stream(ni_ctx* c, void* s) {
  if (!c) return NI_E_ARG;
  c->stream = (hipStream_t)s;
  return NI_OK;
}

ni_status ni_integrate(ni_ctx* c, const float* normals, const uint8_t* mask, int32_t H, int32_t W,
                       const ni_camera* cam, const ni_params* params, float* depth, int32_t* labels,
                       double* log_scale, int64_t cap, int32_t* K, ni_report* rep) {
  Problem pb;
  ni_status s = validate(c, normals, mask, H, W, cam, params, &pb);
  if (s != NI_OK) return s;
  if (!depth || !labels || !K || (cap > 0 && !log_scale) || cap < 0) {
    c->err = "null output pointer or negative cap";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    begin(c, rep);
    stage_setup(c, pb);
    mark(c, 1);
    int k = stage_label(c, pb, labels);
    mark(c, 2);
    *K = k;
    // stage times are read once their end events have completed (an
    // event still pending reads as not ready)
    auto label_times = [&] {
      if (!rep) return;
      check(c, hipEventSynchronize(c->ev[2]), "sync");
      rep->K = k;
      rep->ms_setup = ev_ms(c, 0, 1);
      rep->ms_label = ev_ms(c, 1, 2);
    };
    if ((int64_t)k > cap) {
      label_times();
      c->err = "log_scale capacity smaller than K";
      throw Fail{NI_E_SHAPE};
    }
    Seg sg = build_segments(c, pb, labels, k, false);
    if (rep) rep->n_valid = sg.N;
    float* zf = ptr<float>(c->zgrid);
    ni_status fs = NI_OK;
    try {
      stage_fill(c, pb, labels, sg, zf, rep);
    } catch (const Fail& f) {
      if (f.s != NI_E_NOTCONV) throw;
      fs = f.s;
    }
    ni_status qs = NI_OK;
    try {
      stage_irls(c, pb, labels, sg, zf, depth, log_scale, rep);
    } catch (const Fail& f) {
      if (f.s != NI_E_NOTCONV) throw;
      qs = f.s;
    }
    if (rep) {
      mark(c, 11);
      check(c, hipEventSynchronize(c->ev[11]), "sync");
      label_times();
      rep->ms_segments = ev_ms(c, 2, 3);
      rep->ms_total = ev_ms(c, 0, 11);
    }
    if (fs != NI_OK) throw Fail{fs};
    if (qs != NI_OK) throw Fail{qs};
  });
}

ni_status ni_label(ni_ctx* c, const float* normals, const uint8_t* mask, int32_t H, int32_t W,
                   const ni_camera* cam, const ni_params* params, int32_t* labels, int32_t* K, ni_report* rep) {
  Problem pb;
  ni_status s = validate(c, normals, mask, H, W, cam, params, &pb);
  if (s != NI_OK) return s;
  if (!labels || !K) {
    c->err = "null output pointer";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    begin(c, rep);
    stage_setup(c, pb);
    mark(c, 1);
    *K = stage_label(c, pb, labels);
    mark(c, 2);
    check(c, hipStreamSynchronize(c->stream), "sync");
    if (rep) {
      rep->K = *K;
      rep->ms_setup = ev_ms(c, 0, 1);
      rep->ms_label = ev_ms(c, 1, 2);
    }
  });
}

ni_status ni_label_noalloc(ni_ctx* c, const float* normals, const uint8_t* mask, int32_t H, int32_t W,
                           const ni_camera* cam, const ni_params* params, int32_t* labels, int32_t* K) {
  Problem pb;
  ni_status s = validate(c, normals, mask, H, W, cam, params, &pb);
  if (s != NI_OK) return s;
  if (!labels || !K) {
    c->err = "null output pointer";
    return NI_E_ARG;
  }
  if (H > NOALLOC_MAX_SIDE || W > NOALLOC_MAX_SIDE || (long long)H * W > NOALLOC_MAX_PX) {
    c->err = "map larger than the allocation-free scratch holds (H, W <= 4096, H*W <= 2^20)";
    return NI_E_SHAPE;
  }
  if (!c->noalloc) {
    c->err = "no scratch address for this device";
    return NI_E_DEVICE;
  }
  return guarded(c, [&] {
    check(c, hipSetDevice(c->device), "hipSetDevice");
    const int P = H * W;
    // carve the scratch: counters, ray tables, edge arrays, union-find
    size_t off = 0;
    auto take = [&](size_t bytes) {
      char* p = static_cast<char*>(c->noalloc) + off;
      off += (bytes + 255) & ~(size_t)255;
      return p;
    };
    int* cnt = reinterpret_cast<int*>(take(16 * sizeof(int)));  // [0] K, [8] non-finite flag
    double* tab = reinterpret_cast<double*>(take((2 * (size_t)W + 2 * (size_t)H) * sizeof(double)));
    uint8_t* ebits = reinterpret_cast<uint8_t*>(take(P));
    uint8_t* eb2 = pb.prm.connectivity == 8 ? reinterpret_cast<uint8_t*>(take(P)) : nullptr;
    float* nt = reinterpret_cast<float*>(take((size_t)P * sizeof(float)));
    int* parent = reinterpret_cast<int*>(take((size_t)P * sizeof(int)));
    int* flag = reinterpret_cast<int*>(take((size_t)P * sizeof(int)));
    int* cid = reinterpret_cast<int*>(take((size_t)P * sizeof(int)));
    int* stmp = reinterpret_cast<int*>(take(nil::scan_tmp_ints(P) * sizeof(int)));
    if (off > NOALLOC_BYTES) {
      c->err = "allocation-free scratch too small for this map";
      throw Fail{NI_E_SHAPE};
    }
    hipStream_t st = c->stream;
    check(c, nil::set_i32(cnt, 16, 0, st), "clear counters");
    const bool persp = pb.cam.proj == NI_PERSP;
    if (persp) check(c, nil::ray_tables(H, W, pb.cam.cx, pb.cam.cy, pb.cam.fx, pb.cam.fy, tab, st), "ray tables");
    const double th = pb.prm.theta_c_deg;
    const int use_sim = th > 0 ? 1 : 0;
    const double cth = use_sim ? cos(th * M_PI / 180.0) : 2.0;
    check(c, nil::launch_setup(normals, mask, H, W, persp, pb.cam.pixel_pitch, tab, cth, use_sim, ebits, nullptr,
                               nullptr, nt, cnt + 8, st, eb2, nullptr, nullptr),
          "setup");
    check(c, nil::grid_components(ebits, H, W, EB_SR, EB_SD, parent, flag, cid, labels, cnt, stmp, st, eb2, EB2_SDR,
                                  EB2_SDL),
          "label");
    check(c, hipMemcpyAsync(c->host, cnt, 16 * sizeof(int), hipMemcpyDeviceToHost, st), "D2H");
    check(c, hipStreamSynchronize(st), "sync");
    if (c->host[8]) {
      c->err = "non-finite normal inside the mask";
      throw Fail{NI_E_NONFINITE};
    }
    *K = c->host[0];
  });
}

ni_status ni_fill(ni_ctx* c, const float* normals, const uint8_t* mask, int32_t H, int32_t W, const ni_camera* cam,
                  const ni_params* params, const int32_t* labels, int32_t K, float* zfill, ni_report* rep) {
  Problem pb;
  ni_status s = validate(c, normals, mask, H, W, cam, params, &pb);
  if (s != NI_OK) return s;
  if (!labels || !zfill || K < 0 || (int64_t)K > (int64_t)H * W) {
    c->err = "null pointer or K out of range";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    begin(c, rep);
    stage_setup(c, pb);
    readback(c, misc(c), 16 * sizeof(int), c->host);
    if (c->host[M_ERR]) {
      c->err = "non-finite normal inside the mask";
      throw Fail{NI_E_NONFINITE};
    }
    Seg sg = build_segments(c, pb, labels, K, true);
    if (rep) {
      rep->K = K;
      rep->n_valid = sg.N;
    }
    stage_fill(c, pb, labels, sg, zfill, rep);
    check(c, hipStreamSynchronize(c->stream), "sync");
  });
}

ni_status ni_irls_step(ni_ctx* c, const float* normals, const uint8_t* mask, int32_t H, int32_t W,
                       const ni_camera* cam, const ni_params* params, const int32_t* labels, int32_t K,
                       const float* zfill, const double* S_in, int32_t t, double* s_out, double* energy,
                       ni_report* rep) {
  Problem pb;
  ni_status s = validate(c, normals, mask, H, W, cam, params, &pb);
  if (s != NI_OK) return s;
  if (!labels || !zfill || !energy || K < 0 || (int64_t)K > (int64_t)H * W || (K > 0 && (!S_in || !s_out))) {
    c->err = "null pointer or K out of range";
    return NI_E_ARG;
  }
  if (t < 0 || t >= NI_MAX_IRLS) {
    c->err = "step index out of range";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    begin(c, rep);
    stage_setup(c, pb);
    readback(c, misc(c), 16 * sizeof(int), c->host);
    if (c->host[M_ERR]) {
      c->err = "non-finite normal inside the mask";
      throw Fail{NI_E_NONFINITE};
    }
    Seg sg = build_segments(c, pb, labels, K, true);
    if (rep) {
      rep->K = K;
      rep->n_valid = sg.N;
    }
    if (K == 0) {
      *energy = 0.0;
      return;
    }
    StepHook hook;
    hook.S = S_in;
    hook.t = t;
    hook.s = s_out;
    hook.e = energy;
    stage_irls(c, pb, labels, sg, zfill, nullptr, nullptr, rep, hook);
  });
}

ni_status ni_irls(ni_ctx* c, const float* normals, const uint8_t* mask, int32_t H, int32_t W, const ni_camera* cam,
                  const ni_params* params, const int32_t* labels, int32_t K, const float* zfill, float* depth,
                  double* log_scale, int64_t cap, ni_report* rep) {
  Problem pb;
  ni_status s = validate(c, normals, mask, H, W, cam, params, &pb);
  if (s != NI_OK) return s;
  if (!labels || !zfill || !depth || K < 0 || (int64_t)K > (int64_t)H * W || (K > 0 && !log_scale)) {
    c->err = "null pointer or K out of range";
    return NI_E_ARG;
  }
  if (cap < K) {
    c->err = "log_scale capacity smaller than K";
    return NI_E_SHAPE;
  }
  return guarded(c, [&] {
    begin(c, rep);
    stage_setup(c, pb);
    readback(c, misc(c), 16 * sizeof(int), c->host);
    if (c->host[M_ERR]) {
      c->err = "non-finite normal inside the mask";
      throw Fail{NI_E_NONFINITE};
    }
    Seg sg = build_segments(c, pb, labels, K, true);
    if (rep) {
      rep->K = K;
      rep->n_valid = sg.N;
    }
    stage_irls(c, pb, labels, sg, zfill, depth, log_scale, rep);
  });
}

int32_t ni_unet_param_count(void) { return nil::unet_param_count(); }
size_t ni_unet_blob_size(void) { return nil::unet_blob_size(); }

ni_status ni_unet_init(ni_ctx* c, uint64_t seed) {
  if (!c) return NI_E_ARG;
  return guarded(c, [&] {
    check(c, hipSetDevice(c->device), "hipSetDevice");
    nil::UnetModel* m = nullptr;
    if (!nil::unet_new(&m, seed, &c->err)) throw Fail{NI_E_NOMEM};
    if (c->unet) nil::unet_free(c->unet);
    c->unet = m;
  });
}

ni_status ni_unet_load(ni_ctx* c, const void* blob, size_t nbytes) {
  if (!c || !blob) return NI_E_ARG;
  return guarded(c, [&] {
    check(c, hipSetDevice(c->device), "hipSetDevice");
    nil::UnetModel* m = nullptr;
    if (!nil::unet_load(&m, blob, nbytes, &c->err)) throw Fail{NI_E_MODEL};
    if (c->unet) nil::unet_free(c->unet);
    c->unet = m;
  });
}

static ni_status need_model(ni_ctx* c) {
  if (!c) return NI_E_ARG;
  if (!c->unet) {
    c->err = "no U-Net model (ni_unet_init or ni_unet_load first)";
    return NI_E_MODEL;
  }
  c->err.clear();
  return NI_OK;
}

ni_status ni_unet_save(ni_ctx* c, void* blob, size_t nbytes) {
  ni_status s = need_model(c);
  if (s != NI_OK) return s;
  if (!blob || nbytes != nil::unet_blob_size()) {
    c->err = "blob must be ni_unet_blob_size() bytes";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    check(c, hipSetDevice(c->device), "hipSetDevice");
    check(c, nil::unet_save(c->unet, blob), "save");
  });
}

ni_status ni_unet_get_params(ni_ctx* c, float* host, int32_t n) {
  ni_status s = need_model(c);
  if (s != NI_OK) return s;
  if (!host || n != nil::unet_param_count()) {
    c->err = "need ni_unet_param_count() floats";
    return NI_E_ARG;
  }
  return guarded(c, [&] { check(c, nil::unet_get_params(c->unet, host), "get params"); });
}

ni_status ni_unet_set_params(ni_ctx* c, const float* host, int32_t n) {
  ni_status s = need_model(c);
  if (s != NI_OK) return s;
  if (!host || n != nil::unet_param_count()) {
    c->err = "need ni_unet_param_count() floats";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    check(c, nil::unet_set_params(c->unet, host, c->stream), "set params");
    check(c, hipStreamSynchronize(c->stream), "sync");
  });
}

ni_status ni_unet_predict(ni_ctx* c, const float* normals, const uint8_t* mask, int32_t H, int32_t W,
                          const ni_camera* cam, float* out) {
  ni_status s = need_model(c);
  if (s != NI_OK) return s;
  if (!normals || !mask || !cam || !out || H < 1 || W < 1 || (long long)H * W > (1ll << 28)) {
    c->err = "bad argument";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    check(c, hipSetDevice(c->device), "hipSetDevice");
    check(c, nil::unet_predict(c->unet, normals, mask, H, W, cam, out, nullptr, 0, c->stream), "predict");
    check(c, hipStreamSynchronize(c->stream), "sync");
  });
}

ni_status ni_unet_forward(ni_ctx* c, const float* feat, int32_t B, int32_t H, int32_t W, float* out) {
  ni_status s = need_model(c);
  if (s != NI_OK) return s;
  if (!feat || !out || B < 1 || H < 8 || W < 8 || H % 8 || W % 8 || (long long)B * H * W > (1ll << 28)) {
    c->err = "need B >= 1 and H, W multiples of 8";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    check(c, hipSetDevice(c->device), "hipSetDevice");
    check(c, nil::unet_forward_raw(c->unet, feat, B, H, W, out, c->stream), "forward");
    check(c, hipStreamSynchronize(c->stream), "sync");
  });
}

ni_status ni_unet_backward(ni_ctx* c, const float* dout, float* grad) {
  ni_status s = need_model(c);
  if (s != NI_OK) return s;
  if (!dout || !grad) {
    c->err = "bad argument";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    check(c, hipSetDevice(c->device), "hipSetDevice");
    check(c, nil::unet_backward_raw(c->unet, dout, grad, c->stream), "backward");
    check(c, hipStreamSynchronize(c->stream), "sync");
  });
}

ni_status ni_unet_train_step(ni_ctx* c, const float* normals, const uint8_t* mask, const ni_camera* cams,
                             const float* target, const int32_t* labels, int32_t ncomp, int32_t B, int32_t S,
                             float lr, double* loss) {
  ni_status s = need_model(c);
  if (s != NI_OK) return s;
  if (!normals || !mask || !cams || !target || !labels || !loss || B < 1 || S < 8 || S % 8 || ncomp < 1 ||
      (long long)B * S * S > (1ll << 28)) {
    c->err = "bad argument";
    return NI_E_ARG;
  }
  return guarded(c, [&] {
    check(c, hipSetDevice(c->device), "hipSetDevice");
    check(c, nil::unet_train_step(c->unet, normals, mask, cams, target, labels, ncomp, B, S, lr, loss, c->stream),
          "train step");
    check(c, hipStreamSynchronize(c->stream), "sync");
  });
}

const char* ni_status_str(ni_status s) {
  switch (s) {
    case NI_OK: return "ok";
    case NI_E_ARG: return "invalid argument";
    case NI_E_SHAPE: return "output capacity too small";
    case NI_E_NONFINITE: return "non-finite normal inside the mask";
    case NI_E_NOMEM: return "out of device memory";
    case NI_E_DEVICE: return "HIP runtime error";
    case NI_E_NOTCONV: return "a CG solve hit its iteration cap";
    case NI_E_MODEL: return "bad or missing warm-start model";
  }
  return "unknown status";
}

const char* ni_last_error(const ni_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
