// C ABI of libnlpr: plans and batches, workspace layout, the ADMM solve sequence, per-stage
// entry points for testing, stage timing and graph capture.  See include/nlpr.h.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nlpr_internal.h"

struct nlpr_plan {
  nlpr::Batch B;
};
struct nlpr_batch {
  nlpr::Batch B;
};

namespace nlpr {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

constexpr uint32_t kBatchFlags = NLPR_INIT_ZERO | NLPR_STATE_IN | NLPR_CHECK_FINITE |
                                 NLPR_TIMING | NLPR_GRAPH | NLPR_FUSED_S;

bool factor_23(int n, LineFFT& f) {
  f.n = n;
  f.nfac = 0;
  int m = n;
  while (m % 8 == 0 && f.nfac < kMaxFFTFactors) { f.fac[f.nfac++] = 8; m /= 8; }
  if (m % 4 == 0 && f.nfac < kMaxFFTFactors) { f.fac[f.nfac++] = 4; m /= 4; }
  if (m % 2 == 0 && f.nfac < kMaxFFTFactors) { f.fac[f.nfac++] = 2; m /= 2; }
  while (m % 3 == 0 && f.nfac < kMaxFFTFactors) { f.fac[f.nfac++] = 3; m /= 3; }
  return m == 1;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int check_device_ptr(const void* ptr, const char* name) {
  if (!ptr) return fail(NLPR_ERR_INVALID_ARG, std::string(name) + " is NULL");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(NLPR_ERR_INVALID_ARG, std::string(name) + " is not a HIP device pointer");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(NLPR_ERR_INVALID_ARG, std::string(name) + " is not device memory");
  return NLPR_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

int validate(const nlpr_params& q) {
  auto bad = [](const std::string& m) { return fail(NLPR_ERR_UNSUPPORTED_SHAPE, m); };
  if (q.monitor_every < 0) return fail(NLPR_ERR_INVALID_ARG, "monitor_every must be >= 0");
  if (q.Ls < 0 || q.Ls > std::min(q.L, kMaxLs)) return bad("Ls must lie in [0, min(L, 32)]");
  LineFFT tmp{};
  if (q.p < 8 || q.q < 8 || q.p > kMaxFFTLen || q.q > kMaxFFTLen)
    return bad("p and q must lie in [8, 4096]");
  if (!factor_23(q.p, tmp) || !factor_23(q.q, tmp)) return bad("p and q must be of the form 2^a 3^b");
  if (q.q % 4) return bad("q must be a multiple of 4");
  if (q.d < 1) return fail(NLPR_ERR_INVALID_ARG, "d must be >= 1");
  if (q.p % q.d || q.q % q.d) return bad("d must divide p and q");
  if (q.L < 1 || q.L > 4096) return bad("L must lie in [1, 4096]");
  if (q.Lh < 1 || q.Lh > kMaxLh) return bad("Lh must lie in [1, 16]");
  if (q.blur_radius < 0 || q.blur_radius > kMaxBlurRadius) return bad("blur_radius must lie in [0, 16]");
  if (q.K < 0 || q.K > kMaxK) return bad("K must lie in [0, 4]");
  if (q.Sw < 0 || q.Sw > kMaxSw) return bad("Sw must lie in [0, 8]");
  if (q.Sw >= q.p || q.Sw >= q.q) return bad("Sw must be smaller than p and q");
  if ((q.flags & NLPR_LOCAL_WINDOW) && q.Sw != 1) return bad("NLPR_LOCAL_WINDOW needs Sw == 1");
  if (q.flags & NLPR_FUSED_S) {
    if (q.Ls != 0) return bad("NLPR_FUSED_S takes no subspace basis (Ls must be 0)");
    // the column pass holds d columns of p points and a line of twiddles in 64 KiB of LDS
    if ((size_t)8 * (q.d + 1) * q.p > 65536) return bad("NLPR_FUSED_S needs 8 * (d + 1) * p <= 65536");
  }
  if (q.iters < 0) return fail(NLPR_ERR_INVALID_ARG, "iters must be >= 0");
  if (!(q.lambda >= 0.0) || !std::isfinite(q.lambda)) return fail(NLPR_ERR_INVALID_ARG, "lambda must be >= 0");
  if (!(q.lambda1 > 0.0) || !std::isfinite(q.lambda1)) return fail(NLPR_ERR_INVALID_ARG, "lambda1 must be > 0");
  if (!(q.rho > 0.0) || !std::isfinite(q.rho)) return fail(NLPR_ERR_INVALID_ARG, "rho must be > 0");
  if (!(q.flags & NLPR_UNWEIGHTED) && !(q.h > 0.0 && std::isfinite(q.h)))
    return fail(NLPR_ERR_INVALID_ARG, "h must be > 0");
  // the sweep keeps full image rows of X, mu and its accumulator in LDS
  const int halo = (q.flags & NLPR_LOCAL_WINDOW) ? 1 : q.Sw;
  const SweepShape sh = choose_sweep_shape(q.p, q.q, q.K, halo);
  if (sh.lds > kMaxSweepLds)
    return bad("q too large for the patch / search radii: the sweep tile needs " +
               std::to_string(sh.lds) + " bytes of LDS (max " + std::to_string(kMaxSweepLds) + ")");
  return NLPR_OK;
}

// ---------------------------------------------------------------------------- scenes
void scene_free(Plan* P) {
  if (!P) return;
  hipFree(P->d_E);
  hipFree(P->d_Ep);
  hipFree(P->d_M);
  hipFree(P->d_Rt);
  hipFree(P->d_mon);
  hipFree(P->d_fia);
  hipFree(P->d_fu);
  hipFree(P->d_fv);
  hipFree(P->d_taus);
  hipFree(P->d_invden);
  hipFree(P->d_tw_p);
  hipFree(P->d_tw_q);
  hipFree(P->d_blur);
  hipFree(P->d_R);
  hipFree(P->d_G);
  delete P;
}

// A blur of rank one, b(a, c) = u(a) v(c) up to FP32 rounding (a Gaussian, for one), is
// applied as a pass along rows and one along columns: 2 (2r+1) multiply-adds per output
// instead of (2r+1)^2.  The factors come from the row and the column through the largest
// tap, in FP64; the blur counts as rank one when no tap differs from u(a) v(c) by more than
// 1e-6 of the largest (a Gaussian rounded to FP32 stays near 2e-7).  uv = u then v.
bool separable_factors(const float* b, int r, std::vector<float>& uv) {
  const int w = 2 * r + 1;
  int a0 = 0, c0 = 0;
  double bm = 0.0;
  for (int a = 0; a < w; ++a)
    for (int c = 0; c < w; ++c)
      if (std::fabs((double)b[a * w + c]) > bm) {
        bm = std::fabs((double)b[a * w + c]);
        a0 = a;
        c0 = c;
      }
  if (!(bm > 0.0) || !std::isfinite(bm)) return false;
  std::vector<double> u(w), v(w);
  for (int a = 0; a < w; ++a) u[a] = b[a * w + c0];
  for (int c = 0; c < w; ++c) v[c] = (double)b[a0 * w + c] / (double)b[a0 * w + c0];
  for (int a = 0; a < w; ++a)
    for (int c = 0; c < w; ++c)
      if (!(std::fabs((double)b[a * w + c] - u[a] * v[c]) <= 1e-6 * bm)) return false;
  uv.resize(2 * w);
  for (int a = 0; a < w; ++a) uv[a] = (float)u[a];
  for (int c = 0; c < w; ++c) uv[w + c] = (float)v[c];
  return true;
}

// Validate, upload the blur taps and R, precompute the tables, tune the FFT shapes and lay
// out the scene's part of the workspace.
int scene_create(const nlpr_params& prm, const float* blur_host, const float* R_host,
                 const float* E_host, Plan** out) {
  *out = nullptr;
  int rc = validate(prm);
  if (rc) return rc;
  if ((prm.Ls > 0) != (E_host != nullptr))
    return fail(NLPR_ERR_INVALID_ARG, "a basis E must be given exactly when Ls > 0");
  Plan* P = new (std::nothrow) Plan();
  if (!P) return fail(NLPR_ERR_INVALID_ARG, "out of host memory");
  P->prm = prm;
  P->Lx = prm.Ls > 0 ? prm.Ls : prm.L;
  const int p = prm.p, q = prm.q, L = prm.L, Lh = prm.Lh, r = prm.blur_radius, Lx = P->Lx;
  // W+ in storage order: (0, 1..S), then tau1 = 1..S with tau2 = -S..S
  if (prm.flags & NLPR_LOCAL_WINDOW) {
    P->taus = {0, 1, 1, 0};
  } else {
    const int S = prm.Sw;
    for (int b = 1; b <= S; ++b) { P->taus.push_back(0); P->taus.push_back(b); }
    for (int a = 1; a <= S; ++a)
      for (int b = -S; b <= S; ++b) { P->taus.push_back(a); P->taus.push_back(b); }
  }
  P->npairs = (int)P->taus.size() / 2;
  P->npatch = (2 * prm.K + 1) * (2 * prm.K + 1);
  int hrows = 0;
  for (int n = 0; n < P->npairs; ++n) hrows = std::max(hrows, P->taus[2 * n]);
  factor_23(p, P->fp);
  factor_23(q, P->fq);
  P->sweep = choose_sweep_shape(p, q, prm.K, hrows);
  P->sweep.split = choose_pair_split(P->sweep.ntiles * Lx, P->npairs);
  auto cleanup = [&](int code) {
    scene_free(P);
    return code;
  };
  const size_t plane = (size_t)p * q;
  if (hipMalloc(&P->d_taus, std::max<size_t>(1, P->npairs) * sizeof(int2)) != hipSuccess ||
      hipMalloc(&P->d_invden, plane * sizeof(float)) != hipSuccess ||
      hipMalloc(&P->d_tw_p, p * sizeof(float2)) != hipSuccess ||
      hipMalloc(&P->d_tw_q, q * sizeof(float2)) != hipSuccess ||
      hipMalloc(&P->d_blur, ((2 * r + 1) * (2 * r + 1) + 2 * (2 * r + 1)) * sizeof(float)) !=
          hipSuccess ||
      hipMalloc(&P->d_R, (size_t)L * Lh * sizeof(float)) != hipSuccess ||
      hipMalloc(&P->d_G, (size_t)Lh * Lh * sizeof(float)) != hipSuccess) {
    set_error("hipMalloc of plan tables failed");
    return cleanup(NLPR_ERR_HIP);
  }
  P->fp.tw = P->d_tw_p;
  P->fq.tw = P->d_tw_q;
  if ((P->npairs && hipMemcpy(P->d_taus, P->taus.data(), P->npairs * sizeof(int2),
                              hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(P->d_blur, blur_host, (2 * r + 1) * (2 * r + 1) * sizeof(float),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_R, R_host, (size_t)L * Lh * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("upload of the plan tables failed");
    return cleanup(NLPR_ERR_HIP);
  }
  {
    std::vector<float> uv;
    P->blur_separable = separable_factors(blur_host, r, uv);
    if (P->blur_separable &&
        hipMemcpy(P->d_blur + (2 * r + 1) * (2 * r + 1), uv.data(), uv.size() * sizeof(float),
                  hipMemcpyHostToDevice) != hipSuccess) {
      set_error("upload of the blur factors failed");
      return cleanup(NLPR_ERR_HIP);
    }
  }
  if (E_host) {
    if (hipMalloc(&P->d_E, (size_t)Lx * L * sizeof(float)) != hipSuccess ||
        hipMalloc(&P->d_Ep, (size_t)L * Lx * sizeof(float)) != hipSuccess ||
        hipMalloc(&P->d_M, (size_t)Lx * Lx * sizeof(float)) != hipSuccess ||
        hipMalloc(&P->d_Rt, (size_t)Lx * Lh * sizeof(float)) != hipSuccess ||
        hipMemcpy(P->d_E, E_host, (size_t)Lx * L * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("allocation or upload of the subspace tables failed");
      return cleanup(NLPR_ERR_HIP);
    }
  }
  if (prm.flags & NLPR_FUSED_S) {
    if (hipMalloc(&P->d_fia, plane * sizeof(float)) != hipSuccess ||
        hipMalloc(&P->d_fu, plane * sizeof(float2)) != hipSuccess ||
        hipMalloc(&P->d_fv, plane * sizeof(float2)) != hipSuccess) {
      set_error("allocation of the fused-S tables failed");
      return cleanup(NLPR_ERR_HIP);
    }
  }
  if (prm.monitor_every > 0) {
    P->mon_points = monitor_points(prm.iters, prm.monitor_every);
    const size_t nd = 4 * (size_t)pixel_blocks(*P) + monreg_blocks(*P) + 8 * (size_t)P->mon_points;
    if (hipMalloc(&P->d_mon, std::max<size_t>(nd, 1) * sizeof(double)) != hipSuccess) {
      set_error("allocation of the monitor buffer failed");
      return cleanup(NLPR_ERR_HIP);
    }
  }
  if ((rc = launch_precompute(*P))) return cleanup(rc);
  if (hipDeviceSynchronize() != hipSuccess) {
    set_error("plan precompute failed");
    return cleanup(NLPR_ERR_HIP);
  }
  if ((rc = autotune_fft(*P))) return cleanup(rc);
  // workspace layout
  size_t off = 0;
  auto take = [&](int slot, size_t bytes) {
    P->off[slot] = off;
    P->sz[slot] = bytes;
    off = align256(off + std::max<size_t>(bytes, 4));
  };
  const size_t pl = plane * Lx * sizeof(float);
  take(B_SIGMA, sweep_sigma_bytes(P->sweep, q, Lx, P->npairs, P->npatch));
  take(B_SCODE, P->npairs ? P->sz[B_SIGMA] / 16 : 0);     // one code byte per float4
  take(B_MU, (size_t)P->npairs * plane * sizeof(float));
  take(B_C, pl);
  take(B_L1, pl);
  take(B_L2, pl);
  take(B_BX, pl);
  take(B_W1, pl);
  take(B_W2, pl);
  take(B_F, (size_t)((Lx + 1) / 2) * plane * sizeof(float2));
  take(B_HALO, (size_t)P->sweep.split * Lx * P->sweep.ntiles * P->sweep.halo * q * sizeof(float));
  take(B_CSPLIT, (size_t)(P->sweep.split - 1) * pl);
  if (E_host) {                            // the X iterate and the projected Y_l
    const size_t lowres = (size_t)(p / prm.d) * (q / prm.d) * Lx * sizeof(float);
    take(B_Z, pl);
    take(B_YLE, lowres);
    take(B_YLP, lowres);
  }
  P->ws_bytes = off;
  *out = P;
  return NLPR_OK;
}

SceneDesc static_desc(const Plan& P) {
  SceneDesc d;
  std::memset(&d, 0, sizeof(d));   // padding included: descriptors are compared bytewise
  const nlpr_params& q = P.prm;
  d.p = q.p;
  d.q = q.q;
  d.L = P.Lx;
  d.Lz = q.L;
  d.subspace = P.d_E ? 1 : 0;
  d.E = P.d_E;
  d.Ep = P.d_Ep;
  d.M = P.d_M;
  d.Lh = q.Lh;
  d.d = q.d;
  d.r = q.blur_radius;
  d.K = q.K;
  d.npairs = P.npairs;
  d.npatch = P.npatch;
  d.rows = P.sweep.rows;
  d.ntiles = P.sweep.ntiles;
  d.halo = P.sweep.halo;
  d.psplit = P.sweep.split;
  d.fq_tpl = P.fft.q_tpl;
  d.fq_lpb = P.fft.q_lpb;
  d.fp_tpl = P.fft.p_tpl;
  d.fp_cb = P.fft.p_cb;
  d.init_zero = (q.flags & NLPR_INIT_ZERO) ? 1 : 0;
  d.unweighted = (q.flags & NLPR_UNWEIGHTED) ? 1 : 0;
  d.rho = (float)q.rho;
  d.inv_1prho = (float)(1.0 / (1.0 + q.rho));
  d.mu_scale = (float)(q.lambda / q.rho);
  d.inv_h2 = (q.flags & NLPR_UNWEIGHTED) ? 0.f : (float)(1.0 / (q.h * q.h));
  d.fp = P.fp;
  d.fq = P.fq;
  d.taus = P.d_taus;
  d.invden = P.d_invden;
  d.blur = P.d_blur;
  const int bw = 2 * q.blur_radius + 1;
  d.bsep = P.blur_separable ? P.d_blur + bw * bw : nullptr;
  d.R = P.d_E ? P.d_Rt : P.d_R;
  d.G = P.d_G;
  d.fused = P.d_fia ? 1 : 0;
  d.fia = P.d_fia;
  d.fu = P.d_fu;
  d.fv = P.d_fv;
  d.mon = P.d_mon;
  d.mon_npix = P.d_mon ? pixel_blocks(P) : 0;
  d.mon_nreg = P.d_mon ? monreg_blocks(P) : 0;
  d.rho_d = q.rho;
  d.lam1_d = q.lambda1;
  d.lam_d = q.lambda;
  return d;
}

// ----------------------------------------------------------------------------- batches
void batch_release(Batch& B) {
  for (int k = 0; k < KD_COUNT; ++k) {
    for (Group& g : B.groups[k]) hipFree(g.d_items);
    B.groups[k].clear();
  }
  if (B.upload_ev) hipEventSynchronize(B.upload_ev);
  hipFree(B.d_desc);
  if (B.h_desc) hipHostFree(B.h_desc);
  hipFree(B.d_flag);
  hipFree(B.d_counts);
  if (B.side) {
    hipStreamSynchronize(B.side);
    hipStreamDestroy(B.side);
  }
  if (B.fork_ev) hipEventDestroy(B.fork_ev);
  if (B.join_ev) hipEventDestroy(B.join_ev);
  if (B.upload_ev) hipEventDestroy(B.upload_ev);
  if (B.done_ev) hipEventDestroy(B.done_ev);
  if (B.graph) hipGraphExecDestroy(B.graph);
  for (hipEvent_t e : B.ev_pool) hipEventDestroy(e);
  B.ev_pool.clear();
  for (Plan* P : B.scenes) scene_free(P);
  B.scenes.clear();
  B.d_desc = nullptr;
  B.h_desc = nullptr;
  B.d_flag = nullptr;
  B.d_counts = nullptr;
  B.upload_ev = nullptr;
  B.done_ev = nullptr;
  B.side = nullptr;
  B.fork_ev = nullptr;
  B.join_ev = nullptr;
  B.graph = nullptr;
}

// Work items in the order that gives each XCD a contiguous range of them.  The workgroups
// of a launch go to the 8 XCDs round-robin by workgroup index, each XCD with its own L2, so
// workgroup b runs item start(b % 8) + b / 8, where XCD x owns the next N/8 (+1 for the first
// N mod 8) items.  Neighbouring tiles of one band, whose halos overlap, then share an L2.
std::vector<int2> xcd_order(const std::vector<int2>& items) {
  constexpr int kXcds = 8;
  const int n = (int)items.size(), q = n / kXcds, r = n % kXcds;
  std::vector<int2> out(n);
  for (int b = 0; b < n; ++b) {
    const int x = b % kXcds, s = b / kXcds;
    out[b] = items[x * q + std::min(x, r) + s];
  }
  return out;
}

int add_group(Batch& B, Kind kind, const std::vector<int2>& items, int block, size_t lds, int k0,
              int k1) {
  Group g;
  g.nitems = (int)items.size();
  g.block = block;
  g.lds = lds;
  g.key0 = k0;
  g.key1 = k1;
  if (g.nitems) {
    NLPR_HIP_TRY(hipMalloc(&g.d_items, items.size() * sizeof(int2)));
    NLPR_HIP_TRY(hipMemcpy(g.d_items, items.data(), items.size() * sizeof(int2),
                           hipMemcpyHostToDevice));
  }
  B.groups[kind].push_back(g);
  return NLPR_OK;
}

int block256(const Plan&) { return 256; }
int rows_block(const Plan& P) { return P.fft.q_bs; }
int cols_block(const Plan& P) { return P.fft.p_bs; }
size_t no_lds(const Plan&) { return 0; }

// Work-item tables of every launch kind, descriptors, events.
int batch_build(Batch& B) {
  const int n = (int)B.scenes.size();
  B.base.resize(n);
  size_t off = 0;
  for (int s = 0; s < n; ++s) {
    B.base[s] = off;
    off = align256(off + B.scenes[s]->ws_bytes);
  }
  B.ws_bytes = off;
  auto simple = [&](Kind kind, int (*count)(const Plan&), size_t (*lds)(const Plan&),
                    int (*block)(const Plan&)) -> int {
    std::vector<int2> it;
    size_t l = 0;
    int bs = 256;
    for (int s = 0; s < n; ++s) {
      const Plan& P = *B.scenes[s];
      if (kind == KD_WEIGHTS && P.npairs == 0) continue;
      const int c = count(P);
      for (int i = 0; i < c; ++i) it.push_back(make_int2(s, i));
      l = std::max(l, lds(P));
      bs = std::max(bs, block(P));
    }
    return add_group(B, kind, it, bs, l, 0, 0);
  };
  int rc;
  if ((rc = simple(KD_WEIGHTS, weights_blocks, weights_lds, block256))) return rc;
  if ((rc = simple(KD_PLANE, plane_blocks, no_lds, block256))) return rc;
  for (int cls : {1, 2, 4, 8, kMaxBlurRadius}) {      // blur convolution by radius class
    std::vector<int2> it;
    size_t l = 0;
    for (int s = 0; s < n; ++s) {
      const Plan& P = *B.scenes[s];
      if (conv_class(P.prm.blur_radius) != cls) continue;
      const int c = conv_blocks(P);
      for (int i = 0; i < c; ++i) it.push_back(make_int2(s, i));
      l = std::max(l, conv_lds(P));
    }
    if (!it.empty() && (rc = add_group(B, KD_CONV, xcd_order(it), 256, l, cls, 0))) return rc;
  }
  // per-pixel launches by guide-band class (key0); key1 = threads per pixel, 4 (bands of a
  // pixel split) when the launch covers few pixels in all, else 1
  for (int cls : {1, 4, kMaxLh}) {
    std::vector<int2> it;
    size_t pixels = 0;
    for (int s = 0; s < n; ++s) {
      const Plan& P = *B.scenes[s];
      if (lh_class(P.prm.Lh) != cls) continue;
      pixels += (size_t)P.prm.p * P.prm.q;
      const int c = pixel_blocks(P);
      for (int i = 0; i < c; ++i) it.push_back(make_int2(s, i));
    }
    if (!it.empty() && (rc = add_group(B, KD_PIXEL, it, 256, 0, cls, pixel_split(pixels))))
      return rc;
  }
  // scenes with a subspace basis: low-resolution projections / P1, and Z = X E
  for (Kind kind : {KD_LOWRES, KD_COMPOSE}) {
    std::vector<int2> it;
    for (int s = 0; s < n; ++s) {
      const Plan& P = *B.scenes[s];
      if (!P.d_E) continue;
      const int c = kind == KD_LOWRES ? lowres_blocks(P) : pixel_blocks(P);
      for (int i = 0; i < c; ++i) it.push_back(make_int2(s, i));
    }
    if ((rc = add_group(B, kind, it, 256, 0, 0, 0))) return rc;
  }
  if (B.monitor_every > 0) {
    std::vector<int2> it, sc;
    size_t l = 0;
    for (int s = 0; s < n; ++s) {
      const Plan& P = *B.scenes[s];
      sc.push_back(make_int2(s, 0));
      if (P.npairs == 0) continue;
      const int c = monreg_blocks(P);
      for (int i = 0; i < c; ++i) it.push_back(make_int2(s, i));
      l = std::max(l, monreg_lds(P));
    }
    if ((rc = add_group(B, KD_MONREG, it, 256, l, 0, 0))) return rc;
    if ((rc = add_group(B, KD_SCENE, sc, 256, 0, 0, 0))) return rc;
  }
  if (n == 1 && B.scenes[0]->npairs > 0) {     // reverse mode of a single scene
    const Plan& P = *B.scenes[0];
    std::vector<int2> it;
    const int c = (int)(((size_t)P.npairs * P.prm.p * P.prm.q + 255) / 256);
    for (int i = 0; i < c; ++i) it.push_back(make_int2(0, i));
    if ((rc = add_group(B, KD_MUPLANE, it, 256, 0, 0, 0))) return rc;
    it.clear();
    for (int i = 0; i < weights_bwd_blocks(P); ++i) it.push_back(make_int2(0, i));
    if ((rc = add_group(B, KD_WBWD, it, 256, weights_bwd_lds(P), 0, 0))) return rc;
    if (P.sweep.items == 1 && sweep_bwd_lds(P) <= kMaxSweepLds &&
        (rc = sweep_bwd_prepare(P.prm.K)))
      return rc;
  }
  if ((rc = simple(KD_ROWS, rows_blocks, rows_lds, rows_block))) return rc;
  if ((rc = simple(KD_COLS, cols_blocks, cols_lds, cols_block))) return rc;
  // the sweep: one launch per (patch radius, tile size)
  for (int K = 0; K <= kMaxK; ++K)
    for (int items = 1; items <= 4; items *= 2) {
      std::vector<int2> it;
      size_t l = 0;
      for (int s = 0; s < n; ++s) {
        const Plan& P = *B.scenes[s];
        if (P.npairs == 0 || P.prm.K != K || P.sweep.items != items) continue;
        const int c = sweep_blocks(P);
        for (int i = 0; i < c; ++i) it.push_back(make_int2(s, i));
        l = std::max(l, P.sweep.lds);
      }
      if (it.empty()) continue;
      if ((rc = add_group(B, KD_SWEEP, it, kSweepThreads, l, K, items))) return rc;
      if ((rc = sweep_prepare(K, items))) return rc;
    }
  NLPR_HIP_TRY(hipMalloc(&B.d_desc, n * sizeof(SceneDesc)));
  NLPR_HIP_TRY(hipHostMalloc(&B.h_desc, n * sizeof(SceneDesc)));
  NLPR_HIP_TRY(hipMalloc(&B.d_flag, 256));
  if (B.timing)
    NLPR_HIP_TRY(hipMalloc(&B.d_counts, (size_t)std::max(B.iters, 1) * kCountSlots * kCountStride *
                                            sizeof(unsigned long long)));
  NLPR_HIP_TRY(hipEventCreateWithFlags(&B.upload_ev, hipEventDisableTiming));
  NLPR_HIP_TRY(hipEventCreateWithFlags(&B.done_ev, hipEventDisableTiming));
  size_t pbands = 0;
  bool reg = false;
  for (const Plan* P : B.scenes) {
    pbands += (size_t)P->prm.p * P->prm.q * P->Lx;
    reg = reg || P->npairs > 0;
  }
  if (reg && !B.timing && pbands >= kForkPixelBands) {
    NLPR_HIP_TRY(hipStreamCreateWithFlags(&B.side, hipStreamNonBlocking));
    NLPR_HIP_TRY(hipEventCreateWithFlags(&B.fork_ev, hipEventDisableTiming));
    NLPR_HIP_TRY(hipEventCreateWithFlags(&B.join_ev, hipEventDisableTiming));
  }
  B.uploaded.resize(n);
  B.desc_valid = false;
  return NLPR_OK;
}

// Write the descriptors (sizes, tables, buffers) to the device if they changed.  The pinned
// staging copy is rewritten only after the previous upload from it has completed.  Every
// call that launches work on a plan comes through here first, and its stream waits for the
// device work of the previous call on the plan (done_ev, recorded at the end of each call):
// the previous call's kernels read the device descriptor until they finish, so calls on one
// plan run on the device in the order they were made, whatever streams they use.
int upload_desc(Batch& B, const std::vector<SceneDesc>& descs, hipStream_t s) {
  const size_t n = descs.size();
  NLPR_HIP_TRY(hipStreamWaitEvent(s, B.done_ev, 0));
  if (B.desc_valid && std::memcmp(B.uploaded.data(), descs.data(), n * sizeof(SceneDesc)) == 0)
    return NLPR_OK;
  NLPR_HIP_TRY(hipEventSynchronize(B.upload_ev));
  std::memcpy(B.h_desc, descs.data(), n * sizeof(SceneDesc));
  NLPR_HIP_TRY(hipMemcpyAsync(B.d_desc, B.h_desc, n * sizeof(SceneDesc), hipMemcpyHostToDevice, s));
  NLPR_HIP_TRY(hipEventRecord(B.upload_ev, s));
  std::memcpy(B.uploaded.data(), descs.data(), n * sizeof(SceneDesc));
  B.desc_valid = true;
  return NLPR_OK;
}

// Timing: events bracket each launch group when the batch was created with NLPR_TIMING.
struct StageTimer {
  Batch& B;
  hipStream_t s;
  int stage;
  size_t a = 0;
  bool on = false;
  StageTimer(Batch& b, hipStream_t st, int sg) : B(b), s(st), stage(sg) {
    if (!B.timing || B.ev_used + 2 > B.ev_pool.size()) return;
    a = B.ev_used;
    if (hipEventRecord(B.ev_pool[a], s) == hipSuccess) {
      on = true;
      B.ev_used += 2;
    }
  }
  ~StageTimer() {
    if (!on) return;
    hipEventRecord(B.ev_pool[a + 1], s);
    B.recs.push_back({stage, a, a + 1});
  }
};

int ensure_events(Batch& B) {
  if (!B.timing) return NLPR_OK;
  const size_t need = 2 * (size_t)(7 * std::max(B.iters, 1) + 16);
  while (B.ev_pool.size() < need + B.ev_used) {
    hipEvent_t e;
    NLPR_HIP_TRY(hipEventCreate(&e));
    B.ev_pool.push_back(e);
  }
  return NLPR_OK;
}

// The solve: weights, initial values, then per iteration the X-update, the blur, the
// P/Lambda update, the sweep and the right-hand-side assembly.
int enqueue_solve(Batch& B, bool resume, hipStream_t s) {
  int rc;
  int point = 0;
  bool reg = false, sub = false;
  for (const Plan* P : B.scenes) {
    reg = reg || P->npairs > 0;
    sub = sub || P->d_E != nullptr;
  }
  // fused-S (shared by every scene of a batch): no P1 / Lambda1.  The constant part of
  // every X-update, Xc0 = A^{-1} B^T S^T Y_l / rho, is solved once and added after each
  // solve, so the per-iteration right-hand side W2 + C_reg stays of the size of X.  W1
  // holds Xc0 and L1 serves as scratch.
  const bool fused = (B.flags & NLPR_FUSED_S) != 0;
  const bool check = (B.flags & NLPR_CHECK_FINITE) != 0;
  if (check && (rc = launch_finite_clear(B.d_flag, s))) return rc;
  if (B.d_counts &&
      (rc = launch_zero_u64(B.d_counts, B.iters * kCountSlots * kCountStride, s)))
    return rc;
  if (sub) {
    StageTimer tm(B, s, NLPR_STAGE_INIT);
    if ((rc = launch_project(B, B_YL, B_YLE, B_YLP, s))) return rc;
  }
  {
    StageTimer tm(B, s, NLPR_STAGE_WEIGHTS);
    if ((rc = launch_weights(B, B_YH, B_MU, s))) return rc;
  }
  if (fused) {
    StageTimer tm(B, s, NLPR_STAGE_INIT);
    if ((rc = launch_upsample_zero(B, B_YL, B_L1, s))) return rc;
    if ((rc = launch_conv(B, B_L1, B_W1, true, -1, -1, -1, 0, s))) return rc;
    if ((rc = launch_xsolve(B, B_W1, B_W1, B_F, -1, s))) return rc;
  }
  if (!resume) {
    StageTimer tm(B, s, NLPR_STAGE_INIT);
    // X0 into Z, W2 = P2 + Lambda2 = X0, Lambda = 0, W1 = P1 + Lambda1 = B X0, C = B^T W1 + W2
    // (fused-S: C = W2)
    if ((rc = launch_init(B, B_YL, B_YLP, B_Z, B_L1, B_L2, B_W2, s))) return rc;
    if (fused) {
      if ((rc = launch_conv(B, -1, B_C, false, B_W2, -1, -1, 0, s))) return rc;
    } else {
      if ((rc = launch_conv(B, B_Z, B_W1, false, -1, -1, -1, 0, s))) return rc;
      if ((rc = launch_conv(B, B_W1, B_C, true, B_W2, -1, -1, 0, s))) return rc;
    }
  }
  for (int t = 0; t < B.iters; ++t) {
    const bool mon = B.monitor_every > 0 && ((t + 1) % B.monitor_every == 0 || t + 1 == B.iters);
    {
      StageTimer tm(B, s, NLPR_STAGE_XSOLVE);
      if ((rc = launch_xsolve(B, B_C, B_Z, B_F, fused ? B_W1 : -1, s))) return rc;
    }
    if (check && ((t + 1) % kFiniteEvery == 0 || t + 1 == B.iters) &&
        (rc = launch_finite(B, B_Z, B.d_flag, t + 1, s)))
      return rc;
    // The P-side (blur, P-update, and T = B^T W1 + W2, the part of the right-hand side that
    // does not wait for the sweep, into the BX slot) and the sweep read X and write disjoint
    // buffers.  In a batch with a side stream the P-side forks onto it and joins before the
    // assembly adds the regulariser term, so it runs while the sweep does; a monitor record
    // keeps this iteration on one stream.  C = (B^T W1 + W2) + C_reg either way, with the
    // same additions in the same order.
    const bool fork = B.side != nullptr && !mon;
    const bool tpart = fork && !fused;
    hipStream_t sp = s;
    if (fork) {
      NLPR_HIP_TRY(hipEventRecord(B.fork_ev, s));
      NLPR_HIP_TRY(hipStreamWaitEvent(B.side, B.fork_ev, 0));
      sp = B.side;
    }
    if (!fused || mon) {           // fused-S needs B X only for the monitor's data term
      StageTimer tm(B, sp, NLPR_STAGE_BLUR);
      if ((rc = launch_conv(B, B_Z, B_BX, false, -1, -1, -1, 0, sp))) return rc;
    }
    {
      StageTimer tm(B, sp, NLPR_STAGE_PUPDATE);
      if ((rc = launch_pupdate(B, B_Z, B_BX, B_YL, B_YH, B_L1, B_L2, B_W1, B_W2, B_L1, B_L2, sp)))
        return rc;
      if (sub && (rc = launch_p1_subspace(B, B_BX, B_YLE, B_L1, B_W1, sp))) return rc;
    }
    if (tpart && (rc = launch_conv(B, B_W1, B_BX, true, B_W2, -1, -1, 0, sp))) return rc;
    if (mon) {
      StageTimer tm(B, s, NLPR_STAGE_MONITOR);
      if ((rc = launch_monitor(B, point++, t + 1, s))) return rc;
    }
    if (reg) {
      const bool first = (t == 0 && !resume);
      StageTimer tm(B, s, first ? NLPR_STAGE_SWEEP_FIRST : NLPR_STAGE_SWEEP);
      if ((rc = launch_sweep(B, B_Z, B_MU, B_SIGMA, B_C, B_HALO, first, s, nullptr,
                             B.d_counts ? B.d_counts + (size_t)t * kCountSlots * kCountStride
                                        : nullptr)))
        return rc;
    }
    if (fork) {
      NLPR_HIP_TRY(hipEventRecord(B.join_ev, sp));
      NLPR_HIP_TRY(hipStreamWaitEvent(s, B.join_ev, 0));
    }
    {
      StageTimer tm(B, s, NLPR_STAGE_ASSEMBLE);
      if (tpart) {
        if ((rc = launch_conv(B, -1, B_C, true, B_BX, B_C, B_HALO, 2 | 4, s))) return rc;
      } else if ((rc = launch_conv(B, fused ? -1 : B_W1, B_C, true, B_W2, B_C, B_HALO, 2 | 4,
                                   s))) {
        return rc;
      }
    }
  }
  if (check && B.iters == 0 && (rc = launch_finite(B, B_Z, B.d_flag, 0, s))) return rc;
  if (sub) {
    StageTimer tm(B, s, NLPR_STAGE_INIT);
    if ((rc = launch_compose(B, B_Z, B_OUT, s))) return rc;
  }
  return NLPR_OK;
}

// Descriptor of one scene for a solve: workspace regions, observations and output.
SceneDesc solve_desc(const Plan& P, char* base, const float* Yl, const float* Yh, float* Z) {
  SceneDesc d = static_desc(P);
  for (int k : {B_SIGMA, B_SCODE, B_MU, B_C, B_L1, B_L2, B_BX, B_W1, B_W2, B_F, B_HALO, B_CSPLIT})
    d.buf[k] = base + P.off[k];
  d.buf[B_L1O] = d.buf[B_L1];
  d.buf[B_L2O] = d.buf[B_L2];
  d.buf[B_YL] = const_cast<float*>(Yl);
  d.buf[B_YH] = const_cast<float*>(Yh);
  if (P.d_E) {                       // X lives in the workspace; Z = X E at the end
    d.buf[B_Z] = base + P.off[B_Z];
    d.buf[B_YLE] = base + P.off[B_YLE];
    d.buf[B_YLP] = base + P.off[B_YLP];
    d.buf[B_OUT] = Z;
  } else {
    d.buf[B_Z] = Z;
  }
  d.buf[B_TMP] = base + P.off[B_BX];
  return d;
}

int batch_solve(Batch& B, const float* const* Yl, const float* const* Yh, float* const* Z,
                void* ws, size_t ws_bytes, hipStream_t s, bool ws_is_static = false) {
  const int n = (int)B.scenes.size();
  int rc;
  if (!ws_is_static && (rc = check_device_ptr(ws, "ws"))) return rc;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(NLPR_ERR_INVALID_ARG, "ws must be 256-byte aligned");
  if (ws_bytes < B.ws_bytes)
    return fail(NLPR_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than the required size");
  std::vector<SceneDesc> descs(n);
  for (int i = 0; i < n; ++i) {
    if ((rc = check_device_ptr(Yl[i], "Yl")) || (rc = check_device_ptr(Yh[i], "Yh")) ||
        (rc = check_device_ptr(Z[i], "Z")))
      return rc;
    descs[i] = solve_desc(*B.scenes[i], static_cast<char*>(ws) + B.base[i], Yl[i], Yh[i], Z[i]);
  }
  DeviceGuard dg(B.device);
  if ((rc = ensure_events(B))) return rc;
  if ((rc = upload_desc(B, descs, s))) return rc;
  const bool resume = (B.flags & NLPR_STATE_IN) != 0;
  if (B.use_graph && !B.timing) {
    const uint32_t key = (resume ? 1u : 0u) | ((uint32_t)B.iters << 1) | 0x80000000u;
    if (!B.graph || B.graph_key != key) {
      if (B.graph) {
        hipGraphExecDestroy(B.graph);
        B.graph = nullptr;
      }
      // capture on a private stream (the caller's may be the legacy default stream, which
      // cannot be captured), then launch the instantiated graph on the caller's stream
      hipStream_t cs;
      NLPR_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = enqueue_solve(B, resume, cs);
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
      }
      hipStreamDestroy(cs);
      if (rc || e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        if (rc) return rc;
        return fail(NLPR_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      }
      e = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) {
        B.graph = nullptr;
        return fail(NLPR_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
      B.graph_key = key;
    }
    NLPR_HIP_TRY(hipGraphLaunch(B.graph, s));
  } else {
    if ((rc = enqueue_solve(B, resume, s))) return rc;
  }
  NLPR_HIP_TRY(hipEventRecord(B.done_ev, s));
  B.mon_last = monitor_points(B.iters, B.monitor_every);
  if (B.flags & NLPR_CHECK_FINITE) {
    // the checks ran inside the solve without waiting; read their flag once
    int hflag = 0;
    NLPR_HIP_TRY(hipMemcpyAsync(&hflag, B.d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    NLPR_HIP_TRY(hipStreamSynchronize(s));
    B.nonfinite_iter = hflag == INT_MAX ? -1 : hflag;
    if (B.nonfinite_iter >= 0)
      return fail(NLPR_ERR_NUMERICAL, "NaN or Inf in the iterate X, first found by the check "
                                      "after iteration " + std::to_string(B.nonfinite_iter));
  }
  return NLPR_OK;
}

// ---------------------------------------------------------------------- reverse mode
// Checkpoints, for t = 1 .. T-1: X^t, B X^t and the Lambda1, Lambda2 entering iteration t
// (planes), then the threshold branches of iteration t's sweep (2 bits per dual element).
// Layout: the 4 (T - 1) planes first ([t][X, BX, Lambda1, Lambda2]), then the T - 1 blocks
// of branch codes.
struct GradLayout {
  size_t off[B_COUNT] = {};
  size_t gws_bytes = 0;
  size_t plane_al = 0, code_al = 0, ck_bytes = 0;
  int npix = 0, nw = 0;
};

GradLayout grad_layout(const Plan& P) {
  GradLayout G;
  const size_t pl = (size_t)P.Lx * P.prm.p * P.prm.q * sizeof(float);
  size_t off = 0;
  auto take = [&](int slot, size_t bytes) {
    G.off[slot] = off;
    off = align256(off + std::max<size_t>(bytes, 4));
  };
  for (int k : {B_GC, B_GCP, B_GL1, B_GL2, B_GX, B_GW1, B_GBX, B_GXP, B_GXR}) take(k, pl);
  const size_t mup = (size_t)P.npairs * P.prm.p * P.prm.q * sizeof(float);
  G.npix = pixel_blocks(P);
  G.nw = P.npairs ? weights_bwd_blocks(P) : 0;
  take(B_GSIG, P.sz[B_SIGMA]);
  take(B_GHALO, P.sz[B_HALO]);
  take(B_GMUP, P.npairs ? mubar_partial_elems(P) * sizeof(float) : 4);
  take(B_GMU, mup);
  take(B_GE, mup);
  take(B_GPART, 2 * (size_t)(G.npix + G.nw) * sizeof(double));
  G.gws_bytes = off;
  const int T = P.prm.iters;
  G.plane_al = align256(pl);
  G.code_al = P.npairs ? align256(P.sz[B_SIGMA] / 16) : 0;   // one byte per float4 of Sigma'
  G.ck_bytes = std::max<size_t>(256, (size_t)std::max(T - 1, 0) * (4 * G.plane_al + G.code_al));
  return G;
}

int grad_check(const Batch& B) {
  if (B.scenes.size() != 1) return fail(NLPR_ERR_INVALID_ARG, "reverse mode takes a single scene");
  const Plan& P = *B.scenes[0];
  if (P.d_E) return fail(NLPR_ERR_UNSUPPORTED_SHAPE, "reverse mode is built for E = I");
  if (P.d_fia) return fail(NLPR_ERR_UNSUPPORTED_SHAPE, "reverse mode follows the paper's splitting (no NLPR_FUSED_S)");
  if (B.flags & NLPR_STATE_IN) return fail(NLPR_ERR_INVALID_ARG, "reverse mode starts from the default start (no NLPR_STATE_IN)");
  if (B.iters < 1) return fail(NLPR_ERR_INVALID_ARG, "reverse mode needs iters >= 1");
  if (P.npairs && (P.sweep.items != 1 || sweep_bwd_lds(P) > kMaxSweepLds))
    return fail(NLPR_ERR_UNSUPPORTED_SHAPE,
                "the sweep adjoint needs q <= 1024 and its LDS tile within 160 KiB");
  // the sweep adjoint gives each of its 256 threads one float4 of the tile
  if (P.npairs && (size_t)P.sweep.rows * (P.prm.q / 4) > 256)
    return fail(NLPR_ERR_UNSUPPORTED_SHAPE, "the sweep tile is larger than the adjoint's workgroup");
  return NLPR_OK;
}

// Checkpoint t (1 .. T-1) holds what the reverse step of iteration t reads: plane k = 0 X^t,
// 1 B X^t, 2 Lambda1^{t-1}, 3 Lambda2^{t-1}; then the branch codes of iteration t's sweep.
char* ck_plane(void* ck, const GradLayout& G, int t, int k) {
  return static_cast<char*>(ck) + ((size_t)(t - 1) * 4 + k) * G.plane_al;
}
uint8_t* ck_codes(void* ck, const GradLayout& G, int T, int t) {
  return reinterpret_cast<uint8_t*>(ck) + (size_t)(T - 1) * 4 * G.plane_al +
         (size_t)(t - 1) * G.code_al;
}

// Forward solve that keeps the checkpoints.  Z = X^T equals nlpr_solve's output bit for bit;
// the last iteration stops after its X-update, the only part of it that reaches Z.  Nothing
// is copied: before each iteration the descriptor's slots are re-pointed so that the X-update
// and the blur write X^t and B X^t into checkpoint t, and the P-update reads the Lambda of
// checkpoint t and writes the new Lambda into checkpoint t+1 (the workspace after the last).
// The sweep updates Sigma' in place in the workspace, as in the solve, and writes the branch
// codes of checkpoint t.
int grad_forward(Batch& B, const float* Yl, const float* Yh, float* Z, void* ws, size_t ws_bytes,
                 void* ck, size_t ck_bytes, hipStream_t s) {
  int rc;
  if ((rc = grad_check(B))) return rc;
  const Plan& P = *B.scenes[0];
  const GradLayout G = grad_layout(P);
  if ((rc = check_device_ptr(ws, "ws")) || (rc = check_device_ptr(ck, "ck")) ||
      (rc = check_device_ptr(Yl, "Yl")) || (rc = check_device_ptr(Yh, "Yh")) ||
      (rc = check_device_ptr(Z, "Z")))
    return rc;
  if (reinterpret_cast<uintptr_t>(ws) % 256 || reinterpret_cast<uintptr_t>(ck) % 256)
    return fail(NLPR_ERR_INVALID_ARG, "ws and ck must be 256-byte aligned");
  if (ws_bytes < B.ws_bytes || ck_bytes < G.ck_bytes)
    return fail(NLPR_ERR_WORKSPACE_TOO_SMALL, "workspace or checkpoint buffer too small");
  char* base = static_cast<char*>(ws);
  std::vector<SceneDesc> descs{solve_desc(P, base, Yl, Yh, Z)};
  DeviceGuard dg(B.device);
  if ((rc = upload_desc(B, descs, s))) return rc;
  const int T = B.iters;
  const bool reg = P.npairs > 0;
  B.desc_valid = false;          // the slots below change the device copy
  auto plane = [&](int t, int k) -> void* { return ck_plane(ck, G, t, k); };
  void* wl1 = base + P.off[B_L1];
  void* wl2 = base + P.off[B_L2];
  if ((rc = launch_weights(B, B_YH, B_MU, s))) return rc;
  if (T > 1) {                   // the start's Lambda (zeros) goes into checkpoint 1
    SlotSet st;
    st.add(B_L1, plane(1, 2));
    st.add(B_L2, plane(1, 3));
    if ((rc = launch_set_slots(B, st, s))) return rc;
  }
  if ((rc = launch_init(B, B_YL, B_YLP, B_Z, B_L1, B_L2, B_W2, s))) return rc;
  if ((rc = launch_conv(B, B_Z, B_W1, false, -1, -1, -1, 0, s))) return rc;
  if ((rc = launch_conv(B, B_W1, B_C, true, B_W2, -1, -1, 0, s))) return rc;
  for (int t = 1; t <= T; ++t) {
    if (T > 1) {
      SlotSet st;
      st.add(B_Z, t < T ? plane(t, 0) : static_cast<void*>(Z));
      if (t < T) {
        st.add(B_BX, plane(t, 1));
        st.add(B_L1, plane(t, 2));
        st.add(B_L2, plane(t, 3));
        st.add(B_L1O, t + 1 < T ? plane(t + 1, 2) : wl1);
        st.add(B_L2O, t + 1 < T ? plane(t + 1, 3) : wl2);
      }
      if ((rc = launch_set_slots(B, st, s))) return rc;
    }
    if ((rc = launch_xsolve(B, B_C, B_Z, B_F, -1, s))) return rc;
    if (t == T) break;
    if ((rc = launch_conv(B, B_Z, B_BX, false, -1, -1, -1, 0, s))) return rc;
    if ((rc = launch_pupdate(B, B_Z, B_BX, B_YL, B_YH, B_L1, B_L2, B_W1, B_W2, B_L1O, B_L2O, s)))
      return rc;
    if (reg && (rc = launch_sweep(B, B_Z, B_MU, B_SIGMA, B_C, B_HALO, t == 1, s,
                                  ck_codes(ck, G, T, t))))
      return rc;
    if ((rc = launch_conv(B, B_W1, B_C, true, B_W2, B_C, B_HALO, 2 | 4, s))) return rc;
  }
  NLPR_HIP_TRY(hipEventRecord(B.done_ev, s));
  return NLPR_OK;
}

// Reverse pass: from Z' back through the T iterations (X, B X and the entering Lambda of
// each from its checkpoint), the start and the weights.
int grad_backward(Batch& B, const float* Yl, const float* Yh, const float* dZ, void* ws,
                  size_t ws_bytes, void* ck, size_t ck_bytes, void* gws, size_t gws_bytes,
                  float* dYl, float* dYh, double* dscal, hipStream_t s) {
  int rc;
  if ((rc = grad_check(B))) return rc;
  const Plan& P = *B.scenes[0];
  const GradLayout G = grad_layout(P);
  for (const void* ptr : {(const void*)ws, (const void*)ck, (const void*)gws, (const void*)Yl,
                          (const void*)Yh, (const void*)dZ, (const void*)dYl, (const void*)dYh,
                          (const void*)dscal})
    if ((rc = check_device_ptr(ptr, "reverse-mode buffer"))) return rc;
  if (reinterpret_cast<uintptr_t>(ws) % 256 || reinterpret_cast<uintptr_t>(ck) % 256 ||
      reinterpret_cast<uintptr_t>(gws) % 256)
    return fail(NLPR_ERR_INVALID_ARG, "ws, ck and gws must be 256-byte aligned");
  if (ws_bytes < B.ws_bytes || ck_bytes < G.ck_bytes || gws_bytes < G.gws_bytes)
    return fail(NLPR_ERR_WORKSPACE_TOO_SMALL, "workspace, checkpoint or gradient buffer too small");
  char* base = static_cast<char*>(ws);
  char* gb = static_cast<char*>(gws);
  // X, B X and Lambda of each iteration are read from its checkpoint (slots re-pointed)
  SceneDesc d = solve_desc(P, base, Yl, Yh, reinterpret_cast<float*>(base + P.off[B_W2]));
  for (int k : {B_GC, B_GCP, B_GL1, B_GL2, B_GX, B_GW1, B_GBX, B_GXP, B_GXR, B_GSIG, B_GHALO,
                B_GMUP, B_GMU, B_GE, B_GPART})
    d.buf[k] = gb + G.off[k];
  // C' alternates between two buffers, so that the sweep adjoint of step t still has the C'
  // of step t + 1 (slot B_GCP), from which it rebuilds the Sigma'' that step did not store
  const int T = B.iters;
  char* cbuf[2] = {gb + G.off[B_GC], gb + G.off[B_GCP]};
  d.buf[B_GC] = cbuf[(T - 1) & 1];
  d.buf[B_GCP] = cbuf[T & 1];
  d.buf[B_GZ] = const_cast<float*>(dZ);
  d.buf[B_GYL] = dYl;
  d.buf[B_GYH] = dYh;
  std::vector<SceneDesc> descs{d};
  DeviceGuard dg(B.device);
  if ((rc = upload_desc(B, descs, s))) return rc;
  B.desc_valid = false;          // the checkpoint slots below change the device copy
  const bool reg = P.npairs > 0;
  const int p = P.prm.p, q = P.prm.q, d_ = P.prm.d;
  const size_t pl = (size_t)P.Lx * p * q * sizeof(float);
  NLPR_HIP_TRY(hipMemsetAsync(gb + G.off[B_GL1], 0, pl, s));
  NLPR_HIP_TRY(hipMemsetAsync(gb + G.off[B_GL2], 0, pl, s));
  if (reg)
    NLPR_HIP_TRY(hipMemsetAsync(gb + G.off[B_GMUP], 0, mubar_partial_elems(P) * sizeof(float), s));
  NLPR_HIP_TRY(hipMemsetAsync(gb + G.off[B_GPART], 0, 2 * (size_t)(G.npix + G.nw) * sizeof(double), s));
  NLPR_HIP_TRY(hipMemsetAsync(dYl, 0, (size_t)P.Lx * (p / d_) * (q / d_) * sizeof(float), s));
  NLPR_HIP_TRY(hipMemsetAsync(dYh, 0, (size_t)P.prm.Lh * p * q * sizeof(float), s));
  if ((rc = launch_weights(B, B_YH, B_MU, s))) return rc;
  // Z = X^T = solve(C^{T-1})
  if ((rc = launch_xsolve(B, B_GZ, B_GC, B_F, -1, s))) return rc;
  for (int t = T - 1; t >= 1; --t) {
    SlotSet st;                  // X^t, B X^t and the Lambda entering iteration t; C'
    for (int k = 0; k < 4; ++k) st.add(k == 0 ? B_Z : k == 1 ? B_BX : k == 2 ? B_L1 : B_L2,
                                       ck_plane(ck, G, t, k));
    st.add(B_GC, cbuf[t & 1]);
    st.add(B_GCP, cbuf[(t + 1) & 1]);
    if ((rc = launch_set_slots(B, st, s))) return rc;
    if ((rc = launch_conv(B, B_GC, B_GW1, false, -1, -1, -1, 0, s))) return rc;   // W1' = B C'
    if (reg && (rc = launch_sweep_bwd(B, B_GC, ck_codes(ck, G, T, t), B_GSIG, B_GXR, B_GHALO,
                                      B_GMUP, t + 1 < T ? ck_codes(ck, G, T, t + 1) : nullptr,
                                      B_GCP, s)))
      return rc;
    if ((rc = launch_pupdate_bwd(B, B_Z, B_BX, B_YL, B_YH, B_L1, B_L2, B_GW1, B_GC, B_GL1, B_GL2,
                                 B_GBX, B_GXP, B_GYL, B_GYH, B_GPART, s)))
      return rc;
    // X' = B^T BX' + X'(P-update) + X'(sweep) (+ halo rows)
    if ((rc = launch_conv(B, B_GBX, B_GX, true, B_GXP, B_GXR, B_GHALO, 2, s))) return rc;
    if ((rc = launch_xsolve(B, B_GX, B_GCP, B_F, -1, s))) return rc;   // C' of step t - 1
  }
  if (T > 1) {                   // C' of the start was written into buffer 0
    SlotSet st;
    st.add(B_GC, cbuf[0]);
    st.add(B_GCP, cbuf[1]);
    if ((rc = launch_set_slots(B, st, s))) return rc;
  }
  // start: C^0 = B^T B X0 + X0, X0 = up(Y_l)
  if ((rc = launch_conv(B, B_GC, B_GW1, false, -1, -1, -1, 0, s))) return rc;
  if ((rc = launch_conv(B, B_GW1, B_GX, true, B_GC, -1, -1, 0, s))) return rc;
  if (!(B.flags & NLPR_INIT_ZERO) && (rc = launch_upsample_bwd(B, B_GX, B_GYL, s))) return rc;
  if (reg) {
    if ((rc = launch_mubar_reduce(B, B_GMUP, B_GMU, s))) return rc;
    if ((rc = launch_weights_bwd(B, B_YH, B_GMU, B_GE, B_GPART, 2 * G.npix, s))) return rc;
    if ((rc = launch_yh_bwd(B, B_YH, B_GE, B_GYH, s))) return rc;
  }
  if ((rc = launch_grad_scalars(B, B_GPART, G.npix, G.nw, dscal, s))) return rc;
  NLPR_HIP_TRY(hipEventRecord(B.done_ev, s));
  return NLPR_OK;
}

int batch_stage_time(Batch& B, int stage, double* ms_total, int64_t* launches, int reset) {
  if (!ms_total || !launches) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  if (!B.timing) return fail(NLPR_ERR_NOT_ENABLED, "created without NLPR_TIMING");
  if (stage < 1 || stage >= NLPR_STAGE_COUNT) return fail(NLPR_ERR_INVALID_ARG, "unknown stage");
  DeviceGuard dg(B.device);
  for (const auto& r : B.recs) {
    NLPR_HIP_TRY(hipEventSynchronize(B.ev_pool[r.b]));
    float ms = 0.f;
    NLPR_HIP_TRY(hipEventElapsedTime(&ms, B.ev_pool[r.a], B.ev_pool[r.b]));
    B.acc_ms[r.stage] += ms;
    B.acc_n[r.stage] += 1;
  }
  B.recs.clear();
  B.ev_used = 0;
  *ms_total = B.acc_ms[stage];
  *launches = B.acc_n[stage];
  if (reset) {
    std::fill(std::begin(B.acc_ms), std::end(B.acc_ms), 0.0);
    std::fill(std::begin(B.acc_n), std::end(B.acc_n), int64_t(0));
  }
  return NLPR_OK;
}

int region_of(const Plan& P, int region, size_t* offset, size_t* bytes) {
  static const int slot_of[NLPR_REGION_COUNT] = {B_SIGMA, B_MU, B_C, B_L1, B_L2, B_SCODE};
  if (region < 0 || region >= NLPR_REGION_COUNT) return fail(NLPR_ERR_INVALID_ARG, "unknown workspace region");
  *offset = P.off[slot_of[region]];
  *bytes = P.sz[slot_of[region]];
  return NLPR_OK;
}

int batch_monitor(const Batch& B, int scene, double* trace, int cap, int* n) {
  if (!n || (cap > 0 && !trace)) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  if (cap < 0) return fail(NLPR_ERR_INVALID_ARG, "cap must be >= 0");
  if (scene < 0 || scene >= (int)B.scenes.size()) return fail(NLPR_ERR_INVALID_ARG, "scene out of range");
  if (B.monitor_every <= 0) return fail(NLPR_ERR_NOT_ENABLED, "created with monitor_every == 0");
  const Plan& P = *B.scenes[scene];
  *n = B.mon_last;
  const int k = std::min(cap, B.mon_last);
  if (k <= 0) return NLPR_OK;
  DeviceGuard dg(B.device);
  NLPR_HIP_TRY(hipEventSynchronize(B.done_ev));
  const size_t off = 4 * (size_t)pixel_blocks(P) + (P.npairs ? monreg_blocks(P) : 0);
  NLPR_HIP_TRY(hipMemcpy(trace, P.d_mon + off, (size_t)k * 8 * sizeof(double),
                         hipMemcpyDeviceToHost));
  return NLPR_OK;
}

// Create a batch from scene parameters (n >= 1).
int batch_create(Batch& B, int n, const nlpr_params* params, const float* const* blur,
                 const float* const* R, const float* const* E) {
  if (n < 1 || !params || !blur || !R) return fail(NLPR_ERR_INVALID_ARG, "NULL argument or n < 1");
  const uint32_t bf = params[0].flags & kBatchFlags;
  for (int i = 0; i < n; ++i) {
    if (!blur[i] || !R[i]) return fail(NLPR_ERR_INVALID_ARG, "NULL blur taps or R");
    if ((params[i].flags & kBatchFlags) != bf || params[i].iters != params[0].iters ||
        params[i].monitor_every != params[0].monitor_every)
      return fail(NLPR_ERR_INVALID_ARG,
                  "scenes of a batch must share iters, monitor_every and the flags INIT_ZERO, "
                  "STATE_IN, CHECK_FINITE, TIMING and GRAPH");
    int rc = validate(params[i]);
    if (rc) return rc;
  }
  if (hipGetDevice(&B.device) != hipSuccess) return fail(NLPR_ERR_HIP, "no HIP device");
  B.flags = bf;
  B.iters = params[0].iters;
  B.monitor_every = params[0].monitor_every;
  B.timing = (bf & NLPR_TIMING) != 0;
  B.use_graph = (bf & NLPR_GRAPH) != 0;
  for (int i = 0; i < n; ++i) {
    Plan* P = nullptr;
    int rc = scene_create(params[i], blur[i], R[i], E ? E[i] : nullptr, &P);
    if (rc) {
      batch_release(B);
      return rc;
    }
    B.scenes.push_back(P);
  }
  int rc = batch_build(B);
  if (!rc) rc = ensure_events(B);
  if (rc) batch_release(B);
  return rc;
}

}  // namespace
}  // namespace nlpr

using namespace nlpr;

extern "C" {

const char* nlpr_status_string(int status) {
  switch (status) {
    case NLPR_OK: return "ok";
    case NLPR_ERR_INVALID_ARG: return "invalid argument";
    case NLPR_ERR_UNSUPPORTED_SHAPE: return "unsupported shape";
    case NLPR_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case NLPR_ERR_HIP: return "HIP error";
    case NLPR_ERR_NUMERICAL: return "non-finite values in the result";
    case NLPR_ERR_NOT_ENABLED: return "option not enabled in the plan";
    default: return "unknown status";
  }
}

const char* nlpr_last_error(void) { return g_last_error.c_str(); }

int nlpr_plan_create(const nlpr_params* params, const float* blur_host, const float* R_host,
                     const float* E_host, nlpr_plan** out) {
  if (!params || !blur_host || !R_host || !out) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  int rc = validate(*params);
  if (rc) return rc;
  if ((params->Ls > 0) != (E_host != nullptr))
    return fail(NLPR_ERR_INVALID_ARG, "a basis E must be given exactly when Ls > 0");
  nlpr_plan* h = new (std::nothrow) nlpr_plan();
  if (!h) return fail(NLPR_ERR_INVALID_ARG, "out of host memory");
  rc = batch_create(h->B, 1, params, &blur_host, &R_host, &E_host);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return NLPR_OK;
}

int nlpr_plan_destroy(nlpr_plan* plan) {
  if (!plan) return NLPR_OK;
  DeviceGuard g(plan->B.device);
  batch_release(plan->B);
  delete plan;
  return NLPR_OK;
}

int nlpr_workspace_size(const nlpr_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  *bytes = plan->B.ws_bytes;
  return NLPR_OK;
}

int nlpr_half_window(const nlpr_plan* plan, int32_t* tau, int32_t cap, int32_t* n) {
  if (!plan || !n || (cap > 0 && !tau)) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  const Plan& P = *plan->B.scenes[0];
  *n = P.npairs;
  for (int i = 0; i < std::min(cap, P.npairs); ++i) {
    tau[2 * i] = P.taus[2 * i];
    tau[2 * i + 1] = P.taus[2 * i + 1];
  }
  return NLPR_OK;
}

int nlpr_plan_get_info(const nlpr_plan* plan, nlpr_plan_info* info) {
  if (!plan || !info) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  const Plan& P = *plan->B.scenes[0];
  info->npairs = P.npairs;
  info->npatch = P.npatch;
  info->tile_rows = P.sweep.rows;
  info->ntiles = P.sweep.ntiles;
  info->halo_rows = P.sweep.halo;
  info->blur_separable = P.blur_separable ? 1 : 0;
  info->sweep_split = P.sweep.split;
  info->sigma_elems = P.sz[B_SIGMA] / sizeof(float);
  return NLPR_OK;
}

int nlpr_workspace_region(const nlpr_plan* plan, int region, size_t* offset, size_t* bytes) {
  if (!plan || !offset || !bytes) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  return region_of(*plan->B.scenes[0], region, offset, bytes);
}

int nlpr_solve(nlpr_plan* plan, const float* Yl, const float* Yh, float* Z, void* ws,
               size_t ws_bytes, void* stream) {
  if (!plan) return fail(NLPR_ERR_INVALID_ARG, "plan is NULL");
  return batch_solve(plan->B, &Yl, &Yh, &Z, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------- solve without any allocation
// The workspace of nlpr_solve_noalloc: a file-scope device array.  Each GPU the library runs
// on holds its own copy, at its own address, until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host it is only a stand-in for the
// symbol): it uses the device address that hipGetSymbolAddress returns, looked up once per
// device with that device current and kept below.
static __device__ __align__(256) unsigned char scratch[NLPR_NOALLOC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev`, which must be the current device.
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return fail(NLPR_ERR_HIP, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(NLPR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                    hipGetErrorString(e));
    if (reinterpret_cast<uintptr_t>(ptr) % 256)
      return fail(NLPR_ERR_HIP, "the static workspace is not 256-byte aligned");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NLPR_OK;
}
}  // namespace

int nlpr_solve_noalloc(nlpr_plan* plan, const float* Yl, const float* Yh, float* Z,
                       void* stream) {
  if (!plan) return fail(NLPR_ERR_INVALID_ARG, "plan is NULL");
  Batch& B = plan->B;
  if (B.ws_bytes > NLPR_NOALLOC_WORKSPACE_BYTES)
    return fail(NLPR_ERR_WORKSPACE_TOO_SMALL,
                "nlpr_solve_noalloc: the plan needs a workspace of " + std::to_string(B.ws_bytes) +
                    " bytes, more than the static workspace of " +
                    std::to_string((size_t)NLPR_NOALLOC_WORKSPACE_BYTES) +
                    " bytes; use nlpr_solve with a caller workspace");
  if (B.flags & (NLPR_STATE_IN | NLPR_GRAPH | NLPR_TIMING))
    return fail(NLPR_ERR_INVALID_ARG,
                "nlpr_solve_noalloc takes plans without NLPR_STATE_IN, NLPR_GRAPH and NLPR_TIMING");
  DeviceGuard dg(B.device);
  void* ws = nullptr;
  int rc = scratch_address(B.device, &ws);
  if (rc) return rc;
  return batch_solve(B, &Yl, &Yh, &Z, ws, NLPR_NOALLOC_WORKSPACE_BYTES,
                     static_cast<hipStream_t>(stream), true);
}

int nlpr_sigma_expand(const nlpr_plan* plan, const float* sigma, const void* codes,
                      const float* mu, int32_t c0, int32_t c1, float* out, void* stream) {
  if (!plan || !sigma || !codes || !mu || !out) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  const Batch& B = plan->B;
  const Plan& P = *B.scenes[0];
  if (c0 < 0 || c1 > P.Lx || c0 > c1) return fail(NLPR_ERR_INVALID_ARG, "bad band range");
  if (P.npairs == 0) return NLPR_OK;
  int rc;
  for (const void* ptr : {(const void*)sigma, codes, (const void*)mu, (const void*)out})
    if ((rc = check_device_ptr(ptr, "sigma expand buffer"))) return rc;
  DeviceGuard dg(B.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the kernel reads sizes only (descriptor 0): wait for the plan's previous work as any call
  NLPR_HIP_TRY(hipStreamWaitEvent(s, B.done_ev, 0));
  if (!B.desc_valid) {
    std::vector<SceneDesc> descs{static_desc(P)};
    if ((rc = upload_desc(const_cast<Batch&>(B), descs, s))) return rc;
  }
  if ((rc = launch_sigma_expand(B, sigma, static_cast<const uint8_t*>(codes), mu, c0, c1 - c0,
                                out, s)))
    return rc;
  NLPR_HIP_TRY(hipEventRecord(B.done_ev, s));   // later calls on the plan wait for the reads
  return NLPR_OK;
}

int nlpr_sweep_counts(const nlpr_plan* plan, int64_t* counts, int32_t cap, int32_t* n) {
  if (!plan || !n) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  const Batch& B = plan->B;
  if (!B.timing) return fail(NLPR_ERR_NOT_ENABLED, "created without NLPR_TIMING");
  *n = B.scenes[0]->npairs ? B.iters : 0;
  if (!counts || cap <= 0 || *n == 0) return NLPR_OK;
  DeviceGuard dg(B.device);
  NLPR_HIP_TRY(hipEventSynchronize(B.done_ev));
  const size_t per = (size_t)kCountSlots * kCountStride;
  std::vector<unsigned long long> h(B.iters * per);
  NLPR_HIP_TRY(hipMemcpy(h.data(), B.d_counts, h.size() * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost));
  for (int i = 0; i < std::min(cap, *n); ++i) {
    unsigned long long sum = 0;
    for (int k = 0; k < kCountSlots; ++k) sum += h[i * per + (size_t)k * kCountStride];
    counts[i] = (int64_t)sum;
  }
  return NLPR_OK;
}

int nlpr_nonfinite_iteration(const nlpr_plan* plan, int32_t* iter) {
  if (!plan || !iter) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  if (!(plan->B.flags & NLPR_CHECK_FINITE))
    return fail(NLPR_ERR_NOT_ENABLED, "created without NLPR_CHECK_FINITE");
  *iter = plan->B.nonfinite_iter;
  return NLPR_OK;
}

int nlpr_monitor(const nlpr_plan* plan, double* trace, int32_t cap, int32_t* n) {
  if (!plan) return fail(NLPR_ERR_INVALID_ARG, "plan is NULL");
  return batch_monitor(plan->B, 0, trace, cap, n);
}

int nlpr_grad_sizes(const nlpr_plan* plan, size_t* ck_bytes, size_t* gws_bytes) {
  if (!plan || !ck_bytes || !gws_bytes) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  int rc = grad_check(plan->B);
  if (rc) return rc;
  const GradLayout G = grad_layout(*plan->B.scenes[0]);
  *ck_bytes = G.ck_bytes;
  *gws_bytes = G.gws_bytes;
  return NLPR_OK;
}

int nlpr_forward(nlpr_plan* plan, const float* Yl, const float* Yh, float* Z, void* ws,
                 size_t ws_bytes, void* ck, size_t ck_bytes, void* stream) {
  if (!plan) return fail(NLPR_ERR_INVALID_ARG, "plan is NULL");
  return grad_forward(plan->B, Yl, Yh, Z, ws, ws_bytes, ck, ck_bytes,
                      static_cast<hipStream_t>(stream));
}

int nlpr_backward(nlpr_plan* plan, const float* Yl, const float* Yh, const float* dZ, void* ws,
                  size_t ws_bytes, void* ck, size_t ck_bytes, void* gws, size_t gws_bytes,
                  float* dYl, float* dYh, double* dscal, void* stream) {
  if (!plan) return fail(NLPR_ERR_INVALID_ARG, "plan is NULL");
  return grad_backward(plan->B, Yl, Yh, dZ, ws, ws_bytes, ck, ck_bytes, gws, gws_bytes, dYl, dYh,
                       dscal, static_cast<hipStream_t>(stream));
}

int nlpr_debug_stage(nlpr_plan* plan, int stage, void* const* bufs, int32_t nbufs, void* stream) {
  if (!plan || !bufs) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  Batch& B = plan->B;
  const Plan& P = *B.scenes[0];
  static const int need[NLPR_STAGE_COUNT] = {0, 2, 3, 2, 2, 8, 5, 5, 4, 7, 0};
  if (stage < 1 || stage >= NLPR_STAGE_COUNT) return fail(NLPR_ERR_INVALID_ARG, "unknown stage");
  if (stage == NLPR_STAGE_MONITOR)
    return fail(NLPR_ERR_INVALID_ARG, "the monitor has no per-stage entry point");
  if (nbufs < need[stage]) return fail(NLPR_ERR_INVALID_ARG, "too few buffers for the stage");
  int rc;
  for (int i = 0; i < need[stage]; ++i)
    if ((rc = check_device_ptr(bufs[i], "stage buffer"))) return rc;
  if (P.d_E && (stage == NLPR_STAGE_INIT || stage == NLPR_STAGE_PUPDATE))
    return fail(NLPR_ERR_UNSUPPORTED_SHAPE, "the INIT and PUPDATE stages take no subspace basis");
  if (P.d_fia && stage == NLPR_STAGE_INIT)
    return fail(NLPR_ERR_UNSUPPORTED_SHAPE, "the INIT stage is for the paper's splitting");
  DeviceGuard dg(B.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  SceneDesc d = static_desc(P);
  auto put = [&](int slot, int i) { d.buf[slot] = bufs[i]; };
  auto scratch = [&](int slot, int wsi, int region) {
    d.buf[slot] = static_cast<char*>(bufs[wsi]) + P.off[region];
  };
  std::vector<SceneDesc> descs(1);
  auto run = [&](auto&& body) -> int {
    descs[0] = d;
    int r2 = upload_desc(B, descs, s);
    if (r2) return r2;
    if ((r2 = body())) return r2;
    NLPR_HIP_TRY(hipEventRecord(B.done_ev, s));
    return NLPR_OK;
  };
  switch (stage) {
    case NLPR_STAGE_WEIGHTS:
      put(B_YH, 0); put(B_MU, 1);
      return run([&] { return launch_weights(B, B_YH, B_MU, s); });
    case NLPR_STAGE_XSOLVE:
      put(B_C, 0); put(B_Z, 1); scratch(B_F, 2, B_F);
      return run([&] { return launch_xsolve(B, B_C, B_Z, B_F, -1, s); });
    case NLPR_STAGE_BLUR:
    case NLPR_STAGE_BLUR_T:
      put(B_Z, 0); put(B_BX, 1);
      return run([&] { return launch_conv(B, B_Z, B_BX, stage == NLPR_STAGE_BLUR_T, -1, -1, -1, 0, s); });
    case NLPR_STAGE_PUPDATE:
      put(B_Z, 0); put(B_BX, 1); put(B_YL, 2); put(B_YH, 3); put(B_L1, 4); put(B_L2, 5);
      put(B_W1, 6); put(B_W2, 7);
      return run([&] {
        return launch_pupdate(B, B_Z, B_BX, B_YL, B_YH, B_L1, B_L2, B_W1, B_W2, B_L1, B_L2, s);
      });
    case NLPR_STAGE_SWEEP:
    case NLPR_STAGE_SWEEP_FIRST:
      // Creg = the sweep's own-tile part (scratch TMP) + the folded halo rows, assembled by
      // the B^T kernel over a zero image
      put(B_Z, 0); put(B_MU, 1); put(B_SIGMA, 2); put(B_C, 3);
      scratch(B_SCODE, 4, B_SCODE);
      scratch(B_HALO, 4, B_HALO);
      scratch(B_CSPLIT, 4, B_CSPLIT);
      scratch(B_W1, 4, B_W1);
      scratch(B_TMP, 4, B_BX);
      return run([&] {
        int r2;
        if (P.npairs == 0) return launch_fill(B, B_C, s);
        if ((r2 = launch_sweep(B, B_Z, B_MU, B_SIGMA, B_TMP, B_HALO,
                               stage == NLPR_STAGE_SWEEP_FIRST, s)))
          return r2;
        if ((r2 = launch_fill(B, B_W1, s))) return r2;
        return launch_conv(B, B_W1, B_C, true, B_TMP, -1, B_HALO, 1 | 4, s);
      });
    case NLPR_STAGE_ASSEMBLE:
      put(B_W1, 0); put(B_W2, 1); put(B_TMP, 2); put(B_C, 3);
      return run([&] { return launch_conv(B, B_W1, B_C, true, B_W2, B_TMP, -1, 0, s); });
    case NLPR_STAGE_INIT:
      put(B_YL, 0); put(B_Z, 1); put(B_W1, 2); put(B_W2, 3); put(B_L1, 4); put(B_L2, 5);
      put(B_C, 6);
      return run([&] {
        int r2;
        if ((r2 = launch_init(B, B_YL, B_YLP, B_Z, B_L1, B_L2, B_W2, s))) return r2;
        if ((r2 = launch_conv(B, B_Z, B_W1, false, -1, -1, -1, 0, s))) return r2;
        return launch_conv(B, B_W1, B_C, true, B_W2, -1, -1, 0, s);
      });
    default:
      return fail(NLPR_ERR_INVALID_ARG, "unknown stage");
  }
}

int nlpr_stage_time(nlpr_plan* plan, int stage, double* ms_total, int64_t* launches, int reset) {
  if (!plan) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  return batch_stage_time(plan->B, stage, ms_total, launches, reset);
}

// ------------------------------------------------------------------------------ batch
int nlpr_batch_create(int32_t n, const nlpr_params* params, const float* const* blur_host,
                      const float* const* R_host, const float* const* E_host, nlpr_batch** out) {
  if (!out) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  nlpr_batch* h = new (std::nothrow) nlpr_batch();
  if (!h) return fail(NLPR_ERR_INVALID_ARG, "out of host memory");
  int rc = batch_create(h->B, n, params, blur_host, R_host, E_host);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return NLPR_OK;
}

int nlpr_batch_monitor(const nlpr_batch* batch, int32_t scene, double* trace, int32_t cap,
                       int32_t* n) {
  if (!batch) return fail(NLPR_ERR_INVALID_ARG, "batch is NULL");
  return batch_monitor(batch->B, scene, trace, cap, n);
}

int nlpr_batch_destroy(nlpr_batch* batch) {
  if (!batch) return NLPR_OK;
  DeviceGuard g(batch->B.device);
  batch_release(batch->B);
  delete batch;
  return NLPR_OK;
}

int nlpr_stream_rmw(void* buf, size_t bytes, void* stream) {
  int rc = check_device_ptr(buf, "buf");
  if (rc) return rc;
  if (reinterpret_cast<uintptr_t>(buf) % 16 || bytes % 16)
    return fail(NLPR_ERR_INVALID_ARG, "buf must be 16-byte aligned and bytes a multiple of 16");
  if (bytes / 16 > (size_t)0x7fffffff * 256)
    return fail(NLPR_ERR_INVALID_ARG, "bytes exceeds 2^31 * 4096");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, buf) != hipSuccess) return fail(NLPR_ERR_HIP, "hipPointerGetAttributes failed");
  DeviceGuard g(attr.device);
  return launch_stream_rmw(static_cast<float*>(buf), bytes / 16, static_cast<hipStream_t>(stream));
}

int nlpr_stream_chunks(void* buf, size_t buf_bytes, size_t chunk_bytes, int32_t nchunks,
                       int32_t bands, int32_t planes, size_t lds_bytes, void* stream) {
  int rc = check_device_ptr(buf, "buf");
  if (rc) return rc;
  if (reinterpret_cast<uintptr_t>(buf) % 16) return fail(NLPR_ERR_INVALID_ARG, "buf must be 16-byte aligned");
  if (planes < 1 || planes > 8) return fail(NLPR_ERR_INVALID_ARG, "planes must lie in [1, 8]");
  if (chunk_bytes == 0 || chunk_bytes % ((size_t)4096 * planes))
    return fail(NLPR_ERR_INVALID_ARG, "chunk_bytes must be a positive multiple of 4096 * planes");
  if (bands < 1 || nchunks < 1 || nchunks % bands)
    return fail(NLPR_ERR_INVALID_ARG, "nchunks must be a positive multiple of bands");
  if (chunk_bytes > buf_bytes / (size_t)nchunks)
    return fail(NLPR_ERR_INVALID_ARG, "nchunks * chunk_bytes exceeds buf_bytes");
  if (lds_bytes > kMaxSweepLds) return fail(NLPR_ERR_INVALID_ARG, "lds_bytes exceeds 160 KiB");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, buf) != hipSuccess) return fail(NLPR_ERR_HIP, "hipPointerGetAttributes failed");
  DeviceGuard g(attr.device);
  return launch_stream_chunks(static_cast<float*>(buf), chunk_bytes / 16, nchunks, bands, planes,
                              lds_bytes, static_cast<hipStream_t>(stream));
}

int nlpr_batch_workspace_size(const nlpr_batch* batch, size_t* bytes) {
  if (!batch || !bytes) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  *bytes = batch->B.ws_bytes;
  return NLPR_OK;
}

int nlpr_batch_region(const nlpr_batch* batch, int32_t scene, int region, size_t* offset,
                      size_t* bytes) {
  if (!batch || !offset || !bytes) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  const Batch& B = batch->B;
  if (scene < 0 || scene >= (int)B.scenes.size()) return fail(NLPR_ERR_INVALID_ARG, "scene index out of range");
  int rc = region_of(*B.scenes[scene], region, offset, bytes);
  if (!rc) *offset += B.base[scene];
  return rc;
}

int nlpr_batch_solve(nlpr_batch* batch, const float* const* Yl, const float* const* Yh,
                     float* const* Z, void* ws, size_t ws_bytes, void* stream) {
  if (!batch || !Yl || !Yh || !Z) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  return batch_solve(batch->B, Yl, Yh, Z, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

int nlpr_batch_stage_time(nlpr_batch* batch, int stage, double* ms_total, int64_t* launches,
                          int reset) {
  if (!batch) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  return batch_stage_time(batch->B, stage, ms_total, launches, reset);
}

}  // extern "C"
