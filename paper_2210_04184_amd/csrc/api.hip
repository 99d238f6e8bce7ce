// C ABI of libnlpr: plan creation, workspace layout, the ADMM solve loop, per-stage entry
// points for testing, and stage timing.  See include/nlpr.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "nlpr_internal.h"

struct nlpr_plan {
  nlpr::Plan P;
};

namespace nlpr {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

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

void free_plan(Plan& P) {
  hipFree(P.d_taus);
  hipFree(P.d_invden);
  hipFree(P.d_tw_p);
  hipFree(P.d_tw_q);
  hipFree(P.d_blur);
  hipFree(P.d_R);
  hipFree(P.d_G);
  for (hipEvent_t e : P.ev_pool) hipEventDestroy(e);
  P.ev_pool.clear();
}

int validate(const nlpr_params& q) {
  auto bad = [](const std::string& m) { return fail(NLPR_ERR_UNSUPPORTED_SHAPE, m); };
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

// Timing: events bracket each launch group when the plan was created with NLPR_TIMING.
struct StageTimer {
  Plan& P;
  hipStream_t s;
  int stage;
  size_t a = 0;
  bool on = false;
  StageTimer(Plan& p, hipStream_t st, int sg) : P(p), s(st), stage(sg) {
    if (!P.timing || P.ev_used + 2 > P.ev_pool.size()) return;
    a = P.ev_used;
    if (hipEventRecord(P.ev_pool[a], s) == hipSuccess) {
      on = true;
      P.ev_used += 2;
    }
  }
  ~StageTimer() {
    if (!on) return;
    hipEventRecord(P.ev_pool[a + 1], s);
    P.recs.push_back({stage, a, a + 1});
  }
};

int ensure_events(Plan& P) {
  if (!P.timing) return NLPR_OK;
  const size_t need = 2 * (size_t)(6 * std::max(P.prm.iters, 1) + 16);
  while (P.ev_pool.size() < need + P.ev_used) {
    hipEvent_t e;
    NLPR_HIP_TRY(hipEventCreate(&e));
    P.ev_pool.push_back(e);
  }
  return NLPR_OK;
}

template <typename T>
T* region(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
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
  if (E_host) return fail(NLPR_ERR_UNSUPPORTED_SHAPE, "a subspace basis E is not supported (E must be NULL)");
  int rc = validate(*params);
  if (rc) return rc;
  nlpr_plan* h = new (std::nothrow) nlpr_plan();
  if (!h) return fail(NLPR_ERR_INVALID_ARG, "out of host memory");
  Plan& P = h->P;
  P.prm = *params;
  P.timing = (params->flags & NLPR_TIMING) != 0;
  if (hipGetDevice(&P.device) != hipSuccess) {
    delete h;
    return fail(NLPR_ERR_HIP, "no HIP device");
  }
  const int p = P.prm.p, q = P.prm.q, L = P.prm.L, Lh = P.prm.Lh, r = P.prm.blur_radius;
  // W+ in storage order: (0, 1..S), then tau1 = 1..S with tau2 = -S..S
  if (P.prm.flags & NLPR_LOCAL_WINDOW) {
    P.taus = {0, 1, 1, 0};
  } else {
    const int S = P.prm.Sw;
    for (int b = 1; b <= S; ++b) { P.taus.push_back(0); P.taus.push_back(b); }
    for (int a = 1; a <= S; ++a)
      for (int b = -S; b <= S; ++b) { P.taus.push_back(a); P.taus.push_back(b); }
  }
  P.npairs = (int)P.taus.size() / 2;
  P.npatch = (2 * P.prm.K + 1) * (2 * P.prm.K + 1);
  int hrows = 0;
  for (int n = 0; n < P.npairs; ++n) hrows = std::max(hrows, P.taus[2 * n]);
  factor_23(p, P.fp);
  factor_23(q, P.fq);
  P.sweep = choose_sweep_shape(p, q, P.prm.K, hrows);

  auto cleanup = [&](int code) {
    free_plan(P);
    delete h;
    return code;
  };
  const size_t plane = (size_t)p * q;
  if (hipMalloc(&P.d_taus, std::max<size_t>(1, P.npairs) * sizeof(int2)) != hipSuccess ||
      hipMalloc(&P.d_invden, plane * sizeof(float)) != hipSuccess ||
      hipMalloc(&P.d_tw_p, p * sizeof(float2)) != hipSuccess ||
      hipMalloc(&P.d_tw_q, q * sizeof(float2)) != hipSuccess ||
      hipMalloc(&P.d_blur, (2 * r + 1) * (2 * r + 1) * sizeof(float)) != hipSuccess ||
      hipMalloc(&P.d_R, (size_t)L * Lh * sizeof(float)) != hipSuccess ||
      hipMalloc(&P.d_G, (size_t)Lh * Lh * sizeof(float)) != hipSuccess) {
    set_error("hipMalloc of plan tables failed");
    return cleanup(NLPR_ERR_HIP);
  }
  P.fp.tw = P.d_tw_p;
  P.fq.tw = P.d_tw_q;
  if (P.npairs &&
      hipMemcpy(P.d_taus, P.taus.data(), P.npairs * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("upload of the window failed");
    return cleanup(NLPR_ERR_HIP);
  }
  if (hipMemcpy(P.d_blur, blur_host, (2 * r + 1) * (2 * r + 1) * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P.d_R, R_host, (size_t)L * Lh * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("upload of blur taps / R failed");
    return cleanup(NLPR_ERR_HIP);
  }
  rc = launch_precompute(P, nullptr);
  if (rc) return cleanup(rc);
  if (hipDeviceSynchronize() != hipSuccess) {
    set_error("plan precompute failed");
    return cleanup(NLPR_ERR_HIP);
  }
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  P.sz_plane = plane * L * sizeof(float);
  P.sz_sigma = sweep_sigma_bytes(P.sweep, q, L, P.npairs, P.npatch);
  P.sz_mu = (size_t)P.npairs * plane * sizeof(float);
  P.sz_F = (size_t)((L + 1) / 2) * plane * sizeof(float2);
  P.sz_halo = (size_t)L * P.sweep.ntiles * P.sweep.halo * q * sizeof(float);
  P.off_sigma = take(P.sz_sigma);
  P.off_mu = take(P.sz_mu);
  P.off_C = take(P.sz_plane);
  P.off_L1 = take(P.sz_plane);
  P.off_L2 = take(P.sz_plane);
  P.off_BX = take(P.sz_plane);
  P.off_W1 = take(P.sz_plane);
  P.off_W2 = take(P.sz_plane);
  P.off_F = take(P.sz_F);
  P.off_halo = take(std::max<size_t>(P.sz_halo, 4));
  P.off_flag = take(256);
  P.ws_bytes = off;
  if (int e = ensure_events(P)) return cleanup(e);
  *out = h;
  return NLPR_OK;
}

int nlpr_plan_destroy(nlpr_plan* plan) {
  if (!plan) return NLPR_OK;
  DeviceGuard g(plan->P.device);
  free_plan(plan->P);
  delete plan;
  return NLPR_OK;
}

int nlpr_workspace_size(const nlpr_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  *bytes = plan->P.ws_bytes;
  return NLPR_OK;
}

int nlpr_half_window(const nlpr_plan* plan, int32_t* tau, int32_t cap, int32_t* n) {
  if (!plan || !n || (cap > 0 && !tau)) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  const Plan& P = plan->P;
  *n = P.npairs;
  for (int i = 0; i < std::min(cap, P.npairs); ++i) {
    tau[2 * i] = P.taus[2 * i];
    tau[2 * i + 1] = P.taus[2 * i + 1];
  }
  return NLPR_OK;
}

int nlpr_plan_get_info(const nlpr_plan* plan, nlpr_plan_info* info) {
  if (!plan || !info) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  const Plan& P = plan->P;
  info->npairs = P.npairs;
  info->npatch = P.npatch;
  info->tile_rows = P.sweep.rows;
  info->ntiles = P.sweep.ntiles;
  info->halo_rows = P.sweep.halo;
  info->reserved = 0;
  info->sigma_elems = P.sz_sigma / sizeof(float);
  return NLPR_OK;
}

int nlpr_workspace_region(const nlpr_plan* plan, int region, size_t* offset, size_t* bytes) {
  if (!plan || !offset || !bytes) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  const Plan& P = plan->P;
  switch (region) {
    case NLPR_REGION_SIGMA: *offset = P.off_sigma; *bytes = P.sz_sigma; break;
    case NLPR_REGION_MU: *offset = P.off_mu; *bytes = P.sz_mu; break;
    case NLPR_REGION_C: *offset = P.off_C; *bytes = P.sz_plane; break;
    case NLPR_REGION_LAMBDA1: *offset = P.off_L1; *bytes = P.sz_plane; break;
    case NLPR_REGION_LAMBDA2: *offset = P.off_L2; *bytes = P.sz_plane; break;
    default: return fail(NLPR_ERR_INVALID_ARG, "unknown workspace region");
  }
  return NLPR_OK;
}

int nlpr_solve(nlpr_plan* plan, const float* Yl, const float* Yh, float* Z, void* ws,
               size_t ws_bytes, void* stream) {
  if (!plan) return fail(NLPR_ERR_INVALID_ARG, "plan is NULL");
  Plan& P = plan->P;
  int rc;
  if ((rc = check_device_ptr(Yl, "Yl")) || (rc = check_device_ptr(Yh, "Yh")) ||
      (rc = check_device_ptr(Z, "Z")) || (rc = check_device_ptr(ws, "ws")))
    return rc;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(NLPR_ERR_INVALID_ARG, "ws must be 256-byte aligned");
  if (ws_bytes < P.ws_bytes)
    return fail(NLPR_ERR_WORKSPACE_TOO_SMALL, "workspace smaller than nlpr_workspace_size()");
  DeviceGuard dg(P.device);
  if ((rc = ensure_events(P))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* sigma = region<float>(ws, P.off_sigma);
  float* mu = region<float>(ws, P.off_mu);
  float* C = region<float>(ws, P.off_C);
  float* L1 = region<float>(ws, P.off_L1);
  float* L2 = region<float>(ws, P.off_L2);
  float* BX = region<float>(ws, P.off_BX);
  float* W1 = region<float>(ws, P.off_W1);
  float* W2 = region<float>(ws, P.off_W2);
  float2* F = region<float2>(ws, P.off_F);
  float* halo = region<float>(ws, P.off_halo);
  const bool resume = (P.prm.flags & NLPR_STATE_IN) != 0;
  const bool reg = P.npairs > 0;
  {
    StageTimer tm(P, s, NLPR_STAGE_WEIGHTS);
    if ((rc = launch_weights(P, Yh, mu, s))) return rc;
  }
  if (!resume) {
    StageTimer tm(P, s, NLPR_STAGE_INIT);
    // X0 into Z, W2 = P2 + Lambda2 = X0, Lambda = 0, W1 = P1 + Lambda1 = B X0, C = B^T W1 + W2
    if ((rc = launch_init(P, Yl, Z, L1, L2, W2, s))) return rc;
    if ((rc = launch_conv(P, Z, W1, false, nullptr, nullptr, nullptr, s))) return rc;
    if ((rc = launch_conv(P, W1, C, true, W2, nullptr, nullptr, s))) return rc;
  }
  for (int t = 0; t < P.prm.iters; ++t) {
    {
      StageTimer tm(P, s, NLPR_STAGE_XSOLVE);
      if ((rc = launch_xsolve(P, C, Z, F, s))) return rc;
    }
    {
      StageTimer tm(P, s, NLPR_STAGE_BLUR);
      if ((rc = launch_conv(P, Z, BX, false, nullptr, nullptr, nullptr, s))) return rc;
    }
    {
      StageTimer tm(P, s, NLPR_STAGE_PUPDATE);
      if ((rc = launch_pupdate(P, Z, BX, Yl, Yh, L1, L2, W1, W2, s))) return rc;
    }
    if (reg) {
      const bool first = (t == 0 && !resume);
      StageTimer tm(P, s, first ? NLPR_STAGE_SWEEP_FIRST : NLPR_STAGE_SWEEP);
      if ((rc = launch_sweep(P, Z, mu, sigma, C, halo, first, s))) return rc;
    }
    {
      StageTimer tm(P, s, NLPR_STAGE_ASSEMBLE);
      if ((rc = launch_conv(P, W1, C, true, W2, reg ? C : nullptr, reg ? halo : nullptr, s)))
        return rc;
    }
  }
  if (P.prm.flags & NLPR_CHECK_FINITE) {
    int* flag = region<int>(ws, P.off_flag);
    if ((rc = launch_check_finite(P, Z, flag, s))) return rc;
    int hflag = 0;
    NLPR_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    NLPR_HIP_TRY(hipStreamSynchronize(s));
    if (hflag) return fail(NLPR_ERR_NUMERICAL, "NaN or Inf in Z");
  }
  return NLPR_OK;
}

int nlpr_debug_stage(nlpr_plan* plan, int stage, void* const* bufs, int32_t nbufs, void* stream) {
  if (!plan || !bufs) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  Plan& P = plan->P;
  static const int need[NLPR_STAGE_COUNT] = {0, 2, 3, 2, 2, 8, 5, 5, 4, 7};
  if (stage < 1 || stage >= NLPR_STAGE_COUNT) return fail(NLPR_ERR_INVALID_ARG, "unknown stage");
  if (nbufs < need[stage]) return fail(NLPR_ERR_INVALID_ARG, "too few buffers for the stage");
  int rc;
  for (int i = 0; i < need[stage]; ++i)
    if ((rc = check_device_ptr(bufs[i], "stage buffer"))) return rc;
  DeviceGuard dg(P.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto f = [&](int i) { return static_cast<float*>(bufs[i]); };
  switch (stage) {
    case NLPR_STAGE_WEIGHTS:
      return launch_weights(P, f(0), f(1), s);
    case NLPR_STAGE_XSOLVE:
      return launch_xsolve(P, f(0), f(1), region<float2>(bufs[2], P.off_F), s);
    case NLPR_STAGE_BLUR:
      return launch_conv(P, f(0), f(1), false, nullptr, nullptr, nullptr, s);
    case NLPR_STAGE_BLUR_T:
      return launch_conv(P, f(0), f(1), true, nullptr, nullptr, nullptr, s);
    case NLPR_STAGE_PUPDATE:
      return launch_pupdate(P, f(0), f(1), f(2), f(3), f(4), f(5), f(6), f(7), s);
    case NLPR_STAGE_SWEEP:
    case NLPR_STAGE_SWEEP_FIRST: {
      if (P.npairs == 0) {
        NLPR_HIP_TRY(hipMemsetAsync(f(3), 0, P.sz_plane, s));
        return NLPR_OK;
      }
      float* halo = region<float>(bufs[4], P.off_halo);
      float* tmp = region<float>(bufs[4], P.off_BX);
      if ((rc = launch_sweep(P, f(0), f(1), f(2), tmp, halo, stage == NLPR_STAGE_SWEEP_FIRST, s)))
        return rc;
      // Creg = own-tile part + halo fold: a conv with a zero kernel would do it; use the
      // assembly kernel on zero W1 instead (W1 region of the scratch workspace).
      float* zero = region<float>(bufs[4], P.off_W1);
      NLPR_HIP_TRY(hipMemsetAsync(zero, 0, P.sz_plane, s));
      return launch_conv(P, zero, f(3), true, tmp, nullptr, halo, s);
    }
    case NLPR_STAGE_ASSEMBLE:
      return launch_conv(P, f(0), f(3), true, f(1), f(2), nullptr, s);
    case NLPR_STAGE_INIT: {
      if ((rc = launch_init(P, f(0), f(1), f(4), f(5), f(3), s))) return rc;
      if ((rc = launch_conv(P, f(1), f(2), false, nullptr, nullptr, nullptr, s))) return rc;
      return launch_conv(P, f(2), f(6), true, f(3), nullptr, nullptr, s);
    }
    default:
      return fail(NLPR_ERR_INVALID_ARG, "unknown stage");
  }
}

int nlpr_stage_time(nlpr_plan* plan, int stage, double* ms_total, int64_t* launches, int reset) {
  if (!plan || !ms_total || !launches) return fail(NLPR_ERR_INVALID_ARG, "NULL argument");
  Plan& P = plan->P;
  if (!P.timing) return fail(NLPR_ERR_NOT_ENABLED, "plan created without NLPR_TIMING");
  if (stage < 1 || stage >= NLPR_STAGE_COUNT) return fail(NLPR_ERR_INVALID_ARG, "unknown stage");
  DeviceGuard dg(P.device);
  for (const auto& r : P.recs) {
    NLPR_HIP_TRY(hipEventSynchronize(P.ev_pool[r.b]));
    float ms = 0.f;
    NLPR_HIP_TRY(hipEventElapsedTime(&ms, P.ev_pool[r.a], P.ev_pool[r.b]));
    P.acc_ms[r.stage] += ms;
    P.acc_n[r.stage] += 1;
  }
  P.recs.clear();
  P.ev_used = 0;
  *ms_total = P.acc_ms[stage];
  *launches = P.acc_n[stage];
  if (reset) {
    std::fill(std::begin(P.acc_ms), std::end(P.acc_ms), 0.0);
    std::fill(std::begin(P.acc_n), std::end(P.acc_n), int64_t(0));
  }
  return NLPR_OK;
}

}  // extern "C"
