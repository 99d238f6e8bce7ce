// Internal declarations of libnlpr: plan structure, kernel launchers, helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "nlpr.h"

namespace nlpr {

constexpr int kMaxLh = 16;
constexpr int kMaxK = 4;
constexpr int kMaxSw = 8;
constexpr int kMaxBlurRadius = 16;
constexpr int kMaxFFTFactors = 24;
constexpr int kMaxFFTLen = 4096;
constexpr size_t kMaxSweepLds = 160 * 1024;  // LDS per workgroup on gfx950

// One-dimensional FFT of length n = product of fac[] (each 2, 3, 4 or 8); passed to
// kernels by value.  tw[m] = exp(-2 pi i m / n), m in [0, n).
struct LineFFT {
  int n;
  int nfac;
  int fac[kMaxFFTFactors];
  const float2* tw;
};

// Tiling of the sweep: a workgroup owns `rows` image rows (all q columns) of one band.
struct SweepShape {
  int rows;      // tile height R
  int items;     // float4 items per thread
  int threads;   // workgroup size
  int ntiles;    // ceil(p / R)
  int halo;      // rows above the tile reached by the adjoint scatter (max tau1)
  size_t lds;    // dynamic LDS bytes
};

struct Plan {
  nlpr_params prm{};
  int device = 0;
  int npairs = 0;                 // |W+|
  int npatch = 0;                 // |P|
  std::vector<int32_t> taus;      // host copy of W+ (tau1, tau2 pairs)
  int2* d_taus = nullptr;
  float* d_invden = nullptr;      // [p][q], 1 / (den * p * q)
  float2* d_tw_p = nullptr;
  float2* d_tw_q = nullptr;
  LineFFT fp{}, fq{};
  float* d_blur = nullptr;        // (2r+1)^2 taps
  float* d_R = nullptr;           // [L][Lh]
  float* d_G = nullptr;           // [Lh][Lh]
  SweepShape sweep{};
  // workspace layout
  size_t off_sigma = 0, off_mu = 0, off_C = 0, off_L1 = 0, off_L2 = 0, off_BX = 0,
         off_W1 = 0, off_W2 = 0, off_F = 0, off_halo = 0, off_flag = 0;
  size_t sz_sigma = 0, sz_mu = 0, sz_plane = 0, sz_F = 0, sz_halo = 0;
  size_t ws_bytes = 0;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Rec { int stage; size_t a, b; };
  std::vector<Rec> recs;
  double acc_ms[NLPR_STAGE_COUNT] = {};
  int64_t acc_n[NLPR_STAGE_COUNT] = {};
};

// ---- error plumbing (api.hip)
void set_error(const std::string& msg);
#define NLPR_HIP_TRY(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::nlpr::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));         \
      return NLPR_ERR_HIP;                                                          \
    }                                                                               \
  } while (0)
#define NLPR_LAUNCH_CHECK(what)                                                     \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess) {                                                         \
      ::nlpr::set_error(std::string("launch of ") + (what) + ": " + hipGetErrorString(e_)); \
      return NLPR_ERR_HIP;                                                          \
    }                                                                               \
  } while (0)

// ---- precompute (dense.hip)
int launch_precompute(Plan& P, hipStream_t s);

// ---- dense kernels (dense.hip)
int launch_weights(const Plan& P, const float* Yh, float* mu, hipStream_t s);
int launch_init(const Plan& P, const float* Yl, float* X0, float* Lam1, float* Lam2, float* W2,
                hipStream_t s);
// out = conv(in) (+ add1 + add2 + halo fold); transpose selects B^T.
int launch_conv(const Plan& P, const float* in, float* out, bool transpose, const float* add1,
                const float* add2, const float* halo, hipStream_t s);
int launch_pupdate(const Plan& P, const float* X, const float* BX, const float* Yl,
                   const float* Yh, float* Lam1, float* Lam2, float* W1, float* W2,
                   hipStream_t s);
int launch_check_finite(const Plan& P, const float* Z, int* flag, hipStream_t s);

// ---- FFT solve (fft.hip)
int launch_xsolve(const Plan& P, const float* C, float* X, float2* F, hipStream_t s);

// ---- sweep (sweep.hip)
SweepShape choose_sweep_shape(int p, int q, int K, int halo);
size_t sweep_sigma_bytes(const SweepShape& sh, int q, int L, int npairs, int npatch);
int launch_sweep(const Plan& P, const float* X, const float* mu, float* sigma, float* creg,
                 float* halo, bool first, hipStream_t s);

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

}  // namespace nlpr
