// Dense per-pixel kernels of the NLPR ADMM iteration and the plan precompute.
//
//   precompute : FFT twiddles, the inverse Fourier denominator of eq. (inv) and the
//                L_h x L_h Woodbury block G of the P2-update, all in FP64
//   weights    : guide thresholds mu_{i tau} = lambda omega_{i tau} / rho, eq. (wts)
//   init       : initial values (nearest-neighbour upsample of Y_l)
//   conv       : circular blur B X or B^T Y, optionally plus addends and the halo fold of
//                the sweep (assembles C of eq. (x_linear_system_main))
//   pupdate    : P1 (eq. (Qh_update)), P2 (eq. (Qm_update)) and the duals Lambda1, Lambda2
//                (eqs. (dualvar1_main), (dualvar2_main))
#include <cmath>

#include "nlpr_internal.h"

namespace nlpr {
namespace {

__device__ __forceinline__ int wrapi(int x, int n) {
  x %= n;
  return x < 0 ? x + n : x;
}

// tw[m] = exp(-2 pi i m / n), in FP64, stored FP32.
__global__ void twiddle_kernel(float2* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)n, &s, &c);
  tw[m] = make_float2((float)c, (float)s);
}

// invden(u, v) = 1 / ((1 + |b^(u,v)|^2 + |P| sum_{tau in W} |d^_{tau 0}(u,v)|^2) p q), with
// |d^_{tau 0}|^2 = 2 - 2 cos(2 pi (u tau1 / p + v tau2 / q)) and the sum over W equal to
// twice the sum over W+ (the tau = 0 term vanishes).  Phases are reduced exactly in
// integers before the FP64 sine/cosine.
__global__ void den_kernel(float* invden, int p, int q, const float* blur, int r,
                           const int2* taus, int npairs, int npatch) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int u = blockIdx.y;
  if (v >= q) return;
  double br = 0.0, bi = 0.0;
  const int w = 2 * r + 1;
  for (int m1 = -r; m1 <= r; ++m1) {
    const long a = (((long)u * m1) % p + p) % p;
    for (int m2 = -r; m2 <= r; ++m2) {
      const long b = (((long)v * m2) % q + q) % q;
      const double ph = -2.0 * ((double)a / p + (double)b / q);
      double sn, cs;
      sincospi(ph, &sn, &cs);
      const double tap = (double)blur[(m1 + r) * w + (m2 + r)];
      br += tap * cs;
      bi += tap * sn;
    }
  }
  double dsum = 0.0;
  for (int n = 0; n < npairs; ++n) {
    const int2 t = taus[n];
    const long a = (((long)u * t.x) % p + p) % p;
    const long b = (((long)v * t.y) % q + q) % q;
    dsum += 2.0 - 2.0 * cospi(2.0 * ((double)a / p + (double)b / q));
  }
  const double den = 1.0 + br * br + bi * bi + (double)npatch * 2.0 * dsum;
  invden[(size_t)u * q + v] = (float)(1.0 / (den * (double)p * (double)q));
}

// G = (ratio I + R^T R)^{-1}, L_h x L_h, ratio = rho / lambda1, by Gauss-Jordan elimination
// with partial pivoting in FP64 (one thread; L_h <= 16).
__global__ void g_kernel(const float* R, int L, int Lh, double ratio, float* G) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double A[kMaxLh][2 * kMaxLh];
  for (int a = 0; a < Lh; ++a) {
    for (int b = 0; b < Lh; ++b) {
      double s = 0.0;
      for (int c = 0; c < L; ++c) s += (double)R[c * Lh + a] * (double)R[c * Lh + b];
      A[a][b] = s + (a == b ? ratio : 0.0);
      A[a][Lh + b] = (a == b) ? 1.0 : 0.0;
    }
  }
  for (int col = 0; col < Lh; ++col) {
    int piv = col;
    for (int r = col + 1; r < Lh; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col)
      for (int j = 0; j < 2 * Lh; ++j) {
        const double t = A[col][j];
        A[col][j] = A[piv][j];
        A[piv][j] = t;
      }
    const double inv = 1.0 / A[col][col];
    for (int j = 0; j < 2 * Lh; ++j) A[col][j] *= inv;
    for (int r = 0; r < Lh; ++r) {
      if (r == col) continue;
      const double f = A[r][col];
      if (f != 0.0)
        for (int j = 0; j < 2 * Lh; ++j) A[r][j] -= f * A[col][j];
    }
  }
  for (int a = 0; a < Lh; ++a)
    for (int b = 0; b < Lh; ++b) G[a * Lh + b] = (float)A[a][Lh + b];
}

// ---------------------------------------------------------------------------- weights
// mu_{i tau} = scale * exp(-inv_h2 * sum_{k in P} e_tau(i - k)),
// e_tau(j) = sum_c (Y_c(j) - Y_c(j - tau))^2, for tau = taus[blockIdx.z].
// Tile 16 x 64 per block; e on the tile plus a K halo, then separable box sums in LDS.
constexpr int WT_Y = 16, WT_X = 64;
__global__ void __launch_bounds__(256)
weights_kernel(const float* __restrict__ Yh, float* __restrict__ mu, int p, int q, int Lh, int K,
               const int2* __restrict__ taus, float scale, float inv_h2, int unweighted) {
  extern __shared__ float wsh[];
  const int EY = WT_Y + 2 * K, EX = WT_X + 2 * K;
  float* e = wsh;             // EY x EX
  float* hs = wsh + EY * EX;  // EY x WT_X
  const int x0 = blockIdx.x * WT_X, y0 = blockIdx.y * WT_Y;
  const int n = blockIdx.z;
  const int2 t = taus[n];
  float* mun = mu + (size_t)n * p * q;
  if (unweighted) {
    for (int idx = threadIdx.x; idx < WT_Y * WT_X; idx += blockDim.x) {
      const int y = y0 + idx / WT_X, x = x0 + idx % WT_X;
      if (y < p && x < q) mun[(size_t)y * q + x] = scale;
    }
    return;
  }
  const size_t plane = (size_t)p * q;
  for (int idx = threadIdx.x; idx < EY * EX; idx += blockDim.x) {
    const int yy = idx / EX, xx = idx % EX;
    const int gy = wrapi(y0 - K + yy, p), gx = wrapi(x0 - K + xx, q);
    const int sy = wrapi(gy - t.x, p), sx = wrapi(gx - t.y, q);
    float acc = 0.f;
    for (int c = 0; c < Lh; ++c) {
      const float dlt = Yh[c * plane + (size_t)gy * q + gx] - Yh[c * plane + (size_t)sy * q + sx];
      acc += dlt * dlt;
    }
    e[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < EY * WT_X; idx += blockDim.x) {
    const int yy = idx / WT_X, x = idx % WT_X;
    float acc = 0.f;
    for (int dx = 0; dx <= 2 * K; ++dx) acc += e[yy * EX + x + dx];
    hs[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < WT_Y * WT_X; idx += blockDim.x) {
    const int y = idx / WT_X, x = idx % WT_X;
    float acc = 0.f;
    for (int dy = 0; dy <= 2 * K; ++dy) acc += hs[(y + dy) * WT_X + x];
    if (y0 + y < p && x0 + x < q) mun[(size_t)(y0 + y) * q + x0 + x] = scale * expf(-acc * inv_h2);
  }
}

// ------------------------------------------------------------------------------- init
__global__ void init_kernel(const float* __restrict__ Yl, float* __restrict__ X0,
                            float* __restrict__ L1, float* __restrict__ L2,
                            float* __restrict__ W2, int p, int q, int L, int d, int zero) {
  const size_t total = (size_t)L * p * q;
  const int qd = q / d, pd = p / d;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / ((size_t)p * q));
    const int rem = (int)(e - (size_t)c * p * q);
    const int i1 = rem / q, i2 = rem - i1 * q;
    const float x = zero ? 0.f : Yl[((size_t)c * pd + i1 / d) * qd + i2 / d];
    X0[e] = x;
    W2[e] = x;
    L1[e] = 0.f;
    L2[e] = 0.f;
  }
}

// ------------------------------------------------------------------------------- conv
// out(i) = sum_m b(m) in(i - m)      (B, circular convolution)        TR = false
// out(i) = sum_m b(m) in(i + m)      (B^T, circular correlation)      TR = true
// then out += add1 + add2 + halo fold (each optional).  The halo fold adds the part of the
// regulariser term that the sweep kernel scattered above its tile: halo row h of tile t
// (rows t*tile_rows .. ) belongs to image row (t*tile_rows - hrows + h) mod p.
constexpr int CV_Y = 16, CV_X = 64;
template <bool TR>
__global__ void __launch_bounds__(256)
conv_kernel(const float* __restrict__ in, float* __restrict__ out, const float* __restrict__ taps,
            int r, int p, int q, const float* __restrict__ add1, const float* __restrict__ add2,
            const float* __restrict__ halo, int hrows, int tile_rows, int ntiles) {
  extern __shared__ float csh[];
  const int w = 2 * r + 1;
  const int TY = CV_Y + 2 * r, TX = CV_X + 2 * r;
  float* tile = csh;
  float* tp = csh + TY * TX;
  const int x0 = blockIdx.x * CV_X, y0 = blockIdx.y * CV_Y, c = blockIdx.z;
  const size_t plane = (size_t)p * q;
  const float* inc = in + (size_t)c * plane;
  for (int idx = threadIdx.x; idx < w * w; idx += blockDim.x) tp[idx] = taps[idx];
  for (int idx = threadIdx.x; idx < TY * TX; idx += blockDim.x) {
    const int yy = idx / TX, xx = idx % TX;
    tile[idx] = inc[(size_t)wrapi(y0 - r + yy, p) * q + wrapi(x0 - r + xx, q)];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < CV_Y * CV_X; idx += blockDim.x) {
    const int y = idx / CV_X, x = idx % CV_X;
    const int gy = y0 + y, gx = x0 + x;
    if (gy >= p || gx >= q) continue;
    float acc = 0.f;
    for (int m1 = -r; m1 <= r; ++m1) {
      const int ty = TR ? (y + r + m1) : (y + r - m1);
      for (int m2 = -r; m2 <= r; ++m2) {
        const int tx = TR ? (x + r + m2) : (x + r - m2);
        acc += tp[(m1 + r) * w + (m2 + r)] * tile[ty * TX + tx];
      }
    }
    const size_t o = (size_t)c * plane + (size_t)gy * q + gx;
    if (add1) acc += add1[o];
    if (add2) acc += add2[o];
    if (halo) {
      for (int h = 0; h < hrows; ++h) {
        const int r0 = wrapi(gy + hrows - h, p);
        if (r0 % tile_rows == 0) {
          const int t = r0 / tile_rows;
          acc += halo[(((size_t)c * ntiles + t) * hrows + h) * q + gx];
        }
      }
    }
    out[o] = acc;
  }
}

// ---------------------------------------------------------------------------- pupdate
// One thread per pixel; bands are visited twice.  With E = I:
//   P1 = (rho BX + Y_l - rho Lambda1) / (1 + rho)  on sampled pixels (S^T S = 1)
//   P1 = BX - Lambda1                              elsewhere            (eq. (Qh_update))
//   P2 = (X - Lambda2 + lambda1/rho Y_h R^T) F,  F = (I + lambda1/rho R R^T)^{-1}
//                                                                       (eq. (Qm_update))
// P2 is evaluated as  P2 = A0 + (Y_h - A0 R) G R^T  with A0 = X - Lambda2 and
// G = (rho/lambda1 I + R^T R)^{-1}: Woodbury gives F = I - R G R^T and the push-through
// identity R^T F = (I + lambda1/rho R^T R)^{-1} R^T turns lambda1/rho Y_h R^T F into
// Y_h G R^T.  The rearrangement is exact and keeps every FP32 term O(|X|) instead of
// O(lambda1/rho |Y_h|), which avoids a large cancellation.
//   Lambda1 -= BX - P1,  Lambda2 -= X - P2;  W1 = P1 + Lambda1,  W2 = P2 + Lambda2
template <int LHM>
__global__ void __launch_bounds__(256)
pupdate_kernel(const float* __restrict__ X, const float* __restrict__ BX,
               const float* __restrict__ Yl, const float* __restrict__ Yh,
               float* __restrict__ L1, float* __restrict__ L2, float* __restrict__ W1,
               float* __restrict__ W2, const float* __restrict__ R, const float* __restrict__ G,
               int p, int q, int L, int Lh, int d, float rho, float inv_1prho) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t plane = (size_t)p * q;
  if (j >= (int)plane) return;
  const int i1 = j / q, i2 = j - i1 * q;
  const bool sampled = (i1 % d == 0) && (i2 % d == 0);
  const size_t lj = (size_t)(i1 / d) * (q / d) + i2 / d;
  const size_t lplane = (size_t)(p / d) * (q / d);
  float res[LHM];
#pragma unroll
  for (int h = 0; h < LHM; ++h) res[h] = (h < Lh) ? Yh[h * plane + j] : 0.f;
  // res = Y_h - A0 R
  for (int c = 0; c < L; ++c) {
    const float a0 = X[c * plane + j] - L2[c * plane + j];
#pragma unroll
    for (int h = 0; h < LHM; ++h)
      if (h < Lh) res[h] -= a0 * R[c * Lh + h];
  }
  // u = res G
  float u[LHM];
#pragma unroll
  for (int h2 = 0; h2 < LHM; ++h2) {
    float s = 0.f;
#pragma unroll
    for (int h = 0; h < LHM; ++h)
      if (h < Lh && h2 < Lh) s += res[h] * G[h * Lh + h2];
    u[h2] = s;
  }
  for (int c = 0; c < L; ++c) {
    const size_t o = c * plane + j;
    float corr = 0.f;
#pragma unroll
    for (int h = 0; h < LHM; ++h)
      if (h < Lh) corr += u[h] * R[c * Lh + h];
    const float x = X[o], l2 = L2[o];
    const float p2 = (x - l2) + corr;
    const float l2n = l2 - (x - p2);
    L2[o] = l2n;
    W2[o] = p2 + l2n;
    const float bx = BX[o], l1 = L1[o];
    const float p1 = sampled ? (rho * bx + Yl[c * lplane + lj] - rho * l1) * inv_1prho : bx - l1;
    const float l1n = l1 - (bx - p1);
    L1[o] = l1n;
    W1[o] = p1 + l1n;
  }
}

__global__ void finite_kernel(const float* __restrict__ Z, size_t n, int* flag) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    if (!isfinite(Z[e])) {
      flag[0] = 1;
      return;
    }
  }
}

}  // namespace

int launch_precompute(Plan& P, hipStream_t s) {
  const int p = P.prm.p, q = P.prm.q;
  hipLaunchKernelGGL(twiddle_kernel, dim3(ceil_div(p, 256)), dim3(256), 0, s, P.d_tw_p, p);
  NLPR_LAUNCH_CHECK("twiddle_kernel");
  hipLaunchKernelGGL(twiddle_kernel, dim3(ceil_div(q, 256)), dim3(256), 0, s, P.d_tw_q, q);
  NLPR_LAUNCH_CHECK("twiddle_kernel");
  hipLaunchKernelGGL(den_kernel, dim3(ceil_div(q, 128), p), dim3(128), 0, s, P.d_invden, p, q,
                     P.d_blur, P.prm.blur_radius, P.d_taus, P.npairs, P.npatch);
  NLPR_LAUNCH_CHECK("den_kernel");
  hipLaunchKernelGGL(g_kernel, dim3(1), dim3(1), 0, s, P.d_R, P.prm.L, P.prm.Lh,
                     P.prm.rho / P.prm.lambda1, P.d_G);
  NLPR_LAUNCH_CHECK("g_kernel");
  return NLPR_OK;
}

int launch_weights(const Plan& P, const float* Yh, float* mu, hipStream_t s) {
  if (P.npairs == 0) return NLPR_OK;
  const int p = P.prm.p, q = P.prm.q, K = P.prm.K;
  const size_t lds = (size_t)((WT_Y + 2 * K) * (WT_X + 2 * K) + (WT_Y + 2 * K) * WT_X) * sizeof(float);
  const float scale = (float)(P.prm.lambda / P.prm.rho);
  const float inv_h2 = (P.prm.flags & NLPR_UNWEIGHTED) ? 0.f : (float)(1.0 / (P.prm.h * P.prm.h));
  dim3 grid(ceil_div(q, WT_X), ceil_div(p, WT_Y), P.npairs);
  hipLaunchKernelGGL(weights_kernel, grid, dim3(256), lds, s, Yh, mu, p, q, P.prm.Lh, K, P.d_taus,
                     scale, inv_h2, (P.prm.flags & NLPR_UNWEIGHTED) ? 1 : 0);
  NLPR_LAUNCH_CHECK("weights_kernel");
  return NLPR_OK;
}

int launch_init(const Plan& P, const float* Yl, float* X0, float* Lam1, float* Lam2, float* W2,
                hipStream_t s) {
  const size_t total = (size_t)P.prm.L * P.prm.p * P.prm.q;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, s, Yl, X0, Lam1, Lam2, W2, P.prm.p,
                     P.prm.q, P.prm.L, P.prm.d, (P.prm.flags & NLPR_INIT_ZERO) ? 1 : 0);
  NLPR_LAUNCH_CHECK("init_kernel");
  return NLPR_OK;
}

int launch_conv(const Plan& P, const float* in, float* out, bool transpose, const float* add1,
                const float* add2, const float* halo, hipStream_t s) {
  const int p = P.prm.p, q = P.prm.q, r = P.prm.blur_radius;
  const size_t lds = (size_t)((CV_Y + 2 * r) * (CV_X + 2 * r) + (2 * r + 1) * (2 * r + 1)) * sizeof(float);
  dim3 grid(ceil_div(q, CV_X), ceil_div(p, CV_Y), P.prm.L);
  const int hrows = halo ? P.sweep.halo : 0;
  if (transpose)
    hipLaunchKernelGGL(conv_kernel<true>, grid, dim3(256), lds, s, in, out, P.d_blur, r, p, q, add1,
                       add2, halo, hrows, P.sweep.rows, P.sweep.ntiles);
  else
    hipLaunchKernelGGL(conv_kernel<false>, grid, dim3(256), lds, s, in, out, P.d_blur, r, p, q,
                       add1, add2, halo, hrows, P.sweep.rows, P.sweep.ntiles);
  NLPR_LAUNCH_CHECK("conv_kernel");
  return NLPR_OK;
}

int launch_pupdate(const Plan& P, const float* X, const float* BX, const float* Yl,
                   const float* Yh, float* Lam1, float* Lam2, float* W1, float* W2,
                   hipStream_t s) {
  const int p = P.prm.p, q = P.prm.q;
  const int n = p * q;
  const float rho = (float)P.prm.rho;
  const float inv = (float)(1.0 / (1.0 + P.prm.rho));
  dim3 grid(ceil_div(n, 256));
#define NLPR_PU(LHM)                                                                         \
  hipLaunchKernelGGL(pupdate_kernel<LHM>, grid, dim3(256), 0, s, X, BX, Yl, Yh, Lam1, Lam2, W1, \
                     W2, P.d_R, P.d_G, p, q, P.prm.L, P.prm.Lh, P.prm.d, rho, inv)
  if (P.prm.Lh == 1) NLPR_PU(1);
  else if (P.prm.Lh <= 4) NLPR_PU(4);
  else NLPR_PU(16);
#undef NLPR_PU
  NLPR_LAUNCH_CHECK("pupdate_kernel");
  return NLPR_OK;
}

int launch_check_finite(const Plan& P, const float* Z, int* flag, hipStream_t s) {
  const size_t n = (size_t)P.prm.L * P.prm.p * P.prm.q;
  NLPR_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
  hipLaunchKernelGGL(finite_kernel, dim3(1024), dim3(256), 0, s, Z, n, flag);
  NLPR_LAUNCH_CHECK("finite_kernel");
  return NLPR_OK;
}

}  // namespace nlpr
