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
// All but the precompute run over a batch of scenes (see nlpr_internal.h).
#include <algorithm>
#include <cmath>

#include <climits>

#include "nlpr_internal.h"

namespace nlpr {
namespace {

__device__ __forceinline__ int wrapi(int x, int n) {
  x %= n;
  return x < 0 ? x + n : x;
}

// ------------------------------------------------------------------------- precompute
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

// Tables of the X-update with S inside the system (fused-S).  Per band the system is
//   a(w) x^(w) + conj(b^(w)) / (rho d^2) sum_{w' ~ w} b^(w') x^(w') = c^(w),
// a = 1 + |P| sum_{tau in W} |d^_{tau 0}|^2, w' over the aliasing group of w (the d^2
// frequencies (w1 + m1 p/d, w2 + m2 q/d) the sampling mask S^T S couples).  Each group's
// matrix is diag(a) plus a rank-one term, so Sherman-Morrison gives
//   x_j = c_j / a_j - (conj(b^_j) / a_j) gamma sum_k (b^_k / a_k) c_k,
//   gamma = 1 / (rho d^2 + sum_k |b^_k|^2 / a_k).
// One thread per group, all in FP64; stored FP32 in column-major [q][p] order with the
// 1/(p q) of the unnormalised inverse DFT folded into ia and v:
//   ia = 1 / (a p q),  u = b^ / a,  v = gamma conj(b^) / (a p q).
__device__ void freq_terms(int u, int v, int p, int q, const float* blur, int r, const int2* taus,
                           int npairs, int npatch, double* br, double* bi, double* a) {
  double sr = 0.0, si = 0.0;
  const int w = 2 * r + 1;
  for (int m1 = -r; m1 <= r; ++m1) {
    const long ka = (((long)u * m1) % p + p) % p;
    for (int m2 = -r; m2 <= r; ++m2) {
      const long kb = (((long)v * m2) % q + q) % q;
      double sn, cs;
      sincospi(-2.0 * ((double)ka / p + (double)kb / q), &sn, &cs);
      const double tap = (double)blur[(m1 + r) * w + (m2 + r)];
      sr += tap * cs;
      si += tap * sn;
    }
  }
  double dsum = 0.0;
  for (int n = 0; n < npairs; ++n) {
    const int2 t = taus[n];
    const long ka = (((long)u * t.x) % p + p) % p;
    const long kb = (((long)v * t.y) % q + q) % q;
    dsum += 2.0 - 2.0 * cospi(2.0 * ((double)ka / p + (double)kb / q));
  }
  *br = sr;
  *bi = si;
  *a = 1.0 + (double)npatch * 2.0 * dsum;
}

__global__ void fused_tables_kernel(int p, int q, int d, const float* blur, int r,
                                    const int2* taus, int npairs, int npatch, double rho,
                                    float* ia, float2* fu, float2* fv) {
  const int pd = p / d, qd = q / d;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= pd * qd) return;
  const int w1 = g / qd, w2 = g - (g / qd) * qd;
  double s = 0.0;
  for (int m1 = 0; m1 < d; ++m1)
    for (int m2 = 0; m2 < d; ++m2) {
      double br, bi, a;
      freq_terms(w1 + m1 * pd, w2 + m2 * qd, p, q, blur, r, taus, npairs, npatch, &br, &bi, &a);
      s += (br * br + bi * bi) / a;
    }
  const double gamma = 1.0 / (rho * d * d + s);
  const double pq = (double)p * (double)q;
  for (int m1 = 0; m1 < d; ++m1)
    for (int m2 = 0; m2 < d; ++m2) {
      const int u = w1 + m1 * pd, v = w2 + m2 * qd;
      double br, bi, a;
      freq_terms(u, v, p, q, blur, r, taus, npairs, npatch, &br, &bi, &a);
      const size_t o = (size_t)v * p + u;
      ia[o] = (float)(1.0 / (a * pq));
      fu[o] = make_float2((float)(br / a), (float)(bi / a));
      fv[o] = make_float2((float)(gamma * br / (a * pq)), (float)(-gamma * bi / (a * pq)));
    }
}

// Gauss-Jordan inversion with partial pivoting in FP64, by one workgroup: A is n x 2n in LDS
// (row stride 2 NM), [matrix | I] on entry and [I | inverse] on return.  One thread picks
// the pivot (largest magnitude, first on ties); every element then takes the same sequence
// of operations as in the textbook serial loop.
template <int NM>
__device__ void gauss_jordan_block(double* A, int n) {
  constexpr int RS = 2 * NM;
  __shared__ int piv_s;
  __shared__ double f[NM];
  const int n2 = 2 * n;
  for (int col = 0; col < n; ++col) {
    if (threadIdx.x == 0) {
      int piv = col;
      for (int r = col + 1; r < n; ++r)
        if (fabs(A[r * RS + col]) > fabs(A[piv * RS + col])) piv = r;
      piv_s = piv;
    }
    __syncthreads();
    const int piv = piv_s;
    if (piv != col)
      for (int j = threadIdx.x; j < n2; j += blockDim.x) {
        const double t = A[col * RS + j];
        A[col * RS + j] = A[piv * RS + j];
        A[piv * RS + j] = t;
      }
    __syncthreads();
    const double inv = 1.0 / A[col * RS + col];
    __syncthreads();                       // every thread has read the pivot
    for (int j = threadIdx.x; j < n2; j += blockDim.x) A[col * RS + j] *= inv;
    for (int r = threadIdx.x; r < n; r += blockDim.x) f[r] = 0.0;
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x)
      if (r != col) f[r] = A[r * RS + col];  // factors before any row changes
    __syncthreads();
    for (int e = threadIdx.x; e < n * n2; e += blockDim.x) {
      const int r = e / n2, j = e - (e / n2) * n2;
      if (f[r] != 0.0) A[r * RS + j] -= f[r] * A[col * RS + j];
    }
    __syncthreads();
  }
}

// G = (ratio I + R^T R)^{-1}, L_h x L_h, ratio = rho / lambda1, in FP64 (one workgroup).
__global__ void __launch_bounds__(256) g_kernel(const float* R, int L, int Lh, double ratio,
                                                float* G) {
  __shared__ double A[kMaxLh * 2 * kMaxLh];
  for (int e = threadIdx.x; e < Lh * Lh; e += blockDim.x) {
    const int a = e / Lh, b = e - (e / Lh) * Lh;
    double s = 0.0;
    for (int c = 0; c < L; ++c) s += (double)R[c * Lh + a] * (double)R[c * Lh + b];
    A[a * 2 * kMaxLh + b] = s + (a == b ? ratio : 0.0);
    A[a * 2 * kMaxLh + Lh + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  gauss_jordan_block<kMaxLh>(A, Lh);
  for (int e = threadIdx.x; e < Lh * Lh; e += blockDim.x) {
    const int a = e / Lh, b = e - (e / Lh) * Lh;
    G[a * Lh + b] = (float)A[a * 2 * kMaxLh + Lh + b];
  }
}

// With a subspace basis E (Ls x L), in FP64 (one workgroup; Ls <= 32):
//   M  = (E E^T + rho I)^{-1}            Ls x Ls   (P1-update, eq. (Qh_update))
//   Ep = E^T (E E^T)^{-1}                L x Ls    (default start X0 = up(Y_l) Ep)
//   Rt = E R                             Ls x Lh   (P2-update with E R in place of R)
__global__ void __launch_bounds__(256) subspace_kernel(const float* E, const float* R, int L,
                                                       int Ls, int Lh, double rho, float* M,
                                                       float* Ep, float* Rt) {
  constexpr int RS = 2 * kMaxLs;
  __shared__ double A[kMaxLs * RS];
  __shared__ double EEt[kMaxLs * kMaxLs];
  for (int e = threadIdx.x; e < Ls * Ls; e += blockDim.x) {
    const int a = e / Ls, b = e - (e / Ls) * Ls;
    double s = 0.0;
    for (int c = 0; c < L; ++c) s += (double)E[a * L + c] * (double)E[b * L + c];
    EEt[a * kMaxLs + b] = s;
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {      // pass 0: (E E^T + rho I)^{-1}; 1: (E E^T)^{-1}
    for (int e = threadIdx.x; e < Ls * Ls; e += blockDim.x) {
      const int a = e / Ls, b = e - (e / Ls) * Ls;
      A[a * RS + b] = EEt[a * kMaxLs + b] + (pass == 0 && a == b ? rho : 0.0);
      A[a * RS + Ls + b] = (a == b) ? 1.0 : 0.0;
    }
    __syncthreads();
    gauss_jordan_block<kMaxLs>(A, Ls);
    if (pass == 0) {
      for (int e = threadIdx.x; e < Ls * Ls; e += blockDim.x) {
        const int a = e / Ls, b = e - (e / Ls) * Ls;
        M[a * Ls + b] = (float)A[a * RS + Ls + b];
      }
    } else {
      for (int e = threadIdx.x; e < L * Ls; e += blockDim.x) {
        const int c = e / Ls, b = e - (e / Ls) * Ls;
        double s = 0.0;
        for (int a = 0; a < Ls; ++a) s += (double)E[a * L + c] * A[a * RS + Ls + b];
        Ep[c * Ls + b] = (float)s;
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < Ls * Lh; e += blockDim.x) {
    const int a = e / Lh, h = e - (e / Lh) * Lh;
    double s = 0.0;
    for (int c = 0; c < L; ++c) s += (double)E[a * L + c] * (double)R[c * Lh + h];
    Rt[a * Lh + h] = (float)s;
  }
}

// Y_l E^T and Y_l E^+ at every low-resolution pixel m: [Ls][p/d][q/d] each.
__global__ void __launch_bounds__(256)
project_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int yl_s,
               int yle_s, int ylp_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int nl = (S.p / S.d) * (S.q / S.d);
  const int m = it.y * 256 + threadIdx.x;
  if (m >= nl) return;
  const int Ls = S.L, Lz = S.Lz;
  const gfloat* __restrict__ Yl = gslot<const gfloat>(S, yl_s);
  const gfloat* __restrict__ E = as_global(S.E);
  const gfloat* __restrict__ Ep = as_global(S.Ep);
  float ye[kMaxLs], yp[kMaxLs];
#pragma unroll
  for (int k = 0; k < kMaxLs; ++k) ye[k] = yp[k] = 0.f;
  for (int c = 0; c < Lz; ++c) {
    const float y = Yl[(size_t)c * nl + m];
#pragma unroll
    for (int k = 0; k < kMaxLs; ++k)
      if (k < Ls) {
        ye[k] += y * E[k * Lz + c];
        yp[k] += y * Ep[c * Ls + k];
      }
  }
  gfloat* yle = gslot<gfloat>(S, yle_s);
  gfloat* ylp = gslot<gfloat>(S, ylp_s);
#pragma unroll
  for (int k = 0; k < kMaxLs; ++k)
    if (k < Ls) {
      yle[(size_t)k * nl + m] = ye[k];
      ylp[(size_t)k * nl + m] = yp[k];
    }
}

// P1 on the sampled pixels with a basis (eq. (Qh_update)):
//   P1 = (rho BX + Y_l E^T - rho Lambda1) (E E^T + rho I)^{-1},
// then Lambda1 -= BX - P1 and W1 = P1 + Lambda1.  One thread per low-resolution pixel.
__global__ void __launch_bounds__(256)
p1_subspace_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int bx_s,
                   int yle_s, int l1_s, int w1_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int qd = S.q / S.d;
  const int nl = (S.p / S.d) * qd;
  const int m = it.y * 256 + threadIdx.x;
  if (m >= nl) return;
  const int Ls = S.L;
  const size_t plane = (size_t)S.p * S.q;
  const size_t j = (size_t)(m / qd) * S.d * S.q + (size_t)(m % qd) * S.d;
  const gfloat* __restrict__ BX = gslot<const gfloat>(S, bx_s);
  const gfloat* __restrict__ yle = gslot<const gfloat>(S, yle_s);
  gfloat* __restrict__ L1 = gslot<gfloat>(S, l1_s);
  gfloat* __restrict__ W1 = gslot<gfloat>(S, w1_s);
  const gfloat* __restrict__ M = as_global(S.M);
  const float rho = S.rho;
  float v[kMaxLs], bx[kMaxLs], l1[kMaxLs];
#pragma unroll
  for (int k = 0; k < kMaxLs; ++k)
    if (k < Ls) {
      bx[k] = BX[k * plane + j];
      l1[k] = L1[k * plane + j];
      v[k] = rho * bx[k] + yle[(size_t)k * nl + m] - rho * l1[k];
    }
  float p1[kMaxLs];                       // every read of M before the first store
#pragma unroll
  for (int k2 = 0; k2 < kMaxLs; ++k2) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < kMaxLs; ++k)
      if (k < Ls && k2 < Ls) t += v[k] * M[k * Ls + k2];
    p1[k2] = t;
  }
#pragma unroll
  for (int k2 = 0; k2 < kMaxLs; ++k2)
    if (k2 < Ls) {
      const float l1n = l1[k2] - (bx[k2] - p1[k2]);
      L1[k2 * plane + j] = l1n;
      W1[k2 * plane + j] = p1[k2] + l1n;
    }
}

// Z = X E at every pixel: Z_c = sum_s X_s E[s][c].
__global__ void __launch_bounds__(256)
compose_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int x_s,
               int z_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const size_t plane = (size_t)S.p * S.q;
  const int j = it.y * 256 + threadIdx.x;
  if (j >= (int)plane) return;
  const int Ls = S.L, Lz = S.Lz;
  const gfloat* __restrict__ X = gslot<const gfloat>(S, x_s);
  gfloat* __restrict__ Z = gslot<gfloat>(S, z_s);
  const gfloat* __restrict__ E = as_global(S.E);
  float x[kMaxLs];
#pragma unroll
  for (int k = 0; k < kMaxLs; ++k) x[k] = (k < Ls) ? X[k * plane + j] : 0.f;
  for (int c = 0; c < Lz; ++c) {
    float z = 0.f;
#pragma unroll
    for (int k = 0; k < kMaxLs; ++k)
      if (k < Ls) z += x[k] * E[k * Lz + c];
    Z[c * plane + j] = z;
  }
}

// ---------------------------------------------------------------------------- weights
// mu_{i tau} = scale * exp(-inv_h2 * sum_{k in P} e_tau(i - k)),
// e_tau(j) = sum_c (Y_c(j) - Y_c(j - tau))^2.  Local block = (shift, tile row, tile col);
// 16 x 64 tile, e on the tile plus a K halo, then separable box sums in LDS.
constexpr int WT_Y = 16, WT_X = 64;
__global__ void __launch_bounds__(256)
weights_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int yh_s,
               int mu_s) {
  extern __shared__ float wsh[];
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, K = S.K, Lh = S.Lh;
  const int gx = ceil_div(q, WT_X), gy = ceil_div(p, WT_Y);
  const int n = it.y / (gx * gy);
  const int rem = it.y - n * gx * gy;
  const int y0 = (rem / gx) * WT_Y, x0 = (rem % gx) * WT_X;
  const int EY = WT_Y + 2 * K, EX = WT_X + 2 * K;
  float* e = wsh;             // EY x EX
  float* hs = wsh + EY * EX;  // EY x WT_X
  const int2 t = tau_at(S, n);
  const gfloat* Yh = gslot<const gfloat>(S, yh_s);
  gfloat* mun = gslot<gfloat>(S, mu_s) + (size_t)n * p * q;
  if (S.unweighted) {
    for (int idx = threadIdx.x; idx < WT_Y * WT_X; idx += blockDim.x) {
      const int y = y0 + idx / WT_X, x = x0 + idx % WT_X;
      if (y < p && x < q) mun[(size_t)y * q + x] = S.mu_scale;
    }
    return;
  }
  const size_t plane = (size_t)p * q;
  for (int idx = threadIdx.x; idx < EY * EX; idx += blockDim.x) {
    const int yy = idx / EX, xx = idx % EX;
    const int gyy = wrapi(y0 - K + yy, p), gxx = wrapi(x0 - K + xx, q);
    const int sy = wrapi(gyy - t.x, p), sx = wrapi(gxx - t.y, q);
    float acc = 0.f;
    for (int c = 0; c < Lh; ++c) {
      const float dlt = Yh[c * plane + (size_t)gyy * q + gxx] - Yh[c * plane + (size_t)sy * q + sx];
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
    if (y0 + y < p && x0 + x < q)
      mun[(size_t)(y0 + y) * q + x0 + x] = S.mu_scale * expf(-acc * S.inv_h2);
  }
}

// ------------------------------------------------------------------ elementwise planes
// One thread per element of [L][p][q]; local block lb covers elements lb*256 .. +255.
__global__ void __launch_bounds__(256)
init_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int yl_s, int ylp_s,
            int x0_s, int l1_s, int l2_s, int w2_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, d = S.d;
  const size_t e = (size_t)it.y * 256 + threadIdx.x;
  if (e >= (size_t)S.L * p * q) return;
  const int c = (int)(e / ((size_t)p * q));
  const int rem = (int)(e - (size_t)c * p * q);
  const int i1 = rem / q, i2 = rem - i1 * q;
  // with a basis the start is the upsampled coefficient image Y_l E^+ (Ls bands)
  const gfloat* Yl = gslot<const gfloat>(S, S.subspace ? ylp_s : yl_s);
  const float x = S.init_zero ? 0.f : Yl[((size_t)c * (p / d) + i1 / d) * (q / d) + i2 / d];
  gslot<gfloat>(S, x0_s)[e] = x;
  gslot<gfloat>(S, w2_s)[e] = x;
  gslot<gfloat>(S, l1_s)[e] = 0.f;
  gslot<gfloat>(S, l2_s)[e] = 0.f;
}

// T = S^T Y_l / rho: the low-resolution pixels at (d m1, d m2), zero elsewhere (fused-S).
__global__ void __launch_bounds__(256)
upsample_zero_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int yl_s,
                     int t_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, d = S.d;
  const size_t e = (size_t)it.y * 256 + threadIdx.x;
  if (e >= (size_t)S.L * p * q) return;
  const int c = (int)(e / ((size_t)p * q));
  const int rem = (int)(e - (size_t)c * p * q);
  const int i1 = rem / q, i2 = rem - i1 * q;
  float v = 0.f;
  if (i1 % d == 0 && i2 % d == 0)
    v = gslot<const gfloat>(S, yl_s)[((size_t)c * (p / d) + i1 / d) * (q / d) + i2 / d] / S.rho;
  gslot<gfloat>(S, t_s)[e] = v;
}

__global__ void __launch_bounds__(256)
fill_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int s_) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const size_t e = (size_t)it.y * 256 + threadIdx.x;
  if (e < (size_t)S.L * S.p * S.q) gslot<gfloat>(S, s_)[e] = 0.f;
}

// flag[0] = min(flag[0], iter) if any element of the slot is NaN or Inf.  The flag is set to
// INT_MAX at the start of a solve by a one-thread launch (so no memset is recorded into a
// captured graph); it then holds the first checked iteration that found a non-finite value.
__global__ void __launch_bounds__(256)
finite_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int z_s,
              int* flag, int iter) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const size_t e = (size_t)it.y * 256 + threadIdx.x;
  if (e < (size_t)S.L * S.p * S.q && !isfinite(gslot<const gfloat>(S, z_s)[e]))
    atomicMin(flag, iter);
}

__global__ void clear_flag_kernel(int* flag) { flag[0] = INT_MAX; }

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ------------------------------------------------------------------------------- conv
// out(i) = sum_m b(m) in(i - m)      (B, circular convolution)        TR = false
// out(i) = sum_m b(m) in(i + m)      (B^T, circular correlation)      TR = true
// then out += add1 + add2 + halo fold (each optional).  The halo fold adds the part of the
// regulariser term that the sweep scattered above its tile: halo row h of tile t belongs
// to image row (t * rows - halo + h) mod p.  Bit 0 / bit 1 of reg_mask mark add1 / add2 as
// regulariser terms; they and the halo are skipped for scenes without a search window,
// whose sweep never runs.  Bit 2 adds the planes and halo rows of the sweep's other parts
// when it splits the shifts of a tile over several workgroups.  Local block = (band, tile row, tile col), tile
// 16 x 64; each thread produces 4 consecutive outputs of one row, reusing the LDS row it
// reads for all 4.
// The blur radius is a template bound RM >= r (1, 2, 4, 8 or 16): the tile carries an RM
// halo and the taps are zero-padded to (2 RM + 1)^2, so each thread keeps the 4 + 2 RM input
// values of a tap row in registers and the tap loop is unrolled.  Padded taps add exact
// zeros, so the sum equals the (2r+1)^2 one.
// The tile comes in with 16-byte loads when RM is a multiple of 4 (its columns then start
// on a multiple of 4 and q % 4 == 0, so no access straddles the wrap), else column by
// column; tap rows are read from LDS as float4 when RM is even (rows of 64 + 2 RM floats).
// A rank-one blur b = u v^T (S.bsep) runs as a pass along rows over the tile and its halo
// rows, h = v * in, kept in LDS, then one along columns, out = u * h: 2 (2 RM + 1) instead of
// (2 RM + 1)^2 multiply-adds per output.
constexpr int CV_Y = 16, CV_X = 64;
template <bool TR, int RM>
__global__ void __launch_bounds__(256)
conv_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int in_s, int out_s,
            int add1_s, int add2_s, int halo_s, int reg_mask) {
  extern __shared__ float4 csh4[];           // 16-byte aligned: the rank-one pass stores float4
  float* csh = reinterpret_cast<float*>(csh4);
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, r = S.r;
  const int gx = ceil_div(q, CV_X), gy = ceil_div(p, CV_Y);
  const int c = it.y / (gx * gy);
  const int rem = it.y - c * gx * gy;
  const int y0 = (rem / gx) * CV_Y, x0 = (rem % gx) * CV_X;
  const int w = 2 * r + 1;
  constexpr int W2 = 2 * RM + 1;
  constexpr int TY = CV_Y + 2 * RM, TX = CV_X + 2 * RM;
  float* tile = csh;
  float* tp = csh + TY * TX;
  const size_t plane = (size_t)p * q;
  const int y = threadIdx.x >> 4;            // 16 rows
  const int xb = (threadIdx.x & 15) * 4;     // 4 outputs per thread
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  const int gy2 = y0 + y;
  const bool reg = S.npairs > 0;
  const gfloat* a1 = (reg || !(reg_mask & 1)) ? gslot<const gfloat>(S, add1_s) : nullptr;
  const gfloat* a2 = (reg || !(reg_mask & 2)) ? gslot<const gfloat>(S, add2_s) : nullptr;
  const gfloat* hb = reg ? gslot<const gfloat>(S, halo_s) : nullptr;
  gfloat* out = gslot<gfloat>(S, out_s);
  const int gx0 = x0 + xb;
  const size_t o0 = (size_t)c * plane + (size_t)gy2 * q + gx0;
  // bit 2: the regulariser term comes from a sweep split into psplit parts; parts 1 ..
  // psplit-1 left their planes in slot B_CSPLIT and every part its own halo rows
  const int ns = (reg && (reg_mask & 4)) ? S.psplit : 1;
  const gfloat* cs = ns > 1 ? gslot<const gfloat>(S, B_CSPLIT) : nullptr;
  const uintptr_t align = reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(a1) |
                          reinterpret_cast<uintptr_t>(a2) | reinterpret_cast<uintptr_t>(hb) |
                          reinterpret_cast<uintptr_t>(cs);
  const bool vec = gy2 < p && gx0 + 3 < q && (align & 15) == 0;
  // the addends of the 16-byte path are requested before the convolution, so their latency
  // overlaps it (out may be add2: each thread reads and writes only its own four outputs)
  float4 t1 = make_float4(0.f, 0.f, 0.f, 0.f), t2 = t1;
  if (vec && a1) t1 = ldg4(a1 + o0);
  if (vec && a2) t2 = ldg4(a2 + o0);
  // in_s < 0: no convolution, out = add1 + add2 + halo fold (uniform over the launch)
  if (in_s >= 0) {
    const gfloat* inc = gslot<const gfloat>(S, in_s) + (size_t)c * plane;
    const gfloat* uv = S.bsep ? as_global(S.bsep) : nullptr;
    float* ht = tp;                          // rank one: TY x CV_X row-filtered tile
    float* tu = ht + TY * CV_X;              // rank one: u, v zero-padded to 2 RM + 1
    if (uv) {
      for (int idx = threadIdx.x; idx < 2 * W2; idx += blockDim.x) {
        const int m = (idx < W2 ? idx : idx - W2) - RM;
        tu[idx] = (m >= -r && m <= r) ? uv[(idx < W2 ? 0 : w) + m + r] : 0.f;
      }
    } else {
      for (int idx = threadIdx.x; idx < W2 * W2; idx += blockDim.x) {
        const int a = idx / W2 - RM, b = idx - (idx / W2) * W2 - RM;
        tp[idx] = (a >= -r && a <= r && b >= -r && b <= r)
                      ? as_global(S.blur)[(a + r) * w + (b + r)] : 0.f;
      }
    }
    // tile with a circular RM halo: thread = column (coalesced), rows strided by 2; one wrap
    // of the column per thread, rows wrapped incrementally (TX <= 96 <= 128 columns)
    if (RM % 4 == 0 && (reinterpret_cast<uintptr_t>(inc) & 15) == 0) {
      constexpr int TX4 = TX / 4;
      for (int e = threadIdx.x; e < TY * TX4; e += blockDim.x) {
        const int yy = e / TX4, c4 = e - yy * TX4;
        const int gyy = wrapi(y0 - RM + yy, p), gxx = wrapi(x0 - RM + 4 * c4, q);
        *reinterpret_cast<float4*>(tile + yy * TX + 4 * c4) = ldg4(inc + (size_t)gyy * q + gxx);
      }
    } else {
      const int lane = threadIdx.x & 127;
      if (lane < TX) {
        const int gxx = wrapi(x0 - RM + lane, q);
        int yy = threadIdx.x >> 7;
        int gyy = wrapi(y0 - RM + yy, p);
        for (; yy < TY; yy += 2) {
          tile[yy * TX + lane] = inc[(size_t)gyy * q + gxx];
          gyy += 2;
          if (gyy >= p) gyy -= p;   // p >= 8
        }
      }
    }
    __syncthreads();
    if (uv) {
      const float* tv = tu + W2;
      for (int yy = y; yy < TY; yy += CV_Y) {   // rows of the tile and of its halo
        const float* trow = tile + yy * TX + xb;
        float rv[4 + 2 * RM];
        if constexpr (RM % 2 == 0) {
#pragma unroll
          for (int i4 = 0; i4 < (4 + 2 * RM) / 4; ++i4) {
            const float4 v = reinterpret_cast<const float4*>(trow)[i4];
            rv[4 * i4] = v.x; rv[4 * i4 + 1] = v.y; rv[4 * i4 + 2] = v.z; rv[4 * i4 + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4 + 2 * RM; ++i) rv[i] = trow[i];
        }
        float hs[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m2 = -RM; m2 <= RM; ++m2) {
          const float b = tv[m2 + RM];
          const int o = TR ? (RM + m2) : (RM - m2);
#pragma unroll
          for (int e = 0; e < 4; ++e) hs[e] += b * rv[o + e];
        }
        *reinterpret_cast<float4*>(ht + yy * CV_X + xb) = make_float4(hs[0], hs[1], hs[2], hs[3]);
      }
      __syncthreads();
#pragma unroll
      for (int m1 = -RM; m1 <= RM; ++m1) {
        const float4 h =
            *reinterpret_cast<const float4*>(ht + (TR ? (y + RM + m1) : (y + RM - m1)) * CV_X + xb);
        const float b = tu[m1 + RM];
        acc[0] += b * h.x;
        acc[1] += b * h.y;
        acc[2] += b * h.z;
        acc[3] += b * h.w;
      }
    } else {
      for (int m1 = -RM; m1 <= RM; ++m1) {
        const float* trow = tile + (TR ? (y + RM + m1) : (y + RM - m1)) * TX + xb;
        const float* tap = tp + (m1 + RM) * W2;
        float rv[4 + 2 * RM];
        if constexpr (RM % 2 == 0) {
#pragma unroll
          for (int i4 = 0; i4 < (4 + 2 * RM) / 4; ++i4) {
            const float4 v = reinterpret_cast<const float4*>(trow)[i4];
            rv[4 * i4] = v.x; rv[4 * i4 + 1] = v.y; rv[4 * i4 + 2] = v.z; rv[4 * i4 + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4 + 2 * RM; ++i) rv[i] = trow[i];
        }
#pragma unroll
        for (int m2 = -RM; m2 <= RM; ++m2) {
          const float b = tap[m2 + RM];
          const int o = TR ? (RM + m2) : (RM - m2);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[e] += b * rv[o + e];
        }
      }
    }
  }
  if (gy2 >= p) return;
  // halo rows folded into image row gy2: halo row h of the tile starting at row
  // gy2 + H - h (when that is a tile start); the same for the four columns
  const int H = hb ? S.halo : 0, R = S.rows;
  const size_t cs_stride = (size_t)S.L * plane;
  const size_t hb_stride = (size_t)S.L * S.ntiles * H * q;
  if (vec) {
    float4 v = make_float4(acc[0], acc[1], acc[2], acc[3]);
    if (a1) {
      v.x += t1.x; v.y += t1.y; v.z += t1.z; v.w += t1.w;
    }
    if (a2) {
      v.x += t2.x; v.y += t2.y; v.z += t2.z; v.w += t2.w;
    }
    // the parts are loaded four at a time before they are added (in order; an absent part
    // adds zero), so their latencies overlap
    for (int j = 1; j < ns; j += 4) {
      float4 t[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        t[u] = j + u < ns ? ldg4(cs + (size_t)(j + u - 1) * cs_stride + o0)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) { v.x += t[u].x; v.y += t[u].y; v.z += t[u].z; v.w += t[u].w; }
    }
    for (int h = 0; h < H; ++h) {
      const int r0 = wrapi(gy2 + H - h, p);
      if (r0 % R) continue;
      const size_t ho = (((size_t)c * S.ntiles + r0 / R) * H + h) * q + gx0;
      for (int j = 0; j < ns; j += 4) {
        float4 t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          t[u] = j + u < ns ? ldg4(hb + (size_t)(j + u) * hb_stride + ho)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 4; ++u) { v.x += t[u].x; v.y += t[u].y; v.z += t[u].z; v.w += t[u].w; }
      }
    }
    stg4(out + o0, v);
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int gx2 = gx0 + e;
    if (gx2 >= q) continue;
    const size_t o = o0 + e;
    float v = acc[e];
    if (a1) v += a1[o];
    if (a2) v += a2[o];
    for (int j = 1; j < ns; j += 4) {
      float t[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) t[u] = j + u < ns ? cs[(size_t)(j + u - 1) * cs_stride + o] : 0.f;
#pragma unroll
      for (int u = 0; u < 4; ++u) v += t[u];
    }
    for (int h = 0; h < H; ++h) {
      const int r0 = wrapi(gy2 + H - h, p);
      if (r0 % R) continue;
      const size_t ho = (((size_t)c * S.ntiles + r0 / R) * H + h) * q + gx2;
      for (int j = 0; j < ns; j += 4) {
        float t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = j + u < ns ? hb[(size_t)(j + u) * hb_stride + ho] : 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u) v += t[u];
      }
    }
    out[o] = v;
  }
}

// ---------------------------------------------------------------------------- pupdate
// Work item = 256 pixels; a workgroup of 256 NC threads gives each pixel NC threads (1, or
// 4 when the launch covers few pixels in all, so that it still fills the GPU), each owning
// a contiguous share of the bands.
// With E = I:
//   P1 = (rho BX + Y_l - rho Lambda1) / (1 + rho)  on sampled pixels (S^T S = 1)
//   P1 = BX - Lambda1                              elsewhere            (eq. (Qh_update))
//   P2 = (X - Lambda2 + lambda1/rho Y_h R^T) F,  F = (I + lambda1/rho R R^T)^{-1}
//                                                                       (eq. (Qm_update))
// P2 is evaluated as  P2 = A0 + (Y_h - A0 R) G R^T  with A0 = X - Lambda2 and
// G = (rho/lambda1 I + R^T R)^{-1}: Woodbury gives F = I - R G R^T and the push-through
// identity R^T F = (I + lambda1/rho R^T R)^{-1} R^T turns lambda1/rho Y_h R^T F into
// Y_h G R^T.  The rearrangement is exact and keeps every FP32 term O(|X|) instead of
// O(lambda1/rho |Y_h|), which avoids a large cancellation.  The contraction A0 R over
// bands is summed per band share and the parts are added in share order (through LDS when a
// pixel has several threads).
//   Lambda1 -= BX - P1,  Lambda2 -= X - P2;  W1 = P1 + Lambda1,  W2 = P2 + Lambda2
// Band shares of the contraction A0 R in the P-update: fixed, so that the sum is the same
// whichever number of threads a pixel has.
constexpr int kPuShares = 4;

// rp += sum over bands [c0, c1) of (X - Lambda2)_c R_c, one fused multiply-add per term.
template <int LHM>
__device__ __forceinline__ void pupdate_share(const gfloat* __restrict__ X,
                                              const gfloat* __restrict__ L2,
                                              const gfloat* __restrict__ R, float (&rp)[LHM],
                                              size_t plane, int Lh, int c0, int c1, int j) {
  for (int c = c0; c < c1; ++c) {
    const float a0 = X[c * plane + j] - L2[c * plane + j];
#pragma unroll
    for (int h = 0; h < LHM; ++h)
      if (h < Lh) rp[h] = __builtin_fmaf(a0, R[c * Lh + h], rp[h]);
  }
}

// Bands [c0, c1) of one pixel: P2, Lambda2, W2 and (per p1mode) P1, Lambda1, W1.  Lambda is
// read through L1, L2 and written through L1o, L2o, which may be the same buffers (no
// restrict on those four).  R arrives as a restrict parameter so that the compiler may read
// it with scalar loads across the stores (restrict on local pointer variables is not used
// for that).
template <int LHM>
__device__ __forceinline__ void pupdate_write(
    const gfloat* __restrict__ X, const gfloat* __restrict__ BX, const gfloat* __restrict__ Yl,
    const gfloat* L1, const gfloat* L2, gfloat* L1o, gfloat* L2o, gfloat* __restrict__ W1,
    gfloat* __restrict__ W2, const gfloat* __restrict__ R, const float (&u)[LHM], size_t plane,
    size_t lplane, size_t lj, bool sampled, int p1mode, int Lh, float rho, float inv_1prho,
    int c0, int c1, int j) {
  for (int c = c0; c < c1; ++c) {
    const size_t o = c * plane + j;
    float corr = 0.f;
#pragma unroll
    for (int h = 0; h < LHM; ++h)
      if (h < Lh) corr += u[h] * R[c * Lh + h];
    const float x = X[o], l2 = L2[o];
    const float p2 = (x - l2) + corr;
    const float l2n = l2 - (x - p2);
    L2o[o] = l2n;
    W2[o] = p2 + l2n;
    if (p1mode == 2 || (sampled && p1mode == 1)) continue;
    const float bx = BX[o], l1 = L1[o];
    const float p1 = sampled ? (rho * bx + Yl[c * lplane + lj] - rho * l1) * inv_1prho : bx - l1;
    const float l1n = l1 - (bx - p1);
    L1o[o] = l1n;
    W1[o] = p1 + l1n;
  }
}

// With at most kPuKeep bands per thread, X and Lambda2 are read once: the contraction pass
// keeps them in registers for the write pass (32 bytes per pixel and band instead of 40).
// Same operations in the same order as the two functions above.
constexpr int kPuKeep = 16;

// All loads of the thread's bands up front (X, Lambda2, and for P1 BX and Lambda1), so that
// their latencies overlap: the contraction pass then only waits for X and Lambda2.
template <int LHM>
__device__ __forceinline__ void pupdate_load_keep(const gfloat* __restrict__ X,
                                                  const gfloat* __restrict__ L2,
                                                  const gfloat* __restrict__ BX,
                                                  const gfloat* __restrict__ L1,
                                                  const gfloat* __restrict__ Yl, bool p1,
                                                  bool sampled, size_t plane, size_t lplane,
                                                  size_t lj, int c0, int c1, int j,
                                                  float (&xs)[kPuKeep], float (&l2s)[kPuKeep],
                                                  float (&bxs)[kPuKeep], float (&l1s)[kPuKeep],
                                                  float (&yls)[kPuKeep]) {
#pragma unroll
  for (int i = 0; i < kPuKeep; ++i) {
    const int c = c0 + i;
    if (c < c1) {
      xs[i] = X[c * plane + j];
      l2s[i] = L2[c * plane + j];
    }
  }
  if (!p1) return;
#pragma unroll
  for (int i = 0; i < kPuKeep; ++i) {
    const int c = c0 + i;
    if (c < c1) {
      bxs[i] = BX[c * plane + j];
      l1s[i] = L1[c * plane + j];
      if (sampled) yls[i] = Yl[c * lplane + lj];
    }
  }
}

// rp += sum over bands [cs, ce) of (X - Lambda2)_c R_c, from the kept values (band c at
// register c - c0)
template <int LHM>
__device__ __forceinline__ void pupdate_share_kept(const float (&xs)[kPuKeep],
                                                   const float (&l2s)[kPuKeep],
                                                   const gfloat* __restrict__ R,
                                                   float (&rp)[LHM], int Lh, int c0, int cs,
                                                   int ce) {
#pragma unroll
  for (int i = 0; i < kPuKeep; ++i) {
    const int c = c0 + i;
    if (c >= cs && c < ce) {
      const float a0 = xs[i] - l2s[i];
#pragma unroll
      for (int h = 0; h < LHM; ++h)
        if (h < Lh) rp[h] = __builtin_fmaf(a0, R[c * Lh + h], rp[h]);
    }
  }
}

template <int LHM>
__device__ __forceinline__ void pupdate_write_kept(
    const float (&xs)[kPuKeep], const float (&l2s)[kPuKeep], const float (&bxs)[kPuKeep],
    const float (&l1s)[kPuKeep], const float (&yls)[kPuKeep], gfloat* L1o, gfloat* L2o,
    gfloat* __restrict__ W1, gfloat* __restrict__ W2, const gfloat* __restrict__ R,
    const float (&u)[LHM], size_t plane, bool sampled, int p1mode, int Lh, float rho,
    float inv_1prho, int c0, int c1, int j) {
#pragma unroll
  for (int i = 0; i < kPuKeep; ++i) {
    const int c = c0 + i;
    if (c >= c1) continue;
    const size_t o = c * plane + j;
    float corr = 0.f;
#pragma unroll
    for (int h = 0; h < LHM; ++h)
      if (h < Lh) corr += u[h] * R[c * Lh + h];
    const float x = xs[i], l2 = l2s[i];
    const float p2 = (x - l2) + corr;
    const float l2n = l2 - (x - p2);
    L2o[o] = l2n;
    W2[o] = p2 + l2n;
    if (p1mode == 2 || (sampled && p1mode == 1)) continue;
    const float bx = bxs[i], l1 = l1s[i];
    const float p1 = sampled ? (rho * bx + yls[i] - rho * l1) * inv_1prho : bx - l1;
    const float l1n = l1 - (bx - p1);
    L1o[o] = l1n;
    W1[o] = p1 + l1n;
  }
}

template <int LHM, int PU_NC, bool KEEP>
__global__ void __launch_bounds__(256 * PU_NC)
pupdate_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int x_s,
               int bx_s, int yl_s, int yh_s, int l1_s, int l2_s, int w1_s, int w2_s, int l1o_s,
               int l2o_s) {
  __shared__ float part[PU_NC > 1 ? PU_NC : 1][PU_NC > 1 ? LHM : 1][PU_NC > 1 ? 256 : 1];
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, L = S.L, Lh = S.Lh, d = S.d;
  // the band share is uniform over a wave (256 threads per share); readfirstlane lets the
  // band loops index R and G with scalar loads
  const int pix = threadIdx.x & 255;
  const int ch = PU_NC == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);
  const int j = it.y * 256 + pix;
  const size_t plane = (size_t)p * q;
  const bool act = j < (int)plane;
  const int c0 = (L * ch) / PU_NC, c1 = (L * (ch + 1)) / PU_NC;   // this thread's bands
  const gfloat* __restrict__ X = gslot<const gfloat>(S, x_s);
  const gfloat* L2 = gslot<const gfloat>(S, l2_s);
  const gfloat* __restrict__ R = as_global(S.R);
  const gfloat* __restrict__ G = as_global(S.G);
  const gfloat* __restrict__ Yh = gslot<const gfloat>(S, yh_s);
  // res = Y_h - A0 R.  The bands form kPuShares contiguous shares; each share's part of A0 R
  // is summed on its own and the parts are added in share order, so the result does not
  // depend on how many threads a pixel has.
  float res[LHM];
  // KEEP: every scene of the launch has at most kPuKeep bands per thread
  const int i1 = j / q, i2 = j - i1 * q;
  const bool sampled = (i1 % d == 0) && (i2 % d == 0);
  // p1mode 1: a basis couples the sampled pixels across bands (p1_subspace_kernel);
  // p1mode 2: fused-S splitting, no P1
  const int p1mode = S.fused ? 2 : (S.subspace ? 1 : 0);
  const bool p1 = !(p1mode == 2 || (sampled && p1mode == 1));
  const size_t lplane = (size_t)(p / d) * (q / d), lj = (size_t)(i1 / d) * (q / d) + i2 / d;
  float xs[KEEP ? kPuKeep : 1], l2s[KEEP ? kPuKeep : 1], bxs[KEEP ? kPuKeep : 1],
      l1s[KEEP ? kPuKeep : 1], yls[KEEP ? kPuKeep : 1], yh[LHM];
  if constexpr (KEEP)
    if (act)
    pupdate_load_keep<LHM>(X, L2, gslot<const gfloat>(S, bx_s), gslot<const gfloat>(S, l1_s),
                           gslot<const gfloat>(S, yl_s), p1, sampled, plane, lplane, lj, c0, c1,
                           j, xs, l2s, bxs, l1s, yls);
  if (act) {
#pragma unroll
    for (int h = 0; h < LHM; ++h) yh[h] = (h < Lh) ? Yh[h * plane + j] : 0.f;
  }
  if constexpr (PU_NC == 1) {
    // one thread per pixel: the parts are added in registers, and no barrier sits between
    // the two band loops (with one the memory-bound loops of different waves do not overlap)
    if (!act) return;
    float a[LHM];
#pragma unroll
    for (int h = 0; h < LHM; ++h) a[h] = 0.f;
    for (int k = 0; k < kPuShares; ++k) {
      float rp[LHM];
#pragma unroll
      for (int h = 0; h < LHM; ++h) rp[h] = 0.f;
      if constexpr (KEEP)
        pupdate_share_kept<LHM>(xs, l2s, R, rp, Lh, c0, (L * k) / kPuShares,
                                (L * (k + 1)) / kPuShares);
      else
        pupdate_share<LHM>(X, L2, R, rp, plane, Lh, (L * k) / kPuShares,
                           (L * (k + 1)) / kPuShares, j);
#pragma unroll
      for (int h = 0; h < LHM; ++h) a[h] += rp[h];
    }
#pragma unroll
    for (int h = 0; h < LHM; ++h) res[h] = (h < Lh) ? yh[h] - a[h] : 0.f;
  } else {
    static_assert(PU_NC == kPuShares, "one share per thread");
    float rp[LHM];
#pragma unroll
    for (int h = 0; h < LHM; ++h) rp[h] = 0.f;
    if (act) {
      if constexpr (KEEP) pupdate_share_kept<LHM>(xs, l2s, R, rp, Lh, c0, c0, c1);
      else pupdate_share<LHM>(X, L2, R, rp, plane, Lh, c0, c1, j);
    }
#pragma unroll
    for (int h = 0; h < LHM; ++h) part[ch][h][pix] = rp[h];
    __syncthreads();
    if (!act) return;
#pragma unroll
    for (int h = 0; h < LHM; ++h) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < PU_NC; ++k) a += part[k][h][pix];
      res[h] = (h < Lh) ? yh[h] - a : 0.f;
    }
  }
  float u[LHM];                           // u = res G
#pragma unroll
  for (int h2 = 0; h2 < LHM; ++h2) {
    float sum = 0.f;
#pragma unroll
    for (int h = 0; h < LHM; ++h)
      if (h < Lh && h2 < Lh) sum += res[h] * G[h * Lh + h2];
    u[h2] = sum;
  }
  if constexpr (KEEP)
    pupdate_write_kept<LHM>(xs, l2s, bxs, l1s, yls, gslot<gfloat>(S, l1o_s),
                            gslot<gfloat>(S, l2o_s), gslot<gfloat>(S, w1_s),
                            gslot<gfloat>(S, w2_s), R, u, plane, sampled, p1mode, Lh, S.rho,
                            S.inv_1prho, c0, c1, j);
  else
    pupdate_write<LHM>(X, gslot<const gfloat>(S, bx_s), gslot<const gfloat>(S, yl_s),
                       gslot<const gfloat>(S, l1_s), L2, gslot<gfloat>(S, l1o_s),
                       gslot<gfloat>(S, l2o_s), gslot<gfloat>(S, w1_s), gslot<gfloat>(S, w2_s),
                       R, u, plane, lplane, lj, sampled, p1mode, Lh, S.rho, S.inv_1prho, c0, c1,
                       j);
}

template <typename Kern, typename... Args>
int launch_groups(const Batch& B, Kind kind, const char* name, Kern kern, hipStream_t s,
                  Args... args) {
  for (const Group& g : B.groups[kind]) {
    if (g.nitems == 0) continue;
    hipLaunchKernelGGL(kern, dim3(g.nitems), dim3(g.block), g.lds, s, B.d_desc, g.d_items,
                       args...);
    NLPR_LAUNCH_CHECK(name);
  }
  return NLPR_OK;
}

// Buffer slots of descriptor 0 re-pointed on the stream (one thread per slot).
__global__ void set_slots_kernel(SceneDesc* sd, SlotSet set) {
  const int i = threadIdx.x;
  if (i < set.n) sd->buf[set.slot[i]] = set.ptr[i];
}

// Reference stream with the sweep's access shape and none of its arithmetic: workgroup b owns chunk
// (b mod bands) * per_band + b / bands of chunk4 float4s and negates it in place, P planes of
// 256 float4 (4 KB) at a time, all loads of a step before its stores.  The dynamic LDS the
// launch asks for is reserved per workgroup but not used: it limits the workgroups per CU as
// the sweep's tile does.
template <int P>
__global__ void __launch_bounds__(256) stream_chunks_kernel(float* buf, size_t chunk4,
                                                            int per_band, int bands) {
  const int b = blockIdx.x;
  const size_t c = (size_t)(b % bands) * per_band + b / bands;
  gv4f* base = reinterpret_cast<gv4f*>(as_global(buf)) + c * chunk4 + threadIdx.x;
  const size_t steps = chunk4 / (256 * P);
  for (size_t st = 0; st < steps; ++st) {
    gv4f* p = base + st * (256 * P);
    v4f_t v[P];
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = __builtin_nontemporal_load(p + j * 256);
#pragma unroll
    for (int j = 0; j < P; ++j) __builtin_nontemporal_store(-v[j], p + j * 256);
  }
}

// Reference stream: one 16-byte non-temporal load and store per thread, in place.
__global__ void __launch_bounds__(256) stream_rmw_kernel(float* buf, size_t n4) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n4) return;
  gv4f* p = reinterpret_cast<gv4f*>(as_global(buf)) + i;
  const v4f_t v = __builtin_nontemporal_load(p);
  __builtin_nontemporal_store(-v, p);
}

}  // namespace

// --------------------------------------------------------------------- work-item counts
int weights_blocks(const Plan& P) {
  return ceil_div(P.prm.q, WT_X) * ceil_div(P.prm.p, WT_Y) * P.npairs;
}
size_t weights_lds(const Plan& P) {
  const int K = P.prm.K;
  return (size_t)((WT_Y + 2 * K) * (WT_X + 2 * K) + (WT_Y + 2 * K) * WT_X) * sizeof(float);
}
int plane_blocks(const Plan& P) {
  return (int)(((size_t)P.Lx * P.prm.p * P.prm.q + 255) / 256);
}
int conv_blocks(const Plan& P) {
  return ceil_div(P.prm.q, CV_X) * ceil_div(P.prm.p, CV_Y) * P.Lx;
}
size_t conv_lds(const Plan& P) {
  // tile + the larger of the (2 RM + 1)^2 taps and (rank one) the row-filtered tile with u, v
  const int rm = conv_class(P.prm.blur_radius), w2 = 2 * rm + 1;
  return (size_t)((CV_Y + 2 * rm) * (CV_X + 2 * rm) +
                  std::max(w2 * w2, (CV_Y + 2 * rm) * CV_X + 2 * w2)) * sizeof(float);
}
int pixel_blocks(const Plan& P) { return ceil_div(P.prm.p * P.prm.q, 256); }

// ---------------------------------------------------------------------------- launches
int launch_precompute(Plan& P) {
  const int p = P.prm.p, q = P.prm.q;
  hipLaunchKernelGGL(twiddle_kernel, dim3(ceil_div(p, 256)), dim3(256), 0, nullptr, P.d_tw_p, p);
  NLPR_LAUNCH_CHECK("twiddle_kernel");
  hipLaunchKernelGGL(twiddle_kernel, dim3(ceil_div(q, 256)), dim3(256), 0, nullptr, P.d_tw_q, q);
  NLPR_LAUNCH_CHECK("twiddle_kernel");
  hipLaunchKernelGGL(den_kernel, dim3(ceil_div(q, 128), p), dim3(128), 0, nullptr, P.d_invden, p,
                     q, P.d_blur, P.prm.blur_radius, P.d_taus, P.npairs, P.npatch);
  NLPR_LAUNCH_CHECK("den_kernel");
  if (P.d_E) {
    hipLaunchKernelGGL(subspace_kernel, dim3(1), dim3(256), 0, nullptr, P.d_E, P.d_R, P.prm.L, P.Lx,
                       P.prm.Lh, P.prm.rho, P.d_M, P.d_Ep, P.d_Rt);
    NLPR_LAUNCH_CHECK("subspace_kernel");
  }
  if (P.d_fia) {
    const int groups = (p / P.prm.d) * (q / P.prm.d);
    hipLaunchKernelGGL(fused_tables_kernel, dim3(ceil_div(groups, 64)), dim3(64), 0, nullptr, p, q,
                       P.prm.d, P.d_blur, P.prm.blur_radius, P.d_taus, P.npairs, P.npatch,
                       P.prm.rho, P.d_fia, P.d_fu, P.d_fv);
    NLPR_LAUNCH_CHECK("fused_tables_kernel");
  }
  hipLaunchKernelGGL(g_kernel, dim3(1), dim3(256), 0, nullptr, P.d_E ? P.d_Rt : P.d_R, P.Lx,
                     P.prm.Lh, P.prm.rho / P.prm.lambda1, P.d_G);
  NLPR_LAUNCH_CHECK("g_kernel");
  return NLPR_OK;
}

int launch_weights(const Batch& B, int yh, int mu, hipStream_t s) {
  return launch_groups(B, KD_WEIGHTS, "weights_kernel", weights_kernel, s, yh, mu);
}

int launch_init(const Batch& B, int yl, int ylp, int x0, int l1, int l2, int w2, hipStream_t s) {
  return launch_groups(B, KD_PLANE, "init_kernel", init_kernel, s, yl, ylp, x0, l1, l2, w2);
}

int launch_upsample_zero(const Batch& B, int yl, int t, hipStream_t s) {
  return launch_groups(B, KD_PLANE, "upsample_zero_kernel", upsample_zero_kernel, s, yl, t);
}

int launch_set_slots(const Batch& B, const SlotSet& set, hipStream_t s) {
  if (set.n <= 0) return NLPR_OK;
  hipLaunchKernelGGL(set_slots_kernel, dim3(1), dim3(64), 0, s, B.d_desc, set);
  NLPR_LAUNCH_CHECK("set_slots_kernel");
  return NLPR_OK;
}

int launch_stream_rmw(float* buf, size_t n4, hipStream_t s) {
  if (!n4) return NLPR_OK;
  hipLaunchKernelGGL(stream_rmw_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, buf,
                     n4);
  NLPR_LAUNCH_CHECK("stream_rmw_kernel");
  return NLPR_OK;
}

template <int P>
int launch_chunks_p(float* buf, size_t chunk4, int nchunks, int bands, size_t lds, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    NLPR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(stream_chunks_kernel<P>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kMaxSweepLds));
    attr_set = true;
  }
  hipLaunchKernelGGL(stream_chunks_kernel<P>, dim3((unsigned)nchunks), dim3(256), lds, s, buf,
                     chunk4, nchunks / bands, bands);
  NLPR_LAUNCH_CHECK("stream_chunks_kernel");
  return NLPR_OK;
}

int launch_stream_chunks(float* buf, size_t chunk4, int nchunks, int bands, int planes,
                         size_t lds, hipStream_t s) {
  switch (planes) {
    case 1: return launch_chunks_p<1>(buf, chunk4, nchunks, bands, lds, s);
    case 2: return launch_chunks_p<2>(buf, chunk4, nchunks, bands, lds, s);
    case 3: return launch_chunks_p<3>(buf, chunk4, nchunks, bands, lds, s);
    case 4: return launch_chunks_p<4>(buf, chunk4, nchunks, bands, lds, s);
    case 5: return launch_chunks_p<5>(buf, chunk4, nchunks, bands, lds, s);
    case 6: return launch_chunks_p<6>(buf, chunk4, nchunks, bands, lds, s);
    case 7: return launch_chunks_p<7>(buf, chunk4, nchunks, bands, lds, s);
    default: return launch_chunks_p<8>(buf, chunk4, nchunks, bands, lds, s);
  }
}

int launch_fill(const Batch& B, int slot_, hipStream_t s) {
  return launch_groups(B, KD_PLANE, "fill_kernel", fill_kernel, s, slot_);
}

int launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  if (n <= 0) return NLPR_OK;
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  NLPR_LAUNCH_CHECK("zero_u64_kernel");
  return NLPR_OK;
}

int launch_finite_clear(int* flag, hipStream_t s) {
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
  NLPR_LAUNCH_CHECK("clear_flag_kernel");
  return NLPR_OK;
}

int launch_finite(const Batch& B, int z, int* flag, int iter, hipStream_t s) {
  return launch_groups(B, KD_PLANE, "finite_kernel", finite_kernel, s, z, flag, iter);
}

int conv_class(int r) {
  for (int rm : {1, 2, 4, 8}) if (r <= rm) return rm;
  return kMaxBlurRadius;
}

template <int RM>
int launch_conv_rm(const Group& g, const Batch& B, int in, int out, bool transpose, int add1,
                   int add2, int halo, int reg_mask, hipStream_t s) {
  auto kern = transpose ? conv_kernel<true, RM> : conv_kernel<false, RM>;
  hipLaunchKernelGGL(kern, dim3(g.nitems), dim3(256), g.lds, s, B.d_desc, g.d_items, in, out, add1,
                     add2, halo, reg_mask);
  NLPR_LAUNCH_CHECK("conv_kernel");
  return NLPR_OK;
}

// one launch per blur-radius class (key0 = RM)
int launch_conv(const Batch& B, int in, int out, bool transpose, int add1, int add2, int halo,
                int reg_mask, hipStream_t s) {
  for (const Group& g : B.groups[KD_CONV]) {
    if (!g.nitems) continue;
    int rc;
    switch (g.key0) {
      case 1: rc = launch_conv_rm<1>(g, B, in, out, transpose, add1, add2, halo, reg_mask, s); break;
      case 2: rc = launch_conv_rm<2>(g, B, in, out, transpose, add1, add2, halo, reg_mask, s); break;
      case 4: rc = launch_conv_rm<4>(g, B, in, out, transpose, add1, add2, halo, reg_mask, s); break;
      case 8: rc = launch_conv_rm<8>(g, B, in, out, transpose, add1, add2, halo, reg_mask, s); break;
      default:
        rc = launch_conv_rm<kMaxBlurRadius>(g, B, in, out, transpose, add1, add2, halo, reg_mask, s);
    }
    if (rc) return rc;
  }
  return NLPR_OK;
}

template <int LHM, int NC>
void launch_pu(const Batch& B, const Group& g, int x, int bx, int yl, int yh, int l1, int l2,
               int w1, int w2, int l1o, int l2o, hipStream_t s) {
  int maxL = 0;
  for (const auto& P : B.scenes) maxL = std::max(maxL, P->Lx);
  if (maxL <= kPuKeep * NC)
    hipLaunchKernelGGL((pupdate_kernel<LHM, NC, true>), dim3(g.nitems), dim3(256 * NC), 0, s,
                       B.d_desc, g.d_items, x, bx, yl, yh, l1, l2, w1, w2, l1o, l2o);
  else
    hipLaunchKernelGGL((pupdate_kernel<LHM, NC, false>), dim3(g.nitems), dim3(256 * NC), 0, s,
                       B.d_desc, g.d_items, x, bx, yl, yh, l1, l2, w1, w2, l1o, l2o);
}

int launch_pupdate(const Batch& B, int x, int bx, int yl, int yh, int l1, int l2, int w1, int w2,
                   int l1o, int l2o, hipStream_t s) {
  // one launch per guide-band class (key0 = 1, 4 or 16 register slots) and threads per
  // pixel (key1 = 1 or 4)
  for (const Group& g : B.groups[KD_PIXEL]) {
    if (!g.nitems) continue;
    const bool split = g.key1 == 4;
    if (g.key0 == 1) {
      if (split) launch_pu<1, 4>(B, g, x, bx, yl, yh, l1, l2, w1, w2, l1o, l2o, s);
      else launch_pu<1, 1>(B, g, x, bx, yl, yh, l1, l2, w1, w2, l1o, l2o, s);
    } else if (g.key0 == 4) {
      if (split) launch_pu<4, 4>(B, g, x, bx, yl, yh, l1, l2, w1, w2, l1o, l2o, s);
      else launch_pu<4, 1>(B, g, x, bx, yl, yh, l1, l2, w1, w2, l1o, l2o, s);
    } else {
      if (split) launch_pu<kMaxLh, 4>(B, g, x, bx, yl, yh, l1, l2, w1, w2, l1o, l2o, s);
      else launch_pu<kMaxLh, 1>(B, g, x, bx, yl, yh, l1, l2, w1, w2, l1o, l2o, s);
    }
    NLPR_LAUNCH_CHECK("pupdate_kernel");
  }
  return NLPR_OK;
}

int lowres_blocks(const Plan& P) {
  return ceil_div((P.prm.p / P.prm.d) * (P.prm.q / P.prm.d), 256);
}

int launch_project(const Batch& B, int yl, int yle, int ylp, hipStream_t s) {
  return launch_groups(B, KD_LOWRES, "project_kernel", project_kernel, s, yl, yle, ylp);
}

int launch_p1_subspace(const Batch& B, int bx, int yle, int l1, int w1, hipStream_t s) {
  return launch_groups(B, KD_LOWRES, "p1_subspace_kernel", p1_subspace_kernel, s, bx, yle, l1, w1);
}

int launch_compose(const Batch& B, int x, int z, hipStream_t s) {
  return launch_groups(B, KD_COMPOSE, "compose_kernel", compose_kernel, s, x, z);
}

int lh_class(int Lh) { return Lh == 1 ? 1 : (Lh <= 4 ? 4 : kMaxLh); }

}  // namespace nlpr
