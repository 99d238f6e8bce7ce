// Monitor of the ADMM iteration: the objective of eq. (mainoptim) split into its three
// terms at the current iterate X, and the primal residuals ||B X - P1||, ||X - P2|| of the
// constraints of eq. (fusionoptim).  It runs after the P-update of a monitored iteration,
// when X, B X, P1 + Lambda1, P2 + Lambda2 and the new duals are all in place, and only
// reads them.
//
// Each workgroup forms its terms in FP32 (differences and contractions in FP64 where
// cancellation would cost digits) and writes one FP64 partial sum; one workgroup per
// scene then adds the partials in a fixed order, so the trace is bit-for-bit repeatable.
//
// The regulariser of eq. (regfilt1) uses the same reductions as the sweep: the terms of
// -tau equal those of tau (antisymmetry of omega and D), tau = 0 adds nothing, and with
// D_{tau k} X(i) = g_tau(i - k), g_tau = X - X(. - tau),
//   sum_i omega_{i tau} sum_k |D_{tau k} X(i)| = sum_j |g_tau(j)| sum_k omega_{j+k, tau}.
// With mu = lambda2 omega / rho in the workspace, lambda2 phi(X) =
//   2 rho sum_{tau in W+} sum_j (sum_k mu_{j+k, tau}) sum_c |g_tau(j, c)|.
#include "nlpr_internal.h"

namespace nlpr {
namespace {

constexpr int MR_Y = 32, MR_X = 64;   // regulariser tile: 32 rows x 64 columns, 8 rows/thread

__device__ __forceinline__ int wrapm(int a, int m) {
  a %= m;
  return a < 0 ? a + m : a;
}

// Sum of v[k] over the 256 threads of the workgroup, in a fixed order; thread 0 gets it.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
  __shared__ double red[N][4];
#pragma unroll
  for (int k = 0; k < N; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) red[k][w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
}

// Per pixel: data_l (sampled pixels), data_h, ||B X - P1||^2 and ||X - P2||^2 summed over
// bands; P1 = W1 - Lambda1 and P2 = W2 - Lambda2.  Work items of the pixel launches.
__global__ void __launch_bounds__(256)
monitor_pixel_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int x_s,
                     int bx_s, int yl_s, int yh_s, int l1_s, int l2_s, int w1_s, int w2_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, L = S.L, Lh = S.Lh, d = S.d;
  const size_t plane = (size_t)p * q;
  const int j = it.y * 256 + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};   // data_l, data_h, r1^2, r2^2 (unscaled)
  if (j < (int)plane) {
    const gfloat* X = gslot<const gfloat>(S, x_s);
    const gfloat* BX = gslot<const gfloat>(S, bx_s);
    const gfloat* L1 = gslot<const gfloat>(S, l1_s);
    const gfloat* L2 = gslot<const gfloat>(S, l2_s);
    const gfloat* W1 = gslot<const gfloat>(S, w1_s);
    const gfloat* W2 = gslot<const gfloat>(S, w2_s);
    const gfloat* R = as_global(S.R);   // [L][Lh] (E R with a basis)
    double hr[kMaxLh];
#pragma unroll
    for (int h = 0; h < kMaxLh; ++h) hr[h] = 0.0;
    for (int c = 0; c < L; ++c) {
      const size_t o = (size_t)c * plane + j;
      const double x = X[o], bx = BX[o];
      const double e2 = x - ((double)W2[o] - (double)L2[o]);
      if (!S.fused) {                     // the fused-S splitting has no P1 = B X constraint
        const double e1 = bx - ((double)W1[o] - (double)L1[o]);
        acc[2] += e1 * e1;
      }
      acc[3] += e2 * e2;
#pragma unroll
      for (int h = 0; h < kMaxLh; ++h)
        if (h < Lh) hr[h] += x * (double)R[c * Lh + h];
    }
    const gfloat* Yh = gslot<const gfloat>(S, yh_s);
#pragma unroll
    for (int h = 0; h < kMaxLh; ++h)
      if (h < Lh) {
        const double e = (double)Yh[(size_t)h * plane + j] - hr[h];
        acc[1] += e * e;
      }
    const int i1 = j / q, i2 = j - (j / q) * q;
    if (i1 % d == 0 && i2 % d == 0) {
      const int nl = (p / d) * (q / d);
      const int m = (i1 / d) * (q / d) + i2 / d;
      const gfloat* Yl = gslot<const gfloat>(S, yl_s);
      if (!S.subspace) {
        for (int c = 0; c < L; ++c) {
          const double e = (double)Yl[(size_t)c * nl + m] - (double)BX[(size_t)c * plane + j];
          acc[0] += e * e;
        }
      } else {
        // Y_l has Lz bands; (B X E)_c = sum_s (B X)_s E[s][c]
        const gfloat* E = as_global(S.E);
        float bx[kMaxLs];
#pragma unroll
        for (int s = 0; s < kMaxLs; ++s) bx[s] = s < L ? BX[(size_t)s * plane + j] : 0.f;
        for (int c = 0; c < S.Lz; ++c) {
          double z = 0.0;
#pragma unroll
          for (int s = 0; s < kMaxLs; ++s)
            if (s < L) z += (double)bx[s] * (double)E[s * S.Lz + c];
          const double e = (double)Yl[(size_t)c * nl + m] - z;
          acc[0] += e * e;
        }
      }
    }
  }
  block_sum(acc);
  if (threadIdx.x == 0) {
    gdouble* part = (gdouble*)S.mon + 4 * (size_t)it.y;
#pragma unroll
    for (int k = 0; k < 4; ++k) part[k] = acc[k];
  }
}

// Regulariser partial of one (shift, tile): sum over the tile of
// (sum_k mu_{j+k, tau}) * sum_c |X(j, c) - X(j - tau, c)|.
__global__ void __launch_bounds__(256)
monitor_reg_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int x_s,
                   int mu_s) {
  extern __shared__ float msh[];
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, K = S.K, L = S.L;
  const int gx = ceil_div(q, MR_X), gy = ceil_div(p, MR_Y);
  const int n = it.y / (gx * gy);
  const int rem = it.y - n * gx * gy;
  const int y0 = (rem / gx) * MR_Y, x0 = (rem % gx) * MR_X;
  const int TX = MR_X + 2 * K, TY = MR_Y + 2 * K;
  const size_t plane = (size_t)p * q;
  const int2 t = tau_at(S, n);
  // mu(., tau) on the tile with a K halo (circular)
  const gfloat* mun = gslot<const gfloat>(S, mu_s) + (size_t)n * plane;
  for (int e = threadIdx.x; e < TY * TX; e += 256) {
    const int yy = e / TX, xx = e - (e / TX) * TX;
    msh[e] = mun[(size_t)wrapm(y0 - K + yy, p) * q + wrapm(x0 - K + xx, q)];
  }
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const gfloat* X = gslot<const gfloat>(S, x_s);
  int o1[8], o2[8];
  bool ok[8];
  float g[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int y = y0 + ty + 4 * r, x = x0 + tx;
    ok[r] = y < p && x < q;
    o1[r] = ok[r] ? y * q + x : 0;
    o2[r] = ok[r] ? wrapm(y - t.x, p) * q + wrapm(x - t.y, q) : 0;
    g[r] = 0.f;
  }
  for (int c = 0; c < L; ++c) {
    const gfloat* Xc = X + (size_t)c * plane;
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (ok[r]) g[r] += fabsf(Xc[o1[r]] - Xc[o2[r]]);
  }
  double acc[1] = {0.0};
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (!ok[r]) continue;
    float om = 0.f;
    const float* base = msh + (ty + 4 * r) * TX + tx;
    for (int a = 0; a <= 2 * K; ++a)
      for (int b = 0; b <= 2 * K; ++b) om += base[a * TX + b];
    acc[0] += (double)g[r] * (double)om;
  }
  block_sum(acc);
  if (threadIdx.x == 0) ((gdouble*)S.mon)[4 * (size_t)S.mon_npix + it.y] = acc[0];
}

// One workgroup per scene: add the partials in a fixed order and write record `point`.
__global__ void __launch_bounds__(256)
monitor_reduce_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items,
                      int point, int iter) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const gdouble* part = (const gdouble*)S.mon;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < S.mon_npix; b += 256)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += part[4 * (size_t)b + k];
  for (int b = threadIdx.x; b < S.mon_nreg; b += 256) v[4] += part[4 * (size_t)S.mon_npix + b];
  block_sum(v);
  if (threadIdx.x == 0) {
    gdouble* rec = (gdouble*)S.mon + 4 * (size_t)S.mon_npix + S.mon_nreg + 8 * (size_t)point;
    const double dl = 0.5 * v[0], dh = 0.5 * S.lam1_d * v[1], reg = 2.0 * S.rho_d * v[4];
    rec[0] = iter;
    rec[1] = dl + dh + reg;
    rec[2] = dl;
    rec[3] = dh;
    rec[4] = reg;
    rec[5] = sqrt(v[2]);
    rec[6] = sqrt(v[3]);
    rec[7] = 0.0;
  }
}

}  // namespace

int monreg_blocks(const Plan& P) {
  return P.npairs * ceil_div(P.prm.p, MR_Y) * ceil_div(P.prm.q, MR_X);
}
size_t monreg_lds(const Plan& P) {
  return (size_t)(MR_Y + 2 * P.prm.K) * (MR_X + 2 * P.prm.K) * sizeof(float);
}
int monitor_points(int iters, int every) {
  if (every <= 0 || iters <= 0) return 0;
  return iters / every + (iters % every ? 1 : 0);
}

int launch_monitor(const Batch& B, int point, int iter, hipStream_t s) {
  for (const Group& g : B.groups[KD_PIXEL]) {
    if (!g.nitems) continue;
    hipLaunchKernelGGL(monitor_pixel_kernel, dim3(g.nitems), dim3(256), 0, s, B.d_desc,
                       g.d_items, (int)B_Z, (int)B_BX, (int)B_YL, (int)B_YH, (int)B_L1,
                       (int)B_L2, (int)B_W1, (int)B_W2);
    NLPR_LAUNCH_CHECK("monitor_pixel_kernel");
  }
  for (const Group& g : B.groups[KD_MONREG]) {
    if (!g.nitems) continue;
    hipLaunchKernelGGL(monitor_reg_kernel, dim3(g.nitems), dim3(256), g.lds, s, B.d_desc,
                       g.d_items, (int)B_Z, (int)B_MU);
    NLPR_LAUNCH_CHECK("monitor_reg_kernel");
  }
  for (const Group& g : B.groups[KD_SCENE]) {
    if (!g.nitems) continue;
    hipLaunchKernelGGL(monitor_reduce_kernel, dim3(g.nitems), dim3(256), 0, s, B.d_desc,
                       g.d_items, point, iter);
    NLPR_LAUNCH_CHECK("monitor_reduce_kernel");
  }
  return NLPR_OK;
}

}  // namespace nlpr
