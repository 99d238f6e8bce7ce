// X-update of the ADMM iteration: X_c = IDFT2(DFT2(C_c) / den) for every band c
// (Sec. "Optimization", eqs. (xupdateoper), (inv)).
//
// Two real bands a = 2m, b = 2m+1 are packed into one complex image C_a + i C_b.  The
// spectral weight 1/den is real and even (den(-w) = den(w)), so filtering the packed image
// and splitting real / imaginary parts gives the two filtered bands exactly; one complex
// 2-D transform pair serves two bands.
//
// The 2-D transform runs as three passes over a complex [pairs][p][q] buffer:
//   rows_fwd   : pack two bands, forward DFT along every row
//   cols_solve : forward DFT along columns, multiply by 1/(den p q), inverse DFT along
//                columns (the column data stays in LDS between the two transforms)
//   rows_inv   : inverse DFT along rows, unpack the two bands
// Each 1-D transform is a Stockham autosort FFT (mixed radix 2/3/4/8) staged in LDS:
// every stage reads R values strided by n/R, twiddles them, does an R-point DFT and writes
// them to their natural-order position, so no bit reversal is needed.  Twiddles come from
// a table computed in FP64.
#include "nlpr_internal.h"

namespace nlpr {
namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * (-i) for the forward transform, a * (+i) for the inverse
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV> struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = rot90<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, t3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, t3);
  }
};

template <bool INV> struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    const float c = 0.70710678118654752440f;
    // w8^s, w8 = exp(-+ 2 pi i / 8)
    const float2 w1 = INV ? make_float2(c, c) : make_float2(c, -c);
    const float2 w3 = INV ? make_float2(-c, c) : make_float2(-c, -c);
    float2 o1 = cmul(o[1], w1), o2 = rot90<INV>(o[2]), o3 = cmul(o[3], w3);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <bool INV> struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float s3 = 0.86602540378443864676f;  // sqrt(3)/2
    float2 a = v[0], b = v[1], c = v[2];
    float2 t1 = cadd(b, c);
    float2 t2 = csub(a, cscale(t1, 0.5f));
    float2 t3 = cscale(rot90<INV>(csub(b, c)), s3);
    v[0] = cadd(a, t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
};

// One Stockham stage of radix R on a line of n points in LDS.  Ns is the product of the
// radices of the earlier stages.  Threads t < tpl of the line take part; tpl >= ceil(n/8)
// keeps every thread at <= ceil(8/R) butterflies.  All threads of the block must call it.
template <int R, bool INV>
__device__ void fft_stage(float2* buf, int n, int Ns, const float2* __restrict__ tw, int t,
                          int tpl) {
  constexpr int MAXB = (8 + R - 1) / R;
  const int nb = n / R;
  float2 v[MAXB][R];
#pragma unroll
  for (int u = 0; u < MAXB; ++u) {
    const int j = t + u * tpl;
    if (t < tpl && j < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[u][r] = buf[j + r * nb];
    }
  }
  __syncthreads();
  const int step = n / (Ns * R);
#pragma unroll
  for (int u = 0; u < MAXB; ++u) {
    const int j = t + u * tpl;
    if (t < tpl && j < nb) {
      const int k = j % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * k * step];
        if (INV) w.y = -w.y;
        v[u][r] = cmul(v[u][r], w);
      }
      Dft<R, INV>::run(v[u]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[u][r];
    }
  }
  __syncthreads();
}

template <bool INV>
__device__ void fft_line(float2* buf, const LineFFT& f, int t, int tpl) {
  int Ns = 1;
  for (int s = 0; s < f.nfac; ++s) {
    const int R = f.fac[s];
    if (R == 8) fft_stage<8, INV>(buf, f.n, Ns, f.tw, t, tpl);
    else if (R == 4) fft_stage<4, INV>(buf, f.n, Ns, f.tw, t, tpl);
    else if (R == 2) fft_stage<2, INV>(buf, f.n, Ns, f.tw, t, tpl);
    else fft_stage<3, INV>(buf, f.n, Ns, f.tw, t, tpl);
    Ns *= R;
  }
}

// Pack bands (2m, 2m+1) of C, forward DFT along rows.  grid (ceil(p / lpb), pairs).
__global__ void fft_rows_fwd(const float* __restrict__ C, float2* __restrict__ F, int p, int q,
                             int L, LineFFT fq, int tpl, int lpb) {
  extern __shared__ float2 sh[];
  const int m = blockIdx.y;
  const size_t plane = (size_t)p * q;
  const float* Ca = C + (size_t)(2 * m) * plane;
  const float* Cb = (2 * m + 1 < L) ? C + (size_t)(2 * m + 1) * plane : nullptr;
  const int row0 = blockIdx.x * lpb;
  for (int e = threadIdx.x; e < lpb * q; e += blockDim.x) {
    const int l = e / q, i = e - l * q, r = row0 + l;
    float2 v = make_float2(0.f, 0.f);
    if (r < p) {
      v.x = Ca[(size_t)r * q + i];
      if (Cb) v.y = Cb[(size_t)r * q + i];
    }
    sh[e] = v;
  }
  __syncthreads();
  const int g = threadIdx.x / tpl;
  const int t = (g < lpb) ? threadIdx.x - g * tpl : tpl;
  fft_line<false>(sh + (g < lpb ? g : 0) * q, fq, t, tpl);
  float2* Fm = F + (size_t)m * plane;
  for (int e = threadIdx.x; e < lpb * q; e += blockDim.x) {
    const int l = e / q, i = e - l * q, r = row0 + l;
    if (r < p) Fm[(size_t)r * q + i] = sh[e];
  }
}

// Forward DFT along columns, multiply by invden, inverse DFT along columns.
// grid (ceil(q / cb), pairs); LDS holds cb columns of p points.
__global__ void fft_cols_solve(float2* __restrict__ F, const float* __restrict__ invden, int p,
                               int q, LineFFT fp, int tpl, int cb) {
  extern __shared__ float2 sh[];
  const int m = blockIdx.y;
  const int c0 = blockIdx.x * cb;
  const size_t plane = (size_t)p * q;
  float2* Fm = F + (size_t)m * plane;
  for (int e = threadIdx.x; e < cb * p; e += blockDim.x) {
    const int i = e / cb, l = e - i * cb, col = c0 + l;
    sh[l * p + i] = (col < q) ? Fm[(size_t)i * q + col] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int G = blockDim.x / tpl;
  const int g = threadIdx.x / tpl;
  const int tl = threadIdx.x - g * tpl;
  for (int base = 0; base < cb; base += G) {
    const int l = base + g;
    const bool act = (g < G) && (l < cb);
    const int t = act ? tl : tpl;
    float2* line = sh + (act ? l : 0) * p;
    fft_line<false>(line, fp, t, tpl);
    if (act && c0 + l < q) {
      for (int i = tl; i < p; i += tpl) {
        const float s = invden[(size_t)i * q + c0 + l];
        line[i] = cscale(line[i], s);
      }
    }
    __syncthreads();
    fft_line<true>(line, fp, t, tpl);
  }
  for (int e = threadIdx.x; e < cb * p; e += blockDim.x) {
    const int i = e / cb, l = e - i * cb, col = c0 + l;
    if (col < q) Fm[(size_t)i * q + col] = sh[l * p + i];
  }
}

// Inverse DFT along rows, unpack bands (2m, 2m+1) into X.
__global__ void fft_rows_inv(const float2* __restrict__ F, float* __restrict__ X, int p, int q,
                             int L, LineFFT fq, int tpl, int lpb) {
  extern __shared__ float2 sh[];
  const int m = blockIdx.y;
  const size_t plane = (size_t)p * q;
  const float2* Fm = F + (size_t)m * plane;
  const int row0 = blockIdx.x * lpb;
  for (int e = threadIdx.x; e < lpb * q; e += blockDim.x) {
    const int l = e / q, i = e - l * q, r = row0 + l;
    sh[e] = (r < p) ? Fm[(size_t)r * q + i] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int g = threadIdx.x / tpl;
  const int t = (g < lpb) ? threadIdx.x - g * tpl : tpl;
  fft_line<true>(sh + (g < lpb ? g : 0) * q, fq, t, tpl);
  float* Xa = X + (size_t)(2 * m) * plane;
  float* Xb = (2 * m + 1 < L) ? X + (size_t)(2 * m + 1) * plane : nullptr;
  for (int e = threadIdx.x; e < lpb * q; e += blockDim.x) {
    const int l = e / q, i = e - l * q, r = row0 + l;
    if (r < p) {
      const float2 v = sh[e];
      Xa[(size_t)r * q + i] = v.x;
      if (Xb) Xb[(size_t)r * q + i] = v.y;
    }
  }
}

int block_for(int tpl) {
  int b = 256;
  while (b < tpl) b *= 2;
  return b;
}

}  // namespace

int launch_xsolve(const Plan& P, const float* C, float* X, float2* F, hipStream_t s) {
  const int p = P.prm.p, q = P.prm.q, L = P.prm.L;
  const int pairs = (L + 1) / 2;
  {
    const int tpl = ceil_div(q, 8);
    const int bs = block_for(tpl);
    int lpb = bs / tpl;
    while (lpb > 1 && (size_t)lpb * q * sizeof(float2) > 65536) --lpb;
    dim3 grid(ceil_div(p, lpb), pairs);
    hipLaunchKernelGGL(fft_rows_fwd, grid, dim3(bs), (size_t)lpb * q * sizeof(float2), s, C, F, p,
                       q, L, P.fq, tpl, lpb);
    NLPR_LAUNCH_CHECK("fft_rows_fwd");
  }
  {
    const int tpl = ceil_div(p, 8);
    const int bs = block_for(tpl);
    int cb = 16;
    while (cb > 1 && (size_t)cb * p * sizeof(float2) > 65536) cb /= 2;
    dim3 grid(ceil_div(q, cb), pairs);
    hipLaunchKernelGGL(fft_cols_solve, grid, dim3(bs), (size_t)cb * p * sizeof(float2), s, F,
                       P.d_invden, p, q, P.fp, tpl, cb);
    NLPR_LAUNCH_CHECK("fft_cols_solve");
  }
  {
    const int tpl = ceil_div(q, 8);
    const int bs = block_for(tpl);
    int lpb = bs / tpl;
    while (lpb > 1 && (size_t)lpb * q * sizeof(float2) > 65536) --lpb;
    dim3 grid(ceil_div(p, lpb), pairs);
    hipLaunchKernelGGL(fft_rows_inv, grid, dim3(bs), (size_t)lpb * q * sizeof(float2), s, F, X, p,
                       q, L, P.fq, tpl, lpb);
    NLPR_LAUNCH_CHECK("fft_rows_inv");
  }
  return NLPR_OK;
}

}  // namespace nlpr
