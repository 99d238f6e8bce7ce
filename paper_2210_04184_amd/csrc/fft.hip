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
// Every pass runs over a batch of scenes (see nlpr_internal.h); lines per block and columns
// per block are picked per image size by timing candidates when a plan is created.
// Each 1-D transform is a Stockham autosort FFT (mixed radix 2/3/4/8) staged in LDS:
// every stage reads R values strided by n/R, twiddles them, does an R-point DFT and writes
// them to their natural-order position, so no bit reversal is needed.  Twiddles come from
// a table computed in FP64.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

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
// radices of the earlier stages; tw holds the line's n twiddles, staged in LDS.  Threads
// t < tpl of the line take part; tpl >= ceil(n/8) keeps every thread at <= ceil(8/R)
// butterflies.  All threads of the block must call it.
template <int R, bool INV>
__device__ __forceinline__ void fft_stage(float2* buf, int n, int Ns, const float2* tw, int t,
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

// Twiddles of a line length, copied from the FP64-computed table to LDS (before the
// barrier that follows the data load) so the stages read them without global latency.
__device__ __forceinline__ void stage_twiddles(float2* twl, const LineFFT& f) {
  const gfloat* tw = (const gfloat*)f.tw;
  for (int e = threadIdx.x; e < f.n; e += blockDim.x) twl[e] = ldg2(tw + 2 * e);
}

template <bool INV>
__device__ __forceinline__ void fft_line(float2* buf, const LineFFT& f, int t, int tpl,
                                         const float2* tw) {
  int Ns = 1;
  for (int s = 0; s < f.nfac; ++s) {
    const int R = f.fac[s];
    if (R == 8) fft_stage<8, INV>(buf, f.n, Ns, tw, t, tpl);
    else if (R == 4) fft_stage<4, INV>(buf, f.n, Ns, tw, t, tpl);
    else if (R == 2) fft_stage<2, INV>(buf, f.n, Ns, tw, t, tpl);
    else fft_stage<3, INV>(buf, f.n, Ns, tw, t, tpl);
    Ns *= R;
  }
}

// Pack bands (2m, 2m+1) of C, forward DFT along rows.  Local block = (pair, row block).
__global__ void fft_rows_fwd(const SceneDesc* __restrict__ sd, const int2* __restrict__ items,
                             int c_s, int f_s) {
  extern __shared__ float2 sh[];
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, L = S.L, lpb = S.fq_lpb, tpl = S.fq_tpl;
  const int nrb = ceil_div(p, lpb);
  const int m = it.y / nrb, row0 = (it.y - m * nrb) * lpb;
  const size_t plane = (size_t)p * q;
  const gfloat* C = gslot<const gfloat>(S, c_s);
  float2* twl = sh + lpb * q;
  stage_twiddles(twl, S.fq);
  const gfloat* Ca = C + (size_t)(2 * m) * plane;
  const gfloat* Cb = (2 * m + 1 < L) ? C + (size_t)(2 * m + 1) * plane : nullptr;
  // 16-byte loads (4 points of a row; q % 4 == 0) when the buffer allows, else 4-byte ones
  if ((reinterpret_cast<uintptr_t>(C) & 15) == 0) {
    const int q4 = q >> 2;
    for (int e = threadIdx.x; e < lpb * q4; e += blockDim.x) {
      const int l = e / q4, i4 = e - l * q4, r = row0 + l;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
      if (r < p) {
        a = ldg4(Ca + (size_t)r * q + 4 * i4);
        if (Cb) b = ldg4(Cb + (size_t)r * q + 4 * i4);
      }
      float2* d = sh + l * q + 4 * i4;
      d[0] = make_float2(a.x, b.x);
      d[1] = make_float2(a.y, b.y);
      d[2] = make_float2(a.z, b.z);
      d[3] = make_float2(a.w, b.w);
    }
  } else {
    for (int e = threadIdx.x; e < lpb * q; e += blockDim.x) {
      const int l = e / q, i = e - l * q, r = row0 + l;
      float2 v = make_float2(0.f, 0.f);
      if (r < p) {
        v.x = Ca[(size_t)r * q + i];
        if (Cb) v.y = Cb[(size_t)r * q + i];
      }
      sh[e] = v;
    }
  }
  __syncthreads();
  const int g = threadIdx.x / tpl;
  const int t = (g < lpb) ? threadIdx.x - g * tpl : tpl;
  fft_line<false>(sh + (g < lpb ? g : 0) * q, S.fq, t, tpl, twl);
  gfloat* Fm = gslot<gfloat>(S, f_s) + 2 * (size_t)m * plane;   // complex, interleaved
  const int q2 = q >> 1;                // two complex points per 16-byte store
  for (int e = threadIdx.x; e < lpb * q2; e += blockDim.x) {
    const int l = e / q2, i2 = e - l * q2, r = row0 + l;
    if (r < p) {
      const float2 u = sh[l * q + 2 * i2], w = sh[l * q + 2 * i2 + 1];
      stg4(Fm + 2 * ((size_t)r * q + 2 * i2), make_float4(u.x, u.y, w.x, w.y));
    }
  }
}

// Forward DFT along columns, multiply by invden, inverse DFT along columns.
// Local block = (pair, column block); LDS holds cb columns of p points.
//
// Fused-S scenes solve, per aliasing group of d^2 frequencies, the system of
// fused_tables_kernel instead of the division: line l of the block holds column
// b0 + (l % cbb) + (l / cbb) q/d (cbb = cb / d base columns and their d - 1 column aliases),
// so each group's d^2 entries (rows i1 + m1 p/d of those d columns) are in LDS.  All lines
// are transformed forward, the group solves run, then all lines are transformed back.
__global__ void fft_cols_solve(const SceneDesc* __restrict__ sd, const int2* __restrict__ items,
                               int f_s) {
  extern __shared__ float2 sh[];
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, cb = S.fp_cb, tpl = S.fp_tpl;
  const int ncb = ceil_div(q, cb);
  const int m = it.y / ncb, cblk = it.y - m * ncb;
  const size_t plane = (size_t)p * q;
  gfloat* Fm = gslot<gfloat>(S, f_s) + 2 * (size_t)m * plane;   // complex, interleaved
  float2* twl = sh + cb * p;
  stage_twiddles(twl, S.fp);
  const int d = S.d, cbb = S.fused ? cb / d : cb, qd = q / d;
  // column of LDS line l (-1: past the image)
  auto column = [&](int l) -> int {
    if (!S.fused) {
      const int col = cblk * cb + l;
      return col < q ? col : -1;
    }
    const int bc = cblk * cbb + l % cbb;
    return bc < qd ? bc + (l / cbb) * qd : -1;
  };
  // plain layout with an even block width: two neighbouring columns per 16-byte access
  const bool pairs = !S.fused && (cb & 1) == 0;
  if (pairs) {
    const int cb2 = cb >> 1;
    for (int e = threadIdx.x; e < cb2 * p; e += blockDim.x) {
      const int i = e / cb2, l = 2 * (e - i * cb2), col = cblk * cb + l;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (col + 1 < q) {
        v = ldg4(Fm + 2 * ((size_t)i * q + col));
      } else if (col < q) {
        const float2 u = ldg2(Fm + 2 * ((size_t)i * q + col));
        v.x = u.x;
        v.y = u.y;
      }
      sh[l * p + i] = make_float2(v.x, v.y);
      sh[(l + 1) * p + i] = make_float2(v.z, v.w);
    }
  } else {
    for (int e = threadIdx.x; e < cb * p; e += blockDim.x) {
      const int i = e / cb, l = e - i * cb, col = column(l);
      sh[l * p + i] = (col >= 0) ? ldg2(Fm + 2 * ((size_t)i * q + col)) : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  const int G = blockDim.x / tpl;
  const int g = threadIdx.x / tpl;
  const int tl = threadIdx.x - g * tpl;
  if (!S.fused) {
    // 1/den of the line's points is requested before the forward transform, so its latency
    // overlaps the transform (a line has at most 8 tpl points)
    const gfloat* invden = as_global(S.invden);
    for (int base = 0; base < cb; base += G) {
      const int l = base + g;
      const bool act = (g < G) && (l < cb);
      const int t = act ? tl : tpl;
      float2* line = sh + (act ? l : 0) * p;
      const int col = act ? column(l) : -1;
      float sv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = tl + u * tpl;
        sv[u] = (col >= 0 && i < p) ? invden[(size_t)i * q + col] : 0.f;
      }
      fft_line<false>(line, S.fp, t, tpl, twl);
      if (col >= 0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = tl + u * tpl;
          if (i < p) line[i] = cscale(line[i], sv[u]);
        }
      }
      __syncthreads();
      fft_line<true>(line, S.fp, t, tpl, twl);
    }
  } else {
    for (int base = 0; base < cb; base += G) {
      const int l = base + g;
      const bool act = (g < G) && (l < cb);
      fft_line<false>(sh + (act ? l : 0) * p, S.fp, act ? tl : tpl, tpl, twl);
    }
    // group solves: (i1, base column) pairs, i1 fastest (tables are column-major)
    const int pd = p / d;
    const gfloat* ia = as_global(S.fia);
    const gfloat* fu = (const gfloat*)S.fu;
    const gfloat* fv = (const gfloat*)S.fv;
    for (int e = threadIdx.x; e < pd * cbb; e += blockDim.x) {
      const int bcl = e / pd, i1 = e - bcl * pd;
      if (cblk * cbb + bcl >= qd) continue;
      const int col0 = cblk * cbb + bcl;
      float tr = 0.f, ti = 0.f;          // t = sum_k u_k c_k
      for (int m2 = 0; m2 < d; ++m2) {
        const size_t cbase = (size_t)(col0 + m2 * qd) * p;
        const float2* ln = sh + (m2 * cbb + bcl) * p;
        for (int m1 = 0; m1 < d; ++m1) {
          const int i = i1 + m1 * pd;
          const float2 u = ldg2(fu + 2 * (cbase + i)), c = ln[i];
          tr += u.x * c.x - u.y * c.y;
          ti += u.x * c.y + u.y * c.x;
        }
      }
      for (int m2 = 0; m2 < d; ++m2) {
        const size_t cbase = (size_t)(col0 + m2 * qd) * p;
        float2* ln = sh + (m2 * cbb + bcl) * p;
        for (int m1 = 0; m1 < d; ++m1) {
          const int i = i1 + m1 * pd;
          const float a = ia[cbase + i];
          const float2 v = ldg2(fv + 2 * (cbase + i)), c = ln[i];
          ln[i] = make_float2(a * c.x - (v.x * tr - v.y * ti), a * c.y - (v.x * ti + v.y * tr));
        }
      }
    }
    __syncthreads();
    for (int base = 0; base < cb; base += G) {
      const int l = base + g;
      const bool act = (g < G) && (l < cb);
      fft_line<true>(sh + (act ? l : 0) * p, S.fp, act ? tl : tpl, tpl, twl);
    }
  }
  if (pairs) {
    const int cb2 = cb >> 1;
    for (int e = threadIdx.x; e < cb2 * p; e += blockDim.x) {
      const int i = e / cb2, l = 2 * (e - i * cb2), col = cblk * cb + l;
      const float2 u = sh[l * p + i], w = sh[(l + 1) * p + i];
      if (col + 1 < q)
        stg4(Fm + 2 * ((size_t)i * q + col), make_float4(u.x, u.y, w.x, w.y));
      else if (col < q)
        stg2(Fm + 2 * ((size_t)i * q + col), u);
    }
    return;
  }
  for (int e = threadIdx.x; e < cb * p; e += blockDim.x) {
    const int i = e / cb, l = e - i * cb, col = column(l);
    if (col >= 0) stg2(Fm + 2 * ((size_t)i * q + col), sh[l * p + i]);
  }
}

// Inverse DFT along rows, unpack bands (2m, 2m+1) into X.
__global__ void fft_rows_inv(const SceneDesc* __restrict__ sd, const int2* __restrict__ items,
                             int f_s, int x_s, int add_s) {
  extern __shared__ float2 sh[];
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, L = S.L, lpb = S.fq_lpb, tpl = S.fq_tpl;
  const int nrb = ceil_div(p, lpb);
  const int m = it.y / nrb, row0 = (it.y - m * nrb) * lpb;
  const size_t plane = (size_t)p * q;
  const gfloat* Fm = gslot<const gfloat>(S, f_s) + 2 * (size_t)m * plane;   // complex
  float2* twl = sh + lpb * q;
  stage_twiddles(twl, S.fq);
  const int q2 = q >> 1;                // two complex points per 16-byte load
  for (int e = threadIdx.x; e < lpb * q2; e += blockDim.x) {
    const int l = e / q2, i2 = e - l * q2, r = row0 + l;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < p) v = ldg4(Fm + 2 * ((size_t)r * q + 2 * i2));
    sh[l * q + 2 * i2] = make_float2(v.x, v.y);
    sh[l * q + 2 * i2 + 1] = make_float2(v.z, v.w);
  }
  __syncthreads();
  const int g = threadIdx.x / tpl;
  const int t = (g < lpb) ? threadIdx.x - g * tpl : tpl;
  fft_line<true>(sh + (g < lpb ? g : 0) * q, S.fq, t, tpl, twl);
  gfloat* X = gslot<gfloat>(S, x_s);
  gfloat* Xa = X + (size_t)(2 * m) * plane;
  gfloat* Xb = (2 * m + 1 < L) ? X + (size_t)(2 * m + 1) * plane : nullptr;
  const gfloat* Ad = add_s < 0 ? nullptr : gslot<const gfloat>(S, add_s);
  const gfloat* Aa = Ad ? Ad + (size_t)(2 * m) * plane : nullptr;
  const gfloat* Ab = (Ad && Xb) ? Ad + (size_t)(2 * m + 1) * plane : nullptr;
  const uintptr_t align = reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Ad);
  if ((align & 15) == 0) {              // 16-byte stores of 4 points of a row (q % 4 == 0)
    const int q4 = q >> 2;
    for (int e = threadIdx.x; e < lpb * q4; e += blockDim.x) {
      const int l = e / q4, i4 = e - l * q4, r = row0 + l;
      if (r >= p) continue;
      const float2* s4 = sh + l * q + 4 * i4;
      const float2 v0 = s4[0], v1 = s4[1], v2 = s4[2], v3 = s4[3];
      const size_t o = (size_t)r * q + 4 * i4;
      float4 a = make_float4(v0.x, v1.x, v2.x, v3.x);
      if (Aa) {
        const float4 t = ldg4(Aa + o);
        a.x += t.x; a.y += t.y; a.z += t.z; a.w += t.w;
      }
      stg4(Xa + o, a);
      if (Xb) {
        float4 b = make_float4(v0.y, v1.y, v2.y, v3.y);
        if (Ab) {
          const float4 t = ldg4(Ab + o);
          b.x += t.x; b.y += t.y; b.z += t.z; b.w += t.w;
        }
        stg4(Xb + o, b);
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < lpb * q; e += blockDim.x) {
    const int l = e / q, i = e - l * q, r = row0 + l;
    if (r < p) {
      const float2 v = sh[e];
      const size_t o = (size_t)r * q + i;
      Xa[o] = Aa ? v.x + Aa[o] : v.x;
      if (Xb) Xb[o] = Ab ? v.y + Ab[o] : v.y;
    }
  }
}

constexpr size_t kFftLds = 65536;

int launch_rows(const Batch& B, bool inv, int a, int b, int add, hipStream_t s) {
  for (const Group& g : B.groups[KD_ROWS]) {
    if (!g.nitems) continue;
    if (inv)
      hipLaunchKernelGGL(fft_rows_inv, dim3(g.nitems), dim3(g.block), g.lds, s, B.d_desc,
                         g.d_items, a, b, add);
    else
      hipLaunchKernelGGL(fft_rows_fwd, dim3(g.nitems), dim3(g.block), g.lds, s, B.d_desc,
                         g.d_items, a, b);
    NLPR_LAUNCH_CHECK(inv ? "fft_rows_inv" : "fft_rows_fwd");
  }
  return NLPR_OK;
}

int launch_cols(const Batch& B, int f, hipStream_t s) {
  for (const Group& g : B.groups[KD_COLS]) {
    if (!g.nitems) continue;
    hipLaunchKernelGGL(fft_cols_solve, dim3(g.nitems), dim3(g.block), g.lds, s, B.d_desc,
                       g.d_items, f);
    NLPR_LAUNCH_CHECK("fft_cols_solve");
  }
  return NLPR_OK;
}

}  // namespace

int fft_block(int tpl) {
  int b = 256;
  while (b < tpl) b *= 2;
  return b;
}

// Workgroup size for `lines` lines of tpl threads each: at least fft_block(tpl), and up to
// 1024 so that all lines of the block are transformed in one round.
static int lines_block(int tpl, int lines) {
  int b = fft_block(tpl);
  while (b < lines * tpl && b < 1024) b *= 2;
  return b;
}

int rows_blocks(const Plan& P) {
  return ceil_div(P.prm.p, P.fft.q_lpb) * ((P.Lx + 1) / 2);
}
int cols_blocks(const Plan& P) {
  return ceil_div(P.prm.q, P.fft.p_cb) * ((P.Lx + 1) / 2);
}
// data lines plus one line of twiddles
size_t rows_lds(const Plan& P) { return (size_t)(P.fft.q_lpb + 1) * P.prm.q * sizeof(float2); }
size_t cols_lds(const Plan& P) { return (size_t)(P.fft.p_cb + 1) * P.prm.p * sizeof(float2); }

// d_fused > 0: the columns per block must be a multiple of d (a base column and its aliases)
FftShape default_fft_shape(int p, int q, int d_fused) {
  FftShape f{};
  f.q_tpl = ceil_div(q, 8);
  f.p_tpl = ceil_div(p, 8);
  f.q_lpb = fft_block(f.q_tpl) / f.q_tpl;
  while (f.q_lpb > 1 && (size_t)(f.q_lpb + 1) * q * sizeof(float2) > kFftLds) --f.q_lpb;
  const int unit = d_fused > 0 ? d_fused : 1;
  f.p_cb = unit;
  while (f.p_cb * 2 <= std::max(16, unit) &&
         (size_t)(f.p_cb * 2 + 1) * p * sizeof(float2) <= kFftLds)
    f.p_cb *= 2;
  f.q_bs = fft_block(f.q_tpl);
  f.p_bs = fft_block(f.p_tpl);
  return f;
}

int launch_xsolve(const Batch& B, int c, int x, int f, int add, hipStream_t s) {
  int rc;
  if ((rc = launch_rows(B, false, c, f, -1, s))) return rc;
  if ((rc = launch_cols(B, f, s))) return rc;
  return launch_rows(B, true, f, x, add, s);
}

// Autotuner: time the row and column passes of one band pair for every admissible lines-
// per-block / columns-per-block choice and keep the fastest; results are cached per
// (device, p, q) for the life of the process.
int autotune_fft(Plan& P) {
  static std::mutex mtx;
  static std::map<std::tuple<int, int, int, int>, FftShape> cache;
  const int p = P.prm.p, q = P.prm.q;
  const int dfu = P.d_fia ? P.prm.d : 0;
  int dev = 0;
  NLPR_HIP_TRY(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, p, q, dfu);
  {
    std::lock_guard<std::mutex> lk(mtx);
    auto hit = cache.find(key);
    if (hit != cache.end()) {
      P.fft = hit->second;
      return NLPR_OK;
    }
  }
  FftShape best = default_fft_shape(p, q, dfu);
  const size_t plane = (size_t)p * q;
  // time on up to 16 band pairs so the launch fills the GPU like the real one
  const int tp = std::max(1, std::min((P.Lx + 1) / 2, 16));
  float* d_real = nullptr;
  float2* d_cplx = nullptr;
  SceneDesc* d_sd = nullptr;
  int2* d_items = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int maxitems = std::max(p, q) * tp;
  int rc = NLPR_OK;
  auto cleanup = [&]() {
    hipFree(d_real);
    hipFree(d_cplx);
    hipFree(d_sd);
    hipFree(d_items);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  if (hipMalloc(&d_real, 2 * tp * plane * sizeof(float)) != hipSuccess ||
      hipMalloc(&d_cplx, tp * plane * sizeof(float2)) != hipSuccess ||
      hipMalloc(&d_sd, sizeof(SceneDesc)) != hipSuccess ||
      hipMalloc(&d_items, maxitems * sizeof(int2)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    set_error("autotune: allocation failed");
    return NLPR_ERR_HIP;
  }
  hipMemset(d_real, 0, 2 * tp * plane * sizeof(float));
  std::vector<int2> items(maxitems);
  for (int i = 0; i < maxitems; ++i) items[i] = make_int2(0, i);
  hipMemcpy(d_items, items.data(), maxitems * sizeof(int2), hipMemcpyHostToDevice);
  SceneDesc h{};
  h.p = p;
  h.q = q;
  h.L = 2 * tp;
  h.fp = P.fp;
  h.fq = P.fq;
  h.invden = P.d_invden;
  h.d = P.prm.d;
  h.fused = dfu > 0 ? 1 : 0;
  h.fia = P.d_fia;
  h.fu = P.d_fu;
  h.fv = P.d_fv;
  h.buf[B_C] = d_real;
  h.buf[B_Z] = d_real;
  h.buf[B_F] = d_cplx;
  // best of three runs of 5 launches each (single runs flip between near-equal candidates)
  auto time_it = [&](auto launch) -> float {
    launch();
    float best_ms = 1e30f;
    for (int trial = 0; trial < 3; ++trial) {
      hipEventRecord(e0, nullptr);
      for (int r = 0; r < 5; ++r) launch();
      hipEventRecord(e1, nullptr);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      best_ms = std::min(best_ms, ms);
    }
    return best_ms;
  };
  // rows: lines per block from 1 up to what LDS holds, on a workgroup of lines_block threads
  {
    const int tpl = best.q_tpl;
    float tbest = 1e30f;
    for (int lpb = 1; lpb * tpl <= 1024; lpb *= 2) {
      if ((size_t)(lpb + 1) * q * sizeof(float2) > kFftLds) break;
      const int bs = lines_block(tpl, lpb);
      h.fq_tpl = tpl;
      h.fq_lpb = lpb;
      hipMemcpy(d_sd, &h, sizeof(SceneDesc), hipMemcpyHostToDevice);
      const int nb = ceil_div(p, lpb) * tp;
      const size_t lds = (size_t)(lpb + 1) * q * sizeof(float2);
      const float ms = time_it([&]() {
        hipLaunchKernelGGL(fft_rows_fwd, dim3(nb), dim3(bs), lds, nullptr, d_sd, d_items, (int)B_C,
                           (int)B_F);
        hipLaunchKernelGGL(fft_rows_inv, dim3(nb), dim3(bs), lds, nullptr, d_sd, d_items, (int)B_F,
                           (int)B_Z, -1);
      });
      if (hipGetLastError() != hipSuccess) { rc = NLPR_ERR_HIP; break; }
      if (ms < tbest) { tbest = ms; best.q_lpb = lpb; best.q_bs = bs; }
    }
  }
  // columns: the same over columns per block
  if (rc == NLPR_OK) {
    const int tpl = best.p_tpl;
    float tbest = 1e30f;
    for (int cb = std::max(dfu, 1); cb <= std::max(32, dfu); cb *= 2) {
      if ((size_t)(cb + 1) * p * sizeof(float2) > kFftLds) break;
      const int bs = lines_block(tpl, cb);
      h.fp_tpl = tpl;
      h.fp_cb = cb;
      hipMemcpy(d_sd, &h, sizeof(SceneDesc), hipMemcpyHostToDevice);
      const int nb = ceil_div(q, cb) * tp;
      const size_t lds = (size_t)(cb + 1) * p * sizeof(float2);
      const float ms = time_it([&]() {
        hipLaunchKernelGGL(fft_cols_solve, dim3(nb), dim3(bs), lds, nullptr, d_sd, d_items,
                           (int)B_F);
      });
      if (hipGetLastError() != hipSuccess) { rc = NLPR_ERR_HIP; break; }
      if (ms < tbest) { tbest = ms; best.p_cb = cb; best.p_bs = bs; }
    }
  }
  cleanup();
  if (rc != NLPR_OK) {
    set_error("autotune: a timing launch failed");
    return rc;
  }
  P.fft = best;
  std::lock_guard<std::mutex> lk(mtx);
  cache[key] = best;
  return NLPR_OK;
}

}  // namespace nlpr
