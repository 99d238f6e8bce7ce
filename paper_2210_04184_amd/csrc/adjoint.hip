// Reverse mode of the unrolled ADMM: kernels that carry adjoints (written v') back through
// one iteration of Sec. "Optimization" (paper's splitting, E = I), and through the guide
// weights and the start.  The iteration, in the form the forward kernels compute it:
//   X   = solve(C)                                        (self-adjoint: C' = solve(X'))
//   BX  = B X
//   P1  = M (rho BX + S^T Y_l - rho L1) / (1 + rho) + (1 - M)(BX - L1)   eq. (Qh_update)
//   P2  = A0 + (Y_h - A0 R) G R^T,  A0 = X - L2,  G = (rho/lambda1 I + R^T R)^{-1}
//   L1+ = L1 - (BX - P1),  L2+ = L2 - (X - P2),  W1 = P1 + L1+,  W2 = P2 + L2+
//   per tau in W+, k in P (reduced sweep):  V = g_tau(j) - Sigma'(j),  c = clip(V, +-mu(j+k)),
//     Sigma'+ = -c,  A_tau(j) += V - 2c,  g_tau = X - X(. - tau)
//   C+  = B^T W1 + W2 + 2 sum_tau [A_tau(j) - A_tau(j + tau)]
// The derivative of clip is 1 inside (|V| < mu) and 0 outside, where clip = +-mu moves with
// mu instead.  All sums run in a fixed order (no atomics): gradients repeat bit for bit.
#include "nlpr_internal.h"

namespace nlpr {
namespace {

constexpr int PADW = 4;   // LDS column padding of the mu' accumulator (K <= 4)

__device__ __forceinline__ int wrapg(int a, int m) {
  a %= m;
  return a < 0 ? a + m : a;
}
__device__ __forceinline__ float4 ld4_nt(const gfloat* p) {
  const v4f_t v = __builtin_nontemporal_load((const gv4f*)p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4_nt(gfloat* p, float4 v) {
  v4f_t w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, (gv4f*)p);
}

// Sum of v[k] over the NW waves of the workgroup, in a fixed order; thread 0 gets it.
template <int N, int NW>
__device__ __forceinline__ void block_sum_waves(double (&v)[N]) {
  __shared__ double red[N][NW];
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
    for (int k = 0; k < N; ++k) {
      double a = 0.0;
      for (int i = 0; i < NW; ++i) a += red[k][i];
      v[k] = a;
    }
  __syncthreads();
}

template <int N>
__device__ __forceinline__ void block_sum256(double (&v)[N]) {
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
  __syncthreads();
}

// ------------------------------------------------------------------------ sweep adjoint
// Per workgroup (tile, band) as the forward sweep, one float4 item per thread.  Inputs: the
// threshold branch of every dual element in the forward sweep (codes, 2 bits each, one byte
// per float4 of Sigma', written by the forward's branch-recording variant), C' (adjoint of
// the right-hand side the sweep fed) and Sigma'' (adjoint of the sweep's Sigma' output,
// updated in place to the adjoint of its input).  The branch is all the adjoint needs of
// the forward values: inside the threshold Sigma+ = -V, outside it Sigma+ = -mu sign(V).
// Outputs: X' of the sweep (xr, plus the rows above the tile in the halo buffer, folded like
// the forward's), and mu' accumulated into per-(band, tile) partial tiles covering the rows
// r0 - K .. r0 + R + K - 1 (mup), reduced over bands and tiles by mubar_reduce_kernel.
//   A'(j) = 2 (C'(j) - C'(j - tau));  per k: c' = -Sigma''(j) - 2 A'(j);
//   V' = A'(j) + [|V| < mu] c';  mu'(j + k) += [V >= mu] c' - [V <= -mu] c';
//   Sigma''(j) := -V';  g'(j) = sum_k V';  X'(j) += g'(j),  X'(j - tau) -= g'(j).
// Coded Sigma'': outside the threshold the new Sigma''(j) = -(A'(j) + 0) depends on the shift
// and the pixel only, so a float4 item is stored only if one of its elements is inside
// (branch 0), packed per wave segment as the forward's open items (ballot and mbcnt give the
// slots).  The next backward step, which has the branch codes of this step (pcodes) and this
// step's C' (cbp_s), rebuilds the others with the same operations, so the values are exact.
// FIRST: the first backward step, whose incoming Sigma'' is zero.
// The planes of a workgroup are software-pipelined as in the forward sweep: the codes of this
// step and Sigma'' of plane x + D, and the codes of the previous step of plane x + D + E
// (which place the packed float4s), are in flight while plane x is updated.  The requests
// are issued on every path (lanes past the tile read the plane's first item, a wave with no
// stored item the start of its segment, and past the last plane the last plane again,
// unused), so each wait leaves the later requests in flight.  A plane is read before it is
// written.
template <int K, bool FIRST>
__global__ void __launch_bounds__(256)
sweep_bwd_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int cb_s,
                 const uint8_t* codes, int sb_s, int xr_s, int halo_s, int mup_s,
                 const uint8_t* pcodes, int cbp_s) {
  constexpr int NT = 256;
  constexpr int KW = 2 * K + 1;
  constexpr int NP = KW * KW;
  const int2 it_ = items[blockIdx.x];
  const SceneDesc& S = sd[it_.x];
  const int p = S.p, q = S.q, L = S.L, npairs = S.npairs, R = S.rows, ntiles = S.ntiles,
            H = S.halo;
  const gfloat* Cb = gslot<const gfloat>(S, cb_s);
  const gu8* cod = (const gu8*)codes;
  const gu8* pcod = (const gu8*)pcodes;
  gfloat* sb = gslot<gfloat>(S, sb_s);
  gfloat* mup = gslot<gfloat>(S, mup_s);
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  const int q4 = q >> 2;
  const int ms = q + 2 * PADW;
  const int ER = R + 2 * K;               // extended rows of the mu' tile
  float* Mb = lds;                        // ER x ms   mu' accumulator
  float* Cs = Mb + ER * ms;               // (R + H) x q   C'
  float* As = Cs + (R + H) * q;           // (R + H) x q   X' accumulator
  float* Cps = As + (R + H) * q;          // (R + H) x q   C' of the previous step (not FIRST)
  const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);

  // the forward sweep's work items, y = (tile * psplit + part) * L + band; the adjoint covers
  // all shifts of a tile in one workgroup, so the items of parts 1 .. psplit-1 have no work
  const int tp = it_.y / L;
  const int c = it_.y - tp * L;
  const int tile = tp / S.psplit;
  if (tp - tile * S.psplit != 0) return;
  const int r0 = tile * R;
  const int rows = min(R, p - r0);
  const size_t plane = (size_t)p * q;
  const gfloat* Cc = Cb + (size_t)c * plane;
  const gfloat* Cpc = FIRST ? Cc : gslot<const gfloat>(S, cbp_s) + (size_t)c * plane;
  for (int e = threadIdx.x; e < (R + H) * q4; e += NT) {
    const int rr = e / q4, c4 = e - rr * q4;
    const int gr = wrapg(r0 - H + rr, p);
    reinterpret_cast<float4*>(Cs)[e] = ldg4(Cc + (size_t)gr * q + 4 * c4);
    reinterpret_cast<float4*>(As)[e] = zero4;
    if (!FIRST) reinterpret_cast<float4*>(Cps)[e] = ldg4(Cpc + (size_t)gr * q + 4 * c4);
  }
  __syncthreads();

  const int row = threadIdx.x / q4;
  const int col = (threadIdx.x - row * q4) * 4;
  const bool ok = row < rows;
  const float4 cv = ok ? *reinterpret_cast<const float4*>(Cs + (row + H) * q + col) : zero4;
  const float4 cvp =
      ok && !FIRST ? *reinterpret_cast<const float4*>(Cps + (row + H) * q + col) : zero4;
  float4 cp = zero4;

  const size_t kstride = (size_t)R * q;
  const size_t tstride = (size_t)NP * kstride;
  const size_t tile_off = ((size_t)c * ntiles + tile) * (size_t)npairs * tstride;
  gfloat* mup_tile = mup + ((size_t)c * ntiles + tile) * (size_t)npairs * ER * q;

  // the shifts, one per lane, 64 at a time, packed as (tau1 << 16 | tau2): a load inside the
  // shift loop would wait for every request issued before it
  int tau_lane = 0;
  auto tau_fetch = [&](int n0) {
    const int j = n0 + (int)(threadIdx.x & 63);
    const int2 tj = j < npairs ? tau_at(S, j) : make_int2(0, 0);
    tau_lane = (tj.x << 16) | (tj.y & 0xffff);
  };
  tau_fetch(0);

  // an item with a zero 2-bit field (an element inside the threshold) is stored
  auto stored = [](unsigned b) { return ((b | (b >> 1)) & 0x55u) != 0x55u; };
  constexpr int D = 2, E = FIRST ? 0 : 2;
  const int nplanes = npairs * NP;
  const unsigned itm = ok ? threadIdx.x : 0u;               // the lane's item in a plane
  const unsigned segf = 4u * (threadIdx.x & ~63u);          // float offset of its wave segment
  const unsigned long long okmask = __builtin_amdgcn_ballot_w64(ok);
  auto pbase = [&](int x) { return tile_off + (size_t)min(x, nplanes - 1) * kstride; };
  unsigned cq[D + 1];          // this step's branch codes of planes x .. x + D
  unsigned pq[D + E + 1];      // the previous step's codes of planes x .. x + D + E
  float4 sq[D + 1];            // packed Sigma'' of planes x .. x + D
  auto req_codes = [&](int x, unsigned& cw) { cw = (cod + (pbase(x) >> 2))[itm]; };
  auto req_pcodes = [&](int x, unsigned& pw) { pw = (pcod + (pbase(x) >> 2))[itm]; };
  auto req_sigma = [&](int x, unsigned pw, float4& sv) {
    const unsigned long long bal = __builtin_amdgcn_ballot_w64(stored(pw)) & okmask;
    const unsigned slot = __builtin_amdgcn_mbcnt_hi(
        (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
    sv = ld4_nt((sb + pbase(x)) + (segf + 4u * slot));
  };
  if (nplanes > 0) {
#pragma unroll
    for (int i = 0; i < D; ++i) req_codes(i, cq[i]);
    if (!FIRST) {
#pragma unroll
      for (int i = 0; i < D + E; ++i) req_pcodes(i, pq[i]);
#pragma unroll
      for (int i = 0; i < D; ++i) req_sigma(i, pq[i], sq[i]);
    }
  }

  for (int n = 0; n < npairs; ++n) {
    if (n > 0 && (n & 63) == 0) tau_fetch(n);
    const int tpk = __builtin_amdgcn_readlane(tau_lane, n & 63);
    const int2 t = make_int2(tpk >> 16, (int)(short)(tpk & 0xffff));
    __syncthreads();
    for (int e = threadIdx.x; e < ER * (ms >> 2); e += NT) reinterpret_cast<float4*>(Mb)[e] = zero4;
    __syncthreads();
    // A' at the item's four pixels, and the previous step's Sigma'' of the items it did not
    // store, -(A'_prev + 0)
    float ab[4], dv[4], gb[4] = {0.f, 0.f, 0.f, 0.f};
    {
      const float* cr = Cs + (row + H - t.x) * q;
      const float* crp = Cps + (row + H - t.x) * q;
      const float ca[4] = {cv.x, cv.y, cv.z, cv.w};
      const float cap[4] = {cvp.x, cvp.y, cvp.z, cvp.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int cc = col + e - t.y;
        cc = cc < 0 ? cc + q : (cc >= q ? cc - q : cc);
        ab[e] = ok ? 2.f * (ca[e] - cr[cc]) : 0.f;
        const float abp = ok && !FIRST ? 2.f * (cap[e] - crp[cc]) : 0.f;
        dv[e] = -(abp + 0.f);
      }
    }
#pragma unroll
    for (int k1 = -K; k1 <= K; ++k1) {
#pragma unroll
      for (int k2 = 0; k2 < KW; ++k2) {
        const int x = n * NP + (k1 + K) * KW + k2;   // plane of the workgroup
        req_codes(x + D, cq[D]);
        if (!FIRST) {
          req_pcodes(x + D + E, pq[D + E]);
          req_sigma(x + D, pq[D], sq[D]);
        }
        const unsigned cw = ok ? cq[0] : 0u;
        float b4[4] = {0.f, 0.f, 0.f, 0.f};
        if (!FIRST) {
          const bool ps = ok && stored(pq[0]);
          const float st[4] = {sq[0].x, sq[0].y, sq[0].z, sq[0].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) b4[e] = ps ? st[e] : dv[e];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
          cq[i] = cq[i + 1];
          sq[i] = sq[i + 1];
        }
#pragma unroll
        for (int i = 0; i < D + E; ++i) pq[i] = pq[i + 1];
        const int o = 4 + (k2 - K);
        float vb[4], mb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const unsigned code = (cw >> (2 * e)) & 3u;
          const float cbar = -b4[e] - 2.f * ab[e];
          vb[e] = ab[e] + (code == 0u ? cbar : 0.f);
          mb[e] = code == 1u ? cbar : (code == 2u ? -cbar : 0.f);
          gb[e] += vb[e];
        }
        if (ok) {
          if (stored(cw)) {
            // inside the branch the execution mask is the ballot of the storing lanes
            const unsigned long long bal = __builtin_amdgcn_read_exec();
            const unsigned slot = __builtin_amdgcn_mbcnt_hi(
                (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            st4_nt((sb + tile_off + (size_t)x * kstride) + (segf + 4u * slot),
                   make_float4(-vb[0], -vb[1], -vb[2], -vb[3]));
          }
          float* mrow = Mb + (row + K + k1) * ms + col + o;   // mu' at (row + k1, col + k2 - K + e)
#pragma unroll
          for (int e = 0; e < 4; ++e) mrow[e] += mb[e];
        }
        __syncthreads();   // j -> j + k is one-to-one for a fixed k; k's overlap
      }
    }
    if (ok) {
      cp.x += gb[0]; cp.y += gb[1]; cp.z += gb[2]; cp.w += gb[3];
      float* ar = As + (row + H - t.x) * q;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int cc = col + e - t.y;
        cc = cc < 0 ? cc + q : (cc >= q ? cc - q : cc);
        ar[cc] -= gb[e];
      }
    }
    __syncthreads();
    // fold the padded columns into their wrapped positions and accumulate the partial tile,
    // as float4s, a thread's first MP4 read before one wait: a row of Mb holds PADW = 4
    // columns on either side, one float4 folded into the row's first and last float4
    gfloat* mpn = mup_tile + (size_t)n * ER * q;
    const int mp_n4 = ER * q4;
    auto folded = [&](int e4) {
      const int rr = e4 / q4, c4 = e4 - rr * q4;
      const float4* mrow = reinterpret_cast<const float4*>(Mb + rr * ms);
      float4 v = mrow[1 + c4];
      if (c4 == 0) {                               // columns q .. q + 3
        const float4 w = mrow[1 + q4];
        v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
      }
      if (c4 == q4 - 1) {                          // columns -4 .. -1
        const float4 w = mrow[0];
        v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
      }
      return v;
    };
    constexpr int MP4 = 2;
    float4 mpv[MP4];
#pragma unroll
    for (int u = 0; u < MP4; ++u)
      mpv[u] = ldg4(mpn + 4 * min((int)threadIdx.x + u * NT, mp_n4 - 1));
#pragma unroll
    for (int u = 0; u < MP4; ++u) {
      const int e4 = threadIdx.x + u * NT;
      if (e4 < mp_n4) {
        const float4 v = folded(e4);
        stg4(mpn + 4 * e4, make_float4(mpv[u].x + v.x, mpv[u].y + v.y, mpv[u].z + v.z,
                                       mpv[u].w + v.w));
      }
    }
    for (int e4 = threadIdx.x + MP4 * NT; e4 < mp_n4; e4 += NT) {
      const float4 v = folded(e4), m = ldg4(mpn + 4 * e4);
      stg4(mpn + 4 * e4, make_float4(m.x + v.x, m.y + v.y, m.z + v.z, m.w + v.w));
    }
  }
  __syncthreads();
  gfloat* xro = gslot<gfloat>(S, xr_s) + (size_t)c * plane + (size_t)r0 * q;
  if (ok) {
    const float4 acc = *reinterpret_cast<const float4*>(As + (row + H) * q + col);
    stg4(xro + (size_t)row * q + col,
         make_float4(cp.x + acc.x, cp.y + acc.y, cp.z + acc.z, cp.w + acc.w));
  }
  if (H > 0) {
    gfloat* hb = gslot<gfloat>(S, halo_s) + ((size_t)c * ntiles + tile) * H * q;
    for (int e = threadIdx.x; e < H * q4; e += NT)
      stg4(hb + 4 * e, reinterpret_cast<const float4*>(As)[e]);
  }
}

// mu'(tau, i) = sum over bands and over the tiles whose extended rows cover image row i of
// the partial tiles.  One thread per (tau, pixel).
__global__ void __launch_bounds__(256)
mubar_reduce_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int mup_s,
                    int mub_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, R = S.rows, ntiles = S.ntiles, ER = S.rows + 2 * S.K;
  const size_t plane = (size_t)p * q;
  const size_t e = (size_t)it.y * 256 + threadIdx.x;
  if (e >= (size_t)S.npairs * plane) return;
  const int n = (int)(e / plane);
  const int rem = (int)(e - (size_t)n * plane);
  const int i = rem / q, col = rem - (rem / q) * q;
  const gfloat* mup = gslot<const gfloat>(S, mup_s);
  float acc = 0.f;
  for (int tl = 0; tl < ntiles; ++tl) {
    // extended row er of tile tl is image row (tl R - K + er) mod p
    const int er0 = wrapg(i - tl * R + S.K, p);
    if (er0 >= ER) continue;
    for (int c = 0; c < S.L; ++c)
      for (int er = er0; er < ER; er += p)
        acc += mup[((((size_t)c * ntiles + tl) * S.npairs + n) * ER + er) * q + col];
  }
  gslot<gfloat>(S, mub_s)[e] = acc;
}

// ----------------------------------------------------------------------- P-update adjoint
// Work item = 256 pixels; NC threads per pixel (1 for large images; for small ones 4, or 2
// with up to 16 guide bands, which need more registers), each owning a contiguous share of
// the bands.  Inputs: X, BX of the iteration, Y_l,
// Y_h, Lambda1 and Lambda2 before the update; adjoints W1' (= B C'), W2' (= C'), Lambda1'',
// Lambda2'' of the outputs.  Outputs: BX', X' of this step, Lambda'' of the inputs (in
// place), Y_l' and Y_h' accumulated, and per workgroup two FP64 partial sums of rho', added
// to the workgroup's own slot (repeatable across iterations): through P1, and through G,
// where G' = sum res s^T and dG/drho = -G G / lambda1 give -res^T G (G s) / lambda1 per
// pixel.  The band sums res = Y_h - A0 R and s = P2' R are formed per share and added in
// LDS in a fixed order.
// Bands [c0, c1) of one pixel in the P-update adjoint: X', Lambda2'', BX', Lambda1'' and
// Y_l' of the step; returns the pixel's rho' share through P1.  Restrict parameters let the
// compiler read R with scalar loads across the stores.
template <int LHM>
__device__ __forceinline__ double pupdate_bwd_write(
    const gfloat* __restrict__ BX, const gfloat* __restrict__ Yl, const gfloat* __restrict__ L1,
    const gfloat* __restrict__ W1b, const gfloat* __restrict__ W2b, gfloat* __restrict__ L1b,
    gfloat* __restrict__ L2b, gfloat* __restrict__ BXb, gfloat* __restrict__ Xp,
    gfloat* __restrict__ GYl, const gfloat* __restrict__ R, const float (&v)[LHM], size_t plane,
    size_t lplane, size_t lj, bool sampled, int Lh, float inv, float rr, int c0, int c1, int j) {
  double acc = 0.0;
  for (int c = c0; c < c1; ++c) {
    const size_t o = (size_t)c * plane + j;
    float corr = 0.f;
#pragma unroll
    for (int h = 0; h < LHM; ++h)
      if (h < Lh) corr += v[h] * R[c * Lh + h];
    // with P2' = 2 W2' + Lambda2'' and A0' = P2' - P2' R G R^T = P2' - corr:
    // X' = A0' - W2' - Lambda2'' = W2' - corr and Lambda2''(new) = W2' + Lambda2'' - A0'
    // = corr - W2', so Lambda2'' is not read again here
    const float xp = W2b[o] - corr;
    Xp[o] = xp;
    L2b[o] = -xp;
    const float w1b = W1b[o];
    if (sampled) {
      const float l1b = L1b[o];            // read only where the P1 step keeps it
      const float p1b = 2.f * w1b + l1b;
      const float y = Yl[c * lplane + lj];
      BXb[o] = -w1b - l1b + p1b * rr;
      L1b[o] = w1b + l1b - p1b * rr;
      GYl[c * lplane + lj] += p1b * inv;
      acc += (double)p1b * ((double)BX[o] - (double)L1[o] - (double)y) * (double)inv *
             (double)inv;
    } else {
      BXb[o] = w1b;
      L1b[o] = -w1b;
    }
  }
  return acc;
}

// pupdate_bwd_write with the thread's W2' in registers and every read issued first.
template <int LHM, int KB>
__device__ __forceinline__ double pupdate_bwd_write_kept(
    const gfloat* __restrict__ BX, const gfloat* __restrict__ Yl, const gfloat* __restrict__ L1,
    const gfloat* __restrict__ W1b, const float (&w2k)[KB], gfloat* __restrict__ L1b,
    gfloat* __restrict__ L2b, gfloat* __restrict__ BXb, gfloat* __restrict__ Xp,
    gfloat* __restrict__ GYl, const gfloat* __restrict__ R, const float (&v)[LHM], size_t plane,
    size_t lplane, size_t lj, bool sampled, int Lh, float inv, float rr, int c0, int c1, int j) {
  float w1a[KB], l1ba[KB], yla[KB], bxa[KB], l1a[KB], gya[KB];
#pragma unroll
  for (int i = 0; i < KB; ++i)
    if (c0 + i < c1) {
      const int c = c0 + i;
      const size_t o = (size_t)c * plane + j;
      w1a[i] = W1b[o];
      if (sampled) {
        l1ba[i] = L1b[o];
        yla[i] = Yl[c * lplane + lj];
        bxa[i] = BX[o];
        l1a[i] = L1[o];
        gya[i] = GYl[c * lplane + lj];
      }
    }
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < KB; ++i)
    if (c0 + i < c1) {
      const int c = c0 + i;
      const size_t o = (size_t)c * plane + j;
      float corr = 0.f;
#pragma unroll
      for (int h = 0; h < LHM; ++h)
        if (h < Lh) corr += v[h] * R[c * Lh + h];
      const float xp = w2k[i] - corr;
      Xp[o] = xp;
      L2b[o] = -xp;
      const float w1b = w1a[i];
      if (sampled) {
        const float l1b = l1ba[i];
        const float p1b = 2.f * w1b + l1b;
        const float y = yla[i];
        BXb[o] = -w1b - l1b + p1b * rr;
        L1b[o] = w1b + l1b - p1b * rr;
        GYl[c * lplane + lj] = gya[i] + p1b * inv;
        acc += (double)p1b * ((double)bxa[i] - (double)l1a[i] - (double)y) * (double)inv *
               (double)inv;
      } else {
        BXb[o] = w1b;
        L1b[o] = -w1b;
      }
    }
  return acc;
}

// With at most kPbKeep bands per thread (KEEP), every read of a pass is issued before the
// pass's arithmetic, and W2' is read once, kept in registers between the two passes; the
// arithmetic and its order are those of the band loops.
constexpr int kPbKeep = 8;
template <int LHM, int PB_NC, bool KEEP>
__global__ void __launch_bounds__(256 * PB_NC)
pupdate_bwd_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int x_s,
                   int bx_s, int yl_s, int yh_s, int l1_s, int l2_s, int w1b_s, int w2b_s,
                   int l1b_s, int l2b_s, int bxb_s, int xp_s, int gyl_s, int gyh_s, int part_s) {
  __shared__ float part[PB_NC > 1 ? PB_NC : 1][PB_NC > 1 ? LHM : 1][PB_NC > 1 ? 256 : 1];
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, L = S.L, Lh = S.Lh, d = S.d;
  const size_t plane = (size_t)p * q;
  // the band share is uniform over a wave (256 threads per share); readfirstlane lets the
  // band loops index R and G with scalar loads
  const int pix = threadIdx.x & 255;
  const int ch = PB_NC == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);
  const int j = it.y * 256 + pix;
  const bool act = j < (int)plane;
  const int c0 = (L * ch) / PB_NC, c1 = (L * (ch + 1)) / PB_NC;
  const gfloat* X = gslot<const gfloat>(S, x_s);
  const gfloat* L2 = gslot<const gfloat>(S, l2_s);
  const gfloat* W2b = gslot<const gfloat>(S, w2b_s);
  gfloat* L2b = gslot<gfloat>(S, l2b_s);
  const gfloat* R = as_global(S.R);
  const gfloat* G = as_global(S.G);
  float rp[LHM], sp[LHM];
#pragma unroll
  for (int h = 0; h < LHM; ++h) rp[h] = sp[h] = 0.f;
  constexpr int KB = KEEP ? kPbKeep : 1;
  float w2k[KB];                        // W2' of the thread's bands (KEEP)
  if (KEEP && act) {
    float xa[KB], l2a[KB], l2ba[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i)
      if (c0 + i < c1) {
        const size_t o = (size_t)(c0 + i) * plane + j;
        xa[i] = X[o];
        l2a[i] = L2[o];
        w2k[i] = W2b[o];
        l2ba[i] = L2b[o];
      }
#pragma unroll
    for (int i = 0; i < KB; ++i)
      if (c0 + i < c1) {
        const int c = c0 + i;
        const float a0 = xa[i] - l2a[i];
        const float p2b = 2.f * w2k[i] + l2ba[i];
#pragma unroll
        for (int h = 0; h < LHM; ++h)
          if (h < Lh) {
            rp[h] += a0 * R[c * Lh + h];
            sp[h] += p2b * R[c * Lh + h];
          }
      }
  }
  if (!KEEP && act)
    for (int c = c0; c < c1; ++c) {      // this quarter's A0 R and P2' R
      const size_t o = (size_t)c * plane + j;
      const float a0 = X[o] - L2[o];
      const float p2b = 2.f * W2b[o] + L2b[o];
#pragma unroll
      for (int h = 0; h < LHM; ++h)
        if (h < Lh) {
          rp[h] += a0 * R[c * Lh + h];
          sp[h] += p2b * R[c * Lh + h];
        }
    }
  float res[LHM], sv[LHM];
  if constexpr (PB_NC == 1) {             // one thread per pixel: no exchange
#pragma unroll
    for (int h = 0; h < LHM; ++h) {
      res[h] = rp[h];
      sv[h] = sp[h];
    }
  } else {
#pragma unroll
    for (int h = 0; h < LHM; ++h) part[ch][h][pix] = rp[h];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < LHM; ++h) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < PB_NC; ++k) a += part[k][h][pix];
      res[h] = a;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < LHM; ++h) part[ch][h][pix] = sp[h];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < LHM; ++h) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < PB_NC; ++k) a += part[k][h][pix];
      sv[h] = a;
    }
  }
  double acc[2] = {0.0, 0.0};
  if (act) {
    const gfloat* BX = gslot<const gfloat>(S, bx_s);
    const gfloat* Yl = gslot<const gfloat>(S, yl_s);
    const gfloat* Yh = gslot<const gfloat>(S, yh_s);
    const gfloat* L1 = gslot<const gfloat>(S, l1_s);
    const gfloat* W1b = gslot<const gfloat>(S, w1b_s);
    gfloat* L1b = gslot<gfloat>(S, l1b_s);
    gfloat* BXb = gslot<gfloat>(S, bxb_s);
    gfloat* Xp = gslot<gfloat>(S, xp_s);
    gfloat* GYl = gslot<gfloat>(S, gyl_s);
    gfloat* GYh = gslot<gfloat>(S, gyh_s);
    const float inv = S.inv_1prho, rr = S.rho * S.inv_1prho;   // 1/(1+rho), rho/(1+rho)
    const int i1 = j / q, i2 = j - (j / q) * q;
    const bool sampled = (i1 % d == 0) && (i2 % d == 0);
    const size_t lj = (size_t)(i1 / d) * (q / d) + i2 / d;
    const size_t lplane = (size_t)(p / d) * (q / d);
#pragma unroll
    for (int h = 0; h < LHM; ++h) res[h] = (h < Lh) ? Yh[h * plane + j] - res[h] : 0.f;
    float v[LHM];                        // v = s G  (G symmetric)
#pragma unroll
    for (int h2 = 0; h2 < LHM; ++h2) {
      float t = 0.f;
#pragma unroll
      for (int h = 0; h < LHM; ++h)
        if (h < Lh && h2 < Lh) t += sv[h] * G[h * Lh + h2];
      v[h2] = t;
    }
    if (ch == 0) {                       // the pixel's Y_h' and rho' share through G, once
      float rg = 0.f;                    // res^T G v
#pragma unroll
      for (int h2 = 0; h2 < LHM; ++h2) {
        float w = 0.f;
#pragma unroll
        for (int h = 0; h < LHM; ++h)
          if (h < Lh && h2 < Lh) w += v[h] * G[h * Lh + h2];
        rg += res[h2] * w;
      }
      acc[1] = -(double)rg / S.lam1_d;
#pragma unroll
      for (int h = 0; h < LHM; ++h)      // after every read of G (stores would order them)
        if (h < Lh) GYh[h * plane + j] += v[h];
    }
    if constexpr (KEEP)
      acc[0] = pupdate_bwd_write_kept<LHM, KB>(BX, Yl, L1, W1b, w2k, L1b, L2b, BXb, Xp, GYl, R,
                                               v, plane, lplane, lj, sampled, Lh, inv, rr, c0,
                                               c1, j);
    else
      acc[0] = pupdate_bwd_write<LHM>(BX, Yl, L1, W1b, W2b, L1b, L2b, BXb, Xp, GYl, R, v, plane,
                                      lplane, lj, sampled, Lh, inv, rr, c0, c1, j);
  }
  block_sum_waves<2, 4 * PB_NC>(acc);
  if (threadIdx.x == 0) {
    gdouble* prt = gslot<gdouble>(S, part_s) + 2 * (size_t)it.y;
    prt[0] += acc[0];
    prt[1] += acc[1];
  }
}

// ------------------------------------------------------------------ weights adjoint
// mu = (lambda/rho) omega,  omega(i) = exp(-Bx(e)(i) / h^2),  Bx = box sum over P,
// e_tau(j) = sum_c (Y_h(j) - Y_h(j - tau))^2.  Per (shift, 16 x 64 tile): recompute e on the
// tile plus a 2K halo and omega on the tile plus a K halo, form
// Bx(e)'(i) = -mu'(i) (lambda/rho) omega(i) / h^2 there, and box-sum it back (the box is
// symmetric) into e'_tau on the tile.  FP64 partials of lambda' = sum mu' omega / rho and of
// the thresholds' share of rho' = -sum mu' lambda omega / rho^2, over the tile.
constexpr int WB_Y = 16, WB_X = 64;
__global__ void __launch_bounds__(256)
weights_bwd_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int yh_s,
                   int mub_s, int eb_s, int part_s, int w0) {
  extern __shared__ float wsh[];
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, K = S.K, Lh = S.Lh;
  const int gx = ceil_div(q, WB_X), gy = ceil_div(p, WB_Y);
  const int n = it.y / (gx * gy);
  const int rem = it.y - n * gx * gy;
  const int y0 = (rem / gx) * WB_Y, x0 = (rem % gx) * WB_X;
  const int2 t = tau_at(S, n);
  const size_t plane = (size_t)p * q;
  const int E2Y = WB_Y + 4 * K, E2X = WB_X + 4 * K;    // e on the tile + 2K
  const int E1Y = WB_Y + 2 * K, E1X = WB_X + 2 * K;    // omega, Bx(e)' on the tile + K
  float* e2 = wsh;                    // E2Y x E2X
  float* hs = e2 + E2Y * E2X;         // E2Y x E1X   row box sums, then reused
  float* ob = hs + E2Y * E1X;         // E1Y x E1X   Bx(e)'
  const gfloat* Yh = gslot<const gfloat>(S, yh_s);
  const gfloat* mub = gslot<const gfloat>(S, mub_s) + (size_t)n * plane;
  gfloat* eb = gslot<gfloat>(S, eb_s) + (size_t)n * plane;
  const double lam = S.lam_d, rho = S.rho_d;
  double acc[2] = {0.0, 0.0};
  if (S.unweighted) {
    for (int idx = threadIdx.x; idx < WB_Y * WB_X; idx += blockDim.x) {
      const int y = y0 + idx / WB_X, x = x0 + idx % WB_X;
      if (y < p && x < q) {
        const double m = mub[(size_t)y * q + x];
        acc[0] += m / rho;
        acc[1] -= m * lam / (rho * rho);
        eb[(size_t)y * q + x] = 0.f;
      }
    }
  } else {
    for (int idx = threadIdx.x; idx < E2Y * E2X; idx += blockDim.x) {
      const int yy = idx / E2X, xx = idx % E2X;
      const int gyy = wrapg(y0 - 2 * K + yy, p), gxx = wrapg(x0 - 2 * K + xx, q);
      const int sy = wrapg(gyy - t.x, p), sx = wrapg(gxx - t.y, q);
      float a = 0.f;
      for (int c = 0; c < Lh; ++c) {
        const float dl = Yh[c * plane + (size_t)gyy * q + gxx] - Yh[c * plane + (size_t)sy * q + sx];
        a += dl * dl;
      }
      e2[idx] = a;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < E2Y * E1X; idx += blockDim.x) {
      const int yy = idx / E1X, x = idx % E1X;
      float a = 0.f;
      for (int dx = 0; dx <= 2 * K; ++dx) a += e2[yy * E2X + x + dx];
      hs[idx] = a;
    }
    __syncthreads();
    const float ih2 = S.inv_h2;
    for (int idx = threadIdx.x; idx < E1Y * E1X; idx += blockDim.x) {
      const int yy = idx / E1X, xx = idx % E1X;
      float bxe = 0.f;
      for (int dy = 0; dy <= 2 * K; ++dy) bxe += hs[(yy + dy) * E1X + xx];
      const float om = expf(-bxe * ih2);
      const int gyy = wrapg(y0 - K + yy, p), gxx = wrapg(x0 - K + xx, q);
      const float m = mub[(size_t)gyy * q + gxx];
      ob[idx] = -m * S.mu_scale * om * ih2;
      const bool inside = yy >= K && yy < K + WB_Y && xx >= K && xx < K + WB_X &&
                          y0 - K + yy < p && x0 - K + xx < q;
      if (inside) {
        acc[0] += (double)m * (double)om / rho;
        acc[1] -= (double)m * lam * (double)om / (rho * rho);
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < E1Y * WB_X; idx += blockDim.x) {   // rows of the box
      const int yy = idx / WB_X, x = idx % WB_X;
      float a = 0.f;
      for (int dx = 0; dx <= 2 * K; ++dx) a += ob[yy * E1X + x + dx];
      hs[idx] = a;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < WB_Y * WB_X; idx += blockDim.x) {
      const int y = idx / WB_X, x = idx % WB_X;
      float a = 0.f;
      for (int dy = 0; dy <= 2 * K; ++dy) a += hs[(y + dy) * WB_X + x];
      if (y0 + y < p && x0 + x < q) eb[(size_t)(y0 + y) * q + x0 + x] = a;
    }
  }
  block_sum256(acc);
  if (threadIdx.x == 0) {
    gdouble* part = gslot<gdouble>(S, part_s) + w0 + 2 * (size_t)it.y;
    part[0] = acc[0];
    part[1] = acc[1];
  }
}

// Y_h'(c, i) += sum_tau 2 [e'_tau(i) (Y(i) - Y(i - tau)) - e'_tau(i + tau) (Y(i + tau) - Y(i))].
__global__ void __launch_bounds__(256)
yh_bwd_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int yh_s,
              int eb_s, int gyh_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q;
  const size_t plane = (size_t)p * q;
  const int j = it.y * 256 + threadIdx.x;
  if (j >= (int)plane || S.unweighted) return;
  const int i1 = j / q, i2 = j - (j / q) * q;
  const gfloat* Yh = gslot<const gfloat>(S, yh_s);
  const gfloat* eb = gslot<const gfloat>(S, eb_s);
  gfloat* gyh = gslot<gfloat>(S, gyh_s);
  for (int c = 0; c < S.Lh; ++c) {
    const gfloat* Y = Yh + (size_t)c * plane;
    const float y = Y[j];
    float a = 0.f;
    for (int n = 0; n < S.npairs; ++n) {
      const int2 t = tau_at(S, n);
      const size_t jm = (size_t)wrapg(i1 - t.x, p) * q + wrapg(i2 - t.y, q);
      const size_t jp = (size_t)wrapg(i1 + t.x, p) * q + wrapg(i2 + t.y, q);
      a += eb[(size_t)n * plane + j] * (y - Y[jm]) - eb[(size_t)n * plane + jp] * (Y[jp] - y);
    }
    gyh[(size_t)c * plane + j] += 2.f * a;
  }
}

// Y_l'(c, m) += sum of X0' over the d x d block of m (adjoint of the nearest-neighbour start).
__global__ void __launch_bounds__(256)
upsample_bwd_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int x0b_s,
                    int gyl_s) {
  const int2 it = items[blockIdx.x];
  const SceneDesc& S = sd[it.x];
  const int p = S.p, q = S.q, d = S.d, pd = S.p / S.d, qd = S.q / S.d;
  const size_t e = (size_t)it.y * 256 + threadIdx.x;
  if (e >= (size_t)S.L * pd * qd) return;
  const int c = (int)(e / ((size_t)pd * qd));
  const int rem = (int)(e - (size_t)c * pd * qd);
  const int m1 = rem / qd, m2 = rem - (rem / qd) * qd;
  const gfloat* xb = gslot<const gfloat>(S, x0b_s) + (size_t)c * p * q;
  float a = 0.f;
  for (int u = 0; u < d; ++u)
    for (int v = 0; v < d; ++v) a += xb[(size_t)(m1 * d + u) * q + m2 * d + v];
  gslot<gfloat>(S, gyl_s)[e] += a;
}

// lambda' and rho' from the partial sums (one workgroup, fixed order): the pixel blocks'
// [rho' through P1, rho' through G] pairs, then the weight blocks' [lambda', rho' through
// the thresholds] pairs from offset 2 npix.
__global__ void __launch_bounds__(256)
grad_scalars_kernel(const SceneDesc* __restrict__ sd, int part_s, int npix, int nw,
                    double* out) {
  const SceneDesc& S = sd[0];
  const gdouble* part = gslot<const gdouble>(S, part_s);
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < npix; b += 256) v[1] += part[2 * (size_t)b] + part[2 * (size_t)b + 1];
  for (int b = threadIdx.x; b < nw; b += 256) {
    v[0] += part[2 * (size_t)npix + 2 * (size_t)b];
    v[1] += part[2 * (size_t)npix + 2 * (size_t)b + 1];
  }
  block_sum256(v);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[1];
  }
}

template <typename Kern, typename... Args>
int launch_kind(const Batch& B, Kind kind, const char* name, Kern kern, hipStream_t s,
                Args... args) {
  for (const Group& g : B.groups[kind]) {
    if (g.nitems == 0) continue;
    hipLaunchKernelGGL(kern, dim3(g.nitems), dim3(256), g.lds, s, B.d_desc, g.d_items, args...);
    NLPR_LAUNCH_CHECK(name);
  }
  return NLPR_OK;
}

template <int K>
int launch_sbwd(const Batch& B, const Group& g, size_t lds, int cb, const uint8_t* codes, int sb,
                int xr, int halo, int mup, const uint8_t* pcodes, int cbp, hipStream_t s) {
  if (pcodes) {
    hipLaunchKernelGGL((sweep_bwd_kernel<K, false>), dim3(g.nitems), dim3(256), lds, s,
                       B.d_desc, g.d_items, cb, codes, sb, xr, halo, mup, pcodes, cbp);
  } else {
    hipLaunchKernelGGL((sweep_bwd_kernel<K, true>), dim3(g.nitems), dim3(256), lds, s,
                       B.d_desc, g.d_items, cb, codes, sb, xr, halo, mup, codes, cb);
  }
  NLPR_LAUNCH_CHECK("sweep_bwd_kernel");
  return NLPR_OK;
}

template <int K>
int sbwd_attr() {
  NLPR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_bwd_kernel<K, true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxSweepLds));
  NLPR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(sweep_bwd_kernel<K, false>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxSweepLds));
  return NLPR_OK;
}

}  // namespace

size_t sweep_bwd_lds(const Plan& P) {
  const int R = P.sweep.rows, H = P.sweep.halo, K = P.prm.K, q = P.prm.q;
  return (size_t)((R + 2 * K) * (q + 2 * PADW) + 3 * (R + H) * q) * sizeof(float);
}
size_t weights_bwd_lds(const Plan& P) {
  const int K = P.prm.K;
  const size_t e2 = (size_t)(WB_Y + 4 * K) * (WB_X + 4 * K);
  const size_t hs = (size_t)(WB_Y + 4 * K) * (WB_X + 2 * K);
  const size_t ob = (size_t)(WB_Y + 2 * K) * (WB_X + 2 * K);
  return (e2 + hs + ob) * sizeof(float);
}
int weights_bwd_blocks(const Plan& P) {
  return ceil_div(P.prm.q, WB_X) * ceil_div(P.prm.p, WB_Y) * P.npairs;
}
size_t mubar_partial_elems(const Plan& P) {
  return (size_t)P.prm.L * P.sweep.ntiles * P.npairs * (P.sweep.rows + 2 * P.prm.K) * P.prm.q;
}

int sweep_bwd_prepare(int K) {
  switch (K) {
    case 0: return sbwd_attr<0>();
    case 1: return sbwd_attr<1>();
    case 2: return sbwd_attr<2>();
    case 3: return sbwd_attr<3>();
    default: return sbwd_attr<4>();
  }
}

int launch_sweep_bwd(const Batch& B, int cb, const uint8_t* codes, int sb, int xr, int halo,
                     int mup, const uint8_t* pcodes, int cbp, hipStream_t s) {
  const Plan& P = *B.scenes[0];
  const size_t lds = sweep_bwd_lds(P);
  for (const Group& g : B.groups[KD_SWEEP]) {
    if (!g.nitems) continue;
    int rc;
    switch (g.key0) {
      case 0: rc = launch_sbwd<0>(B, g, lds, cb, codes, sb, xr, halo, mup, pcodes, cbp, s); break;
      case 1: rc = launch_sbwd<1>(B, g, lds, cb, codes, sb, xr, halo, mup, pcodes, cbp, s); break;
      case 2: rc = launch_sbwd<2>(B, g, lds, cb, codes, sb, xr, halo, mup, pcodes, cbp, s); break;
      case 3: rc = launch_sbwd<3>(B, g, lds, cb, codes, sb, xr, halo, mup, pcodes, cbp, s); break;
      case 4: rc = launch_sbwd<4>(B, g, lds, cb, codes, sb, xr, halo, mup, pcodes, cbp, s); break;
      default:
        set_error("sweep adjoint: unsupported patch radius");
        return NLPR_ERR_UNSUPPORTED_SHAPE;
    }
    if (rc) return rc;
  }
  return NLPR_OK;
}

int launch_mubar_reduce(const Batch& B, int mup, int mub, hipStream_t s) {
  return launch_kind(B, KD_MUPLANE, "mubar_reduce_kernel", mubar_reduce_kernel, s, mup, mub);
}

template <int LHM, int NC>
void launch_pb(const Batch& B, const Group& g, int x, int bx, int yl, int yh, int l1, int l2,
               int w1b, int w2b, int l1b, int l2b, int bxb, int xp, int gyl, int gyh, int part,
               hipStream_t s) {
  // the reverse mode takes one scene: its bands per thread decide the variant
  if (ceil_div(B.scenes[0]->Lx, NC) <= kPbKeep)
    hipLaunchKernelGGL((pupdate_bwd_kernel<LHM, NC, true>), dim3(g.nitems), dim3(256 * NC), 0,
                       s, B.d_desc, g.d_items, x, bx, yl, yh, l1, l2, w1b, w2b, l1b, l2b, bxb,
                       xp, gyl, gyh, part);
  else
    hipLaunchKernelGGL((pupdate_bwd_kernel<LHM, NC, false>), dim3(g.nitems), dim3(256 * NC), 0,
                       s, B.d_desc, g.d_items, x, bx, yl, yh, l1, l2, w1b, w2b, l1b, l2b, bxb,
                       xp, gyl, gyh, part);
}

int launch_pupdate_bwd(const Batch& B, int x, int bx, int yl, int yh, int l1, int l2, int w1b,
                       int w2b, int l1b, int l2b, int bxb, int xp, int gyl, int gyh, int part,
                       hipStream_t s) {
  for (const Group& g : B.groups[KD_PIXEL]) {
    if (!g.nitems) continue;
    const bool split = g.key1 == 4;
#define NLPR_PB(LHM, NC) \
  launch_pb<LHM, NC>(B, g, x, bx, yl, yh, l1, l2, w1b, w2b, l1b, l2b, bxb, xp, gyl, gyh, part, s)
    if (g.key0 == 1) {
      if (split) NLPR_PB(1, 4); else NLPR_PB(1, 1);
    } else if (g.key0 == 4) {
      if (split) NLPR_PB(4, 4); else NLPR_PB(4, 1);
    } else {
      if (split) NLPR_PB(kMaxLh, 2); else NLPR_PB(kMaxLh, 1);   // registers: 2 at most
    }
#undef NLPR_PB
    NLPR_LAUNCH_CHECK("pupdate_bwd_kernel");
  }
  return NLPR_OK;
}

int launch_weights_bwd(const Batch& B, int yh, int mub, int eb, int part, int w0, hipStream_t s) {
  return launch_kind(B, KD_WBWD, "weights_bwd_kernel", weights_bwd_kernel, s, yh, mub, eb, part,
                     w0);
}

int launch_yh_bwd(const Batch& B, int yh, int eb, int gyh, hipStream_t s) {
  for (const Group& g : B.groups[KD_PIXEL]) {
    if (!g.nitems) continue;
    hipLaunchKernelGGL(yh_bwd_kernel, dim3(g.nitems), dim3(256), 0, s, B.d_desc, g.d_items, yh,
                       eb, gyh);
    NLPR_LAUNCH_CHECK("yh_bwd_kernel");
  }
  return NLPR_OK;
}

int launch_upsample_bwd(const Batch& B, int x0b, int gyl, hipStream_t s) {
  return launch_kind(B, KD_PLANE, "upsample_bwd_kernel", upsample_bwd_kernel, s, x0b, gyl);
}

int launch_grad_scalars(const Batch& B, int part, int npix, int nw, double* out, hipStream_t s) {
  hipLaunchKernelGGL(grad_scalars_kernel, dim3(1), dim3(256), 0, s, B.d_desc, part, npix, nw,
                     out);
  NLPR_LAUNCH_CHECK("grad_scalars_kernel");
  return NLPR_OK;
}

}  // namespace nlpr
