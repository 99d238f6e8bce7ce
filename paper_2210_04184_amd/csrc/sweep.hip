// The regulariser sweep: the Q-update (eq. (Qj_main)), the Sigma-update (eq. (dualvar3_main))
// and the regulariser part of the next right-hand side (after eq. (x_linear_system_main)),
// fused into one pass over the dual state.  This is where nearly all HBM traffic of an
// iteration goes: every Sigma value is read once and written once.
//
// Reduced form used here (all identities are exact):
//  * Q-elimination.  With V = D_{tau k} X - Sigma_{tau k}, the soft-threshold gives
//    Q+ = V - clip(V, +-mu) and then Sigma+ = Sigma - (D X - Q+) = -clip(V, +-mu), so Q
//    need not be stored and Q+ + Sigma+ = V - 2 clip(V, +-mu).
//  * Half window.  omega_{i-tau,-tau} = omega_{i tau} and D_{-tau,k} X(i - tau) = -D_{tau k} X(i),
//    so from Sigma = 0 the duals of -tau stay minus those of tau (shifted by tau) and the
//    adjoint terms of tau and -tau are equal; tau = 0 contributes nothing.  Only the half
//    window W+ is visited and its adjoint terms count twice.
//  * Source alignment.  D_{tau k} X(i) = g_tau(i - k) with g_tau = X - X(. - tau) (the shift
//    property of the difference filters).  Storing Sigma'_{tau k}(j) = Sigma_{tau k}(j + k)
//    makes every update at j read g_tau(j) and the threshold mu(j + k, tau), and turns
//    sum_k D_{tau k}^T U_{tau k} into A_tau(j) - A_tau(j + tau) with A_tau = sum_k U'_{tau k}.
// So, per band and pixel j:   Creg(j) = 2 sum_{tau in W+} [A_tau(j) - A_tau(j + tau)].
//
// Work decomposition.  A workgroup owns a tile of `rows` full image rows of one band and
// loops over tau in W+.  Per tau it stages the thresholds mu(., tau) of the tile plus a K
// halo in LDS, forms g_tau from the X tile in LDS, then streams the (2K+1)^2 planes of
// Sigma' for its tile with 16-byte loads and stores, issuing all loads of one patch row
// before any compute.  A_tau is added to the thread's own pixels in registers and
// subtracted at j - tau in an LDS accumulator that spans the tile plus `halo` rows above
// it; since j -> j - tau is one-to-one, the LDS updates of one tau never collide.  The rows
// above the tile go to a small halo buffer that the right-hand-side assembly folds in, so
// the result is deterministic (no atomics).
//
// Split.  A scene with fewer (tile, band) pairs than the GPU has CUs would leave most of it
// idle, so each pair is then served by `psplit` workgroups, part j taking the contiguous
// shifts [j Npairs / psplit, (j+1) Npairs / psplit) of W+.  Part 0 writes the regulariser
// plane and its halo rows as above, part j > 0 its own plane (slot B_CSPLIT) and halo rows;
// the assembly adds the parts in a fixed order, so results stay bit-for-bit repeatable.
#include "nlpr_internal.h"

namespace nlpr {
namespace {


// Sigma' is touched once per iteration: stream it with non-temporal loads and stores so it
// does not evict X and mu from the caches.
#ifndef NLPR_SWEEP_NT
#define NLPR_SWEEP_NT 1
#endif
// cache policy of a buffer access: non-temporal
constexpr int kCacheNT = 2;
// last word of a raw byte-addressed buffer resource: 32-bit data format (bits 15-18 = 4),
// no stride, no swizzle; offsets are bytes from the base
constexpr int kRawBufferFlags = 0x00020000;
__device__ __forceinline__ float4 ld_nt(const gfloat* p) {
#if NLPR_SWEEP_NT
  const v4f_t v = __builtin_nontemporal_load((const gv4f*)p);
#else
  const v4f_t v = *(const gv4f*)p;
#endif
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_nt(gfloat* p, float4 v) {
  v4f_t w = {v.x, v.y, v.z, v.w};
#if NLPR_SWEEP_NT
  __builtin_nontemporal_store(w, (gv4f*)p);
#else
  *(gv4f*)p = w;
#endif
}
__device__ __forceinline__ float clampf(float v, float m) { return fminf(fmaxf(v, -m), m); }

// ---- sweep kernel begin (the traffic record of the benchmark is keyed to this text)
// Storage of Sigma' (coded).  Every new dual value is -clip(V, +-mu), so an element that
// reached the threshold (|V| >= mu) holds exactly -mu (V > 0) or +mu (V < 0): its value
// follows from the threshold, which the sweep has at hand, and one sign bit.  Per float4
// item of a plane the state keeps a code byte, for element e:
//   bit e     the sign bit of V (set: the value is +mu when on the threshold, else -mu);
//   bit 4 + e off the threshold: the sign bit of |V| - mu, i.e. |V| < mu (a NaN V gives a
//             NaN with the sign of |V|, so it counts as on; the NaN reaches C through A).
// The bits are shifted in one at a time with alignbit.  An item with any element off the
// threshold (byte >= 16) is "open": its four values are stored as a float4, as
// clip(V, +-mu) = -Sigma' (so the next sweep adds them: V = g - Sigma').  Open items are
// packed per wave: the 64 items a wave owns in a plane (one 1 KB
// segment of the plane) keep the float4s of their open items at the start of that segment,
// in lane order, so a wave reads and writes only as many 16-byte slots as it has open
// items (mbcnt of the ballot gives each open lane its slot).  A wave reads its whole old
// run before it writes the new one, and each segment belongs to one wave, so the update is
// in place.  Decoding is exact: the stored values are the values, and -mu, +mu are the
// thresholds that produced the on-threshold ones.
// CODES (differentiated form): also record, per dual element, which branch of the
// threshold it took, which is all the sweep's adjoint needs of this iteration: 2 bits, 0 for
// |V| < mu, 1 for V >= mu, 2 for V <= -mu, 3 for V = 0 with mu = 0 (or V not a number).  The
// four elements of a float4 item share one byte, at the item's float offset / 4.
// COUNT: add the number of open items written by each wave to one of the kCountSlots
// counters at count (kCountStride apart); their sum is the launch's count.
template <int K, int ITEMS, int NT, bool FIRST, bool CODES>
__global__ void __launch_bounds__(NT)
sweep_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int x_s, int mu_s,
             int sig_s, int code_s, int creg_s, int halo_s, uint8_t* codes,
             unsigned long long* count) {
  const int2 it_ = items[blockIdx.x];
  const SceneDesc& S = sd[it_.x];
  const int p = S.p, q = S.q, L = S.L, npairs = S.npairs, R = S.rows, ntiles = S.ntiles,
            H = S.halo, split = S.psplit;
  const gfloat* __restrict__ X = gslot<const gfloat>(S, x_s);
  const gfloat* __restrict__ mu = gslot<const gfloat>(S, mu_s);
  gfloat* sig = gslot<gfloat>(S, sig_s);   // updated in place
  gu8* scode = gslot<gu8>(S, code_s);      // updated in place
  constexpr int KW = 2 * K + 1;
  constexpr int NP = KW * KW;
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  const int q4 = q >> 2;
  float* Ms = lds;                      // (R + 2K) x q        mu(., tau), rows r0-K .. r0+R+K-1
  float* Xs = Ms + (R + 2 * K) * q;     // (R + H) x q         X rows r0-H .. r0+R-1
  float* Cs = Xs + (R + H) * q;         // (R + H) x q         adjoint accumulator

  // work item y = (tile * split + part) * L + band: bands fastest, so that the workgroups
  // resident together share the tile's thresholds in L2
  const int tp = it_.y / L;
  const int c = it_.y - tp * L;
  const int tile = tp / split;
  const int part = tp - tile * split;
  const int n_begin = part * npairs / split, n_end = (part + 1) * npairs / split;
  const int r0 = tile * R;
  const int rows = min(R, p - r0);
  const size_t plane = (size_t)p * q;
  gfloat* creg = part == 0 ? gslot<gfloat>(S, creg_s)
                           : gslot<gfloat>(S, B_CSPLIT) + (size_t)(part - 1) * L * plane;
  gfloat* halo = gslot<gfloat>(S, halo_s) + (size_t)part * L * ntiles * H * q;
  const gfloat* Xc = X + (size_t)c * plane;

  for (int e = threadIdx.x; e < (R + H) * q4; e += NT) {
    const int rr = e / q4, c4 = e - rr * q4;
    int gr = (r0 - H + rr) % p;
    if (gr < 0) gr += p;
    reinterpret_cast<float4*>(Xs)[e] = ldg4(Xc + (size_t)gr * q + 4 * c4);
    reinterpret_cast<float4*>(Cs)[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();

  int row[ITEMS], col[ITEMS], seg[ITEMS];
  bool ok[ITEMS];
  float4 xv[ITEMS], cp[ITEMS];
#pragma unroll
  for (int m = 0; m < ITEMS; ++m) {
    const int it = threadIdx.x + NT * m;
    row[m] = it / q4;
    col[m] = (it - row[m] * q4) * 4;
    seg[m] = 4 * (it & ~63);            // float offset of the wave's segment in a plane
    ok[m] = row[m] < rows;
    xv[m] = ok[m] ? *reinterpret_cast<const float4*>(Xs + (row[m] + H) * q + col[m])
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    cp[m] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  unsigned open_written = 0;            // open items this wave wrote (wave-uniform)

  // Sigma' as [L][tiles][Npairs][|P|][R][q]: the whole state of one workgroup is one
  // contiguous stream, each (tau, k) slab of it R*q floats.
  const size_t kstride = (size_t)R * q;             // between patch offsets
  const size_t tstride = (size_t)NP * kstride;      // between shifts
  const size_t tile_off = ((size_t)c * ntiles + tile) * (size_t)npairs * tstride;
  // without the pipeline below (several items per thread): code bytes of the next patch
  // row to process, requested one row ahead
  unsigned cbn[KW][ITEMS];
  auto load_codes = [&](size_t row_off) {
#pragma unroll
    for (int k2 = 0; k2 < KW; ++k2) {
      const gu8* cbp = scode + ((row_off + (size_t)k2 * kstride) >> 2);
#pragma unroll
      for (int m = 0; m < ITEMS; ++m)
        cbn[k2][m] = __builtin_nontemporal_load(cbp + (threadIdx.x + NT * m));
    }
  };
  // the open items' float4s of a patch row, from the waves' packed runs: a wave with open
  // items loads on every lane (lanes past the tile from the start of the segment): the closed
  // lanes' slots lie inside the open run, so no extra line is read and no lane branches
  auto load_open = [&](size_t row_off, const unsigned (&cbx)[KW][ITEMS],
                       float4 (&sx)[KW][ITEMS]) {
#pragma unroll
    for (int k2 = 0; k2 < KW; ++k2) {
      const gfloat* vb = sig + row_off + (size_t)k2 * kstride;
#pragma unroll
      for (int m = 0; m < ITEMS; ++m) {
        const bool open = ok[m] && cbx[k2][m] >= 16u;
        const unsigned long long bal = __builtin_amdgcn_ballot_w64(open);
        const unsigned slot = __builtin_amdgcn_mbcnt_hi(
            (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
        if (bal) sx[k2][m] = ld_nt(vb + (seg[m] + 4u * (ok[m] ? slot : 0u)));
      }
    }
  };

  // the shifts of this workgroup, one per lane, 64 at a time, packed as (tau1 << 16 | tau2):
  // read before the planes' requests, since a load inside the shift loop would wait for
  // every request issued before it
  int tau_lane = 0;
  auto tau_fetch = [&](int n0) {
    const int j = n0 + (int)(threadIdx.x & 63);
    const int2 tj = j < n_end ? tau_at(S, j) : make_int2(0, 0);
    tau_lane = (tj.x << 16) | (tj.y & 0xffff);
  };
  tau_fetch(n_begin);

  // With one item per thread the planes are software-pipelined.  The planes of a workgroup
  // form one contiguous sequence over its shifts (plane x at base + x kstride); while plane x
  // is updated, the open float4s of plane x + D and the code bytes of plane x + D + E are in
  // flight.  These requests are issued on every path (a wave with no open item reads the
  // start of its segment; past the last plane the last plane is read again, unused), so the
  // number of memory operations after each is fixed and the wait for plane x leaves the later
  // ones in flight.  A plane is read only before it is written: its own requests come D and
  // D + E planes earlier, repeats of the last plane up to its own update.
  constexpr bool PIPE = !FIRST && ITEMS == 1;
  constexpr int D = K <= 1 ? 6 : 5, E = D;
  const int nplanes = (n_end - n_begin) * NP;
  const size_t base = tile_off + (size_t)n_begin * tstride;
  uint8_t cq[D + E + 1];   // code bytes of planes x .. x + D + E (kept as bytes: a widening
                           // at the loop's back edge would wait for the loads in flight)
  float4 sb[D + 1];        // open float4s of planes x .. x + D
  // the workgroup's code bytes as one buffer, plane x at byte x * cstride: a lane's byte is
  // addressed by the plane offset (a scalar) and the thread index, with no vector arithmetic
  // (accesses past the range would be dropped)
  const unsigned cstride = (unsigned)(kstride >> 2);
  const __amdgpu_buffer_rsrc_t crs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(uint8_t*)(scode + (base >> 2)), (short)0, PIPE ? nplanes * (int)cstride : 0,
      kRawBufferFlags);
  auto pipe_codes = [&](int x) -> uint8_t {
    return __builtin_amdgcn_raw_buffer_load_b8(crs, threadIdx.x, min(x, nplanes - 1) * cstride,
                                               kCacheNT);
  };
  // the ballot of a plain comparison is one instruction: the lanes past the tile are cleared
  // with a mask taken once; each lane without an open item reads the slot after the open
  // lanes below it, inside the segment
  const unsigned long long okmask = __builtin_amdgcn_ballot_w64(ok[0]);
  const unsigned segb = 4u * (unsigned)seg[0];  // byte offset of the wave's segment
  auto pipe_open = [&](int x, unsigned cx) -> float4 {
    const gfloat* pb = sig + base + (size_t)min(x, nplanes - 1) * kstride;
    const unsigned long long bal = __builtin_amdgcn_ballot_w64(cx >= 16u) & okmask;
    const unsigned slot = __builtin_amdgcn_mbcnt_hi(
        (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
    return ld_nt((const gfloat*)((const gu8*)pb + (segb + 16u * slot)));
  };
  if constexpr (PIPE) {
    if (nplanes > 0) {
#pragma unroll
      for (int i = 0; i < D + E; ++i) cq[i] = pipe_codes(i);
#pragma unroll
      for (int i = 0; i < D; ++i) sb[i] = pipe_open(i, cq[i]);
    }
  } else if (!FIRST && n_begin < n_end) {
    load_codes(tile_off + (size_t)n_begin * tstride);
  }

  // thresholds mu(., tau) of the tile rows and their K halo, (R + 2K) q4 float4s per shift.
  // When they fit MUR per thread their offsets in a mu plane are computed once (no integer
  // division per shift), and for patches of at most 3 x 3 they are requested one shift ahead
  // into registers, so their latency hides behind the previous shift (at 5 x 5 the extra
  // registers would cost a wave per SIMD).
  constexpr int MUR = K <= 1 ? 2 : 3;
  constexpr bool MU_AHEAD = K <= 1;
  const int mu_n4 = (R + 2 * K) * q4;
  const bool mu_hoist = mu_n4 <= MUR * NT;
  int mu_off[MUR];
  float4 mv[MU_AHEAD ? MUR : 1];
#pragma unroll
  for (int u = 0; u < MUR; ++u) {
    const int e = threadIdx.x + u * NT;
    const int rr = e / q4, c4 = e - rr * q4;
    int gr = (r0 - K + rr) % p;
    if (gr < 0) gr += p;
    mu_off[u] = e < mu_n4 ? gr * q + 4 * c4 : -1;
  }
  auto mu_fetch = [&](int n) {
    const gfloat* mun = mu + (size_t)n * plane;
#pragma unroll
    for (int u = 0; u < MUR; ++u)
      if (mu_off[u] >= 0) mv[MU_AHEAD ? u : 0] = ldg4(mun + mu_off[u]);
  };
  if (MU_AHEAD && mu_hoist && n_begin < n_end) mu_fetch(n_begin);

  for (int n = n_begin; n < n_end; ++n) {
    if (n > n_begin && ((n - n_begin) & 63) == 0) tau_fetch(n);
    const int tpk = __builtin_amdgcn_readlane(tau_lane, (n - n_begin) & 63);
    const int2 t = make_int2(tpk >> 16, (int)(short)(tpk & 0xffff));
    __syncthreads();  // the previous shift's reads of Ms and updates of Cs are done
    if (MU_AHEAD && mu_hoist) {
#pragma unroll
      for (int u = 0; u < MUR; ++u)
        if (mu_off[u] >= 0) reinterpret_cast<float4*>(Ms)[threadIdx.x + u * NT] = mv[u];
      if (n + 1 < n_end) mu_fetch(n + 1);
    } else if (mu_hoist) {
      // all of a thread's requests first (lanes without a float4 read the plane's first),
      // then the stores: one wait per shift
      const gfloat* mun = mu + (size_t)n * plane;
      float4 mt[MUR];
#pragma unroll
      for (int u = 0; u < MUR; ++u) mt[u] = ldg4(mun + max(mu_off[u], 0));
#pragma unroll
      for (int u = 0; u < MUR; ++u)
        if (mu_off[u] >= 0) reinterpret_cast<float4*>(Ms)[threadIdx.x + u * NT] = mt[u];
    } else {
      const gfloat* mun = mu + (size_t)n * plane;
      for (int e = threadIdx.x; e < mu_n4; e += NT) {
        const int rr = e / q4, c4 = e - rr * q4;
        int gr = (r0 - K + rr) % p;
        if (gr < 0) gr += p;
        reinterpret_cast<float4*>(Ms)[e] = ldg4(mun + (size_t)gr * q + 4 * c4);
      }
    }
    __syncthreads();

    float4 g[ITEMS], A[ITEMS];
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
      const float* xr = Xs + (row[m] + H - t.x) * q;
      float sh[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int cc = col[m] + e - t.y;
        cc = cc < 0 ? cc + q : (cc >= q ? cc - q : cc);
        sh[e] = xr[cc];
      }
      g[m] = make_float4(xv[m].x - sh[0], xv[m].y - sh[1], xv[m].z - sh[2], xv[m].w - sh[3]);
      A[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    const size_t n_off = tile_off + (size_t)n * tstride;
#pragma unroll
    for (int k1 = -K; k1 <= K; ++k1) {
      // thresholds mu(j + k, tau) for k2 in [-K, K]: columns col-4 .. col+7 of row + k1, the
      // float4 before and after wrapped around the full-width row (no padding columns, so
      // four workgroups fit a CU's LDS at q = 512)
      float mw[ITEMS][12];
#pragma unroll
      for (int m = 0; m < ITEMS; ++m) {
        const float4* mr = reinterpret_cast<const float4*>(Ms + (row[m] + K + k1) * q);
        const int c4 = col[m] >> 2;
        const float4 a = mr[c4 == 0 ? q4 - 1 : c4 - 1], b = mr[c4],
                     d = mr[c4 + 1 == q4 ? 0 : c4 + 1];
        mw[m][0] = a.x; mw[m][1] = a.y; mw[m][2] = a.z; mw[m][3] = a.w;
        mw[m][4] = b.x; mw[m][5] = b.y; mw[m][6] = b.z; mw[m][7] = b.w;
        mw[m][8] = d.x; mw[m][9] = d.y; mw[m][10] = d.z; mw[m][11] = d.w;
      }
      const size_t row_off = n_off + (size_t)((k1 + K) * KW) * kstride;
      // without the pipeline (several items per thread), the old state of this patch row's
      // planes: the code bytes (loaded with the previous row), then the open items' float4s
      // from the waves' packed runs; the next row's code bytes (or the next shift's first
      // row) are requested before this row's values
      unsigned cb[KW][ITEMS];
      float4 s[KW][ITEMS];
      if (!FIRST && !PIPE) {
#pragma unroll
        for (int k2 = 0; k2 < KW; ++k2)
#pragma unroll
          for (int m = 0; m < ITEMS; ++m) cb[k2][m] = cbn[k2][m];
        if (k1 < K || n + 1 < n_end) load_codes(row_off + (size_t)KW * kstride);
        load_open(row_off, cb, s);
      }
#pragma unroll
      for (int k2 = 0; k2 < KW; ++k2) {
        const size_t pl_off = row_off + (size_t)k2 * kstride;
        gfloat* vb = sig + pl_off;
        gu8* cbp = scode + (pl_off >> 2);
#pragma unroll
        for (int m = 0; m < ITEMS; ++m) {
          const int o = 4 + (k2 - K);  // window index of column col + (k2 - K)
          const float mu4[4] = {mw[m][o + 0], mw[m][o + 1], mw[m][o + 2], mw[m][o + 3]};
          float sv[4];
          unsigned cbv = 0;  // this plane's old code byte and open float4
          float4 s4 = make_float4(0.f, 0.f, 0.f, 0.f);
          const int x = (n - n_begin) * NP + (k1 + K) * KW + k2;  // plane of the workgroup
          if constexpr (PIPE) {
            cq[D + E] = pipe_codes(x + D + E);
            sb[D] = pipe_open(x + D, cq[D]);
            cbv = cq[0];
            s4 = sb[0];
#pragma unroll
            for (int i = 0; i < D + E; ++i) cq[i] = cq[i + 1];
#pragma unroll
            for (int i = 0; i < D; ++i) sb[i] = sb[i + 1];
          } else if (!FIRST) {
            cbv = cb[k2][m];
            s4 = s[k2][m];
          }
          if (FIRST) {
            sv[0] = sv[1] = sv[2] = sv[3] = 0.f;
          } else {
            // sv = -Sigma' = clip(V_old, +-mu): the stored value, or on the threshold mu with
            // the sign of V_old (bit e), i.e. mu's magnitude under that sign bit
            const bool open = ok[m] && cbv >= 16u;
            const float st[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float on = __uint_as_float((cbv >> e) << 31 | __float_as_uint(mu4[e]));
              sv[e] = open ? st[e] : on;
            }
          }
          const float gv[4] = {g[m].x, g[m].y, g[m].z, g[m].w};
          float nv[4], acc[4];
          unsigned code = 0, branch = 0;
          float vv[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float v = gv[e] + sv[e];
            const float cl = __builtin_amdgcn_fmed3f(v, -mu4[e], mu4[e]);
            vv[e] = v;
            acc[e] = __builtin_fmaf(-2.f, cl, v);
            nv[e] = cl;
            if (CODES) {
              const unsigned bc = fabsf(v) < mu4[e] ? 0u : (v > 0.f ? 1u : (v < 0.f ? 2u : 3u));
              branch |= bc << (2 * e);
            }
          }
          // the code byte, shifted in one bit at a time (alignbit(c, x, 31) = c << 1 | x >> 31):
          // the off flags (sign bits of |V| - mu) of elements 3..0, then the signs of V
#pragma unroll
          for (int e = 3; e >= 0; --e)
            code = __builtin_amdgcn_alignbit(code, __float_as_uint(fabsf(vv[e]) - mu4[e]), 31);
#pragma unroll
          for (int e = 3; e >= 0; --e)
            code = __builtin_amdgcn_alignbit(code, __float_as_uint(vv[e]), 31);
          if (ok[m]) {
            A[m].x += acc[0];
            A[m].y += acc[1];
            A[m].z += acc[2];
            A[m].w += acc[3];
          }
          const bool opn = ok[m] && code >= 16u;
          if (opn) {
            // inside the branch the execution mask is the ballot of the open lanes (every
            // lane of the wave reaches this point)
            const unsigned long long bal = __builtin_amdgcn_read_exec();
            const unsigned slot = __builtin_amdgcn_mbcnt_hi(
                (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            st_nt(vb + (seg[m] + 4u * slot), make_float4(nv[0], nv[1], nv[2], nv[3]));
          }
          if (count)
            open_written += (unsigned)__builtin_popcountll(__builtin_amdgcn_ballot_w64(opn));
          if (ok[m]) {
            if constexpr (PIPE)
              __builtin_amdgcn_raw_buffer_store_b8((uint8_t)code, crs, threadIdx.x, x * cstride,
                                                   kCacheNT);
            else
              __builtin_nontemporal_store((uint8_t)code, cbp + (threadIdx.x + NT * m));
            if (CODES) ((gu8*)codes)[(pl_off >> 2) + threadIdx.x + NT * m] = (uint8_t)branch;
          }
        }
      }
    }

#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
      if (!ok[m]) continue;
      cp[m].x += A[m].x; cp[m].y += A[m].y; cp[m].z += A[m].z; cp[m].w += A[m].w;
      float* cr = Cs + (row[m] + H - t.x) * q;
      const float a4[4] = {A[m].x, A[m].y, A[m].z, A[m].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int cc = col[m] + e - t.y;
        cc = cc < 0 ? cc + q : (cc >= q ? cc - q : cc);
        cr[cc] -= a4[e];
      }
    }
  }
  if (count && (threadIdx.x & 63) == 0) {
    // spread over kCountSlots counters a cache line apart: waves that end together on one
    // address would queue behind each other at the L2
    const unsigned slot = (blockIdx.x * (NT / 64) + threadIdx.x / 64) % kCountSlots;
    atomicAdd(count + (size_t)slot * kCountStride, (unsigned long long)open_written);
  }
  __syncthreads();

  gfloat* cregc = creg + (size_t)c * plane + (size_t)r0 * q;
#pragma unroll
  for (int m = 0; m < ITEMS; ++m) {
    if (!ok[m]) continue;
    const float4 acc = *reinterpret_cast<const float4*>(Cs + (row[m] + H) * q + col[m]);
    stg4(cregc + (size_t)row[m] * q + col[m],
         make_float4(2.f * (cp[m].x + acc.x), 2.f * (cp[m].y + acc.y), 2.f * (cp[m].z + acc.z),
                     2.f * (cp[m].w + acc.w)));
  }
  if (H > 0) {
    gfloat* hb = halo + ((size_t)c * ntiles + tile) * H * q;
    for (int e = threadIdx.x; e < H * q4; e += NT) {
      const float4 v = reinterpret_cast<const float4*>(Cs)[e];
      stg4(hb + 4 * e, make_float4(2.f * v.x, 2.f * v.y, 2.f * v.z, 2.f * v.w));
    }
  }
}

// ---- sweep kernel end

// Tiles and launch shapes.  A tile is 1024 * items pixels (items = 1, 2 or 4: the fewest with
// one full image row per tile), i.e. 256 * items float4 items, on a workgroup of 256 threads
// with `items` items each; the layout of Sigma' and of its codes depends on the tile only
// (segments of 64 items).  For 3 x 3 patches at 256 x 256 x 31 this shape was faster than
// 128 threads with two items each (89 against 154 VGPRs at the time: five waves per SIMD
// instead of three; 20-iteration solve 2.88 against 3.16 ms).

template <int K, int ITEMS, int NT, bool FIRST, bool CODES>
int launch_k(const Batch& B, const Group& g, int x, int mu, int sig, int creg, int halo,
             uint8_t* codes, unsigned long long* count, hipStream_t s) {
  auto kern = sweep_kernel<K, ITEMS, NT, FIRST, CODES>;
  hipLaunchKernelGGL(kern, dim3(g.nitems), dim3(NT), g.lds, s, B.d_desc, g.d_items, x, mu,
                     sig, (int)B_SCODE, creg, halo, codes, count);
  NLPR_LAUNCH_CHECK("sweep_kernel");
  return NLPR_OK;
}

// Allow the sweep's dynamic LDS beyond the default limit (done when a batch is built, not
// during graph capture).  The branch-recording variant exists for single-item tiles.
template <int K, int ITEMS, int NT>
int set_lds_limit() {
  const bool single = ITEMS == 1;
  const void* kern[4] = {
      reinterpret_cast<const void*>(sweep_kernel<K, ITEMS, NT, true, false>),
      reinterpret_cast<const void*>(sweep_kernel<K, ITEMS, NT, false, false>),
      single ? reinterpret_cast<const void*>(sweep_kernel<K, ITEMS, NT, true, true>) : nullptr,
      single ? reinterpret_cast<const void*>(sweep_kernel<K, ITEMS, NT, false, true>) : nullptr};
  for (const void* k : kern)
    if (k) NLPR_HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)kMaxSweepLds));
  return NLPR_OK;
}

template <int K>
int set_lds_limit_items(int items) {
  switch (items) {
    case 1: return set_lds_limit<K, 1, kSweepThreads>();
    case 2: return set_lds_limit<K, 2, kSweepThreads>();
    default: return set_lds_limit<K, 4, kSweepThreads>();
  }
}

// g.key1 = tile items
template <int K, bool FIRST>
int launch_items(const Batch& B, const Group& g, int x, int mu, int sig, int creg, int halo,
                 uint8_t* codes, unsigned long long* count, hipStream_t s) {
  if (codes && g.key1 != 1) {
    set_error("sweep: branch codes need single-item tiles");
    return NLPR_ERR_UNSUPPORTED_SHAPE;
  }
  if (codes) return launch_k<K, 1, kSweepThreads, FIRST, true>(B, g, x, mu, sig, creg, halo, codes, count, s);
  switch (g.key1) {
    case 1:
      return launch_k<K, 1, kSweepThreads, FIRST, false>(B, g, x, mu, sig, creg, halo, nullptr, count, s);
    case 2:
      return launch_k<K, 2, kSweepThreads, FIRST, false>(B, g, x, mu, sig, creg, halo, nullptr, count, s);
    default:
      return launch_k<K, 4, kSweepThreads, FIRST, false>(B, g, x, mu, sig, creg, halo, nullptr, count, s);
  }
}

}  // namespace

SweepShape choose_sweep_shape(int p, int q, int K, int halo) {
  SweepShape sh{};
  int items = 1;
  while (items < 4 && kSweepThreads * items * 4 < q) items *= 2;
  sh.items = items;
  const int per_block = kSweepThreads * items * 4;  // pixels per workgroup
  sh.rows = std::max(1, std::min(p, per_block / q));
  sh.ntiles = ceil_div(p, sh.rows);
  sh.halo = halo;
  sh.lds = (size_t)((sh.rows + 2 * K) * q + 2 * (sh.rows + halo) * q) * sizeof(float);
  return sh;
}

size_t sweep_sigma_bytes(const SweepShape& sh, int q, int L, int npairs, int npatch) {
  return (size_t)L * sh.ntiles * npairs * npatch * sh.rows * q * sizeof(float);
}

// Workgroups per (tile, band): 1 unless the scene has fewer (tile, band) pairs than the GPU
// has CUs, then enough parts of W+ (at most one shift each) for about one workgroup per CU.
int choose_pair_split(int blocks, int npairs) {
  constexpr int kCus = 256;
  if (blocks <= 0 || blocks >= kCus || npairs <= 1) return 1;
  return std::min(npairs, (kCus + blocks - 1) / blocks);
}

int sweep_blocks(const Plan& P) { return P.sweep.ntiles * P.Lx * P.sweep.split; }

int sweep_prepare(int K, int items) {
  switch (K) {
    case 0: return set_lds_limit_items<0>(items);
    case 1: return set_lds_limit_items<1>(items);
    case 2: return set_lds_limit_items<2>(items);
    case 3: return set_lds_limit_items<3>(items);
    case 4: return set_lds_limit_items<4>(items);
    default: set_error("sweep: unsupported patch radius"); return NLPR_ERR_UNSUPPORTED_SHAPE;
  }
}

int launch_sweep(const Batch& B, int x, int mu, int sig, int creg, int halo, bool first,
                 hipStream_t s, uint8_t* codes, unsigned long long* count) {
  for (const Group& g : B.groups[KD_SWEEP]) {
    if (!g.nitems) continue;
    int rc;
    switch (g.key0) {
#define NLPR_SW(KK)                                                                            \
  case KK:                                                                                     \
    rc = first ? launch_items<KK, true>(B, g, x, mu, sig, creg, halo, codes, count, s)        \
               : launch_items<KK, false>(B, g, x, mu, sig, creg, halo, codes, count, s);      \
    break;
      NLPR_SW(0)
      NLPR_SW(1)
      NLPR_SW(2)
      NLPR_SW(3)
      NLPR_SW(4)
#undef NLPR_SW
      default:
        set_error("sweep: unsupported patch radius");
        return NLPR_ERR_UNSUPPORTED_SHAPE;
    }
    if (rc) return rc;
  }
  return NLPR_OK;
}

// ------------------------------------------------------------------ decoding Sigma'
namespace {
// Dense Sigma' of bands [c0, c0 + nb) from the coded state: out[c - c0][n][k][i1][i2] =
// Sigma'_{tau_n, k}(i1, i2) of band c (image rows, not tiles).  One thread per float4 item of a
// plane, in the sweep's order (ITEMS * NT items per plane, 64 per wave), so every wave sees
// the packed run of the segment the sweep's wave wrote.
__global__ void __launch_bounds__(256)
sigma_expand_kernel(const SceneDesc* __restrict__ sd, const gfloat* __restrict__ sig,
                    const gu8* __restrict__ scode, const gfloat* __restrict__ mu, int c0, int nb,
                    int per_plane, gfloat* __restrict__ out) {
  const SceneDesc& S = sd[0];
  const int p = S.p, q = S.q, K = S.K, npairs = S.npairs, npatch = S.npatch, R = S.rows,
            ntiles = S.ntiles, q4 = q >> 2, KW = 2 * K + 1;
  const size_t g = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t planes = (size_t)nb * ntiles * npairs * npatch;
  const bool live = g < planes * per_plane;        // whole waves are live or not
  const size_t pi = live ? g / per_plane : 0;
  const int it = (int)(g - pi * per_plane);
  // plane index pi = ((cl * ntiles + tile) * npairs + n) * npatch + k
  const int k = (int)(pi % npatch);
  const size_t r1 = pi / npatch;
  const int n = (int)(r1 % npairs);
  const size_t r2 = r1 / npairs;
  const int tile = (int)(r2 % ntiles);
  const int cl = (int)(r2 / ntiles);
  const int r0 = tile * R, rows = min(R, p - r0);
  const int row = it / q4, col = (it - row * q4) * 4;
  const bool ok = live && row < rows;
  const size_t pl_off = (((size_t)(c0 + cl) * ntiles + tile) * npairs + n) * npatch * ((size_t)R * q) +
                        (size_t)k * R * q;
  const unsigned cb = ok ? scode[(pl_off >> 2) + it] : 0u;
  const bool open = ok && cb >= 16u;
  const unsigned long long bal = __builtin_amdgcn_ballot_w64(open);
  const unsigned slot = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
  if (!ok) return;
  float v[4];
  if (open) {
    const float4 t = ldg4(sig + pl_off + 4 * (it & ~63) + 4 * slot);   // clip(V) = -Sigma'
    v[0] = -t.x; v[1] = -t.y; v[2] = -t.z; v[3] = -t.w;
  } else {
    const int k1 = k / KW - K, k2 = k % KW - K;
    const int mr = (r0 + row + k1 + p) % p;
    const gfloat* mun = mu + (size_t)n * p * q + (size_t)mr * q;
    for (int e = 0; e < 4; ++e) {
      const float m = mun[(col + e + k2 + q) % q];
      v[e] = (cb >> e) & 1u ? m : -m;
    }
  }
  const size_t o = ((((size_t)cl * npairs + n) * npatch + k) * p + (r0 + row)) * q + col;
  stg4(out + o, make_float4(v[0], v[1], v[2], v[3]));
}
}  // namespace

int launch_sigma_expand(const Batch& B, const float* sig, const uint8_t* codes, const float* mu,
                        int c0, int nb, float* out, hipStream_t s) {
  const Plan& P = *B.scenes[0];
  const int per_plane = kSweepThreads * P.sweep.items;
  const size_t total = (size_t)nb * P.sweep.ntiles * P.npairs * P.npatch * per_plane;
  if (total == 0) return NLPR_OK;
  const size_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffffu) {
    set_error("sigma expand: too many bands at once");
    return NLPR_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(sigma_expand_kernel, dim3((unsigned)blocks), dim3(256), 0, s, B.d_desc,
                     (const gfloat*)sig, (const gu8*)codes, (const gfloat*)mu, c0, nb, per_plane,
                     (gfloat*)out);
  NLPR_LAUNCH_CHECK("sigma_expand_kernel");
  return NLPR_OK;
}

}  // namespace nlpr
