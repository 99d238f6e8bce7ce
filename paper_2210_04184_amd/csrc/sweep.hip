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
// CODES (differentiated form): also record, per dual element, which branch of the
// threshold it took, which is all the sweep's adjoint needs of this iteration: 2 bits, 0 for
// |V| < mu, 1 for V >= mu, 2 for V <= -mu, 3 for V = 0 with mu = 0 (or V not a number).  The
// four elements of a float4 item share one byte, at the item's float offset / 4.
template <int K, int ITEMS, int NT, bool FIRST, bool CODES>
__global__ void __launch_bounds__(NT)
sweep_kernel(const SceneDesc* __restrict__ sd, const int2* __restrict__ items, int x_s, int mu_s,
             int sig_s, int creg_s, int halo_s, uint8_t* codes) {
  const int2 it_ = items[blockIdx.x];
  const SceneDesc& S = sd[it_.x];
  const int p = S.p, q = S.q, L = S.L, npairs = S.npairs, R = S.rows, ntiles = S.ntiles,
            H = S.halo, split = S.psplit;
  const gfloat* __restrict__ X = gslot<const gfloat>(S, x_s);
  const gfloat* __restrict__ mu = gslot<const gfloat>(S, mu_s);
  gfloat* sig = gslot<gfloat>(S, sig_s);   // updated in place
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

  int row[ITEMS], col[ITEMS];
  bool ok[ITEMS];
  float4 xv[ITEMS], cp[ITEMS];
#pragma unroll
  for (int m = 0; m < ITEMS; ++m) {
    const int it = threadIdx.x + NT * m;
    row[m] = it / q4;
    col[m] = (it - row[m] * q4) * 4;
    ok[m] = row[m] < rows;
    xv[m] = ok[m] ? *reinterpret_cast<const float4*>(Xs + (row[m] + H) * q + col[m])
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    cp[m] = make_float4(0.f, 0.f, 0.f, 0.f);
  }

  // Sigma' as [L][tiles][Npairs][|P|][R][q]: the whole state of one workgroup is one
  // contiguous stream, each (tau, k) slab of it R*q floats.
  const size_t kstride = (size_t)R * q;             // between patch offsets
  const size_t tstride = (size_t)NP * kstride;      // between shifts
  const size_t tile_off = ((size_t)c * ntiles + tile) * (size_t)npairs * tstride;

  for (int n = n_begin; n < n_end; ++n) {
    const int2 t = tau_at(S, n);
    __syncthreads();  // the previous shift's reads of Ms and updates of Cs are done
    {
      const gfloat* mun = mu + (size_t)n * plane;
      for (int e = threadIdx.x; e < (R + 2 * K) * q4; e += NT) {
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
      float4 s[KW][ITEMS];
      if (!FIRST) {
#pragma unroll
        for (int k2 = 0; k2 < KW; ++k2) {
          const gfloat* base = sig + n_off + (size_t)((k1 + K) * KW + k2) * kstride;
#pragma unroll
          for (int m = 0; m < ITEMS; ++m)
            s[k2][m] = ok[m] ? ld_nt(base + (size_t)row[m] * q + col[m])
                             : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
#pragma unroll
      for (int k2 = 0; k2 < KW; ++k2) {
        const size_t pl_off = n_off + (size_t)((k1 + K) * KW + k2) * kstride;
        gfloat* base = sig + pl_off;
#pragma unroll
        for (int m = 0; m < ITEMS; ++m) {
          if (!ok[m]) continue;
          const float4 sv = FIRST ? make_float4(0.f, 0.f, 0.f, 0.f) : s[k2][m];
          const int o = 4 + (k2 - K);  // window index of column col + (k2 - K)
          float4 v, cl;
          v.x = g[m].x - sv.x; cl.x = clampf(v.x, mw[m][o + 0]);
          v.y = g[m].y - sv.y; cl.y = clampf(v.y, mw[m][o + 1]);
          v.z = g[m].z - sv.z; cl.z = clampf(v.z, mw[m][o + 2]);
          v.w = g[m].w - sv.w; cl.w = clampf(v.w, mw[m][o + 3]);
          A[m].x += v.x - 2.f * cl.x;
          A[m].y += v.y - 2.f * cl.y;
          A[m].z += v.z - 2.f * cl.z;
          A[m].w += v.w - 2.f * cl.w;
          st_nt(base + (size_t)row[m] * q + col[m], make_float4(-cl.x, -cl.y, -cl.z, -cl.w));
          if (CODES) {
            const float va[4] = {v.x, v.y, v.z, v.w};
            unsigned byte = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const unsigned code = fabsf(va[e]) < mw[m][o + e] ? 0u
                                    : (va[e] > 0.f ? 1u : (va[e] < 0.f ? 2u : 3u));
              byte |= code << (2 * e);
            }
            ((gu8*)codes)[(pl_off + (size_t)row[m] * q + col[m]) >> 2] =
                (uint8_t)byte;
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

#ifndef NLPR_SWEEP_THREADS
#define NLPR_SWEEP_THREADS 256
#endif
#ifndef NLPR_SWEEP_MIN_ITEMS
#define NLPR_SWEEP_MIN_ITEMS 1
#endif
// Workgroup size and the smallest number of float4 items per thread.  One item per thread
// (tiles of 2 rows at q = 512, 90 VGPRs, three workgroups per CU) streamed Sigma' fastest
// among 1, 2 and 4 items and 256 / 512 / 1024 threads; wider images take 2 or 4 items so
// that one workgroup covers at least one full row.
constexpr int kThreads = NLPR_SWEEP_THREADS;
constexpr int kMinItems = NLPR_SWEEP_MIN_ITEMS;

template <int K, int ITEMS, bool FIRST, bool CODES>
int launch_k(const Batch& B, const Group& g, int x, int mu, int sig, int creg, int halo,
             uint8_t* codes, hipStream_t s) {
  auto kern = sweep_kernel<K, ITEMS, kThreads, FIRST, CODES>;
  hipLaunchKernelGGL(kern, dim3(g.nitems), dim3(kThreads), g.lds, s, B.d_desc, g.d_items, x, mu,
                     sig, creg, halo, codes);
  NLPR_LAUNCH_CHECK("sweep_kernel");
  return NLPR_OK;
}

// Allow the sweep's dynamic LDS beyond the default limit (done when a batch is built, not
// during graph capture).  The branch-recording variant exists for one item per thread only.
template <int K, int ITEMS>
int set_lds_limit() {
  const void* kern[4] = {
      reinterpret_cast<const void*>(sweep_kernel<K, ITEMS, kThreads, true, false>),
      reinterpret_cast<const void*>(sweep_kernel<K, ITEMS, kThreads, false, false>),
      ITEMS == 1 ? reinterpret_cast<const void*>(sweep_kernel<K, 1, kThreads, true, true>) : nullptr,
      ITEMS == 1 ? reinterpret_cast<const void*>(sweep_kernel<K, 1, kThreads, false, true>) : nullptr};
  for (const void* k : kern)
    if (k) NLPR_HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)kMaxSweepLds));
  return NLPR_OK;
}

template <int K>
int set_lds_limit_items(int items) {
  switch (items) {
    case 1: return set_lds_limit<K, (kMinItems > 1 ? kMinItems : 1)>();
    case 2: return set_lds_limit<K, (kMinItems > 2 ? kMinItems : 2)>();
    default: return set_lds_limit<K, 4>();
  }
}

template <int K, bool FIRST>
int launch_items(const Batch& B, const Group& g, int x, int mu, int sig, int creg, int halo,
                 uint8_t* codes, hipStream_t s) {
  if (codes) {
    if (g.key1 != 1 || kMinItems != 1) {
      set_error("sweep: branch codes need one item per thread");
      return NLPR_ERR_UNSUPPORTED_SHAPE;
    }
    return launch_k<K, 1, FIRST, true>(B, g, x, mu, sig, creg, halo, codes, s);
  }
  switch (g.key1) {
    case 1:
      return launch_k<K, (kMinItems > 1 ? kMinItems : 1), FIRST, false>(B, g, x, mu, sig, creg,
                                                                         halo, nullptr, s);
    case 2:
      return launch_k<K, (kMinItems > 2 ? kMinItems : 2), FIRST, false>(B, g, x, mu, sig, creg,
                                                                         halo, nullptr, s);
    default: return launch_k<K, 4, FIRST, false>(B, g, x, mu, sig, creg, halo, nullptr, s);
  }
}

}  // namespace

SweepShape choose_sweep_shape(int p, int q, int K, int halo) {
  SweepShape sh{};
  sh.threads = kThreads;
  int items = kMinItems;
  while (items < 4 && kThreads * items * 4 < q) items *= 2;
  sh.items = items;
  const int per_block = kThreads * items * 4;  // pixels per workgroup
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
                 hipStream_t s, uint8_t* codes) {
  for (const Group& g : B.groups[KD_SWEEP]) {
    if (!g.nitems) continue;
    int rc;
    switch (g.key0) {
#define NLPR_SW(KK)                                                                            \
  case KK:                                                                                     \
    rc = first ? launch_items<KK, true>(B, g, x, mu, sig, creg, halo, codes, s)               \
               : launch_items<KK, false>(B, g, x, mu, sig, creg, halo, codes, s);             \
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

}  // namespace nlpr
