// Internal declarations of libnlpr: scene plans, the batch every launch runs over, device
// scene descriptors and kernel launchers.
//
// Every kernel runs over a batch of scenes.  Block b of a launch reads its work item
// items[b] = (scene, local block), takes the scene's sizes, tables and buffers from the
// device descriptor sd[scene] and does the work of that local block.  A single-scene plan
// is a batch of one, so one code path serves both.  Kernels reach buffers through slots
// (SceneDesc::buf[slot]), so the same kernel serves the solve and the per-stage entry
// points with different buffers.
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
constexpr int kMaxLs = 32;                    // bands of X with a subspace basis

// One-dimensional FFT of length n = product of fac[] (each 2, 3, 4 or 8).
// tw[m] = exp(-2 pi i m / n), m in [0, n).
struct LineFFT {
  int n;
  int nfac;
  int fac[kMaxFFTFactors];
  const float2* tw;
};

// Buffer slots of a scene descriptor.
enum Slot {
  B_YL = 0, B_YH, B_Z, B_SIGMA, B_MU, B_C, B_L1, B_L2, B_BX, B_W1, B_W2, B_F, B_HALO, B_TMP,
  B_OUT,     // Z = X E when a subspace basis is used (B_Z is then the X iterate)
  B_YLE,     // Y_l E^T, [Ls][p/d][q/d]
  B_YLP,     // Y_l E^+, [Ls][p/d][q/d]
  B_L1O, B_L2O,   // where the P-update writes Lambda1, Lambda2 when not in place (checkpoints)
  B_CSPLIT,  // regulariser planes of sweep parts 1 .. psplit-1, [psplit-1][L][p][q]
  B_SCODE,   // Sigma' codes: one byte per float4 item of Sigma' (sweep.hip)
  // reverse mode (single scene): adjoints of the iteration's variables and the outputs
  B_GZ,      // Z' (input)
  B_GC,      // C'
  B_GCP,     // C' of the backward step before (the sweep adjoint rebuilds Sigma'' from it)
  B_GL1, B_GL2,   // Lambda1'', Lambda2''
  B_GSIG,    // Sigma'' (coded: float4 items with an element inside the threshold, packed)
  B_GX,      // X'
  B_GW1,     // W1' = B C'
  B_GBX,     // BX'
  B_GXP,     // X' of the P-update
  B_GXR,     // X' of the sweep (+ halo rows in B_GHALO)
  B_GHALO,
  B_GMUP,    // mu' partial tiles [L][ntiles][Npairs][R + 2K][q]
  B_GMU,     // mu' [Npairs][p][q]
  B_GE,      // e' [Npairs][p][q]
  B_GYL, B_GYH,   // Y_l', Y_h' (outputs)
  B_GPART,   // FP64 partial sums
  B_COUNT
};

// Everything a kernel needs to know about one scene.  Lives in device memory.
struct SceneDesc {
  int p, q, L, Lh, d, r, K, npairs, npatch;
  int rows, ntiles, halo;          // sweep tiling
  int psplit;                      // sweep workgroups per (tile, band), each over a part of W+
  int fq_tpl, fq_lpb;              // row FFT: threads per line, lines per block
  int fp_tpl, fp_cb;               // column FFT: threads per line, columns per block
  int init_zero, unweighted;
  int subspace, Lz;                // basis in use; bands of Z (L is the number of X bands)
  int fused;                       // S inside the X-system (no P1)
  float rho, inv_1prho, mu_scale, inv_h2;
  LineFFT fp, fq;
  const int2* taus;
  const float* invden;
  const float* blur;
  const float* bsep;               // u then v (2r+1 each) of a rank-one blur b = u v^T, else null
  const float* R;
  const float* G;
  const float* E;                  // [Ls][Lz]
  const float* Ep;                 // E^+ = E^T (E E^T)^{-1}, [Lz][Ls]
  const float* M;                  // (E E^T + rho I)^{-1}, [Ls][Ls]
  // fused-S X-update tables, column-major [q][p]: 1/(a p q), b^/a, gamma conj(b^)/(a p q)
  const float* fia;
  const float2* fu;
  const float2* fv;
  // monitor: partial sums [mon_npix][4] (data_l, data_h, r1^2, r2^2 per pixel block), then
  // [mon_nreg] (regulariser per (shift, tile) block), then the trace [points][8]
  double* mon;
  int mon_npix, mon_nreg;
  double rho_d, lam1_d, lam_d;
  void* buf[B_COUNT];
};

constexpr int kSweepThreads = 256;   // workgroup size of the sweep
// Batches of at least this many pixel-bands (summed over scenes) run the P-side of each
// iteration on a second stream, concurrently with the sweep.  Below it the two cross-stream
// waits of an iteration (about 6 and 11 us on MI355X) and the sweep's hold on the CUs cost
// more than the overlap gains (256 x 256 x 31: 2.77 -> 2.90 ms per solve; 512 x 512 x 128:
// 3.03 -> 2.98 s).
constexpr size_t kForkPixelBands = (size_t)1 << 22;
// open-item counters of one sweep launch (timing plans): kCountSlots, kCountStride apart
constexpr int kCountSlots = 64;
constexpr int kCountStride = 16;

struct SweepShape {
  int rows;      // tile height R
  int items;     // tile size in units of 256 float4 items (1024 pixels): 1, 2 or 4
  int ntiles;    // ceil(p / R)
  int halo;      // rows above the tile reached by the adjoint scatter (max tau1)
  int split;     // workgroups per (tile, band), each over a contiguous part of W+
  size_t lds;    // dynamic LDS bytes
};

struct FftShape {
  int q_tpl, q_lpb, q_bs;   // row passes: threads per line, lines per block, block size
  int p_tpl, p_cb, p_bs;    // column pass: threads per line, columns per block, block size
};

// One scene: parameters, device tables and its part of the workspace.
struct Plan {
  nlpr_params prm{};
  int npairs = 0;
  int npatch = 0;
  std::vector<int32_t> taus;      // W+ (tau1, tau2 pairs)
  int2* d_taus = nullptr;
  float* d_invden = nullptr;      // [p][q], 1 / (den * p * q)
  float2* d_tw_p = nullptr;
  float2* d_tw_q = nullptr;
  LineFFT fp{}, fq{};
  FftShape fft{};
  float* d_blur = nullptr;          // (2r+1)^2 taps, then u and v when blur_separable
  bool blur_separable = false;
  float* d_R = nullptr;
  float* d_G = nullptr;
  int Lx = 0;                     // bands of X: Ls with a basis, else L
  float* d_E = nullptr;           // [Ls][L]
  float* d_Ep = nullptr;          // [L][Ls]
  float* d_M = nullptr;           // [Ls][Ls]
  float* d_Rt = nullptr;          // E R, [Ls][Lh]
  double* d_mon = nullptr;        // monitor partials and trace (monitor_every > 0)
  float* d_fia = nullptr;         // fused-S tables (NLPR_FUSED_S)
  float2* d_fu = nullptr;
  float2* d_fv = nullptr;
  int mon_points = 0;             // records per solve
  SweepShape sweep{};
  // workspace layout relative to the scene's base
  size_t off[B_COUNT] = {};
  size_t sz[B_COUNT] = {};
  size_t ws_bytes = 0;
};

// A launch: the work items of the scenes that share its template parameters.
struct Group {
  int2* d_items = nullptr;
  int nitems = 0;
  int block = 256;
  size_t lds = 0;
  int key0 = 0, key1 = 0;   // sweep: K, items per thread
};

enum Kind { KD_WEIGHTS = 0, KD_PLANE, KD_CONV, KD_PIXEL, KD_SWEEP, KD_ROWS, KD_COLS,
            KD_LOWRES,   // one thread per low-resolution pixel of scenes with a basis
            KD_COMPOSE,  // one thread per pixel of scenes with a basis
            KD_MONREG,   // monitor regulariser: (shift, 32 x 64 tile) of scenes with a window
            KD_SCENE,    // one workgroup per scene
            KD_MUPLANE,  // one thread per (shift, pixel): single-scene reverse mode
            KD_WBWD,     // weights adjoint: (shift, 16 x 64 tile), single-scene reverse mode
            KD_COUNT };

struct Batch {
  int device = 0;
  uint32_t flags = 0;              // flags shared by every scene (INIT_ZERO, STATE_IN, ...)
  int iters = 0;
  int monitor_every = 0;           // shared by every scene
  int mon_last = 0;                // monitor records written by the last solve
  hipEvent_t done_ev = nullptr;    // recorded after each solve
  // second stream of the iteration (large batches only): the P-side (blur, P-update and the
  // part of the right-hand side that does not wait for the sweep) runs on it while the sweep
  // runs on the solve's stream
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  std::vector<Plan*> scenes;       // owned
  std::vector<size_t> base;        // workspace base of each scene
  size_t ws_bytes = 0;
  SceneDesc* d_desc = nullptr;     // device descriptors, one per scene
  SceneDesc* h_desc = nullptr;     // pinned staging copy
  std::vector<SceneDesc> uploaded; // what d_desc holds
  bool desc_valid = false;
  hipEvent_t upload_ev = nullptr;
  std::vector<Group> groups[KD_COUNT];
  unsigned long long* d_counts = nullptr;  // open Sigma' items written per sweep (timing)
  int* d_flag = nullptr;           // finite check: first checked iteration with NaN / Inf
  int nonfinite_iter = -1;         // what the last checked solve found (-1: nothing)
  // graph
  bool use_graph = false;
  hipGraphExec_t graph = nullptr;
  uint32_t graph_key = 0;
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

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Pointers read from a descriptor are generic (flat); kernels convert them to the global
// address space so the compiler emits global loads, and scalar loads for uniform addresses.
// Vector elements move through clang ext-vector types (HIP's vector structs cannot be
// copied out of an address-space-qualified object).
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) uint8_t gu8;
typedef __attribute__((address_space(1))) double gdouble;
typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef int v2i_t __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) v2f_t gv2f;
typedef __attribute__((address_space(1))) v4f_t gv4f;
typedef __attribute__((address_space(1))) v2i_t gv2i;
__device__ __forceinline__ const gfloat* as_global(const float* p) { return (const gfloat*)p; }
__device__ __forceinline__ gfloat* as_global(float* p) { return (gfloat*)p; }
template <typename G>
__device__ __forceinline__ G* gslot(const SceneDesc& S, int k) {
  return k < 0 ? nullptr : (G*)(S.buf[k]);
}
__device__ __forceinline__ float2 ldg2(const gfloat* p) {
  const v2f_t v = *(const gv2f*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void stg2(gfloat* p, float2 a) {
  const v2f_t v = {a.x, a.y};
  *(gv2f*)p = v;
}
__device__ __forceinline__ float4 ldg4(const gfloat* p) {
  const v4f_t v = *(const gv4f*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stg4(gfloat* p, float4 a) {
  const v4f_t v = {a.x, a.y, a.z, a.w};
  *(gv4f*)p = v;
}
__device__ __forceinline__ int2 tau_at(const SceneDesc& S, int n) {
  const v2i_t v = ((const gv2i*)S.taus)[n];
  return make_int2(v.x, v.y);
}

// ---- plan precompute (dense.hip); runs once per scene on the null stream
int launch_precompute(Plan& P);

// ---- local work-item counts per scene for each kind of launch
int weights_blocks(const Plan& P);
int plane_blocks(const Plan& P);      // elementwise over [L][p][q], 256 elements per block
int conv_blocks(const Plan& P);
int pixel_blocks(const Plan& P);      // one thread per pixel
int rows_blocks(const Plan& P);
int cols_blocks(const Plan& P);
int sweep_blocks(const Plan& P);
size_t weights_lds(const Plan& P);
size_t conv_lds(const Plan& P);
int conv_class(int r);                // template bound of a blur radius: 1, 2, 4, 8 or 16
size_t rows_lds(const Plan& P);
size_t cols_lds(const Plan& P);

// ---- batched kernels: each launches the groups of one kind with buffer slots (< 0: none)
int launch_weights(const Batch& B, int yh, int mu, hipStream_t s);
int launch_init(const Batch& B, int yl, int ylp, int x0, int l1, int l2, int w2, hipStream_t s);
// reg_mask: bit 0 / 1 mark add1 / add2 as regulariser terms (skipped, like the halo, for
// scenes without a search window); bit 2 marks them as the forward sweep's output, whose
// parts 1 .. psplit-1 (slot B_CSPLIT) and halo parts are then added as well
int launch_conv(const Batch& B, int in, int out, bool transpose, int add1, int add2, int halo,
                int reg_mask, hipStream_t s);
// Lambda1, Lambda2 are read from slots l1, l2 and written to l1o, l2o (the same slots for an
// update in place)
int launch_pupdate(const Batch& B, int x, int bx, int yl, int yh, int l1, int l2, int w1, int w2,
                   int l1o, int l2o, hipStream_t s);
// Re-point buffer slots of the descriptor of scene 0 on the stream: kernels enqueued after it
// see the new buffers.  The reverse-mode passes move through their checkpoints this way.
struct SlotSet {
  int n = 0;
  int slot[6];
  void* ptr[6];
  void add(int sl, void* p) {      // at most 6 (the callers add 2, 4 or 6)
    if (n < 6) { slot[n] = sl; ptr[n] = p; ++n; }
  }
};
int launch_set_slots(const Batch& B, const SlotSet& set, hipStream_t s);
int lh_class(int Lh);                // pupdate template class of a guide-band count: 1, 4 or 16
// threads per pixel of a P-update launch over `pixels` pixels in all: 4 (bands split) below
// 131072, where one thread per pixel would leave most of the GPU idle, else 1
inline int pixel_split(size_t pixels) { return pixels < 131072 ? 4 : 1; }
int lowres_blocks(const Plan& P);
// in-place negation of n4 float4 values with non-temporal 16-byte accesses (reference stream)
int launch_stream_rmw(float* buf, size_t n4, hipStream_t s);
int launch_stream_chunks(float* buf, size_t chunk4, int nchunks, int bands, int planes,
                         size_t lds, hipStream_t s);
// with a subspace basis: Y_l E^T and Y_l E^+ (once per solve), the P1-update on sampled
// pixels, and Z = X E
int launch_project(const Batch& B, int yl, int yle, int ylp, hipStream_t s);
int launch_p1_subspace(const Batch& B, int bx, int yle, int l1, int w1, hipStream_t s);
int launch_compose(const Batch& B, int x, int z, hipStream_t s);
// monitor (monitor.hip): objective terms and primal residuals after iteration `iter`,
// written to record `point` of each scene's trace
int monreg_blocks(const Plan& P);
size_t monreg_lds(const Plan& P);
int monitor_points(int iters, int every);
int launch_monitor(const Batch& B, int point, int iter, hipStream_t s);
// reverse mode (adjoint.hip); single-scene batches
size_t sweep_bwd_lds(const Plan& P);
size_t weights_bwd_lds(const Plan& P);
int weights_bwd_blocks(const Plan& P);
size_t mubar_partial_elems(const Plan& P);
int sweep_bwd_prepare(int K);
// codes: the forward sweep's threshold branches of the iteration (launch_sweep's codes);
// pcodes, cbp: those of the iteration whose backward step ran last and its C' (null on the
// first backward step, whose incoming Sigma'' is zero)
int launch_sweep_bwd(const Batch& B, int cb, const uint8_t* codes, int sb, int xr, int halo,
                     int mup, const uint8_t* pcodes, int cbp, hipStream_t s);
int launch_mubar_reduce(const Batch& B, int mup, int mub, hipStream_t s);
int launch_pupdate_bwd(const Batch& B, int x, int bx, int yl, int yh, int l1, int l2, int w1b,
                       int w2b, int l1b, int l2b, int bxb, int xp, int gyl, int gyh, int part,
                       hipStream_t s);
int launch_weights_bwd(const Batch& B, int yh, int mub, int eb, int part, int w0, hipStream_t s);
int launch_yh_bwd(const Batch& B, int yh, int eb, int gyh, hipStream_t s);
int launch_upsample_bwd(const Batch& B, int x0b, int gyl, hipStream_t s);
int launch_grad_scalars(const Batch& B, int part, int npix, int nw, double* out, hipStream_t s);
// Finite check every kFiniteEvery iterations (and after the last) with NLPR_CHECK_FINITE.
constexpr int kFiniteEvery = 8;
int launch_finite_clear(int* flag, hipStream_t s);
int launch_finite(const Batch& B, int z, int* flag, int iter, hipStream_t s);
int launch_fill(const Batch& B, int slot, hipStream_t s);   // zero a [L][p][q] slot
int launch_upsample_zero(const Batch& B, int yl, int t, hipStream_t s);   // S^T Y_l / rho
// X = solve(C) (+ add, a [L][p][q] slot, when add >= 0); the fused-S system for fused scenes
int launch_xsolve(const Batch& B, int c, int x, int f, int add, hipStream_t s);
// Sigma' (coded: values in slot `sigma`, code bytes in slot B_SCODE) is updated in place.
// codes (differentiated form, one item per thread): also write each dual element's 2-bit
// threshold branch there, one byte per float4 of Sigma'.  count: if not null, add the
// number of open items written (float4s stored) to *count.
int launch_sweep(const Batch& B, int x, int mu, int sigma, int creg, int halo, bool first,
                 hipStream_t s, uint8_t* codes = nullptr, unsigned long long* count = nullptr);
// Dense Sigma' of bands [c0, c0 + nb) of scene 0: [nb][Npairs][|P|][p][q]
int launch_sigma_expand(const Batch& B, const float* sig, const uint8_t* codes, const float* mu,
                        int c0, int nb, float* out, hipStream_t s);
// zero n 64-bit counters
int launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
int sweep_prepare(int K, int items);   // kernel attributes; before launches or capture

// ---- shapes and tuning
SweepShape choose_sweep_shape(int p, int q, int K, int halo);
int choose_pair_split(int blocks, int npairs);   // SweepShape.split for `blocks` (tile, band) pairs
size_t sweep_sigma_bytes(const SweepShape& sh, int q, int L, int npairs, int npatch);
int fft_block(int tpl);             // workgroup size of a line FFT with tpl threads per line
int autotune_fft(Plan& P);          // picks P.fft by timing candidates (cached per (p, q, d if fused))
FftShape default_fft_shape(int p, int q, int d_fused);

}  // namespace nlpr
