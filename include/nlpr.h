/*
 * nlpr.h - C ABI of libnlpr, an MI355X (gfx950) implementation of the ADMM solver of
 * guided nonlocal patch-regularised (NLPR) multiband fusion:
 *
 *   Unni V. S., P. Nair, K. N. Chaudhury, "Guided Nonlocal Patch Regularization and
 *   Efficient Filtering-Based Inversion for Multiband Fusion", arXiv 2210.04184.
 *
 * Problem (Sec. "Variational models", eqs. (model), (mainoptim); Sec. "Definition",
 * eqs. (reg1), (wts)): recover Z (n_h pixels x L bands) from
 *     Y_l = S B Z + N_l   (L bands, decimated by d, blurred by the circular kernel b)
 *     Y_h = Z R + N_h     (L_h bands at full resolution; R is L x L_h)
 * by minimising
 *     1/2 ||Y_l - S B Z||^2 + lambda1/2 ||Y_h - Z R||^2
 *       + lambda * sum_i sum_{tau in W} omega_{i tau} ||P_{i tau}(Z)||_1,
 *     omega_{i tau} = exp(-||P_{i tau}(Y_h)||_2^2 / h^2),
 * where P_{i tau} is the difference of the (2K+1)x(2K+1) patches at i and i - tau on the
 * periodic image domain and W = [-Sw, Sw]^2.  The solver runs the ADMM iteration of
 * Sec. "Optimization" (eqs. (inv), (Qh_update), (Qm_update), (Qj_main),
 * (dualvar1_main)-(dualvar3_main)) with E = I (Z coincides with the paper's X).
 *
 * Conventions shared by every entry point
 *   - Images are planar, band-major, row-major float32: element (c, i1, i2) of an image
 *     with p rows and q columns lives at [(c * p + i1) * q + i2].
 *   - Device pointers are HIP device allocations on the device that was current when the
 *     plan was created.  Host pointers are plain host memory.  The caller owns every
 *     buffer it passes; the library never frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream).
 *     Work is enqueued asynchronously; completion is observed by synchronising the
 *     stream.  Plans and batches of at least 2^22 pixel-bands (without NLPR_TIMING) run
 *     part of each iteration on a second stream of their own, forked from `stream` and
 *     joined back into it within the call, so `stream` still orders all of the call's work.
 *   - Every function returns an nlpr_status.  No C++ exception crosses the ABI.  On error
 *     nlpr_last_error() returns a message for the calling thread.
 *   - Functions are thread-safe for distinct plans.  Host calls that share a plan must not
 *     overlap (one host thread at a time per plan).  On the device, the work of successive
 *     calls on one plan runs in call order even when the calls pass different streams:
 *     each call's stream first waits for the device work of the previous call on that
 *     plan.  Concurrent solves therefore need one plan each; calls that share a workspace
 *     must not run concurrently on the device.
 */
#ifndef NLPR_H
#define NLPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nlpr_status {
  NLPR_OK = 0,
  NLPR_ERR_INVALID_ARG = 1,        /* null pointer, negative size, host pointer where a device one is needed */
  NLPR_ERR_UNSUPPORTED_SHAPE = 2,  /* a size outside the limits documented at nlpr_params              */
  NLPR_ERR_WORKSPACE_TOO_SMALL = 3,/* ws_bytes < nlpr_workspace_size()                                  */
  NLPR_ERR_HIP = 4,                /* a HIP runtime call or a kernel launch failed                      */
  NLPR_ERR_NUMERICAL = 5,          /* NaN or Inf found in the result (NLPR_CHECK_FINITE)                */
  NLPR_ERR_NOT_ENABLED = 6         /* the plan was not created with the option this call needs          */
} nlpr_status;

/* nlpr_params.flags */
enum {
  NLPR_INIT_ZERO = 1u << 0,     /* start every ADMM variable at 0 instead of the default start:
                                   X0 = nearest-neighbour upsample of Y_l, P1 = B X0, P2 = X0,
                                   Q = Sigma = Lambda1 = Lambda2 = 0 (the paper names but does not
                                   give the initial values, Sec. "Optimization")                       */
  NLPR_STATE_IN = 1u << 1,      /* resume: the workspace holds the state left by an earlier
                                   nlpr_solve with the same plan and the same Y_h (the dual state
                                   keeps elements on the threshold by reference to the thresholds,
                                   which each solve derives from Y_h); run `iters` more iterations */
  NLPR_UNWEIGHTED = 1u << 2,    /* omega = 1 (ablation cases C2 / C4 of the paper)                    */
  NLPR_LOCAL_WINDOW = 1u << 3,  /* W = {0, +-e1, +-e2}: local pixel differences (ablation C5);
                                   requires Sw == 1                                                  */
  NLPR_CHECK_FINITE = 1u << 4,  /* check the iterate X for NaN/Inf on the device after every 8th
                                   iteration and after the last one, without waiting; the
                                   first checked iteration that finds one is kept in a device
                                   flag, which nlpr_solve reads once at the end (this
                                   synchronises the stream) and then returns NLPR_ERR_NUMERICAL
                                   (see nlpr_nonfinite_iteration)                                   */
  NLPR_TIMING = 1u << 5,        /* record HIP events around every stage; read with nlpr_stage_time   */
  NLPR_GRAPH = 1u << 6,         /* capture the whole solve (weights, start, all iterations) in a HIP
                                   graph on the first call and replay it on later calls; ignored
                                   with NLPR_TIMING.  The graph reads buffer addresses from a
                                   device descriptor written before each launch, so later calls
                                   may pass other buffers.                                          */
  NLPR_FUSED_S = 1u << 7        /* splitting without P1: the X-update keeps S B in its system,
                                   (I + sum D^T D + B^T S^T S B / rho) X = B^T S^T Y_l / rho + P2
                                   + Lambda2 + sum D^T (Q + Sigma), solved in Fourier per
                                   aliasing group of d^2 frequencies (Sherman-Morrison, tables in
                                   FP64).  Same minimiser as the paper's splitting of eq.
                                   (fusionoptim), different iterates.  Requires Ls == 0 and
                                   8 * (d + 1) * p <= 65536 (a column group and the twiddles fit
                                   one FFT workgroup).  */
};

/*
 * Problem size and parameters.  Limits (else NLPR_ERR_UNSUPPORTED_SHAPE):
 *   p, q       : image rows / columns, each of the form 2^a 3^b, 8 <= p, q <= 4096, q % 4 == 0;
 *                p % d == 0 and q % d == 0.
 *   L          : bands of Y_l and Z, 1 <= L <= 4096.
 *   Lh         : bands of Y_h, 1 <= Lh <= 16.
 *   d          : decimation factor >= 1; S keeps the pixels (d*m1, d*m2).
 *   blur_radius: r, the blur kernel is (2r+1) x (2r+1), centred, 0 <= r <= 16.
 *   K          : patch radius, P = [-K, K]^2, 0 <= K <= 4.
 *   Sw         : search radius, W = [-Sw, Sw]^2, 0 <= Sw <= 8, Sw < p and Sw < q.
 *   The sweep keeps full image rows in LDS: with R = max(1, 1024 * items / q) rows per tile
 *   (items = 1, 2 or 4, the smallest with 1024 * items >= q),
 *   4 * ((R + 2K) q + 2 (R + Sw) q) must not exceed 160 KiB (e.g. q <= 2048 for
 *   K = 2, Sw = 5).
 *   iters      : ADMM iterations, >= 0.
 *   Ls         : 0 = no subspace (Z is the ADMM variable X).  1 <= Ls <= min(L, 32): Z = X E
 *                with the fixed basis E (Ls x L) passed to nlpr_plan_create; X has Ls bands
 *                and the dual state shrinks by L / Ls (Sec. "Variational models").
 *   monitor_every : 0 = no monitor.  N > 0: after iterations N, 2N, ... and after the last
 *                iteration of each solve, record the objective of eq. (mainoptim) with its
 *                terms and the primal residuals of eq. (fusionoptim) (read with nlpr_monitor).
 *   lambda     : regulariser weight lambda_2 >= 0.  The soft-threshold of eq. (Qj_main) is
 *                lambda * omega / rho.
 *   lambda1    : weight of the Y_h term, > 0.
 *   rho        : ADMM penalty, > 0.
 *   h          : width of the guide weights of eq. (wts), > 0 (ignored with NLPR_UNWEIGHTED).
 */
typedef struct nlpr_params {
  int32_t p, q;
  int32_t L, Lh;
  int32_t d;
  int32_t blur_radius;
  int32_t K, Sw;
  int32_t iters;
  uint32_t flags;
  int32_t Ls;
  int32_t monitor_every;
  double lambda;
  double lambda1;
  double rho;
  double h;
} nlpr_params;

typedef struct nlpr_plan nlpr_plan;

/*
 * Create a plan on the current HIP device: validate the parameters, upload the blur taps
 * and R, and precompute the tables the iteration reuses (Sec. "Computational details"):
 * the inverse Fourier denominator 1/(1 + |b^|^2 + |P| sum_{tau in W} |d^_{tau 0}|^2) of
 * eq. (inv), computed in FP64 and stored FP32, the FFT twiddles, and the L_h x L_h
 * matrix G = (rho/lambda1 I + R^T R)^{-1} (FP64) with which the P2-update of
 * eq. (Qm_update) applies F = (I + lambda1/rho R R^T)^{-1} = I - R G R^T.
 *   blur_host : host, (2r+1)^2 floats, row-major, tap b(m1, m2) at [(m1 + r)(2r+1) + m2 + r];
 *               B X (i) = sum_m b(m) X(i - m), circular.  When b has rank one up to FP32
 *               rounding (no tap off by more than 1e-6 of the largest; a Gaussian, for
 *               one), the plan also stores its row and column factors (derived in FP64)
 *               and applies B as a row and a column pass; nlpr_plan_info.blur_separable
 *               reports it.
 *   R_host    : host, L x Lh floats, row-major (R[c][h] at [c * Lh + h]).
 *   With NLPR_FUSED_S the plan also holds, per frequency, the FP64-derived factors of the
 *   aliasing-group solve (1/a, b^/a and gamma conj(b^)/a, with a the denominator of
 *   eq. (inv) without |b^|^2 and gamma = 1/(rho d^2 + sum_group |b^|^2/a)).
 *   E_host    : host, Ls x L floats, row-major (E[s][c] at [s * L + c]), the subspace basis
 *               (rows need not be orthonormal, E E^T must be invertible); NULL iff Ls == 0.
 *               With a basis the plan also holds, computed in FP64: (E E^T + rho I)^{-1} for
 *               the P1-update (eq. (Qh_update)), E^+ = E^T (E E^T)^{-1} for the default start
 *               X0 = up(Y_l) E^+, and E R, with which the P2-update runs as without a basis.
 *   out       : receives the plan.  The plan owns its small device tables only.
 * Allocates device memory for the tables (a few MB at 512 x 512).
 */
int nlpr_plan_create(const nlpr_params* params, const float* blur_host, const float* R_host,
                     const float* E_host, nlpr_plan** out);

/* Bytes of device workspace nlpr_solve needs for this plan.  The dominant part is the
 * dual state Sigma' (see nlpr_workspace_region): about 4 * Npairs * (2K+1)^2 * L * p * q bytes. */
int nlpr_workspace_size(const nlpr_plan* plan, size_t* bytes);

/*
 * Run params.iters ADMM iterations and write Z = X^(iters).
 *   Yl : device, [L][p/d][q/d]     low-resolution observation.
 *   Yh : device, [Lh][p][q]        high-resolution guide observation.
 *   Z  : device, [L][p][q]         output; also used as the X iterate during the solve.
 *   ws : device workspace of at least nlpr_workspace_size() bytes, 256-byte aligned.  It
 *        holds the ADMM state on return, so a later call with NLPR_STATE_IN continues the
 *        iteration (T1 iterations then T2 resumed iterations give the same Z, bit for bit,
 *        as T1 + T2 iterations at once).
 * Never allocates device memory.  Asynchronous on `stream` unless NLPR_CHECK_FINITE is set.
 */
int nlpr_solve(nlpr_plan* plan, const float* Yl, const float* Yh, float* Z, void* ws,
               size_t ws_bytes, void* stream);

/*
 * nlpr_solve for callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it).  Same result as
 * nlpr_solve, bit for bit, but the workspace is a static device array inside the library
 * of NLPR_NOALLOC_WORKSPACE_BYTES (64 MiB); each GPU the library runs on holds one until
 * the process ends.  No device memory is allocated or freed by this call.
 *   Yl, Yh, Z : as for nlpr_solve.
 * Errors: NLPR_ERR_WORKSPACE_TOO_SMALL when nlpr_workspace_size() exceeds
 * NLPR_NOALLOC_WORKSPACE_BYTES; NLPR_ERR_INVALID_ARG for a plan created with NLPR_STATE_IN,
 * NLPR_GRAPH or NLPR_TIMING.  Every call on one GPU shares that GPU's array and leaves its
 * state there: calls that overlap on one GPU (from any plan, stream or thread) race and
 * give undefined results.  Asynchronous on `stream` unless NLPR_CHECK_FINITE is set.
 */
#define NLPR_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
int nlpr_solve_noalloc(nlpr_plan* plan, const float* Yl, const float* Yh, float* Z,
                       void* stream);

/*
 * Decode the coded dual state (NLPR_REGION_SIGMA with its NLPR_REGION_SIGMA_CODES) of bands
 * [c0, c1) into dense FP32: out[c - c0][n][k][i1][i2] = Sigma'_{tau_n, k}(i1, i2) of band c,
 * tau_n the n-th shift of nlpr_half_window, k as in NLPR_REGION_SIGMA, (i1, i2) image pixels.
 *   sigma, codes : device, the two regions (of a workspace, or the Sigma' buffer of the SWEEP
 *                  stage and the code region of its ws);
 *   mu           : device, the thresholds [Npairs][p][q] the state was produced with
 *                  (NLPR_REGION_MU);
 *   out          : device, (c1 - c0) * Npairs * (2K+1)^2 * p * q floats.
 * Asynchronous on `stream`; ordered after the plan's earlier calls like any call on the plan.
 */
int nlpr_sigma_expand(const nlpr_plan* plan, const float* sigma, const void* codes,
                      const float* mu, int32_t c0, int32_t c1, float* out, void* stream);

/*
 * For plans created with NLPR_TIMING (else NLPR_ERR_NOT_ENABLED): the number of open items
 * (float4s of NLPR_REGION_SIGMA stored) each sweep of the last solve wrote, one count per
 * iteration.  counts : host, receives min(cap, n) values; n : receives iters (0 without a
 * search window).  Waits for the last solve.  The next sweep reads what the previous one
 * wrote, so these counts give the dual state's HBM bytes of every launch.
 */
int nlpr_sweep_counts(const nlpr_plan* plan, int64_t* counts, int32_t cap, int32_t* n);

/* For plans created with NLPR_CHECK_FINITE (else NLPR_ERR_NOT_ENABLED): the iteration t
 * whose check (t = 8, 16, ... and the last; 0 for a solve of 0 iterations) first found NaN
 * or Inf in the iterate during the last solve, or -1 if none did.  iter : host, receives t. */
int nlpr_nonfinite_iteration(const nlpr_plan* plan, int32_t* iter);

/* Release the plan and its device tables.  NULL is accepted. */
int nlpr_plan_destroy(nlpr_plan* plan);

/* Static description of a status code. */
const char* nlpr_status_string(int status);

/* Message of the last failed call on this thread ("" if none). */
const char* nlpr_last_error(void);

/*
 * The half window W+ = {tau in W : tau1 > 0, or tau1 == 0 and tau2 > 0} in the order the
 * library stores it.  By the antisymmetry omega_{i-tau,-tau} = omega_{i tau} and
 * D_{-tau,k} X(i - tau) = -D_{tau k} X(i), the duals of -tau are minus the duals of tau
 * and tau = 0 contributes nothing, so only W+ is stored.
 *   tau : host, receives 2 * min(cap, Npairs) int32 (tau1, tau2 pairs);   n : receives Npairs.
 */
int nlpr_half_window(const nlpr_plan* plan, int32_t* tau, int32_t cap, int32_t* n);

/* Geometry of a plan that callers need to read the dual state. */
typedef struct nlpr_plan_info {
  int32_t npairs;       /* |W+|, number of stored shifts                                    */
  int32_t npatch;       /* |P| = (2K+1)^2                                                   */
  int32_t tile_rows;    /* R: image rows per sweep tile                                      */
  int32_t ntiles;       /* ceil(p / R)                                                      */
  int32_t halo_rows;    /* largest tau1 in W+ (rows the adjoint scatter reaches above a tile) */
  int32_t blur_separable; /* 1: the blur has rank one and runs as a row and a column pass  */
  int32_t sweep_split;  /* workgroups per (tile, band) in the sweep, each over a contiguous
                           part of W+ (more than 1 for scenes with few tiles x bands)        */
  size_t sigma_elems;   /* floats in the Sigma' region (= L * ntiles * npairs * npatch * R * q) */
} nlpr_plan_info;
int nlpr_plan_get_info(const nlpr_plan* plan, nlpr_plan_info* info);

/* Workspace regions (byte offset and size inside ws). */
typedef enum nlpr_region {
  NLPR_REGION_SIGMA = 0,  /* Sigma', the dual of eq. (dualvar3_main) for tau in W+ (order of
                             nlpr_half_window) and k in P (k1 major, then k2, each from -K to
                             K), stored source-aligned: Sigma'_{tau k}(j) = Sigma_{tau k}(j + k),
                             in coded form (with NLPR_REGION_SIGMA_CODES; read it with
                             nlpr_sigma_expand).  Its planes are laid out
                             [L][ntiles][Npairs][|P|][R][q] (nlpr_plan_get_info): image row i
                             of band c lives in tile i / R at row i % R, so one sweep workgroup
                             streams one contiguous block.  Each plane is cut into items of 4
                             consecutive floats and segments of 64 items (1 KB).  Every dual
                             value is -clip(V, +-mu) (eqs. (Qj_main), (dualvar3_main)), so an
                             element on the threshold is -mu (V > 0) or +mu (V < 0) and is not
                             stored; for an item with any element off the threshold ("open")
                             the 4 values -Sigma' = clip(V, +-mu) are stored, packed at the
                             start of the item's segment in item order.                      */
  NLPR_REGION_MU = 1,     /* mu [Npairs][p][q] = lambda * omega_{i tau} / rho, the thresholds         */
  NLPR_REGION_C = 2,      /* C [L][p][q], right-hand side of eq. (x_linear_system_main)                */
  NLPR_REGION_LAMBDA1 = 3,/* Lambda1 [L][p][q]                                                       */
  NLPR_REGION_LAMBDA2 = 4,/* Lambda2 [L][p][q]                                                       */
  NLPR_REGION_SIGMA_CODES = 5, /* one byte per item of NLPR_REGION_SIGMA (byte index = float
                             offset of the item / 4); for element e, bit e is the sign bit
                             of V (set: an element on the threshold holds +mu, else -mu) and
                             bit 4 + e is set if |V| < mu (off the threshold); an item whose
                             byte is below 16 is on the threshold in all four elements     */
  NLPR_REGION_COUNT = 6
} nlpr_region;
int nlpr_workspace_region(const nlpr_plan* plan, int region, size_t* offset, size_t* bytes);

/*
 * Run one step of the iteration on caller buffers (per-kernel testing).  bufs holds device
 * pointers in the order listed; `ws` means a workspace of nlpr_workspace_size() bytes used
 * as scratch.
 *   NLPR_STAGE_WEIGHTS     {Yh, mu}                   mu = lambda omega / rho for tau in W+ (eq. (wts))
 *   NLPR_STAGE_XSOLVE      {C, X, ws}                 X = IDFT(DFT(C) / den) per band (eq. (inv))
 *   NLPR_STAGE_BLUR        {X, BX}                    BX = B X
 *   NLPR_STAGE_BLUR_T      {Y, BtY}                   BtY = B^T Y
 *   NLPR_STAGE_PUPDATE     {X, BX, Yl, Yh, Lambda1, Lambda2, W1, W2}
 *                          P1 by eq. (Qh_update), P2 by eq. (Qm_update), then eqs.
 *                          (dualvar1_main), (dualvar2_main) update Lambda1, Lambda2 in place;
 *                          W1 = P1 + Lambda1 and W2 = P2 + Lambda2 with the new duals.
 *   NLPR_STAGE_SWEEP       {X, mu, Sigma', Creg, ws}  Q-update (eq. (Qj_main)) and Sigma-update
 *                          (eq. (dualvar3_main)) for every tau in W, k in P, in place on Sigma'
 *                          (sigma_elems floats, coded as NLPR_REGION_SIGMA, with its code bytes
 *                          in the NLPR_REGION_SIGMA_CODES region of ws);
 *                          Creg = sum_{tau in W} sum_k D_{tau k}^T (Q_{tau k} + Sigma_{tau k}).
 *   NLPR_STAGE_SWEEP_FIRST same, with Sigma' taken as 0 on input (only written).
 *   NLPR_STAGE_ASSEMBLE    {W1, W2, Creg, C}          C = B^T W1 + W2 + Creg
 *   NLPR_STAGE_INIT        {Yl, X0, W1, W2, Lambda1, Lambda2, C}   the initial values and C^(0)
 * All stages act on X-space buffers (Ls bands with a basis); INIT and PUPDATE are for plans
 * without a basis (else NLPR_ERR_UNSUPPORTED_SHAPE).
 */
enum {
  NLPR_STAGE_WEIGHTS = 1,
  NLPR_STAGE_XSOLVE = 2,
  NLPR_STAGE_BLUR = 3,
  NLPR_STAGE_BLUR_T = 4,
  NLPR_STAGE_PUPDATE = 5,
  NLPR_STAGE_SWEEP = 6,
  NLPR_STAGE_SWEEP_FIRST = 7,
  NLPR_STAGE_ASSEMBLE = 8,
  NLPR_STAGE_INIT = 9,
  NLPR_STAGE_MONITOR = 10,      /* timing only (no per-stage entry point)                         */
  NLPR_STAGE_COUNT = 11
};
int nlpr_debug_stage(nlpr_plan* plan, int stage, void* const* bufs, int32_t nbufs, void* stream);

/*
 * Accumulated device time of one stage over the solves since the last reset, from the HIP
 * events recorded on the solve's stream (plans created with NLPR_TIMING only).
 * Synchronises on the recorded events.  ms_total: sum of launch durations in ms;
 * launches: number of timed launches.  reset != 0 clears the totals after reading.
 */
int nlpr_stage_time(nlpr_plan* plan, int stage, double* ms_total, int64_t* launches, int reset);

/*
 * Monitor trace of the last solve (plans created with monitor_every > 0, else
 * NLPR_ERR_NOT_ENABLED).  One record of NLPR_MON_FIELDS doubles per monitored iteration
 * t (t = N, 2N, ... and the last iteration of the solve, counted from 1 in each call):
 *   [NLPR_MON_ITER]      t
 *   [NLPR_MON_OBJECTIVE] f(X^(t)) = data_l + data_h + reg, eq. (mainoptim) (the quantity the
 *                        paper plots against t in its convergence figure)
 *   [NLPR_MON_DATA_L]    1/2 ||Y_l - S B X^(t) E||^2
 *   [NLPR_MON_DATA_H]    lambda1/2 ||Y_h - X^(t) E R||^2
 *   [NLPR_MON_REG]       lambda2 sum_{i, c} sum_{tau in W} sum_{k in P} omega_{i tau}
 *                        |D_{tau k} X^(t)(i, c)|, eq. (regfilt1), evaluated as
 *                        2 rho sum_{tau in W+} sum_j (sum_{k in P} mu_{j+k, tau})
 *                        sum_c |X(j, c) - X(j - tau, c)| (mu = lambda2 omega / rho)
 *   [NLPR_MON_R1]        ||B X^(t) - P1^(t)||,   [NLPR_MON_R2] ||X^(t) - P2^(t)||:
 *                        the primal residuals of the constraints of eq. (fusionoptim)
 *   [7]                  0
 * Terms are formed in FP32 from the iterate and summed in FP64 in a fixed order (the
 * trace is bit-for-bit repeatable).  Monitoring does not change the iterates.
 *   trace : host, receives min(cap, n) records (cap * NLPR_MON_FIELDS doubles);
 *   n     : receives the number of records of the last solve (0 before the first).
 * Waits for the last solve to complete.
 */
enum {
  NLPR_MON_ITER = 0, NLPR_MON_OBJECTIVE = 1, NLPR_MON_DATA_L = 2, NLPR_MON_DATA_H = 3,
  NLPR_MON_REG = 4, NLPR_MON_R1 = 5, NLPR_MON_R2 = 6, NLPR_MON_FIELDS = 8
};
int nlpr_monitor(const nlpr_plan* plan, double* trace, int32_t cap, int32_t* n);

/*
 * Reverse mode (the differentiated form): the gradient of a loss of Z = X^(iters) with
 * respect to Y_l, Y_h, lambda_2 and rho, through every unrolled iteration of the paper's
 * splitting (Sec. "Optimization": eqs. (inv), (Qh_update), (Qm_update), (Qj_main),
 * (dualvar1_main) - (dualvar3_main)), the default start and the guide weights of eq. (wts)
 * (Y_h reaches Z both through Y_h R^T and through the weights).  The derivative of the
 * soft threshold is taken as 1 where |V| > mu and 0 elsewhere (its value at |V| = mu is
 * immaterial for almost every input).  Plans with E = I, the paper's splitting (no
 * NLPR_FUSED_S), without NLPR_STATE_IN, iters >= 1, and (with a search window) q <= 1024
 * with the sweep adjoint's LDS tile within 160 KiB; else NLPR_ERR_UNSUPPORTED_SHAPE or
 * NLPR_ERR_INVALID_ARG.
 *
 * nlpr_grad_sizes: bytes of the checkpoint buffer and of the gradient workspace.  For
 *   t = 1 .. iters-1 the checkpoints hold X^t, B X^t, the Lambda1 and Lambda2 entering
 *   iteration t, and which branch of the threshold every dual element of its sweep took
 *   (2 bits each: |V| < mu, V >= mu or V <= -mu; the adjoint needs nothing else of Sigma).
 *   They take (iters - 1) * (16 + Npairs |P| / 4) * L * p * q bytes, each part rounded up to
 *   a multiple of 256 (at least 256 in all).
 * nlpr_forward: like nlpr_solve (Z equal bit for bit) and also writes the checkpoints to ck
 *   (device, 256-byte aligned).  ws as for nlpr_solve; the dual state is updated in it in
 *   place, as by nlpr_solve.
 * nlpr_backward: given dZ = dloss/dZ (device, [L][p][q]), reloads each iteration's X, B X
 *   and Lambda from its checkpoint and carries the adjoints back; writes dYl ([L][p/d][q/d]),
 *   dYh ([Lh][p][q]) and dscal (device, 2 doubles: dloss/dlambda_2, dloss/drho).  ws, ck
 *   from the matching nlpr_forward (same Yl, Yh); gws: gradient workspace (device,
 *   256-byte aligned).  Never allocates; asynchronous on `stream`; sums run in a fixed
 *   order, so gradients repeat bit for bit.
 */
int nlpr_grad_sizes(const nlpr_plan* plan, size_t* ck_bytes, size_t* gws_bytes);
int nlpr_forward(nlpr_plan* plan, const float* Yl, const float* Yh, float* Z, void* ws,
                 size_t ws_bytes, void* ck, size_t ck_bytes, void* stream);
int nlpr_backward(nlpr_plan* plan, const float* Yl, const float* Yh, const float* dZ, void* ws,
                  size_t ws_bytes, void* ck, size_t ck_bytes, void* gws, size_t gws_bytes,
                  float* dYl, float* dYh, double* dscal, void* stream);

/*
 * Batches: many independent scenes solved together (the multi-scene workload).  Every stage
 * of the iteration is one kernel launch over all scenes: a table of (scene, block) work
 * items maps each workgroup to a scene, whose sizes, tables and buffers a device
 * descriptor holds.  With NLPR_GRAPH the whole batched solve is one HIP graph.
 *   n        : number of scenes >= 1.
 *   params   : host array of n parameter sets.  Scenes may differ in every size and
 *              parameter, but must share iters, monitor_every and the flags
 *              NLPR_INIT_ZERO, NLPR_STATE_IN, NLPR_CHECK_FINITE, NLPR_TIMING and NLPR_GRAPH
 *              (else NLPR_ERR_INVALID_ARG).
 *   blur_host, R_host, E_host : host arrays of n host pointers, as for nlpr_plan_create
 *              (E_host may be NULL when no scene has a basis).
 * The workspace of a batch is the concatenation of the scenes' workspaces;
 * nlpr_batch_region gives a region of one scene (offset from the start of ws).
 * nlpr_batch_solve takes host arrays of n device pointers Yl[s], Yh[s], Z[s] laid out as
 * for nlpr_solve; it never allocates device memory.
 */
typedef struct nlpr_batch nlpr_batch;
int nlpr_batch_create(int32_t n, const nlpr_params* params, const float* const* blur_host,
                      const float* const* R_host, const float* const* E_host, nlpr_batch** out);
int nlpr_batch_workspace_size(const nlpr_batch* batch, size_t* bytes);
int nlpr_batch_region(const nlpr_batch* batch, int32_t scene, int region, size_t* offset,
                      size_t* bytes);
int nlpr_batch_solve(nlpr_batch* batch, const float* const* Yl, const float* const* Yh,
                     float* const* Z, void* ws, size_t ws_bytes, void* stream);
int nlpr_batch_stage_time(nlpr_batch* batch, int stage, double* ms_total, int64_t* launches,
                          int reset);
/* The monitor trace of one scene of the last batched solve, as nlpr_monitor. */
int nlpr_batch_monitor(const nlpr_batch* batch, int32_t scene, double* trace, int32_t cap,
                       int32_t* n);
int nlpr_batch_destroy(nlpr_batch* batch);

/*
 * Reference stream for the HBM roofline, not part of the method: negates the `bytes / 4`
 * floats at `buf` in place with one 16-byte non-temporal load and store per thread, the
 * access pattern of the dual sweep, so that its rate is the practical ceiling the sweep is
 * held against.  buf: device memory, 16-byte aligned; bytes: a multiple of 16, at most
 * 2^31 * 4096.  Asynchronous on `stream`.  NLPR_ERR_INVALID_ARG for a null, host or
 * misaligned buffer or a bad size.
 */
int nlpr_stream_rmw(void* buf, size_t bytes, void* stream);

/*
 * A second reference stream, with the sweep's own access shape and none of its arithmetic,
 * for the ceiling that pattern reaches on a given footprint.  nchunks workgroups of 256
 * threads; workgroup b owns chunk (b mod bands) * (nchunks / bands) + b / bands of
 * chunk_bytes contiguous bytes (bands fastest, the order in which the sweep visits its
 * tile-major dual state).  It negates that chunk in place in steps of `planes` 4 KB planes:
 * all 16-byte non-temporal loads of a step, then its stores.  lds_bytes of dynamic LDS per
 * workgroup (not used) limits the workgroups per CU as the sweep's tile does.
 *   buf: device memory, 16-byte aligned, buf_bytes long; nchunks * chunk_bytes <= buf_bytes.
 *   chunk_bytes: a positive multiple of 4096 * planes; planes in [1, 8]; nchunks a positive
 *   multiple of bands; lds_bytes <= 160 KiB.
 * Asynchronous on `stream`.  NLPR_ERR_INVALID_ARG for a null, host or misaligned buffer or
 * a bad size.
 */
int nlpr_stream_chunks(void* buf, size_t buf_bytes, size_t chunk_bytes, int32_t nchunks,
                       int32_t bands, int32_t planes, size_t lds_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NLPR_H */
