/*
 * Drives libnlpr through its C ABI alone (include/nlpr.h): plan creation from host tables,
 * workspace size, device buffers from hipMalloc, one solve on a HIP stream, copy back.
 * No Python or torch is involved.
 *
 * Usage: abi_solve <in.bin> <out.bin>
 *   in.bin : int32 [p, q, L, Lh, d, r, K, Sw, iters], float64 [lambda, lambda1, rho, h],
 *            float32 blur[(2r+1)^2], R[L*Lh], Yl[L*(p/d)*(q/d)], Yh[Lh*p*q]
 *   out.bin: float32 Z[L*p*q]
 * Exit status 0 on success; on a library error prints the status and message.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nlpr.h"

static int read_all(FILE* f, void* dst, size_t bytes) { return fread(dst, 1, bytes, f) == bytes; }

#define CHECK_NLPR(call)                                                                  \
  do {                                                                                    \
    int rc_ = (call);                                                                     \
    if (rc_ != NLPR_OK) {                                                                 \
      fprintf(stderr, "%s: %s (%s)\n", #call, nlpr_status_string(rc_), nlpr_last_error()); \
      return 2;                                                                           \
    }                                                                                     \
  } while (0)
#define CHECK_HIP(call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                          \
      return 3;                                                                           \
    }                                                                                     \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
    return 1;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 1;
  int32_t h[9];
  double dv[4];
  if (!read_all(f, h, sizeof h) || !read_all(f, dv, sizeof dv)) return 1;
  nlpr_params prm;
  memset(&prm, 0, sizeof prm);
  prm.p = h[0]; prm.q = h[1]; prm.L = h[2]; prm.Lh = h[3]; prm.d = h[4];
  prm.blur_radius = h[5]; prm.K = h[6]; prm.Sw = h[7]; prm.iters = h[8];
  prm.lambda = dv[0]; prm.lambda1 = dv[1]; prm.rho = dv[2]; prm.h = dv[3];
  const size_t nb = (size_t)(2 * prm.blur_radius + 1) * (2 * prm.blur_radius + 1);
  const size_t nR = (size_t)prm.L * prm.Lh;
  const size_t nYl = (size_t)prm.L * (prm.p / prm.d) * (prm.q / prm.d);
  const size_t nYh = (size_t)prm.Lh * prm.p * prm.q;
  const size_t nZ = (size_t)prm.L * prm.p * prm.q;
  float* blur = malloc(nb * 4);
  float* R = malloc(nR * 4);
  float* Yl = malloc(nYl * 4);
  float* Yh = malloc(nYh * 4);
  float* Z = malloc(nZ * 4);
  if (!blur || !R || !Yl || !Yh || !Z) return 1;
  if (!read_all(f, blur, nb * 4) || !read_all(f, R, nR * 4) || !read_all(f, Yl, nYl * 4) ||
      !read_all(f, Yh, nYh * 4))
    return 1;
  fclose(f);

  nlpr_plan* plan = NULL;
  CHECK_NLPR(nlpr_plan_create(&prm, blur, R, NULL, &plan));
  size_t ws_bytes = 0;
  CHECK_NLPR(nlpr_workspace_size(plan, &ws_bytes));
  void *d_ws = NULL, *d_Yl = NULL, *d_Yh = NULL, *d_Z = NULL;
  CHECK_HIP(hipMalloc(&d_ws, ws_bytes));
  CHECK_HIP(hipMalloc(&d_Yl, nYl * 4));
  CHECK_HIP(hipMalloc(&d_Yh, nYh * 4));
  CHECK_HIP(hipMalloc(&d_Z, nZ * 4));
  CHECK_HIP(hipMemcpy(d_Yl, Yl, nYl * 4, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_Yh, Yh, nYh * 4, hipMemcpyHostToDevice));
  hipStream_t stream;
  CHECK_HIP(hipStreamCreate(&stream));
  CHECK_NLPR(nlpr_solve(plan, d_Yl, d_Yh, d_Z, d_ws, ws_bytes, stream));
  CHECK_HIP(hipStreamSynchronize(stream));
  CHECK_HIP(hipMemcpy(Z, d_Z, nZ * 4, hipMemcpyDeviceToHost));
  CHECK_NLPR(nlpr_plan_destroy(plan));
  CHECK_HIP(hipStreamDestroy(stream));
  hipFree(d_ws);
  hipFree(d_Yl);
  hipFree(d_Yh);
  hipFree(d_Z);

  FILE* o = fopen(argv[2], "wb");
  if (!o || fwrite(Z, 4, nZ, o) != nZ) return 1;
  fclose(o);
  printf("abi_solve: %dx%dx%d, %d iterations, workspace %zu bytes\n", prm.p, prm.q, prm.L,
         prm.iters, ws_bytes);
  free(blur); free(R); free(Yl); free(Yh); free(Z);
  return 0;
}
