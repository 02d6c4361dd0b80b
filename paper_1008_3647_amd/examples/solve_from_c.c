/*
 * solve_from_c -- the library used from plain C through include/ufg.h alone:
 * no Python, no torch. Reads a lattice problem from a file, applies
 * M (paper, Sec. 1, Eq. MatrixM) to the right-hand sides, solves M x = b by
 * BiCGStab (Sec. 1, Eq. 2 with one operator) on a stream of its own, and
 * writes both results.
 *
 *   solve_from_c IN OUT
 *
 * IN  (little-endian, packed): int32 nx, ntau, nrhs; float64 tau, g;
 *     float64 sigma[ntau][nx][nx][nx]; complex128 b[nrhs][ntau][nx][nx][nx]
 *     as interleaved (re, im) float64 pairs.
 * OUT: complex128 y[nrhs][...] = M b; complex128 x[nrhs][...] with
 *     ||b - M x|| <= 1e-12 ||b||; int32 status, iters; float64 relres.
 *
 * Exit status 0 on success; 1 with a message on stderr for a bad file, a HIP
 * error or a library error (the library's own text from ufg_last_error).
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "ufg.h"

static int fail_hip(const char* what, hipError_t e) {
  fprintf(stderr, "solve_from_c: %s: %s\n", what, hipGetErrorString(e));
  return 1;
}

static int fail_ufg(const char* what, int code) {
  fprintf(stderr, "solve_from_c: %s returned %d: %s\n", what, code, ufg_last_error());
  return 1;
}

#define HIP_TRY(call)                             \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return fail_hip(#call, e_); \
  } while (0)

static int run(FILE* in, FILE* out) {
  int dims[3];
  double tg[2];
  if (fread(dims, sizeof(int), 3, in) != 3 || fread(tg, sizeof(double), 2, in) != 2) {
    fprintf(stderr, "solve_from_c: short header\n");
    return 1;
  }
  const int nx = dims[0], ntau = dims[1], nrhs = dims[2];
  if (nx < 2 || nx > 16 || ntau < 2 || ntau > (1 << 20) || nrhs < 1 || nrhs > 64) {
    fprintf(stderr, "solve_from_c: sizes out of range (nx %d, ntau %d, nrhs %d)\n", nx, ntau,
            nrhs);
    return 1;
  }
  const size_t n = (size_t)nx * nx * nx * ntau;   /* sites */
  const size_t nv = n * (size_t)nrhs * 2;          /* float64 per vector set */
  double* sigma = malloc(n * sizeof(double));
  double* buf = malloc(nv * sizeof(double));
  if (!sigma || !buf) {
    fprintf(stderr, "solve_from_c: out of host memory\n");
    return 1;
  }
  if (fread(sigma, sizeof(double), n, in) != n || fread(buf, sizeof(double), nv, in) != nv) {
    fprintf(stderr, "solve_from_c: short body\n");
    return 1;
  }

  hipStream_t stream;
  HIP_TRY(hipStreamCreate(&stream));
  void *sigma_d, *b_d, *y_d, *x_d;
  HIP_TRY(hipMalloc(&sigma_d, n * sizeof(double)));
  HIP_TRY(hipMalloc(&b_d, nv * sizeof(double)));
  HIP_TRY(hipMalloc(&y_d, nv * sizeof(double)));
  HIP_TRY(hipMalloc(&x_d, nv * sizeof(double)));
  HIP_TRY(hipMemcpy(sigma_d, sigma, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b_d, buf, nv * sizeof(double), hipMemcpyHostToDevice));

  ufg_lattice L = NULL;
  int rc = create_lattice(nx, ntau, tg[0], tg[1], UFG_C128, (void*)stream, &L);
  if (rc != UFG_OK) return fail_ufg("create_lattice", rc);
  if ((rc = set_aux_field(L, (const double*)sigma_d)) != UFG_OK)
    return fail_ufg("set_aux_field", rc);

  /* y = M b is enqueued on the lattice's stream */
  if ((rc = apply_M(L, b_d, y_d, nrhs)) != UFG_OK) return fail_ufg("apply_M", rc);
  HIP_TRY(hipStreamSynchronize(stream));
  HIP_TRY(hipMemcpy(buf, y_d, nv * sizeof(double), hipMemcpyDeviceToHost));
  if (fwrite(buf, sizeof(double), nv, out) != nv) return 1;

  /* M x = b, unpreconditioned, all in FP64; the solve returns when done */
  ufg_solve_opts o = {0};
  o.tol = 1e-12;
  o.maxit = 10000;
  o.delta = 0.1;
  o.check_every = 10;
  ufg_solve_stats st;
  rc = solve_bicgstab(L, NULL, UFG_OP_M, b_d, x_d, nrhs, &o, &st);
  if (rc < 0) return fail_ufg("solve_bicgstab", rc);
  HIP_TRY(hipMemcpy(buf, x_d, nv * sizeof(double), hipMemcpyDeviceToHost));
  if (fwrite(buf, sizeof(double), nv, out) != nv) return 1;
  const int tail[2] = {st.status, st.iters[0]};
  if (fwrite(tail, sizeof(int), 2, out) != 2 || fwrite(&st.relres[0], sizeof(double), 1, out) != 1)
    return 1;
  printf("solve_from_c: %dx%dx%dx%d, %d rhs: status %d, %d iterations, relres %.3e\n", nx, nx,
         nx, ntau, nrhs, st.status, st.iters[0], st.relres[0]);

  if ((rc = destroy_lattice(L)) != UFG_OK) return fail_ufg("destroy_lattice", rc);
  HIP_TRY(hipFree(sigma_d));
  HIP_TRY(hipFree(b_d));
  HIP_TRY(hipFree(y_d));
  HIP_TRY(hipFree(x_d));
  HIP_TRY(hipStreamDestroy(stream));
  free(sigma);
  free(buf);
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: solve_from_c IN OUT\n");
    return 1;
  }
  FILE* in = fopen(argv[1], "rb");
  FILE* out = fopen(argv[2], "wb");
  if (!in || !out) {
    fprintf(stderr, "solve_from_c: cannot open %s or %s\n", argv[1], argv[2]);
    return 1;
  }
  const int rc = run(in, out);
  fclose(in);
  if (fclose(out) != 0) return 1;
  return rc;
}
