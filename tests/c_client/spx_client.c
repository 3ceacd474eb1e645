/* A plain C client of libspx: the library driven through include/spx.h alone,
 * with device memory from the HIP runtime's C API and no Python or torch.
 *
 *   spx_client --version          print spx_version() (no HIP call)
 *   spx_client IN OUT             run the calls below on IN, write OUT
 *
 * IN (little-endian): int32 m, n, nnz_in, k; int32 r[nnz_in], c[nnz_in];
 * f64 v[nnz_in], x[n], X[n*k] (row-major), dy[m].
 *
 * Calls, in order: csr_from_coo_host and csr_validate_host (host CRS arrays,
 * Sec. 3); csr_from_coo on the device, compared byte for byte with the host
 * assembly; csr_validate; plans for k = 1 and k; csr_spmv; csr_spmm;
 * csr_transpose_index and csr_spmv_t in both modes; csr_sddmm; two calls
 * that must fail with SPX_ERR_INVALID and a message.
 *
 * OUT (little-endian): int32 nnz; int32 rowptr[m+1], colind[nnz]; f64
 * values[nnz], y[m], Y[m*k], dx[n] (CSC gather), dx_atomic[n], dvalues[nnz].
 * Exit status 0 on success; 2 bad input, 3 HIP error, 4 library error,
 * 5 a check failed. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "spx.h"

#define HIP_CHECK(e)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (e);                                                                        \
    if (e_ != hipSuccess) {                                                                     \
      fprintf(stderr, "spx_client: HIP error %s (line %d)\n", hipGetErrorString(e_), __LINE__); \
      exit(3);                                                                                  \
    }                                                                                           \
  } while (0)

#define SPX_CHECK(e)                                                                                  \
  do {                                                                                                \
    spx_status s_ = (e);                                                                              \
    if (s_ != SPX_OK) {                                                                               \
      fprintf(stderr, "spx_client: status %d: %s (line %d)\n", (int)s_, spx_last_error(), __LINE__); \
      exit(4);                                                                                        \
    }                                                                                                 \
  } while (0)

static void fail_check(const char *what) {
  fprintf(stderr, "spx_client: check failed: %s\n", what);
  exit(5);
}

static void *xmalloc(size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p) {
    fprintf(stderr, "spx_client: out of host memory\n");
    exit(2);
  }
  return p;
}

static void read_exact(FILE *f, void *dst, size_t bytes) {
  if (bytes && fread(dst, 1, bytes, f) != bytes) {
    fprintf(stderr, "spx_client: short input\n");
    exit(2);
  }
}

static void write_exact(FILE *f, const void *src, size_t bytes) {
  if (bytes && fwrite(src, 1, bytes, f) != bytes) {
    fprintf(stderr, "spx_client: short write\n");
    exit(2);
  }
}

/* device copy of a host array */
static void *to_device(const void *h, size_t bytes) {
  void *d = NULL;
  HIP_CHECK(hipMalloc(&d, bytes ? bytes : 1));
  if (bytes) HIP_CHECK(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
  return d;
}

static void *device_buffer(size_t bytes) {
  void *d = NULL;
  HIP_CHECK(hipMalloc(&d, bytes ? bytes : 1));
  return d;
}

static void to_host(void *h, const void *d, size_t bytes) {
  if (bytes) HIP_CHECK(hipMemcpy(h, d, bytes, hipMemcpyDeviceToHost));
}

static spx_plan *make_plan(int32_t m, int32_t n, int32_t nnz, const int32_t *d_rowptr, int32_t k,
                           void **ws_out) {
  spx_plan_opts o;
  size_t bytes = 0;
  spx_plan *p = NULL;
  SPX_CHECK(spx_plan_default_opts(k, SPX_F64, &o));
  SPX_CHECK(csr_plan_workspace_bytes(m, nnz, &o, &bytes));
  *ws_out = device_buffer(bytes);
  SPX_CHECK(csr_plan_create(m, n, nnz, d_rowptr, &o, *ws_out, bytes, NULL, &p));
  return p;
}

int main(int argc, char **argv) {
  if (argc == 2 && strcmp(argv[1], "--version") == 0) {
    printf("%s\n", spx_version());
    return 0;
  }
  if (argc != 3) {
    fprintf(stderr, "usage: spx_client --version | spx_client IN OUT\n");
    return 2;
  }
  FILE *in = fopen(argv[1], "rb");
  if (!in) {
    fprintf(stderr, "spx_client: cannot open %s\n", argv[1]);
    return 2;
  }
  int32_t hdr[4];
  read_exact(in, hdr, sizeof(hdr));
  const int32_t m = hdr[0], n = hdr[1], nnz_in = hdr[2], k = hdr[3];
  if (m < 1 || n < 1 || nnz_in < 0 || k < 1) {
    fprintf(stderr, "spx_client: bad header\n");
    return 2;
  }
  int32_t *r = xmalloc(sizeof(int32_t) * (size_t)nnz_in);
  int32_t *c = xmalloc(sizeof(int32_t) * (size_t)nnz_in);
  double *v = xmalloc(sizeof(double) * (size_t)nnz_in);
  double *x = xmalloc(sizeof(double) * (size_t)n);
  double *X = xmalloc(sizeof(double) * (size_t)n * (size_t)k);
  double *dy = xmalloc(sizeof(double) * (size_t)m);
  read_exact(in, r, sizeof(int32_t) * (size_t)nnz_in);
  read_exact(in, c, sizeof(int32_t) * (size_t)nnz_in);
  read_exact(in, v, sizeof(double) * (size_t)nnz_in);
  read_exact(in, x, sizeof(double) * (size_t)n);
  read_exact(in, X, sizeof(double) * (size_t)n * (size_t)k);
  read_exact(in, dy, sizeof(double) * (size_t)m);
  fclose(in);

  /* host assembly (no HIP call) */
  int32_t *h_rowptr = xmalloc(sizeof(int32_t) * (size_t)(m + 1));
  int32_t *h_colind = xmalloc(sizeof(int32_t) * (size_t)nnz_in);
  double *h_values = xmalloc(sizeof(double) * (size_t)nnz_in);
  int32_t h_nnz = -1;
  SPX_CHECK(csr_from_coo_host(m, n, nnz_in, r, c, v, h_rowptr, h_colind, h_values, &h_nnz));
  SPX_CHECK(csr_validate_host(m, n, h_nnz, h_rowptr, h_colind));
  const int32_t nnz = h_nnz;

  /* device assembly from the same triplets */
  int32_t *d_r = to_device(r, sizeof(int32_t) * (size_t)nnz_in);
  int32_t *d_c = to_device(c, sizeof(int32_t) * (size_t)nnz_in);
  double *d_v = to_device(v, sizeof(double) * (size_t)nnz_in);
  int32_t *d_rowptr = device_buffer(sizeof(int32_t) * (size_t)(m + 1));
  int32_t *d_colind = device_buffer(sizeof(int32_t) * (size_t)nnz_in);
  double *d_values = device_buffer(sizeof(double) * (size_t)nnz_in);
  int32_t *d_scalar = device_buffer(sizeof(int32_t));
  size_t ws_bytes = 0;
  SPX_CHECK(csr_from_coo_workspace_bytes(m, n, nnz_in, &ws_bytes));
  void *d_ws = device_buffer(ws_bytes);
  SPX_CHECK(csr_from_coo(m, n, nnz_in, d_r, d_c, d_v, d_rowptr, d_colind, d_values, d_scalar, d_ws, ws_bytes,
                         NULL));
  int32_t d_nnz = -2;
  to_host(&d_nnz, d_scalar, sizeof(int32_t));
  if (d_nnz != nnz) fail_check("device and host assembly store different counts");
  {
    int32_t *t_rowptr = xmalloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t *t_colind = xmalloc(sizeof(int32_t) * (size_t)nnz);
    double *t_values = xmalloc(sizeof(double) * (size_t)nnz);
    to_host(t_rowptr, d_rowptr, sizeof(int32_t) * (size_t)(m + 1));
    to_host(t_colind, d_colind, sizeof(int32_t) * (size_t)nnz);
    to_host(t_values, d_values, sizeof(double) * (size_t)nnz);
    if (memcmp(t_rowptr, h_rowptr, sizeof(int32_t) * (size_t)(m + 1)) ||
        memcmp(t_colind, h_colind, sizeof(int32_t) * (size_t)nnz) ||
        memcmp(t_values, h_values, sizeof(double) * (size_t)nnz))
      fail_check("device assembly differs from host assembly");
    free(t_rowptr);
    free(t_colind);
    free(t_values);
  }
  int32_t status = -1;
  SPX_CHECK(csr_validate(m, n, nnz, d_rowptr, d_colind, 1, d_scalar, NULL));
  to_host(&status, d_scalar, sizeof(int32_t));
  if (status != 0) fail_check("csr_validate on the assembled matrix");

  /* products */
  void *ws1 = NULL, *wsk = NULL;
  spx_plan *p1 = make_plan(m, n, nnz, d_rowptr, 1, &ws1);
  spx_plan *pk = make_plan(m, n, nnz, d_rowptr, k, &wsk);
  double *d_x = to_device(x, sizeof(double) * (size_t)n);
  double *d_X = to_device(X, sizeof(double) * (size_t)n * (size_t)k);
  double *d_dy = to_device(dy, sizeof(double) * (size_t)m);
  double *d_y = device_buffer(sizeof(double) * (size_t)m);
  double *d_Y = device_buffer(sizeof(double) * (size_t)m * (size_t)k);
  SPX_CHECK(csr_spmv(m, n, nnz, d_rowptr, d_colind, d_values, SPX_F64, d_x, d_y, SPX_F64, p1, NULL));
  SPX_CHECK(csr_spmm(m, n, nnz, d_rowptr, d_colind, d_values, SPX_F64, k, d_X, k, d_Y, k, SPX_F64, pk, NULL));

  /* transpose and sampled dot */
  int32_t *d_colptr = device_buffer(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *d_rowind = device_buffer(sizeof(int32_t) * (size_t)nnz);
  int32_t *d_perm = device_buffer(sizeof(int32_t) * (size_t)nnz);
  size_t tbytes = 0;
  SPX_CHECK(csr_transpose_index_workspace_bytes(m, n, nnz, &tbytes));
  void *d_tws = device_buffer(tbytes);
  SPX_CHECK(csr_transpose_index(m, n, nnz, d_rowptr, d_colind, d_colptr, d_rowind, d_perm, d_tws, tbytes, NULL));
  double *d_dx = device_buffer(sizeof(double) * (size_t)n);
  double *d_dxa = device_buffer(sizeof(double) * (size_t)n);
  double *d_dv = device_buffer(sizeof(double) * (size_t)nnz);
  SPX_CHECK(csr_spmv_t(m, n, nnz, d_rowptr, d_colind, d_colptr, d_rowind, d_perm, d_values, SPX_F64, 1, d_dy, 1,
                       d_dx, 1, SPX_F64, 0, NULL, NULL));
  SPX_CHECK(csr_spmv_t(m, n, nnz, d_rowptr, d_colind, NULL, NULL, NULL, d_values, SPX_F64, 1, d_dy, 1, d_dxa, 1,
                       SPX_F64, 1, p1, NULL));
  SPX_CHECK(csr_sddmm(m, n, nnz, d_rowptr, d_colind, 1, d_dy, 1, d_x, 1, d_dv, SPX_F64, p1, NULL));

  /* errors are reported, not launched */
  if (csr_spmv(-1, n, nnz, d_rowptr, d_colind, d_values, SPX_F64, d_x, d_y, SPX_F64, NULL, NULL) !=
          SPX_ERR_INVALID ||
      spx_last_error()[0] == '\0')
    fail_check("negative m is rejected with a message");
  if (csr_spmm(m, n, nnz, d_rowptr, d_colind, d_values, SPX_F64, k, d_X, k - 1, d_Y, k, SPX_F64, pk, NULL) !=
      SPX_ERR_INVALID)
    fail_check("ldx < k is rejected");
  HIP_CHECK(hipDeviceSynchronize());

  /* results */
  double *y = xmalloc(sizeof(double) * (size_t)m);
  double *Y = xmalloc(sizeof(double) * (size_t)m * (size_t)k);
  double *dx = xmalloc(sizeof(double) * (size_t)n);
  double *dxa = xmalloc(sizeof(double) * (size_t)n);
  double *dv = xmalloc(sizeof(double) * (size_t)nnz);
  to_host(y, d_y, sizeof(double) * (size_t)m);
  to_host(Y, d_Y, sizeof(double) * (size_t)m * (size_t)k);
  to_host(dx, d_dx, sizeof(double) * (size_t)n);
  to_host(dxa, d_dxa, sizeof(double) * (size_t)n);
  to_host(dv, d_dv, sizeof(double) * (size_t)nnz);
  FILE *out = fopen(argv[2], "wb");
  if (!out) {
    fprintf(stderr, "spx_client: cannot open %s\n", argv[2]);
    return 2;
  }
  write_exact(out, &nnz, sizeof(int32_t));
  write_exact(out, h_rowptr, sizeof(int32_t) * (size_t)(m + 1));
  write_exact(out, h_colind, sizeof(int32_t) * (size_t)nnz);
  write_exact(out, h_values, sizeof(double) * (size_t)nnz);
  write_exact(out, y, sizeof(double) * (size_t)m);
  write_exact(out, Y, sizeof(double) * (size_t)m * (size_t)k);
  write_exact(out, dx, sizeof(double) * (size_t)n);
  write_exact(out, dxa, sizeof(double) * (size_t)n);
  write_exact(out, dv, sizeof(double) * (size_t)nnz);
  if (fclose(out) != 0) return 2;

  csr_plan_destroy(p1);
  csr_plan_destroy(pk);
  void *bufs[] = {d_r, d_c, d_v, d_rowptr, d_colind, d_values, d_scalar, d_ws, ws1, wsk, d_x, d_X, d_dy, d_y,
                  d_Y, d_colptr, d_rowind, d_perm, d_tws, d_dx, d_dxa, d_dv};
  for (size_t i = 0; i < sizeof(bufs) / sizeof(bufs[0]); ++i) HIP_CHECK(hipFree(bufs[i]));
  free(r);
  free(c);
  free(v);
  free(x);
  free(X);
  free(dy);
  free(h_rowptr);
  free(h_colind);
  free(h_values);
  free(y);
  free(Y);
  free(dx);
  free(dxa);
  free(dv);
  printf("spx_client: m=%d n=%d nnz=%d k=%d ok\n", m, n, nnz, k);
  return 0;
}
