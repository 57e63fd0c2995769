/* The C ABI used from plain C (no Python, no torch): a flat tied interface,
 * slave 8 x 8 and master 7 x 7 quad4 elements on the unit square at z = 0,
 * through upload, workspace, pair search, CSR pattern, integration and the
 * backward pass.  Checked against what the geometry fixes: sum(D) equals the
 * covered area (1), every row of M sums to the same row of D (partition of
 * unity of the master shape functions), the gap of tied meshes is zero,
 * and the gradient of sum(D) vanishes for in-plane motion of interior nodes
 * (the covered area does not change).  Prints "c abi ok" and returns 0 on
 * success. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "mortar_mi355x.h"

#define CHECK(x)                                                           \
  do {                                                                     \
    int rc_ = (x);                                                         \
    if (rc_ != MT_OK) {                                                    \
      fprintf(stderr, "%s -> %d: %s\n", #x, rc_, mt_last_error());         \
      return 1;                                                            \
    }                                                                      \
  } while (0)
#define HCHECK(x)                                                          \
  do {                                                                     \
    hipError_t e_ = (x);                                                   \
    if (e_ != hipSuccess) {                                                \
      fprintf(stderr, "%s -> %s\n", #x, hipGetErrorString(e_));            \
      return 1;                                                            \
    }                                                                      \
  } while (0)

/* n x n quad4 grid of the unit square at z = 0, nodes (i, j) -> j (n + 1) + i */
static void grid(int n, double* x, double* y, double* z, int32_t* conn) {
  for (int j = 0; j <= n; ++j)
    for (int i = 0; i <= n; ++i) {
      const int k = j * (n + 1) + i;
      x[k] = (double)i / n;
      y[k] = (double)j / n;
      z[k] = 0.0;
    }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int32_t* c = conn + 4 * (j * n + i);
      c[0] = j * (n + 1) + i;
      c[1] = c[0] + 1;
      c[2] = c[1] + n + 1;
      c[3] = c[0] + n + 1;
    }
}

static int to_device(void** d, const void* h, size_t bytes) {
  if (hipMalloc(d, bytes < 16 ? 16 : bytes) != hipSuccess) return 1;
  return hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice) != hipSuccess;
}

int main(void) {
  const int n[2] = {8, 7};
  double* X[2][3];
  int32_t* C[2];
  int nn[2], ne[2];
  double* hx[2][3];
  for (int s = 0; s < 2; ++s) {
    nn[s] = (n[s] + 1) * (n[s] + 1);
    ne[s] = n[s] * n[s];
    double* h = (double*)malloc(3 * sizeof(double) * nn[s]);
    int32_t* hc = (int32_t*)malloc(4 * sizeof(int32_t) * ne[s]);
    grid(n[s], h, h + nn[s], h + 2 * nn[s], hc);
    for (int d = 0; d < 3; ++d) {
      hx[s][d] = h + d * nn[s];
      if (to_device((void**)&X[s][d], hx[s][d], sizeof(double) * nn[s])) return 1;
    }
    if (to_device((void**)&C[s], hc, 4 * sizeof(int32_t) * ne[s])) return 1;
    free(hc);
  }

  mt_ctx* ctx = NULL;
  CHECK(mt_create(&ctx, 0));
  mt_params p;
  CHECK(mt_default_params(&p));
  CHECK(mt_set_params(ctx, &p));
  CHECK(mt_upload(ctx, MT_SIDE_SLAVE, nn[0], X[0][0], X[0][1], X[0][2], ne[0], C[0], NULL));
  CHECK(mt_upload(ctx, MT_SIDE_MASTER, nn[1], X[1][0], X[1][1], X[1][2], ne[1], C[1], NULL));

  size_t ws_bytes = 0;
  CHECK(mt_workspace_size(ctx, NULL, &ws_bytes));
  void* ws = NULL;
  HCHECK(hipMalloc(&ws, ws_bytes));  /* hipMalloc memory is 256-byte aligned */
  int64_t n_cand = 0, n_pairs = 0, nnz_D = 0, nnz_M = 0;
  CHECK(mt_build_pairs(ctx, NULL, ws, ws_bytes, &n_cand, &n_pairs, NULL));
  CHECK(mt_csr_pattern(ctx, &nnz_D, &nnz_M, NULL));

  const int ns = nn[0], nm = nn[1];
  double *D, *M, *g, *WD, *WM, *wg, *gXs, *gXm;
  int32_t *Drp, *Dcol, *Mrp, *Mcol;
  HCHECK(hipMalloc((void**)&D, sizeof(double) * nnz_D));
  HCHECK(hipMalloc((void**)&M, sizeof(double) * nnz_M));
  HCHECK(hipMalloc((void**)&g, sizeof(double) * ns));
  HCHECK(hipMalloc((void**)&Drp, sizeof(int32_t) * (ns + 1)));
  HCHECK(hipMalloc((void**)&Mrp, sizeof(int32_t) * (ns + 1)));
  HCHECK(hipMalloc((void**)&Dcol, sizeof(int32_t) * nnz_D));
  HCHECK(hipMalloc((void**)&Mcol, sizeof(int32_t) * nnz_M));
  CHECK(mt_get_csr(ctx, Drp, Dcol, Mrp, Mcol, NULL));
  CHECK(mt_integrate(ctx, D, M, g, NULL));

  /* weights of L = sum(D): W_D = 1, W_M = 0, w_g = 0 */
  double* h1 = (double*)malloc(sizeof(double) * (nnz_D > ns ? nnz_D : ns));
  double* h0 = (double*)calloc((size_t)(nnz_M > ns ? nnz_M : ns), sizeof(double));
  for (int64_t i = 0; i < nnz_D; ++i) h1[i] = 1.0;
  if (to_device((void**)&WD, h1, sizeof(double) * nnz_D)) return 1;
  if (to_device((void**)&WM, h0, sizeof(double) * nnz_M)) return 1;
  if (to_device((void**)&wg, h0, sizeof(double) * ns)) return 1;
  HCHECK(hipMalloc((void**)&gXs, 3 * sizeof(double) * ns));
  HCHECK(hipMalloc((void**)&gXm, 3 * sizeof(double) * nm));
  CHECK(mt_backward(ctx, WD, WM, wg, gXs, gXm, NULL));
  HCHECK(hipDeviceSynchronize());
  CHECK(mt_check(ctx));

  double* hD = (double*)malloc(sizeof(double) * nnz_D);
  double* hM = (double*)malloc(sizeof(double) * nnz_M);
  double* hg = (double*)malloc(sizeof(double) * ns);
  double* hgs = (double*)malloc(3 * sizeof(double) * ns);
  double* hgm = (double*)malloc(3 * sizeof(double) * nm);
  int32_t* hDrp = (int32_t*)malloc(sizeof(int32_t) * (ns + 1));
  int32_t* hMrp = (int32_t*)malloc(sizeof(int32_t) * (ns + 1));
  HCHECK(hipMemcpy(hD, D, sizeof(double) * nnz_D, hipMemcpyDeviceToHost));
  HCHECK(hipMemcpy(hM, M, sizeof(double) * nnz_M, hipMemcpyDeviceToHost));
  HCHECK(hipMemcpy(hg, g, sizeof(double) * ns, hipMemcpyDeviceToHost));
  HCHECK(hipMemcpy(hgs, gXs, 3 * sizeof(double) * ns, hipMemcpyDeviceToHost));
  HCHECK(hipMemcpy(hgm, gXm, 3 * sizeof(double) * nm, hipMemcpyDeviceToHost));
  HCHECK(hipMemcpy(hDrp, Drp, sizeof(int32_t) * (ns + 1), hipMemcpyDeviceToHost));
  HCHECK(hipMemcpy(hMrp, Mrp, sizeof(int32_t) * (ns + 1), hipMemcpyDeviceToHost));

  int bad = 0;
  double sumD = 0.0, worst_row = 0.0, worst_gap = 0.0, worst_grad = 0.0;
  for (int i = 0; i < ns; ++i) {
    double rd = 0.0, rm = 0.0;
    for (int k = hDrp[i]; k < hDrp[i + 1]; ++k) rd += hD[k];
    for (int k = hMrp[i]; k < hMrp[i + 1]; ++k) rm += hM[k];
    sumD += rd;
    worst_row = fmax(worst_row, fabs(rd - rm));
    worst_gap = fmax(worst_gap, fabs(hg[i]));
  }
  /* in-plane gradient components of interior nodes, both sides */
  for (int s = 0; s < 2; ++s) {
    const int m = n[s], nodes = nn[s];
    const double* gx = s ? hgm : hgs;
    for (int j = 1; j < m; ++j)
      for (int i = 1; i < m; ++i) {
        const int k = j * (m + 1) + i;
        worst_grad = fmax(worst_grad, fmax(fabs(gx[k]), fabs(gx[nodes + k])));
      }
  }
  if (n_pairs <= 0 || nnz_D <= 0 || nnz_M <= 0) bad = 1;
  if (fabs(sumD - 1.0) > 1e-13) bad = 1;
  if (worst_row > 1e-14) bad = 1;
  if (worst_gap > 1e-15) bad = 1;
  if (worst_grad > 1e-13) bad = 1;
  printf("pairs %lld candidates %lld nnz(D) %lld nnz(M) %lld sum(D) %.17g |rowD-rowM| %.3g |gap| %.3g "
         "|grad in plane| %.3g\n",
         (long long)n_pairs, (long long)n_cand, (long long)nnz_D, (long long)nnz_M, sumD, worst_row, worst_gap,
         worst_grad);
  CHECK(mt_destroy(ctx));
  if (bad) {
    printf("c abi FAILED\n");
    return 1;
  }
  printf("c abi ok\n");
  return 0;
}
