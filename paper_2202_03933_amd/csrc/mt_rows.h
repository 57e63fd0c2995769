// Row-owner device functions of the deterministic assembly: one thread owns
// one output row (slave node) or one node's gradient and adds its
// contributions in a fixed order (incident elements ascending, then pairs in
// (slave, master) order).  Shared by the single-interface and batched kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mt {

// Row a of D, M and the gap from the staged local blocks blk[c * stride + p].
__device__ __forceinline__ void assemble_row(int a, const int32_t* __restrict__ inc_off,
                                             const int32_t* __restrict__ inc_list,
                                             const int32_t* __restrict__ pair_off,
                                             const int32_t* __restrict__ D_rowptr,
                                             const int32_t* __restrict__ M_rowptr,
                                             const int32_t* __restrict__ posD, int32_t n_s_el,
                                             const int32_t* __restrict__ posM, const double* __restrict__ blk,
                                             int64_t stride, double* __restrict__ D_val, double* __restrict__ M_val,
                                             double* __restrict__ gap) {
  for (int i = D_rowptr[a]; i < D_rowptr[a + 1]; ++i) D_val[i] = 0.0;
  for (int i = M_rowptr[a]; i < M_rowptr[a + 1]; ++i) M_val[i] = 0.0;
  double g = 0.0;
  for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
    const int e = inc_list[i] >> 2, j = inc_list[i] & 3;
    const int p0 = pair_off[e], p1 = pair_off[e + 1];
    if (p0 == p1) continue;
    int pd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pd[k] = posD[(int64_t)(j * 4 + k) * n_s_el + e];
    for (int p = p0; p < p1; ++p) {
#pragma unroll
      for (int k = 0; k < 4; ++k) D_val[pd[k]] += blk[(int64_t)(j * 4 + k) * stride + p];
#pragma unroll
      for (int l = 0; l < 4; ++l)
        M_val[posM[(int64_t)(j * 4 + l) * stride + p]] += blk[(int64_t)(16 + j * 4 + l) * stride + p];
      g += blk[(int64_t)(32 + j) * stride + p];
    }
  }
  gap[a] = g;
}

// Same as assemble_row, accumulating the row in a per-thread scratch segment
// acc[i * stride] (D entries first, then M) and writing it once; rows longer
// than cap entries fall back to assemble_row.
__device__ __forceinline__ void assemble_row_acc(int a, const int32_t* __restrict__ inc_off,
                                                 const int32_t* __restrict__ inc_list,
                                                 const int32_t* __restrict__ pair_off,
                                                 const int32_t* __restrict__ D_rowptr,
                                                 const int32_t* __restrict__ M_rowptr,
                                                 const int32_t* __restrict__ posD, int32_t n_s_el,
                                                 const int32_t* __restrict__ posM, const double* __restrict__ blk,
                                                 int64_t stride, double* __restrict__ D_val,
                                                 double* __restrict__ M_val, double* __restrict__ gap, double* acc,
                                                 int astride, int cap) {
  const int d0 = D_rowptr[a], d1 = D_rowptr[a + 1];
  const int m0 = M_rowptr[a], m1 = M_rowptr[a + 1];
  const int nd = d1 - d0, nm = m1 - m0;
  if (nd + nm > cap) {
    assemble_row(a, inc_off, inc_list, pair_off, D_rowptr, M_rowptr, posD, n_s_el, posM, blk, stride, D_val, M_val,
                 gap);
    return;
  }
  for (int i = 0; i < nd + nm; ++i) acc[i * astride] = 0.0;
  double g = 0.0;
  const int moff = nd - m0;  // M position q accumulates at acc[(q + moff) * astride]
  for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
    const int e = inc_list[i] >> 2, j = inc_list[i] & 3;
    const int p0 = pair_off[e], p1 = pair_off[e + 1];
    if (p0 == p1) continue;
    int pd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pd[k] = posD[(int64_t)(j * 4 + k) * n_s_el + e] - d0;
    for (int p = p0; p < p1; ++p) {
      double vd[4], vm[4];
      int pm[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        vd[k] = blk[(int64_t)(j * 4 + k) * stride + p];
        vm[k] = blk[(int64_t)(16 + j * 4 + k) * stride + p];
        pm[k] = posM[(int64_t)(j * 4 + k) * stride + p] + moff;
      }
      g += blk[(int64_t)(32 + j) * stride + p];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[pd[k] * astride] += vd[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[pm[k] * astride] += vm[k];
    }
  }
  for (int i = 0; i < nd; ++i) D_val[d0 + i] = acc[i * astride];
  for (int i = 0; i < nm; ++i) M_val[m0 + i] = acc[(nd + i) * astride];
  gap[a] = g;
}

// Gradient of slave node a (structure-of-arrays gX[3 * n]).
__device__ __forceinline__ void grad_slave_row(int a, int32_t n, const int32_t* __restrict__ inc_off,
                                               const int32_t* __restrict__ inc_list,
                                               const int32_t* __restrict__ pair_off,
                                               const double* __restrict__ gpair, int64_t stride,
                                               double* __restrict__ gX) {
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
    const int e = inc_list[i] >> 2, j = inc_list[i] & 3;
    for (int p = pair_off[e]; p < pair_off[e + 1]; ++p) {
      g0 += gpair[(int64_t)(3 * j + 0) * stride + p];
      g1 += gpair[(int64_t)(3 * j + 1) * stride + p];
      g2 += gpair[(int64_t)(3 * j + 2) * stride + p];
    }
  }
  gX[a] = g0;
  gX[(int64_t)n + a] = g1;
  gX[2 * (int64_t)n + a] = g2;
}

// Gradient of master node b: the master components of the pairs are staged
// in pairs-by-master order (position k of pair p = its rank in that order),
// so the pairs of master element m are the contiguous range
// mstart[m] .. mend[m].
__device__ __forceinline__ void grad_master_row(int b, int32_t n, const int32_t* __restrict__ inc_off,
                                                const int32_t* __restrict__ inc_list,
                                                const int32_t* __restrict__ mstart, const int32_t* __restrict__ mend,
                                                const double* __restrict__ gpair, int64_t stride,
                                                double* __restrict__ gX) {
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int i = inc_off[b]; i < inc_off[b + 1]; ++i) {
    const int m = inc_list[i] >> 2, l = inc_list[i] & 3;
    for (int k = mstart[m]; k < mend[m]; ++k) {
      g0 += gpair[(int64_t)(12 + 3 * l + 0) * stride + k];
      g1 += gpair[(int64_t)(12 + 3 * l + 1) * stride + k];
      g2 += gpair[(int64_t)(12 + 3 * l + 2) * stride + k];
    }
  }
  gX[b] = g0;
  gX[(int64_t)n + b] = g1;
  gX[2 * (int64_t)n + b] = g2;
}

}  // namespace mt
