// Row-owner device functions of the deterministic assembly: one thread owns
// one output row (slave node) or one node's gradient and adds its
// contributions in a fixed order (incident elements ascending, then pairs in
// (slave, master) order).  Shared by the single-interface and batched kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mt {

// The pairs that one node's row gathers, as one flat sequence k = 0 .. n-1:
// the pairs of its incident elements (ascending), each element's pairs in
// their order.  Up to four incident elements are held in registers, so the
// loads of several consecutive pairs can be issued before any of them is
// added; the additions still run in the sequence order, so the sums are the
// same bit for bit as those of the plain nested loops (used for nodes with
// more than four elements).
constexpr int ROW_RUNS = 4;

struct RowRuns {
  int e[ROW_RUNS];   // incident element
  int j[ROW_RUNS];   // local index of the node in it
  int p0[ROW_RUNS];  // first pair (or pair position) of the element
  int c1, c2, c3;    // flat index at which elements 1, 2, 3 start
  int n;             // number of pairs in all
};

// Runs of the ni <= ROW_RUNS incidences inc_list[i0 ..]; element e's pairs
// are lo[e] .. hi[e] - 1.
__device__ __forceinline__ void load_runs(int i0, int ni, const int32_t* __restrict__ inc_list,
                                          const int32_t* __restrict__ lo, const int32_t* __restrict__ hi,
                                          RowRuns& R) {
  int l[ROW_RUNS], h[ROW_RUNS];
#pragma unroll
  for (int t = 0; t < ROW_RUNS; ++t) {
    const int v = t < ni ? inc_list[i0 + t] : 0;
    R.e[t] = v >> 2;
    R.j[t] = v & 3;
  }
#pragma unroll
  for (int t = 0; t < ROW_RUNS; ++t) {
    l[t] = t < ni ? lo[R.e[t]] : 0;
    h[t] = t < ni ? hi[R.e[t]] : 0;
    R.p0[t] = l[t];
  }
  R.c1 = h[0] - l[0];
  R.c2 = R.c1 + (h[1] - l[1]);
  R.c3 = R.c2 + (h[2] - l[2]);
  R.n = R.c3 + (h[3] - l[3]);
}

// Local index j and pair p of flat position k (0 <= k < n); empty elements
// are skipped because their start equals the next one's.
__device__ __forceinline__ int run_at(const RowRuns& R, int k, int& j) {
  int base = 0, p0 = R.p0[0];
  j = R.j[0];
  if (k >= R.c1) { base = R.c1; p0 = R.p0[1]; j = R.j[1]; }
  if (k >= R.c2) { base = R.c2; p0 = R.p0[2]; j = R.j[2]; }
  if (k >= R.c3) { base = R.c3; p0 = R.p0[3]; j = R.j[3]; }
  return p0 + (k - base);
}

// pairs whose loads the gradient gathers issue together
constexpr int ROW_BATCH = 8;

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

// One sweep over the pairs of row a (incident elements ascending, then their
// pairs), adding the D part (DP: entry q at acc[(q - d0) * astride], and the
// gap, returned) and/or the M part (MP: entry q at acc[(q + moff) * astride]).
template <bool DP, bool MP>
__device__ __forceinline__ double row_sweep(int a, const int32_t* __restrict__ inc_off,
                                            const int32_t* __restrict__ inc_list,
                                            const int32_t* __restrict__ pair_off, int d0, int moff,
                                            const int32_t* __restrict__ posD, int32_t n_s_el,
                                            const int32_t* __restrict__ posM, const double* __restrict__ blk,
                                            int64_t stride, double* acc, int astride) {
  double g = 0.0;
  for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
    const int e = inc_list[i] >> 2, j = inc_list[i] & 3;
    const int p0 = pair_off[e], p1 = pair_off[e + 1];
    if (p0 == p1) continue;
    int pd[4];
    if (DP) {
#pragma unroll
      for (int k = 0; k < 4; ++k) pd[k] = posD[(int64_t)(j * 4 + k) * n_s_el + e] - d0;
    }
    for (int p = p0; p < p1; ++p) {
      double vd[4], vm[4];
      int pm[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (DP) vd[k] = blk[(int64_t)(j * 4 + k) * stride + p];
        if (MP) {
          vm[k] = blk[(int64_t)(16 + j * 4 + k) * stride + p];
          pm[k] = posM[(int64_t)(j * 4 + k) * stride + p] + moff;
        }
      }
      if (DP) g += blk[(int64_t)(32 + j) * stride + p];
      if (DP) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[pd[k] * astride] += vd[k];
      }
      if (MP) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[pm[k] * astride] += vm[k];
      }
    }
  }
  return g;
}

// Same as assemble_row, accumulating the row in a per-thread scratch segment
// of cap entries, acc[i * astride], and writing it once: D and M entries
// together in one sweep when they fit, else in two sweeps (D with the gap,
// then M) when each part fits; longer rows fall back to assemble_row.  Every
// entry receives its contributions in the same order in all three forms.
// (Issuing the loads of several pairs together, as the gradient gathers
// below do, measured slower here: the row's LDS updates, not its loads, set
// the pace.)
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
  double g;
  if (nd + nm <= cap) {
    for (int i = 0; i < nd + nm; ++i) acc[i * astride] = 0.0;
    g = row_sweep<true, true>(a, inc_off, inc_list, pair_off, d0, nd - m0, posD, n_s_el, posM, blk, stride, acc,
                              astride);
    for (int i = 0; i < nd; ++i) D_val[d0 + i] = acc[i * astride];
    for (int i = 0; i < nm; ++i) M_val[m0 + i] = acc[(nd + i) * astride];
  } else if (nd <= cap && nm <= cap) {
    for (int i = 0; i < nd; ++i) acc[i * astride] = 0.0;
    g = row_sweep<true, false>(a, inc_off, inc_list, pair_off, d0, 0, posD, n_s_el, posM, blk, stride, acc,
                               astride);
    for (int i = 0; i < nd; ++i) D_val[d0 + i] = acc[i * astride];
    for (int i = 0; i < nm; ++i) acc[i * astride] = 0.0;
    row_sweep<false, true>(a, inc_off, inc_list, pair_off, d0, -m0, posD, n_s_el, posM, blk, stride, acc, astride);
    for (int i = 0; i < nm; ++i) M_val[m0 + i] = acc[i * astride];
  } else {
    assemble_row(a, inc_off, inc_list, pair_off, D_rowptr, M_rowptr, posD, n_s_el, posM, blk, stride, D_val, M_val,
                 gap);
    return;
  }
  gap[a] = g;
}

// Sum over the flat pair sequence of R of the three components
// gpair[(c0 + 3 j + d) * stride + p], d = 0, 1, 2, in sequence order.
__device__ __forceinline__ void gather3(const RowRuns& R, int c0, const double* __restrict__ gpair, int64_t stride,
                                        double& g0, double& g1, double& g2) {
  constexpr int U = ROW_BATCH;
  for (int k0 = 0; k0 < R.n; k0 += U) {
    double v[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // positions past the end reload the last pair and are not added
      int j;
      const int p = run_at(R, min(k0 + u, R.n - 1), j);
#pragma unroll
      for (int d = 0; d < 3; ++d) v[u][d] = gpair[(int64_t)(c0 + 3 * j + d) * stride + p];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (k0 + u < R.n) {
        g0 += v[u][0];
        g1 += v[u][1];
        g2 += v[u][2];
      }
    }
  }
}

// Gradient of slave node a (structure-of-arrays gX[3 * n]).
__device__ __forceinline__ void grad_slave_row(int a, int32_t n, const int32_t* __restrict__ inc_off,
                                               const int32_t* __restrict__ inc_list,
                                               const int32_t* __restrict__ pair_off,
                                               const double* __restrict__ gpair, int64_t stride,
                                               double* __restrict__ gX) {
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  const int i0 = inc_off[a], ni = inc_off[a + 1] - i0;
  if (ni <= ROW_RUNS) {
    RowRuns R;
    load_runs(i0, ni, inc_list, pair_off, pair_off + 1, R);
    gather3(R, 0, gpair, stride, g0, g1, g2);
  } else {
    for (int i = i0; i < i0 + ni; ++i) {
      const int e = inc_list[i] >> 2, j = inc_list[i] & 3;
      for (int p = pair_off[e]; p < pair_off[e + 1]; ++p) {
        g0 += gpair[(int64_t)(3 * j + 0) * stride + p];
        g1 += gpair[(int64_t)(3 * j + 1) * stride + p];
        g2 += gpair[(int64_t)(3 * j + 2) * stride + p];
      }
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
  const int i0 = inc_off[b], ni = inc_off[b + 1] - i0;
  if (ni <= ROW_RUNS) {
    RowRuns R;
    load_runs(i0, ni, inc_list, mstart, mend, R);
    gather3(R, 12, gpair, stride, g0, g1, g2);
  } else {
    for (int i = i0; i < i0 + ni; ++i) {
      const int m = inc_list[i] >> 2, l = inc_list[i] & 3;
      for (int k = mstart[m]; k < mend[m]; ++k) {
        g0 += gpair[(int64_t)(12 + 3 * l + 0) * stride + k];
        g1 += gpair[(int64_t)(12 + 3 * l + 1) * stride + k];
        g2 += gpair[(int64_t)(12 + 3 * l + 2) * stride + k];
      }
    }
  }
  gX[b] = g0;
  gX[(int64_t)n + b] = g1;
  gX[2 * (int64_t)n + b] = g2;
}

}  // namespace mt
