// Gradient through the dual basis coefficients of a slave element (shared by
// the single-interface and the batched backward).
#pragma once

#include "mt_pair_eval.h"

namespace mt {

// Dependence of the dual coefficients on the slave nodes, for one slave
// element.  Its dual blocks are A times the standard ones, A = diag(De)
// Me^-1 (2x2 Gauss on the projected slave quad), so the loss
// L = sum over the element's pairs of <WD, D> + <WM, M> + <wg, g> has
// Abar = G A^-T with G = sum_pairs (WD D^T + WM M^T + wg g^T) over the dual
// blocks; with A^-T = diag(1/De) Me this gives Abar Me^-1 = G diag(1/De),
// Debar_j = G_jj / De_j and Mebar_jk = -(sum_m Me^-1_jm De_m G_mk) / De_k,
// then through the Jacobian determinants at the Gauss points to the projected
// slave nodes, and through the projection and the frame to the slave
// coordinates (added to Xsb) and, with the continuous normal field (ns), to
// the element's plane normal (added to n0b).
__device__ __forceinline__ void dual_adjoint(const double Xs[4][3], const double* ns, const double G[16],
                                             double Xsb[4][3], double n0b[3]) {
#pragma clang fp contract(fast)
  double f[12];
  slave_frame_p(Xs, ns, f);
  V2 S[4];
  double hs[4], As, hmax;
  slave_setup(Xs, f, S, hs, As, hmax);
  // forward of the coefficients
  const double gp = 0.5773502691896257;
  double Me[16], De[4];
#pragma unroll
  for (int i = 0; i < 16; ++i) Me[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) De[i] = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double x1 = a ? gp : -gp, x2 = b ? gp : -gp;
      double N[4];
      shape4(x1, x2, N);
      const double d1[4] = {-0.25 * (1.0 - x2), 0.25 * (1.0 - x2), 0.25 * (1.0 + x2), -0.25 * (1.0 + x2)};
      const double d2[4] = {-0.25 * (1.0 - x1), -0.25 * (1.0 + x1), 0.25 * (1.0 + x1), 0.25 * (1.0 - x1)};
      double j00 = 0, j01 = 0, j10 = 0, j11 = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        j00 += d1[k] * S[k].u; j01 += d2[k] * S[k].u;
        j10 += d1[k] * S[k].v; j11 += d2[k] * S[k].v;
      }
      const double det = j00 * j11 - j01 * j10;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        De[j] += N[j] * det;
#pragma unroll
        for (int k = 0; k < 4; ++k) Me[j * 4 + k] += N[j] * N[k] * det;
      }
    }
  double inv[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) inv[i] = (i % 5 == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double r = 1.0 / Me[c * 4 + c];
#pragma unroll
    for (int k = 0; k < 4; ++k) { Me[c * 4 + k] *= r; inv[c * 4 + k] *= r; }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      if (rr == c) continue;
      const double fct = Me[rr * 4 + c];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Me[rr * 4 + k] -= fct * Me[c * 4 + k];
        inv[rr * 4 + k] -= fct * inv[c * 4 + k];
      }
    }
  }
  double rDe[4], Mb[16], Db[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) rDe[j] = 1.0 / De[j];
#pragma unroll
  for (int j = 0; j < 4; ++j) Db[j] = G[5 * j] * rDe[j];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double a = 0.0;
#pragma unroll
      for (int m = 0; m < 4; ++m) a += inv[4 * j + m] * De[m] * G[4 * m + k];
      Mb[4 * j + k] = -a * rDe[k];
    }
  // to the projected slave nodes through det J at the Gauss points
  double ub[4] = {0, 0, 0, 0}, vb[4] = {0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double x1 = a ? gp : -gp, x2 = b ? gp : -gp;
      double N[4];
      shape4(x1, x2, N);
      const double d1[4] = {-0.25 * (1.0 - x2), 0.25 * (1.0 - x2), 0.25 * (1.0 + x2), -0.25 * (1.0 + x2)};
      const double d2[4] = {-0.25 * (1.0 - x1), -0.25 * (1.0 + x1), 0.25 * (1.0 + x1), 0.25 * (1.0 - x1)};
      double j00 = 0, j01 = 0, j10 = 0, j11 = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        j00 += d1[k] * S[k].u; j01 += d2[k] * S[k].u;
        j10 += d1[k] * S[k].v; j11 += d2[k] * S[k].v;
      }
      double detb = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double t = Db[j];
#pragma unroll
        for (int k = 0; k < 4; ++k) t += Mb[4 * j + k] * N[k];
        detb += N[j] * t;
      }
      const double jb00 = detb * j11, jb11 = detb * j00, jb01 = -detb * j10, jb10 = -detb * j01;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ub[k] += jb00 * d1[k] + jb01 * d2[k];
        vb[k] += jb10 * d1[k] + jb11 * d2[k];
      }
    }
  double nb[8][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    nb[k][0] = ub[k];
    nb[k][1] = vb[k];
    nb[k][2] = 0.0;
    nb[4 + k][0] = nb[4 + k][1] = nb[4 + k][2] = 0.0;
  }
  double gsb[4][3], gmb[4][3];
  projection_adjoint(Xs, Xs, ns, nb, gsb, gmb, n0b);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) Xsb[k][d] += gsb[k][d];
}

// G = WD D^T + WM M^T + wg g^T of pair p from its dual blocks blk[c * stride + p].
__device__ __forceinline__ void dual_gram(const double WD[16], const double WM[16], const double wg[4],
                                          const double* __restrict__ blk, int64_t stride, int64_t p, double G[16]) {
#pragma clang fp contract(fast)
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      double a = wg[j] * blk[(int64_t)(32 + m) * stride + p];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        a += WD[4 * j + k] * blk[(int64_t)(4 * m + k) * stride + p] + WM[4 * j + k] * blk[(int64_t)(16 + 4 * m + k) * stride + p];
      G[4 * j + m] = a;
    }
}

// The dual-coefficient part of pair p's gradient, written to the slave
// slots of gpair[c * stride + p] (and, with the continuous normal field, the
// plane-normal part to gn0[d * stride + p]); the sweep adds its own terms
// there afterwards.  WD, WM, wg = the pair's upstream weights.
template <bool NODAL>
__device__ __forceinline__ void pair_dual_adjoint(const MeshPtrs& S, int s, int4 csn, const double WD[16],
                                                  const double WM[16], const double wg[4],
                                                  const double* __restrict__ blk, int64_t stride, int64_t p,
                                                  double* __restrict__ gpair, double* __restrict__ gn0) {
  double G[16];
  dual_gram(WD, WM, wg, blk, stride, p, G);
  double Xs[4][3], Xd[4][3];
  load_nodes(S.x, S.y, S.z, csn, Xs);
#pragma unroll
  for (int k = 0; k < 4; ++k) Xd[k][0] = Xd[k][1] = Xd[k][2] = 0.0;
  double n0d[3] = {0.0, 0.0, 0.0};
  dual_adjoint(Xs, NODAL ? elem_nrm(S, s) : nullptr, G, Xd, n0d);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) gpair[(int64_t)(3 * k + d) * stride + p] = Xd[k][d];
  if (NODAL)
#pragma unroll
    for (int d = 0; d < 3; ++d) gn0[(int64_t)d * stride + p] = n0d[d];
}

}  // namespace mt
