// Evaluation of one (slave, master) element pair, forward and backward, as
// device functions shared by the single-interface kernels and the persistent
// batched kernels.  The triangle rule (3 or 7 points) and the basis (standard
// or dual) are template parameters, so rule points fold into constants.
#pragma once

#include "mt_geometry.h"
#include "mt_internal.h"

namespace mt {

// Triangle rules as (l0, l1, l2, w) rows, barycentric coordinates with
// weights summing to one: 7 points of degree 5 (Radon's rule) and 3 points of
// degree 2 (the rule of Fig. 1).  The point index is uniform across a
// wavefront, so reads are scalar constant-cache loads.
__constant__ double c_rule7[7][4] = {
    {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 9.0 / 40.0},
    {0.7974269853530873, 0.10128650732345634, 0.10128650732345634, 0.12593918054482714},
    {0.10128650732345634, 0.7974269853530873, 0.10128650732345634, 0.12593918054482714},
    {0.10128650732345634, 0.10128650732345634, 0.7974269853530873, 0.12593918054482714},
    {0.05971587178976982, 0.4701420641051151, 0.4701420641051151, 0.1323941527885062},
    {0.4701420641051151, 0.05971587178976982, 0.4701420641051151, 0.1323941527885062},
    {0.4701420641051151, 0.4701420641051151, 0.05971587178976982, 0.1323941527885062}};
__constant__ double c_rule3[3][4] = {{2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 3.0},
                                     {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0, 1.0 / 3.0},
                                     {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0, 1.0 / 3.0}};

template <int NQ>
__device__ __forceinline__ void rule_point(int q, double& l0, double& l1, double& l2, double& w) {
  const double* r = NQ == 3 ? c_rule3[q] : c_rule7[q];
  l0 = r[0];
  l1 = r[1];
  l2 = r[2];
  w = r[3];
}

// Forward: projection, clip, cleanup, fan triangulation and quadrature of the
// local blocks
//   D[j][k] = sum w A_t Phi_j N_k(xi),  M[j][l] = sum w A_t Phi_j N_l(eta),
//   g[j]    = sum w A_t Phi_j (sum_l N_l(eta) hm_l - sum_k N_k(xi) hs_k).
// Returns the clip vertex count (0: not a pair, blocks zero).
template <int NQ, bool DUAL, bool LAB>
__device__ __forceinline__ int pair_forward(const double Xs[4][3], const double Xm[4][3], const KParams& kp,
                                            const LdsPoly<LAB>& P, double D[16], double M[16], double g[4],
                                            unsigned& noconv) {
  double f[12];
  slave_frame(Xs, f);
  V2 S[4], Mn[4];
  double hs[4], hm[4];
  int res, st;
  bool flip;
  const int n = pair_geometry<LAB>(Xs, Xm, f, kp.eps_d, kp.eps_a, S, Mn, hs, hm, flip, P, res, st);
#pragma unroll
  for (int k = 0; k < 16; ++k) { D[k] = 0.0; M[k] = 0.0; }
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = 0.0;
  double A[16];
  if (DUAL) dual_coefficients(S, A);
  {
#pragma clang fp contract(fast)
  const double u0 = P.u[P.at(res, 0)], v0 = P.v[P.at(res, 0)];
  for (int i = 1; i + 1 < n; ++i) {
    const double u1 = P.u[P.at(res, i)], v1 = P.v[P.at(res, i)];
    const double u2 = P.u[P.at(res, i + 1)], v2 = P.v[P.at(res, i + 1)];
    const double At = 0.5 * ((u1 - u0) * (v2 - v0) - (v1 - v0) * (u2 - u0));
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      double l0, l1, l2, w;
      rule_point<NQ>(q, l0, l1, l2, w);
      const double pu = l0 * u0 + l1 * u1 + l2 * u2;
      const double pv = l0 * v0 + l1 * v1 + l2 * v2;
      const double wA = w * At;
      double a1, a2, b1, b2;
      if (!inverse_bilinear(S, pu, pv, kp.newton_tol, kp.newton_maxit, a1, a2)) ++noconv;
      if (!inverse_bilinear(Mn, pu, pv, kp.newton_tol, kp.newton_maxit, b1, b2)) ++noconv;
      double Ns[4], Nm[4];
      shape4(a1, a2, Ns);
      shape4(b1, b2, Nm);
      double Phi[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        Phi[j] = DUAL ? A[j * 4 + 0] * Ns[0] + A[j * 4 + 1] * Ns[1] + A[j * 4 + 2] * Ns[2] + A[j * 4 + 3] * Ns[3]
                      : Ns[j];
      const double gap = (Nm[0] * hm[0] + Nm[1] * hm[1] + Nm[2] * hm[2] + Nm[3] * hm[3]) -
                         (Ns[0] * hs[0] + Ns[1] * hs[1] + Ns[2] * hs[2] + Ns[3] * hs[3]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double wp = wA * Phi[j];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          D[j * 4 + k] += wp * Ns[k];
          M[j * 4 + k] += wp * Nm[k];
        }
        g[j] += wp * gap;
      }
    }
  }
  }
  return n;
}

// ---- backward ----------------------------------------------------------------

struct Map2 {
  double e1u, e1v, e2u, e2v, fu, fv;
};

__device__ __forceinline__ Map2 bilinear_map(const V2 X[4]) {
  Map2 m;
  m.e1u = 0.25 * ((X[1].u - X[0].u) + (X[2].u - X[3].u));
  m.e1v = 0.25 * ((X[1].v - X[0].v) + (X[2].v - X[3].v));
  m.e2u = 0.25 * ((X[2].u - X[1].u) + (X[3].u - X[0].u));
  m.e2v = 0.25 * ((X[2].v - X[1].v) + (X[3].v - X[0].v));
  m.fu = 0.25 * ((X[0].u - X[1].u) + (X[2].u - X[3].u));
  m.fv = 0.25 * ((X[0].v - X[1].v) + (X[2].v - X[3].v));
  return m;
}

// Reverse of xi = inverse map at point p: given xibar returns
// lambda = J^-T xibar (then pbar += lambda, Xbar_k -= N_k lambda).
__device__ __forceinline__ void ift_adjoint(const Map2& m, double x1, double x2, double xb1, double xb2, double& l0,
                                            double& l1) {
#pragma clang fp contract(fast)
  const double j00 = m.e1u + m.fu * x2, j01 = m.e2u + m.fu * x1;
  const double j10 = m.e1v + m.fv * x2, j11 = m.e2v + m.fv * x1;
  const double rdet = 1.0 / (j00 * j11 - j01 * j10);
  l0 = (j11 * xb1 - j10 * xb2) * rdet;
  l1 = (j00 * xb2 - j01 * xb1) * rdet;
}

__device__ __forceinline__ void shape_grad(double x1, double x2, double d1[4], double d2[4]) {
#pragma clang fp contract(fast)
  d1[0] = -0.25 * (1.0 - x2); d1[1] = 0.25 * (1.0 - x2); d1[2] = 0.25 * (1.0 + x2); d1[3] = -0.25 * (1.0 + x2);
  d2[0] = -0.25 * (1.0 - x1); d2[1] = -0.25 * (1.0 + x1); d2[2] = 0.25 * (1.0 + x1); d2[3] = 0.25 * (1.0 - x1);
}

// Adjoint of the intersection X of line A (A1 -> A2) and line B (B1 -> B2):
// X = A1 + s (A2 - A1), s = cross(B1 - A1, dB) / cross(dA, dB).  Parallel
// lines (no defined intersection) contribute nothing.
__device__ __forceinline__ void intersect_adjoint(V2 A1, V2 A2, V2 B1, V2 B2, double xu, double xv, V2& a1, V2& a2,
                                                  V2& b1, V2& b2) {
#pragma clang fp contract(fast)
  const double dAu = A2.u - A1.u, dAv = A2.v - A1.v;
  const double dBu = B2.u - B1.u, dBv = B2.v - B1.v;
  const double wu = B1.u - A1.u, wv = B1.v - A1.v;
  const double den = dAu * dBv - dAv * dBu;
  const double scale = (fabs(dAu) + fabs(dAv)) * (fabs(dBu) + fabs(dBv));
  a1 = a2 = b1 = b2 = V2{0.0, 0.0};
  if (!(fabs(den) > 1e-14 * scale)) return;
  const double num = wu * dBv - wv * dBu;
  const double s = num / den;
  double dAbu = s * xu, dAbv = s * xv;
  const double sb = xu * dAu + xv * dAv;
  const double numb = sb / den;
  const double denb = -sb * s / den;
  const double wbu = numb * dBv, wbv = -numb * dBu;
  double dBbu = -numb * wv, dBbv = numb * wu;
  dAbu += denb * dBv;
  dAbv += -denb * dBu;
  dBbu += -denb * dAv;
  dBbv += denb * dAu;
  b1.u = wbu - dBbu;
  b1.v = wbv - dBbv;
  a1.u = xu - wbu - dAbu;
  a1.v = xv - wbv - dAbv;
  a2.u = dAbu;
  a2.v = dAbv;
  b2.u = dBbu;
  b2.v = dBbv;
}

// Backward of one pair (standard basis): gradient of
// L = sum WD[j][k] D[j][k] + sum WM[j][l] M[j][l] + sum wg[j] g[j]
// with respect to the slave (Xsb) and master (Xmb) nodal coordinates.  The
// clip is recomputed with vertex provenance; reverse mode runs through the
// quadrature, the inverse maps (implicit-function derivative), the clip
// vertices (line intersections), the projection and the slave frame.
// Vertex adjoints of the clip polygon live in a per-lane LDS slot array
// (au, av: CAP0 lane-interleaved entries, lane stride P.bs).
template <int NQ>
__device__ __forceinline__ void pair_backward(const double Xs[4][3], const double Xm[4][3], const KParams& kp,
                                              const LdsPoly<true>& P, double* au, double* av,
                                              const double WD[16], const double WM[16],
                                              const double wg[4], double Xsb[4][3], double Xmb[4][3],
                                              unsigned& noconv) {
  double f[12];
  slave_frame(Xs, f);
  V2 S[4], Mn[4];
  double hs[4], hm[4];
  int res, st;
  bool flip;
  const int n = pair_geometry<true>(Xs, Xm, f, kp.eps_d, kp.eps_a, S, Mn, hs, hm, flip, P, res, st);

  V2 Sb[4], Mb[4];
  double hsb[4], hmb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Sb[k] = V2{0.0, 0.0};
    Mb[k] = V2{0.0, 0.0};
    hsb[k] = 0.0;
    hmb[k] = 0.0;
  }
  const int bs = P.bs;
  for (int i = 0; i < n; ++i) {
    au[i * bs] = 0.0;
    av[i * bs] = 0.0;
  }
  const Map2 ms = bilinear_map(S), mm = bilinear_map(Mn);
  {
#pragma clang fp contract(fast)
    const double u0 = P.u[P.at(res, 0)], v0 = P.v[P.at(res, 0)];
    for (int i = 1; i + 1 < n; ++i) {
      const double u1 = P.u[P.at(res, i)], v1 = P.v[P.at(res, i)];
      const double u2 = P.u[P.at(res, i + 1)], v2 = P.v[P.at(res, i + 1)];
      const double At = 0.5 * ((u1 - u0) * (v2 - v0) - (v1 - v0) * (u2 - u0));
      double Atb = 0.0;
      double pb0u = 0.0, pb0v = 0.0, pb1u = 0.0, pb1v = 0.0, pb2u = 0.0, pb2v = 0.0;
#pragma unroll 1
      for (int q = 0; q < NQ; ++q) {
        double l0, l1, l2, w;
        rule_point<NQ>(q, l0, l1, l2, w);
        const double pu = l0 * u0 + l1 * u1 + l2 * u2;
        const double pv = l0 * v0 + l1 * v1 + l2 * v2;
        const double wA = w * At;
        double a1, a2, b1, b2;
        if (!inverse_bilinear(S, pu, pv, kp.newton_tol, kp.newton_maxit, a1, a2)) ++noconv;
        if (!inverse_bilinear(Mn, pu, pv, kp.newton_tol, kp.newton_maxit, b1, b2)) ++noconv;
        double Ns[4], Nm[4], ds1[4], ds2[4], dm1[4], dm2[4];
        shape4(a1, a2, Ns);
        shape4(b1, b2, Nm);
        shape_grad(a1, a2, ds1, ds2);
        shape_grad(b1, b2, dm1, dm2);
        const double gap = (Nm[0] * hm[0] + Nm[1] * hm[1] + Nm[2] * hm[2] + Nm[3] * hm[3]) -
                           (Ns[0] * hs[0] + Ns[1] * hs[1] + Ns[2] * hs[2] + Ns[3] * hs[3]);
        // f = sum_j Ns_j a_j,  a_j = sum_k WD_jk Ns_k + sum_l WM_jl Nm_l + wg_j gap
        double fval = 0.0, G = 0.0;
        double nsb[4], nmb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          nsb[k] = 0.0;
          nmb[k] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double aj = wg[j] * gap;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            aj += WD[j * 4 + k] * Ns[k] + WM[j * 4 + k] * Nm[k];
            nsb[k] += Ns[j] * WD[j * 4 + k];
            nmb[k] += Ns[j] * WM[j * 4 + k];
          }
          fval += Ns[j] * aj;
          nsb[j] += aj;
          G += wg[j] * Ns[j];
        }
        Atb += w * fval;
        double xb1 = 0.0, xb2 = 0.0, eb1 = 0.0, eb2 = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double ns = wA * (nsb[k] - G * hs[k]);
          const double nm = wA * (nmb[k] + G * hm[k]);
          hsb[k] -= wA * G * Ns[k];
          hmb[k] += wA * G * Nm[k];
          xb1 += ns * ds1[k];
          xb2 += ns * ds2[k];
          eb1 += nm * dm1[k];
          eb2 += nm * dm2[k];
        }
        double ls0, ls1, lm0, lm1;
        ift_adjoint(ms, a1, a2, xb1, xb2, ls0, ls1);
        ift_adjoint(mm, b1, b2, eb1, eb2, lm0, lm1);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          Sb[k].u -= Ns[k] * ls0;
          Sb[k].v -= Ns[k] * ls1;
          Mb[k].u -= Nm[k] * lm0;
          Mb[k].v -= Nm[k] * lm1;
        }
        const double pbu = ls0 + lm0, pbv = ls1 + lm1;
        pb0u += l0 * pbu; pb0v += l0 * pbv;
        pb1u += l1 * pbu; pb1v += l1 * pbv;
        pb2u += l2 * pbu; pb2v += l2 * pbv;
      }
      // triangle area
      const double hA = 0.5 * Atb;
      au[0] += pb0u + hA * (v1 - v2);
      av[0] += pb0v + hA * (u2 - u1);
      au[i * bs] += pb1u + hA * (v2 - v0);
      av[i * bs] += pb1v - hA * (u2 - u0);
      au[(i + 1) * bs] += pb2u - hA * (v1 - v0);
      av[(i + 1) * bs] += pb2v + hA * (u1 - u0);
    }
  }

  // clip vertices -> projected nodes, through each vertex's provenance
  for (int i = 0; i < n; ++i) {
    const double xu = au[i * bs], xv = av[i * bs];
    const uint8_t lab = P.vl[P.at(res, i)];
    if (lab & 0x80) {
      const int k = lab & 3;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        if (kk == k) {
          Sb[kk].u += xu;
          Sb[kk].v += xv;
        }
      continue;
    }
    const int la = lab >> 4, lb = lab & 15;
    // line ids 0..3: slave edges k -> k+1; 4..7: master clip edges l -> l+1,
    // whose endpoints are master nodes (4 - l) % 4 when the master is walked
    // in reverse
    const bool ma = la >= 4, mb = lb >= 4;
    const int la4 = la & 3, lb4 = lb & 3;
    const int ia0 = ma && flip ? (4 - la4) & 3 : la4;
    const int ia1 = ma && flip ? (3 - la4) & 3 : (la4 + 1) & 3;
    const int ib0 = mb && flip ? (4 - lb4) & 3 : lb4;
    const int ib1 = mb && flip ? (3 - lb4) & 3 : (lb4 + 1) & 3;
    V2 A1 = ma ? Mn[0] : S[0], A2 = A1, B1 = mb ? Mn[0] : S[0], B2 = B1;
#pragma unroll
    for (int kk = 1; kk < 4; ++kk) {
      const V2 ak = ma ? Mn[kk] : S[kk], bk = mb ? Mn[kk] : S[kk];
      if (ia0 == kk) A1 = ak;
      if (ia1 == kk) A2 = ak;
      if (ib0 == kk) B1 = bk;
      if (ib1 == kk) B2 = bk;
    }
    V2 a1, a2, b1, b2;
    intersect_adjoint(A1, A2, B1, B2, xu, xv, a1, a2, b1, b2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double du = 0.0, dv = 0.0;
      if (ia0 == k) { du += a1.u; dv += a1.v; }
      if (ia1 == k) { du += a2.u; dv += a2.v; }
      if (ma) { Mb[k].u += du; Mb[k].v += dv; } else { Sb[k].u += du; Sb[k].v += dv; }
      du = 0.0;
      dv = 0.0;
      if (ib0 == k) { du += b1.u; dv += b1.v; }
      if (ib1 == k) { du += b2.u; dv += b2.v; }
      if (mb) { Mb[k].u += du; Mb[k].v += dv; } else { Sb[k].u += du; Sb[k].v += dv; }
    }
  }

  // projection: (u, v, h) = ((X - x0).t1, (X - x0).t2, (X - x0).n0)
  {
#pragma clang fp contract(fast)
  double x0b[3] = {0, 0, 0}, t1b[3] = {0, 0, 0}, t2b[3] = {0, 0, 0}, n0b[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double* X = k < 4 ? Xs[k] : Xm[k - 4];
    const double ub = k < 4 ? Sb[k].u : Mb[k - 4].u;
    const double vbb = k < 4 ? Sb[k].v : Mb[k - 4].v;
    const double hb = k < 4 ? hsb[k] : hmb[k - 4];
    double* Xb = k < 4 ? Xsb[k] : Xmb[k - 4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double dd = X[d] - f[d];
      const double gg = ub * f[6 + d] + vbb * f[9 + d] + hb * f[3 + d];
      Xb[d] = gg;
      x0b[d] -= gg;
      t1b[d] += ub * dd;
      t2b[d] += vbb * dd;
      n0b[d] += hb * dd;
    }
  }
  // t2 = n0 x t1
  const double* n0 = f + 3;
  const double* t1 = f + 6;
  n0b[0] += t1[1] * t2b[2] - t1[2] * t2b[1];
  n0b[1] += t1[2] * t2b[0] - t1[0] * t2b[2];
  n0b[2] += t1[0] * t2b[1] - t1[1] * t2b[0];
  t1b[0] += t2b[1] * n0[2] - t2b[2] * n0[1];
  t1b[1] += t2b[2] * n0[0] - t2b[0] * n0[2];
  t1b[2] += t2b[0] * n0[1] - t2b[1] * n0[0];
  // frame from the slave nodes: g1, g2, n = g1 x g2, n0 = n/|n|, t1 = g1/|g1|
  double g1[3], g2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g1[d] = 0.25 * (((Xs[1][d] - Xs[0][d]) + Xs[2][d]) - Xs[3][d]);
    g2[d] = 0.25 * (((Xs[2][d] + Xs[3][d]) - Xs[0][d]) - Xs[1][d]);
  }
  const double nn[3] = {g1[1] * g2[2] - g1[2] * g2[1], g1[2] * g2[0] - g1[0] * g2[2], g1[0] * g2[1] - g1[1] * g2[0]};
  const double rln = 1.0 / sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
  const double rlg = 1.0 / sqrt(g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]);
  const double tt = t1[0] * t1b[0] + t1[1] * t1b[1] + t1[2] * t1b[2];
  const double nt = n0[0] * n0b[0] + n0[1] * n0b[1] + n0[2] * n0b[2];
  double g1b[3], g2b[3], nb[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g1b[d] = (t1b[d] - t1[d] * tt) * rlg;
    nb[d] = (n0b[d] - n0[d] * nt) * rln;
  }
  g1b[0] += g2[1] * nb[2] - g2[2] * nb[1];
  g1b[1] += g2[2] * nb[0] - g2[0] * nb[2];
  g1b[2] += g2[0] * nb[1] - g2[1] * nb[0];
  g2b[0] = nb[1] * g1[2] - nb[2] * g1[1];
  g2b[1] = nb[2] * g1[0] - nb[0] * g1[2];
  g2b[2] = nb[0] * g1[1] - nb[1] * g1[0];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double c0 = 0.25 * x0b[d], c1 = 0.25 * g1b[d], c2 = 0.25 * g2b[d];
    Xsb[0][d] += c0 - c1 - c2;
    Xsb[1][d] += c0 + c1 - c2;
    Xsb[2][d] += c0 + c1 + c2;
    Xsb[3][d] += c0 - c1 + c2;
  }
  }
}

}  // namespace mt
