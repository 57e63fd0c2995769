// Evaluation of one (slave, master) element pair, forward and backward, as
// device functions shared by the single-interface kernels and the persistent
// batched kernels.
//
// The clip polygon of a pair is computed once (k_pair_poly, in LDS) and
// stored structure-of-arrays in HBM with each vertex's provenance; the
// integration and its reverse mode read it from there and need no LDS.
//
// Quadrature works in the monomial basis m(xi) = (1, xi1, xi2, xi1 xi2) of
// the bilinear element: N(xi) = C m(xi) with C = H / 4,
//   H = [[1,-1,-1, 1], [1, 1,-1,-1], [1, 1, 1, 1], [1,-1, 1,-1]],
// (row k: (1, s1, s2, s1 s2), (s1, s2) the corner of node k), H H^T = 4 I.
// A quad's map x(xi) = sum_k N_k(xi) X_k = c + e1 xi1 + e2 xi2 + f xi1 xi2
// has coefficients (c, e1, e2, f) = C^T X and nodes X = H (c, e1, e2, f).
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

// ---- clip polygons in HBM (layout: PolyBuf) ------------------------------------
struct GPoly {
  const double* __restrict__ u;
  const double* __restrict__ v;
  const uint8_t* __restrict__ l;
  int64_t stride, p;
  __device__ __forceinline__ double U(int i) const { return u[(int64_t)i * stride + p]; }
  __device__ __forceinline__ double V(int i) const { return v[(int64_t)i * stride + p]; }
  __device__ __forceinline__ uint8_t L(int i) const { return l[(int64_t)i * stride + p]; }
};

// Polygon of pair p (at its entry of the buffer).
__device__ __forceinline__ GPoly gpoly(const PolyBuf& b, int64_t p) {
  return GPoly{b.u, b.v, b.lab, b.stride, b.at(p)};
}
__device__ __forceinline__ uint8_t gpoly_nf(const PolyBuf& b, int64_t p) { return b.nf[b.at(p)]; }

// Copies a clip polygon (n vertices in LDS buffer res) and its provenance to
// entry idx of a polygon buffer.
__device__ __forceinline__ void poly_store(const LdsPoly<true>& P, int res, int n, bool flip, const PolyBuf& out,
                                           int64_t idx) {
  out.nf[idx] = (uint8_t)(n | (flip ? 0x80 : 0));
  for (int i = 0; i < n; ++i) {
    out.u[(int64_t)i * out.stride + idx] = P.u[P.at(res, i)];
    out.v[(int64_t)i * out.stride + idx] = P.v[P.at(res, i)];
    out.lab[(int64_t)i * out.stride + idx] = P.vl[P.at(res, i)];
  }
}

// Frame, projection, orientation, clip and cleanup of pair p; stores the
// polygon and its provenance.  Returns the clip status bits (PS_*), with
// PS_LOST when the polygon is no longer a segment at these coordinates (the
// pair then contributes nothing).
__device__ __forceinline__ int store_pair_polygon(const double Xs[4][3], const double Xm[4][3], const double* ns,
                                                   const KParams& kp, const LdsPoly<true>& P, const PolyBuf& out,
                                                   int64_t p) {
  double f[12];
  slave_frame_p(Xs, ns, f);
  V2 S[4], Mn[4];
  double hs[4], hm[4];
  int res, st;
  bool flip;
  const int n = pair_geometry<true>(Xs, Xm, f, kp.eps_d, kp.eps_a, S, Mn, hs, hm, flip, P, res, st);
  poly_store(P, res, n, flip, out, out.at(p));
  return st | (n >= 3 ? 0 : PS_LOST);
}

// Projected nodes and heights of both elements on the slave plane f.
__device__ __forceinline__ void pair_project(const double Xs[4][3], const double Xm[4][3], const double f[12],
                                             V2 S[4], V2 Mn[4], double hs[4], double hm[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    project(Xs[k], f, S[k], hs[k]);
    project(Xm[k], f, Mn[k], hm[k]);
  }
}

// ---- monomial basis helpers ------------------------------------------------------

// y = H x
__device__ __forceinline__ void h_apply(const double x[4], double y[4]) {
  const double am = x[0] - x[2], ap = x[0] + x[2], bm = x[1] - x[3], bp = x[1] + x[3];
  y[0] = am - bm;
  y[1] = am + bm;
  y[2] = ap + bp;
  y[3] = ap - bp;
}
// y = H^T x
__device__ __forceinline__ void ht_apply(const double x[4], double y[4]) {
  const double s03 = x[0] + x[3], s12 = x[1] + x[2];
  y[0] = s03 + s12;
  y[1] = s12 - s03;
  y[2] = (x[2] + x[3]) - (x[0] + x[1]);
  y[3] = (x[0] + x[2]) - (x[1] + x[3]);
}
// Y = s H X H^T for a row-major 4x4 X.
__device__ __forceinline__ void h_sandwich(const double X[16], double s, double Y[16]) {
  double T[16];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double col[4] = {X[c], X[4 + c], X[8 + c], X[12 + c]};
    double y[4];
    h_apply(col, y);
#pragma unroll
    for (int r = 0; r < 4; ++r) T[r * 4 + c] = y[r];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double y[4];
    h_apply(T + 4 * r, y);
#pragma unroll
    for (int k = 0; k < 4; ++k) Y[r * 4 + k] = s * y[k];
  }
}
// Y = s H^T X H for a row-major 4x4 X.
__device__ __forceinline__ void ht_sandwich(const double X[16], double s, double Y[16]) {
  double T[16];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double col[4] = {X[c], X[4 + c], X[8 + c], X[12 + c]};
    double y[4];
    ht_apply(col, y);
#pragma unroll
    for (int r = 0; r < 4; ++r) T[r * 4 + c] = y[r];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double y[4];
    ht_apply(T + 4 * r, y);
#pragma unroll
    for (int k = 0; k < 4; ++k) Y[r * 4 + k] = s * y[k];
  }
}

// Launders an index so that loads through it are not merged with earlier
// loads of the same address (the values are reloaded instead of being kept
// in registers across the quadrature loop).
__device__ __forceinline__ int launder(int i) {
  asm volatile("" : "+v"(i));
  return i;
}

// Reciprocal: hardware estimate refined by two Newton-Raphson steps.
__device__ __forceinline__ double rcp_nr(double d) {
#pragma clang fp contract(fast)
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// Map coefficients (c, e1, e2, f) of a projected quad and the reciprocal
// determinant of its Jacobian at xi = 0.
struct QMap {
  double cu, cv, e1u, e1v, e2u, e2v, fu, fv, r0;
};

__device__ __forceinline__ QMap qmap(const V2 X[4]) {
#pragma clang fp contract(fast)
  QMap m;
  m.cu = 0.25 * ((X[0].u + X[1].u) + (X[2].u + X[3].u));
  m.cv = 0.25 * ((X[0].v + X[1].v) + (X[2].v + X[3].v));
  m.e1u = 0.25 * ((X[1].u - X[0].u) + (X[2].u - X[3].u));
  m.e1v = 0.25 * ((X[1].v - X[0].v) + (X[2].v - X[3].v));
  m.e2u = 0.25 * ((X[2].u - X[1].u) + (X[3].u - X[0].u));
  m.e2v = 0.25 * ((X[2].v - X[1].v) + (X[3].v - X[0].v));
  m.fu = 0.25 * ((X[0].u - X[1].u) + (X[2].u - X[3].u));
  m.fv = 0.25 * ((X[0].v - X[1].v) + (X[2].v - X[3].v));
  m.r0 = rcp_nr(m.e1u * m.e2v - m.e2u * m.e1v);
  return m;
}

// Node k of a quad from its map coefficients: c + s1 e1 + s2 e2 + s1 s2 f.
__device__ __forceinline__ V2 qmap_node(const QMap& m, int k) {
#pragma clang fp contract(fast)
  const double s1 = (k == 1 || k == 2) ? 1.0 : -1.0;
  const double s2 = k >= 2 ? 1.0 : -1.0;
  const double s12 = s1 * s2;
  return V2{m.cu + s1 * m.e1u + s2 * m.e2u + s12 * m.fu, m.cv + s1 * m.e1v + s2 * m.e2v + s12 * m.fv};
}

// One Newton step for x(xi) = p, d = p - c: stops (conv) once the step
// J^-1 r is at most tol in both components, tested as |adj(J) r| <= tol |det J|
// without the division.
__device__ __forceinline__ void newton_step(const QMap& m, double du, double dv, double tol, double& x1, double& x2,
                                            bool& conv) {
#pragma clang fp contract(fast)
  const double x12 = x1 * x2;
  const double ru = m.e1u * x1 + m.e2u * x2 + m.fu * x12 - du;
  const double rv = m.e1v * x1 + m.e2v * x2 + m.fv * x12 - dv;
  const double j00 = m.e1u + m.fu * x2, j01 = m.e2u + m.fu * x1;
  const double j10 = m.e1v + m.fv * x2, j11 = m.e2v + m.fv * x1;
  const double det = j00 * j11 - j01 * j10;
  const double n1 = j11 * ru - j01 * rv;
  const double n2 = j00 * rv - j10 * ru;
  const bool ok = fmax(fabs(n1), fabs(n2)) <= tol * fabs(det);
  const bool upd = !(conv || ok);
  const double r = rcp_nr(det);
  x1 = upd ? x1 - n1 * r : x1;
  x2 = upd ? x2 - n2 * r : x2;
  conv = conv || ok;
}

// Inverse bilinear maps of point p on the slave quad (a) and the master quad
// (b) by Newton's method from xi = 0, interleaved.  The first step uses the
// precomputed Jacobian at 0; at most maxit steps per map.  Counts maps that
// did not converge in noconv.
__device__ __forceinline__ void inverse2(const QMap& A, const QMap& B, double pu, double pv, double tol, int maxit,
                                         double& a1, double& a2, double& b1, double& b2, unsigned& noconv) {
#pragma clang fp contract(fast)
  const double dau = pu - A.cu, dav = pv - A.cv, dbu = pu - B.cu, dbv = pv - B.cv;
  a1 = (A.e2v * dau - A.e2u * dav) * A.r0;
  a2 = (A.e1u * dav - A.e1v * dau) * A.r0;
  b1 = (B.e2v * dbu - B.e2u * dbv) * B.r0;
  b2 = (B.e1u * dbv - B.e1v * dbu) * B.r0;
  bool ca = false, cb = false;
  for (int it = 1; it < maxit && !(ca && cb); ++it) {
    newton_step(A, dau, dav, tol, a1, a2, ca);
    newton_step(B, dbu, dbv, tol, b1, b2, cb);
  }
  noconv += (ca ? 0u : 1u) + (cb ? 0u : 1u);
}

// ---- forward -------------------------------------------------------------------
// Blocks from the monomial moments of a quadrature: mu_ij = sum w xi1^i
// xi2^j (i, j <= 2) and Mm[p][r] = sum w m_p(xi) m_r(eta), with the nodal
// heights: D = C Dm C^T (Dm[p][r] the moment of m_p m_r), M = C Mm C^T,
// g = C (Mm ht_m - Dm ht_s), ht = C^T h; for the dual basis Phi = A N:
// D, M, g <- A D, A M, A g.
template <bool DUAL>
__device__ __forceinline__ void moments_to_blocks(const QMap& ms, const double mu[9], const double Mm[16],
                                                  const double hs[4], const double hm[4], double D[16],
                                                  double M[16], double g[4]) {
#pragma clang fp contract(fast)
  // Dm[p][r]: monomial exponents (0,0), (1,0), (0,1), (1,1) added
  const double Dm[16] = {mu[0], mu[1], mu[2], mu[3], mu[1], mu[4], mu[3], mu[6],
                         mu[2], mu[3], mu[5], mu[7], mu[3], mu[6], mu[7], mu[8]};
  double hts[4], htm[4];
  ht_apply(hs, hts);
  ht_apply(hm, htm);
  double gm[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    gm[p] = 0.25 * ((Mm[4 * p] * htm[0] + Mm[4 * p + 1] * htm[1] + Mm[4 * p + 2] * htm[2] + Mm[4 * p + 3] * htm[3]) -
                    (Dm[4 * p] * hts[0] + Dm[4 * p + 1] * hts[1] + Dm[4 * p + 2] * hts[2] + Dm[4 * p + 3] * hts[3]));
  }
  double gs[4];
  h_apply(gm, gs);
  double Ds[16], Ms[16];
  h_sandwich(Dm, 0.0625, Ds);
  h_sandwich(Mm, 0.0625, Ms);
  if (DUAL) {
    const V2 S[4] = {qmap_node(ms, 0), qmap_node(ms, 1), qmap_node(ms, 2), qmap_node(ms, 3)};
    double A[16];
    dual_coefficients(S, A);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        D[4 * j + k] = A[4 * j] * Ds[k] + A[4 * j + 1] * Ds[4 + k] + A[4 * j + 2] * Ds[8 + k] + A[4 * j + 3] * Ds[12 + k];
        M[4 * j + k] = A[4 * j] * Ms[k] + A[4 * j + 1] * Ms[4 + k] + A[4 * j + 2] * Ms[8 + k] + A[4 * j + 3] * Ms[12 + k];
      }
      g[j] = 0.25 * (A[4 * j] * gs[0] + A[4 * j + 1] * gs[1] + A[4 * j + 2] * gs[2] + A[4 * j + 3] * gs[3]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      D[k] = Ds[k];
      M[k] = Ms[k];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) g[j] = 0.25 * gs[j];
  }
}

// Local blocks of one pair from its stored polygon (n vertices):
//   D[j][k] = sum w A_t Phi_j N_k(xi),  M[j][l] = sum w A_t Phi_j N_l(eta),
//   g[j]    = sum w A_t Phi_j (sum_l N_l(eta) hm_l - sum_k N_k(xi) hs_k),
// over the fan triangles from vertex 0 and the rule points.  Accumulates the
// moments mu_ij = sum w A_t xi1^i xi2^j (i, j <= 2) and
// Mm[p][r] = sum w A_t m_p(xi) m_r(eta); then D = C Dm C^T (Dm[p][r] the
// moment of m_p m_r), M = C Mm C^T, g = C (Mm ht_m - Dm ht_s) with
// ht = C^T h, and for the dual basis Phi = A N: D, M, g <- A D, A M, A g.
template <int NQ, bool DUAL, class Heights>
__device__ __forceinline__ void pair_integrate(const QMap& ms, const QMap& mm, const Heights& heights,
                                             const GPoly& P, int n, const KParams& kp, double D[16], double M[16],
                                             double g[4], unsigned& noconv) {
double mu[9], Mm[16];
#pragma unroll
for (int k = 0; k < 9; ++k) mu[k] = 0.0;
#pragma unroll
for (int k = 0; k < 16; ++k) Mm[k] = 0.0;
if (n >= 3) {
#pragma clang fp contract(fast)
  const double u0 = P.U(0), v0 = P.V(0);
  double u1 = P.U(1), v1 = P.V(1);
  for (int i = 1; i + 1 < n; ++i) {
    const double u2 = P.U(i + 1), v2 = P.V(i + 1);
    const double At = 0.5 * ((u1 - u0) * (v2 - v0) - (v1 - v0) * (u2 - u0));
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      double l0, l1, l2, w;
      rule_point<NQ>(q, l0, l1, l2, w);
      const double pu = l0 * u0 + l1 * u1 + l2 * u2;
      const double pv = l0 * v0 + l1 * v1 + l2 * v2;
      double a1, a2, b1, b2;
      inverse2(ms, mm, pu, pv, kp.newton_tol, kp.newton_maxit, a1, a2, b1, b2, noconv);
      const double t[4] = {w * At, w * At * a1, w * At * a2, w * At * a1 * a2};
      mu[0] += t[0];
      mu[1] += t[1];
      mu[2] += t[2];
      mu[3] += t[3];
      mu[4] += t[1] * a1;
      mu[5] += t[2] * a2;
      mu[6] += t[3] * a1;
      mu[7] += t[3] * a2;
      mu[8] += t[3] * (a1 * a2);
      const double b12 = b1 * b2;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        Mm[4 * p] += t[p];
        Mm[4 * p + 1] += t[p] * b1;
        Mm[4 * p + 2] += t[p] * b2;
        Mm[4 * p + 3] += t[p] * b12;
      }
    }
    u1 = u2;
    v1 = v2;
  }
}
if (n < 3) {
  // no segment (a pair lost after a coordinate update): no contribution, and
  // no dual coefficients of a possibly degenerate slave element
#pragma unroll
  for (int k = 0; k < 16; ++k) D[k] = M[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) g[k] = 0.0;
  return;
}
double hs[4], hm[4];
heights(hs, hm);
moments_to_blocks<DUAL>(ms, mu, Mm, hs, hm, D, M, g);
}

// ---- backward ------------------------------------------------------------------

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
  const double rden = rcp_nr(den);
  const double num = wu * dBv - wv * dBu;
  const double s = num * rden;
  double dAbu = s * xu, dAbv = s * xv;
  const double sb = xu * dAu + xv * dAv;
  const double numb = sb * rden;
  const double denb = -numb * s;
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

// Adjoint of node k of a quad, added in map-coefficient form:
// (c, e1, e2, f)-bar += H[k][.] d (the node adjoint is then C times it).
__device__ __forceinline__ void add_node_adj(double cb[8], int k, double du, double dv) {
#pragma clang fp contract(fast)
  const double s1 = (k == 1 || k == 2) ? 1.0 : -1.0;
  const double s2 = k >= 2 ? 1.0 : -1.0;
  const double s12 = s1 * s2;
  cb[0] += du;
  cb[1] += dv;
  cb[2] += s1 * du;
  cb[3] += s1 * dv;
  cb[4] += s2 * du;
  cb[5] += s2 * dv;
  cb[6] += s12 * du;
  cb[7] += s12 * dv;
}

// Pull the adjoint (xu, xv) of one clip vertex back to the projected nodes
// through its provenance: a slave node directly; otherwise the intersection
// of its two lines (the second always a master clip edge).  Master clip edge
// l runs Mo[l] -> Mo[l+1] with Mo[j] = Mn[(4 - j) % 4] when flipped.
__device__ __forceinline__ void vertex_adjoint(uint8_t lab, double xu, double xv, const QMap& ms, const QMap& mm,
                                               bool flip, double cbs[8], double cbm[8]) {
  if (lab & 0x80) {
    add_node_adj(cbs, lab & 3, xu, xv);
    return;
  }
  const int la = lab >> 4, lb = lab & 15;
  const bool ma = la >= 4;
  const int la4 = la & 3, lb4 = lb & 3;
  const int ia0 = ma && flip ? (4 - la4) & 3 : la4;
  const int ia1 = ma && flip ? (3 - la4) & 3 : (la4 + 1) & 3;
  const int ib0 = flip ? (4 - lb4) & 3 : lb4;
  const int ib1 = flip ? (3 - lb4) & 3 : (lb4 + 1) & 3;
  const QMap& mA = ma ? mm : ms;
  const V2 A1 = qmap_node(mA, ia0), A2 = qmap_node(mA, ia1);
  const V2 B1 = qmap_node(mm, ib0), B2 = qmap_node(mm, ib1);
  V2 a1, a2, b1, b2;
  intersect_adjoint(A1, A2, B1, B2, xu, xv, a1, a2, b1, b2);
  if (ma) {
    add_node_adj(cbm, ia0, a1.u, a1.v);
    add_node_adj(cbm, ia1, a2.u, a2.v);
  } else {
    add_node_adj(cbs, ia0, a1.u, a1.v);
    add_node_adj(cbs, ia1, a2.u, a2.v);
  }
  add_node_adj(cbm, ib0, b1.u, b1.v);
  add_node_adj(cbm, ib1, b2.u, b2.v);
}

// Adjoint of the projection (u, v, h) = ((X - x0).t1, (X - x0).t2,
// (X - x0).n0) of the 8 nodes (slave 0..3, master 4..7) and of the slave
// frame (x0, n0 = g1 x g2 / |g1 x g2|, t1 = g1 / |g1|, t2 = n0 x t1):
// given nb[k] = (ubar, vbar, hbar) of node k, writes the coordinate
// gradients Xsb (slave) and Xmb (master).  With the continuous normal field
// (ns, the element's plane normal: n0 = ns, t1 = the part of g1 orthogonal to
// n0, normalised) the gradient with respect to n0 is added to n0b instead.
__device__ __forceinline__ void projection_adjoint(const double Xs[4][3], const double Xm[4][3], const double* ns,
                                                   const double nb[8][3], double Xsb[4][3], double Xmb[4][3],
                                                   double n0b_out[3]) {
#pragma clang fp contract(fast)
  double f[12];
  slave_frame_p(Xs, ns, f);
  double x0b[3] = {0, 0, 0}, t1b[3] = {0, 0, 0}, t2b[3] = {0, 0, 0}, n0b[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double* X = k < 4 ? Xs[k] : Xm[k - 4];
    const double ub = nb[k][0], vbb = nb[k][1], hb = nb[k][2];
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
  double g1[3], g2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g1[d] = 0.25 * (((Xs[1][d] - Xs[0][d]) + Xs[2][d]) - Xs[3][d]);
    g2[d] = 0.25 * (((Xs[2][d] + Xs[3][d]) - Xs[0][d]) - Xs[1][d]);
  }
  if (ns) {
    // t1 = w / |w|, w = g1 - (g1.n0) n0; n0 is an input
    const double gn = g1[0] * n0[0] + g1[1] * n0[1] + g1[2] * n0[2];
    double w[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) w[d] = g1[d] - gn * n0[d];
    const double rlw = 1.0 / sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    const double tt = t1[0] * t1b[0] + t1[1] * t1b[1] + t1[2] * t1b[2];
    double wb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) wb[d] = (t1b[d] - t1[d] * tt) * rlw;
    const double nw = n0[0] * wb[0] + n0[1] * wb[1] + n0[2] * wb[2];
    double g1b[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      g1b[d] = wb[d] - n0[d] * nw;
      n0b_out[d] += n0b[d] - g1[d] * nw - gn * wb[d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double c0 = 0.25 * x0b[d], c1 = 0.25 * g1b[d];
      Xsb[0][d] += c0 - c1;
      Xsb[1][d] += c0 + c1;
      Xsb[2][d] += c0 + c1;
      Xsb[3][d] += c0 - c1;
    }
    return;
  }
  // frame from the slave nodes: g1, g2, n = g1 x g2, n0 = n/|n|, t1 = g1/|g1|
  const double nn[3] = {g1[1] * g2[2] - g1[2] * g2[1], g1[2] * g2[0] - g1[0] * g2[2], g1[0] * g2[1] - g1[1] * g2[0]};
  const double rln = 1.0 / sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
  const double rlg = 1.0 / sqrt(g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]);
  const double tt = t1[0] * t1b[0] + t1[1] * t1b[1] + t1[2] * t1b[2];
  const double nt = n0[0] * n0b[0] + n0[1] * n0b[1] + n0[2] * n0b[2];
  double g1b[3], g2b[3], nbv[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    g1b[d] = (t1b[d] - t1[d] * tt) * rlg;
    nbv[d] = (n0b[d] - n0[d] * nt) * rln;
  }
  g1b[0] += g2[1] * nbv[2] - g2[2] * nbv[1];
  g1b[1] += g2[2] * nbv[0] - g2[0] * nbv[2];
  g1b[2] += g2[0] * nbv[1] - g2[1] * nbv[0];
  g2b[0] = nbv[1] * g1[2] - nbv[2] * g1[1];
  g2b[1] = nbv[2] * g1[0] - nbv[0] * g1[2];
  g2b[2] = nbv[0] * g1[1] - nbv[1] * g1[0];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double c0 = 0.25 * x0b[d], c1 = 0.25 * g1b[d], c2 = 0.25 * g2b[d];
    Xsb[0][d] += c0 - c1 - c2;
    Xsb[1][d] += c0 + c1 - c2;
    Xsb[2][d] += c0 + c1 + c2;
    Xsb[3][d] += c0 - c1 + c2;
  }
}

// Backward of one pair: gradient of
// L = sum WD[j][k] D[j][k] + sum WM[j][l] M[j][l] + sum wg[j] g[j]
// with respect to the slave (Xsb) and master (Xmb) nodal coordinates, from
// the stored polygon (nf = count | flip << 7).  Per rule point the
// integrand is F = 1/2 ma^T Q ma + ma^T W mb (ma = m(xi), mb = m(eta)), with
// Q = C^T (WD + WD^T) C - (wt ht_s^T + ht_s wt^T), W = C^T WM C + wt ht_m^T,
// wt = C^T wg, ht = C^T h; reverse mode runs through the quadrature, the
// inverse maps (implicit-function derivative), the clip vertices (line
// intersections, each vertex once: the fan's pending vertex is carried to the
// next triangle), the projection and the slave frame.
template <int NQ, bool DUAL, bool NODAL = false>
__device__ __forceinline__ void pair_backward(const MeshPtrs& SM, int s, int4 cs, const MeshPtrs& MM, int4 cm,
                                              const GPoly& P, int nf, const KParams& kp, const double WD_in[16],
                                              const double WM_in[16], const double wg_in[4], double Xsb[4][3],
                                              double Xmb[4][3], double n0b[3], unsigned& noconv) {
  const int n = nf & 0x7f;
  const bool flip = (nf & 0x80) != 0;
  QMap ms, mm;
  double Qs[10], W[16], wt[4];
  {
#pragma clang fp contract(fast)
    double Xs[4][3], Xm[4][3], f[12];
    load_nodes(SM.x, SM.y, SM.z, cs, Xs);
    load_nodes(MM.x, MM.y, MM.z, cm, Xm);
    slave_frame_p(Xs, NODAL ? elem_nrm(SM, s) : nullptr, f);
    V2 S[4], Mn[4];
    double hs[4], hm[4];
    pair_project(Xs, Xm, f, S, Mn, hs, hm);
    ms = qmap(S);
    mm = qmap(Mn);
    // dual basis: the blocks are A times the standard ones, so the standard
    // sweep runs on the weights A^T W (the dependence of A on the slave
    // nodes is added by dual_adjoint)
    double WD[16], WM[16], wg[4];
    if (DUAL) {
      double A[16];
      dual_coefficients(S, A);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          WD[4 * m + k] = A[m] * WD_in[k] + A[4 + m] * WD_in[4 + k] + A[8 + m] * WD_in[8 + k] + A[12 + m] * WD_in[12 + k];
          WM[4 * m + k] = A[m] * WM_in[k] + A[4 + m] * WM_in[4 + k] + A[8 + m] * WM_in[8 + k] + A[12 + m] * WM_in[12 + k];
        }
        wg[m] = A[m] * wg_in[0] + A[4 + m] * wg_in[1] + A[8 + m] * wg_in[2] + A[12 + m] * wg_in[3];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        WD[k] = WD_in[k];
        WM[k] = WM_in[k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) wg[k] = wg_in[k];
    }
    double hts[4], htm[4];
    ht_apply(hs, hts);
    ht_apply(hm, htm);
    ht_apply(wg, wt);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      hts[k] *= 0.25;
      htm[k] *= 0.25;
      wt[k] *= 0.25;
    }
    double WDs[16], Q[16];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < 4; ++k) WDs[4 * j + k] = WD[4 * j + k] + WD[4 * k + j];
    ht_sandwich(WDs, 0.0625, Q);
    ht_sandwich(WM, 0.0625, W);
    int z = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int r = p; r < 4; ++r) Qs[z++] = Q[4 * p + r] - (wt[p] * hts[r] + hts[p] * wt[r]);
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) W[4 * p + r] += wt[p] * htm[r];
  }
  // Qs: q00 q01 q02 q03 q11 q12 q13 q22 q23 q33
  double cbs[8], cbm[8], htsb[4], htmb[4];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    cbs[k] = 0.0;
    cbm[k] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    htsb[k] = 0.0;
    htmb[k] = 0.0;
  }
  if (n >= 3) {
#pragma clang fp contract(fast)
    const double u0 = P.U(0), v0 = P.V(0);
    double u1 = P.U(1), v1 = P.V(1);
    double x0bu = 0.0, x0bv = 0.0, pendu = 0.0, pendv = 0.0;
    for (int i = 1; i + 1 < n; ++i) {
      const double u2 = P.U(i + 1), v2 = P.V(i + 1);
      const double At = 0.5 * ((u1 - u0) * (v2 - v0) - (v1 - v0) * (u2 - u0));
      double Atb = 0.0;
      double pb0u = 0.0, pb0v = 0.0, pb1u = 0.0, pb1v = 0.0, pb2u = 0.0, pb2v = 0.0;
#pragma unroll 1
      for (int q = 0; q < NQ; ++q) {
        double l0, l1, l2, w;
        rule_point<NQ>(q, l0, l1, l2, w);
        const double pu = l0 * u0 + l1 * u1 + l2 * u2;
        const double pv = l0 * v0 + l1 * v1 + l2 * v2;
        double a1, a2, b1, b2;
        inverse2(ms, mm, pu, pv, kp.newton_tol, kp.newton_maxit, a1, a2, b1, b2, noconv);
        const double a12 = a1 * a2, b12 = b1 * b2;
        const double qa0 = Qs[0] + Qs[1] * a1 + Qs[2] * a2 + Qs[3] * a12;
        const double qa1 = Qs[1] + Qs[4] * a1 + Qs[5] * a2 + Qs[6] * a12;
        const double qa2 = Qs[2] + Qs[5] * a1 + Qs[7] * a2 + Qs[8] * a12;
        const double qa3 = Qs[3] + Qs[6] * a1 + Qs[8] * a2 + Qs[9] * a12;
        const double wb0 = W[0] + W[1] * b1 + W[2] * b2 + W[3] * b12;
        const double wb1 = W[4] + W[5] * b1 + W[6] * b2 + W[7] * b12;
        const double wb2 = W[8] + W[9] * b1 + W[10] * b2 + W[11] * b12;
        const double wb3 = W[12] + W[13] * b1 + W[14] * b2 + W[15] * b12;
        const double wa1 = W[1] + W[5] * a1 + W[9] * a2 + W[13] * a12;
        const double wa2 = W[2] + W[6] * a1 + W[10] * a2 + W[14] * a12;
        const double wa3 = W[3] + W[7] * a1 + W[11] * a2 + W[15] * a12;
        const double F = (0.5 * qa0 + wb0) + (0.5 * qa1 + wb1) * a1 + (0.5 * qa2 + wb2) * a2 + (0.5 * qa3 + wb3) * a12;
        const double G = wt[0] + wt[1] * a1 + wt[2] * a2 + wt[3] * a12;
        const double wA = w * At;
        Atb += w * F;
        const double ga3 = qa3 + wb3;
        const double xa1 = wA * ((qa1 + wb1) + a2 * ga3), xa2 = wA * ((qa2 + wb2) + a1 * ga3);
        const double xb1 = wA * (wa1 + b2 * wa3), xb2 = wA * (wa2 + b1 * wa3);
        const double wAG = wA * G;
        htsb[0] -= wAG;
        htsb[1] -= wAG * a1;
        htsb[2] -= wAG * a2;
        htsb[3] -= wAG * a12;
        htmb[0] += wAG;
        htmb[1] += wAG * b1;
        htmb[2] += wAG * b2;
        htmb[3] += wAG * b12;
        // implicit-function adjoint: lambda = J^-T xibar at the solution
        double lau, lav, lbu, lbv;
        {
          const double j00 = ms.e1u + ms.fu * a2, j01 = ms.e2u + ms.fu * a1;
          const double j10 = ms.e1v + ms.fv * a2, j11 = ms.e2v + ms.fv * a1;
          const double r = rcp_nr(j00 * j11 - j01 * j10);
          lau = (j11 * xa1 - j10 * xa2) * r;
          lav = (j00 * xa2 - j01 * xa1) * r;
        }
        {
          const double j00 = mm.e1u + mm.fu * b2, j01 = mm.e2u + mm.fu * b1;
          const double j10 = mm.e1v + mm.fv * b2, j11 = mm.e2v + mm.fv * b1;
          const double r = rcp_nr(j00 * j11 - j01 * j10);
          lbu = (j11 * xb1 - j10 * xb2) * r;
          lbv = (j00 * xb2 - j01 * xb1) * r;
        }
        cbs[0] -= lau;
        cbs[1] -= lav;
        cbs[2] -= a1 * lau;
        cbs[3] -= a1 * lav;
        cbs[4] -= a2 * lau;
        cbs[5] -= a2 * lav;
        cbs[6] -= a12 * lau;
        cbs[7] -= a12 * lav;
        cbm[0] -= lbu;
        cbm[1] -= lbv;
        cbm[2] -= b1 * lbu;
        cbm[3] -= b1 * lbv;
        cbm[4] -= b2 * lbu;
        cbm[5] -= b2 * lbv;
        cbm[6] -= b12 * lbu;
        cbm[7] -= b12 * lbv;
        const double pbu = lau + lbu, pbv = lav + lbv;
        pb0u += l0 * pbu;
        pb0v += l0 * pbv;
        pb1u += l1 * pbu;
        pb1v += l1 * pbv;
        pb2u += l2 * pbu;
        pb2v += l2 * pbv;
      }
      // triangle area, then vertex i is complete
      const double hA = 0.5 * Atb;
      x0bu += pb0u + hA * (v1 - v2);
      x0bv += pb0v + hA * (u2 - u1);
      vertex_adjoint(P.L(i), pendu + pb1u + hA * (v2 - v0), pendv + pb1v - hA * (u2 - u0), ms, mm, flip, cbs, cbm);
      pendu = pb2u - hA * (v1 - v0);
      pendv = pb2v + hA * (u1 - u0);
      u1 = u2;
      v1 = v2;
    }
    vertex_adjoint(P.L(n - 1), pendu, pendv, ms, mm, flip, cbs, cbm);
    vertex_adjoint(P.L(0), x0bu, x0bv, ms, mm, flip, cbs, cbm);
  }

  // node adjoints: Xbar = C (coefficient adjoint), hbar = C htbar (the 1/4
  // of C is applied in projection_adjoint)
  {
    double nb[8][3];
    {
      const double cu[4] = {cbs[0], cbs[2], cbs[4], cbs[6]}, cv[4] = {cbs[1], cbs[3], cbs[5], cbs[7]};
      double u[4], v[4], h[4];
      h_apply(cu, u);
      h_apply(cv, v);
      h_apply(htsb, h);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        nb[k][0] = 0.25 * u[k];
        nb[k][1] = 0.25 * v[k];
        nb[k][2] = 0.25 * h[k];
      }
    }
    {
      const double cu[4] = {cbm[0], cbm[2], cbm[4], cbm[6]}, cv[4] = {cbm[1], cbm[3], cbm[5], cbm[7]};
      double u[4], v[4], h[4];
      h_apply(cu, u);
      h_apply(cv, v);
      h_apply(htmb, h);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        nb[4 + k][0] = 0.25 * u[k];
        nb[4 + k][1] = 0.25 * v[k];
        nb[4 + k][2] = 0.25 * h[k];
      }
    }
    // on reloaded nodes and a recomputed frame
    const int4 cs2{launder(cs.x), launder(cs.y), launder(cs.z), launder(cs.w)};
    const int4 cm2{launder(cm.x), launder(cm.y), launder(cm.z), launder(cm.w)};
    double Xs[4][3], Xm[4][3];
    load_nodes(SM.x, SM.y, SM.z, cs2, Xs);
    load_nodes(MM.x, MM.y, MM.z, cm2, Xm);
    n0b[0] = n0b[1] = n0b[2] = 0.0;
    projection_adjoint(Xs, Xm, NODAL ? elem_nrm(SM, launder(s)) : nullptr, nb, Xsb, Xmb, n0b);
  }
}

}  // namespace mt

namespace mt {

// Forward of pair p from its stored polygon: nodes, slave frame, projection,
// then the quadrature of pair_integrate.  The heights are recomputed after
// the quadrature from reloaded nodes rather than kept in registers.
template <int NQ, bool DUAL>
__device__ __forceinline__ void pair_forward(const MeshPtrs& SM, int s, int4 cs, const MeshPtrs& MM, int4 cm,
                                             const GPoly& P, int nf, const KParams& kp, double D[16], double M[16],
                                             double g[4], unsigned& noconv) {
  QMap ms, mm;
  {
    double Xs[4][3], Xm[4][3], f[12];
    load_nodes(SM.x, SM.y, SM.z, cs, Xs);
    load_nodes(MM.x, MM.y, MM.z, cm, Xm);
    slave_frame_p(Xs, elem_nrm(SM, s), f);
    V2 S[4], Mn[4];
    double hs[4], hm[4];
    pair_project(Xs, Xm, f, S, Mn, hs, hm);
    ms = qmap(S);
    mm = qmap(Mn);
  }
  auto heights = [&](double hs[4], double hm[4]) {
    const int4 cs2{launder(cs.x), launder(cs.y), launder(cs.z), launder(cs.w)};
    const int4 cm2{launder(cm.x), launder(cm.y), launder(cm.z), launder(cm.w)};
    double Xs[4][3], Xm[4][3], f[12];
    load_nodes(SM.x, SM.y, SM.z, cs2, Xs);
    load_nodes(MM.x, MM.y, MM.z, cm2, Xm);
    slave_frame_p(Xs, elem_nrm(SM, launder(s)), f);
    V2 S[4], Mn[4];
    pair_project(Xs, Xm, f, S, Mn, hs, hm);
  };
  pair_integrate<NQ, DUAL>(ms, mm, heights, P, nf & 0x7f, kp, D, M, g, noconv);
}

}  // namespace mt
