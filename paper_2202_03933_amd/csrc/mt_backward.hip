// Backward pass of the pair evaluation: gradient of
//   L = <W_D, D> + <W_M, M> + <w_g, g>
// with respect to the 24 nodal coordinates of each pair (the linearisation
// of the mortar terms the paper requires in every nonlinear iteration).
//
// The clip geometry is recomputed (bitwise equal to the forward pass) with
// vertex provenance: each clip vertex is a projected slave node or the
// intersection of two lines (slave edges / master edges).  Reverse mode then
// runs through the quadrature (triangle areas, rule points), the inverse
// bilinear maps (implicit-function derivative: with J = dx/dxi,
// dxi = J^-1 (dp - sum_k N_k dX_k)), the line intersections, the projection
// onto the auxiliary plane and the slave frame (normalisations and cross
// products).  Per-pair gradients are staged structure-of-arrays,
// gpair[c * stride + p], c = 3 * node + axis (slave nodes 0..3, then master
// nodes 0..3), and reduced per node by the assembly kernels.
#include "mt_geometry.h"
#include "mt_internal.h"

namespace mt {

namespace {

constexpr int BSC = 64;

struct Map2 {
  double cu, cv, e1u, e1v, e2u, e2v, fu, fv;
};

__device__ __forceinline__ Map2 bilinear_map(const V2 X[4]) {
  Map2 m;
  m.cu = 0.25 * ((X[0].u + X[1].u) + (X[2].u + X[3].u));
  m.cv = 0.25 * ((X[0].v + X[1].v) + (X[2].v + X[3].v));
  m.e1u = 0.25 * ((X[1].u - X[0].u) + (X[2].u - X[3].u));
  m.e1v = 0.25 * ((X[1].v - X[0].v) + (X[2].v - X[3].v));
  m.e2u = 0.25 * ((X[2].u - X[1].u) + (X[3].u - X[0].u));
  m.e2v = 0.25 * ((X[2].v - X[1].v) + (X[3].v - X[0].v));
  m.fu = 0.25 * ((X[0].u - X[1].u) + (X[2].u - X[3].u));
  m.fv = 0.25 * ((X[0].v - X[1].v) + (X[2].v - X[3].v));
  return m;
}

// Reverse of xi = inverse map at point p: given xibar, returns
// lambda = J^-T xibar (then pbar += lambda, Xbar_k -= N_k lambda).
__device__ __forceinline__ void ift_adjoint(const Map2& m, double x1, double x2, double xb1, double xb2,
                                            double& l0, double& l1) {
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
// X = A1 + s (A2 - A1), s = cross(B1 - A1, dB) / cross(dA, dB).
__device__ __forceinline__ void intersect_adjoint(V2 A1, V2 A2, V2 B1, V2 B2, double xu, double xv, V2& a1,
                                                  V2& a2, V2& b1, V2& b2) {
#pragma clang fp contract(fast)
  const double dAu = A2.u - A1.u, dAv = A2.v - A1.v;
  const double dBu = B2.u - B1.u, dBv = B2.v - B1.v;
  const double wu = B1.u - A1.u, wv = B1.v - A1.v;
  const double den = dAu * dBv - dAv * dBu;
  const double scale = (fabs(dAu) + fabs(dAv)) * (fabs(dBu) + fabs(dBv));
  a1 = a2 = b1 = b2 = V2{0.0, 0.0};
  if (!(fabs(den) > 1e-14 * scale)) return;  // parallel lines: no defined intersection
  const double num = wu * dBv - wv * dBu;
  const double s = num / den;
  // X = A1 + s dA
  double A1u = xu, A1v = xv;
  double dAbu = s * xu, dAbv = s * xv;
  const double sb = xu * dAu + xv * dAv;
  const double numb = sb / den;
  const double denb = -sb * s / den;
  // num = wu dBv - wv dBu
  const double wbu = numb * dBv, wbv = -numb * dBu;
  double dBbu = -numb * wv, dBbv = numb * wu;
  // den = dAu dBv - dAv dBu
  dAbu += denb * dBv;
  dAbv += -denb * dBu;
  dBbu += -denb * dAv;
  dBbv += denb * dAu;
  // w = B1 - A1, dA = A2 - A1, dB = B2 - B1
  b1.u = wbu - dBbu; b1.v = wbv - dBbv;
  A1u += -wbu - dAbu; A1v += -wbv - dAbv;
  a1.u = A1u; a1.v = A1v;
  a2.u = dAbu; a2.v = dAbv;
  b2.u = dBbu; b2.v = dBbv;
}

__global__ __launch_bounds__(BSC) void k_pair_bwd(const double* __restrict__ xs, const double* __restrict__ ys,
                                                   const double* __restrict__ zs, const int32_t* __restrict__ cs,
                                                   int32_t n_s, const double* __restrict__ xm,
                                                   const double* __restrict__ ym, const double* __restrict__ zm,
                                                   const int32_t* __restrict__ cm, KParams kp, const int32_t* __restrict__ pair_s,
                                                   const int32_t* __restrict__ pair_m, int64_t n_pairs,
                                                   const int32_t* __restrict__ posD, const int32_t* __restrict__ posM,
                                                   const double* __restrict__ W_D, const double* __restrict__ W_M,
                                                   const double* __restrict__ w_g, double* __restrict__ gpair,
                                                   int64_t stride, Counters* cnt) {
  __shared__ double su[2 * CAP * BSC], sv[2 * CAP * BSC];
  __shared__ uint8_t sl[2 * CAP * BSC], se[2 * CAP * BSC];
  const int64_t p = (int64_t)blockIdx.x * BSC + threadIdx.x;
  if (p >= n_pairs) return;
  const int s = pair_s[p], m = pair_m[p];
  const int4 csn = load_conn(cs, s);
  double f[12], Xs[4][3], Xm[4][3];
  load_nodes(xs, ys, zs, csn, Xs);
  load_nodes(xm, ym, zm, load_conn(cm, m), Xm);
  slave_frame(Xs, f);
  LdsPoly<true> P{su + threadIdx.x, sv + threadIdx.x, sl + threadIdx.x, se + threadIdx.x, BSC};
  V2 S[4], Mn[4];
  double hs[4], hm[4];
  int mo[4], res, st;
  const int n = pair_geometry<true>(Xs, Xm, f, kp.eps_d, kp.eps_a, S, Mn, hs, hm, mo, P, res, st);

  double WD[16], WM[16], wg[4];
#pragma unroll
  for (int k = 0; k < 16; ++k) WD[k] = W_D[posD[(int64_t)k * n_s + s]];
#pragma unroll
  for (int k = 0; k < 16; ++k) WM[k] = W_M[posM[(int64_t)k * stride + p]];
  wg[0] = w_g[csn.x]; wg[1] = w_g[csn.y]; wg[2] = w_g[csn.z]; wg[3] = w_g[csn.w];

  // adjoints of the projected nodes and heights
  V2 Sb[4], Mb[4];
  double hsb[4], hmb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Sb[k] = V2{0.0, 0.0}; Mb[k] = V2{0.0, 0.0}; hsb[k] = 0.0; hmb[k] = 0.0;
  }
  // adjoints of the clip vertices live in the free LDS buffer
  const int vb = res ^ 1;
  for (int i = 0; i < n; ++i) { P.u[P.at(vb, i)] = 0.0; P.v[P.at(vb, i)] = 0.0; }

  double rl[7][3], rw[7];
  int nq;
  get_rule(kp.rule, rl, rw, nq);
  const Map2 ms = bilinear_map(S), mm = bilinear_map(Mn);
  unsigned long long noconv = 0;
  {
#pragma clang fp contract(fast)
    const double u0 = P.u[P.at(res, 0)], v0 = P.v[P.at(res, 0)];
    for (int i = 1; i + 1 < n; ++i) {
      const double u1 = P.u[P.at(res, i)], v1 = P.v[P.at(res, i)];
      const double u2 = P.u[P.at(res, i + 1)], v2 = P.v[P.at(res, i + 1)];
      const double At = 0.5 * ((u1 - u0) * (v2 - v0) - (v1 - v0) * (u2 - u0));
      double Atb = 0.0;
      double pb0u = 0.0, pb0v = 0.0, pb1u = 0.0, pb1v = 0.0, pb2u = 0.0, pb2v = 0.0;
      for (int q = 0; q < nq; ++q) {
        const double pu = rl[q][0] * u0 + rl[q][1] * u1 + rl[q][2] * u2;
        const double pv = rl[q][0] * v0 + rl[q][1] * v1 + rl[q][2] * v2;
        const double wA = rw[q] * At;
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
        for (int k = 0; k < 4; ++k) { nsb[k] = 0.0; nmb[k] = 0.0; }
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
        Atb += rw[q] * fval;
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
          Sb[k].u -= Ns[k] * ls0; Sb[k].v -= Ns[k] * ls1;
          Mb[k].u -= Nm[k] * lm0; Mb[k].v -= Nm[k] * lm1;
        }
        const double pbu = ls0 + lm0, pbv = ls1 + lm1;
        pb0u += rl[q][0] * pbu; pb0v += rl[q][0] * pbv;
        pb1u += rl[q][1] * pbu; pb1v += rl[q][1] * pbv;
        pb2u += rl[q][2] * pbu; pb2v += rl[q][2] * pbv;
      }
      // triangle area
      const double hA = 0.5 * Atb;
      P.u[P.at(vb, 0)] += pb0u + hA * (v1 - v2);
      P.v[P.at(vb, 0)] += pb0v + hA * (u2 - u1);
      P.u[P.at(vb, i)] += pb1u + hA * (v2 - v0);
      P.v[P.at(vb, i)] += pb1v - hA * (u2 - u0);
      P.u[P.at(vb, i + 1)] += pb2u - hA * (v1 - v0);
      P.v[P.at(vb, i + 1)] += pb2v + hA * (u1 - u0);
    }
  }

  // clip vertices -> projected nodes, through each vertex's provenance
  for (int i = 0; i < n; ++i) {
    const double xu = P.u[P.at(vb, i)], xv = P.v[P.at(vb, i)];
    const uint8_t lab = P.vl[P.at(res, i)];
    if (lab & 0x80) {
      const int k = lab & 3;
      Sb[k].u += xu;
      Sb[k].v += xv;
      continue;
    }
    const int la = lab >> 4, lb = lab & 15;
    // endpoints of the two lines; ids 0..3 slave edges, 4..7 master clip edges
    int ia[2], ib[2];
    bool ma, mb;
    if (la < 4) { ia[0] = la; ia[1] = (la + 1) & 3; ma = false; }
    else { ia[0] = mo[la - 4]; ia[1] = mo[(la - 3) & 3]; ma = true; }
    if (lb < 4) { ib[0] = lb; ib[1] = (lb + 1) & 3; mb = false; }
    else { ib[0] = mo[lb - 4]; ib[1] = mo[(lb - 3) & 3]; mb = true; }
    const V2 A1 = ma ? Mn[ia[0]] : S[ia[0]], A2 = ma ? Mn[ia[1]] : S[ia[1]];
    const V2 B1 = mb ? Mn[ib[0]] : S[ib[0]], B2 = mb ? Mn[ib[1]] : S[ib[1]];
    V2 a1, a2, b1, b2;
    intersect_adjoint(A1, A2, B1, B2, xu, xv, a1, a2, b1, b2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double du = 0.0, dv = 0.0;
      if (ia[0] == k) { du += a1.u; dv += a1.v; }
      if (ia[1] == k) { du += a2.u; dv += a2.v; }
      if (ma) { Mb[k].u += du; Mb[k].v += dv; } else { Sb[k].u += du; Sb[k].v += dv; }
      du = 0.0; dv = 0.0;
      if (ib[0] == k) { du += b1.u; dv += b1.v; }
      if (ib[1] == k) { du += b2.u; dv += b2.v; }
      if (mb) { Mb[k].u += du; Mb[k].v += dv; } else { Sb[k].u += du; Sb[k].v += dv; }
    }
  }

  // projection: (u, v, h) = ((X - x0).t1, (X - x0).t2, (X - x0).n0)
  double Xsb[4][3], Xmb[4][3], x0b[3] = {0, 0, 0}, t1b[3] = {0, 0, 0}, t2b[3] = {0, 0, 0}, n0b[3] = {0, 0, 0};
  {
#pragma clang fp contract(fast)
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
        const double g = ub * f[6 + d] + vbb * f[9 + d] + hb * f[3 + d];
        Xb[d] = g;
        x0b[d] -= g;
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
    // frame from the slave nodes
    double g1[3], g2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      g1[d] = 0.25 * (((Xs[1][d] - Xs[0][d]) + Xs[2][d]) - Xs[3][d]);
      g2[d] = 0.25 * (((Xs[2][d] + Xs[3][d]) - Xs[0][d]) - Xs[1][d]);
    }
    const double nn[3] = {g1[1] * g2[2] - g1[2] * g2[1], g1[2] * g2[0] - g1[0] * g2[2], g1[0] * g2[1] - g1[1] * g2[0]};
    const double ln = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    const double lg = sqrt(g1[0] * g1[0] + g1[1] * g1[1] + g1[2] * g1[2]);
    // t1 = g1 / |g1|, n0 = n / |n|
    const double tt = t1[0] * t1b[0] + t1[1] * t1b[1] + t1[2] * t1b[2];
    const double nt = n0[0] * n0b[0] + n0[1] * n0b[1] + n0[2] * n0b[2];
    double g1b[3], g2b[3], nb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      g1b[d] = (t1b[d] - t1[d] * tt) / lg;
      nb[d] = (n0b[d] - n0[d] * nt) / ln;
    }
    // n = g1 x g2
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
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      gpair[(int64_t)(3 * k + d) * stride + p] = Xsb[k][d];
      gpair[(int64_t)(12 + 3 * k + d) * stride + p] = Xmb[k][d];
    }
  if (noconv) atomicAdd(&cnt->noconv, noconv);
}

}  // namespace

hipError_t launch_pair_bwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp,
                           const int32_t* pair_s, const int32_t* pair_m, int64_t n_pairs, const int32_t* posD,
                           int32_t n_s_el, const int32_t* posM, const double* W_D, const double* W_M,
                           const double* w_g, double* gpair, int64_t stride, Counters* cnt, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  (void)n_s_el;
  k_pair_bwd<<<(unsigned)((n_pairs + BSC - 1) / BSC), BSC, 0, s>>>(S.x, S.y, S.z, S.conn, S.n_el, M.x, M.y, M.z,
                                                                   M.conn, kp, pair_s, pair_m, n_pairs, posD,
                                                                   posM, W_D, W_M, w_g, gpair, stride, cnt);
  return hipGetLastError();
}

}  // namespace mt
