// Backward pass of the pair evaluation: gradient of
//   L = <W_D, D> + <W_M, M> + <w_g, g>
// with respect to the 24 nodal coordinates of each pair (the linearisation
// of the mortar terms required in every nonlinear iteration), staged
// structure-of-arrays gpair[c * stride + p], c = 3 * node + axis (slave nodes
// 0..3, then master nodes 0..3), and reduced per node by the assembly kernels.
#include "mt_pair_eval.h"

namespace mt {

namespace {

constexpr int BSC = 64;

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

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

// Upstream weights of pair p gathered through the position maps.
__device__ __forceinline__ void gather_weights(int s, int64_t p, int4 csn, const int32_t* __restrict__ posD,
                                               int32_t n_s, const int32_t* __restrict__ posM, int64_t stride,
                                               const double* __restrict__ W_D, const double* __restrict__ W_M,
                                               const double* __restrict__ w_g, double WD[16], double WM[16],
                                               double wg[4]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) WD[k] = W_D[posD[(int64_t)k * n_s + s]];
#pragma unroll
  for (int k = 0; k < 16; ++k) WM[k] = W_M[posM[(int64_t)k * stride + p]];
  wg[0] = w_g[csn.x];
  wg[1] = w_g[csn.y];
  wg[2] = w_g[csn.z];
  wg[3] = w_g[csn.w];
}

template <int NQ, bool DUAL, bool NODAL>
__global__ __launch_bounds__(BSC) __attribute__((amdgpu_waves_per_eu(2))) void k_pair_bwd(MeshPtrs S, int32_t n_s, MeshPtrs M, KParams kp,
                                                   const int32_t* __restrict__ pair_s,
                                                   const int32_t* __restrict__ pair_m, int64_t n_pairs, PolyBuf poly,
                                                   const int32_t* __restrict__ mpos,
                                                   const int32_t* __restrict__ posD, const int32_t* __restrict__ posM,
                                                   const double* __restrict__ W_D, const double* __restrict__ W_M,
                                                   const double* __restrict__ w_g, const double* __restrict__ blk,
                                                   double* __restrict__ gpair, double* __restrict__ gn0,
                                                   int64_t stride, Counters* cnt) {
  const int64_t p = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * BSC + threadIdx.x;
  unsigned noconv = 0;
  if (p < n_pairs) {
    const int s = pair_s[p];
    const int4 csn = load_conn(S.conn, s);
    if (DUAL) {
      // dependence of the dual coefficients on the slave nodes, from the
      // pair's dual blocks G = WD D^T + WM M^T + wg g^T; parked in the slave
      // slots of gpair during the sweep (the weights are gathered again for
      // the sweep rather than kept live through this part)
      double WD[16], WM[16], wg[4];
      gather_weights(s, p, csn, posD, n_s, posM, stride, W_D, W_M, w_g, WD, WM, wg);
      double G[16];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          double a = wg[j] * blk[(int64_t)(32 + m) * stride + p];
#pragma unroll
          for (int k = 0; k < 4; ++k)
            a += WD[4 * j + k] * blk[(int64_t)(4 * m + k) * stride + p] +
                 WM[4 * j + k] * blk[(int64_t)(16 + 4 * m + k) * stride + p];
          G[4 * j + m] = a;
        }
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
    double WD[16], WM[16], wg[4];
    {
      const int s2 = DUAL ? launder(s) : s;
      const int4 c2 = DUAL ? int4{launder(csn.x), launder(csn.y), launder(csn.z), launder(csn.w)} : csn;
      gather_weights(s2, p, c2, posD, n_s, posM, stride, W_D, W_M, w_g, WD, WM, wg);
    }
    double Xsb[4][3], Xmb[4][3], n0b[3];
    pair_backward<NQ, DUAL, NODAL>(S, s, csn, M, load_conn(M.conn, pair_m[p]), gpoly(poly, p), poly.nf[p], kp, WD, WM, wg,
                            Xsb, Xmb, n0b, noconv);
    if (NODAL)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double v = n0b[d];
        if (DUAL) v += gn0[(int64_t)d * stride + p];
        gn0[(int64_t)d * stride + p] = v;
      }
    const int64_t q = mpos[p];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double v = Xsb[k][d];
        if (DUAL) v += gpair[(int64_t)(3 * k + d) * stride + p];
        gpair[(int64_t)(3 * k + d) * stride + p] = v;
        gpair[(int64_t)(12 + 3 * k + d) * stride + q] = Xmb[k][d];
      }
  }
  const unsigned long long nc = wave_sum_u64(noconv);
  if (threadIdx.x == 0 && nc) atomicAdd(&cnt->noconv, nc);
}

}  // namespace

hipError_t launch_pair_bwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                           const int32_t* pair_m, int64_t n_pairs, const PolyBuf& poly, const int32_t* mpos,
                           const int32_t* posD, int32_t n_s_el,
                           const int32_t* posM, const double* W_D, const double* W_M, const double* w_g,
                           const double* blk, double* gpair, double* gn0, int64_t stride, Counters* cnt,
                           hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  const unsigned nb = xcd_grid((unsigned)((n_pairs + BSC - 1) / BSC));
  const MeshPtrs ms{S.x, S.y, S.z, S.conn, S.nrm}, mm{M.x, M.y, M.z, M.conn, nullptr};
  const bool nodal = S.nrm != nullptr;
  auto* k = kp.rule == 3
                ? (kp.dual ? (nodal ? k_pair_bwd<3, true, true> : k_pair_bwd<3, true, false>)
                           : (nodal ? k_pair_bwd<3, false, true> : k_pair_bwd<3, false, false>))
                : (kp.dual ? (nodal ? k_pair_bwd<7, true, true> : k_pair_bwd<7, true, false>)
                           : (nodal ? k_pair_bwd<7, false, true> : k_pair_bwd<7, false, false>));
  hipLaunchKernelGGL(k, dim3(nb), dim3(BSC), 0, s, ms, n_s_el, mm, kp, pair_s, pair_m, n_pairs, poly, mpos, posD, posM,
                     W_D, W_M, w_g, blk, gpair, gn0, stride, cnt);
  return hipGetLastError();
}

}  // namespace mt
