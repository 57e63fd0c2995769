// Backward pass of the pair evaluation: gradient of
//   L = <W_D, D> + <W_M, M> + <w_g, g>
// with respect to the 24 nodal coordinates of each pair (the linearisation
// of the mortar terms required in every nonlinear iteration), staged
// structure-of-arrays gpair[c * stride + p], c = 3 * node + axis (slave nodes
// 0..3, then master nodes 0..3), and reduced per node by the assembly kernels.
#include "mt_dual.h"

namespace mt {

namespace {

constexpr int BSC = 64;

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
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

// Dual basis: the dependence of the dual coefficients on the slave nodes
// (pair_dual_adjoint), before the sweep.  A kernel of its own, so that its
// registers do not add to those of the sweep.
template <bool NODAL>
__global__ __launch_bounds__(BSC) __attribute__((amdgpu_waves_per_eu(2))) void k_pair_dual_adj(MeshPtrs S, int32_t n_s, const int32_t* __restrict__ pair_s,
                                                        const int32_t* __restrict__ n_dev,
                                                        const int32_t* __restrict__ posD,
                                                        const int32_t* __restrict__ posM,
                                                        const double* __restrict__ W_D, const double* __restrict__ W_M,
                                                        const double* __restrict__ w_g,
                                                        const double* __restrict__ blk, double* __restrict__ gpair,
                                                        double* __restrict__ gn0, int64_t stride) {
  const int64_t n_pairs = *n_dev;
  const int64_t tile = dyn_tile(blockIdx.x, n_pairs, BSC);
  if (tile < 0) return;
  const int64_t p = tile * BSC + threadIdx.x;
  if (p >= n_pairs) return;
  const int s = pair_s[p];
  const int4 csn = load_conn(S.conn, s);
  double WD[16], WM[16], wg[4];
  gather_weights(s, p, csn, posD, n_s, posM, stride, W_D, W_M, w_g, WD, WM, wg);
  pair_dual_adjoint<NODAL>(S, s, csn, WD, WM, wg, blk, stride, p, gpair, gn0);
}

template <int NQ, bool DUAL, bool NODAL>
__global__ __launch_bounds__(BSC) __attribute__((amdgpu_waves_per_eu(2))) void k_pair_bwd(MeshPtrs S, int32_t n_s, MeshPtrs M, KParams kp,
                                                   const int32_t* __restrict__ pair_s,
                                                   const int32_t* __restrict__ pair_m,
                                                   const int32_t* __restrict__ n_dev, PolyBuf poly,
                                                   const int32_t* __restrict__ mpos,
                                                   const int32_t* __restrict__ posD, const int32_t* __restrict__ posM,
                                                   const double* __restrict__ W_D, const double* __restrict__ W_M,
                                                   const double* __restrict__ w_g, double* __restrict__ gpair,
                                                   double* __restrict__ gn0, int64_t stride, Counters* cnt) {
  const int64_t n_pairs = *n_dev;
  const int64_t tile = dyn_tile(blockIdx.x, n_pairs, BSC);
  if (tile < 0) return;
  const int64_t p = tile * BSC + threadIdx.x;
  unsigned noconv = 0;
  if (p < n_pairs) {
    const int s = pair_s[p];
    const int4 csn = load_conn(S.conn, s);
    double WD[16], WM[16], wg[4];
    gather_weights(s, p, csn, posD, n_s, posM, stride, W_D, W_M, w_g, WD, WM, wg);
    double Xsb[4][3], Xmb[4][3], n0b[3];
    pair_backward<NQ, DUAL, NODAL>(S, s, csn, M, load_conn(M.conn, pair_m[p]), gpoly(poly, p), gpoly_nf(poly, p), kp, WD, WM, wg,
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
                           const int32_t* pair_m, const int32_t* n_pairs, int64_t cap, const PolyBuf& poly,
                           const int32_t* mpos,
                           const int32_t* posD, int32_t n_s_el,
                           const int32_t* posM, const double* W_D, const double* W_M, const double* w_g,
                           const double* blk, double* gpair, double* gn0, int64_t stride, Counters* cnt,
                           hipStream_t s) {
  if (cap == 0) return hipSuccess;
  const unsigned nb = xcd_grid((unsigned)((cap + BSC - 1) / BSC));
  const MeshPtrs ms{S.x, S.y, S.z, S.conn, S.nrm}, mm{M.x, M.y, M.z, M.conn, nullptr};
  const bool nodal = S.nrm != nullptr;
  auto* k = kp.rule == 3
                ? (kp.dual ? (nodal ? k_pair_bwd<3, true, true> : k_pair_bwd<3, true, false>)
                           : (nodal ? k_pair_bwd<3, false, true> : k_pair_bwd<3, false, false>))
                : (kp.dual ? (nodal ? k_pair_bwd<7, true, true> : k_pair_bwd<7, true, false>)
                           : (nodal ? k_pair_bwd<7, false, true> : k_pair_bwd<7, false, false>));
  if (kp.dual) {
    auto* kd = nodal ? k_pair_dual_adj<true> : k_pair_dual_adj<false>;
    hipLaunchKernelGGL(kd, dim3(nb), dim3(BSC), 0, s, ms, n_s_el, pair_s, n_pairs, posD, posM, W_D, W_M, w_g, blk,
                       gpair, gn0, stride);
  }
  hipLaunchKernelGGL(k, dim3(nb), dim3(BSC), 0, s, ms, n_s_el, mm, kp, pair_s, pair_m, n_pairs, poly, mpos, posD, posM,
                     W_D, W_M, w_g, gpair, gn0, stride, cnt);
  return hipGetLastError();
}

}  // namespace mt
