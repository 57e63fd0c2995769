// Per-pair kernels of Alg. 1: projection onto the slave auxiliary plane,
// clipping, cleanup (candidate pass), compaction into the pair list, and the
// segment-based integration of the local D, M and weighted-gap blocks.
//
// One lane owns one (slave, master) pair; its clip polygons live in LDS,
// lane-interleaved.  Local blocks are staged structure-of-arrays,
// blk[c * stride + p] for the 36 components c = [D 4x4 | M 4x4 | g 4], so
// the stores of a wavefront are coalesced.
#include "mt_geometry.h"
#include "mt_internal.h"

namespace mt {

namespace {

constexpr int BSC = 64;   // clip / integrate block: one wavefront
constexpr int BS = 256;

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__global__ __launch_bounds__(BSC) void k_clip_count(const double* __restrict__ xs, const double* __restrict__ ys,
                                                     const double* __restrict__ zs, const int32_t* __restrict__ cs,
                                                     int32_t n_s, const double* __restrict__ xm,
                                                     const double* __restrict__ ym, const double* __restrict__ zm,
                                                     const int32_t* __restrict__ cm, KParams kp, const int32_t* __restrict__ cand_s,
                                                     const int32_t* __restrict__ cand_m, int64_t n_cand,
                                                     uint8_t* __restrict__ nv_out, int32_t* __restrict__ flag,
                                                     Counters* cnt) {
  __shared__ double su[2 * CAP * BSC], sv[2 * CAP * BSC];
  __shared__ unsigned int hist[20];
  if (threadIdx.x < 20) hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * BSC + threadIdx.x;
  if (c < n_cand) {
    const int s = cand_s[c], m = cand_m[c];
    double f[12], Xs[4][3], Xm[4][3];
    load_nodes(xs, ys, zs, load_conn(cs, s), Xs);
    load_nodes(xm, ym, zm, load_conn(cm, m), Xm);
    slave_frame(Xs, f);
    LdsPoly<false> P{su + threadIdx.x, sv + threadIdx.x, nullptr, nullptr, BSC};
    V2 S[4], Mn[4];
    double hs[4], hm[4];
    int mo[4], res, st;
    const int n = pair_geometry<false>(Xs, Xm, f, kp.eps_d, kp.eps_a, S, Mn, hs, hm, mo, P, res, st);
    nv_out[c] = (uint8_t)n;
    flag[c] = n >= 3 ? 1 : 0;
    atomicAdd(&hist[n], 1u);
    if (st & PS_DEGEN_SLAVE) atomicAdd(&hist[17], 1u);
    if (st & PS_DEGEN_MASTER) atomicAdd(&hist[18], 1u);
    if (st & PS_OVERFLOW) atomicAdd(&hist[19], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 20 && hist[threadIdx.x]) {
    const unsigned long long v = hist[threadIdx.x];
    if (threadIdx.x < 17) atomicAdd(&cnt->hist[threadIdx.x], v);
    else if (threadIdx.x == 17) atomicAdd(&cnt->degen_slave, v);
    else if (threadIdx.x == 18) atomicAdd(&cnt->degen_master, v);
    else atomicAdd(&cnt->overflow, v);
  }
}

__global__ __launch_bounds__(BS) void k_compact(const int32_t* __restrict__ cand_s, const int32_t* __restrict__ cand_m,
                                                 const uint8_t* __restrict__ nv, const int32_t* __restrict__ scan,
                                                 int64_t n_cand, int32_t* __restrict__ ps, int32_t* __restrict__ pm,
                                                 uint8_t* __restrict__ pnv) {
  const int64_t c = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (c >= n_cand) return;
  const uint8_t n = nv[c];
  if (n >= 3) {
    const int p = scan[c];
    ps[p] = cand_s[c];
    pm[p] = cand_m[c];
    pnv[p] = n;
  }
}

__global__ __launch_bounds__(BS) void k_pair_off(const int32_t* __restrict__ cand_off, const int32_t* __restrict__ scan,
                                                  int32_t n_s, int32_t* __restrict__ pair_off) {
  const int s = blockIdx.x * BS + threadIdx.x;
  if (s > n_s) return;
  pair_off[s] = scan[cand_off[s]];
}

// Segment-based integration of one pair: fan triangles (v0, v_i, v_{i+1})
// of the clip polygon, rule points p, slave / master parameter coordinates
// by the inverse bilinear maps, and the local blocks
//   D[j][k] += w Phi_j N_k(xi), M[j][l] += w Phi_j N_l(eta),
//   g[j]    += w Phi_j (sum_l N_l(eta) hm_l - sum_k N_k(xi) hs_k).
__global__ __launch_bounds__(BSC) void k_pair_fwd(const double* __restrict__ xs, const double* __restrict__ ys,
                                                   const double* __restrict__ zs, const int32_t* __restrict__ cs,
                                                   int32_t n_s, const double* __restrict__ xm,
                                                   const double* __restrict__ ym, const double* __restrict__ zm,
                                                   const int32_t* __restrict__ cm, KParams kp,
                                                   const int32_t* __restrict__ pair_s,
                                                   const int32_t* __restrict__ pair_m, int64_t n_pairs,
                                                   double* __restrict__ blk, int64_t stride, Counters* cnt) {
  __shared__ double su[2 * CAP * BSC], sv[2 * CAP * BSC];
  const int64_t p = (int64_t)blockIdx.x * BSC + threadIdx.x;
  unsigned long long noconv = 0;
  if (p < n_pairs) {
    const int s = pair_s[p], m = pair_m[p];
    double f[12], Xs[4][3], Xm[4][3];
    load_nodes(xs, ys, zs, load_conn(cs, s), Xs);
    load_nodes(xm, ym, zm, load_conn(cm, m), Xm);
    slave_frame(Xs, f);
    LdsPoly<false> P{su + threadIdx.x, sv + threadIdx.x, nullptr, nullptr, BSC};
    V2 S[4], Mn[4];
    double hs[4], hm[4];
    int mo[4], res, st;
    const int n = pair_geometry<false>(Xs, Xm, f, kp.eps_d, kp.eps_a, S, Mn, hs, hm, mo, P, res, st);
    double A[16];
    if (kp.dual) dual_coefficients(S, A);
    double D[16], M[16], g[4];
#pragma unroll
    for (int k = 0; k < 16; ++k) { D[k] = 0.0; M[k] = 0.0; }
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = 0.0;
    double rl[7][3], rw[7];
    int nq;
    get_rule(kp.rule, rl, rw, nq);
    {
#pragma clang fp contract(fast)
      const double u0 = P.u[P.at(res, 0)], v0 = P.v[P.at(res, 0)];
      for (int i = 1; i + 1 < n; ++i) {
        const double u1 = P.u[P.at(res, i)], v1 = P.v[P.at(res, i)];
        const double u2 = P.u[P.at(res, i + 1)], v2 = P.v[P.at(res, i + 1)];
        const double At = 0.5 * ((u1 - u0) * (v2 - v0) - (v1 - v0) * (u2 - u0));
        for (int q = 0; q < nq; ++q) {
          const double pu = rl[q][0] * u0 + rl[q][1] * u1 + rl[q][2] * u2;
          const double pv = rl[q][0] * v0 + rl[q][1] * v1 + rl[q][2] * v2;
          const double wA = rw[q] * At;
          double a1, a2, b1, b2;
          if (!inverse_bilinear(S, pu, pv, kp.newton_tol, kp.newton_maxit, a1, a2)) ++noconv;
          if (!inverse_bilinear(Mn, pu, pv, kp.newton_tol, kp.newton_maxit, b1, b2)) ++noconv;
          double Ns[4], Nm[4];
          shape4(a1, a2, Ns);
          shape4(b1, b2, Nm);
          double Phi[4];
          if (kp.dual) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              Phi[j] = A[j * 4 + 0] * Ns[0] + A[j * 4 + 1] * Ns[1] + A[j * 4 + 2] * Ns[2] + A[j * 4 + 3] * Ns[3];
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) Phi[j] = Ns[j];
          }
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
#pragma unroll
    for (int k = 0; k < 16; ++k) blk[(int64_t)k * stride + p] = D[k];
#pragma unroll
    for (int k = 0; k < 16; ++k) blk[(int64_t)(16 + k) * stride + p] = M[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) blk[(int64_t)(32 + k) * stride + p] = g[k];
  }
  noconv = wave_sum_u64(noconv);
  if (threadIdx.x == 0 && noconv) atomicAdd(&cnt->noconv, noconv);
}

}  // namespace

hipError_t launch_clip_count(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp,
                             const int32_t* cand_s, const int32_t* cand_m, int64_t n_cand, uint8_t* nv,
                             int32_t* flag, Counters* cnt, hipStream_t s) {
  if (n_cand == 0) return hipSuccess;
  k_clip_count<<<(unsigned)((n_cand + BSC - 1) / BSC), BSC, 0, s>>>(S.x, S.y, S.z, S.conn, S.n_el, M.x, M.y, M.z,
                                                                    M.conn, kp, cand_s, cand_m, n_cand, nv,
                                                                    flag, cnt);
  return hipGetLastError();
}

hipError_t launch_compact(const int32_t* cand_s, const int32_t* cand_m, const uint8_t* cand_nv, const int32_t* scan,
                          int64_t n_cand, int32_t* pair_s, int32_t* pair_m, uint8_t* pair_nv, hipStream_t s) {
  if (n_cand == 0) return hipSuccess;
  k_compact<<<(unsigned)((n_cand + BS - 1) / BS), BS, 0, s>>>(cand_s, cand_m, cand_nv, scan, n_cand, pair_s, pair_m,
                                                              pair_nv);
  return hipGetLastError();
}

hipError_t launch_pair_off(const int32_t* cand_off, const int32_t* scan, int32_t n_s, int32_t* pair_off,
                           hipStream_t s) {
  k_pair_off<<<(n_s + 1 + BS - 1) / BS, BS, 0, s>>>(cand_off, scan, n_s, pair_off);
  return hipGetLastError();
}

hipError_t launch_pair_fwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s, const int32_t* pair_m, int64_t n_pairs,
                           double* blk, int64_t stride, Counters* cnt, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  k_pair_fwd<<<(unsigned)((n_pairs + BSC - 1) / BSC), BSC, 0, s>>>(S.x, S.y, S.z, S.conn, S.n_el, M.x, M.y, M.z,
                                                                   M.conn, kp, pair_s, pair_m, n_pairs,
                                                                   blk, stride, cnt);
  return hipGetLastError();
}

}  // namespace mt
