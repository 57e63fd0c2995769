// Per-pair kernels of Alg. 1: projection onto the slave auxiliary plane,
// clipping, cleanup (candidate pass), compaction into the pair list, and the
// segment-based integration of the local D, M and weighted-gap blocks.
//
// One lane owns one (slave, master) pair; its clip polygons live in LDS,
// lane-interleaved.  Local blocks are staged structure-of-arrays,
// blk[c * stride + p] for the 36 components c = [D 4x4 | M 4x4 | g 4], so
// the stores of a wavefront are coalesced.
#include "mt_pair_eval.h"

namespace mt {

namespace {

constexpr int BSC = 64;   // clip / integrate block: one wavefront
constexpr int CPT = 4;    // candidates per thread in the candidate pass
constexpr int BS = 256;

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Candidate pass: projection of the master element onto the precomputed
// slave plane, clip and cleanup; writes the vertex count (0: not a pair).
__global__ __launch_bounds__(BSC) void k_clip_count(const double* __restrict__ sd, int32_t n_s,
                                                     const double* __restrict__ xm, const double* __restrict__ ym,
                                                     const double* __restrict__ zm, const int32_t* __restrict__ cm,
                                                     KParams kp, const int32_t* __restrict__ cand_s,
                                                     const int32_t* __restrict__ cand_m, int64_t n_cand,
                                                     uint8_t* __restrict__ nv_out, int32_t* __restrict__ flag,
                                                     Counters* cnt) {
  __shared__ double su[CAPT * BSC], sv[CAPT * BSC];
  __shared__ unsigned int hist[20];
  if (threadIdx.x < 20) hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t tile = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * (BSC * CPT);
#pragma unroll 1
  for (int it = 0; it < CPT; ++it) {
  const int64_t c = tile + it * BSC + threadIdx.x;
  if (c < n_cand) {
    const int s = cand_s[c], m = cand_m[c];
    double f[12], Xm[4][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) f[k] = sd[(int64_t)k * n_s + s];
    V2 S[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      S[k].u = sd[(int64_t)(12 + k) * n_s + s];
      S[k].v = sd[(int64_t)(16 + k) * n_s + s];
    }
    const double As = sd[(int64_t)20 * n_s + s], hmax = sd[(int64_t)21 * n_s + s];
    load_nodes(xm, ym, zm, load_conn(cm, m), Xm);
    LdsPoly<false> P{su + threadIdx.x, sv + threadIdx.x, nullptr, nullptr, BSC};
    V2 Mn[4];
    double hm[4];
    int res, st;
    bool flip;
    const int n = pair_clip<false>(S, As, hmax, Xm, f, kp.eps_d, kp.eps_a, Mn, hm, flip, P, res, st);
    nv_out[c] = (uint8_t)n;
    flag[c] = n >= 3 ? 1 : 0;
    atomicAdd(&hist[n], 1u);
    if (st & PS_DEGEN_SLAVE) atomicAdd(&hist[17], 1u);
    if (st & PS_DEGEN_MASTER) atomicAdd(&hist[18], 1u);
    if (st & PS_OVERFLOW) atomicAdd(&hist[19], 1u);
  }
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

// Clip polygon of every pair (projection, clip and cleanup in LDS), stored
// with its provenance for the integration and its reverse mode.
__global__ __launch_bounds__(BSC) void k_pair_poly(MeshPtrs S, MeshPtrs M, KParams kp,
                                                    const int32_t* __restrict__ pair_s,
                                                    const int32_t* __restrict__ pair_m, int64_t n_pairs,
                                                    PolyBuf out) {
  __shared__ double su[CAPT * BSC], sv[CAPT * BSC];
  __shared__ uint8_t sl[CAPT * BSC], se[CAPT * BSC];
  const int64_t p = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * BSC + threadIdx.x;
  if (p >= n_pairs) return;
  double Xs[4][3], Xm[4][3];
  load_nodes(S.x, S.y, S.z, load_conn(S.conn, pair_s[p]), Xs);
  load_nodes(M.x, M.y, M.z, load_conn(M.conn, pair_m[p]), Xm);
  const LdsPoly<true> P{su + threadIdx.x, sv + threadIdx.x, sl + threadIdx.x, se + threadIdx.x, BSC};
  store_pair_polygon(Xs, Xm, kp, P, out, p);
}

// Segment-based integration of every pair from its stored polygon; local
// blocks staged structure-of-arrays.  Blocks are mapped XCD-major:
// consecutive blocks are dispatched to different XCDs, so block b works on
// tile (b % 8) * ceil(nb / 8) + b / 8 and each XCD's L2 sees one contiguous
// eighth of the pair list (neighbouring pairs share slave nodes).
template <int NQ, bool DUAL>
__global__ __launch_bounds__(BSC) __attribute__((amdgpu_waves_per_eu(3))) void k_pair_fwd(MeshPtrs S, MeshPtrs M, KParams kp,
                                                   const int32_t* __restrict__ pair_s,
                                                   const int32_t* __restrict__ pair_m, int64_t n_pairs,
                                                   PolyBuf poly, double* __restrict__ blk, int64_t stride,
                                                   Counters* cnt) {
  const int64_t p = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * BSC + threadIdx.x;
  unsigned noconv = 0;
  if (p < n_pairs) {
    double D[16], Mv[16], g[4];
    pair_forward<NQ, DUAL>(S, load_conn(S.conn, pair_s[p]), M, load_conn(M.conn, pair_m[p]), gpoly(poly, p),
                           poly.nf[p], kp, D, Mv, g, noconv);
#pragma unroll
    for (int k = 0; k < 16; ++k) blk[(int64_t)k * stride + p] = D[k];
#pragma unroll
    for (int k = 0; k < 16; ++k) blk[(int64_t)(16 + k) * stride + p] = Mv[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) blk[(int64_t)(32 + k) * stride + p] = g[k];
  }
  const unsigned long long nc = wave_sum_u64(noconv);
  if (threadIdx.x == 0 && nc) atomicAdd(&cnt->noconv, nc);
}

}  // namespace

hipError_t launch_clip_count(const DeviceMesh& S, const DeviceMesh& M, const double* sdata, const KParams& kp,
                             const int32_t* cand_s, const int32_t* cand_m, int64_t n_cand, uint8_t* nv,
                             int32_t* flag, Counters* cnt, hipStream_t s) {
  if (n_cand == 0) return hipSuccess;
  k_clip_count<<<xcd_grid((unsigned)((n_cand + BSC * CPT - 1) / (BSC * CPT))), BSC, 0, s>>>(sdata, S.n_el, M.x, M.y, M.z, M.conn,
                                                                              kp, cand_s, cand_m, n_cand, nv, flag,
                                                                              cnt);
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

hipError_t launch_pair_poly(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                            const int32_t* pair_m, int64_t n_pairs, const PolyBuf& poly, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  const unsigned nb = xcd_grid((unsigned)((n_pairs + BSC - 1) / BSC));
  const MeshPtrs ms{S.x, S.y, S.z, S.conn}, mm{M.x, M.y, M.z, M.conn};
  k_pair_poly<<<nb, BSC, 0, s>>>(ms, mm, kp, pair_s, pair_m, n_pairs, poly);
  return hipGetLastError();
}

hipError_t launch_pair_fwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                           const int32_t* pair_m, int64_t n_pairs, const PolyBuf& poly, double* blk, int64_t stride,
                           Counters* cnt, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  const unsigned nb = xcd_grid((unsigned)((n_pairs + BSC - 1) / BSC));
  const MeshPtrs ms{S.x, S.y, S.z, S.conn}, mm{M.x, M.y, M.z, M.conn};
  if (kp.rule == 3) {
    if (kp.dual) k_pair_fwd<3, true><<<nb, BSC, 0, s>>>(ms, mm, kp, pair_s, pair_m, n_pairs, poly, blk, stride, cnt);
    else k_pair_fwd<3, false><<<nb, BSC, 0, s>>>(ms, mm, kp, pair_s, pair_m, n_pairs, poly, blk, stride, cnt);
  } else {
    if (kp.dual) k_pair_fwd<7, true><<<nb, BSC, 0, s>>>(ms, mm, kp, pair_s, pair_m, n_pairs, poly, blk, stride, cnt);
    else k_pair_fwd<7, false><<<nb, BSC, 0, s>>>(ms, mm, kp, pair_s, pair_m, n_pairs, poly, blk, stride, cnt);
  }
  return hipGetLastError();
}

}  // namespace mt
