// Per-pair kernels of Alg. 1: projection onto the slave auxiliary plane,
// clipping, cleanup (candidate pass), compaction into the pair list, and the
// segment-based integration of the local D, M and weighted-gap blocks.
//
// One lane owns one (slave, master) pair; its clip polygons live in LDS,
// lane-interleaved.  Local blocks are staged structure-of-arrays,
// blk[c * stride + p] for the 36 components c = [D 4x4 | M 4x4 | g 4], so
// the stores of a wavefront are coalesced.
#include <algorithm>

#include "mt_pair_eval.h"

namespace mt {

namespace {

constexpr int BSC = 64;   // clip / integrate block: one wavefront
constexpr int BS = 256;

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Slave data of candidate pass kernels: frame, projected slave polygon,
// its area and longest edge, precomputed per slave element.
__device__ __forceinline__ void load_slave_data(const double* __restrict__ sd, int32_t n_s, int s, double f[12],
                                                V2 S[4], double& As, double& hmax) {
#pragma unroll
  for (int k = 0; k < 12; ++k) f[k] = sd[(int64_t)k * n_s + s];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    S[k].u = sd[(int64_t)(12 + k) * n_s + s];
    S[k].v = sd[(int64_t)(16 + k) * n_s + s];
  }
  As = sd[(int64_t)20 * n_s + s];
  hmax = sd[(int64_t)21 * n_s + s];
}

// Totals of one stage of the build into the device state, clamped to the
// stage's capacity (the flag records an excess):
//  0 candidates: cand_off[n_s];
//  1 screened candidates: scr_off[n_s];
//  2 pairs: maybe_scan[n_screened].
__global__ void k_stage_totals(int stage, const int32_t* __restrict__ vec, int64_t idx, int64_t cap,
                               DevState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (stage == 2) idx = st->n_screened;
  const int64_t total = vec[idx];
  const bool over = total < 0 || total > cap;  // negative: the int32 scan overflowed (more than 2^31)
  const int32_t kept = (int32_t)(total < 0 ? 0 : (total < cap ? total : cap));
  if (stage == 0) {
    st->n_cand = (int32_t)(total < 0 ? 0x7fffffff : total);
    if (over) st->flags |= DS_CAP_CAND;
  } else if (stage == 1) {
    st->need_screened = (int32_t)(total < 0 ? 0x7fffffff : total);
    st->n_screened = kept;
    if (over) st->flags |= DS_CAP_SCREENED;
  } else {
    st->need_pairs = (int32_t)(total < 0 ? 0x7fffffff : total);
    st->n_pairs = kept;
    if (over) st->flags |= DS_CAP_PAIRS;
  }
}

// Screened candidates in candidate order: slave s writes its screened
// candidates from mlist[scr_off[s]] on, in order; a slave whose candidates
// were not stored (beyond their capacity) has none, and nothing is written
// at or past the capacity of the list.
__global__ __launch_bounds__(BS) void k_maybe_list(const int32_t* __restrict__ flag, const int32_t* __restrict__ cand_off,
                                                    const int32_t* __restrict__ scr_off, int32_t n_s,
                                                    int64_t cap_cand, int64_t cap, int32_t* __restrict__ mlist) {
  const int s = blockIdx.x * BS + threadIdx.x;
  if (s >= n_s) return;
  const int c0 = cand_off[s], c1 = cand_off[s + 1];
  if (c0 < 0 || (int64_t)c1 > cap_cand) return;
  int64_t o = scr_off[s];
  for (int c = c0; c < c1 && o < cap; ++c)
    if (flag[c]) mlist[o++] = c;
}

// Clip and cleanup of every screened candidate (LDS clip buffers with
// provenance): vertex count to nv[c], pair flag to flag2[i], polygon to
// entry i of the screened-candidate polygon buffer.
__global__ __launch_bounds__(BSC) void k_clip_screened(const double* __restrict__ sd, int32_t n_s,
                                                        const double* __restrict__ md, KParams kp, const int32_t* __restrict__ cand_s,
                                                        const int32_t* __restrict__ cand_m,
                                                        const int32_t* __restrict__ mlist,
                                                        const int32_t* __restrict__ n_dev,
                                                        uint8_t* __restrict__ nv_out, int32_t* __restrict__ flag2,
                                                        PolyBuf out, Counters* cnt) {
  __shared__ double su[CAPT * BSC], sv[CAPT * BSC];
  __shared__ uint8_t sl[CAPT * BSC], se[CAPT * BSC];
  const int64_t n_maybe = *n_dev;
  const int64_t tile = dyn_tile(blockIdx.x, n_maybe, BSC);
  if (tile < 0) return;
  const int64_t i = tile * BSC + threadIdx.x;
  if (i < n_maybe) {
    const int c = mlist[i];
    const int s = cand_s[c], m = cand_m[c];
    double f[12], Xm[4][3], As, hmax;
    V2 S[4];
    load_slave_data(sd, n_s, s, f, S, As, hmax);
    {
      const double2* src = reinterpret_cast<const double2*>(md + (int64_t)12 * m);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double2 t = src[k];
        Xm[(2 * k) / 3][(2 * k) % 3] = t.x;
        Xm[(2 * k + 1) / 3][(2 * k + 1) % 3] = t.y;
      }
    }
    V2 Mn[4];
    double hm[4];
    int st, res;
    bool flip;
    pair_screen(S, As, Xm, f, kp.eps_a, Mn, hm, flip, st);
    const LdsPoly<true> P{su + threadIdx.x, sv + threadIdx.x, sl + threadIdx.x, se + threadIdx.x, BSC};
    const int n = pair_clip_screened<true>(S, As, hmax, Mn, flip, kp.eps_d, kp.eps_a, P, res, st);
    nv_out[c] = (uint8_t)n;
    flag2[i] = n >= 3 ? 1 : 0;
    poly_store(P, res, n, flip, out, i);
    if (st & PS_OVERFLOW) atomicAdd(&cnt->overflow, 1ull);
  }
}

// Histogram of the candidates' clip vertex counts (computed on demand for
// the statistics): grid-stride over the counts, per-block LDS histogram.
__global__ __launch_bounds__(BS) void k_nv_hist(const uint8_t* __restrict__ nv, int64_t n,
                                                 unsigned long long* __restrict__ hist) {
  __shared__ unsigned int h[17];
  if (threadIdx.x < 17) h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const unsigned v = nv[i];
    atomicAdd(&h[v < 17 ? v : 16], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 17 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// Pair list from the screened candidates that are pairs; each pair's polygon
// stays where the clip stored it (entry slot[p] of the screened-candidate
// polygon buffer).  Pairs at or past the capacity are not stored.
__global__ __launch_bounds__(BS) void k_compact_pairs(const int32_t* __restrict__ cand_s,
                                                       const int32_t* __restrict__ cand_m,
                                                       const int32_t* __restrict__ mlist,
                                                       const int32_t* __restrict__ flag2,
                                                       const int32_t* __restrict__ scan2,
                                                       const int32_t* __restrict__ n_dev, int64_t cap,
                                                       const uint8_t* __restrict__ nf, int32_t* __restrict__ ps,
                                                       int32_t* __restrict__ pm, uint8_t* __restrict__ pnv,
                                                       int32_t* __restrict__ slot) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= *n_dev || !flag2[i]) return;
  const int64_t p = scan2[i];
  if (p >= cap) return;
  const int c = mlist[i];
  ps[p] = cand_s[c];
  pm[p] = cand_m[c];
  pnv[p] = (uint8_t)(nf[i] & 0x7f);
  slot[p] = (int32_t)i;
}

// First pair of each slave element: pairs among the screened candidates
// before its first one (both clamped to what was kept).
__global__ __launch_bounds__(BS) void k_pair_off(const int32_t* __restrict__ scr_off,
                                                  const int32_t* __restrict__ scan2, int32_t n_s,
                                                  const DevState* __restrict__ st, int32_t* __restrict__ pair_off) {
  const int s = blockIdx.x * BS + threadIdx.x;
  if (s > n_s) return;
  const int32_t i = min(scr_off[s], st->n_screened);
  pair_off[s] = min(scan2[i < 0 ? 0 : i], st->n_pairs);
}

// Clip polygon of every pair (projection, clip and cleanup in LDS), stored
// with its provenance for the integration and its reverse mode.
// A pair that is no longer a segment (or whose slave element degenerated)
// is counted in Counters::degen_poly.
__global__ __launch_bounds__(BSC) void k_pair_poly(MeshPtrs S, MeshPtrs M, KParams kp,
                                                    const int32_t* __restrict__ pair_s,
                                                    const int32_t* __restrict__ pair_m,
                                                    const int32_t* __restrict__ n_dev, PolyBuf out, Counters* cnt) {
  __shared__ double su[CAPT * BSC], sv[CAPT * BSC];
  __shared__ uint8_t sl[CAPT * BSC], se[CAPT * BSC];
  const int64_t n_pairs = *n_dev;
  const int64_t tile = dyn_tile(blockIdx.x, n_pairs, BSC);
  if (tile < 0) return;
  const int64_t p = tile * BSC + threadIdx.x;
  if (p >= n_pairs) return;
  double Xs[4][3], Xm[4][3];
  const int s = pair_s[p];
  load_nodes(S.x, S.y, S.z, load_conn(S.conn, s), Xs);
  load_nodes(M.x, M.y, M.z, load_conn(M.conn, pair_m[p]), Xm);
  const LdsPoly<true> P{su + threadIdx.x, sv + threadIdx.x, sl + threadIdx.x, se + threadIdx.x, BSC};
  const int st = store_pair_polygon(Xs, Xm, elem_nrm(S, s), kp, P, out, p);
  if (st) atomicAdd(&cnt->degen_poly, 1ull);
}

// Segment-based integration of every pair from its stored polygon; local
// blocks staged structure-of-arrays.  Blocks are mapped XCD-major:
// consecutive blocks are dispatched to different XCDs, so block b works on
// tile (b % 8) * ceil(nb / 8) + b / 8 and each XCD's L2 sees one contiguous
// eighth of the pair list (neighbouring pairs share slave nodes).
template <int NQ, bool DUAL>
__global__ __launch_bounds__(BSC) __attribute__((amdgpu_waves_per_eu(3))) void k_pair_fwd(MeshPtrs S, MeshPtrs M, KParams kp,
                                                   const int32_t* __restrict__ pair_s,
                                                   const int32_t* __restrict__ pair_m,
                                                   const int32_t* __restrict__ n_dev, PolyBuf poly,
                                                   double* __restrict__ blk, int64_t stride, Counters* cnt) {
  const int64_t n_pairs = *n_dev;
  const int64_t tile = dyn_tile(blockIdx.x, n_pairs, BSC);
  if (tile < 0) return;
  const int64_t p = tile * BSC + threadIdx.x;
  unsigned noconv = 0;
  if (p < n_pairs) {
    double D[16], Mv[16], g[4];
    const int s = pair_s[p];
    pair_forward<NQ, DUAL>(S, s, load_conn(S.conn, s), M, load_conn(M.conn, pair_m[p]), gpoly(poly, p),
                           gpoly_nf(poly, p), kp, D, Mv, g, noconv);
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

hipError_t launch_nv_hist(const uint8_t* nv, int64_t n, unsigned long long* hist, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<int64_t>(1024, (n + BS - 1) / BS);
  k_nv_hist<<<nb, BS, 0, s>>>(nv, n, hist);
  return hipGetLastError();
}

hipError_t launch_stage_totals(int stage, const int32_t* vec, int64_t idx, int64_t cap, DevState* st,
                               hipStream_t s) {
  k_stage_totals<<<1, 64, 0, s>>>(stage, vec, idx, cap, st);
  return hipGetLastError();
}

hipError_t launch_maybe_list(const int32_t* flag, const int32_t* cand_off, const int32_t* scr_off, int32_t n_s,
                             int64_t cap_cand, int64_t cap, int32_t* mlist, hipStream_t s) {
  if (n_s == 0) return hipSuccess;
  k_maybe_list<<<(unsigned)((n_s + BS - 1) / BS), BS, 0, s>>>(flag, cand_off, scr_off, n_s, cap_cand, cap, mlist);
  return hipGetLastError();
}

hipError_t launch_clip_screened(const double* mdata, const double* sdata, int32_t n_s, const KParams& kp,
                                const int32_t* cand_s, const int32_t* cand_m, const int32_t* mlist,
                                const int32_t* n_maybe, int64_t cap, uint8_t* nv, int32_t* flag2, const PolyBuf& out,
                                Counters* cnt, hipStream_t s) {
  if (cap == 0) return hipSuccess;
  k_clip_screened<<<xcd_grid((unsigned)((cap + BSC - 1) / BSC)), BSC, 0, s>>>(
      sdata, n_s, mdata, kp, cand_s, cand_m, mlist, n_maybe, nv, flag2, out, cnt);
  return hipGetLastError();
}

hipError_t launch_compact_pairs(const int32_t* cand_s, const int32_t* cand_m, const int32_t* mlist,
                                const int32_t* flag2, const int32_t* scan2, const int32_t* n_maybe, int64_t cap_maybe,
                                const uint8_t* nf, int32_t* pair_s, int32_t* pair_m, uint8_t* pair_nv,
                                int32_t* pair_slot, int64_t cap_pairs, hipStream_t s) {
  if (cap_maybe == 0) return hipSuccess;
  k_compact_pairs<<<(unsigned)((cap_maybe + BS - 1) / BS), BS, 0, s>>>(cand_s, cand_m, mlist, flag2, scan2, n_maybe,
                                                                       cap_pairs, nf, pair_s, pair_m, pair_nv,
                                                                       pair_slot);
  return hipGetLastError();
}

hipError_t launch_pair_off(const int32_t* scr_off, const int32_t* scan2, int32_t n_s, const DevState* st,
                           int32_t* pair_off, hipStream_t s) {
  k_pair_off<<<(n_s + 1 + BS - 1) / BS, BS, 0, s>>>(scr_off, scan2, n_s, st, pair_off);
  return hipGetLastError();
}

hipError_t launch_pair_poly(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                            const int32_t* pair_m, const int32_t* n_pairs, int64_t cap, const PolyBuf& poly,
                            Counters* cnt, hipStream_t s) {
  if (cap == 0) return hipSuccess;
  const unsigned nb = xcd_grid((unsigned)((cap + BSC - 1) / BSC));
  const MeshPtrs ms{S.x, S.y, S.z, S.conn, S.nrm}, mm{M.x, M.y, M.z, M.conn, nullptr};
  k_pair_poly<<<nb, BSC, 0, s>>>(ms, mm, kp, pair_s, pair_m, n_pairs, poly, cnt);
  return hipGetLastError();
}

hipError_t launch_pair_fwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                           const int32_t* pair_m, const int32_t* n_pairs, int64_t cap, const PolyBuf& poly,
                           double* blk, int64_t stride, Counters* cnt, hipStream_t s) {
  if (cap == 0) return hipSuccess;
  const unsigned nb = xcd_grid((unsigned)((cap + BSC - 1) / BSC));
  const MeshPtrs ms{S.x, S.y, S.z, S.conn, S.nrm}, mm{M.x, M.y, M.z, M.conn, nullptr};
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
