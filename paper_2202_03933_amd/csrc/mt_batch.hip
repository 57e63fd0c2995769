// Batched evaluation of many independent interfaces with one persistent
// launch per phase (the single-GPU analogue of the paper's independent
// interface load balancing, Sec. "Interface domain decompositions for
// dynamically evolving interfaces": work is distributed over all compute
// units regardless of which interface it belongs to).
//
// Work items are buckets of consecutive pairs of one instance, each taken by
// one wavefront.  They are split into 8 contiguous queues, one per XCD; the
// wavefronts of a block start on the queue of the block's XCD (blocks are
// dispatched round-robin over XCDs, so block b runs on XCD b % 8) and then
// take items from the other queues, so each XCD's L2 first sees one
// contiguous part of the meshes.  Queue counters are reset by a fill kernel,
// so the launch sequence can be captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <vector>

#include "mt_dual.h"
#include "mt_rows.h"

namespace mt {

constexpr int NQUEUE = 8;
constexpr int ROWS_PER_ITEM = 128;

struct BatchInst {
  MeshPtrs S, M;
  int32_t n_s_el, n_s_nodes, n_m_el, n_m_nodes;
  const int32_t* pair_s;
  const int32_t* pair_m;
  int64_t n_pairs;
  int64_t stride;  // of the per-pair arrays (the instance's pair capacity)
  const int32_t* pair_off;
  const int32_t* inc_off;
  const int32_t* inc_list;
  const int32_t* D_rowptr;
  const int32_t* M_rowptr;
  const int32_t* posD;
  const int32_t* posM;
  const int32_t* minc_off;
  const int32_t* minc_list;
  const int32_t* mstart;
  const int32_t* mend;
  const int32_t* mpos;
  double* blk;
  double* gpair;
  double* gn0;  // [3][stride] dL/dn0 per pair (continuous normal field), else null
  PolyBuf poly;
  Counters* cnt;  // the instance's counters (pairs lost after a coordinate update)
  // per call
  double* D_val;
  double* M_val;
  double* gap;
  const double* W_D;
  const double* W_M;
  const double* w_g;
  double* gXs;
  double* gXm;
  KParams kp;
};

struct WorkItem {
  int32_t inst, begin, end, pad;
};

namespace {

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__global__ void k_reset_queues(int32_t* qnext) {
  if (threadIdx.x < NQUEUE) qnext[threadIdx.x] = 0;
}

// Takes the next work item for this wavefront: its block's XCD queue first,
// then the others in order; returns -1 when every queue is drained.  Each
// wavefront fetches on its own (lane 0 takes the item, every lane reads it
// from lane 0), so no wavefront waits at a barrier for another's pairs.
// Uniform across the wavefront; all its lanes are active here.
__device__ __forceinline__ int next_item(const int32_t* __restrict__ qbeg, int32_t* qnext, int& qi) {
  const int home = blockIdx.x % NQUEUE;
  const bool lead = (threadIdx.x & 63) == 0;
  while (qi < NQUEUE) {
    const int q = (home + qi) % NQUEUE;
    int it = -1;
    if (lead) {
      const int k = atomicAdd(&qnext[q], 1);
      it = qbeg[q] + k < qbeg[q + 1] ? qbeg[q] + k : -1;
    }
    // lane 0's value, in a scalar register: the item and instance records
    // are then read with scalar loads and their pointers stay out of the
    // vector registers of the pair evaluation
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= 0) return it;
    ++qi;
  }
  return -1;
}

// Clip polygons of every pair of every instance (LDS clip buffers).
template <int BSZ>
__global__ __launch_bounds__(BSZ) void k_batch_poly(const BatchInst* __restrict__ inst,
                                                     const WorkItem* __restrict__ items,
                                                     const int32_t* __restrict__ qbeg, int32_t* qnext) {
  __shared__ double su[CAPT * BSZ], sv[CAPT * BSZ];
  __shared__ uint8_t sl[CAPT * BSZ], se[CAPT * BSZ];
  int qi = 0;
  const LdsPoly<true> P{su + threadIdx.x, sv + threadIdx.x, sl + threadIdx.x, se + threadIdx.x, BSZ};
  for (int it = next_item(qbeg, qnext, qi); it >= 0; it = next_item(qbeg, qnext, qi)) {
    const WorkItem w = items[it];
    const BatchInst& I = inst[w.inst];
    for (int64_t p = w.begin + (int)(threadIdx.x & 63); p < w.end; p += 64) {
      double Xs[4][3], Xm[4][3];
      load_nodes(I.S.x, I.S.y, I.S.z, load_conn(I.S.conn, I.pair_s[p]), Xs);
      load_nodes(I.M.x, I.M.y, I.M.z, load_conn(I.M.conn, I.pair_m[p]), Xm);
      if (store_pair_polygon(Xs, Xm, elem_nrm(I.S, I.pair_s[p]), I.kp, P, I.poly, p))
        atomicAdd(&I.cnt->degen_poly, 1ull);
    }
  }
}

template <int BSZ, int NQ, bool DUAL>
__global__ __launch_bounds__(BSZ) __attribute__((amdgpu_waves_per_eu(3))) void k_batch_fwd(const BatchInst* __restrict__ inst,
                                                    const WorkItem* __restrict__ items,
                                                    const int32_t* __restrict__ qbeg, int32_t* qnext, Counters* cnt) {
  unsigned noconv = 0;
  int qi = 0;
  for (int it = next_item(qbeg, qnext, qi); it >= 0; it = next_item(qbeg, qnext, qi)) {
    const WorkItem w = items[it];
    const BatchInst& I = inst[w.inst];
    for (int64_t p = w.begin + (int)(threadIdx.x & 63); p < w.end; p += 64) {
      double D[16], Mv[16], g[4];
      const int s = I.pair_s[p];
      pair_forward<NQ, DUAL>(I.S, s, load_conn(I.S.conn, s), I.M, load_conn(I.M.conn, I.pair_m[p]),
                             gpoly(I.poly, p), gpoly_nf(I.poly, p), I.kp, D, Mv, g, noconv);
      const int64_t st = I.stride;
#pragma unroll
      for (int k = 0; k < 16; ++k) I.blk[(int64_t)k * st + p] = D[k];
#pragma unroll
      for (int k = 0; k < 16; ++k) I.blk[(int64_t)(16 + k) * st + p] = Mv[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) I.blk[(int64_t)(32 + k) * st + p] = g[k];
    }
  }
  const unsigned long long nc = wave_sum_u64(noconv);
  if ((threadIdx.x & 63) == 0 && nc) atomicAdd(&cnt->noconv, nc);
}

// Upstream weights of pair p of instance I.
__device__ __forceinline__ void batch_weights(const BatchInst& I, int s, int4 c, int64_t p, double WD[16],
                                              double WM[16], double wg[4]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) WD[k] = I.W_D[I.posD[(int64_t)k * I.n_s_el + s]];
#pragma unroll
  for (int k = 0; k < 16; ++k) WM[k] = I.W_M[I.posM[(int64_t)k * I.stride + p]];
  wg[0] = I.w_g[c.x];
  wg[1] = I.w_g[c.y];
  wg[2] = I.w_g[c.z];
  wg[3] = I.w_g[c.w];
}

// Dual basis: gradient through the dual coefficients of every pair, from its
// dual blocks (computed by the forward launch that precedes this one), into
// the slave slots of gpair before the sweep (a launch of its own, so that its
// registers do not add to those of the sweep).
template <int BSZ, bool NODAL>
__global__ __launch_bounds__(BSZ) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_dual_adj(
    const BatchInst* __restrict__ inst, const WorkItem* __restrict__ items, const int32_t* __restrict__ qbeg,
    int32_t* qnext, Counters* cnt) {
  int qi = 0;
  for (int it = next_item(qbeg, qnext, qi); it >= 0; it = next_item(qbeg, qnext, qi)) {
    const WorkItem w = items[it];
    const BatchInst& I = inst[w.inst];
    for (int64_t p = w.begin + (int)(threadIdx.x & 63); p < w.end; p += 64) {
      const int s = I.pair_s[p];
      const int4 csn = load_conn(I.S.conn, s);
      double WD[16], WM[16], wg[4];
      batch_weights(I, s, csn, p, WD, WM, wg);
      pair_dual_adjoint<NODAL>(I.S, s, csn, WD, WM, wg, I.blk, I.stride, p, I.gpair, I.gn0);
    }
  }
}

template <int BSZ, int NQ, bool DUAL, bool NODAL>
__global__ __launch_bounds__(BSZ) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_bwd(const BatchInst* __restrict__ inst,
                                                    const WorkItem* __restrict__ items,
                                                    const int32_t* __restrict__ qbeg, int32_t* qnext, Counters* cnt) {
  unsigned noconv = 0;
  int qi = 0;
  for (int it = next_item(qbeg, qnext, qi); it >= 0; it = next_item(qbeg, qnext, qi)) {
    const WorkItem w = items[it];
    const BatchInst& I = inst[w.inst];
    const int64_t st = I.stride;
    for (int64_t p = w.begin + (int)(threadIdx.x & 63); p < w.end; p += 64) {
      const int s = I.pair_s[p];
      const int4 csn = load_conn(I.S.conn, s);
      double WD[16], WM[16], wg[4];
      batch_weights(I, s, csn, p, WD, WM, wg);
      double Xsb[4][3], Xmb[4][3], n0b[3];
      pair_backward<NQ, DUAL, NODAL>(I.S, s, csn, I.M, load_conn(I.M.conn, I.pair_m[p]), gpoly(I.poly, p),
                                     gpoly_nf(I.poly, p), I.kp, WD, WM, wg, Xsb, Xmb, n0b, noconv);
      if (NODAL)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double v = n0b[d];
          if (DUAL) v += I.gn0[(int64_t)d * st + p];
          I.gn0[(int64_t)d * st + p] = v;
        }
      const int64_t q = I.mpos[p];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double v = Xsb[k][d];
          if (DUAL) v += I.gpair[(int64_t)(3 * k + d) * st + p];
          I.gpair[(int64_t)(3 * k + d) * st + p] = v;
          I.gpair[(int64_t)(12 + 3 * k + d) * st + q] = Xmb[k][d];
        }
    }
  }
  const unsigned long long nc = wave_sum_u64(noconv);
  if ((threadIdx.x & 63) == 0 && nc) atomicAdd(&cnt->noconv, nc);
}

// Row phases: one block per item of ROWS_PER_ITEM rows of one instance.
constexpr int BATCH_ACAP = 32;  // per-thread row accumulator of the batched assembly

__global__ __launch_bounds__(ROWS_PER_ITEM) void k_batch_assemble(const BatchInst* __restrict__ inst,
                                                                   const WorkItem* __restrict__ items) {
  __shared__ double acc[BATCH_ACAP * ROWS_PER_ITEM];
  const WorkItem w = items[blockIdx.x];
  const int a = w.begin + threadIdx.x;
  if (a >= w.end) return;
  const BatchInst& I = inst[w.inst];
  assemble_row_acc(a, I.inc_off, I.inc_list, I.pair_off, I.D_rowptr, I.M_rowptr, I.posD, I.n_s_el, I.posM, I.blk,
                   I.stride, I.D_val, I.M_val, I.gap, acc + threadIdx.x, ROWS_PER_ITEM, BATCH_ACAP);
}

__global__ __launch_bounds__(ROWS_PER_ITEM) void k_batch_grad_rows(const BatchInst* __restrict__ inst,
                                                                    const WorkItem* __restrict__ items) {
  const WorkItem w = items[blockIdx.x];
  const int a = w.begin + threadIdx.x;
  if (a >= w.end) return;
  const BatchInst& I = inst[w.inst];
  if (w.pad == 0)
    grad_slave_row(a, I.n_s_nodes, I.inc_off, I.inc_list, I.pair_off, I.gpair, I.stride, I.gXs);
  else
    grad_master_row(a, I.n_m_nodes, I.minc_off, I.minc_list, I.mstart, I.mend, I.gpair, I.stride, I.gXm);
}

using PolyFn = void (*)(const BatchInst*, const WorkItem*, const int32_t*, int32_t*);
using FwdFn = void (*)(const BatchInst*, const WorkItem*, const int32_t*, int32_t*, Counters*);
using BwdFn = void (*)(const BatchInst*, const WorkItem*, const int32_t*, int32_t*, Counters*);

template <int BSZ>
FwdFn fwd_kernel(int nq, bool dual) {
  if (nq == 3) return dual ? k_batch_fwd<BSZ, 3, true> : k_batch_fwd<BSZ, 3, false>;
  return dual ? k_batch_fwd<BSZ, 7, true> : k_batch_fwd<BSZ, 7, false>;
}
template <int BSZ, bool NODAL>
BwdFn bwd_kernel(int nq, bool dual) {
  if (nq == 3) return dual ? k_batch_bwd<BSZ, 3, true, NODAL> : k_batch_bwd<BSZ, 3, false, NODAL>;
  return dual ? k_batch_bwd<BSZ, 7, true, NODAL> : k_batch_bwd<BSZ, 7, false, NODAL>;
}

PolyFn pick_poly(int bsz) {
  if (bsz == 256) return k_batch_poly<256>;
  if (bsz == 128) return k_batch_poly<128>;
  return k_batch_poly<64>;
}
FwdFn pick_fwd(int bsz, int nq, bool dual) {
  if (bsz == 256) return fwd_kernel<256>(nq, dual);
  if (bsz == 128) return fwd_kernel<128>(nq, dual);
  return fwd_kernel<64>(nq, dual);
}
BwdFn pick_dual(int bsz, bool nodal) {
  if (bsz == 256) return nodal ? k_batch_dual_adj<256, true> : k_batch_dual_adj<256, false>;
  if (bsz == 128) return nodal ? k_batch_dual_adj<128, true> : k_batch_dual_adj<128, false>;
  return nodal ? k_batch_dual_adj<64, true> : k_batch_dual_adj<64, false>;
}
BwdFn pick_bwd(int bsz, int nq, bool dual, bool nodal) {
  if (nodal) {
    if (bsz == 256) return bwd_kernel<256, true>(nq, dual);
    if (bsz == 128) return bwd_kernel<128, true>(nq, dual);
    return bwd_kernel<64, true>(nq, dual);
  }
  if (bsz == 256) return bwd_kernel<256, false>(nq, dual);
  if (bsz == 128) return bwd_kernel<128, false>(nq, dual);
  return bwd_kernel<64, false>(nq, dual);
}

// Blocks of kernel fn (block size bsz) resident on one compute unit, from
// its register and LDS footprint.
int resident_blocks(const void* fn, int bsz) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, bsz, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace
}  // namespace mt

struct mt_batch {
  int device = 0;
  int num_cu = 256;
  std::vector<mt_ctx*> ctxs;
  bool built = false;
  mt_batch_tuning tune{};
  int nq = 7;
  bool dual = false;
  bool nodal = false;
  std::vector<mt::BatchInst> h_inst;
  std::vector<int64_t> pattern_gen;  // each instance's pattern generation at mt_batch_build
  mt::BatchInst* pinned = nullptr;
  // regions of the caller's batch workspace
  mt::Buf d_inst, d_pitems, d_qbeg, d_qnext, d_ritems_s, d_ritems_sm, counters;
  int n_pitems = 0, n_ritems_s = 0, n_ritems_sm = 0;
  int64_t max_pitems = 0;  // pair items the workspace holds (buckets of at least MIN_BUCKET pairs)
  hipGraphExec_t g_fwd = nullptr, g_bwd = nullptr;
  hipStream_t g_fwd_stream = nullptr, g_bwd_stream = nullptr;
  // the search of all instances (mt_batch_search): instances spread over
  // internal streams forked from and joined back into the caller's
  static constexpr int NSEARCH = 8;
  hipStream_t s_stream[NSEARCH] = {};
  hipEvent_t s_fork = nullptr, s_join[NSEARCH] = {};
  // the search captured in a HIP graph: replayed while the capture stream
  // and every instance's search signature are unchanged
  hipGraphExec_t g_search = nullptr;
  hipStream_t g_search_stream = nullptr;
  std::vector<std::string> g_search_sig;
};

using namespace mt;

namespace {

int bfail(int code, const char* msg) {
  set_error(msg);
  return code;
}

#define B_HIP(call)                                              \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) {                                      \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
      return MT_EHIP;                                            \
    }                                                            \
  } while (0)

void drop_graphs(mt_batch* b) {
  if (b->g_fwd) (void)hipGraphExecDestroy(b->g_fwd);
  if (b->g_bwd) (void)hipGraphExecDestroy(b->g_bwd);
  b->g_fwd = b->g_bwd = nullptr;
}

// Pair work items (buckets of `bucket` consecutive pairs of one instance),
// split into NQUEUE contiguous queues of about equal pair counts.
int build_items(mt_batch* b, hipStream_t st) {
  const int bucket = std::max(1, b->tune.bucket);
  std::vector<WorkItem> items;
  int64_t total = 0;
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    const int64_t np = b->ctxs[i]->n_pairs;
    for (int64_t p = 0; p < np; p += bucket)
      items.push_back({(int32_t)i, (int32_t)p, (int32_t)std::min<int64_t>(np, p + bucket), 0});
    total += np;
  }
  std::vector<int32_t> qbeg(NQUEUE + 1, (int32_t)items.size());
  qbeg[0] = 0;
  int64_t acc = 0;
  int q = 1;
  for (size_t k = 0; k < items.size() && q < NQUEUE; ++k) {
    while (q < NQUEUE && acc >= (total * q) / NQUEUE) qbeg[q++] = (int32_t)k;
    acc += items[k].end - items[k].begin;
  }
  b->n_pitems = (int)items.size();
  if ((int64_t)items.size() > b->max_pitems) return bfail(MT_ECAPACITY, "batch: more work items than the workspace holds");
  B_HIP(hipStreamSynchronize(st));
  if (!items.empty())
    B_HIP(hipMemcpy(b->d_pitems.p, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
  B_HIP(hipMemcpy(b->d_qbeg.p, qbeg.data(), sizeof(int32_t) * (NQUEUE + 1), hipMemcpyHostToDevice));
  drop_graphs(b);
  return MT_OK;
}

// Current coordinate arrays of every instance (they may have been replaced
// with mt_update_coordinates since mt_batch_build); an instance whose pair
// list or pattern was rebuilt needs a new mt_batch_build.
int sync_instances(mt_batch* b, hipStream_t st) {
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    mt_ctx* c = b->ctxs[i];
    if (!c->have_pattern || c->pattern_gen != b->pattern_gen[i])
      return bfail(MT_ESTATE, "batch: an instance was rebuilt since mt_batch_build; build the batch again");
    if (b->nodal) {
      // the normal field of the current coordinates, before any polygon refresh
      int rc = ensure_normals(c, st);
      if (rc) return rc;
    }
    const DeviceMesh& S = c->side[0];
    const DeviceMesh& M = c->side[1];
    b->h_inst[i].S = MeshPtrs{S.x, S.y, S.z, S.conn, S.nrm};
    b->h_inst[i].M = MeshPtrs{M.x, M.y, M.z, M.conn, nullptr};
  }
  return MT_OK;
}

int upload_inst(mt_batch* b, hipStream_t st) {
  const size_t bytes = sizeof(BatchInst) * b->h_inst.size();
  if (std::memcmp(b->pinned, b->h_inst.data(), bytes) == 0) return MT_OK;
  B_HIP(hipStreamSynchronize(st));  // the previous copy from the pinned table has completed
  std::memcpy(b->pinned, b->h_inst.data(), bytes);
  B_HIP(hipMemcpyAsync(b->d_inst.p, b->pinned, bytes, hipMemcpyHostToDevice, st));
  return MT_OK;
}

int launch_poly(mt_batch* b, hipStream_t st) {
  const int bsz = b->tune.block;
  PolyFn f = pick_poly(bsz);
  const int grid = b->num_cu * resident_blocks(reinterpret_cast<const void*>(f), bsz);
  k_reset_queues<<<1, 64, 0, st>>>(b->d_qnext.as<int32_t>());
  B_HIP(hipGetLastError());
  hipLaunchKernelGGL(f, dim3(grid), dim3(bsz), 0, st, b->d_inst.as<BatchInst>(), b->d_pitems.as<WorkItem>(),
                     b->d_qbeg.as<int32_t>(), b->d_qnext.as<int32_t>());
  B_HIP(hipGetLastError());
  return MT_OK;
}

int launch_fwd(mt_batch* b, hipStream_t st) {
  const int bsz = b->tune.block;
  FwdFn f = pick_fwd(bsz, b->nq, b->dual);
  const int grid = b->num_cu * std::min(std::max(1, b->tune.blocks_per_cu),
                                        resident_blocks(reinterpret_cast<const void*>(f), bsz));
  k_reset_queues<<<1, 64, 0, st>>>(b->d_qnext.as<int32_t>());
  B_HIP(hipGetLastError());
  hipLaunchKernelGGL(f, dim3(grid), dim3(bsz), 0, st, b->d_inst.as<BatchInst>(), b->d_pitems.as<WorkItem>(),
                     b->d_qbeg.as<int32_t>(), b->d_qnext.as<int32_t>(), b->counters.as<Counters>());
  B_HIP(hipGetLastError());
  return MT_OK;
}

int launch_fwd_all(mt_batch* b, hipStream_t st) {
  int rc = launch_fwd(b, st);
  if (rc) return rc;
  if (b->n_ritems_s) {
    k_batch_assemble<<<b->n_ritems_s, ROWS_PER_ITEM, 0, st>>>(b->d_inst.as<BatchInst>(), b->d_ritems_s.as<WorkItem>());
    B_HIP(hipGetLastError());
  }
  return MT_OK;
}

int launch_bwd_all(mt_batch* b, hipStream_t st) {
  if (b->dual) {
    // the dual adjoint reads every pair's dual blocks
    int rc = launch_fwd(b, st);
    if (rc) return rc;
  }
  const int bsz = b->tune.block;
  if (b->dual) {
    BwdFn fd = pick_dual(bsz, b->nodal);
    const int gd = b->num_cu * resident_blocks(reinterpret_cast<const void*>(fd), bsz);
    k_reset_queues<<<1, 64, 0, st>>>(b->d_qnext.as<int32_t>());
    B_HIP(hipGetLastError());
    hipLaunchKernelGGL(fd, dim3(gd), dim3(bsz), 0, st, b->d_inst.as<BatchInst>(), b->d_pitems.as<WorkItem>(),
                       b->d_qbeg.as<int32_t>(), b->d_qnext.as<int32_t>(), b->counters.as<Counters>());
    B_HIP(hipGetLastError());
  }
  BwdFn f = pick_bwd(bsz, b->nq, b->dual, b->nodal);
  const int grid = b->num_cu * resident_blocks(reinterpret_cast<const void*>(f), bsz);
  k_reset_queues<<<1, 64, 0, st>>>(b->d_qnext.as<int32_t>());
  B_HIP(hipGetLastError());
  hipLaunchKernelGGL(f, dim3(grid), dim3(bsz), 0, st, b->d_inst.as<BatchInst>(), b->d_pitems.as<WorkItem>(),
                     b->d_qbeg.as<int32_t>(), b->d_qnext.as<int32_t>(), b->counters.as<Counters>());
  B_HIP(hipGetLastError());
  if (b->n_ritems_sm) {
    k_batch_grad_rows<<<b->n_ritems_sm, ROWS_PER_ITEM, 0, st>>>(b->d_inst.as<BatchInst>(),
                                                                 b->d_ritems_sm.as<WorkItem>());
    B_HIP(hipGetLastError());
  }
  if (b->nodal)
    // the chain through each instance's normal field (small kernels per
    // instance); the output pointer is read from the device instance table,
    // which is updated per call also when the launches replay from a graph
    for (size_t i = 0; i < b->ctxs.size(); ++i) {
      mt_ctx* c = b->ctxs[i];
      const char* rec = reinterpret_cast<const char*>(b->d_inst.p) + i * sizeof(BatchInst);
      double* const* gx_at = reinterpret_cast<double* const*>(rec + offsetof(BatchInst, gXs));
      const MeshPtrs* s_at = reinterpret_cast<const MeshPtrs*>(rec + offsetof(BatchInst, S));
      B_HIP(launch_normal_chain(c->side[0], c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(),
                                c->pair_off.as<int32_t>(), c->gn0.as<double>(), c->cap.pairs,
                                c->nrm_node.as<double>(), c->nrm_el.as<double>(), c->nrm_sb.as<double>(),
                                c->nrm_ub.as<double>(), c->nrm_cg.as<double>(), nullptr, gx_at, s_at, st));
    }
  return MT_OK;
}

// Recomputes the clip polygons of every instance (one persistent launch,
// outside any graph) when some instance's coordinates changed since its
// polygons were computed.
int refresh_polygons(mt_batch* b, hipStream_t st) {
  bool stale = false;
  for (mt_ctx* c : b->ctxs) stale = stale || c->poly_gen != c->coord_gen;
  if (!stale) return MT_OK;
  int rc = launch_poly(b, st);
  if (rc) return rc;
  for (mt_ctx* c : b->ctxs) c->poly_gen = c->coord_gen;
  return MT_OK;
}

// Capture `launch` on stream st into *exec once, then replay it.
template <class F>
int run_graph(hipGraphExec_t* exec, hipStream_t* cap_stream, hipStream_t st, F launch) {
  if (*exec && *cap_stream != st) {
    (void)hipGraphExecDestroy(*exec);
    *exec = nullptr;
  }
  if (!*exec) {
    hipGraph_t g = nullptr;
    B_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = launch();
    hipError_t e = hipStreamEndCapture(st, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return bfail(MT_EHIP, "hipStreamEndCapture failed");
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      *exec = nullptr;
      return bfail(MT_EHIP, "hipGraphInstantiate failed");
    }
    *cap_stream = st;
  }
  B_HIP(hipGraphLaunch(*exec, st));
  return MT_OK;
}

}  // namespace

extern "C" {

int mt_batch_create(mt_batch** out, int device) {
  if (!out) return bfail(MT_EINVAL, "mt_batch_create: null");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return bfail(MT_EINVAL, "mt_batch_create: no such device");
  mt_batch* b = new mt_batch();
  b->device = device;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
    b->num_cu = cu;
  *out = b;
  return MT_OK;
}

int mt_batch_destroy(mt_batch* b) {
  if (!b) return MT_OK;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  drop_graphs(b);
  if (b->g_search) (void)hipGraphExecDestroy(b->g_search);
  for (int k = 0; k < mt_batch::NSEARCH; ++k) {
    if (b->s_stream[k]) (void)hipStreamDestroy(b->s_stream[k]);
    if (b->s_join[k]) (void)hipEventDestroy(b->s_join[k]);
  }
  if (b->s_fork) (void)hipEventDestroy(b->s_fork);
  if (b->pinned) (void)hipHostFree(b->pinned);
  delete b;
  return MT_OK;
}

int mt_batch_add(mt_batch* b, mt_ctx* c, int32_t* index) {
  if (!b || !c) return bfail(MT_EINVAL, "mt_batch_add: null");
  if (c->device != b->device) return bfail(MT_EINVAL, "mt_batch_add: context on another device");
  if (!c->have_pattern) return bfail(MT_ESTATE, "mt_batch_add: run mt_build_pairs and mt_csr_pattern first");
  b->ctxs.push_back(c);
  b->built = false;
  drop_graphs(b);
  if (index) *index = (int32_t)b->ctxs.size() - 1;
  return MT_OK;
}

// Checks shared by the size query and the build.
static int batch_check(mt_batch* b, const char* who) {
  if (!b) return bfail(MT_EINVAL, who);
  if (b->ctxs.empty()) return bfail(MT_ESTATE, "batch: no instances");
  const mt_params& p0 = b->ctxs[0]->params;
  for (mt_ctx* c : b->ctxs) {
    if (!c->have_pattern) return bfail(MT_ESTATE, "batch: an instance has no pattern");
    if (c->params.rule != p0.rule || c->params.lm_basis != p0.lm_basis)
      return bfail(MT_EINVAL, "batch: all instances must share the rule and the basis");
    if (c->params.normals != p0.normals)
      return bfail(MT_EINVAL, "batch: all instances must share the normal field");
    if (c->params.element_rule != 0) return bfail(MT_EUNSUPPORTED, "batch: segment-based integration only");
    int rc = host_counts(c);
    if (rc) return rc;
  }
  return MT_OK;
}

constexpr int MIN_BUCKET = 64;  // smallest pair bucket (the autotuner's)

// Layout of the batch workspace for the current instances.
static void batch_layout(mt_batch* b, Arena& A, int64_t& max_pitems, int64_t& n_rs, int64_t& n_rsm) {
  max_pitems = 0;
  n_rs = n_rsm = 0;
  for (mt_ctx* c : b->ctxs) {
    max_pitems += (c->n_pairs + MIN_BUCKET - 1) / MIN_BUCKET;
    const int64_t rs = (c->side[0].n_nodes + ROWS_PER_ITEM - 1) / ROWS_PER_ITEM;
    n_rs += rs;
    n_rsm += rs + (c->side[1].n_nodes + ROWS_PER_ITEM - 1) / ROWS_PER_ITEM;
  }
  A.take(b->d_inst, sizeof(BatchInst) * b->ctxs.size());
  A.take(b->d_pitems, sizeof(WorkItem) * (size_t)std::max<int64_t>(1, max_pitems));
  A.take(b->d_qbeg, sizeof(int32_t) * (NQUEUE + 1));
  A.take(b->d_qnext, sizeof(int32_t) * NQUEUE);
  A.take(b->d_ritems_s, sizeof(WorkItem) * (size_t)std::max<int64_t>(1, n_rs));
  A.take(b->d_ritems_sm, sizeof(WorkItem) * (size_t)std::max<int64_t>(1, n_rsm));
  A.take(b->counters, sizeof(Counters));
}

int mt_batch_workspace_size(mt_batch* b, size_t* bytes) {
  if (!bytes) return bfail(MT_EINVAL, "mt_batch_workspace_size: null");
  int rc = batch_check(b, "mt_batch_workspace_size: null");
  if (rc) return rc;
  mt_batch probe;
  probe.ctxs = b->ctxs;
  Arena A;
  int64_t a, r1, r2;
  batch_layout(&probe, A, a, r1, r2);
  *bytes = A.off;
  return MT_OK;
}

int mt_batch_build(mt_batch* b, const mt_batch_tuning* tuning, void* ws, size_t ws_bytes, void* stream) {
  int rc = batch_check(b, "mt_batch_build: null");
  if (rc) return rc;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
    return bfail(MT_EINVAL, "mt_batch_build: workspace null or not 256-byte aligned");
  (void)hipSetDevice(b->device);
  hipStream_t st = (hipStream_t)stream;
  const mt_params& p0 = b->ctxs[0]->params;
  {
    Arena A;
    A.base = static_cast<char*>(ws);
    int64_t r1, r2;
    batch_layout(b, A, b->max_pitems, r1, r2);
    if (A.off > ws_bytes) {
      b->built = false;
      return bfail(MT_ECAPACITY, "mt_batch_build: workspace smaller than mt_batch_workspace_size");
    }
  }
  drop_graphs(b);
  b->nq = p0.rule;
  b->dual = p0.lm_basis == MT_BASIS_DUAL;
  b->nodal = p0.normals == MT_NORMALS_NODAL;
  mt_batch_tuning t{};
  if (tuning) t = *tuning;
  if (t.block != 64 && t.block != 128 && t.block != 256) t.block = 64;
  const int resident = resident_blocks(reinterpret_cast<const void*>(pick_fwd(t.block, p0.rule, p0.lm_basis == MT_BASIS_DUAL)), t.block);
  if (t.blocks_per_cu <= 0) t.blocks_per_cu = resident;
  t.blocks_per_cu = std::min(t.blocks_per_cu, resident);
  if (t.bucket <= 0) t.bucket = 4 * 64;
  t.bucket = std::max(t.bucket, MIN_BUCKET);
  b->tune = t;

  b->h_inst.assign(b->ctxs.size(), BatchInst{});
  b->pattern_gen.assign(b->ctxs.size(), 0);
  std::vector<WorkItem> rs, rsm;
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    mt_ctx* c = b->ctxs[i];
    {
      int rc2 = ensure_master_index(c, st);
      if (!rc2 && b->nodal) rc2 = ensure_normals(c, st);
      if (rc2) return rc2;
    }
    const DeviceMesh& S = c->side[0];
    const DeviceMesh& M = c->side[1];
    BatchInst& I = b->h_inst[i];
    b->pattern_gen[i] = c->pattern_gen;
    I.S = MeshPtrs{S.x, S.y, S.z, S.conn, S.nrm};
    I.M = MeshPtrs{M.x, M.y, M.z, M.conn};
    I.n_s_el = S.n_el;
    I.n_s_nodes = S.n_nodes;
    I.n_m_el = M.n_el;
    I.n_m_nodes = M.n_nodes;
    I.pair_s = c->pair_s.as<int32_t>();
    I.pair_m = c->pair_m.as<int32_t>();
    I.n_pairs = c->n_pairs;
    I.stride = c->cap.pairs;
    I.pair_off = c->pair_off.as<int32_t>();
    I.inc_off = c->inc_off.as<int32_t>();
    I.inc_list = c->inc_list.as<int32_t>();
    I.D_rowptr = c->D_rowptr.as<int32_t>();
    I.M_rowptr = c->M_rowptr.as<int32_t>();
    I.posD = c->posD.as<int32_t>();
    I.posM = c->posM.as<int32_t>();
    I.minc_off = c->minc_off.as<int32_t>();
    I.minc_list = c->minc_list.as<int32_t>();
    I.mstart = c->mp_off.as<int32_t>();
    I.mend = c->mp_off.as<int32_t>() + 1;
    I.mpos = c->mp_pos.as<int32_t>();
    I.blk = c->blk.as<double>();
    I.gpair = c->gpair.as<double>();
    I.gn0 = b->nodal ? c->gn0.as<double>() : nullptr;
    {
      int rc2 = ensure_poly(c);
      if (rc2) return rc2;
    }
    I.poly = poly_buf(c);
    I.cnt = c->counters.as<Counters>();
    I.kp = kparams(c->params);
    for (int r = 0; r < S.n_nodes; r += ROWS_PER_ITEM) {
      const WorkItem w{(int32_t)i, r, std::min(S.n_nodes, r + ROWS_PER_ITEM), 0};
      rs.push_back(w);
      rsm.push_back(w);
    }
    for (int r = 0; r < M.n_nodes; r += ROWS_PER_ITEM)
      rsm.push_back({(int32_t)i, r, std::min(M.n_nodes, r + ROWS_PER_ITEM), 1});
  }
  b->n_ritems_s = (int)rs.size();
  b->n_ritems_sm = (int)rsm.size();
  B_HIP(hipStreamSynchronize(st));
  if (!rs.empty()) B_HIP(hipMemcpy(b->d_ritems_s.p, rs.data(), sizeof(WorkItem) * rs.size(), hipMemcpyHostToDevice));
  if (!rsm.empty())
    B_HIP(hipMemcpy(b->d_ritems_sm.p, rsm.data(), sizeof(WorkItem) * rsm.size(), hipMemcpyHostToDevice));
  const size_t ib = sizeof(BatchInst) * b->h_inst.size();
  B_HIP(fill_i32(b->counters.as<int32_t>(), 0, sizeof(Counters) / 4, st));
  if (b->pinned) (void)hipHostFree(b->pinned);
  b->pinned = nullptr;
  B_HIP(hipHostMalloc((void**)&b->pinned, ib, hipHostMallocDefault));
  std::memcpy(b->pinned, b->h_inst.data(), ib);
  B_HIP(hipMemcpy(b->d_inst.p, b->pinned, ib, hipMemcpyHostToDevice));
  rc = build_items(b, st);
  if (rc) return rc;
  b->built = true;
  return MT_OK;
}

int mt_batch_forward(mt_batch* b, double* const* D_val, double* const* M_val, double* const* gap, int use_graph,
                     void* stream) {
  if (!b) return bfail(MT_EINVAL, "mt_batch_forward: null");
  if (!b->built) return bfail(MT_ESTATE, "mt_batch_forward: mt_batch_build first");
  if (!D_val || !M_val || !gap) return bfail(MT_EINVAL, "mt_batch_forward: null output table");
  hipStream_t st = (hipStream_t)stream;
  if (use_graph && st == nullptr) return bfail(MT_EINVAL, "mt_batch_forward: graph capture needs a created stream");
  (void)hipSetDevice(b->device);
  for (size_t i = 0; i < b->h_inst.size(); ++i) {
    b->h_inst[i].D_val = D_val[i];
    b->h_inst[i].M_val = M_val[i];
    b->h_inst[i].gap = gap[i];
  }
  int rc = sync_instances(b, st);
  if (rc) return rc;
  rc = upload_inst(b, st);
  if (rc) return rc;
  rc = refresh_polygons(b, st);
  if (rc) return rc;
  // the instances' block staging buffers are overwritten with the batch's
  // parameters: no longer those of their last mt_integrate
  for (mt_ctx* c : b->ctxs) {
    c->blk_gen = -1;
    c->blk_pending = false;
  }
  if (use_graph) return run_graph(&b->g_fwd, &b->g_fwd_stream, st, [&]() { return launch_fwd_all(b, st); });
  return launch_fwd_all(b, st);
}

int mt_batch_backward(mt_batch* b, const double* const* W_D, const double* const* W_M, const double* const* w_g,
                      double* const* gXs, double* const* gXm, int use_graph, void* stream) {
  if (!b) return bfail(MT_EINVAL, "mt_batch_backward: null");
  if (!b->built) return bfail(MT_ESTATE, "mt_batch_backward: mt_batch_build first");
  if (!W_D || !W_M || !w_g || !gXs || !gXm) return bfail(MT_EINVAL, "mt_batch_backward: null table");
  hipStream_t st = (hipStream_t)stream;
  if (use_graph && st == nullptr) return bfail(MT_EINVAL, "mt_batch_backward: graph capture needs a created stream");
  (void)hipSetDevice(b->device);
  for (size_t i = 0; i < b->h_inst.size(); ++i) {
    b->h_inst[i].W_D = W_D[i];
    b->h_inst[i].W_M = W_M[i];
    b->h_inst[i].w_g = w_g[i];
    b->h_inst[i].gXs = gXs[i];
    b->h_inst[i].gXm = gXm[i];
  }
  int rc = sync_instances(b, st);
  if (rc) return rc;
  rc = upload_inst(b, st);
  if (rc) return rc;
  rc = refresh_polygons(b, st);
  if (rc) return rc;
  if (b->dual)  // the launch recomputes the dual blocks into the staging buffers
    for (mt_ctx* c : b->ctxs) {
      c->blk_gen = -1;
      c->blk_pending = false;
    }
  if (use_graph) return run_graph(&b->g_bwd, &b->g_bwd_stream, st, [&]() { return launch_bwd_all(b, st); });
  return launch_bwd_all(b, st);
}

int mt_batch_search(mt_batch* b, int use_graph, void* stream) {
  if (!b) return bfail(MT_EINVAL, "mt_batch_search: null");
  if (b->ctxs.empty()) return bfail(MT_ESTATE, "mt_batch_search: no instances");
  hipStream_t st = (hipStream_t)stream;
  if (use_graph && st == nullptr) return bfail(MT_EINVAL, "mt_batch_search: graph capture needs a created stream");
  B_HIP(hipSetDevice(b->device));
  for (mt_ctx* c : b->ctxs) {
    if (!c->ws || c->static_gen != 0)
      return bfail(MT_ESTATE, "mt_batch_search: every instance needs its own workspace bound by mt_build_pairs");
    if (!c->side[0].set || !c->side[1].set) return bfail(MT_ESTATE, "mt_batch_search: an instance is not uploaded");
  }
  if (!b->s_fork) {
    B_HIP(hipEventCreateWithFlags(&b->s_fork, hipEventDisableTiming));
    for (int k = 0; k < mt_batch::NSEARCH; ++k) {
      B_HIP(hipStreamCreateWithFlags(&b->s_stream[k], hipStreamNonBlocking));
      B_HIP(hipEventCreateWithFlags(&b->s_join[k], hipEventDisableTiming));
    }
  }
  // Instances go round-robin onto the internal streams, forked from and
  // joined back into st.  Eagerly, each instance's pattern may fork again to
  // its own internal streams; in a graph it does not (one level of streams
  // under the capture: a capture that forked again from the forked streams
  // ended the process with a segmentation fault inside the capturing call).
  auto search_all = [&](bool fork) -> int {
    B_HIP(hipEventRecord(b->s_fork, st));
    for (int k = 0; k < mt_batch::NSEARCH; ++k) B_HIP(hipStreamWaitEvent(b->s_stream[k], b->s_fork, 0));
    int rc = MT_OK;
    for (size_t i = 0; i < b->ctxs.size() && rc == MT_OK; ++i)
      rc = search_no_wait(b->ctxs[i], b->s_stream[i % mt_batch::NSEARCH], fork);
    // joined back also after an error, so that st orders after whatever was
    // launched (and a capture ends on a joined graph)
    for (int k = 0; k < mt_batch::NSEARCH; ++k) {
      B_HIP(hipEventRecord(b->s_join[k], b->s_stream[k]));
      B_HIP(hipStreamWaitEvent(st, b->s_join[k], 0));
    }
    return rc;
  };
  int rc = MT_OK;
  if (!use_graph) {
    rc = search_all(true);
  } else {
    std::vector<std::string> sig;
    sig.reserve(b->ctxs.size());
    for (mt_ctx* c : b->ctxs) sig.push_back(search_signature(c));
    if (b->g_search && (b->g_search_stream != st || sig != b->g_search_sig)) {
      (void)hipGraphExecDestroy(b->g_search);
      b->g_search = nullptr;
    }
    if (b->g_search) {
      B_HIP(hipGraphLaunch(b->g_search, st));
      for (mt_ctx* c : b->ctxs) search_replayed(c, st);
    } else {
      // the host side of every call runs once here, while the kernels are
      // recorded; the graph launch below runs them
      hipGraph_t g = nullptr;
      B_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      rc = search_all(false);
      const hipError_t e = hipStreamEndCapture(st, &g);
      if (rc == MT_OK && e != hipSuccess) rc = bfail(MT_EHIP, "mt_batch_search: hipStreamEndCapture failed");
      if (rc == MT_OK) {
        const hipError_t ei = hipGraphInstantiate(&b->g_search, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
          b->g_search = nullptr;
          rc = bfail(MT_EHIP, "mt_batch_search: hipGraphInstantiate failed");
        }
      }
      if (g) (void)hipGraphDestroy(g);
      if (rc == MT_OK) {
        b->g_search_stream = st;
        b->g_search_sig = std::move(sig);
        B_HIP(hipGraphLaunch(b->g_search, st));
      } else {
        // nothing ran: the instances hold no valid pair list
        for (mt_ctx* c : b->ctxs) c->have_pairs = c->have_pattern = false;
      }
    }
  }
  // read-backs of the instances' counts wait on the caller's stream
  for (mt_ctx* c : b->ctxs) c->last_stream = st;
  return rc;
}

int mt_batch_autotune(mt_batch* b, mt_batch_tuning* out, void* stream) {
  if (!b) return bfail(MT_EINVAL, "mt_batch_autotune: null");
  if (!b->built) return bfail(MT_ESTATE, "mt_batch_autotune: mt_batch_build first");
  (void)hipSetDevice(b->device);
  hipStream_t st = (hipStream_t)stream;
  struct Cand { int block, bpc, bucket_mul; };
  std::vector<Cand> cands;
  for (int block : {64, 128, 256})
    for (int bpc : {1, 2, 4, 6, 8})
      for (int mul : {1, 2, 4, 8, 16})
        if (bpc <= resident_blocks(reinterpret_cast<const void*>(pick_fwd(block, b->nq, b->dual)), block))
          cands.push_back({block, bpc, mul});
  hipEvent_t e0, e1;
  B_HIP(hipEventCreate(&e0));
  B_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  mt_batch_tuning best_t = b->tune;
  for (const Cand& c : cands) {
    b->tune.block = c.block;
    b->tune.blocks_per_cu = c.bpc;
    b->tune.bucket = 64 * c.bucket_mul;  // pairs per wavefront item
    int rc = build_items(b, st);
    if (rc) return rc;
    rc = launch_fwd(b, st);  // warm-up
    if (rc) return rc;
    B_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r) {
      rc = launch_fwd(b, st);
      if (rc) return rc;
    }
    B_HIP(hipEventRecord(e1, st));
    B_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    B_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      best_t = b->tune;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->tune = best_t;
  int rc = build_items(b, st);
  if (rc) return rc;
  if (out) *out = best_t;
  return MT_OK;
}

}  // extern "C"
