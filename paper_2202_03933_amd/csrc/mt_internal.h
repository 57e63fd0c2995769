// Internal host-side declarations of the mortar library: context layout,
// device buffers and the launch wrappers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "mortar_mi355x.h"

namespace mt {

// A region of the caller's workspace.  The library allocates no device
// memory: every buffer is carved from the workspace bound by mt_build_pairs
// (or mt_batch_build) at a fixed offset, so its size is known up front.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Carves buffers from a base pointer in a fixed order (256-byte aligned);
// with a null base it only sums their sizes.
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  void take(Buf& b, size_t bytes) {
    off = (off + 255) & ~size_t(255);
    if (bytes == 0) bytes = 16;
    b.p = base ? base + off : nullptr;
    b.bytes = bytes;
    off += bytes;
  }
};
struct DeviceMesh {
  const double* x = nullptr;
  const double* y = nullptr;
  const double* z = nullptr;
  const int32_t* conn = nullptr;  // [n_el][4]
  // slave side with the continuous normal field: element plane normals
  // [n_el][4] (unit normal, length of the sum it was normalised from)
  const double* nrm = nullptr;
  int32_t n_nodes = 0;
  int32_t n_el = 0;
  bool set = false;
};

// Cartesian search grid (cells indexed ix + nx * (iy + ny * iz)).
struct Grid {
  double lo[3];
  double inv_beta[3];
  double beta[3];
  int32_t n[3];
  int64_t ncells;
  double reach;  // delta + half the largest element box extent, padded: a master whose box
                 // touches the delta-enlarged slave box has its centre within this of the slave box
  // quantisation of box bounds for the candidate prefilter: level q of axis d
  // stands for qo[d] + q qu[d] (qu a power of two, q < 2^21)
  double qo[3];
  double qu[3];
};

// Device-side scalar reductions of the element preparation step.
struct PrepReduce {
  unsigned long long emax_bits;   // largest element box extent (non-negative double bits)
  unsigned long long edge_bits;   // longest slave element edge
  unsigned long long lo_key[3];   // node bounding box, order-preserving keys
  unsigned long long hi_key[3];
  int32_t bad_index;              // connectivity out of range
  int32_t pad;
};

// Device counters of the pair pipeline (hist: filled on demand from the
// candidates' vertex counts by mt_get_stats).
struct Counters {
  unsigned long long hist[17];
  unsigned long long noconv;
  unsigned long long overflow;
  unsigned long long degen_slave;
  unsigned long long degen_master;
  unsigned long long degen_poly;  // pair polygons lost after a coordinate update
};

// Device-side state of a build: the search grid and the data-dependent
// counts, which the kernels read so that the host need not (no read-back
// between the launches of a build).  Counts are clamped to the capacities;
// the flags say which capacity was exceeded.
enum : uint32_t {
  DS_CAP_CAND = 1u,      // more candidates than their capacity
  DS_CAP_SCREENED = 2u,  // more screened candidates than their capacity
  DS_CAP_PAIRS = 4u,     // more pairs than their capacity
  DS_NONFINITE = 8u,     // a coordinate is NaN or infinite
};
struct DevState {
  Grid grid;
  int32_t n_cand;         // candidates found (may exceed the capacity: DS_CAP_CAND)
  int32_t n_screened;     // screened candidates kept, <= capacity
  int32_t n_pairs;        // pairs kept, <= capacity
  int32_t need_screened;  // screened candidates among the kept candidates
  int32_t need_pairs;     // pairs among the kept screened candidates
  uint32_t flags;         // DS_* bits
  int32_t pad[2];
};

// Clip polygons of the pairs, structure-of-arrays over the pair index p:
// vertex i at u[i * stride + p], v[...], provenance lab[...] (slave node k:
// 0x80 | k; else (la << 4) | lb, the two lines the vertex lies on: 0..3 slave
// edges k -> k+1, 4..7 master clip edges); nf[p] = vertex count | flip << 7
// (flip: the projected master polygon is clockwise and is clipped as
// (M0, M3, M2, M1)).
struct PolyBuf {
  double* u;
  double* v;
  uint8_t* lab;
  uint8_t* nf;
  int64_t stride;
  const int32_t* slot;  // entry of pair p: slot[p] (nullptr: entry p)
  __host__ __device__ __forceinline__ int64_t at(int64_t p) const { return slot ? (int64_t)slot[p] : p; }
};

struct KParams {
  double delta;
  double eps_d;
  double eps_a;
  double newton_tol;
  int32_t newton_maxit;
  int32_t dual;
  int32_t rule;
  int32_t elem;  // 0: segment-based integration; n: element-based, n x n Gauss points
};

}  // namespace mt

struct mt_ctx {
  int device = 0;
  // phase timers
  bool timing = false;
  uint32_t timing_mask = ~0u;  // phases recorded while timing is on
  struct Interval { int phase; hipEvent_t a, b; };
  std::vector<Interval> intervals;
  std::vector<hipEvent_t> event_pool;
  double t_ms[MT_T_COUNT] = {};
  int64_t t_n[MT_T_COUNT] = {};
  mt_params params{};
  mt::DeviceMesh side[2];
  hipStream_t last_stream = nullptr;

  // the caller's workspace bound by the last mt_build_pairs and its layout
  void* ws = nullptr;
  size_t ws_bytes = 0;
  mt_capacity cap{};
  int32_t lay_n[4] = {-1, -1, -1, -1};  // slave/master nodes and elements the layout was made for
  int32_t lay_nodal = -1;
  uint64_t static_gen = 0;  // binding of the static scratch (mt_build_pairs_static), 0: none

  // state flags
  bool have_pairs = false;
  bool have_pattern = false;
  bool have_master_index = false;
  bool have_inc[2] = {false, false};  // node incidence of each side (depends on connectivity only)
  bool counts_known = false;  // n_cand .. nnz_M read back since the last build / pattern
  int64_t n_cand = 0, n_maybe = 0, n_pairs = 0, nnz_D = 0, nnz_M = 0;
  mt::Grid grid{};

  // element preparation
  mt::Buf box_s, box_m;    // [6][n_el] lo xyz, hi xyz
  mt::Buf sdata;           // [SD_N][n_s_el] precomputed slave frame and polygon
  mt::Buf mdata;           // [n_m_el][12] master element node coordinates
  mt::Buf reduce;          // PrepReduce
  mt::Buf prep_part;       // per-block partials of the element preparation
  mt::Buf counters;        // Counters
  mt::Buf state;           // DevState
  // binning
  mt::Buf keys, vals, keys_tmp, vals_tmp;  // [max(n_m_el, pair capacity)]
  mt::Buf cell_range;      // int2 [cell capacity]: sorted-master range of each cell
  mt::Buf sbox;            // [n_m_el][6] master boxes in cell order
  mt::Buf qbox;            // uint64 [n_m_el][2] their bounds quantised (candidate prefilter)
  // candidates
  mt::Buf cand_cnt;        // [n_s_el + 1]
  mt::Buf cand_tmp;        // [CTMP][n_s_el] candidates kept by the count pass
  mt::Buf cand_off;        // [n_s_el + 1]
  mt::Buf cand_s, cand_m;  // [candidate capacity]
  mt::Buf cand_nv;         // uint8 [candidate capacity]
  mt::Buf cand_flag;       // int32 [candidate capacity] 1 = screened in (to be clipped)
  mt::Buf scr_cnt;         // int32 [n_s + 1] screened-in candidates per slave element
  mt::Buf scr_off;         // int32 [n_s + 1] exclusive scan of scr_cnt
  // screened candidates (index i < DevState::n_screened)
  mt::Buf maybe_list;      // int32 [screened capacity] candidate index
  mt::Buf maybe_flag;      // int32 [screened capacity + 1] 1 = pair
  mt::Buf maybe_scan;      // int32 [screened capacity + 1] exclusive scan of maybe_flag
  mt::Buf mpoly_u, mpoly_v, mpoly_lab, mpoly_nf;  // their clip polygons (PolyBuf layout)
  int64_t mpoly_stride = 1;
  // pairs (index p < DevState::n_pairs; per-pair arrays have stride cap.pairs)
  mt::Buf pair_s, pair_m;  // [pair capacity]
  mt::Buf pair_nv;         // uint8 [pair capacity]
  mt::Buf pair_off;        // [n_s_el + 1] first pair of each slave element
  // pattern
  mt::Buf inc_cnt, inc_off, inc_cur, inc_list;     // slave node -> (element*4 + local)
  mt::Buf minc_cnt, minc_off, minc_cur, minc_list; // master node -> (element*4 + local)
  mt::Buf pat_keep;        // per-row column lists kept between the pattern passes
  mt::Buf pat_ecnt;        // int32 [n_s_el] master nodes of each slave element's pairs (-1: too many)
  mt::Buf pat_elist;       // int32 [EL][n_s_el] those master nodes, sorted
  mt::Buf D_cnt, D_rowptr, D_col;  // D_col: [16 n_s_el] (bound of nnz(D))
  mt::Buf M_cnt, M_rowptr, M_col;  // M_col: [16 pair capacity] (bound of nnz(M))
  mt::Buf posD;            // [16][n_s_el]
  mt::Buf posM;            // [16][pair capacity]
  // clip polygons of the pairs (mt::PolyBuf); valid for the coordinates of
  // generation poly_gen (coord_gen counts coordinate and pair-list changes)
  mt::Buf pair_slot;       // int32 [pair capacity] entry of each pair's polygon in the mpoly buffers
  int64_t coord_gen = 0, poly_gen = -1;
  int64_t pattern_gen = 0;  // counts completed mt_csr_pattern calls
  int64_t upload_gen = 0;   // counts mt_upload calls (connectivity possibly new)
  // forward / backward staging
  mt::Buf nrm_node;        // [n_s_nodes][4] nodal normals (continuous normal field)
  mt::Buf nrm_el;          // [n_s_el][4] element plane normals
  mt::Buf gn0;             // [3][pair capacity] dL/dn0 per pair
  mt::Buf nrm_sb, nrm_ub, nrm_cg;
  int64_t nrm_gen = -1;    // coord_gen of nrm_node / nrm_el
  // internal streams on which mt_csr_pattern computes the pair blocks (aux)
  // and the pairs-by-master index (aux2) while the pattern is built on the
  // caller's stream
  hipStream_t aux = nullptr;
  hipEvent_t aux_fork = nullptr, aux_join = nullptr;
  hipStream_t aux2 = nullptr;
  hipEvent_t aux2_join = nullptr;
  mt::Buf aux_scan;
  mt::Buf blk;             // [36][pair capacity]
  int64_t blk_gen = -1;    // coord_gen of the blocks in blk (mt_integrate)
  bool blk_pending = false;  // blocks computed by mt_csr_pattern, not yet assembled
  mt::Buf gpair;           // [24][pair capacity]
  mt::Buf mp_cnt, mp_cur;  // int32 [n_m_el + 1] counting-sort scratch of the pairs-by-master index
  mt::Buf mp_off;          // int32 [n_m_el + 1] range of each master element in that order
  mt::Buf mp_vals;         // uint32 [pair capacity] pairs sorted by master element
  mt::Buf mp_tmp;          // uint32 [pair capacity] merge scratch of that sort
  mt::Buf mp_pos;          // int32 [pair capacity]: rank of each pair in that order
  // scan / sort scratch
  mt::Buf scan_tmp, sort_hist;
  void* pin = nullptr;     // pinned host memory: read-backs and the connectivity check
};

namespace mt {

// ---- primitives (mt_prims.hip) ------------------------------------------
// Scratch (int32 elements) of a scan of up to n values.
int64_t scan_tmp_elems(int64_t n);
// Exclusive prefix sum of n int32 values into out[0..n]; out[n] = total.
// max_blocks > 0 caps the workgroups per launch (for a scan that runs beside
// a long kernel on another stream).
hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, const Buf& tmp, hipStream_t s,
                          int64_t max_blocks = 0);
// Two such scans of arrays of the same length (in into out, in2 into out2)
// in the launches of one; the same scratch.
hipError_t scan_exclusive2(const int32_t* in, int32_t* out, const int32_t* in2, int32_t* out2, int64_t n,
                           const Buf& tmp, hipStream_t s, int64_t max_blocks = 0);
// Workgroup cap of scans that run beside the pair kernels.
constexpr int64_t SCAN_BLOCKS_BESIDE = 256;
// The same over a count the device holds (*n_dev <= cap): out[0..cap] with
// the values from *n_dev on taken as zero, so out[*n_dev] = total.
hipError_t scan_exclusive_dev(const int32_t* in, int32_t* out, const int32_t* n_dev, int64_t cap, const Buf& tmp,
                              hipStream_t s);
// Histogram scratch (int32 elements) of a radix sort of up to n keys.
int64_t radix_hist_elems(int64_t n);
// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).
// Results end in (keys, vals); (keys_tmp, vals_tmp) are scratch of size n.
// With n_dev, only the first *n_dev <= n pairs are sorted.
// in_tmp: the input is in (keys_tmp, vals_tmp) instead (then an odd number
// of passes ends in (keys, vals) without a copy).
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                            const int32_t* n_dev, int bits, const Buf& hist, const Buf& scan_tmp, hipStream_t s,
                            bool in_tmp = false);
// Passes of radix_sort_pairs for `bits` key bits.
inline int radix_passes(int bits) { return (bits + 7) / 8; }
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t s);

// ---- search (mt_search.hip) ------------------------------------------------
// Element preparation of both sides in one launch; per-block partial
// reductions go to part[prep_blocks(S.n_el) + prep_blocks(M.n_el)][9] (slave
// blocks first), reduced by launch_prep_reduce.
int prep_blocks(int32_t n_el);
hipError_t launch_prep(const DeviceMesh& S, const DeviceMesh& M, double* box_s, double* sd, double* box_m,
                       double* md, double* part, hipStream_t s);
// The reductions of both sides, then the search grid (st->grid) from them,
// at most max_cells cells; flags non-finite coordinates.
hipError_t launch_prep_reduce(const double* part, int nb_s, int nb_m, PrepReduce* red, double delta,
                              double bin_size, int64_t max_cells, DevState* st, hipStream_t s);
// Master keys and values for the bin sort; the cell table cleared in the
// same launch.
hipError_t launch_master_keys(const double* box_m, int32_t n_m, const Grid* g, int64_t max_cells, uint32_t* keys,
                              uint32_t* vals, int2* range, hipStream_t s);
hipError_t launch_cell_ranges(const uint32_t* keys, const uint32_t* vals, int32_t n, const double* box_m,
                              const Grid* g, int2* range, double* sbox, uint64_t* qbox, hipStream_t s);
hipError_t launch_cand_count(const double* box_s, int32_t n_s, const double* sbox, const uint64_t* qbox,
                             const uint32_t* mvals, const int2* range, const Grid* g, double delta, int32_t* count,
                             int32_t* tmp, hipStream_t s);
// Candidates of slave s go to [off[s], off[s + 1]) of cand_s / cand_m / nv /
// flag, whose length is cap: a slave whose range ends beyond cap writes
// nothing and gets scr_cnt[s] = 0 (the stage totals flag the excess).
hipError_t launch_cand_fill(const double* box_s, int32_t n_s, const double* sbox, const uint32_t* mvals,
                            const int2* range, const Grid* g, double delta, const int32_t* tmp, const int32_t* off,
                            int32_t* cand_s, int32_t* cand_m, const double* sd, const double* md, double eps_a,
                            uint8_t* nv, int32_t* flag, int32_t* scr_cnt, Counters* cnt, int64_t cap,
                            hipStream_t s);
int cand_tmp_per_slave();

// ---- pairs (mt_pairs.hip) ----------------------------------------------------
// Stage totals into the device state: stage 0 candidates (vec[idx]), 1
// screened candidates (vec[idx]), 2 pairs (vec[st->n_screened]); clamped to
// cap, the excess flagged.
hipError_t launch_stage_totals(int stage, const int32_t* vec, int64_t idx, int64_t cap, DevState* st,
                               hipStream_t s);
// Histogram of clip vertex counts nv[0..n) added to hist[17].
hipError_t launch_nv_hist(const uint8_t* nv, int64_t n, unsigned long long* hist, hipStream_t s);
hipError_t launch_maybe_list(const int32_t* flag, const int32_t* cand_off, const int32_t* scr_off, int32_t n_s,
                             int64_t cap_cand, int64_t cap, int32_t* mlist, hipStream_t s);
hipError_t launch_clip_screened(const double* mdata, const double* sdata, int32_t n_s, const KParams& kp,
                                const int32_t* cand_s, const int32_t* cand_m, const int32_t* mlist,
                                const int32_t* n_maybe, int64_t cap, uint8_t* nv, int32_t* flag2, const PolyBuf& out,
                                Counters* cnt, hipStream_t s);
hipError_t launch_compact_pairs(const int32_t* cand_s, const int32_t* cand_m, const int32_t* mlist,
                                const int32_t* flag2, const int32_t* scan2, const int32_t* n_maybe, int64_t cap_maybe,
                                const uint8_t* nf, int32_t* pair_s, int32_t* pair_m, uint8_t* pair_nv,
                                int32_t* pair_slot, int64_t cap_pairs, hipStream_t s);
hipError_t launch_pair_off(const int32_t* scr_off, const int32_t* scan2, int32_t n_s, const DevState* st,
                           int32_t* pair_off, hipStream_t s);
// Kernels over the pairs take the device count n_pairs (<= cap, the stride
// of the per-pair arrays).
hipError_t launch_pair_poly(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                            const int32_t* pair_m, const int32_t* n_pairs, int64_t cap, const PolyBuf& poly,
                            Counters* cnt, hipStream_t s);
hipError_t launch_pair_fwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                           const int32_t* pair_m, const int32_t* n_pairs, int64_t cap, const PolyBuf& poly,
                           double* blk, int64_t blk_stride, Counters* cnt, hipStream_t s);

// ---- element-based integration (mt_elements.hip) -----------------------------
// Blocks of every pair by the kp.elem x kp.elem Gauss rule on each slave
// element (pairs sorted by slave; those of element e: pair_off[e] ..
// pair_off[e + 1]).
hipError_t launch_elem_fwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                           const int32_t* pair_m, const int32_t* pair_off, const int32_t* n_pairs, int64_t cap,
                           double* blk, int64_t stride, Counters* cnt, hipStream_t s);

// ---- assembly (mt_assemble.hip) ----------------------------------------------
hipError_t launch_inc_count(const int32_t* conn, int32_t n_el, int32_t* cnt, hipStream_t s);
hipError_t launch_inc_fill(const int32_t* conn, int32_t n_el, const int32_t* off, int32_t* cur,
                           int32_t* list, hipStream_t s);
hipError_t launch_inc_sort(const int32_t* off, int32_t n_nodes, int32_t* list, hipStream_t s);
hipError_t launch_pattern_rows(bool fill, const int32_t* inc_off, const int32_t* inc_list, int32_t n_nodes,
                               const int32_t* pair_off, const int32_t* pair_m, const int32_t* conn_s,
                               const int32_t* conn_m, int32_t* D_cnt, int32_t* M_cnt, const int32_t* D_rowptr,
                               const int32_t* M_rowptr, int32_t* D_col, int32_t* M_col, int32_t* keep,
                               int32_t n_s_el, int32_t* ecnt, int32_t* elist, hipStream_t s);
// CSR positions of every local block entry (posD[(4 j + k) * n_s_el + e],
// posM[(4 j + l) * cap + p]) from the filled column arrays.
hipError_t launch_pattern_positions(const int32_t* pair_s, const int32_t* pair_m, const int32_t* n_pairs,
                                    int64_t cap, const int32_t* conn_s, const int32_t* conn_m, int32_t n_s_el,
                                    const int32_t* pair_off, const int32_t* D_rowptr, const int32_t* D_col,
                                    const int32_t* M_rowptr, const int32_t* M_col, int32_t* posD, int32_t* posM,
                                    hipStream_t s);
hipError_t launch_elem_mlist(int32_t n_s_el, const int32_t* pair_off, const int32_t* pair_m, const int32_t* conn_m,
                             int32_t* ecnt, int32_t* elist, hipStream_t s);
int pattern_keep_per_row();
int pattern_elem_list();
hipError_t launch_assemble(const int32_t* inc_off, const int32_t* inc_list, int32_t n_nodes,
                           const int32_t* pair_off, const int32_t* D_rowptr, const int32_t* M_rowptr,
                           const int32_t* posD, int32_t n_s_el, const int32_t* posM, const double* blk,
                           int64_t blk_stride, double* D_val, double* M_val, double* gap, hipStream_t s);
hipError_t launch_grad_slave(const int32_t* inc_off, const int32_t* inc_list, int32_t n_nodes,
                             const int32_t* pair_off, const double* gpair, int64_t stride, double* gX,
                             hipStream_t s);
// Pairs by master element: off[m] .. off[m + 1] the range of master element
// m in vals (pair indices, ascending within the range), mpos[p] the rank of
// pair p in that order; cnt, cur scratch of n_m_el + 1, tmp of cap.
hipError_t launch_master_index(const int32_t* pair_m, const int32_t* n_pairs, int64_t cap, int32_t n_m_el,
                               int32_t* cnt, int32_t* cur, int32_t* off, uint32_t* vals, uint32_t* tmp, int32_t* mpos,
                               const Buf& scan_tmp, hipStream_t s);
hipError_t launch_grad_master(const int32_t* inc_off, const int32_t* inc_list, int32_t n_nodes,
                              const int32_t* mstart, const int32_t* mend, const double* gpair, int64_t stride,
                              double* gX, hipStream_t s);

// ---- backward (mt_backward.hip) ----------------------------------------------
// Backward of every pair: slave gradient components at gpair[c * stride + p],
// master components at gpair[(12 + c) * stride + mpos[p]].  With the dual
// basis, blk holds the pairs' dual blocks [36][stride] (the gradient through
// the dual coefficients needs them); unused otherwise.  With the continuous
// normal field (S.nrm), gn0[d * stride + p] receives the gradient with
// respect to the slave element's plane normal; else gn0 is null.
hipError_t launch_pair_bwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s, const int32_t* pair_m,
                           const int32_t* n_pairs, int64_t cap, const PolyBuf& poly, const int32_t* mpos, const int32_t* posD, int32_t n_s_el, const int32_t* posM,
                           const double* W_D, const double* W_M, const double* w_g, const double* blk,
                           double* gpair, double* gn0, int64_t stride, Counters* cnt, hipStream_t s);

// ---- continuous normal field (mt_normals.hip) --------------------------------
struct MeshPtrs;
// The slave side's normal field for the current coordinates (S.nrm set), or
// S.nrm = null with element normals.
int ensure_normals(mt_ctx* c, hipStream_t st);
// Nodal normals nn[4 a + 0..3] (unit normal, length before normalising) and
// element plane normals ne[4 e + 0..3] of the slave side.
hipError_t launch_normals(const DeviceMesh& S, const int32_t* inc_off, const int32_t* inc_list, double* nn,
                          double* ne, hipStream_t s);
// Adds to gX (SoA [3][n_nodes]) the gradient through the element plane
// normals, from dL/dn0 per pair (gn0[d * stride + p]); sb, ub, cg scratch of
// 4 n_el, 4 n_nodes and 12 n_el doubles.  With gX_at / S_at (device memory
// holding the output pointer / the slave coordinate pointers) those are read
// there when the kernels run, so that launches recorded in a graph follow a
// table updated per call.
hipError_t launch_normal_chain(const DeviceMesh& S, const int32_t* inc_off, const int32_t* inc_list,
                               const int32_t* pair_off, const double* gn0, int64_t stride, const double* nn,
                               const double* ne, double* sb, double* ub, double* cg, double* gX,
                               double* const* gX_at, const MeshPtrs* S_at, hipStream_t s);

KParams kparams(const mt_params& p);
// Node incidence of the master side and the pairs-by-master permutation
// (needed by the backward's master-node reduction); built once per pattern.
int ensure_master_index(mt_ctx* c, hipStream_t st);
// The same on a given stream with its own scan scratch (the master incidence
// must exist already).
int build_master_index(mt_ctx* c, hipStream_t st, const Buf& scan_tmp);
// Polygon buffers of the current pair list, and their view.
int ensure_poly(mt_ctx* c);
PolyBuf poly_buf(mt_ctx* c);
// Device count of pairs of the current build.
const int32_t* dev_n_pairs(mt_ctx* c);
// The counts of the last build / pattern on the host (synchronises the last
// stream when they have not been read back yet).
int host_counts(mt_ctx* c);
// MT_OK while the context's workspace still holds its build (MT_ESTATE once
// another context bound the static scratch this one was built in).
int ws_live(mt_ctx* c);

// ---- search of many interfaces (mt_batch_search) ------------------------------
// mt_build_pairs into the bound workspace and capacities, then mt_csr_pattern,
// without read-back (and without phase timers) on stream st; without `fork`
// every kernel on st (none on the context's internal streams; the
// pairs-by-master index is then built by the first backward).
int search_no_wait(mt_ctx* c, hipStream_t st, bool fork = true);
// The host side of search_no_wait(c, st, false) for a replay of a graph
// captured from it: the flags and generations that call sets.
void search_replayed(mt_ctx* c, hipStream_t st);
// What a captured search_no_wait(c, st, false) depends on besides device
// memory contents: workspace, capacities, parameters, mesh arrays, uploads.
std::string search_signature(const mt_ctx* c);
// mt_csr_pattern on stream st; without `blocks` the pair blocks of the coming
// integration are not computed beside it (a batch computes its own); without
// `fork` nothing runs on the internal streams.
int csr_pattern(mt_ctx* c, int64_t* nnz_D, int64_t* nnz_M, hipStream_t st, bool blocks, bool fork = true);
// The context's internal streams and their events, created on first use.
int ensure_aux(mt_ctx* c);

void set_error(const std::string& msg);

}  // namespace mt
