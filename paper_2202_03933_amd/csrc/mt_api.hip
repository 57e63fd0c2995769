// Host side of the C ABI declared in mortar_mi355x.h: context, argument
// checks, device buffers and the launch sequence of each entry point.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <string>

#include "mt_geometry.h"
#include "mt_internal.h"

namespace mt {

namespace {
thread_local std::string g_err;

// Makes the context's device current for the duration of a call.
struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    err = hipSetDevice(dev);
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return MT_EHIP;
}

#define MT_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

hipEvent_t take_event(mt_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one phase with two events on the stream when timing is enabled.
struct PhaseTimer {
  mt_ctx* c;
  int phase;
  hipStream_t st;
  hipEvent_t a = nullptr;
  PhaseTimer(mt_ctx* c_, int ph, hipStream_t s) : c(c_), phase(ph), st(s) {
    if (c->timing && ((c->timing_mask >> ph) & 1u) && (a = take_event(c)) != nullptr) (void)hipEventRecord(a, st);
  }
  ~PhaseTimer() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, st);
    c->intervals.push_back({phase, a, b});
  }
};

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

KParams kparams(const mt_params& p) {
  KParams k{};
  k.delta = p.delta;
  k.eps_d = p.eps_d;
  k.eps_a = p.eps_a;
  k.newton_tol = p.newton_tol;
  k.newton_maxit = p.newton_maxit;
  k.dual = p.lm_basis == MT_BASIS_DUAL ? 1 : 0;
  k.rule = p.rule;
  k.elem = p.element_rule;
  return k;
}

}  // namespace mt

using namespace mt;

namespace {

constexpr size_t PIN_BYTES = 1024;
constexpr int64_t CAP_MAX = (int64_t(1) << 31) - 1;

int64_t scan_max(const mt_ctx* c, const mt_capacity& cap) {
  const int64_t nm = c->side[1].n_el;
  const int64_t sortn = std::max<int64_t>(nm, cap.pairs);
  const int64_t hist = radix_hist_elems(sortn);
  int64_t m = std::max<int64_t>({(int64_t)c->side[0].n_el, (int64_t)c->side[0].n_nodes, (int64_t)c->side[1].n_nodes,
                                 nm, cap.screened, hist});
  return m + 1;
}

// Workspace layout for capacities `cap` and the current meshes and
// parameters: every buffer of a build, in a fixed order.
void layout(mt_ctx* c, const mt_capacity& cap, Arena& A) {
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const size_t ns = (size_t)S.n_el, nm = (size_t)M.n_el, nsn = (size_t)S.n_nodes, nmn = (size_t)M.n_nodes;
  const size_t C = (size_t)cap.candidates, SC = (size_t)cap.screened, P = (size_t)cap.pairs, G = (size_t)cap.cells;
  const bool nodal = c->params.normals == MT_NORMALS_NODAL;
  const size_t sortn = std::max(nm, P);
  const size_t hist = sizeof(int32_t) * (size_t)radix_hist_elems((int64_t)sortn);
  const size_t scan = sizeof(int32_t) * (size_t)scan_tmp_elems(scan_max(c, cap));
  A.take(c->reduce, sizeof(PrepReduce));
  A.take(c->counters, sizeof(Counters));
  A.take(c->state, sizeof(DevState));
  A.take(c->box_s, 48 * ns);
  A.take(c->box_m, 48 * nm);
  A.take(c->sdata, 8 * SD_N * ns);
  A.take(c->mdata, 96 * nm);
  A.take(c->prep_part, 72 * (size_t)(prep_blocks(S.n_el) + prep_blocks(M.n_el)));
  for (Buf* b : {&c->keys, &c->vals, &c->keys_tmp, &c->vals_tmp}) A.take(*b, 4 * sortn);
  A.take(c->cell_range, 8 * G);
  A.take(c->sbox, 48 * nm);
  A.take(c->qbox, 16 * nm);
  A.take(c->sort_hist, hist);
  A.take(c->scan_tmp, scan);
  A.take(c->aux_scan, scan);
  A.take(c->cand_cnt, 4 * (ns + 1));
  A.take(c->cand_off, 4 * (ns + 1));
  A.take(c->cand_tmp, 4 * (size_t)cand_tmp_per_slave() * ns);
  A.take(c->cand_s, 4 * C);
  A.take(c->cand_m, 4 * C);
  A.take(c->cand_nv, C);
  A.take(c->cand_flag, 4 * C);
  A.take(c->scr_cnt, 4 * (ns + 1));
  A.take(c->scr_off, 4 * (ns + 1));
  A.take(c->maybe_list, 4 * SC);
  A.take(c->maybe_flag, 4 * (SC + 1));
  A.take(c->maybe_scan, 4 * (SC + 1));
  A.take(c->mpoly_u, 8 * CAP0 * SC);
  A.take(c->mpoly_v, 8 * CAP0 * SC);
  A.take(c->mpoly_lab, CAP0 * SC);
  A.take(c->mpoly_nf, SC);
  A.take(c->pair_s, 4 * P);
  A.take(c->pair_m, 4 * P);
  A.take(c->pair_nv, P);
  A.take(c->pair_slot, 4 * P);
  A.take(c->pair_off, 4 * (ns + 1));
  for (Buf* b : {&c->inc_cnt, &c->inc_off, &c->inc_cur}) A.take(*b, 4 * (nsn + 1));
  A.take(c->inc_list, 16 * ns);
  for (Buf* b : {&c->minc_cnt, &c->minc_off, &c->minc_cur}) A.take(*b, 4 * (nmn + 1));
  A.take(c->minc_list, 16 * nm);
  A.take(c->pat_keep, 4 * (size_t)pattern_keep_per_row() * nsn);
  A.take(c->pat_ecnt, 4 * ns);
  A.take(c->pat_elist, 4 * (size_t)pattern_elem_list() * ns);
  for (Buf* b : {&c->D_cnt, &c->M_cnt, &c->D_rowptr, &c->M_rowptr}) A.take(*b, 4 * (nsn + 1));
  A.take(c->D_col, 64 * ns);
  A.take(c->M_col, 64 * P);
  A.take(c->posD, 64 * ns);
  A.take(c->posM, 64 * P);
  if (nodal) {
    A.take(c->nrm_node, 32 * nsn);
    A.take(c->nrm_el, 32 * ns);
    A.take(c->gn0, 24 * P);
    A.take(c->nrm_sb, 32 * ns);
    A.take(c->nrm_ub, 32 * nsn);
    A.take(c->nrm_cg, 96 * ns);
  } else {
    for (Buf* b : {&c->nrm_node, &c->nrm_el, &c->gn0, &c->nrm_sb, &c->nrm_ub, &c->nrm_cg}) *b = Buf{};
  }
  A.take(c->blk, 288 * P);
  A.take(c->gpair, 192 * P);
  A.take(c->mp_cnt, 4 * (nm + 1));
  A.take(c->mp_cur, 4 * (nm + 1));
  A.take(c->mp_off, 4 * (nm + 1));
  A.take(c->mp_vals, 4 * P);
  A.take(c->mp_tmp, 4 * P);
  A.take(c->mp_pos, 4 * P);
}

int check_cap(const mt_capacity& cap) {
  for (int64_t v : {cap.candidates, cap.screened, cap.pairs, cap.cells})
    if (v < 1 || v > CAP_MAX) return fail(MT_EINVAL, "capacity out of range (1 .. 2^31 - 1)");
  return MT_OK;
}

mt_capacity default_cap(const mt_ctx* c) {
  const int64_t e = (int64_t)c->side[0].n_el + c->side[1].n_el;
  mt_capacity k;
  k.candidates = std::min<int64_t>(CAP_MAX, 20 * e + 1024);
  k.screened = std::min<int64_t>(CAP_MAX, (5 * e) / 2 + 1024);
  k.pairs = k.screened;
  k.cells = std::min<int64_t>(int64_t(1) << 24, std::max<int64_t>(int64_t(1) << 16, 64 * e));
  return k;
}

// Small device-to-host reads through the pinned staging buffer of the
// context: one stream synchronisation for all of them.
struct ReadBack {
  void* dst;
  const void* src;
  size_t bytes;
};

hipError_t read_back(mt_ctx* c, std::initializer_list<ReadBack> items, hipStream_t st) {
  size_t off = 0;
  for (const ReadBack& r : items) {
    off = (off + 15) & ~size_t(15);
    if (off + r.bytes > PIN_BYTES) return hipErrorInvalidValue;
    hipError_t e = hipMemcpyAsync(static_cast<char*>(c->pin) + off, r.src, r.bytes, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    off += r.bytes;
  }
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  off = 0;
  for (const ReadBack& r : items) {
    off = (off + 15) & ~size_t(15);
    std::memcpy(r.dst, static_cast<const char*>(c->pin) + off, r.bytes);
    off += r.bytes;
  }
  return hipSuccess;
}

// Status of the device checks from the read-back state and counters.
int device_status(const DevState& ds, const Counters& hc, bool with_noconv) {
  if (ds.flags & DS_NONFINITE) return fail(MT_EINVAL, "a coordinate is NaN or infinite");
  if (ds.flags & (DS_CAP_CAND | DS_CAP_SCREENED | DS_CAP_PAIRS))
    return fail(MT_ECAPACITY, std::string("capacity exceeded:") + ((ds.flags & DS_CAP_CAND) ? " candidates" : "") +
                                  ((ds.flags & DS_CAP_SCREENED) ? " screened" : "") +
                                  ((ds.flags & DS_CAP_PAIRS) ? " pairs" : "") + " (see mt_required_capacity)");
  if (hc.degen_slave || hc.overflow)
    return fail(MT_EDEGENERATE, "degenerate slave element or clip capacity exceeded");
  if (hc.degen_poly) return fail(MT_EDEGENERATE, "pairs lost after a coordinate update (no longer segments)");
  if (with_noconv && hc.noconv) return fail(MT_ENOCONV, "an inverse bilinear map did not converge");
  return MT_OK;
}

// Node -> (element * 4 + local index) incidence, sorted per node.
int build_incidence(mt_ctx* c, const DeviceMesh& mesh, Buf& cntb, Buf& offb, Buf& curb, Buf& listb,
                    hipStream_t st) {
  const int32_t n = mesh.n_nodes;
  MT_HIP(fill_i32(cntb.as<int32_t>(), 0, (int64_t)n + 1, st));
  MT_HIP(fill_i32(curb.as<int32_t>(), 0, (int64_t)n + 1, st));
  MT_HIP(launch_inc_count(mesh.conn, mesh.n_el, cntb.as<int32_t>(), st));
  MT_HIP(scan_exclusive(cntb.as<int32_t>(), offb.as<int32_t>(), n, c->scan_tmp, st));
  MT_HIP(launch_inc_fill(mesh.conn, mesh.n_el, offb.as<int32_t>(), curb.as<int32_t>(), listb.as<int32_t>(), st));
  MT_HIP(launch_inc_sort(offb.as<int32_t>(), n, listb.as<int32_t>(), st));
  return MT_OK;
}

// The slave side's continuous normal field for the current coordinates (the
// element plane normals the frames use), or none for element normals.
int normals_for_coords(mt_ctx* c, hipStream_t st) {
  DeviceMesh& S = c->side[0];
  if (c->params.normals != MT_NORMALS_NODAL) {
    S.nrm = nullptr;
    return MT_OK;
  }
  if (S.nrm && c->nrm_gen == c->coord_gen) return MT_OK;
  if (!c->have_inc[0]) {
    int rc = build_incidence(c, S, c->inc_cnt, c->inc_off, c->inc_cur, c->inc_list, st);
    if (rc) return rc;
    c->have_inc[0] = true;
  }
  MT_HIP(launch_normals(S, c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), c->nrm_node.as<double>(),
                        c->nrm_el.as<double>(), st));
  S.nrm = c->nrm_el.as<double>();
  c->nrm_gen = c->coord_gen;
  return MT_OK;
}

}  // namespace

int mt::host_counts(mt_ctx* c) {
  if (int rc = ws_live(c)) return rc;
  if (c->counts_known || !c->have_pairs) return MT_OK;
  DeviceScope ds(c->device);
  DevState hs;
  int32_t nnz[2] = {0, 0};
  const int32_t n = c->side[0].n_nodes;
  if (c->have_pattern) {
    MT_HIP(read_back(c, {{&hs, c->state.p, sizeof(hs)}, {&nnz[0], c->D_rowptr.as<int32_t>() + n, 4},
                         {&nnz[1], c->M_rowptr.as<int32_t>() + n, 4}}, c->last_stream));
  } else {
    MT_HIP(read_back(c, {{&hs, c->state.p, sizeof(hs)}}, c->last_stream));
  }
  c->n_cand = hs.n_cand;
  c->n_maybe = hs.n_screened;
  c->n_pairs = hs.n_pairs;
  c->nnz_D = nnz[0];
  c->nnz_M = nnz[1];
  c->grid = hs.grid;
  c->counts_known = true;
  return MT_OK;
}

const int32_t* mt::dev_n_pairs(mt_ctx* c) { return &c->state.as<DevState>()->n_pairs; }

namespace {

// Argument checks of mt_integrate / mt_backward (sizes not read back: any
// slave element may have pairs).
int check_integrate(mt_ctx* c, const double* D_val, const double* M_val, const double* gap, const char* who) {
  if (!c) return fail(MT_EINVAL, std::string(who) + ": null ctx");
  if (!c->have_pattern) return fail(MT_ESTATE, std::string(who) + ": build pairs and pattern first");
  if (int rc = ws_live(c)) return rc;
  const bool known = c->counts_known;
  const bool needD = known ? c->nnz_D > 0 : c->side[0].n_el > 0;
  const bool needM = known ? c->nnz_M > 0 : c->side[0].n_el > 0;
  if ((needD && !D_val) || (needM && !M_val) || (c->side[0].n_nodes && !gap))
    return fail(MT_EINVAL, std::string(who) + ": null output");
  return MT_OK;
}

int check_backward(mt_ctx* c, const double* W_D, const double* W_M, const double* w_g, const double* gXs,
                   const double* gXm, const char* who) {
  if (!c) return fail(MT_EINVAL, std::string(who) + ": null ctx");
  if (c->params.element_rule > 0)
    return fail(MT_EUNSUPPORTED, std::string(who) + ": element-based integration has no backward pass");
  if (!c->have_pattern) return fail(MT_ESTATE, std::string(who) + ": build pairs and pattern first");
  if (int rc = ws_live(c)) return rc;
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const bool known = c->counts_known;
  const bool needD = known ? c->nnz_D > 0 : S.n_el > 0;
  const bool needM = known ? c->nnz_M > 0 : S.n_el > 0;
  if ((needD && !W_D) || (needM && !W_M) || (S.n_nodes && (!w_g || !gXs)) || (M.n_nodes && !gXm))
    return fail(MT_EINVAL, std::string(who) + ": null argument");
  return MT_OK;
}

// The clip polygons and the normal field of the current coordinates.
int prepare_pairs(mt_ctx* c, hipStream_t st) {
  int rc = ensure_poly(c);
  if (!rc) rc = normals_for_coords(c, st);
  if (rc) return rc;
  if (c->params.element_rule == 0 && c->poly_gen != c->coord_gen) {
    PhaseTimer t(c, MT_T_PAIR_POLY, st);
    MT_HIP(launch_pair_poly(c->side[0], c->side[1], kparams(c->params), c->pair_s.as<int32_t>(),
                            c->pair_m.as<int32_t>(), dev_n_pairs(c), c->cap.pairs, poly_buf(c),
                            c->counters.as<Counters>(), st));
    c->poly_gen = c->coord_gen;
  }
  return MT_OK;
}

// The per-pair blocks the assembly reads: those mt_csr_pattern computed
// serve the first integration after it (for unchanged coordinates); every
// other one computes them.
int ensure_blocks(mt_ctx* c, hipStream_t st) {
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const int64_t P = c->cap.pairs;
  if (c->params.element_rule > 0) {
    // element-based integration: no clip polygons
    PhaseTimer t(c, MT_T_PAIR_FWD, st);
    MT_HIP(launch_elem_fwd(S, M, kparams(c->params), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(),
                           c->pair_off.as<int32_t>(), dev_n_pairs(c), P, c->blk.as<double>(), P,
                           c->counters.as<Counters>(), st));
    c->blk_gen = -1;
  } else if (!(c->blk_pending && c->blk_gen == c->coord_gen)) {
    PhaseTimer t(c, MT_T_PAIR_FWD, st);
    MT_HIP(launch_pair_fwd(S, M, kparams(c->params), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(),
                           dev_n_pairs(c), P, poly_buf(c), c->blk.as<double>(), P, c->counters.as<Counters>(), st));
    c->blk_gen = c->coord_gen;
  }
  c->blk_pending = false;
  return MT_OK;
}

int enqueue_assemble(mt_ctx* c, double* D_val, double* M_val, double* gap, hipStream_t st) {
  const DeviceMesh& S = c->side[0];
  PhaseTimer t(c, MT_T_ASSEMBLE, st);
  MT_HIP(launch_assemble(c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), S.n_nodes, c->pair_off.as<int32_t>(),
                         c->D_rowptr.as<int32_t>(), c->M_rowptr.as<int32_t>(), c->posD.as<int32_t>(), S.n_el,
                         c->posM.as<int32_t>(), c->blk.as<double>(), c->cap.pairs, D_val, M_val, gap, st));
  return MT_OK;
}

// The reverse sweep of every pair and the nodal gradient sums (the
// polygons, normal field, master index and, for the dual basis, the pair
// blocks of the current coordinates in place).
int enqueue_backward(mt_ctx* c, const double* W_D, const double* W_M, const double* w_g, double* gXs, double* gXm,
                     hipStream_t st) {
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const int64_t P = c->cap.pairs;
  const bool nodal = c->params.normals == MT_NORMALS_NODAL;
  {
    PhaseTimer t(c, MT_T_PAIR_BWD, st);
    const KParams kp = kparams(c->params);
    MT_HIP(launch_pair_bwd(S, M, kp, c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), dev_n_pairs(c), P,
                           poly_buf(c), c->mp_pos.as<int32_t>(), c->posD.as<int32_t>(), S.n_el,
                           c->posM.as<int32_t>(), W_D, W_M, w_g, kp.dual ? c->blk.as<double>() : nullptr,
                           c->gpair.as<double>(), nodal ? c->gn0.as<double>() : nullptr, P,
                           c->counters.as<Counters>(), st));
  }
  PhaseTimer t(c, MT_T_GRAD_REDUCE, st);
  MT_HIP(launch_grad_slave(c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), S.n_nodes, c->pair_off.as<int32_t>(),
                           c->gpair.as<double>(), P, gXs, st));
  const int32_t* mo = c->mp_off.as<int32_t>();
  MT_HIP(launch_grad_master(c->minc_off.as<int32_t>(), c->minc_list.as<int32_t>(), M.n_nodes, mo, mo + 1,
                            c->gpair.as<double>(), P, gXm, st));
  if (nodal) {
    // through the element plane normals to the nodal normals and the
    // coordinates of the neighbouring elements
    MT_HIP(launch_normal_chain(S, c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), c->pair_off.as<int32_t>(),
                               c->gn0.as<double>(), P, c->nrm_node.as<double>(), c->nrm_el.as<double>(),
                               c->nrm_sb.as<double>(), c->nrm_ub.as<double>(), c->nrm_cg.as<double>(), gXs, nullptr,
                               nullptr, st));
  }
  return MT_OK;
}

}  // namespace

extern "C" {

const char* mt_last_error(void) { return mt::g_err.c_str(); }

int mt_default_params(mt_params* p) {
  if (!p) return fail(MT_EINVAL, "mt_default_params: null");
  std::memset(p, 0, sizeof(*p));
  p->delta = 0.0;
  p->bin_size = 0.0;
  p->lm_basis = MT_BASIS_STANDARD;
  p->rule = 7;
  p->eps_d = 1e-12;
  p->eps_a = 1e-12;
  p->newton_tol = 1e-14;
  p->newton_maxit = 30;
  return MT_OK;
}

int mt_create(mt_ctx** ctx, int device) {
  if (!ctx) return fail(MT_EINVAL, "mt_create: null ctx");
  *ctx = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(MT_EINVAL, "mt_create: no such device");
  DeviceScope ds(device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
  void* pin = nullptr;
  e = hipHostMalloc(&pin, PIN_BYTES, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
  mt_ctx* c = new mt_ctx();
  c->device = device;
  c->pin = pin;
  mt_default_params(&c->params);
  *ctx = c;
  return MT_OK;
}

int mt_destroy(mt_ctx* c) {
  if (!c) return MT_OK;
  DeviceScope ds(c->device);
  (void)hipDeviceSynchronize();
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->aux) {
    (void)hipEventDestroy(c->aux_fork);
    (void)hipEventDestroy(c->aux_join);
    (void)hipEventDestroy(c->aux2_join);
    (void)hipStreamDestroy(c->aux);
    (void)hipStreamDestroy(c->aux2);
  }
  for (auto& iv : c->intervals) {
    (void)hipEventDestroy(iv.a);
    (void)hipEventDestroy(iv.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  delete c;
  return MT_OK;
}

int mt_set_params(mt_ctx* c, const mt_params* p) {
  if (!c || !p) return fail(MT_EINVAL, "mt_set_params: null");
  if (p->rule != 3 && p->rule != 7) return fail(MT_EINVAL, "mt_set_params: rule must be 3 or 7");
  if (p->lm_basis != MT_BASIS_STANDARD && p->lm_basis != MT_BASIS_DUAL)
    return fail(MT_EINVAL, "mt_set_params: lm_basis");
  if (p->element_rule < 0 || p->element_rule > 8)
    return fail(MT_EINVAL, "mt_set_params: element_rule must be 0 (segments) or 1..8");
  if (p->normals != MT_NORMALS_ELEMENT && p->normals != MT_NORMALS_NODAL)
    return fail(MT_EINVAL, "mt_set_params: normals");
  if (p->single_stream != 0 && p->single_stream != 1) return fail(MT_EINVAL, "mt_set_params: single_stream");
  if (!(p->delta >= 0) || !(p->bin_size >= 0) || !(p->eps_d >= 0) || !(p->eps_a >= 0) || !(p->newton_tol > 0) ||
      p->newton_maxit < 1)
    return fail(MT_EINVAL, "mt_set_params: negative or invalid tolerance");
  c->params = *p;
  c->have_pairs = c->have_pattern = c->have_master_index = false;
  ++c->coord_gen;
  return MT_OK;
}

int mt_upload(mt_ctx* c, int side, int64_t n_nodes, const double* x, const double* y, const double* z, int64_t n_el,
              const int32_t* conn, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_upload: null ctx");
  if (side != MT_SIDE_SLAVE && side != MT_SIDE_MASTER) return fail(MT_EINVAL, "mt_upload: bad side");
  if (n_nodes < 0 || n_el < 0 || n_nodes >= (int64_t(1) << 31) || n_el >= (int64_t(1) << 29))
    return fail(MT_EINVAL, "mt_upload: size out of range");
  if ((n_nodes > 0 && (!x || !y || !z)) || (n_el > 0 && !conn)) return fail(MT_EINVAL, "mt_upload: null array");
  if (n_el > 0 && (reinterpret_cast<uintptr_t>(conn) & 15))
    return fail(MT_EINVAL, "mt_upload: connectivity must be 16-byte aligned");
  DeviceScope ds(c->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
  DeviceMesh& m = c->side[side];
  m.set = false;
  c->have_inc[side] = false;
  ++c->upload_gen;
  c->have_pairs = c->have_pattern = c->have_master_index = false;
  ++c->coord_gen;
  if (n_el > 0) {
    // connectivity range check (argument validation, once per upload): every
    // later kernel gathers nodes through it without bounds checks
    std::vector<int32_t> h((size_t)n_el * 4);
    hipStream_t st = (hipStream_t)stream;
    MT_HIP(hipMemcpyAsync(h.data(), conn, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    MT_HIP(hipStreamSynchronize(st));
    for (int32_t v : h)
      if (v < 0 || v >= n_nodes) return fail(MT_EINVAL, "mt_upload: connectivity index out of range");
  }
  m.x = x; m.y = y; m.z = z; m.conn = conn;
  m.nrm = nullptr;
  m.n_nodes = (int32_t)n_nodes;
  m.n_el = (int32_t)n_el;
  m.set = true;
  return MT_OK;
}

int mt_update_coordinates(mt_ctx* c, int side, const double* x, const double* y, const double* z, void* stream) {
  (void)stream;
  if (!c) return fail(MT_EINVAL, "mt_update_coordinates: null ctx");
  if (side != MT_SIDE_SLAVE && side != MT_SIDE_MASTER) return fail(MT_EINVAL, "mt_update_coordinates: bad side");
  DeviceMesh& m = c->side[side];
  if (!m.set) return fail(MT_ESTATE, "mt_update_coordinates: side not uploaded");
  if (m.n_nodes > 0 && (!x || !y || !z)) return fail(MT_EINVAL, "mt_update_coordinates: null array");
  m.x = x; m.y = y; m.z = z;
  ++c->coord_gen;
  return MT_OK;
}

int mt_default_capacity(mt_ctx* c, mt_capacity* cap) {
  if (!c || !cap) return fail(MT_EINVAL, "mt_default_capacity: null");
  if (!c->side[0].set || !c->side[1].set) return fail(MT_ESTATE, "mt_default_capacity: upload both sides first");
  *cap = default_cap(c);
  return MT_OK;
}

int mt_workspace_size(mt_ctx* c, const mt_capacity* cap_in, size_t* bytes) {
  if (!c || !bytes) return fail(MT_EINVAL, "mt_workspace_size: null");
  if (!c->side[0].set || !c->side[1].set) return fail(MT_ESTATE, "mt_workspace_size: upload both sides first");
  const mt_capacity cap = cap_in ? *cap_in : default_cap(c);
  if (int rc = check_cap(cap)) return rc;
  // a size query must not disturb the bound layout
  mt_ctx probe;
  probe.side[0] = c->side[0];
  probe.side[1] = c->side[1];
  probe.params = c->params;
  Arena A;
  layout(&probe, cap, A);
  *bytes = A.off;
  return MT_OK;
}

int mt_build_pairs(mt_ctx* c, const mt_capacity* cap_in, void* ws, size_t ws_bytes, int64_t* n_cand_out,
                   int64_t* n_pairs_out, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_build_pairs: null ctx");
  if (!c->side[0].set || !c->side[1].set) return fail(MT_ESTATE, "mt_build_pairs: upload both sides first");
  const mt_capacity cap = cap_in ? *cap_in : default_cap(c);
  if (int rc = check_cap(cap)) return rc;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
    return fail(MT_EINVAL, "mt_build_pairs: workspace null or not 256-byte aligned");
  DeviceScope ds(c->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  c->have_pairs = c->have_pattern = c->have_master_index = false;
  c->counts_known = false;
  ++c->coord_gen;
  c->side[0].nrm = nullptr;
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const int32_t ns = S.n_el, nm = M.n_el;
  // bind the workspace: the layout is a function of the capacities, the
  // mesh sizes and the normal field; buffers that depend on the
  // connectivity only (node incidence) are kept while it is unchanged
  {
    const int nodal = c->params.normals == MT_NORMALS_NODAL ? 1 : 0;
    const int32_t sizes[4] = {S.n_nodes, S.n_el, M.n_nodes, M.n_el};
    const bool same = ws == c->ws && std::memcmp(&cap, &c->cap, sizeof(cap)) == 0 &&
                      std::memcmp(sizes, c->lay_n, sizeof(sizes)) == 0 && nodal == c->lay_nodal;
    Arena A;
    A.base = static_cast<char*>(ws);
    layout(c, cap, A);
    if (A.off > ws_bytes) {
      c->ws = nullptr;
      c->lay_nodal = -1;
      c->have_inc[0] = c->have_inc[1] = false;
      return fail(MT_ECAPACITY, "mt_build_pairs: workspace smaller than mt_workspace_size");
    }
    if (!same) c->have_inc[0] = c->have_inc[1] = false;
    c->static_gen = 0;
    c->ws = ws;
    c->ws_bytes = ws_bytes;
    c->cap = cap;
    std::memcpy(c->lay_n, sizes, sizeof(sizes));
    c->lay_nodal = nodal;
  }
  DevState* dst = c->state.as<DevState>();
  Counters* cnt = c->counters.as<Counters>();
  PrepReduce* red = c->reduce.as<PrepReduce>();
  const KParams kp = kparams(c->params);
  const int nb_s = prep_blocks(ns), nb_m = prep_blocks(nm);
  {
    PhaseTimer t(c, MT_T_PREP, st);
    // counters and state start at zero (a fill kernel: no memset node)
    static_assert(sizeof(Counters) % 4 == 0 && sizeof(DevState) % 4 == 0, "word fills");
    MT_HIP(fill_i32(c->counters.as<int32_t>(), 0, sizeof(Counters) / 4, st));
    MT_HIP(fill_i32(c->state.as<int32_t>(), 0, sizeof(DevState) / 4, st));
    // the continuous normal field first: the slave frames use it
    int rc = normals_for_coords(c, st);
    if (rc) return rc;
    double* part = c->prep_part.as<double>();
    MT_HIP(launch_prep(S, M, c->box_s.as<double>(), c->sdata.as<double>(), c->box_m.as<double>(),
                       c->mdata.as<double>(), part, st));
    MT_HIP(launch_prep_reduce(part, nb_s, nb_m, red, c->params.delta, c->params.bin_size, cap.cells, dst, st));
  }
  const Grid* g = &dst->grid;
  {
    // master elements sorted by cell, cell ranges from segment heads
    PhaseTimer t(c, MT_T_BIN_SORT, st);
    int bits = 1;
    while ((int64_t(1) << bits) < cap.cells) ++bits;
    // keys written where an odd number of sort passes starts, so that the
    // sorted pairs end in (keys, vals) without a copy
    const bool in_tmp = radix_passes(bits) % 2 == 1;
    MT_HIP(launch_master_keys(c->box_m.as<double>(), nm, g, cap.cells,
                              (in_tmp ? c->keys_tmp : c->keys).as<uint32_t>(),
                              (in_tmp ? c->vals_tmp : c->vals).as<uint32_t>(), c->cell_range.as<int2>(), st));
    MT_HIP(radix_sort_pairs(c->keys.as<uint32_t>(), c->vals.as<uint32_t>(), c->keys_tmp.as<uint32_t>(),
                            c->vals_tmp.as<uint32_t>(), nm, nullptr, bits, c->sort_hist, c->scan_tmp, st, in_tmp));
    MT_HIP(launch_cell_ranges(c->keys.as<uint32_t>(), c->vals.as<uint32_t>(), nm, c->box_m.as<double>(), g,
                              c->cell_range.as<int2>(), c->sbox.as<double>(), c->qbox.as<uint64_t>(), st));
  }
  {
    // candidates: count, scan, fill (sorted by master within each slave),
    // each screened as it is written (projection onto the slave plane,
    // degeneracy checks, separating-line test)
    PhaseTimer t(c, MT_T_CAND, st);
    MT_HIP(launch_cand_count(c->box_s.as<double>(), ns, c->sbox.as<double>(), c->qbox.as<uint64_t>(),
                             c->vals.as<uint32_t>(), c->cell_range.as<int2>(), g, c->params.delta,
                             c->cand_cnt.as<int32_t>(), c->cand_tmp.as<int32_t>(), st));
    MT_HIP(scan_exclusive(c->cand_cnt.as<int32_t>(), c->cand_off.as<int32_t>(), ns, c->scan_tmp, st));
    MT_HIP(launch_stage_totals(0, c->cand_off.as<int32_t>(), ns, cap.candidates, dst, st));
    MT_HIP(launch_cand_fill(c->box_s.as<double>(), ns, c->sbox.as<double>(), c->vals.as<uint32_t>(),
                            c->cell_range.as<int2>(), g, c->params.delta, c->cand_tmp.as<int32_t>(),
                            c->cand_off.as<int32_t>(), c->cand_s.as<int32_t>(), c->cand_m.as<int32_t>(),
                            c->sdata.as<double>(), c->mdata.as<double>(), kp.eps_a, c->cand_nv.as<uint8_t>(),
                            c->cand_flag.as<int32_t>(), c->scr_cnt.as<int32_t>(), cnt, cap.candidates, st));
  }
  const int64_t SC = cap.screened;
  c->mpoly_stride = SC;
  const PolyBuf mpoly{c->mpoly_u.as<double>(), c->mpoly_v.as<double>(), c->mpoly_lab.as<uint8_t>(),
                      c->mpoly_nf.as<uint8_t>(), SC, nullptr};
  {
    PhaseTimer t(c, MT_T_COMPACT, st);
    MT_HIP(scan_exclusive(c->scr_cnt.as<int32_t>(), c->scr_off.as<int32_t>(), ns, c->scan_tmp, st));
    MT_HIP(launch_stage_totals(1, c->scr_off.as<int32_t>(), ns, SC, dst, st));
    MT_HIP(launch_maybe_list(c->cand_flag.as<int32_t>(), c->cand_off.as<int32_t>(), c->scr_off.as<int32_t>(), ns,
                             cap.candidates, SC, c->maybe_list.as<int32_t>(), st));
  }
  {
    PhaseTimer t(c, MT_T_CLIP, st);
    MT_HIP(launch_clip_screened(c->mdata.as<double>(), c->sdata.as<double>(), ns, kp, c->cand_s.as<int32_t>(),
                                c->cand_m.as<int32_t>(), c->maybe_list.as<int32_t>(), &dst->n_screened, SC,
                                c->cand_nv.as<uint8_t>(), c->maybe_flag.as<int32_t>(), mpoly, cnt, st));
  }
  {
    PhaseTimer t(c, MT_T_COMPACT, st);
    MT_HIP(scan_exclusive_dev(c->maybe_flag.as<int32_t>(), c->maybe_scan.as<int32_t>(), &dst->n_screened, SC,
                              c->scan_tmp, st));
    MT_HIP(launch_stage_totals(2, c->maybe_scan.as<int32_t>(), 0, cap.pairs, dst, st));
    MT_HIP(launch_compact_pairs(c->cand_s.as<int32_t>(), c->cand_m.as<int32_t>(), c->maybe_list.as<int32_t>(),
                                c->maybe_flag.as<int32_t>(), c->maybe_scan.as<int32_t>(), &dst->n_screened, SC,
                                c->mpoly_nf.as<uint8_t>(), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(),
                                c->pair_nv.as<uint8_t>(), c->pair_slot.as<int32_t>(), cap.pairs, st));
    MT_HIP(launch_pair_off(c->scr_off.as<int32_t>(), c->maybe_scan.as<int32_t>(), ns, dst,
                           c->pair_off.as<int32_t>(), st));
  }
  c->poly_gen = c->coord_gen;
  c->have_pairs = true;
  if (!n_cand_out && !n_pairs_out) return MT_OK;
  DevState hs;
  Counters hc;
  MT_HIP(read_back(c, {{&hs, dst, sizeof(hs)}, {&hc, cnt, sizeof(hc)}}, st));
  c->n_cand = hs.n_cand;
  c->n_maybe = hs.n_screened;
  c->n_pairs = hs.n_pairs;
  c->grid = hs.grid;
  c->counts_known = true;
  if (n_cand_out) *n_cand_out = c->n_cand;
  if (n_pairs_out) *n_pairs_out = c->n_pairs;
  return device_status(hs, hc, false);
}

int mt_required_capacity(mt_ctx* c, mt_capacity* need) {
  if (!c || !need) return fail(MT_EINVAL, "mt_required_capacity: null");
  if (!c->ws || !c->state.p) return fail(MT_ESTATE, "mt_required_capacity: no build");
  if (int rc = ws_live(c)) return rc;
  DeviceScope ds(c->device);
  DevState hs;
  MT_HIP(read_back(c, {{&hs, c->state.p, sizeof(hs)}}, c->last_stream));
  need->candidates = hs.n_cand;
  need->screened = hs.need_screened;
  need->pairs = hs.need_pairs;
  need->cells = hs.grid.ncells;
  return MT_OK;
}

int mt_check(mt_ctx* c) {
  if (!c) return fail(MT_EINVAL, "mt_check: null");
  if (!c->have_pairs) return fail(MT_ESTATE, "mt_check: no build");
  if (int rc = ws_live(c)) return rc;
  DeviceScope ds(c->device);
  DevState hs;
  Counters hc;
  MT_HIP(read_back(c, {{&hs, c->state.p, sizeof(hs)}, {&hc, c->counters.p, sizeof(hc)}}, c->last_stream));
  return device_status(hs, hc, true);
}

int mt_get_pairs(mt_ctx* c, int32_t* s, int32_t* m, uint8_t* nv, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_get_pairs: null ctx");
  if (!c->have_pairs) return fail(MT_ESTATE, "mt_get_pairs: no pair list");
  if (int rc = host_counts(c)) return rc;
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)c->n_pairs;
  if (n == 0) return MT_OK;
  if (s) MT_HIP(hipMemcpyAsync(s, c->pair_s.p, 4 * n, hipMemcpyDeviceToDevice, st));
  if (m) MT_HIP(hipMemcpyAsync(m, c->pair_m.p, 4 * n, hipMemcpyDeviceToDevice, st));
  if (nv) MT_HIP(hipMemcpyAsync(nv, c->pair_nv.p, n, hipMemcpyDeviceToDevice, st));
  return MT_OK;
}

int mt_get_candidates(mt_ctx* c, int32_t* s, int32_t* m, uint8_t* nv, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_get_candidates: null ctx");
  if (!c->have_pairs) return fail(MT_ESTATE, "mt_get_candidates: no candidate list");
  if (int rc = host_counts(c)) return rc;
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)std::min<int64_t>(c->n_cand, c->cap.candidates);
  if (n == 0) return MT_OK;
  if (s) MT_HIP(hipMemcpyAsync(s, c->cand_s.p, 4 * n, hipMemcpyDeviceToDevice, st));
  if (m) MT_HIP(hipMemcpyAsync(m, c->cand_m.p, 4 * n, hipMemcpyDeviceToDevice, st));
  if (nv) MT_HIP(hipMemcpyAsync(nv, c->cand_nv.p, n, hipMemcpyDeviceToDevice, st));
  return MT_OK;
}

int mt_csr_pattern(mt_ctx* c, int64_t* nnz_D, int64_t* nnz_M, void* stream) {
  return csr_pattern(c, nnz_D, nnz_M, (hipStream_t)stream, true);
}

}  // extern "C"

// The pattern, and with `blocks` the pair blocks of the coming integration
// beside it.
int mt::csr_pattern(mt_ctx* c, int64_t* nnz_D, int64_t* nnz_M, hipStream_t st, bool blocks, bool fork) {
  if (!c) return fail(MT_EINVAL, "mt_csr_pattern: null ctx");
  if (!c->have_pairs) return fail(MT_ESTATE, "mt_csr_pattern: build the pair list first");
  if (int rc = ws_live(c)) return rc;
  DeviceScope ds(c->device);
  c->last_stream = st;
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const int32_t n = S.n_nodes;
  const int64_t P = c->cap.pairs;
  // the local block entries (16 per pair) bound nnz(M), so the int32 row
  // pointers cannot overflow below this size
  if (16 * (int64_t)S.n_el >= (int64_t(1) << 31) || 16 * P >= (int64_t(1) << 31))
    return fail(MT_ECAPACITY, "mt_csr_pattern: more than 2^31 block entries");
  c->have_pattern = false;
  c->counts_known = false;
  const int32_t* np_dev = dev_n_pairs(c);
  PhaseTimer timer(c, MT_T_PATTERN, st);
  if (!c->have_inc[0]) {
    int rc = build_incidence(c, S, c->inc_cnt, c->inc_off, c->inc_cur, c->inc_list, st);
    if (rc) return rc;
    c->have_inc[0] = true;
  }
  c->have_master_index = false;
  // per-element master-node lists of the M rows, before the fork: a short
  // kernel that would otherwise wait behind the forward's blocks
  MT_HIP(launch_elem_mlist(S.n_el, c->pair_off.as<int32_t>(), c->pair_m.as<int32_t>(), M.conn,
                           c->pat_ecnt.as<int32_t>(), c->pat_elist.as<int32_t>(), st));
  // The pair blocks of segment-based integration and the pairs-by-master
  // index of the backward depend on the pair list alone: they run on an
  // internal stream (the FP64-bound quadrature beside the latency-bound
  // pattern kernels) and are joined back into the caller's stream before
  // this call returns.  mt_integrate then only assembles.  Enqueue order:
  // the forward, the pattern passes, then the index (a chain of short sort
  // kernels, needed by the backward only), so that no pattern kernel waits
  // for the host to enqueue that chain behind the forward.
  const bool aux =
      fork && c->params.element_rule == 0 && c->poly_gen == c->coord_gen && !c->params.single_stream;
  if (aux) {
    if (!c->have_inc[1]) {
      int rc = build_incidence(c, M, c->minc_cnt, c->minc_off, c->minc_cur, c->minc_list, st);
      if (rc) return rc;
      c->have_inc[1] = true;
    }
    if (int rc = ensure_aux(c)) return rc;
    MT_HIP(hipEventRecord(c->aux_fork, st));
    MT_HIP(hipStreamWaitEvent(c->aux, c->aux_fork, 0));
    MT_HIP(hipStreamWaitEvent(c->aux2, c->aux_fork, 0));
  }
  // from the fork on, errors still join the internal streams back, so that
  // the caller's stream orders after whatever was launched
  auto body = [&]() -> int {
    if (aux && blocks) {
      PhaseTimer t(c, MT_T_PAIR_FWD, c->aux);
      MT_HIP(launch_pair_fwd(S, M, kparams(c->params), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), np_dev, P,
                             poly_buf(c), c->blk.as<double>(), P, c->counters.as<Counters>(), c->aux));
    }
    MT_HIP(launch_pattern_rows(false, c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), n,
                               c->pair_off.as<int32_t>(), c->pair_m.as<int32_t>(), S.conn, M.conn,
                               c->D_cnt.as<int32_t>(), c->M_cnt.as<int32_t>(), nullptr, nullptr, nullptr, nullptr,
                               c->pat_keep.as<int32_t>(), S.n_el, c->pat_ecnt.as<int32_t>(),
                               c->pat_elist.as<int32_t>(), st));
    MT_HIP(scan_exclusive2(c->D_cnt.as<int32_t>(), c->D_rowptr.as<int32_t>(), c->M_cnt.as<int32_t>(),
                           c->M_rowptr.as<int32_t>(), n, c->scan_tmp, st, aux ? SCAN_BLOCKS_BESIDE : 0));
    // the column arrays are sized by the local block entries (16 per slave
    // element for D, 16 per pair for M); then the CSR position of every
    // local block entry, pair by pair
    MT_HIP(launch_pattern_rows(true, c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), n,
                               c->pair_off.as<int32_t>(), c->pair_m.as<int32_t>(), S.conn, M.conn, nullptr, nullptr,
                               c->D_rowptr.as<int32_t>(), c->M_rowptr.as<int32_t>(), c->D_col.as<int32_t>(),
                               c->M_col.as<int32_t>(), c->pat_keep.as<int32_t>(), S.n_el, nullptr, nullptr, st));
    MT_HIP(launch_pattern_positions(c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), np_dev, P, S.conn, M.conn,
                                    S.n_el, c->pair_off.as<int32_t>(), c->D_rowptr.as<int32_t>(),
                                    c->D_col.as<int32_t>(), c->M_rowptr.as<int32_t>(), c->M_col.as<int32_t>(),
                                    c->posD.as<int32_t>(), c->posM.as<int32_t>(), st));
    if (aux) {
      // on the second internal stream: the index's short atomic and sort
      // kernels run beside the forward instead of after it
      PhaseTimer t(c, MT_T_GRAD_REDUCE, c->aux2);
      return build_master_index(c, c->aux2, c->aux_scan);
    }
    return MT_OK;
  };
  const int rc = body();
  if (aux) {
    MT_HIP(hipEventRecord(c->aux_join, c->aux));
    MT_HIP(hipEventRecord(c->aux2_join, c->aux2));
    MT_HIP(hipStreamWaitEvent(st, c->aux_join, 0));
    MT_HIP(hipStreamWaitEvent(st, c->aux2_join, 0));
  }
  if (rc) return rc;
  if (aux && blocks) {
    c->blk_gen = c->coord_gen;
    c->blk_pending = true;
  }
  c->have_pattern = true;
  ++c->pattern_gen;
  if (!nnz_D && !nnz_M) return MT_OK;
  int32_t tot[2] = {0, 0};
  DevState hs;
  MT_HIP(read_back(c, {{&tot[0], c->D_rowptr.as<int32_t>() + n, 4}, {&tot[1], c->M_rowptr.as<int32_t>() + n, 4},
                       {&hs, c->state.p, sizeof(hs)}}, st));
  c->nnz_D = tot[0];
  c->nnz_M = tot[1];
  c->n_cand = hs.n_cand;
  c->n_maybe = hs.n_screened;
  c->n_pairs = hs.n_pairs;
  c->grid = hs.grid;
  c->counts_known = true;
  if (nnz_D) *nnz_D = c->nnz_D;
  if (nnz_M) *nnz_M = c->nnz_M;
  return MT_OK;
}

extern "C" {

int mt_get_csr(mt_ctx* c, int32_t* D_rowptr, int32_t* D_col, int32_t* M_rowptr, int32_t* M_col, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_get_csr: null ctx");
  if (!c->have_pattern) return fail(MT_ESTATE, "mt_get_csr: no pattern");
  if (int rc = host_counts(c)) return rc;
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t nr = (size_t)c->side[0].n_nodes + 1;
  if (D_rowptr) MT_HIP(hipMemcpyAsync(D_rowptr, c->D_rowptr.p, 4 * nr, hipMemcpyDeviceToDevice, st));
  if (M_rowptr) MT_HIP(hipMemcpyAsync(M_rowptr, c->M_rowptr.p, 4 * nr, hipMemcpyDeviceToDevice, st));
  if (D_col && c->nnz_D) MT_HIP(hipMemcpyAsync(D_col, c->D_col.p, 4 * (size_t)c->nnz_D, hipMemcpyDeviceToDevice, st));
  if (M_col && c->nnz_M) MT_HIP(hipMemcpyAsync(M_col, c->M_col.p, 4 * (size_t)c->nnz_M, hipMemcpyDeviceToDevice, st));
  return MT_OK;
}

int mt_integrate(mt_ctx* c, double* D_val, double* M_val, double* gap, void* stream) {
  if (int rc = check_integrate(c, D_val, M_val, gap, "mt_integrate")) return rc;
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  if (int rc = prepare_pairs(c, st)) return rc;
  if (int rc = ensure_blocks(c, st)) return rc;
  return enqueue_assemble(c, D_val, M_val, gap, st);
}

}  // extern "C"

// The pair polygons live in the screened-candidate polygon buffer of the
// last mt_build_pairs (pair p at entry pair_slot[p]); it holds an entry for
// every pair, also when the polygons are recomputed for new coordinates.
int mt::ensure_poly(mt_ctx* c) {
  if (!c->have_pairs || !c->pair_slot.p || !c->mpoly_nf.p)
    return fail(MT_ESTATE, "pair polygons: build the pair list first");
  return MT_OK;
}

mt::PolyBuf mt::poly_buf(mt_ctx* c) {
  return PolyBuf{c->mpoly_u.as<double>(), c->mpoly_v.as<double>(), c->mpoly_lab.as<uint8_t>(),
                 c->mpoly_nf.as<uint8_t>(), c->mpoly_stride, c->pair_slot.as<int32_t>()};
}

int mt::ensure_master_index(mt_ctx* c, hipStream_t st) {
  if (c->have_master_index) return MT_OK;
  const DeviceMesh& M = c->side[1];
  if (!c->have_inc[1]) {
    int rc = build_incidence(c, M, c->minc_cnt, c->minc_off, c->minc_cur, c->minc_list, st);
    if (rc) return rc;
    c->have_inc[1] = true;
  }
  return build_master_index(c, st, c->scan_tmp);
}

int mt::build_master_index(mt_ctx* c, hipStream_t st, const Buf& scan_tmp) {
  const DeviceMesh& M = c->side[1];
  MT_HIP(launch_master_index(c->pair_m.as<int32_t>(), dev_n_pairs(c), c->cap.pairs, M.n_el, c->mp_cnt.as<int32_t>(),
                             c->mp_cur.as<int32_t>(), c->mp_off.as<int32_t>(), c->mp_vals.as<uint32_t>(),
                             c->mp_tmp.as<uint32_t>(), c->mp_pos.as<int32_t>(), scan_tmp, st));
  c->have_master_index = true;
  return MT_OK;
}

extern "C" {

int mt_backward(mt_ctx* c, const double* W_D, const double* W_M, const double* w_g, double* gXs, double* gXm,
                void* stream) {
  if (int rc = check_backward(c, W_D, W_M, w_g, gXs, gXm, "mt_backward")) return rc;
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  {
    PhaseTimer t(c, MT_T_GRAD_REDUCE, st);
    if (int rc = ensure_master_index(c, st)) return rc;
  }
  if (int rc = prepare_pairs(c, st)) return rc;
  if (c->params.lm_basis == MT_BASIS_DUAL && c->blk_gen != c->coord_gen) {
    // the dual adjoint reads each pair's dual blocks: those staged by the
    // last mt_integrate unless the coordinates or pairs changed since
    PhaseTimer t(c, MT_T_PAIR_BWD, st);
    MT_HIP(launch_pair_fwd(c->side[0], c->side[1], kparams(c->params), c->pair_s.as<int32_t>(),
                           c->pair_m.as<int32_t>(), dev_n_pairs(c), c->cap.pairs, poly_buf(c), c->blk.as<double>(),
                           c->cap.pairs, c->counters.as<Counters>(), st));
    c->blk_gen = c->coord_gen;
  }
  return enqueue_backward(c, W_D, W_M, w_g, gXs, gXm, st);
}

int mt_integrate_backward(mt_ctx* c, double* D_val, double* M_val, double* gap, const double* W_D,
                          const double* W_M, const double* w_g, double* gXs, double* gXm, void* stream) {
  if (int rc = check_backward(c, W_D, W_M, w_g, gXs, gXm, "mt_integrate_backward")) return rc;
  if (int rc = check_integrate(c, D_val, M_val, gap, "mt_integrate_backward")) return rc;
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  {
    PhaseTimer t(c, MT_T_GRAD_REDUCE, st);
    if (int rc = ensure_master_index(c, st)) return rc;
  }
  if (int rc = prepare_pairs(c, st)) return rc;
  if (int rc = ensure_blocks(c, st)) return rc;  // also the dual adjoint's blocks
  if (c->params.single_stream) {
    const int rc = enqueue_assemble(c, D_val, M_val, gap, st);
    return rc ? rc : enqueue_backward(c, W_D, W_M, w_g, gXs, gXm, st);
  }
  // the assembly (bound by memory) on the caller's stream, the reverse sweep
  // (bound by FP64 issue) and the gradient sums on an internal stream; the
  // assembly is enqueued first, so that its workgroups are dispatched before
  // the sweep's fill the register files
  if (int rc = ensure_aux(c)) return rc;
  MT_HIP(hipEventRecord(c->aux_fork, st));
  int rc = enqueue_assemble(c, D_val, M_val, gap, st);
  MT_HIP(hipStreamWaitEvent(c->aux, c->aux_fork, 0));
  if (rc == MT_OK) rc = enqueue_backward(c, W_D, W_M, w_g, gXs, gXm, c->aux);
  // joined also after an error, so that the caller's stream orders after
  // whatever was launched
  MT_HIP(hipEventRecord(c->aux_join, c->aux));
  MT_HIP(hipStreamWaitEvent(st, c->aux_join, 0));
  return rc;
}

int mt_set_timing_phases(mt_ctx* c, uint32_t mask) {
  if (!c) return fail(MT_EINVAL, "mt_set_timing_phases: null ctx");
  c->timing = mask != 0;
  c->timing_mask = mask;
  return MT_OK;
}

int mt_set_timing(mt_ctx* c, int enable) {
  if (!c) return fail(MT_EINVAL, "mt_set_timing: null ctx");
  c->timing = enable != 0;
  c->timing_mask = ~0u;
  return MT_OK;
}

int mt_get_timings(mt_ctx* c, mt_timings* t, int reset) {
  if (!c || !t) return fail(MT_EINVAL, "mt_get_timings: null");
  DeviceScope ds(c->device);
  for (auto& iv : c->intervals) {
    MT_HIP(hipEventSynchronize(iv.b));
    float ms = 0.f;
    MT_HIP(hipEventElapsedTime(&ms, iv.a, iv.b));
    c->t_ms[iv.phase] += ms;
    c->t_n[iv.phase] += 1;
    c->event_pool.push_back(iv.a);
    c->event_pool.push_back(iv.b);
  }
  c->intervals.clear();
  for (int i = 0; i < MT_T_COUNT; ++i) {
    t->ms[i] = c->t_ms[i];
    t->intervals[i] = c->t_n[i];
  }
  if (reset) {
    for (int i = 0; i < MT_T_COUNT; ++i) { c->t_ms[i] = 0.0; c->t_n[i] = 0; }
  }
  return MT_OK;
}

int mt_get_stats(mt_ctx* c, mt_stats* out) {
  if (!c || !out) return fail(MT_EINVAL, "mt_get_stats: null");
  std::memset(out, 0, sizeof(*out));
  if (!c->have_pairs || !c->counters.p) return MT_OK;
  if (int rc = host_counts(c)) return rc;
  out->n_candidates = c->n_cand;
  out->n_pairs = c->n_pairs;
  out->nnz_D = c->have_pattern ? c->nnz_D : 0;
  out->nnz_M = c->have_pattern ? c->nnz_M : 0;
  for (int d = 0; d < 3; ++d) {
    out->n_bins[d] = c->grid.n[d];
    out->bin_size[d] = c->grid.beta[d];
  }
  DeviceScope ds(c->device);
  Counters* dc = c->counters.as<Counters>();
  MT_HIP(fill_i32(reinterpret_cast<int32_t*>(dc->hist), 0, 2 * 17, c->last_stream));
  MT_HIP(launch_nv_hist(c->cand_nv.as<uint8_t>(), std::min<int64_t>(c->n_cand, c->cap.candidates), dc->hist,
                        c->last_stream));
  Counters hc;
  MT_HIP(read_back(c, {{&hc, c->counters.p, sizeof(hc)}}, c->last_stream));
  for (int i = 0; i < 17; ++i) out->nverts_hist[i] = (int64_t)hc.hist[i];
  out->n_noconv = (int64_t)hc.noconv;
  out->n_overflow = (int64_t)hc.overflow;
  out->n_degenerate_slave = (int64_t)hc.degen_slave;
  out->n_degenerate_master = (int64_t)hc.degen_master;
  out->n_lost_pairs = (int64_t)hc.degen_poly;
  return MT_OK;
}

}  // extern "C"

int mt::ensure_normals(mt_ctx* c, hipStream_t st) { return normals_for_coords(c, st); }

int mt::ensure_aux(mt_ctx* c) {
  if (c->aux) return MT_OK;
  MT_HIP(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
  MT_HIP(hipStreamCreateWithFlags(&c->aux2, hipStreamNonBlocking));
  MT_HIP(hipEventCreateWithFlags(&c->aux_fork, hipEventDisableTiming));
  MT_HIP(hipEventCreateWithFlags(&c->aux_join, hipEventDisableTiming));
  MT_HIP(hipEventCreateWithFlags(&c->aux2_join, hipEventDisableTiming));
  return MT_OK;
}

// ---- search of many interfaces ------------------------------------------------
int mt::search_no_wait(mt_ctx* c, hipStream_t st, bool fork) {
  const bool timing = c->timing;
  c->timing = false;
  int rc = mt_build_pairs(c, &c->cap, c->ws, c->ws_bytes, nullptr, nullptr, st);
  // the batch's forward computes the pair blocks itself
  if (rc == MT_OK) rc = csr_pattern(c, nullptr, nullptr, st, false, fork);
  c->timing = timing;
  return rc;
}

void mt::search_replayed(mt_ctx* c, hipStream_t st) {
  // mt_build_pairs (same workspace binding, no read-back)
  c->last_stream = st;
  c->have_master_index = false;
  c->counts_known = false;
  ++c->coord_gen;
  DeviceMesh& S = c->side[0];
  if (c->params.normals == MT_NORMALS_NODAL) {  // recomputed by the graph
    S.nrm = c->nrm_el.as<double>();
    c->nrm_gen = c->coord_gen;
  } else {
    S.nrm = nullptr;
  }
  c->static_gen = 0;
  c->mpoly_stride = c->cap.screened;
  c->poly_gen = c->coord_gen;
  c->have_pairs = true;
  // mt_csr_pattern without the internal streams
  c->have_pattern = true;
  ++c->pattern_gen;
}

std::string mt::search_signature(const mt_ctx* c) {
  std::string s;
  auto add = [&s](const void* p, size_t n) { s.append(static_cast<const char*>(p), n); };
  add(&c->device, sizeof(c->device));
  add(&c->ws, sizeof(c->ws));
  add(&c->ws_bytes, sizeof(c->ws_bytes));
  add(&c->cap, sizeof(c->cap));
  add(&c->params, sizeof(c->params));
  // a new upload may bring other connectivity at the same addresses, and
  // the graph does not rebuild node incidences it found built
  add(&c->upload_gen, sizeof(c->upload_gen));
  for (const DeviceMesh& m : c->side) {
    const void* ptrs[4] = {m.x, m.y, m.z, m.conn};
    const int32_t n[2] = {m.n_nodes, m.n_el};
    add(ptrs, sizeof(ptrs));
    add(n, sizeof(n));
  }
  return s;
}

// ---- the build that allocates nothing ------------------------------------------
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid it): the workspace of
// mt_build_pairs is a static device array of the library instead of caller
// memory.  Each GPU the library runs on holds its own copy until the process
// ends; in host code the array's name is no device address, so its address
// is taken once per device with hipGetSymbolAddress and used from then on.
namespace {

constexpr size_t STATIC_SCRATCH_BYTES = size_t(256) << 20;  // 256 MiB per device
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
uint64_t g_scratch_gen[MAX_DEVICES] = {};  // counts bindings of each device's scratch

}  // namespace

int mt::ws_live(mt_ctx* c) {
  if (c->static_gen == 0) return MT_OK;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (c->device < MAX_DEVICES && g_scratch_gen[c->device] == c->static_gen) return MT_OK;
  c->have_pairs = c->have_pattern = c->have_master_index = false;
  return fail(MT_ESTATE, "the static scratch was bound by another context since this context's build");
}

extern "C" int mt_build_pairs_static(mt_ctx* c, const mt_capacity* cap, int64_t* n_cand, int64_t* n_pairs,
                                     void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_build_pairs_static: null ctx");
  if (c->device < 0 || c->device >= MAX_DEVICES) return fail(MT_EINVAL, "mt_build_pairs_static: device index");
  size_t need = 0;
  if (int rc = mt_workspace_size(c, cap, &need)) return rc;
  if (need > STATIC_SCRATCH_BYTES)
    return fail(MT_ECAPACITY, "mt_build_pairs_static: the workspace needs " + std::to_string(need) +
                                  " bytes; the static scratch holds " + std::to_string(STATIC_SCRATCH_BYTES));
  DeviceScope ds(c->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
  void* ptr = nullptr;
  uint64_t gen = 0;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
      // first call on this device, with it current: the device address of
      // this device's copy of the array
      void* p = nullptr;
      hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
      g_scratch_ptr[c->device] = p;
    }
    ptr = g_scratch_ptr[c->device];
    gen = ++g_scratch_gen[c->device];
  }
  const int rc = mt_build_pairs(c, cap, ptr, STATIC_SCRATCH_BYTES, n_cand, n_pairs, stream);
  c->static_gen = gen;
  return rc;
}
