// Host side of the C ABI declared in mortar_mi355x.h: context, argument
// checks, device buffers and the launch sequence of each entry point.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <initializer_list>
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

int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

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

hipError_t ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (bytes <= b.bytes) return hipSuccess;
  if (b.p) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    e = hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (e != hipSuccess) return e;
  }
  const size_t want = bytes + bytes / 4;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return e;
  }
  b.bytes = want;
  return hipSuccess;
}

void release(Buf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

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
  mt_ctx* c = new mt_ctx();
  c->device = device;
  mt_default_params(&c->params);
  *ctx = c;
  return MT_OK;
}

int mt_destroy(mt_ctx* c) {
  if (!c) return MT_OK;
  DeviceScope ds(c->device);
  (void)hipDeviceSynchronize();
  Buf* bufs[] = {&c->box_s, &c->box_m, &c->sdata, &c->mdata, &c->reduce, &c->counters, &c->keys, &c->vals,
                 &c->keys_tmp, &c->vals_tmp, &c->cell_range, &c->sbox, &c->cand_cnt, &c->cand_tmp, &c->cand_off,
                 &c->cand_s, &c->cand_m, &c->cand_nv, &c->cand_flag, &c->scr_cnt, &c->scr_off, &c->pair_s, &c->pair_m,
                 &c->pair_nv, &c->pair_off, &c->inc_cnt, &c->inc_off, &c->inc_cur, &c->inc_list, &c->minc_cnt,
                 &c->minc_off, &c->minc_cur, &c->minc_list, &c->pat_keep, &c->pat_ecnt, &c->pat_elist, &c->D_cnt, &c->D_rowptr, &c->D_col, &c->M_cnt, &c->M_rowptr,
                 &c->M_col, &c->posD, &c->posM, &c->pair_slot, &c->maybe_list,
                 &c->maybe_flag, &c->maybe_scan, &c->mpoly_u, &c->mpoly_v, &c->mpoly_lab, &c->mpoly_nf, &c->blk, &c->gpair, &c->nrm_node, &c->nrm_el, &c->gn0, &c->nrm_sb, &c->nrm_ub, &c->nrm_cg, &c->aux_hist, &c->aux_scan, &c->mp_keys, &c->mp_vals, &c->mp_off, &c->mp_pos,
                 &c->scan_tmp, &c->sort_hist};
  for (Buf* b : bufs) release(*b);
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->aux) {
    (void)hipEventDestroy(c->aux_fork);
    (void)hipEventDestroy(c->aux_join);
    (void)hipStreamDestroy(c->aux);
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
  (void)stream;
  if (!c) return fail(MT_EINVAL, "mt_upload: null ctx");
  if (side != MT_SIDE_SLAVE && side != MT_SIDE_MASTER) return fail(MT_EINVAL, "mt_upload: bad side");
  if (n_nodes < 0 || n_el < 0 || n_nodes >= (int64_t(1) << 31) || n_el >= (int64_t(1) << 29))
    return fail(MT_EINVAL, "mt_upload: size out of range");
  if ((n_nodes > 0 && (!x || !y || !z)) || (n_el > 0 && !conn)) return fail(MT_EINVAL, "mt_upload: null array");
  if (n_el > 0 && (reinterpret_cast<uintptr_t>(conn) & 15))
    return fail(MT_EINVAL, "mt_upload: connectivity must be 16-byte aligned");
  DeviceMesh& m = c->side[side];
  m.x = x; m.y = y; m.z = z; m.conn = conn;
  m.nrm = nullptr;
  m.n_nodes = (int32_t)n_nodes;
  m.n_el = (int32_t)n_el;
  m.set = true;
  c->have_inc[side] = false;
  c->have_pairs = c->have_pattern = c->have_master_index = false;
  ++c->coord_gen;
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

static int normals_for_coords(mt_ctx* c, hipStream_t st);

// Small device-to-host reads (totals of a scan, reduction maxima, counters)
// through a pinned staging buffer of the context: the copies go straight to
// host memory, one stream synchronisation covers all of them, and the values
// are then copied to their destinations.
struct ReadBack {
  void* dst;
  const void* src;
  size_t bytes;
};
static constexpr size_t PIN_BYTES = 1024;

static hipError_t read_back(mt_ctx* c, std::initializer_list<ReadBack> items, hipStream_t st) {
  if (!c->pin) {
    hipError_t e = hipHostMalloc(&c->pin, PIN_BYTES, hipHostMallocDefault);
    if (e != hipSuccess) {
      c->pin = nullptr;
      return e;
    }
  }
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

int mt_build_pairs(mt_ctx* c, int64_t* n_cand_out, int64_t* n_pairs_out, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_build_pairs: null ctx");
  if (!c->side[0].set || !c->side[1].set) return fail(MT_ESTATE, "mt_build_pairs: upload both sides first");
  DeviceScope ds(c->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  c->have_pairs = c->have_pattern = c->have_master_index = false;
  ++c->coord_gen;
  c->side[0].nrm = nullptr;  // element frames until the nodal field is built below
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const int32_t ns = S.n_el, nm = M.n_el;

  MT_HIP(ensure(c->reduce, sizeof(PrepReduce)));
  MT_HIP(ensure(c->counters, sizeof(Counters)));
  MT_HIP(ensure(c->box_s, sizeof(double) * 6 * (size_t)ns));
  MT_HIP(ensure(c->box_m, sizeof(double) * 6 * (size_t)nm));
  MT_HIP(ensure(c->sdata, sizeof(double) * SD_N * (size_t)ns));
  MT_HIP(ensure(c->mdata, sizeof(double) * 12 * (size_t)std::max(nm, 1)));
  PrepReduce* red = c->reduce.as<PrepReduce>();
  const int nb_s = prep_blocks(ns), nb_m = prep_blocks(nm);
  MT_HIP(ensure(c->prep_part, sizeof(double) * 9 * (size_t)std::max(nb_s + nb_m, 1)));
  {
    PhaseTimer t(c, MT_T_PREP, st);
    MT_HIP(hipMemsetAsync(c->counters.p, 0, sizeof(Counters), st));
    double* part = c->prep_part.as<double>();
    MT_HIP(launch_prep(S, true, c->box_s.as<double>(), c->sdata.as<double>(), nullptr, part, st));
    MT_HIP(launch_prep(M, false, c->box_m.as<double>(), nullptr, c->mdata.as<double>(), part + 9 * (size_t)nb_s, st));
    MT_HIP(launch_prep_reduce(part, nb_s, nb_m, red, st));
  }
  PrepReduce hr;
  MT_HIP(read_back(c, {{&hr, red, sizeof(hr)}}, st));
  if (hr.bad_index) return fail(MT_EINVAL, "mt_build_pairs: connectivity index out of range");
  if (c->params.normals == MT_NORMALS_NODAL) {
    // connectivity checked: the continuous normal field, then the slave
    // frames of the candidate pass again with its plane normals
    PhaseTimer t(c, MT_T_PREP, st);
    int rc = normals_for_coords(c, st);
    if (rc) return rc;
    MT_HIP(launch_prep(S, true, c->box_s.as<double>(), c->sdata.as<double>(), nullptr, c->prep_part.as<double>(), st));
  }
  grid_from_reduce(hr, c->params.delta, c->params.bin_size, c->grid);
  const Grid& g = c->grid;

  // master elements sorted by cell, cell ranges from segment heads
  MT_HIP(ensure(c->keys, sizeof(uint32_t) * (size_t)nm));
  MT_HIP(ensure(c->vals, sizeof(uint32_t) * (size_t)nm));
  MT_HIP(ensure(c->keys_tmp, sizeof(uint32_t) * (size_t)nm));
  MT_HIP(ensure(c->vals_tmp, sizeof(uint32_t) * (size_t)nm));
  MT_HIP(ensure(c->cell_range, sizeof(int2) * (size_t)g.ncells));
  MT_HIP(ensure(c->sbox, sizeof(double) * 6 * (size_t)std::max(nm, 1)));
  MT_HIP(ensure(c->sort_hist, sizeof(int32_t) * (size_t)(2 * 256 * ((nm + 2047) / 2048 + 1) + 1)));
  MT_HIP(ensure(c->scan_tmp, 1 << 20));
  {
    PhaseTimer t(c, MT_T_BIN_SORT, st);
    MT_HIP(launch_master_keys(c->box_m.as<double>(), nm, g, c->keys.as<uint32_t>(), c->vals.as<uint32_t>(), st));
    MT_HIP(radix_sort_pairs(c->keys.as<uint32_t>(), c->vals.as<uint32_t>(), c->keys_tmp.as<uint32_t>(),
                            c->vals_tmp.as<uint32_t>(), nm, bits_for(g.ncells), c->sort_hist, c->scan_tmp, st));
    MT_HIP(hipMemsetAsync(c->cell_range.p, 0, sizeof(int2) * (size_t)g.ncells, st));
    MT_HIP(launch_cell_ranges(c->keys.as<uint32_t>(), c->vals.as<uint32_t>(), nm, c->box_m.as<double>(),
                              c->cell_range.as<int2>(), c->sbox.as<double>(), st));
  }

  // candidates: count, scan, fill (sorted by master within each slave)
  MT_HIP(ensure(c->cand_cnt, sizeof(int32_t) * ((size_t)ns + 1)));
  MT_HIP(ensure(c->cand_off, sizeof(int32_t) * ((size_t)ns + 1)));
  MT_HIP(ensure(c->cand_tmp, sizeof(int32_t) * (size_t)cand_tmp_per_slave() * (size_t)std::max(ns, 1)));
  {
    PhaseTimer t(c, MT_T_CAND, st);
    MT_HIP(launch_cand_count(c->box_s.as<double>(), ns, c->sbox.as<double>(), c->vals.as<uint32_t>(),
                             c->cell_range.as<int2>(), g, c->params.delta, c->cand_cnt.as<int32_t>(),
                             c->cand_tmp.as<int32_t>(), st));
    MT_HIP(scan_exclusive(c->cand_cnt.as<int32_t>(), c->cand_off.as<int32_t>(), ns, c->scan_tmp, st));
  }
  MT_HIP(ensure(c->scr_cnt, sizeof(int32_t) * ((size_t)ns + 1)));
  MT_HIP(ensure(c->scr_off, sizeof(int32_t) * ((size_t)ns + 1)));
  // Candidates, each screened as it is written (projection onto the slave
  // plane, degeneracy checks, separating-line test).  The candidate arrays
  // keep their size from call to call: the fill pass runs against the present
  // size and the total comes back with the screened count in one read; only
  // when the total outgrew the arrays are they enlarged and the pass repeated.
  // The first call reads the total before the fill.
  const KParams kp = kparams(c->params);
  Counters* cnt = c->counters.as<Counters>();
  auto size_cand = [c](int64_t n) -> hipError_t {
    hipError_t e = ensure(c->cand_s, sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess) e = ensure(c->cand_m, sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess) e = ensure(c->cand_nv, (size_t)n);
    if (e == hipSuccess) e = ensure(c->cand_flag, sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
    return e;
  };
  int32_t ncand32 = 0, nmaybe32 = 0;
  if (!c->cand_s.p) {
    MT_HIP(read_back(c, {{&ncand32, c->cand_off.as<int32_t>() + ns, sizeof(int32_t)}}, st));
    if (ncand32 < 0) return fail(MT_ECAPACITY, "mt_build_pairs: more than 2^31 candidates");
    MT_HIP(size_cand(ncand32));
  }
  for (int pass = 0;; ++pass) {
    const int64_t cap = (int64_t)std::min(std::min(c->cand_s.bytes, c->cand_m.bytes) / sizeof(int32_t),
                                          std::min(c->cand_nv.bytes, c->cand_flag.bytes / sizeof(int32_t)));
    {
      PhaseTimer t(c, MT_T_CAND, st);
      MT_HIP(launch_cand_fill(c->box_s.as<double>(), ns, c->sbox.as<double>(), c->vals.as<uint32_t>(),
                              c->cell_range.as<int2>(), g, c->params.delta, c->cand_tmp.as<int32_t>(),
                              c->cand_off.as<int32_t>(), c->cand_s.as<int32_t>(), c->cand_m.as<int32_t>(),
                              c->sdata.as<double>(), c->mdata.as<double>(), kp.eps_a, c->cand_nv.as<uint8_t>(),
                              c->cand_flag.as<int32_t>(), c->scr_cnt.as<int32_t>(), cnt, cap, st));
    }
    {
      PhaseTimer t(c, MT_T_COMPACT, st);
      MT_HIP(scan_exclusive(c->scr_cnt.as<int32_t>(), c->scr_off.as<int32_t>(), ns, c->scan_tmp, st));
    }
    MT_HIP(read_back(c, {{&ncand32, c->cand_off.as<int32_t>() + ns, sizeof(int32_t)},
                         {&nmaybe32, c->scr_off.as<int32_t>() + ns, sizeof(int32_t)}}, st));
    if (ncand32 < 0) return fail(MT_ECAPACITY, "mt_build_pairs: more than 2^31 candidates");
    if (ncand32 <= cap) break;
    if (pass > 0) return fail(MT_ECAPACITY, "mt_build_pairs: candidate arrays not sized");
    MT_HIP(size_cand(ncand32));
    // the degenerate-element counts of the partial pass are dropped
    static_assert(offsetof(Counters, degen_master) == offsetof(Counters, degen_slave) + sizeof(unsigned long long),
                  "degen_slave and degen_master are cleared together");
    MT_HIP(hipMemsetAsync(&cnt->degen_slave, 0, 2 * sizeof(unsigned long long), st));
  }
  const int64_t n_cand = ncand32;
  const int64_t n_maybe = nmaybe32;
  const size_t nmb = (size_t)std::max<int64_t>(n_maybe, 1);
  MT_HIP(ensure(c->maybe_list, sizeof(int32_t) * nmb));
  MT_HIP(ensure(c->maybe_flag, sizeof(int32_t) * (nmb + 1)));
  MT_HIP(ensure(c->maybe_scan, sizeof(int32_t) * (nmb + 1)));
  MT_HIP(ensure(c->mpoly_u, sizeof(double) * CAP0 * nmb));
  MT_HIP(ensure(c->mpoly_v, sizeof(double) * CAP0 * nmb));
  MT_HIP(ensure(c->mpoly_lab, CAP0 * nmb));
  MT_HIP(ensure(c->mpoly_nf, nmb));
  c->mpoly_stride = (int64_t)nmb;
  const PolyBuf mpoly{c->mpoly_u.as<double>(), c->mpoly_v.as<double>(), c->mpoly_lab.as<uint8_t>(),
                      c->mpoly_nf.as<uint8_t>(), (int64_t)nmb, nullptr};
  {
    PhaseTimer t(c, MT_T_COMPACT, st);
    MT_HIP(launch_maybe_list(c->cand_flag.as<int32_t>(), c->cand_off.as<int32_t>(), c->scr_off.as<int32_t>(), ns,
                             c->maybe_list.as<int32_t>(), st));
  }
  {
    PhaseTimer t(c, MT_T_CLIP, st);
    MT_HIP(launch_clip_screened(c->mdata.as<double>(), c->sdata.as<double>(), ns, kp, c->cand_s.as<int32_t>(), c->cand_m.as<int32_t>(),
                                c->maybe_list.as<int32_t>(), n_maybe, c->cand_nv.as<uint8_t>(),
                                c->maybe_flag.as<int32_t>(), mpoly, cnt, st));
  }
  {
    PhaseTimer t(c, MT_T_COMPACT, st);
    MT_HIP(scan_exclusive(c->maybe_flag.as<int32_t>(), c->maybe_scan.as<int32_t>(), n_maybe, c->scan_tmp, st));
  }
  int32_t np32 = 0;
  Counters hc;
  MT_HIP(read_back(c, {{&np32, c->maybe_scan.as<int32_t>() + n_maybe, sizeof(int32_t)}, {&hc, cnt, sizeof(hc)}}, st));
  const int64_t n_pairs = np32;
  MT_HIP(ensure(c->pair_s, sizeof(int32_t) * (size_t)n_pairs));
  MT_HIP(ensure(c->pair_m, sizeof(int32_t) * (size_t)n_pairs));
  MT_HIP(ensure(c->pair_nv, (size_t)n_pairs));
  MT_HIP(ensure(c->pair_slot, sizeof(int32_t) * (size_t)std::max<int64_t>(n_pairs, 1)));
  MT_HIP(ensure(c->pair_off, sizeof(int32_t) * ((size_t)ns + 1)));
  c->n_cand = n_cand;
  c->n_maybe = n_maybe;
  c->n_pairs = n_pairs;
  {
    PhaseTimer t(c, MT_T_COMPACT, st);
    MT_HIP(launch_compact_pairs(c->cand_s.as<int32_t>(), c->cand_m.as<int32_t>(), c->maybe_list.as<int32_t>(),
                                c->maybe_flag.as<int32_t>(), c->maybe_scan.as<int32_t>(), n_maybe,
                                c->mpoly_nf.as<uint8_t>(), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(),
                                c->pair_nv.as<uint8_t>(), c->pair_slot.as<int32_t>(), st));
    MT_HIP(launch_pair_off(c->scr_off.as<int32_t>(), c->maybe_scan.as<int32_t>(), ns, c->pair_off.as<int32_t>(), st));
  }
  c->poly_gen = c->coord_gen;
  c->have_pairs = true;
  if (n_cand_out) *n_cand_out = n_cand;
  if (n_pairs_out) *n_pairs_out = n_pairs;
  if (hc.degen_slave || hc.overflow)
    return fail(MT_EDEGENERATE, "mt_build_pairs: degenerate slave element or clip capacity exceeded");
  return MT_OK;
}

int mt_get_pairs(mt_ctx* c, int32_t* s, int32_t* m, uint8_t* nv, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_get_pairs: null ctx");
  if (!c->have_pairs) return fail(MT_ESTATE, "mt_get_pairs: no pair list");
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
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)c->n_cand;
  if (n == 0) return MT_OK;
  if (s) MT_HIP(hipMemcpyAsync(s, c->cand_s.p, 4 * n, hipMemcpyDeviceToDevice, st));
  if (m) MT_HIP(hipMemcpyAsync(m, c->cand_m.p, 4 * n, hipMemcpyDeviceToDevice, st));
  if (nv) MT_HIP(hipMemcpyAsync(nv, c->cand_nv.p, n, hipMemcpyDeviceToDevice, st));
  return MT_OK;
}

// Node -> (element * 4 + local index) incidence, sorted per node.
static int build_incidence(mt_ctx* c, const DeviceMesh& mesh, Buf& cntb, Buf& offb, Buf& curb, Buf& listb,
                           hipStream_t st) {
  const int32_t n = mesh.n_nodes;
  MT_HIP(ensure(cntb, sizeof(int32_t) * ((size_t)n + 1)));
  MT_HIP(ensure(offb, sizeof(int32_t) * ((size_t)n + 1)));
  MT_HIP(ensure(curb, sizeof(int32_t) * ((size_t)n + 1)));
  MT_HIP(ensure(listb, sizeof(int32_t) * 4 * (size_t)mesh.n_el));
  MT_HIP(hipMemsetAsync(cntb.p, 0, sizeof(int32_t) * ((size_t)n + 1), st));
  MT_HIP(hipMemsetAsync(curb.p, 0, sizeof(int32_t) * ((size_t)n + 1), st));
  MT_HIP(launch_inc_count(mesh.conn, mesh.n_el, cntb.as<int32_t>(), st));
  MT_HIP(scan_exclusive(cntb.as<int32_t>(), offb.as<int32_t>(), n, c->scan_tmp, st));
  MT_HIP(launch_inc_fill(mesh.conn, mesh.n_el, offb.as<int32_t>(), curb.as<int32_t>(), listb.as<int32_t>(), st));
  MT_HIP(launch_inc_sort(offb.as<int32_t>(), n, listb.as<int32_t>(), st));
  return MT_OK;
}

// The slave side's continuous normal field for the current coordinates (the
// element plane normals the frames use), or none for element normals.
static int normals_for_coords(mt_ctx* c, hipStream_t st) {
  DeviceMesh& S = c->side[0];
  if (c->params.normals != MT_NORMALS_NODAL) {
    S.nrm = nullptr;
    return MT_OK;
  }
  if (S.nrm && c->nrm_gen == c->coord_gen) return MT_OK;
  MT_HIP(ensure(c->scan_tmp, 1 << 20));
  if (!c->have_inc[0]) {
    int rc = build_incidence(c, S, c->inc_cnt, c->inc_off, c->inc_cur, c->inc_list, st);
    if (rc) return rc;
    c->have_inc[0] = true;
  }
  MT_HIP(ensure(c->nrm_node, sizeof(double) * 4 * (size_t)std::max(S.n_nodes, 1)));
  MT_HIP(ensure(c->nrm_el, sizeof(double) * 4 * (size_t)std::max(S.n_el, 1)));
  MT_HIP(launch_normals(S, c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), c->nrm_node.as<double>(),
                        c->nrm_el.as<double>(), st));
  S.nrm = c->nrm_el.as<double>();
  c->nrm_gen = c->coord_gen;
  return MT_OK;
}

int mt_csr_pattern(mt_ctx* c, int64_t* nnz_D, int64_t* nnz_M, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_csr_pattern: null ctx");
  if (!c->have_pairs) return fail(MT_ESTATE, "mt_csr_pattern: build the pair list first");
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const int32_t n = S.n_nodes;
  // the local block entries (16 per pair) bound nnz(M), so the int32 row
  // pointers cannot overflow below this size
  if (16 * (int64_t)S.n_el >= (int64_t(1) << 31) || 16 * c->n_pairs >= (int64_t(1) << 31))
    return fail(MT_ECAPACITY, "mt_csr_pattern: more than 2^31 block entries");
  PhaseTimer timer(c, MT_T_PATTERN, st);
  if (!c->have_inc[0]) {
    int rc = build_incidence(c, S, c->inc_cnt, c->inc_off, c->inc_cur, c->inc_list, st);
    if (rc) return rc;
    c->have_inc[0] = true;
  }
  c->have_master_index = false;
  // per-element master-node lists of the M rows, before the fork: a short
  // kernel that would otherwise wait behind the forward's blocks
  MT_HIP(ensure(c->pat_ecnt, sizeof(int32_t) * (size_t)std::max(S.n_el, 1)));
  MT_HIP(ensure(c->pat_elist, sizeof(int32_t) * (size_t)pattern_elem_list() * (size_t)std::max(S.n_el, 1)));
  MT_HIP(ensure(c->pat_keep, sizeof(int32_t) * (size_t)pattern_keep_per_row() * (size_t)std::max(n, 1)));
  MT_HIP(ensure(c->D_cnt, sizeof(int32_t) * ((size_t)n + 1)));
  MT_HIP(ensure(c->M_cnt, sizeof(int32_t) * ((size_t)n + 1)));
  MT_HIP(ensure(c->D_rowptr, sizeof(int32_t) * ((size_t)n + 1)));
  MT_HIP(ensure(c->M_rowptr, sizeof(int32_t) * ((size_t)n + 1)));
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
  const bool aux = c->params.element_rule == 0 && c->n_pairs > 0 && c->poly_gen == c->coord_gen;
  if (aux) {
    if (!c->have_inc[1]) {
      int rc = build_incidence(c, M, c->minc_cnt, c->minc_off, c->minc_cur, c->minc_list, st);
      if (rc) return rc;
      c->have_inc[1] = true;
    }
    const int64_t np = c->n_pairs;
    MT_HIP(ensure(c->blk, sizeof(double) * 36 * (size_t)np));
    if (!c->aux) {
      MT_HIP(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
      MT_HIP(hipEventCreateWithFlags(&c->aux_fork, hipEventDisableTiming));
      MT_HIP(hipEventCreateWithFlags(&c->aux_join, hipEventDisableTiming));
    }
    MT_HIP(hipEventRecord(c->aux_fork, st));
    MT_HIP(hipStreamWaitEvent(c->aux, c->aux_fork, 0));
    {
      PhaseTimer t(c, MT_T_PAIR_FWD, c->aux);
      MT_HIP(launch_pair_fwd(S, M, kparams(c->params), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), np,
                             poly_buf(c), c->blk.as<double>(), np, c->counters.as<Counters>(), c->aux));
    }
  }
  MT_HIP(launch_pattern_rows(false, c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), n, c->pair_off.as<int32_t>(),
                             c->pair_m.as<int32_t>(), S.conn, M.conn, c->D_cnt.as<int32_t>(), c->M_cnt.as<int32_t>(),
                             nullptr, nullptr, nullptr, nullptr, c->pat_keep.as<int32_t>(), nullptr, S.n_el, nullptr,
                             c->n_pairs, c->pat_ecnt.as<int32_t>(), c->pat_elist.as<int32_t>(), st));
  int32_t tot[2] = {0, 0};
  MT_HIP(scan_exclusive(c->D_cnt.as<int32_t>(), c->D_rowptr.as<int32_t>(), n, c->scan_tmp, st));
  MT_HIP(scan_exclusive(c->M_cnt.as<int32_t>(), c->M_rowptr.as<int32_t>(), n, c->scan_tmp, st));
  // The fill pass needs the row pointers on the device only: the column arrays
  // are sized by the local block entries (16 per slave element for D, 16 per
  // pair for M), so the pass is launched before the totals are read back and
  // the host waits once, after it.
  MT_HIP(ensure(c->D_col, sizeof(int32_t) * 16 * (size_t)std::max(S.n_el, 1)));
  MT_HIP(ensure(c->M_col, sizeof(int32_t) * 16 * (size_t)std::max<int64_t>(c->n_pairs, 1)));
  // the fill pass also writes the CSR positions of every local block entry
  MT_HIP(ensure(c->posD, sizeof(int32_t) * 16 * (size_t)std::max(S.n_el, 1)));
  MT_HIP(ensure(c->posM, sizeof(int32_t) * 16 * (size_t)std::max<int64_t>(c->n_pairs, 1)));
  MT_HIP(launch_pattern_rows(true, c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), n, c->pair_off.as<int32_t>(),
                             c->pair_m.as<int32_t>(), S.conn, M.conn, nullptr, nullptr, c->D_rowptr.as<int32_t>(), c->M_rowptr.as<int32_t>(), c->D_col.as<int32_t>(),
                             c->M_col.as<int32_t>(), c->pat_keep.as<int32_t>(), c->posD.as<int32_t>(), S.n_el,
                             c->posM.as<int32_t>(), c->n_pairs, nullptr, nullptr, st));
  if (aux) {
    {
      PhaseTimer t(c, MT_T_GRAD_REDUCE, c->aux);
      int rc = build_master_index(c, c->aux, c->aux_hist, c->aux_scan);
      if (rc) return rc;
    }
    MT_HIP(hipEventRecord(c->aux_join, c->aux));
    c->blk_gen = c->coord_gen;
    c->blk_pending = true;
  }
  MT_HIP(read_back(c, {{&tot[0], c->D_rowptr.as<int32_t>() + n, 4}, {&tot[1], c->M_rowptr.as<int32_t>() + n, 4}}, st));
  c->nnz_D = tot[0];
  c->nnz_M = tot[1];
  if (aux) MT_HIP(hipStreamWaitEvent(st, c->aux_join, 0));
  c->have_pattern = true;
  ++c->pattern_gen;
  if (nnz_D) *nnz_D = c->nnz_D;
  if (nnz_M) *nnz_M = c->nnz_M;
  return MT_OK;
}

int mt_get_csr(mt_ctx* c, int32_t* D_rowptr, int32_t* D_col, int32_t* M_rowptr, int32_t* M_col, void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_get_csr: null ctx");
  if (!c->have_pattern) return fail(MT_ESTATE, "mt_get_csr: no pattern");
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
  if (!c) return fail(MT_EINVAL, "mt_integrate: null ctx");
  if (!c->have_pattern) return fail(MT_ESTATE, "mt_integrate: build pairs and pattern first");
  if ((c->nnz_D && !D_val) || (c->nnz_M && !M_val) || (c->side[0].n_nodes && !gap))
    return fail(MT_EINVAL, "mt_integrate: null output");
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  const int64_t np = c->n_pairs;
  MT_HIP(ensure(c->blk, sizeof(double) * 36 * (size_t)std::max<int64_t>(np, 1)));
  {
    int rc = ensure_poly(c);
    if (!rc) rc = normals_for_coords(c, st);
    if (rc) return rc;
  }
  const PolyBuf poly = poly_buf(c);
  if (c->params.element_rule > 0) {
    // element-based integration: no clip polygons
    PhaseTimer t(c, MT_T_PAIR_FWD, st);
    MT_HIP(launch_elem_fwd(S, M, kparams(c->params), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(),
                           c->pair_off.as<int32_t>(), np, c->blk.as<double>(), np, c->counters.as<Counters>(), st));
    c->blk_gen = -1;
  } else {
    if (c->poly_gen != c->coord_gen) {
      PhaseTimer t(c, MT_T_PAIR_POLY, st);
      MT_HIP(launch_pair_poly(S, M, kparams(c->params), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), np, poly,
                              st));
      c->poly_gen = c->coord_gen;
    }
    // the blocks mt_csr_pattern computed serve the first mt_integrate after
    // it (for unchanged coordinates); every other call computes them
    if (!(c->blk_pending && c->blk_gen == c->coord_gen)) {
      PhaseTimer t(c, MT_T_PAIR_FWD, st);
      MT_HIP(launch_pair_fwd(S, M, kparams(c->params), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), np, poly,
                             c->blk.as<double>(), np, c->counters.as<Counters>(), st));
      c->blk_gen = c->coord_gen;
    }
  }
  c->blk_pending = false;
  PhaseTimer t(c, MT_T_ASSEMBLE, st);
  MT_HIP(launch_assemble(c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), S.n_nodes, c->pair_off.as<int32_t>(),
                         c->D_rowptr.as<int32_t>(), c->M_rowptr.as<int32_t>(), c->posD.as<int32_t>(), S.n_el,
                         c->posM.as<int32_t>(), c->blk.as<double>(), np, D_val, M_val, gap, st));
  return MT_OK;
}

namespace {
__global__ void k_iota(uint32_t* v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (uint32_t)i;
}
}  // namespace

}  // extern "C"

// The pair polygons live in the screened-candidate polygon buffer of the
// last mt_build_pairs (pair p at entry pair_slot[p]); it holds an entry for
// every pair, also when the polygons are recomputed for new coordinates.
int mt::ensure_poly(mt_ctx* c) {
  if (c->n_pairs > 0 && (!c->pair_slot.p || !c->mpoly_nf.p))
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
  return build_master_index(c, st, c->sort_hist, c->scan_tmp);
}

int mt::build_master_index(mt_ctx* c, hipStream_t st, Buf& hist, Buf& scan_tmp) {
  const DeviceMesh& M = c->side[1];
  const int64_t np = c->n_pairs;
  MT_HIP(ensure(c->mp_keys, sizeof(uint32_t) * (size_t)np));
  MT_HIP(ensure(c->mp_vals, sizeof(uint32_t) * (size_t)np));
  MT_HIP(ensure(c->keys_tmp, sizeof(uint32_t) * (size_t)np));
  MT_HIP(ensure(c->vals_tmp, sizeof(uint32_t) * (size_t)np));
  MT_HIP(ensure(c->mp_off, sizeof(int32_t) * 2 * ((size_t)M.n_el + 1)));
  if (np > 0) {
    MT_HIP(hipMemcpyAsync(c->mp_keys.p, c->pair_m.p, 4 * (size_t)np, hipMemcpyDeviceToDevice, st));
    k_iota<<<(unsigned)((np + 255) / 256), 256, 0, st>>>(c->mp_vals.as<uint32_t>(), np);
    MT_HIP(hipGetLastError());
  }
  MT_HIP(radix_sort_pairs(c->mp_keys.as<uint32_t>(), c->mp_vals.as<uint32_t>(), c->keys_tmp.as<uint32_t>(),
                          c->vals_tmp.as<uint32_t>(), np, bits_for(std::max<int32_t>(M.n_el, 2)), hist,
                          scan_tmp, st));
  MT_HIP(hipMemsetAsync(c->mp_off.p, 0, sizeof(int32_t) * 2 * ((size_t)M.n_el + 1), st));
  MT_HIP(ensure(c->mp_pos, sizeof(int32_t) * (size_t)std::max<int64_t>(np, 1)));
  MT_HIP(launch_mpair_off(c->mp_keys.as<uint32_t>(), c->mp_vals.as<uint32_t>(), np, M.n_el, c->mp_off.as<int32_t>(),
                          c->mp_pos.as<int32_t>(), st));
  c->have_master_index = true;
  return MT_OK;
}

extern "C" {

int mt_backward(mt_ctx* c, const double* W_D, const double* W_M, const double* w_g, double* gXs, double* gXm,
                void* stream) {
  if (!c) return fail(MT_EINVAL, "mt_backward: null ctx");
  if (c->params.element_rule > 0)
    return fail(MT_EUNSUPPORTED, "mt_backward: element-based integration has no backward pass");
  if (!c->have_pattern) return fail(MT_ESTATE, "mt_backward: build pairs and pattern first");
  const DeviceMesh& S = c->side[0];
  const DeviceMesh& M = c->side[1];
  if ((c->nnz_D && !W_D) || (c->nnz_M && !W_M) || (S.n_nodes && (!w_g || !gXs)) || (M.n_nodes && !gXm))
    return fail(MT_EINVAL, "mt_backward: null argument");
  DeviceScope ds(c->device);
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  {
    PhaseTimer t(c, MT_T_GRAD_REDUCE, st);
    int rc = ensure_master_index(c, st);
    if (rc) return rc;
  }
  const int64_t np = c->n_pairs;
  MT_HIP(ensure(c->gpair, sizeof(double) * 24 * (size_t)std::max<int64_t>(np, 1)));
  {
    int rc = ensure_poly(c);
    if (!rc) rc = normals_for_coords(c, st);
    if (rc) return rc;
  }
  const bool nodal = c->params.normals == MT_NORMALS_NODAL;
  if (nodal) MT_HIP(ensure(c->gn0, sizeof(double) * 3 * (size_t)std::max<int64_t>(np, 1)));
  const PolyBuf poly = poly_buf(c);
  if (c->poly_gen != c->coord_gen) {
    PhaseTimer t(c, MT_T_PAIR_POLY, st);
    MT_HIP(launch_pair_poly(S, M, kparams(c->params), c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), np, poly, st));
    c->poly_gen = c->coord_gen;
  }
  {
    PhaseTimer t(c, MT_T_PAIR_BWD, st);
    const KParams kp = kparams(c->params);
    if (kp.dual && c->blk_gen != c->coord_gen) {
      // the dual adjoint reads each pair's dual blocks: those staged by the
      // last mt_integrate unless the coordinates or pairs changed since
      MT_HIP(ensure(c->blk, sizeof(double) * 36 * (size_t)std::max<int64_t>(np, 1)));
      MT_HIP(launch_pair_fwd(S, M, kp, c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), np, poly,
                             c->blk.as<double>(), np, c->counters.as<Counters>(), st));
      c->blk_gen = c->coord_gen;
    }
    MT_HIP(launch_pair_bwd(S, M, kp, c->pair_s.as<int32_t>(), c->pair_m.as<int32_t>(), np, poly,
                           c->mp_pos.as<int32_t>(),
                           c->posD.as<int32_t>(), S.n_el, c->posM.as<int32_t>(), W_D, W_M, w_g,
                           kp.dual ? c->blk.as<double>() : nullptr, c->gpair.as<double>(),
                           nodal ? c->gn0.as<double>() : nullptr, np, c->counters.as<Counters>(), st));
  }
  PhaseTimer t(c, MT_T_GRAD_REDUCE, st);
  MT_HIP(launch_grad_slave(c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), S.n_nodes, c->pair_off.as<int32_t>(),
                           c->gpair.as<double>(), np, gXs, st));
  const int32_t* mo = c->mp_off.as<int32_t>();
  MT_HIP(launch_grad_master(c->minc_off.as<int32_t>(), c->minc_list.as<int32_t>(), M.n_nodes, mo, mo + M.n_el,
                            c->gpair.as<double>(), np, gXm, st));
  if (nodal) {
    // through the element plane normals to the nodal normals and the
    // coordinates of the neighbouring elements
    MT_HIP(ensure(c->nrm_sb, sizeof(double) * 4 * (size_t)std::max(S.n_el, 1)));
    MT_HIP(ensure(c->nrm_ub, sizeof(double) * 4 * (size_t)std::max(S.n_nodes, 1)));
    MT_HIP(ensure(c->nrm_cg, sizeof(double) * 12 * (size_t)std::max(S.n_el, 1)));
    MT_HIP(launch_normal_chain(S, c->inc_off.as<int32_t>(), c->inc_list.as<int32_t>(), c->pair_off.as<int32_t>(),
                               c->gn0.as<double>(), np, c->nrm_node.as<double>(), c->nrm_el.as<double>(),
                               c->nrm_sb.as<double>(), c->nrm_ub.as<double>(), c->nrm_cg.as<double>(), gXs, nullptr,
                               nullptr, st));
  }
  return MT_OK;
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
  out->n_candidates = c->n_cand;
  out->n_pairs = c->n_pairs;
  out->nnz_D = c->nnz_D;
  out->nnz_M = c->nnz_M;
  for (int d = 0; d < 3; ++d) {
    out->n_bins[d] = c->grid.n[d];
    out->bin_size[d] = c->grid.beta[d];
  }
  if (!c->counters.p) return MT_OK;
  DeviceScope ds(c->device);
  Counters* dc = c->counters.as<Counters>();
  MT_HIP(hipMemsetAsync(dc->hist, 0, sizeof(dc->hist), c->last_stream));
  if (c->have_pairs)
    MT_HIP(launch_nv_hist(c->cand_nv.as<uint8_t>(), c->n_cand, dc->hist, c->last_stream));
  Counters hc;
  MT_HIP(read_back(c, {{&hc, c->counters.p, sizeof(hc)}}, c->last_stream));
  for (int i = 0; i < 17; ++i) out->nverts_hist[i] = (int64_t)hc.hist[i];
  out->n_noconv = (int64_t)hc.noconv;
  out->n_overflow = (int64_t)hc.overflow;
  out->n_degenerate_slave = (int64_t)hc.degen_slave;
  out->n_degenerate_master = (int64_t)hc.degen_master;
  return MT_OK;
}

}  // extern "C"

int mt::ensure_normals(mt_ctx* c, hipStream_t st) { return normals_for_coords(c, st); }
