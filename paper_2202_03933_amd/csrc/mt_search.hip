// Contact search on the GPU: element preparation, Cartesian bins sorted by
// radix sort with bin ranges from segment heads, and the candidate lists of
// every slave element from its own bin and the 26 neighbouring bins
// (Alg. 2 and its bin-sizing rule, Sec. "Distributed storage: going to large
// problems").
#include <cmath>
#include <algorithm>
#include <cstring>

#include "mt_geometry.h"
#include "mt_internal.h"

namespace mt {

namespace {

constexpr int BS = 256;
constexpr int PREP_PART = 9;  // per-block partials: ext, edge, -lo xyz, hi xyz, bad (bits)

__device__ __forceinline__ unsigned long long order_key(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__host__ __device__ inline double from_order_key(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  double x;
  memcpy(&x, &b, sizeof(x));
  return x;
}

template <class T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const T y = __shfl_xor(x, d, 64);
    x = x > y ? x : y;
  }
  return x;
}
template <class T>
__device__ __forceinline__ T wave_min(T x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const T y = __shfl_xor(x, d, 64);
    x = x < y ? x : y;
  }
  return x;
}

// Element preparation: bounding boxes, the grid reductions (largest box
// extent, longest slave edge, bounding box of all element boxes), for slave
// elements the precomputed frame and projected polygon of the candidate
// pass, for master elements their node coordinates gathered element by
// element (md[12 e + 3 k + d], read with 16-byte loads by the candidate
// pass).  Both sides in one launch (blockIdx.y: 0 slave, 1 master), so that
// the shorter master pass fills the slave pass's tail; within a side a
// grid-stride loop over its P.nb blocks, each writing its partials of the
// reductions to P.part[block].
struct PrepSide {
  const double* x;
  const double* y;
  const double* z;
  const int32_t* conn;
  const double* nrm;  // slave element plane normals (continuous field) or null
  double* box;
  double* sd;  // slave: frame data
  double* md;  // master: gathered node coordinates
  double* part;
  int32_t n_el, n_nodes, nb;
};

__global__ __launch_bounds__(BS) void k_prep(PrepSide s_side, PrepSide m_side) {
  const bool slave = blockIdx.y == 0;
  const PrepSide& P = slave ? s_side : m_side;
  if ((int)blockIdx.x >= P.nb) return;  // the whole block: the side has fewer blocks
  const double* __restrict__ x = P.x;
  const double* __restrict__ y = P.y;
  const double* __restrict__ z = P.z;
  const int32_t* __restrict__ conn = P.conn;
  const int32_t n_el = P.n_el, n_nodes = P.n_nodes;
  const double* __restrict__ nrm = P.nrm;
  double* __restrict__ box = P.box;
  double* __restrict__ sd = P.sd;
  double* __restrict__ md = P.md;
  double* __restrict__ part = P.part;
  __shared__ double sh[BS / 64][8];
  __shared__ int bad;  // 1: connectivity out of range, 2: a coordinate not finite
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double ext = 0.0, edge = 0.0;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int e = blockIdx.x * BS + threadIdx.x; e < n_el; e += P.nb * BS) {
    const int4 c = load_conn(conn, e);
    const bool ok = c.x >= 0 && c.y >= 0 && c.z >= 0 && c.w >= 0 && c.x < n_nodes && c.y < n_nodes &&
                    c.z < n_nodes && c.w < n_nodes;
    if (!ok) {
      atomicOr(&bad, 1);
      continue;
    }
    double X[4][3];
    load_nodes(x, y, z, c, X);
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int d = 0; d < 3; ++d) fin = fin && isfinite(X[k][d]);
    if (!fin) atomicOr(&bad, 2);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double l = fmin(fmin(X[0][d], X[1][d]), fmin(X[2][d], X[3][d]));
      const double h = fmax(fmax(X[0][d], X[1][d]), fmax(X[2][d], X[3][d]));
      box[(int64_t)d * n_el + e] = l;
      box[(int64_t)(3 + d) * n_el + e] = h;
      ext = fmax(ext, h - l);
      lo[d] = fmin(lo[d], l);
      hi[d] = fmax(hi[d], h);
    }
    if (slave) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const double a = X[k1][0] - X[k][0], b = X[k1][1] - X[k][1], cc = X[k1][2] - X[k][2];
        edge = fmax(edge, sqrt(a * a + b * b + cc * cc));
      }
      double f[12], hs[4], As, hmax;
      V2 S[4];
      slave_frame_p(X, nrm ? nrm + 4 * (int64_t)e : nullptr, f);
      slave_setup(X, f, S, hs, As, hmax);
#pragma unroll
      for (int k = 0; k < 12; ++k) sd[(int64_t)k * n_el + e] = f[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        sd[(int64_t)(12 + k) * n_el + e] = S[k].u;
        sd[(int64_t)(16 + k) * n_el + e] = S[k].v;
      }
      sd[(int64_t)20 * n_el + e] = As;
      sd[(int64_t)21 * n_el + e] = hmax;
    } else {
      double2* dst = reinterpret_cast<double2*>(md + (int64_t)12 * e);
#pragma unroll
      for (int k = 0; k < 6; ++k) dst[k] = make_double2(X[(2 * k) / 3][(2 * k) % 3], X[(2 * k + 1) / 3][(2 * k + 1) % 3]);
    }
  }
  double v[8] = {ext, edge, -lo[0], -lo[1], -lo[2], hi[0], hi[1], hi[2]};
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = wave_max(v[k]);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 8) {
    double m = sh[0][threadIdx.x];
#pragma unroll
    for (int i = 1; i < BS / 64; ++i) m = fmax(m, sh[i][threadIdx.x]);
    part[(int64_t)blockIdx.x * PREP_PART + threadIdx.x] = m;
  }
  if (threadIdx.x == 8) part[(int64_t)blockIdx.x * PREP_PART + 8] = (double)bad;
}

__device__ void grid_from(const PrepReduce* __restrict__ red, double delta, double bin_size, int64_t max_cells,
                          DevState* st);

// Final reduction of the per-block partials of both sides (nb_s slave
// blocks first, then nb_m master blocks) into the grid quantities, then the
// search grid from them (grid_from, by the same thread).
__global__ __launch_bounds__(BS) void k_prep_reduce(const double* __restrict__ part, int nb_s, int nb_m,
                                                     PrepReduce* red, double delta, double bin_size,
                                                     int64_t max_cells, DevState* st) {
  __shared__ double sh[BS / 64][PREP_PART];
  double v[PREP_PART];
#pragma unroll
  for (int k = 0; k < PREP_PART; ++k) v[k] = k == 0 || k == 1 || k == 8 ? 0.0 : -INFINITY;
  int bits = 0;
  for (int b = threadIdx.x; b < nb_s + nb_m; b += BS) {
#pragma unroll
    for (int k = 0; k < PREP_PART - 1; ++k) {
      const double x = part[(int64_t)b * PREP_PART + k];
      if (k != 1 || b < nb_s) v[k] = fmax(v[k], x);
    }
    bits |= (int)part[(int64_t)b * PREP_PART + 8];
  }
  __shared__ int sbits;
  if (threadIdx.x == 0) sbits = 0;
  __syncthreads();
  if (bits) atomicOr(&sbits, bits);
#pragma unroll
  for (int k = 0; k < PREP_PART; ++k) v[k] = wave_max(v[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < PREP_PART; ++k) sh[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[PREP_PART];
#pragma unroll
    for (int k = 0; k < PREP_PART; ++k) {
      r[k] = sh[0][k];
#pragma unroll
      for (int i = 1; i < BS / 64; ++i) r[k] = fmax(r[k], sh[i][k]);
    }
    red->emax_bits = (unsigned long long)__double_as_longlong(r[0]);
    red->edge_bits = (unsigned long long)__double_as_longlong(r[1]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red->lo_key[d] = r[2 + d] > -INFINITY ? order_key(-r[2 + d]) : ~0ull;
      red->hi_key[d] = r[5 + d] > -INFINITY ? order_key(r[5 + d]) : 0ull;
    }
    red->bad_index = sbits;
    red->pad = 0;
    grid_from(red, delta, bin_size, max_cells, st);
  }
}

// Cell index along one axis, clamped to [0, n); a NaN position (a
// non-finite coordinate, reported by the preparation) lands in cell 0.
__device__ __forceinline__ int cell_coord(double c, double lo, double inv_beta, int n) {
  double t = floor((c - lo) * inv_beta);
  t = fmax(t, 0.0);
  t = fmin(t, (double)(n - 1));
  return (int)t;
}

// ---- box prefilter ------------------------------------------------------------
// The candidate test compares (slave lo - delta) with master hi and master lo
// with (slave hi + delta) on each axis.  Master box bounds are stored as
// quantisation levels (21 bits each, one 16-byte record per master): level q
// of axis d stands for B(q) = qo + q qu, computed the same way wherever it is
// used, so B is non-decreasing in q, and a master bound x is stored as the
// largest q with B(q) <= x (then B(q) <= x < B(q + 1)).  For each slave the
// walk computes, per axis, the levels around a = lo - delta and c = hi +
// delta; a test is then decided by integer comparisons when the levels
// separate the values, and by the exact FP64 test otherwise, so the
// candidate list is the one of the exact test.
constexpr int QBITS = 21;
constexpr int64_t QMAX = (int64_t(1) << QBITS) - 1;
constexpr uint64_t QMASK = (uint64_t(1) << QBITS) - 1;
constexpr uint64_t QEXACT = uint64_t(1) << 63;  // record flag: exact test only

__device__ __forceinline__ double qlevel(const Grid& g, int d, int64_t q) { return g.qo[d] + (double)q * g.qu[d]; }

// max{q in [0, QMAX + 1] : B(q) <= x (B(q) < x when strict)}, -1 when there is
// none; x finite.  A guess, a few unit steps, then bisection.
__device__ int64_t q_max_le(const Grid& g, int d, double x, bool strict) {
  auto ok = [&](int64_t q) {
    const double b = qlevel(g, d, q);
    return strict ? b < x : b <= x;
  };
  const double f = floor((x - g.qo[d]) / g.qu[d]);
  int64_t q = (int64_t)fmin(fmax(f, -1.0), (double)(QMAX + 1));
  for (int it = 0; it < 4; ++it) {
    if (q >= 0 && !ok(q)) {
      --q;
    } else if (q <= QMAX && ok(q + 1)) {
      ++q;
    } else {
      return q;
    }
  }
  int64_t lo = -1, hi = QMAX + 2;  // ok(lo) and !ok(hi), taken as given at the ends
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (ok(mid))
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Per-slave thresholds of the prefilter: on axis d a master with levels
// (ql, qh) fails when qh < ea or ql > ecf, passes when qh > la and ql < ecp;
// anything else goes to the exact test.
struct QSlave {
  int32_t la[3], ea[3], ecp[3], ecf[3];
};

__device__ __forceinline__ QSlave q_slave(const Grid& g, const double lo[3], const double hi[3], double delta) {
  QSlave t;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double a = lo[d] - delta, c = hi[d] + delta;  // as in the exact test
    if (isfinite(a) && isfinite(c)) {
      t.la[d] = (int32_t)q_max_le(g, d, a, true);
      t.ea[d] = (int32_t)q_max_le(g, d, a, false);
      t.ecp[d] = t.ecf[d] = (int32_t)q_max_le(g, d, c, false);
    } else {  // never decided by the levels
      t.la[d] = (int32_t)QMAX + 1;
      t.ea[d] = -1;
      t.ecp[d] = -1;
      t.ecf[d] = (int32_t)QMAX + 1;
    }
  }
  return t;
}

// Search grid from the element reductions (one thread):
// beta_min = max(longest slave edge, largest box extent + delta, bin_size)
// (the paper's rule without a motion term, raised so that 27 cells are
// complete), the node bounding box expanded by beta_min, max(1, floor(L /
// beta_min)) cells per axis, the dense cell table coarsened to at most
// max_cells cells (coarser cells stay complete).
__device__ void grid_from(const PrepReduce* __restrict__ red, double delta, double bin_size, int64_t max_cells,
                          DevState* st) {
  const double emax = __longlong_as_double((long long)red->emax_bits);
  const double edge = __longlong_as_double((long long)red->edge_bits);
  double beta_min = fmax(fmax(edge, emax + delta), bin_size) * (1.0 + 0x1p-20);
  if (!(beta_min > 0.0) || !isfinite(beta_min)) beta_min = 1.0;
  Grid g;
  double L[3];
  int64_t n[3];
  for (int d = 0; d < 3; ++d) {
    double lo = from_order_key(red->lo_key[d]);
    double hi = from_order_key(red->hi_key[d]);
    if (!(lo <= hi) || !isfinite(lo) || !isfinite(hi)) { lo = 0.0; hi = 0.0; }
    g.lo[d] = lo - beta_min;
    L[d] = (hi + beta_min) - g.lo[d];
    const double q = floor(L[d] / beta_min);
    n[d] = q >= 1.0 ? (q < (double)max_cells ? (int64_t)q : max_cells) : 1;
  }
  // (the product in double: three factors up to max_cells overflow int64)
  while ((double)n[0] * (double)n[1] * (double)n[2] > (double)max_cells) {
    const double f = cbrt((double)n[0] * (double)n[1] * (double)n[2] / (double)max_cells) * 1.01;
    for (int d = 0; d < 3; ++d) {
      const double q = floor((double)n[d] / f);
      n[d] = q >= 1.0 ? (int64_t)q : 1;
    }
  }
  for (int d = 0; d < 3; ++d) {
    g.n[d] = (int32_t)n[d];
    g.beta[d] = L[d] / (double)n[d];
    g.inv_beta[d] = 1.0 / g.beta[d];
  }
  g.ncells = n[0] * n[1] * n[2];
  // quantisation of the prefilter: levels from the grid's low corner in
  // steps of a power of two, QMAX + 1 of them spanning at least twice the
  // grid, so every box bound of the grid lies between levels 0 and QMAX
  for (int d = 0; d < 3; ++d) {
    g.qo[d] = g.lo[d];
    int e = 0;
    (void)frexp(2.0 * L[d] / (double)QMAX, &e);
    g.qu[d] = L[d] > 0.0 && isfinite(L[d]) ? ldexp(1.0, e) : 1.0;
  }
  // padded so that rounding in the box centres cannot move a centre across
  g.reach = (delta + 0.5 * emax) * (1.0 + 1e-9) + 1e-9 * beta_min;
  st->grid = g;
  if (red->bad_index & 2) st->flags |= DS_NONFINITE;
}


// Master keys (cell of each master box centre, master index as value); the
// same launch clears the cell table over the grid's cells (grid-stride).
__global__ __launch_bounds__(BS) void k_master_keys(const double* __restrict__ box, int32_t n,
                                                     const Grid* __restrict__ gp, uint32_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals, int2* __restrict__ range) {
  const int64_t nc = gp->ncells;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < nc; i += (int64_t)gridDim.x * BS)
    range[i] = make_int2(0, 0);
  const int m = blockIdx.x * BS + threadIdx.x;
  if (m >= n) return;
  const Grid g = *gp;
  int ix[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double c = 0.5 * (box[(int64_t)d * n + m] + box[(int64_t)(3 + d) * n + m]);
    ix[d] = cell_coord(c, g.lo[d], g.inv_beta[d], g.n[d]);
  }
  keys[m] = (uint32_t)(ix[0] + g.n[0] * (ix[1] + g.n[1] * ix[2]));
  vals[m] = (uint32_t)m;
}

// Cell ranges [x, y) of the cell-sorted master list from segment heads, and
// the master boxes copied into cell order (sbox[i] = lo xyz, hi xyz of the
// i-th sorted master) so that the candidate walks read them contiguously.
__global__ __launch_bounds__(BS) void k_cell_ranges(const uint32_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ vals, int32_t n,
                                                     const double* __restrict__ box_m, const Grid* __restrict__ gp,
                                                     int2* __restrict__ range, double* __restrict__ sbox,
                                                     uint64_t* __restrict__ qbox) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i];
  if (i == 0 || keys[i - 1] != k) range[k].x = i;
  if (i == n - 1 || keys[i + 1] != k) range[k].y = i + 1;
  const int m = (int)vals[i];
  double bx[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) bx[j] = box_m[(int64_t)j * n + m];
  double2* dst = reinterpret_cast<double2*>(sbox + (int64_t)6 * i);
  dst[0] = make_double2(bx[0], bx[1]);
  dst[1] = make_double2(bx[2], bx[3]);
  dst[2] = make_double2(bx[4], bx[5]);
  // quantised record: lo levels in the first word, hi levels in the second
  const Grid g = *gp;
  uint64_t w[2] = {0, 0};
  bool exact = false;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int d = j % 3;
    int64_t q = -1;
    if (isfinite(bx[j])) q = q_max_le(g, d, bx[j], false);
    if (q < 0 || q > QMAX) {
      exact = true;
      q = 0;
    }
    w[j / 3] |= (uint64_t)q << (QBITS * d);
  }
  if (exact) w[1] |= QEXACT;
  reinterpret_cast<ulonglong2*>(qbox)[i] = make_ulonglong2(w[0], w[1]);
}

struct SlaveBox {
  double lo[3], hi[3];
};

__device__ __forceinline__ SlaveBox load_box(const double* __restrict__ box, int32_t n, int e) {
  SlaveBox b;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = box[(int64_t)d * n + e];
    b.hi[d] = box[(int64_t)(3 + d) * n + e];
  }
  return b;
}

// Candidate test: closed overlap of the delta-enlarged slave box and the
// i-th master box in cell order on all three axes.
__device__ __forceinline__ bool touch(const SlaveBox& s, const double* __restrict__ sbox, int i, double delta) {
  const double2* b = reinterpret_cast<const double2*>(sbox + (int64_t)6 * i);
  const double2 b0 = b[0], b1 = b[1], b2 = b[2];
  const double mlo[3] = {b0.x, b0.y, b1.x}, mhi[3] = {b1.y, b2.x, b2.y};
  bool t = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) t = t && (s.lo[d] - delta) <= mhi[d] && mlo[d] <= (s.hi[d] + delta);
  return t;
}

// The candidate test through the quantised record first (one 16-byte load);
// the exact test only when the levels do not decide it.
__device__ __forceinline__ bool touch_q(const SlaveBox& s, const QSlave& t, const double* __restrict__ sbox,
                                        const uint64_t* __restrict__ qbox, int i, double delta) {
  const ulonglong2 rec = reinterpret_cast<const ulonglong2*>(qbox)[i];
  bool fail = false, pass = (rec.y & QEXACT) == 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int32_t ql = (int32_t)((rec.x >> (QBITS * d)) & QMASK);
    const int32_t qh = (int32_t)((rec.y >> (QBITS * d)) & QMASK);
    fail = fail || qh < t.ea[d] || ql > t.ecf[d];
    pass = pass && qh > t.la[d] && ql < t.ecp[d];
  }
  if ((rec.y & QEXACT) == 0) {
    if (fail) return false;
    if (pass) return true;
  }
  return touch(s, sbox, i, delta);
}

constexpr int CCAP = 48;  // per-thread LDS segment of the long-list fill (masters)
constexpr int CTMP = 32;  // candidates per slave kept by the count pass
constexpr int G = 2;      // lanes per slave element in the count and fill passes
static_assert(64 % G == 0 && BS % G == 0, "groups must not straddle a wave");
constexpr int OWN = CTMP / G;  // candidates per lane in the grouped fill

// The 27 cells around the slave centre's cell, restricted to those that can
// hold the centre of a touching master (within g.reach of the box).
__device__ __forceinline__ void cell_window(const SlaveBox& b, const Grid& g, int c0[3], int c1[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ic = cell_coord(0.5 * (b.lo[d] + b.hi[d]), g.lo[d], g.inv_beta[d], g.n[d]);
    c0[d] = max(ic - 1, cell_coord(b.lo[d] - g.reach, g.lo[d], g.inv_beta[d], g.n[d]));
    c1[d] = min(ic + 1, cell_coord(b.hi[d] + g.reach, g.lo[d], g.inv_beta[d], g.n[d]));
  }
}

// The cells c0[0] .. c1[0] of one (y, z) row have consecutive keys, so their
// masters form one run [lo, hi) of the cell-sorted list (empty cells hold the
// range (0, 0)); walking it visits them in the same order as cell by cell.
__device__ __forceinline__ void row_run(const int2* __restrict__ range, int64_t row, int x0, int x1, int& lo,
                                        int& hi) {
  lo = 0x7fffffff;
  hi = 0;
  for (int xx = x0; xx <= x1; ++xx) {
    const int2 r = range[row + xx];
    if (r.y > r.x) {
      lo = min(lo, r.x);
      hi = max(hi, r.y);
    }
  }
}

// Candidates of one slave element: masters of its own and the 26 neighbouring
// cells whose boxes touch its delta-enlarged box, in walk order; the first
// vcap go to v[k * vs].  One lane per slave.
__device__ __forceinline__ int walk_cells(const SlaveBox& b, const double* __restrict__ sbox,
                                          const uint32_t* __restrict__ mvals, const int2* __restrict__ range,
                                          const Grid& g, double delta, int32_t* v, int64_t vs, int vcap) {
  int c0[3], c1[3];
  cell_window(b, g, c0, c1);
  int c = 0;
  for (int zz = c0[2]; zz <= c1[2]; ++zz) {
    for (int yy = c0[1]; yy <= c1[1]; ++yy) {
      int lo, hi;
      row_run(range, (int64_t)g.n[0] * (yy + (int64_t)g.n[1] * zz), c0[0], c1[0], lo, hi);
      for (int i = lo; i < hi; ++i) {
        if (touch(b, sbox, i, delta)) {
          if (c < vcap) v[c * vs] = (int)mvals[i];
          ++c;
        }
      }
    }
  }
  return c;
}

// Same walk by a group of G lanes of one wave (lane r of the group tests
// masters lo + r, lo + r + G, ...): the group's hits of one step are ranked
// by a wave ballot, so v receives the same candidates in the same order as
// the one-lane walk, and the boxes a group reads in one step are adjacent.
__device__ __forceinline__ int walk_cells_group(const SlaveBox& b, const double* __restrict__ sbox,
                                                const uint64_t* __restrict__ qbox,
                                                const uint32_t* __restrict__ mvals, const int2* __restrict__ range,
                                                const Grid& g, double delta, int32_t* v, int64_t vs, int vcap, int r,
                                                int gshift) {
  int c0[3], c1[3];
  cell_window(b, g, c0, c1);
  const QSlave qs = q_slave(g, b.lo, b.hi, delta);
  const unsigned below = (1u << r) - 1u;
  int c = 0;
  for (int zz = c0[2]; zz <= c1[2]; ++zz) {
    for (int yy = c0[1]; yy <= c1[1]; ++yy) {
      // the run of the row's cells: the group's lanes read alternate cells
      // and combine their bounds (the same run as row_run)
      const int64_t row = (int64_t)g.n[0] * (yy + (int64_t)g.n[1] * zz);
      int lo = 0x7fffffff, hi = 0;
      for (int xx = c0[0] + r; xx <= c1[0]; xx += G) {
        const int2 cr = range[row + xx];
        if (cr.y > cr.x) {
          lo = min(lo, cr.x);
          hi = max(hi, cr.y);
        }
      }
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        lo = min(lo, __shfl_xor(lo, d, 64));
        hi = max(hi, __shfl_xor(hi, d, 64));
      }
      for (int i0 = lo; i0 < hi; i0 += G) {
        const int i = i0 + r;
        const bool hit = i < hi && touch_q(b, qs, sbox, qbox, i, delta);
        const unsigned m = (unsigned)(__ballot(hit) >> gshift) & ((1u << G) - 1u);
        if (hit) {
          const int k = c + __popc(m & below);
          if (k < vcap) v[k * vs] = (int)mvals[i];
        }
        c += __popc(m);
      }
    }
  }
  return c;
}

// Count pass, G lanes per slave: the number of candidates, and the first
// CTMP of them (walk order) in the lane-interleaved scratch tmp[k * n_s + s].
__global__ __launch_bounds__(BS) void k_cand_count(const double* __restrict__ box_s, int32_t n_s,
                                                    const double* __restrict__ sbox,
                                                    const uint64_t* __restrict__ qbox,
                                                    const uint32_t* __restrict__ mvals,
                                                    const int2* __restrict__ range, const Grid* __restrict__ gp,
                                                    double delta, int32_t* __restrict__ count,
                                                    int32_t* __restrict__ tmp) {
  const int64_t t = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
  const int s = (int)(t / G), r = (int)(t % G);
  if (s >= n_s) return;  // whole groups leave together
  const Grid g = *gp;
  const SlaveBox b = load_box(box_s, n_s, s);
  const int c = walk_cells_group(b, sbox, qbox, mvals, range, g, delta, tmp + s, n_s, CTMP, r,
                                 (int)(__lane_id() & ~(G - 1)));
  if (r == 0) count[s] = c;
}

__device__ __forceinline__ void load_master_data(const double* __restrict__ md, int m, double X[4][3]) {
  const double2* src = reinterpret_cast<const double2*>(md + (int64_t)12 * m);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double2 t = src[k];
    X[(2 * k) / 3][(2 * k) % 3] = t.x;
    X[(2 * k + 1) / 3][(2 * k + 1) % 3] = t.y;
  }
}

// Screening of one candidate (master m of slave s, output slot ci) against
// the slave plane data: projection of the master nodes, degeneracy checks and
// the separating-line quick exit decide flag[ci] (1: to be clipped;
// otherwise the vertex count is 0).
struct SlavePlane {
  double f[12], As;
  V2 S[4];
};

__device__ __forceinline__ void load_plane(const double* __restrict__ sd, int32_t n_s, int s, SlavePlane& P) {
#pragma unroll
  for (int k = 0; k < 12; ++k) P.f[k] = sd[(int64_t)k * n_s + s];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    P.S[k].u = sd[(int64_t)(12 + k) * n_s + s];
    P.S[k].v = sd[(int64_t)(16 + k) * n_s + s];
  }
  P.As = sd[(int64_t)20 * n_s + s];
}

struct ScreenOut {
  unsigned degen_s, degen_m;
};

__device__ __forceinline__ bool screen_one(const SlavePlane& P, int s, int m, int64_t ci,
                                           const double* __restrict__ md, double eps_a, int32_t* __restrict__ cand_s,
                                           int32_t* __restrict__ cand_m, uint8_t* __restrict__ nv_out,
                                           int32_t* __restrict__ flag, ScreenOut& so) {
  double Xm[4][3];
  load_master_data(md, m, Xm);
  V2 Mn[4];
  double hm[4];
  int st;
  bool flip;
  const bool clip = pair_screen(P.S, P.As, Xm, P.f, eps_a, Mn, hm, flip, st);
  flag[ci] = clip ? 1 : 0;
  if (!clip) nv_out[ci] = 0;
  so.degen_s += (st & PS_DEGEN_SLAVE) ? 1u : 0u;
  so.degen_m += (st & PS_DEGEN_MASTER) ? 1u : 0u;
  cand_m[ci] = m;
  cand_s[ci] = s;
  return clip;
}

__device__ __forceinline__ void count_degenerate(const ScreenOut& so, Counters* cnt) {
  // degenerate elements are rare: count them with global atomics
  if (so.degen_s) atomicAdd(&cnt->degen_slave, (unsigned long long)so.degen_s);
  if (so.degen_m) atomicAdd(&cnt->degen_master, (unsigned long long)so.degen_m);
}

// Fill pass for slaves with at most CTMP candidates, G lanes per slave: lane
// r takes the candidates r, r + G, ... of the count pass's list, finds the
// place of each in the master-sorted order by counting the smaller masters
// of the list (the masters of one slave are distinct), screens it and writes
// it there.  No lane reads what another lane wrote; the group's number of
// screened-in candidates (to scr_cnt[s]) is summed by lane shuffles.
__global__ __launch_bounds__(BS) void k_cand_fill(int32_t n_s, const int32_t* __restrict__ tmp,
                                                   const int32_t* __restrict__ off, int32_t* __restrict__ cand_s,
                                                   int32_t* __restrict__ cand_m, const double* __restrict__ sd,
                                                   const double* __restrict__ md, double eps_a,
                                                   uint8_t* __restrict__ nv_out, int32_t* __restrict__ flag,
                                                   int32_t* __restrict__ scr_cnt, Counters* cnt, int64_t cap) {
  const int64_t t = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
  const int s = (int)(t / G), r = (int)(t % G);
  if (s >= n_s) return;  // whole groups leave together
  const int base = off[s];
  const int c = off[s + 1] - base;
  if (c > CTMP) return;  // k_cand_fill_long
  if (base < 0 || (int64_t)base + c > cap) {  // output too short: the host sizes it, runs the pass again
    if (r == 0) scr_cnt[s] = 0;
    return;
  }
  int nscr = 0;
  if (r < c) {
    int own[OWN], rank[OWN];
#pragma unroll
    for (int q = 0; q < OWN; ++q) {
      const int k = r + q * G;
      own[q] = k < c ? tmp[(int64_t)k * n_s + s] : 0x7fffffff;
      rank[q] = 0;
    }
    for (int k = 0; k < c; ++k) {
      const int x = tmp[(int64_t)k * n_s + s];
#pragma unroll
      for (int q = 0; q < OWN; ++q) rank[q] += x < own[q] ? 1 : 0;
    }
    SlavePlane P;
    load_plane(sd, n_s, s, P);
    ScreenOut so{0u, 0u};
    for (int q = 0; q < OWN && r + q * G < c; ++q)
      nscr += screen_one(P, s, own[q], (int64_t)base + rank[q], md, eps_a, cand_s, cand_m, nv_out, flag, so) ? 1 : 0;
    count_degenerate(so, cnt);
  }
  // all G lanes of the group are active here
#pragma unroll
  for (int d = 1; d < G; d <<= 1) nscr += __shfl_xor(nscr, d, 64);
  if (r == 0) scr_cnt[s] = nscr;
}

// Fill pass for slaves with more than CTMP candidates (rare), one lane per
// slave: the walk again, an insertion sort by master index in a
// lane-interleaved LDS segment (in place in the output when longer than
// CCAP; two call sites, so that each pointer has a known address space),
// then the screening.
__device__ __forceinline__ void fill_long(int s, int32_t n_s, int base, int c, int32_t* v, int vs,
                                          const double* __restrict__ box_s, const double* __restrict__ sbox,
                                          const uint32_t* __restrict__ mvals, const int2* __restrict__ range,
                                          const Grid& g, double delta, int32_t* __restrict__ cand_s,
                                          int32_t* __restrict__ cand_m, const double* __restrict__ sd,
                                          const double* __restrict__ md, double eps_a, uint8_t* __restrict__ nv_out,
                                          int32_t* __restrict__ flag, ScreenOut& so, int& nscr) {
  walk_cells(load_box(box_s, n_s, s), sbox, mvals, range, g, delta, v, vs, c);
  for (int i = 1; i < c; ++i) {
    const int x = v[i * vs];
    int j = i - 1;
    while (j >= 0 && v[j * vs] > x) {
      v[(j + 1) * vs] = v[j * vs];
      --j;
    }
    v[(j + 1) * vs] = x;
  }
  SlavePlane P;
  load_plane(sd, n_s, s, P);
  for (int i = 0; i < c; ++i)
    nscr += screen_one(P, s, v[i * vs], (int64_t)base + i, md, eps_a, cand_s, cand_m, nv_out, flag, so) ? 1 : 0;
}

__global__ __launch_bounds__(BS) void k_cand_fill_long(const double* __restrict__ box_s, int32_t n_s,
                                                        const double* __restrict__ sbox,
                                                        const uint32_t* __restrict__ mvals,
                                                        const int2* __restrict__ range, const Grid* __restrict__ gp,
                                                        double delta,
                                                        const int32_t* __restrict__ off, int32_t* __restrict__ cand_s,
                                                        int32_t* __restrict__ cand_m, const double* __restrict__ sd,
                                                        const double* __restrict__ md, double eps_a,
                                                        uint8_t* __restrict__ nv_out, int32_t* __restrict__ flag,
                                                        int32_t* __restrict__ scr_cnt, Counters* cnt,
                                                        int64_t cap) {
  __shared__ int32_t lds[CCAP * BS];
  const int s = xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
  if (s >= n_s) return;
  const int base = off[s];
  const int c = off[s + 1] - base;
  if (c <= CTMP) return;
  if (base < 0 || (int64_t)base + c > cap) {
    scr_cnt[s] = 0;
    return;
  }
  const Grid g = *gp;
  ScreenOut so{0u, 0u};
  int nscr = 0;
  if (c <= CCAP)
    fill_long(s, n_s, base, c, lds + threadIdx.x, BS, box_s, sbox, mvals, range, g, delta, cand_s, cand_m, sd,
              md, eps_a, nv_out, flag, so, nscr);
  else
    fill_long(s, n_s, base, c, cand_m + base, 1, box_s, sbox, mvals, range, g, delta, cand_s, cand_m, sd, md,
              eps_a, nv_out, flag, so, nscr);
  count_degenerate(so, cnt);
  scr_cnt[s] = nscr;
}

}  // namespace

int prep_blocks(int32_t n_el) { return n_el == 0 ? 0 : std::min(2048, (n_el + BS - 1) / BS); }

hipError_t launch_prep(const DeviceMesh& S, const DeviceMesh& M, double* box_s, double* sd, double* box_m,
                       double* md, double* part, hipStream_t s) {
  const int nb_s = prep_blocks(S.n_el), nb_m = prep_blocks(M.n_el);
  if (nb_s == 0 && nb_m == 0) return hipSuccess;
  const PrepSide ps{S.x, S.y, S.z, S.conn, S.nrm, box_s, sd, nullptr, part, S.n_el, S.n_nodes, nb_s};
  const PrepSide pm{M.x, M.y, M.z, M.conn, nullptr, box_m, nullptr, md, part + (size_t)PREP_PART * nb_s,
                    M.n_el, M.n_nodes, nb_m};
  k_prep<<<dim3((unsigned)std::max(nb_s, nb_m), 2), BS, 0, s>>>(ps, pm);
  return hipGetLastError();
}

hipError_t launch_prep_reduce(const double* part, int nb_s, int nb_m, PrepReduce* red, double delta,
                              double bin_size, int64_t max_cells, DevState* st, hipStream_t s) {
  k_prep_reduce<<<1, BS, 0, s>>>(part, nb_s, nb_m, red, delta, bin_size, max_cells, st);
  return hipGetLastError();
}

hipError_t launch_master_keys(const double* box_m, int32_t n_m, const Grid* g, int64_t max_cells, uint32_t* keys,
                              uint32_t* vals, int2* range, hipStream_t s) {
  const int64_t nb = std::max<int64_t>((n_m + BS - 1) / BS, std::min<int64_t>(2048, (max_cells + BS - 1) / BS));
  k_master_keys<<<(unsigned)std::max<int64_t>(nb, 1), BS, 0, s>>>(box_m, n_m, g, keys, vals, range);
  return hipGetLastError();
}

hipError_t launch_cell_ranges(const uint32_t* keys, const uint32_t* vals, int32_t n, const double* box_m,
                              const Grid* g, int2* range, double* sbox, uint64_t* qbox, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_cell_ranges<<<(n + BS - 1) / BS, BS, 0, s>>>(keys, vals, n, box_m, g, range, sbox, qbox);
  return hipGetLastError();
}

// Grids of the candidate passes: XCD-aware (each XCD's L2 serves a
// contiguous eighth of the slave elements, whose masters are neighbours).
unsigned group_blocks(int32_t n_s) { return xcd_grid((unsigned)(((int64_t)n_s * G + BS - 1) / BS)); }

hipError_t launch_cand_count(const double* box_s, int32_t n_s, const double* sbox, const uint64_t* qbox,
                             const uint32_t* mvals,
                             const int2* range, const Grid* g, double delta, int32_t* count, int32_t* tmp,
                             hipStream_t s) {
  if (n_s == 0) return hipSuccess;
  k_cand_count<<<group_blocks(n_s), BS, 0, s>>>(box_s, n_s, sbox, qbox, mvals, range, g, delta, count, tmp);
  return hipGetLastError();
}

hipError_t launch_cand_fill(const double* box_s, int32_t n_s, const double* sbox, const uint32_t* mvals,
                            const int2* range, const Grid* g, double delta, const int32_t* tmp, const int32_t* off,
                            int32_t* cand_s, int32_t* cand_m, const double* sd, const double* md, double eps_a,
                            uint8_t* nv, int32_t* flag, int32_t* scr_cnt, Counters* cnt, int64_t cap,
                            hipStream_t s) {
  if (n_s == 0) return hipSuccess;
  k_cand_fill<<<group_blocks(n_s), BS, 0, s>>>(n_s, tmp, off, cand_s, cand_m, sd, md, eps_a, nv, flag, scr_cnt, cnt,
                                               cap);
  k_cand_fill_long<<<xcd_grid((unsigned)((n_s + BS - 1) / BS)), BS, 0, s>>>(box_s, n_s, sbox, mvals, range, g, delta,
                                                                            off, cand_s, cand_m, sd, md, eps_a, nv,
                                                                            flag, scr_cnt, cnt, cap);
  return hipGetLastError();
}

int cand_tmp_per_slave() { return CTMP; }

}  // namespace mt
