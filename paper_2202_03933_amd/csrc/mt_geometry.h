// Device-side geometry of one slave/master element pair: auxiliary plane,
// projection, Sutherland-Hodgman clipping with cleanup, triangle rules and
// the inverse bilinear map.
//
// Every expression that decides topology (which candidates are pairs, how
// many vertices a clip polygon has) is written in one fixed evaluation order
// and compiled without fused multiply-add (-ffp-contract=off), so the clip
// polygons are bitwise identical to any implementation evaluating the same
// expressions under IEEE-754 double arithmetic.  Integration code opts back
// into contraction locally.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mt {

// Working capacities of the two clip buffers (vertices): buffer 0 holds the
// slave polygon and the outputs of clip stages 2 and 4, buffer 1 the outputs
// of stages 1 and 3.  A convex quad clipped by k half planes has at most
// 4 + k vertices; two vertices of headroom absorb near-duplicates from
// rounding.  A stage exceeding its buffer marks the candidate degenerate.
constexpr int CAP0 = 10;
constexpr int CAP1 = 9;
constexpr int CAPT = CAP0 + CAP1;  // LDS vertex slots per lane

struct V2 {
  double u, v;
};

// ---- node / element access -------------------------------------------------

struct MeshPtrs {
  const double* x;
  const double* y;
  const double* z;
  const int32_t* conn;
  // slave side with the continuous normal field: per element the unit plane
  // normal and the length it was normalised from, nrm[4 e + 0..3]; else null
  const double* nrm;
};

// Blocks of a grid are dispatched round-robin over the 8 XCDs of an MI355X;
// remap block b to tile (b % 8) * ceil(nb / 8) + b / 8 so that each XCD works
// on one contiguous range of tiles (and its L2 holds one region of the mesh).
// The grid must have xcd_grid(n_tiles) = 8 * ceil(n_tiles / 8) blocks: the
// mapping is a bijection of [0, 8 * per) onto itself, and tiles at or past
// n_tiles are skipped by the caller's bounds check.
__host__ __device__ __forceinline__ unsigned xcd_grid(unsigned n_tiles) { return (n_tiles + 7) / 8 * 8; }
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned grid) {
  const unsigned per = grid / 8;
  return (b % 8) * per + b / 8;
}

// Launches over a count the device holds (the grid sized for a capacity):
// block b takes tile xcd_tile(b, g) of the g = xcd_grid(tiles of n) blocks a
// launch over exactly n items would have; blocks past g have no tile (-1).
__device__ __forceinline__ int64_t dyn_tile(unsigned b, int64_t n, int bs) {
  const unsigned g = xcd_grid((unsigned)((n + bs - 1) / bs));
  return b < g ? (int64_t)xcd_tile(b, g) : int64_t(-1);
}

__device__ __forceinline__ int4 load_conn(const int32_t* conn, int e) {
  return reinterpret_cast<const int4*>(conn)[e];
}

__device__ __forceinline__ void load_nodes(const double* __restrict__ x, const double* __restrict__ y,
                                           const double* __restrict__ z, int4 c, double X[4][3]) {
  const int id[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    X[k][0] = x[id[k]];
    X[k][1] = y[id[k]];
    X[k][2] = z[id[k]];
  }
}

// ---- auxiliary plane of a slave element (Fig. 1: centre x0, normal n0) -----

// f[0..2] = x0, f[3..5] = n0, f[6..8] = t1, f[9..11] = t2.
__device__ __forceinline__ void slave_frame(const double X[4][3], double f[12]) {
  double g1[3], g2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    f[d] = 0.25 * (((X[0][d] + X[1][d]) + X[2][d]) + X[3][d]);
    g1[d] = 0.25 * (((X[1][d] - X[0][d]) + X[2][d]) - X[3][d]);
    g2[d] = 0.25 * (((X[2][d] + X[3][d]) - X[0][d]) - X[1][d]);
  }
  const double n0 = g1[1] * g2[2] - g1[2] * g2[1];
  const double n1 = g1[2] * g2[0] - g1[0] * g2[2];
  const double n2 = g1[0] * g2[1] - g1[1] * g2[0];
  const double ln = sqrt((n0 * n0 + n1 * n1) + n2 * n2);
  const double lg = sqrt((g1[0] * g1[0] + g1[1] * g1[1]) + g1[2] * g1[2]);
  f[3] = n0 / ln;
  f[4] = n1 / ln;
  f[5] = n2 / ln;
  f[6] = g1[0] / lg;
  f[7] = g1[1] / lg;
  f[8] = g1[2] / lg;
  f[9] = f[4] * f[8] - f[5] * f[7];
  f[10] = f[5] * f[6] - f[3] * f[8];
  f[11] = f[3] * f[7] - f[4] * f[6];
}

// Frame with a given unit plane normal n (the continuous normal field at the
// element centre): centre x0, n0 = n, t1 = the part of g1 orthogonal to n,
// normalised, t2 = n0 x t1.
__device__ __forceinline__ void slave_frame_n(const double X[4][3], const double n[3], double f[12]) {
  double g1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    f[d] = 0.25 * (((X[0][d] + X[1][d]) + X[2][d]) + X[3][d]);
    g1[d] = 0.25 * (((X[1][d] - X[0][d]) + X[2][d]) - X[3][d]);
    f[3 + d] = n[d];
  }
  const double gn = (g1[0] * n[0] + g1[1] * n[1]) + g1[2] * n[2];
  double w[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) w[d] = g1[d] - gn * n[d];
  const double lw = sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
  f[6] = w[0] / lw;
  f[7] = w[1] / lw;
  f[8] = w[2] / lw;
  f[9] = f[4] * f[8] - f[5] * f[7];
  f[10] = f[5] * f[6] - f[3] * f[8];
  f[11] = f[3] * f[7] - f[4] * f[6];
}

// Frame of a slave element: from the continuous normal field when nrm (the
// element's entry of MeshPtrs::nrm) is given, else from its own geometry.
__device__ __forceinline__ void slave_frame_p(const double X[4][3], const double* nrm, double f[12]) {
  if (nrm) {
    const double n[3] = {nrm[0], nrm[1], nrm[2]};
    slave_frame_n(X, n, f);
  } else {
    slave_frame(X, f);
  }
}

__device__ __forceinline__ const double* elem_nrm(const MeshPtrs& S, int s) {
  return S.nrm ? S.nrm + 4 * (int64_t)s : nullptr;
}

// In-plane coordinates and height of one node.
__device__ __forceinline__ void project(const double X[3], const double f[12], V2& p, double& h) {
  const double d0 = X[0] - f[0], d1 = X[1] - f[1], d2 = X[2] - f[2];
  p.u = (d0 * f[6] + d1 * f[7]) + d2 * f[8];
  p.v = (d0 * f[9] + d1 * f[10]) + d2 * f[11];
  h = (d0 * f[3] + d1 * f[4]) + d2 * f[5];
}

__device__ __forceinline__ double quad_fan_area(const V2 p[4]) {
  double a = 0.0;
#pragma unroll
  for (int i = 1; i < 3; ++i)
    a = a + ((p[i].u - p[0].u) * (p[i + 1].v - p[0].v) - (p[i].v - p[0].v) * (p[i + 1].u - p[0].u));
  return 0.5 * a;
}

__device__ __forceinline__ double linf(double du, double dv) { return fmax(fabs(du), fabs(dv)); }

// ---- per-lane polygon storage in LDS ---------------------------------------
// Two ping-pong buffers (CAP0 + CAP1 vertices) per lane, lane-interleaved so that a
// wavefront touching vertex i of its polygons hits consecutive addresses.
// With labels, each vertex also carries its provenance (slave node k:
// 0x80|k, else the two lines it lies on, (la << 4) | lb, line ids 0..3 =
// slave edges k -> k+1, 4..7 = master clip edges) and the line id of the
// edge leaving it.
template <bool LAB>
struct LdsPoly {
  double* u;
  double* v;
  uint8_t* vl;
  uint8_t* el;
  int bs;
  __device__ __forceinline__ int at(int b, int i) const { return ((b ? CAP0 : 0) + i) * bs; }
};

// Clip the slave polygon S (counter-clockwise) by the master polygon Mo
// (counter-clockwise) with Sutherland-Hodgman: per master edge a -> b keep
// the closed left half plane, walking subject edges P -> E from vertex 0,
// emitting P when inside and then the crossing when the sides differ.
// Returns the vertex count; the polygon is in buffer `res`.  Sets *ovf on
// capacity overflow (then returns 0).
//
// The first stage reads the slave polygon from registers and writes buffer
// 1; the later stages alternate between the LDS buffers, each first reading
// its whole input polygon into registers (one round trip of independent LDS
// reads instead of one per edge).

// Side value of point (u, v) for the line a -> b (>= 0: inside).
__device__ __forceinline__ double side_of(V2 a, double dbu, double dbv, double u, double v) {
  return dbu * (v - a.v) - dbv * (u - a.u);
}

template <bool LAB>
__device__ __forceinline__ void emit_vertex(const LdsPoly<LAB>& P, int b, int k, double u, double v, uint8_t vl,
                                            uint8_t el) {
  P.u[P.at(b, k)] = u;
  P.v[P.at(b, k)] = v;
  if (LAB) {
    P.vl[P.at(b, k)] = vl;
    P.el[P.at(b, k)] = el;
  }
}

template <bool LAB>
__device__ __forceinline__ int clip_polygon(const V2 S[4], const V2 Mo[4], const LdsPoly<LAB>& P, int& res,
                                            bool& ovf) {
  ovf = false;
  int n;
  // stage 1: slave polygon (registers) against master edge 0, into buffer 1
  {
    const V2 a = Mo[0], b = Mo[1];
    const double dbu = b.u - a.u, dbv = b.v - a.v;
    double c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = side_of(a, dbu, dbv, S[k].u, S[k].v);
    int k = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = (j + 1) & 3;
      const bool pin = c[j] >= 0.0, ein = c[e] >= 0.0;
      if (pin) {
        emit_vertex<LAB>(P, 1, k, S[j].u, S[j].v, (uint8_t)(0x80 | j), (uint8_t)j);
        ++k;
      }
      if (pin != ein) {
        const double t = c[j] / (c[j] - c[e]);
        emit_vertex<LAB>(P, 1, k, S[j].u + t * (S[e].u - S[j].u), S[j].v + t * (S[e].v - S[j].v),
                         (uint8_t)((j << 4) | 4), pin ? (uint8_t)4 : (uint8_t)j);
        ++k;
      }
    }
    n = k;
  }
  int cur = 1;
  constexpr int CIN = CAP0 > CAP1 ? CAP0 : CAP1;  // a stage's input fits its buffer
#pragma unroll
  for (int l = 1; l < 4; ++l) {
    if (n == 0) break;
    const V2 a = Mo[l];
    const V2 b = Mo[(l + 1) & 3];
    const double dbu = b.u - a.u, dbv = b.v - a.v;
    const int nxt = cur ^ 1;
    const int cap = nxt ? CAP1 : CAP0;
    // the stage's whole input polygon to registers first (independent LDS
    // reads, one round trip), then the walk with static register indices
    double qu[CIN], qv[CIN], qc[CIN];
    uint8_t ql[CIN], qe[CIN];
#pragma unroll
    for (int i = 0; i < CIN; ++i) {
      qu[i] = 0.0;
      qv[i] = 0.0;
      ql[i] = 0;
      qe[i] = 0;
      if (i < n) {
        qu[i] = P.u[P.at(cur, i)];
        qv[i] = P.v[P.at(cur, i)];
        if (LAB) { ql[i] = P.vl[P.at(cur, i)]; qe[i] = P.el[P.at(cur, i)]; }
      }
    }
#pragma unroll
    for (int i = 0; i < CIN; ++i) qc[i] = side_of(a, dbu, dbv, qu[i], qv[i]);
    int k = 0;
#pragma unroll
    for (int j = 0; j < CIN; ++j) {
      if (j < n) {
        // edge from vertex j to the next one (vertex 0 after the last)
        const int jn = j + 1 < CIN ? j + 1 : 0;
        const bool wrap = j + 1 == n;
        const double Eu = wrap ? qu[0] : qu[jn], Ev = wrap ? qv[0] : qv[jn];
        const double cP = qc[j], cE = wrap ? qc[0] : qc[jn];
        const bool pin = cP >= 0.0;
        const bool ein = cE >= 0.0;
        if (pin) {
          if (k == cap) { ovf = true; return 0; }
          emit_vertex<LAB>(P, nxt, k, qu[j], qv[j], ql[j], qe[j]);
          ++k;
        }
        if (pin != ein) {
          if (k == cap) { ovf = true; return 0; }
          const double t = cP / (cP - cE);
          emit_vertex<LAB>(P, nxt, k, qu[j] + t * (Eu - qu[j]), qv[j] + t * (Ev - qv[j]),
                           (uint8_t)((qe[j] << 4) | (4 + l)), pin ? (uint8_t)(4 + l) : qe[j]);
          ++k;
        }
      }
    }
    n = k;
    cur = nxt;
  }
  res = cur;
  return n;
}

template <bool LAB>
__device__ __forceinline__ void poly_move(const LdsPoly<LAB>& P, int b, int dst, int src) {
  P.u[P.at(b, dst)] = P.u[P.at(b, src)];
  P.v[P.at(b, dst)] = P.v[P.at(b, src)];
  if (LAB) {
    P.vl[P.at(b, dst)] = P.vl[P.at(b, src)];
    P.el[P.at(b, dst)] = P.el[P.at(b, src)];
  }
}

// Cleanup of a raw clip polygon in buffer b: (i) one pass dropping vertices
// within tol (max-norm) of the previously kept one, vertex 0 always kept and
// the last kept one dropped if within tol of vertex 0; (ii) repeated sweeps in
// index order removing any vertex with |cross(next-prev, v-prev)| <=
// tol * maxnorm(next-prev), until a sweep removes nothing or n < 3.
template <bool LAB>
__device__ __forceinline__ int cleanup(const LdsPoly<LAB>& P, int b, int n, double tol) {
  if (n == 0) return 0;
  int m = 1;
  double lu = P.u[P.at(b, 0)], lv = P.v[P.at(b, 0)];
  for (int i = 1; i < n; ++i) {
    const double cu = P.u[P.at(b, i)], cv = P.v[P.at(b, i)];
    if (linf(cu - lu, cv - lv) > tol) {
      if (m != i) poly_move(P, b, m, i);
      ++m;
      lu = cu;
      lv = cv;
    }
  }
  if (m > 1 && linf(lu - P.u[P.at(b, 0)], lv - P.v[P.at(b, 0)]) <= tol) --m;
  n = m;
  bool changed = true;
  while (changed && n >= 3) {
    changed = false;
    int i = 0;
    while (i < n && n >= 3) {
      const int ia = (i + n - 1) % n, ib = (i + 1) % n;
      const double au = P.u[P.at(b, ia)], av = P.v[P.at(b, ia)];
      const double bu = P.u[P.at(b, ib)] - au, bv = P.v[P.at(b, ib)] - av;
      const double cr = bu * (P.v[P.at(b, i)] - av) - bv * (P.u[P.at(b, i)] - au);
      if (fabs(cr) <= tol * linf(bu, bv)) {
        for (int j = i; j + 1 < n; ++j) poly_move(P, b, j, j + 1);
        --n;
        changed = true;
      } else {
        ++i;
      }
    }
  }
  return n;
}

template <bool LAB>
__device__ __forceinline__ double poly_fan_area(const LdsPoly<LAB>& P, int b, int n) {
  const double u0 = P.u[P.at(b, 0)], v0 = P.v[P.at(b, 0)];
  double a = 0.0;
  for (int i = 1; i + 1 < n; ++i) {
    const double u1 = P.u[P.at(b, i)], v1 = P.v[P.at(b, i)];
    const double u2 = P.u[P.at(b, i + 1)], v2 = P.v[P.at(b, i + 1)];
    a = a + ((u1 - u0) * (v2 - v0) - (v1 - v0) * (u2 - u0));
  }
  return 0.5 * a;
}

// Status bits of one pair evaluation.
enum : int { PS_DEGEN_SLAVE = 1, PS_DEGEN_MASTER = 2, PS_OVERFLOW = 4, PS_LOST = 8 };

// Projection, orientation, clip and cleanup of one candidate.  On return:
// S, Mn = projected slave / master nodes (node order), hs, hm = heights,
// Mo = master polygon walked counter-clockwise (flip: Mo = (M0, M3, M2, M1),
// i.e. Mo[l] = Mn[(4 - l) % 4]; otherwise Mo = Mn),
// polygon in buffer `res` with `n` vertices (0: not a pair).
// Slave-only part of the pair geometry: projected slave nodes, their area and
// the longest projected edge (max-norm), from the slave frame f.
__device__ __forceinline__ void slave_setup(const double Xs[4][3], const double f[12], V2 S[4], double hs[4],
                                            double& As, double& hmax) {
#pragma unroll
  for (int k = 0; k < 4; ++k) project(Xs[k], f, S[k], hs[k]);
  As = quad_fan_area(S);
  hmax = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = (k + 1) & 3;
    hmax = fmax(hmax, linf(S[e].u - S[k].u, S[e].v - S[k].v));
  }
}

// Screening part of the master side: projection of the master nodes onto
// the slave plane, degeneracy checks, orientation and the separating-line
// quick exit.  Returns true when the candidate has to be clipped.
__device__ __forceinline__ bool pair_screen(const V2 S[4], double As, const double Xm[4][3], const double f[12],
                                            double eps_a, V2 Mn[4], double hm[4], bool& flip, int& status) {
  status = 0;
  flip = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) project(Xm[k], f, Mn[k], hm[k]);
  if (!(As > 0.0)) { status = PS_DEGEN_SLAVE; return false; }
  const double tol_a = eps_a * As;
  const double Am = quad_fan_area(Mn);
  if (fabs(Am) <= tol_a) { status = PS_DEGEN_MASTER; return false; }
  flip = Am < 0.0;
  const V2 Mo[4] = {Mn[0], flip ? Mn[3] : Mn[1], Mn[2], flip ? Mn[1] : Mn[3]};
  // Separating-line quick exit (exact): every slave vertex strictly outside
  // one master edge line, or every master vertex strictly outside one slave
  // edge line, means no overlap.  Same side test as the clip.
#pragma unroll
  for (int side = 0; side < 2; ++side) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const V2 a = side == 0 ? Mo[l] : S[l];
      const V2 b = side == 0 ? Mo[(l + 1) & 3] : S[(l + 1) & 3];
      const double dbu = b.u - a.u, dbv = b.v - a.v;
      bool all_out = true;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const V2 q = side == 0 ? S[k] : Mo[k];
        const double c = dbu * (q.v - a.v) - dbv * (q.u - a.u);
        all_out = all_out && !(c >= 0.0);
      }
      if (all_out) return false;
    }
  }
  return true;
}

// Clip and cleanup of a screened candidate; the polygon ends in buffer
// `res` with the returned vertex count (0: not a pair).
template <bool LAB>
__device__ __forceinline__ int pair_clip_screened(const V2 S[4], double As, double hmax, const V2 Mn[4], bool flip,
                                                  double eps_d, double eps_a, const LdsPoly<LAB>& P, int& res,
                                                  int& status) {
  const V2 Mo[4] = {Mn[0], flip ? Mn[3] : Mn[1], Mn[2], flip ? Mn[1] : Mn[3]};
  bool ovf;
  res = 0;
  int n = clip_polygon<LAB>(S, Mo, P, res, ovf);
  if (ovf) { status = PS_OVERFLOW; return 0; }
  n = cleanup<LAB>(P, res, n, eps_d * hmax);
  if (n < 3) return 0;
  const double Ap = poly_fan_area<LAB>(P, res, n);
  if (!(Ap > eps_a * As)) return 0;
  return n;
}

// Master part: projection of the master nodes onto the slave plane,
// orientation, clip and cleanup, given the slave setup.
template <bool LAB>
__device__ __forceinline__ int pair_clip(const V2 S[4], double As, double hmax, const double Xm[4][3],
                                         const double f[12], double eps_d, double eps_a, V2 Mn[4], double hm[4],
                                         bool& flip, const LdsPoly<LAB>& P, int& res, int& status) {
  res = 0;
  if (!pair_screen(S, As, Xm, f, eps_a, Mn, hm, flip, status)) return 0;
  return pair_clip_screened<LAB>(S, As, hmax, Mn, flip, eps_d, eps_a, P, res, status);
}

template <bool LAB>
__device__ __forceinline__ int pair_geometry(const double Xs[4][3], const double Xm[4][3], const double f[12],
                                             double eps_d, double eps_a, V2 S[4], V2 Mn[4], double hs[4],
                                             double hm[4], bool& flip, const LdsPoly<LAB>& P, int& res,
                                             int& status) {
  double As, hmax;
  slave_setup(Xs, f, S, hs, As, hmax);
  return pair_clip<LAB>(S, As, hmax, Xm, f, eps_d, eps_a, Mn, hm, flip, P, res, status);
}

// Precomputed slave data for the candidate pass, structure-of-arrays
// sd[k * n + e]: frame (12), projected nodes u (4), v (4), area, max edge.
constexpr int SD_N = 22;

// ---- quadrature ------------------------------------------------------------

// Bilinear shape functions, nodes at (-1,-1), (1,-1), (1,1), (-1,1).
__device__ __forceinline__ void shape4(double x1, double x2, double N[4]) {
#pragma clang fp contract(fast)
  const double a0 = 1.0 - x1, a1 = 1.0 + x1, b0 = 1.0 - x2, b1 = 1.0 + x2;
  N[0] = 0.25 * a0 * b0;
  N[1] = 0.25 * a1 * b0;
  N[2] = 0.25 * a1 * b1;
  N[3] = 0.25 * a0 * b1;
}

// Inverse of the bilinear map xi -> sum_k N_k(xi) X_k by Newton's method
// from xi = 0; stops when max |dxi| <= tol.  Returns false when it did not
// converge in maxit iterations.  The map is written as
// x(xi) = c + e1 xi1 + e2 xi2 + e12 xi1 xi2.
__device__ __forceinline__ bool inverse_bilinear(const V2 X[4], double pu, double pv, double tol, int maxit,
                                                 double& x1, double& x2) {
#pragma clang fp contract(fast)
  const double cu = 0.25 * ((X[0].u + X[1].u) + (X[2].u + X[3].u));
  const double cv = 0.25 * ((X[0].v + X[1].v) + (X[2].v + X[3].v));
  const double e1u = 0.25 * ((X[1].u - X[0].u) + (X[2].u - X[3].u));
  const double e1v = 0.25 * ((X[1].v - X[0].v) + (X[2].v - X[3].v));
  const double e2u = 0.25 * ((X[2].u - X[1].u) + (X[3].u - X[0].u));
  const double e2v = 0.25 * ((X[2].v - X[1].v) + (X[3].v - X[0].v));
  const double fu = 0.25 * ((X[0].u - X[1].u) + (X[2].u - X[3].u));
  const double fv = 0.25 * ((X[0].v - X[1].v) + (X[2].v - X[3].v));
  x1 = 0.0;
  x2 = 0.0;
  const double ru0 = cu - pu, rv0 = cv - pv;
  for (int it = 0; it < maxit; ++it) {
    const double ru = ru0 + e1u * x1 + e2u * x2 + fu * x1 * x2;
    const double rv = rv0 + e1v * x1 + e2v * x2 + fv * x1 * x2;
    const double j00 = e1u + fu * x2, j01 = e2u + fu * x1;
    const double j10 = e1v + fv * x2, j11 = e2v + fv * x1;
    const double rdet = 1.0 / (j00 * j11 - j01 * j10);
    const double s1 = (j11 * ru - j01 * rv) * rdet;
    const double s2 = (j00 * rv - j10 * ru) * rdet;
    x1 -= s1;
    x2 -= s2;
    if (fmax(fabs(s1), fabs(s2)) <= tol) return true;
  }
  return false;
}

// Dual basis coefficients A = De Me^-1 of one slave element from its
// projected nodes (2x2 Gauss; De = diag int N_j, Me = int N N^T).
__device__ __forceinline__ void dual_coefficients(const V2 S[4], double A[16]) {
#pragma clang fp contract(fast)
  const double g = 0.5773502691896257;
  double Me[16], De[4];
#pragma unroll
  for (int i = 0; i < 16; ++i) Me[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) De[i] = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const double x1 = a ? g : -g, x2 = b ? g : -g;
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
  // Gauss-Jordan inverse of Me (symmetric positive definite: no pivoting).
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
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int k = 0; k < 4; ++k) A[j * 4 + k] = De[j] * inv[j * 4 + k];
}

}  // namespace mt
