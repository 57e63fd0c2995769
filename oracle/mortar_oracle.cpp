// Plain serial CPU oracle for segment-based mortar coupling (FP64).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg load this library.  It shares no code with
// the HIP path and is deliberately slow and literal.
//
// What it computes (Mayr & Popp, "Scalable computational kernels for mortar
// finite element methods"):
//  * contact search: every (slave, master) element pair whose axis-aligned
//    bounding boxes overlap once the slave box is enlarged by delta; by brute
//    force over all pairs, and by Cartesian binning (Sec. "Distributed
//    storage: going to large problems", Alg. 2 and the bin sizing rule above
//    it).
//  * per pair, the steps of Alg. 1 (Sec. "Evaluation of mortar integrals"):
//    project both elements onto the auxiliary plane of the slave element
//    (centre x0, normal n0; Fig. 1 and the piecewise-flat integration the
//    same section describes), clip the slave polygon against the master
//    polygon (Sutherland-Hodgman), split the clip polygon into a triangle fan
//    (Fig. 1), and integrate the nodal blocks of D and M of
//    eq. (DiscreteWeakFormInterfaceFlux) and a weighted gap with a triangle
//    Gauss rule.
//  * standard or dual (biorthogonal) Lagrange multiplier basis (same section,
//    after eq. (AnsatzDiscretizationLagrangeMult)).
//  * element-based integration, the alternative to the segments of Alg. 1
//    that the same section names (a Gauss product rule on the whole slave
//    element, each point assigned to the master it projects into).
//  * exact derivatives by forward-mode dual numbers over the 24 nodal
//    coordinates of a pair (the linearisation the paper requires in every
//    nonlinear iteration, Sec. "Introduction" after Fig. 1).
//
// Readings where the paper is silent (projection plane, clip loop variant and
// start vertex, boundary test, cleanup tolerances, triangulation, rule,
// weighted-gap definition) are listed at each function.
//
// Fixed evaluation order.  Topology (which candidates become pairs and how
// many vertices a clip polygon has) hinges on exact comparisons.  All
// expressions that feed those comparisons are written with explicit
// parenthesisation and built without fused multiply-add, so any other
// implementation evaluating the same expressions in the same order under
// IEEE-754 double arithmetic reproduces the vertex counts bit for bit.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ----------------------------------------------------------------- scalars

inline double val(double x) { return x; }

template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT
};
template <int N> inline double val(const Dual<N>& a) { return a.v; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.v * b.d[i] + b.v * a.d[i]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r; }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) {
  Dual<N> r; r.v = a * b.v; for (int i = 0; i < N; ++i) r.d[i] = a * b.d[i]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) { return b * a; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r; r.v = std::sqrt(a.v);
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
  return r; }
template <int N> inline Dual<N> fabs(const Dual<N>& a) { return a.v < 0 ? -a : a; }

// Flop-counting scalar: one count per add, subtract, multiply, divide and
// square root executed by the algorithm.  Comparisons, abs, min and max are
// not counted.  Operations outside the inverse bilinear maps are also tallied
// by kind, for the reverse-mode cost model of or_count_flops.
thread_local uint64_t g_flops = 0;
thread_local uint64_t g_kind[4] = {0, 0, 0, 0};  // add/sub, mul, div, sqrt outside inverse maps
thread_local bool g_in_inverse_map = false;
thread_local uint64_t g_inverse_maps = 0;
inline void count_op(int kind) {
  ++g_flops;
  if (!g_in_inverse_map) ++g_kind[kind];
}
struct Cnt { double v; Cnt() : v(0.0) {} Cnt(double x) : v(x) {} };  // NOLINT
inline double val(const Cnt& a) { return a.v; }
inline Cnt operator+(Cnt a, Cnt b) { count_op(0); return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { count_op(0); return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { count_op(1); return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { count_op(2); return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator+(double a, Cnt b) { return Cnt(a) + b; }
inline Cnt operator+(Cnt a, double b) { return a + Cnt(b); }
inline Cnt operator-(double a, Cnt b) { return Cnt(a) - b; }
inline Cnt operator-(Cnt a, double b) { return a - Cnt(b); }
inline Cnt operator*(double a, Cnt b) { return Cnt(a) * b; }
inline Cnt operator*(Cnt a, double b) { return a * Cnt(b); }
inline Cnt operator/(Cnt a, double b) { return a / Cnt(b); }
inline Cnt sqrt(Cnt a) { count_op(3); return Cnt(std::sqrt(a.v)); }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }

using std::fabs;
using std::sqrt;

// ------------------------------------------------------------- parameters

struct Params {
  double delta;       // slave bounding-box enlargement of the search
  int dual;           // 0: standard LM basis (Phi = N); 1: dual basis
  int rule;           // triangle rule: 3 (degree 2) or 7 (degree 5)
  double eps_d;       // relative vertex-merge / collinearity tolerance
  double eps_a;       // relative area tolerance
  double newton_tol;  // inverse bilinear map: stop when max |d xi| <= tol
  int newton_maxit;   // ... or fail after this many iterations
  int normals;        // auxiliary-plane normal: 0 element (g1 x g2), 1 averaged nodal normals
};

enum {
  ST_NOCONV = 1,        // inverse bilinear map did not converge
  ST_OVERFLOW = 2,      // unused here (clip polygons grow); reserved for the status layout
  ST_DEGEN_SLAVE = 4,   // projected slave polygon has non-positive area
  ST_DEGEN_MASTER = 8,  // projected master polygon has (near) zero area
};

// Clip polygons are growable: Alg. 1 clips with plain Sutherland-Hodgman
// and neither it nor Fig. 1 sets a vertex limit, so no stage can overflow
// here.  OR_MAX_VERTICES only sizes the output buffers of the test entry
// points below (a cleaned clip of two quads has at most 8 vertices).
constexpr int OR_MAX_VERTICES = 64;

template <class T> struct P2 { T u, v; };
template <class T> using Poly = std::vector<P2<T>>;

// ------------------------------------------------------- shape functions

// Bilinear quad4 shape functions; node k sits at (A[k], B[k]).
constexpr double NA[4] = {-1.0, 1.0, 1.0, -1.0};
constexpr double NB[4] = {-1.0, -1.0, 1.0, 1.0};

template <class T>
void shape(const T& x1, const T& x2, T N[4], T d1[4], T d2[4]) {
  for (int k = 0; k < 4; ++k) {
    T a = 1.0 + NA[k] * x1;
    T b = 1.0 + NB[k] * x2;
    N[k] = 0.25 * (a * b);
    d1[k] = (0.25 * NA[k]) * b;
    d2[k] = (0.25 * NB[k]) * a;
  }
}

// ---------------------------------------------------- slave element frame

// Auxiliary plane of a slave element: centre x0 (parameter origin), unit
// normal n0 at the centre, and an orthonormal in-plane basis (t1, t2) with
// t1 along the first covariant base vector.  Fig. 1 projects along n0 at x0.
// n0 is the element normal g1 x g2 / |g1 x g2| at the centre, or, when nin is
// given, that unit vector (the continuous normal field of the slave side at
// the element centre, see element_normals); t1 is then the part of g1
// orthogonal to n0, normalised.
template <class T>
void slave_frame(const T X[4][3], const T* nin, T x0[3], T n0[3], T t1[3], T t2[3]) {
  T g1[3], g2[3];
  for (int d = 0; d < 3; ++d) {
    x0[d] = 0.25 * (((X[0][d] + X[1][d]) + X[2][d]) + X[3][d]);
    g1[d] = 0.25 * (((X[1][d] - X[0][d]) + X[2][d]) - X[3][d]);
    g2[d] = 0.25 * (((X[2][d] + X[3][d]) - X[0][d]) - X[1][d]);
  }
  if (nin) {
    for (int d = 0; d < 3; ++d) n0[d] = nin[d];
    const T gn = (g1[0] * n0[0] + g1[1] * n0[1]) + g1[2] * n0[2];
    T w[3];
    for (int d = 0; d < 3; ++d) w[d] = g1[d] - gn * n0[d];
    const T lw = sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
    for (int d = 0; d < 3; ++d) t1[d] = w[d] / lw;
  } else {
    T n[3] = {g1[1] * g2[2] - g1[2] * g2[1],
              g1[2] * g2[0] - g1[0] * g2[2],
              g1[0] * g2[1] - g1[1] * g2[0]};
    T ln = sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
    T lg = sqrt((g1[0] * g1[0] + g1[1] * g1[1]) + g1[2] * g1[2]);
    for (int d = 0; d < 3; ++d) {
      n0[d] = n[d] / ln;
      t1[d] = g1[d] / lg;
    }
  }
  t2[0] = n0[1] * t1[2] - n0[2] * t1[1];
  t2[1] = n0[2] * t1[0] - n0[0] * t1[2];
  t2[2] = n0[0] * t1[1] - n0[1] * t1[0];
}

// Unit normal of a quad at its corner k: the cross product of the edges to
// the next and to the previous node (the normal of the bilinear map there).
template <class T>
void corner_normal(const T X[4][3], int k, T v[3]) {
  const int a = (k + 1) % 4, b = (k + 3) % 4;
  T e1[3], e2[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = X[a][d] - X[k][d];
    e2[d] = X[b][d] - X[k][d];
  }
  const T c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const T l = sqrt((c[0] * c[0] + c[1] * c[1]) + c[2] * c[2]);
  for (int d = 0; d < 3; ++d) v[d] = c[d] / l;
}

// In-plane coordinates (u, v) and signed height h above the plane.
template <class T>
void project(const T X[3], const T x0[3], const T n0[3], const T t1[3],
             const T t2[3], P2<T>& p, T& h) {
  T d0 = X[0] - x0[0], d1 = X[1] - x0[1], d2 = X[2] - x0[2];
  p.u = (d0 * t1[0] + d1 * t1[1]) + d2 * t1[2];
  p.v = (d0 * t2[0] + d1 * t2[1]) + d2 * t2[2];
  h = (d0 * n0[0] + d1 * n0[1]) + d2 * n0[2];
}

// Signed area of a polygon as the sum of its fan triangles from vertex 0.
template <class T>
T fan_area(int n, const P2<T>* p) {
  T a = 0.0;
  for (int i = 1; i + 1 < n; ++i)
    a = a + ((p[i].u - p[0].u) * (p[i + 1].v - p[0].v) -
             (p[i].v - p[0].v) * (p[i + 1].u - p[0].u));
  return 0.5 * a;
}

// ------------------------------------------------------------------ clip

// One Sutherland-Hodgman stage (Foley et al., cited by Alg. 1): keep the
// closed left half plane of the directed line a->b.  Walk the subject edges
// P=v_j -> E=v_{j+1}; emit P when it is inside, then the crossing point when
// P and E lie on different sides.  This loop, started at slave node 0 with
// master edge 0 as the first clip line, reproduces Fig. 1's clip polygon and
// vertex order exactly.
template <class T>
void clip_stage(const Poly<T>& in, const P2<T>& a, const P2<T>& b, Poly<T>& out) {
  out.clear();
  const int n = (int)in.size();
  if (n == 0) return;
  std::vector<T> c(n);
  for (int j = 0; j < n; ++j)
    c[j] = (b.u - a.u) * (in[j].v - a.v) - (b.v - a.v) * (in[j].u - a.u);
  for (int j = 0; j < n; ++j) {
    const int e = (j + 1) % n;
    const bool pin = val(c[j]) >= 0.0;
    const bool ein = val(c[e]) >= 0.0;
    if (pin) out.push_back(in[j]);
    if (pin != ein) {
      T t = c[j] / (c[j] - c[e]);
      P2<T> x;
      x.u = in[j].u + t * (in[e].u - in[j].u);
      x.v = in[j].v + t * (in[e].v - in[j].v);
      out.push_back(x);
    }
  }
}

inline double linf(double du, double dv) { return std::max(std::fabs(du), std::fabs(dv)); }

// Cleanup of a raw clip polygon (the paper is silent; this is our reading):
//  (i)  walk the vertices once, dropping any vertex within tol (max-norm) of
//       the previously kept one; vertex 0 is always kept, and the last kept
//       vertex is dropped if it lies within tol of vertex 0;
//  (ii) repeatedly sweep in index order removing any vertex whose distance to
//       the line through its two cyclic neighbours is at most tol, measured
//       as |cross(next-prev, v-prev)| <= tol * maxnorm(next-prev), until a
//       sweep removes nothing or fewer than 3 vertices remain.
template <class T>
void cleanup(Poly<T>& p, double tol) {
  int n = (int)p.size();
  if (n == 0) return;
  int m = 1;
  for (int i = 1; i < n; ++i) {
    if (linf(val(p[i].u) - val(p[m - 1].u), val(p[i].v) - val(p[m - 1].v)) > tol)
      p[m++] = p[i];
  }
  if (m > 1 && linf(val(p[m - 1].u) - val(p[0].u), val(p[m - 1].v) - val(p[0].v)) <= tol) --m;
  p.resize(m);
  bool changed = true;
  while (changed && p.size() >= 3) {
    changed = false;
    size_t i = 0;
    while (i < p.size() && p.size() >= 3) {
      const size_t k = p.size();
      const P2<T>& a = p[(i + k - 1) % k];
      const P2<T>& b = p[(i + 1) % k];
      const double bu = val(b.u) - val(a.u), bv = val(b.v) - val(a.v);
      const double cr = bu * (val(p[i].v) - val(a.v)) - bv * (val(p[i].u) - val(a.u));
      if (std::fabs(cr) <= tol * linf(bu, bv)) {
        p.erase(p.begin() + (std::ptrdiff_t)i);
        changed = true;
      } else {
        ++i;
      }
    }
  }
}

// ----------------------------------------------------------- quadrature

struct Rule { int n; double l[7][3]; double w[7]; };

// Barycentric triangle rules with weights summing to one.
//  3 points: degree 2, points (2/3, 1/6, 1/6) and permutations (Fig. 1).
//  7 points: degree 5 (Radon's rule, as tabulated by Dunavant 1985).
Rule make_rule(int which) {
  Rule r{};
  if (which == 3) {
    r.n = 3;
    const double a = 2.0 / 3.0, b = 1.0 / 6.0;
    const double L[3][3] = {{a, b, b}, {b, a, b}, {b, b, a}};
    for (int q = 0; q < 3; ++q) { for (int i = 0; i < 3; ++i) r.l[q][i] = L[q][i]; r.w[q] = 1.0 / 3.0; }
    return r;
  }
  r.n = 7;
  const double s15 = std::sqrt(15.0);
  const double a1 = (6.0 - s15) / 21.0, b1 = 1.0 - 2.0 * a1, w1 = (155.0 - s15) / 1200.0;
  const double a2 = (6.0 + s15) / 21.0, b2 = 1.0 - 2.0 * a2, w2 = (155.0 + s15) / 1200.0;
  const double L[7][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
                          {b1, a1, a1}, {a1, b1, a1}, {a1, a1, b1},
                          {b2, a2, a2}, {a2, b2, a2}, {a2, a2, b2}};
  const double W[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
  for (int q = 0; q < 7; ++q) { for (int i = 0; i < 3; ++i) r.l[q][i] = L[q][i]; r.w[q] = W[q]; }
  return r;
}

// Parameter coordinates xi of an in-plane point p on the bilinear map of the
// projected quad X: Newton's method from xi = 0 on sum_k N_k(xi) X_k = p.
// Equivalent to projecting p along n0 back onto the element.
template <class T> struct InverseMapScope {
  InverseMapScope() {}
};
template <> struct InverseMapScope<Cnt> {
  InverseMapScope() { g_in_inverse_map = true; ++g_inverse_maps; }
  ~InverseMapScope() { g_in_inverse_map = false; }
};

template <class T>
int inverse_bilinear(const P2<T> X[4], const P2<T>& p, const Params& prm, T& x1, T& x2) {
  InverseMapScope<T> scope;
  x1 = 0.0; x2 = 0.0;
  for (int it = 0; it < prm.newton_maxit; ++it) {
    T N[4], d1[4], d2[4];
    shape(x1, x2, N, d1, d2);
    T xu = 0.0, xv = 0.0, j00 = 0.0, j01 = 0.0, j10 = 0.0, j11 = 0.0;
    for (int k = 0; k < 4; ++k) {
      xu = xu + N[k] * X[k].u;   xv = xv + N[k] * X[k].v;
      j00 = j00 + d1[k] * X[k].u; j01 = j01 + d2[k] * X[k].u;
      j10 = j10 + d1[k] * X[k].v; j11 = j11 + d2[k] * X[k].v;
    }
    T ru = xu - p.u, rv = xv - p.v;
    T det = j00 * j11 - j01 * j10;
    T s1 = (j11 * ru - j01 * rv) / det;
    T s2 = (j00 * rv - j10 * ru) / det;
    x1 = x1 - s1;
    x2 = x2 - s2;
    if (std::max(std::fabs(val(s1)), std::fabs(val(s2))) <= prm.newton_tol) return 0;
  }
  return ST_NOCONV;
}

// Dual (biorthogonal) basis coefficients: Phi_j = sum_k A[j][k] N_k with
// A = De Me^-1, De = diag(int N_j), Me = int N N^T over the projected slave
// quad, integrated by 2x2 Gauss (exact for these bilinear integrands).  Then
// int Phi_j N_k = delta_jk int N_k, which makes D diagonal.
template <class T>
void dual_coefficients(const P2<T> S[4], T A[16]) {
  const double g = 1.0 / std::sqrt(3.0);
  const double gp[2] = {-g, g};
  T Me[16], De[4];
  for (int i = 0; i < 16; ++i) Me[i] = 0.0;
  for (int i = 0; i < 4; ++i) De[i] = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      T x1 = gp[a], x2 = gp[b];
      T N[4], d1[4], d2[4];
      shape(x1, x2, N, d1, d2);
      T j00 = 0.0, j01 = 0.0, j10 = 0.0, j11 = 0.0;
      for (int k = 0; k < 4; ++k) {
        j00 = j00 + d1[k] * S[k].u; j01 = j01 + d2[k] * S[k].u;
        j10 = j10 + d1[k] * S[k].v; j11 = j11 + d2[k] * S[k].v;
      }
      T det = j00 * j11 - j01 * j10;
      for (int j = 0; j < 4; ++j) {
        De[j] = De[j] + N[j] * det;
        for (int k = 0; k < 4; ++k) Me[j * 4 + k] = Me[j * 4 + k] + (N[j] * N[k]) * det;
      }
    }
  // Gauss-Jordan inverse of Me with partial pivoting.
  T inv[16];
  for (int i = 0; i < 16; ++i) inv[i] = (i % 5 == 0) ? T(1.0) : T(0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (std::fabs(val(Me[r * 4 + c])) > std::fabs(val(Me[piv * 4 + c]))) piv = r;
    if (piv != c)
      for (int k = 0; k < 4; ++k) { std::swap(Me[c * 4 + k], Me[piv * 4 + k]); std::swap(inv[c * 4 + k], inv[piv * 4 + k]); }
    T d = Me[c * 4 + c];
    for (int k = 0; k < 4; ++k) { Me[c * 4 + k] = Me[c * 4 + k] / d; inv[c * 4 + k] = inv[c * 4 + k] / d; }
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      T f = Me[r * 4 + c];
      for (int k = 0; k < 4; ++k) {
        Me[r * 4 + k] = Me[r * 4 + k] - f * Me[c * 4 + k];
        inv[r * 4 + k] = inv[r * 4 + k] - f * inv[c * 4 + k];
      }
    }
  }
  for (int j = 0; j < 4; ++j)
    for (int k = 0; k < 4; ++k) A[j * 4 + k] = De[j] * inv[j * 4 + k];
}

// ------------------------------------------------------------- one pair

template <class T>
struct PairOut {
  int nv = 0;          // clip polygon vertex count after cleanup (0: no pair)
  int status = 0;
  Poly<T> poly;        // the cleaned clip polygon of a pair
  T D[16], M[16], g[4];
};

// Alg. 1 for one (slave, master) candidate.  Local blocks:
//   D[j][k] = int_seg Phi_j N_k(xi),  M[j][l] = int_seg Phi_j N_l(eta),
//   g[j]    = int_seg Phi_j (h_m(eta) - h_s(xi)),
// integrals over the clip polygon in the slave auxiliary plane, with xi and
// eta the slave / master parameter coordinates of the in-plane point and h
// the heights of the master / slave surfaces above the plane along n0.  The
// weighted gap is our reading of the paper's "normal distance" gap: positive
// when the master lies on the +n0 side of the slave.
template <class T>
void eval_pair(const T Xs[4][3], const T Xm[4][3], const Params& prm,
               const Rule& rule, bool integrate, PairOut<T>& out, const T* nin = nullptr) {
  out.nv = 0;
  out.status = 0;
  out.poly.clear();
  for (int i = 0; i < 16; ++i) { out.D[i] = 0.0; out.M[i] = 0.0; }
  for (int i = 0; i < 4; ++i) out.g[i] = 0.0;

  T x0[3], n0[3], t1[3], t2[3];
  slave_frame(Xs, nin, x0, n0, t1, t2);
  P2<T> S[4], Mn[4];
  T hs[4], hm[4];
  for (int k = 0; k < 4; ++k) project(Xs[k], x0, n0, t1, t2, S[k], hs[k]);
  for (int k = 0; k < 4; ++k) project(Xm[k], x0, n0, t1, t2, Mn[k], hm[k]);

  T As = fan_area(4, S);
  if (!(val(As) > 0.0)) { out.status |= ST_DEGEN_SLAVE; return; }
  double hmax = 0.0;
  for (int k = 0; k < 4; ++k) {
    const int e = (k + 1) % 4;
    hmax = std::max(hmax, linf(val(S[e].u) - val(S[k].u), val(S[e].v) - val(S[k].v)));
  }
  const double tol_d = prm.eps_d * hmax;
  const double tol_a = prm.eps_a * val(As);

  T Am = fan_area(4, Mn);
  if (std::fabs(val(Am)) <= tol_a) { out.status |= ST_DEGEN_MASTER; return; }
  // Clip with a counter-clockwise master polygon; a clockwise projection
  // (opposing normals, as in contact) is walked as M0, M3, M2, M1.
  P2<T> Mo[4] = {Mn[0], Mn[1], Mn[2], Mn[3]};
  if (val(Am) < 0.0) { Mo[1] = Mn[3]; Mo[3] = Mn[1]; }

  // Sutherland-Hodgman: the slave polygon from node 0 is the subject, the
  // oriented master edges from edge 0 the clip lines.
  Poly<T> cur(S, S + 4), nxt;
  for (int l = 0; l < 4 && !cur.empty(); ++l) {
    clip_stage(cur, Mo[l], Mo[(l + 1) % 4], nxt);
    cur.swap(nxt);
  }
  cleanup(cur, tol_d);
  const int n = (int)cur.size();
  if (n < 3) return;
  T Ap = fan_area(n, cur.data());
  if (!(val(Ap) > tol_a)) return;
  out.nv = n;
  out.poly = cur;
  if (!integrate) return;

  T A[16];
  if (prm.dual) dual_coefficients(S, A);

  const P2<T>* P = out.poly.data();
  for (int i = 1; i + 1 < n; ++i) {
    const P2<T>& V0 = P[0];
    const P2<T>& V1 = P[i];
    const P2<T>& V2 = P[i + 1];
    T At = 0.5 * ((V1.u - V0.u) * (V2.v - V0.v) - (V1.v - V0.v) * (V2.u - V0.u));
    for (int q = 0; q < rule.n; ++q) {
      P2<T> p;
      p.u = (rule.l[q][0] * V0.u + rule.l[q][1] * V1.u) + rule.l[q][2] * V2.u;
      p.v = (rule.l[q][0] * V0.v + rule.l[q][1] * V1.v) + rule.l[q][2] * V2.v;
      T wA = rule.w[q] * At;
      T xs1, xs2, xm1, xm2;
      out.status |= inverse_bilinear(S, p, prm, xs1, xs2);
      out.status |= inverse_bilinear(Mn, p, prm, xm1, xm2);
      T Ns[4], Nm[4], d1[4], d2[4];
      shape(xs1, xs2, Ns, d1, d2);
      shape(xm1, xm2, Nm, d1, d2);
      T Phi[4];
      for (int j = 0; j < 4; ++j) {
        if (prm.dual) {
          Phi[j] = 0.0;
          for (int k = 0; k < 4; ++k) Phi[j] = Phi[j] + A[j * 4 + k] * Ns[k];
        } else {
          Phi[j] = Ns[j];
        }
      }
      T gap = 0.0;
      for (int k = 0; k < 4; ++k) gap = gap + Nm[k] * hm[k];
      for (int k = 0; k < 4; ++k) gap = gap - Ns[k] * hs[k];
      for (int j = 0; j < 4; ++j) {
        T wp = wA * Phi[j];
        for (int k = 0; k < 4; ++k) {
          out.D[j * 4 + k] = out.D[j * 4 + k] + wp * Ns[k];
          out.M[j * 4 + k] = out.M[j * 4 + k] + wp * Nm[k];
        }
        out.g[j] = out.g[j] + wp * gap;
      }
    }
  }
}

// ------------------------------------------------ element-based integration

// Gauss-Legendre points and weights on [-1, 1] in ascending order, exact for
// polynomials up to degree 2n - 1.  The points are the roots of the Legendre
// polynomial P_n: root i of the upper half by Newton's method from
// cos(pi (i + 3/4) / (n + 1/2)), mirrored for the lower half, 0 in the middle
// for odd n.  P_n and P_n' come from the recurrence (k + 1) P_{k+1} =
// (2k + 1) x P_k - k P_{k-1} and P_n' = n (x P_n - P_{n-1}) / (x^2 - 1); the
// weight is 2 / ((1 - x^2) P_n'(x)^2).
void legendre(int n, double z, double& pn, double& dpn) {
  double p0 = 1.0, p1 = z;
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  dpn = n * (z * p1 - p0) / (z * z - 1.0);
}

void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = (2 * i + 1 == n) ? 0.0 : std::cos(std::acos(-1.0) * (i + 0.75) / (n + 0.5));
    double pn, dp;
    for (int it = 0; it < 100 && z != 0.0; ++it) {
      legendre(n, z, pn, dp);
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) <= 1e-16) break;
    }
    legendre(n, z, pn, dp);
    const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    w[i] = wi;
    x[n - 1 - i] = z;
    w[n - 1 - i] = wi;
  }
}

// Element-based integration of one slave element (Sec. "Evaluation of mortar
// integrals": no clipping or triangulation, a higher-order rule over the
// whole slave element).  The paper gives no formulas for it; our reading:
//  * the rule is the ng x ng Gauss-Legendre product rule in the parameter
//    space of the projected slave quad, with the measure det J of that map
//    (area in the auxiliary plane, the measure of the segment-based
//    integrals, so that both converge to the same values);
//  * the point of the auxiliary plane at xi is the bilinear map of the
//    projected slave quad written in monomial form,
//    P = ((c + e1 xi1) + e2 xi2) + f (xi1 xi2) with c = (S0 + S1 + S2 + S3)/4,
//    e1 = (S1 - S0 + S2 - S3)/4, e2 = (S2 - S1 + S3 - S0)/4,
//    f = (S0 - S1 + S2 - S3)/4 (the same map as sum_k N_k(xi) S_k);
//  * P belongs to the first of the element's pairs (pair order, i.e.
//    ascending master) whose counter-clockwise projected master quad
//    contains it: inside the closed bounding box of the quad and on the
//    closed inner side of its four edges by the clip's side test; points in
//    no master are dropped;
//  * the master coordinates of P come from the inverse bilinear map and the
//    integrands are those of eval_pair.
// XmK holds the K masters' nodes (12 per master); blk receives 36 values per
// pair (layout of eval_pair's D, M, g).  Returns status bits.
template <class T>
int eval_element(const T Xs[4][3], int K, const T* XmK, const Params& prm, int ng, const double* gx,
                 const double* gw, T* blk, const T* nin = nullptr) {
  int status = 0;
  for (int i = 0; i < 36 * K; ++i) blk[i] = 0.0;
  T x0[3], n0[3], t1[3], t2[3];
  slave_frame(Xs, nin, x0, n0, t1, t2);
  P2<T> S[4];
  T hs[4];
  for (int k = 0; k < 4; ++k) project(Xs[k], x0, n0, t1, t2, S[k], hs[k]);
  T A[16];
  if (prm.dual) dual_coefficients(S, A);
  std::vector<P2<T>> Mn(4 * K), Mo(4 * K);
  std::vector<T> hm(4 * K);
  for (int i = 0; i < K; ++i) {
    for (int k = 0; k < 4; ++k) {
      T X[3] = {XmK[12 * i + 3 * k], XmK[12 * i + 3 * k + 1], XmK[12 * i + 3 * k + 2]};
      project(X, x0, n0, t1, t2, Mn[4 * i + k], hm[4 * i + k]);
    }
    const T Am = fan_area(4, &Mn[4 * i]);
    for (int k = 0; k < 4; ++k) Mo[4 * i + k] = Mn[4 * i + k];
    if (val(Am) < 0.0) { Mo[4 * i + 1] = Mn[4 * i + 3]; Mo[4 * i + 3] = Mn[4 * i + 1]; }
  }
  P2<T> c, e1, e2, f;
  c.u = 0.25 * ((S[0].u + S[1].u) + (S[2].u + S[3].u));
  c.v = 0.25 * ((S[0].v + S[1].v) + (S[2].v + S[3].v));
  e1.u = 0.25 * ((S[1].u - S[0].u) + (S[2].u - S[3].u));
  e1.v = 0.25 * ((S[1].v - S[0].v) + (S[2].v - S[3].v));
  e2.u = 0.25 * ((S[2].u - S[1].u) + (S[3].u - S[0].u));
  e2.v = 0.25 * ((S[2].v - S[1].v) + (S[3].v - S[0].v));
  f.u = 0.25 * ((S[0].u - S[1].u) + (S[2].u - S[3].u));
  f.v = 0.25 * ((S[0].v - S[1].v) + (S[2].v - S[3].v));
  for (int b = 0; b < ng; ++b)
    for (int a = 0; a < ng; ++a) {
      const T x1 = gx[a], x2 = gx[b];
      T Ns[4], d1[4], d2[4];
      shape(x1, x2, Ns, d1, d2);
      P2<T> P;
      P.u = ((c.u + e1.u * x1) + e2.u * x2) + f.u * (x1 * x2);
      P.v = ((c.v + e1.v * x1) + e2.v * x2) + f.v * (x1 * x2);
      int owner = -1;
      for (int i = 0; i < K && owner < 0; ++i) {
        bool inside = true;
        double lo_u = val(Mo[4 * i].u), hi_u = lo_u, lo_v = val(Mo[4 * i].v), hi_v = lo_v;
        for (int k = 1; k < 4; ++k) {
          lo_u = std::min(lo_u, val(Mo[4 * i + k].u)); hi_u = std::max(hi_u, val(Mo[4 * i + k].u));
          lo_v = std::min(lo_v, val(Mo[4 * i + k].v)); hi_v = std::max(hi_v, val(Mo[4 * i + k].v));
        }
        if (val(P.u) < lo_u || val(P.u) > hi_u || val(P.v) < lo_v || val(P.v) > hi_v) inside = false;
        for (int l = 0; l < 4; ++l) {
          const P2<T>& ea = Mo[4 * i + l];
          const P2<T>& eb = Mo[4 * i + (l + 1) % 4];
          const T c = (eb.u - ea.u) * (P.v - ea.v) - (eb.v - ea.v) * (P.u - ea.u);
          if (!(val(c) >= 0.0)) inside = false;
        }
        if (inside) owner = i;
      }
      if (owner < 0) continue;
      T j00 = 0.0, j01 = 0.0, j10 = 0.0, j11 = 0.0;
      for (int k = 0; k < 4; ++k) {
        j00 = j00 + d1[k] * S[k].u; j01 = j01 + d2[k] * S[k].u;
        j10 = j10 + d1[k] * S[k].v; j11 = j11 + d2[k] * S[k].v;
      }
      const T wJ = (gw[a] * gw[b]) * (j00 * j11 - j01 * j10);
      T xm1, xm2;
      status |= inverse_bilinear(&Mn[4 * owner], P, prm, xm1, xm2);
      T Nm[4], e1[4], e2[4];
      shape(xm1, xm2, Nm, e1, e2);
      T Phi[4];
      for (int j = 0; j < 4; ++j) {
        if (prm.dual) {
          Phi[j] = 0.0;
          for (int k = 0; k < 4; ++k) Phi[j] = Phi[j] + A[j * 4 + k] * Ns[k];
        } else {
          Phi[j] = Ns[j];
        }
      }
      T gap = 0.0;
      for (int k = 0; k < 4; ++k) gap = gap + Nm[k] * hm[4 * owner + k];
      for (int k = 0; k < 4; ++k) gap = gap - Ns[k] * hs[k];
      T* o = blk + 36 * owner;
      for (int j = 0; j < 4; ++j) {
        const T wp = wJ * Phi[j];
        for (int k = 0; k < 4; ++k) {
          o[j * 4 + k] = o[j * 4 + k] + wp * Ns[k];
          o[16 + j * 4 + k] = o[16 + j * 4 + k] + wp * Nm[k];
        }
        o[32 + j] = o[32 + j] + wp * gap;
      }
    }
  return status;
}

// ---------------------------------------------------------------- search

struct Box { double lo[3], hi[3]; };

Box element_box(const double* X, const int32_t* C, int64_t e) {
  Box b;
  for (int d = 0; d < 3; ++d) { b.lo[d] = X[3 * C[4 * e] + d]; b.hi[d] = b.lo[d]; }
  for (int k = 1; k < 4; ++k)
    for (int d = 0; d < 3; ++d) {
      const double x = X[3 * C[4 * e + k] + d];
      b.lo[d] = std::min(b.lo[d], x);
      b.hi[d] = std::max(b.hi[d], x);
    }
  return b;
}

// Candidate test: the slave box enlarged by delta on every side and the
// master box overlap as closed intervals on all three axes.
inline bool boxes_touch(const Box& s, const Box& m, double delta) {
  for (int d = 0; d < 3; ++d)
    if (!((s.lo[d] - delta) <= m.hi[d] && m.lo[d] <= (s.hi[d] + delta))) return false;
  return true;
}

struct MeshView {
  int64_t n_nodes; const double* X; int64_t n_el; const int32_t* C;
};

void search_brute(const MeshView& S, const MeshView& M, double delta,
                  std::vector<int32_t>& os, std::vector<int32_t>& om) {
  std::vector<Box> mb(M.n_el);
  for (int64_t e = 0; e < M.n_el; ++e) mb[e] = element_box(M.X, M.C, e);
  for (int64_t s = 0; s < S.n_el; ++s) {
    Box sb = element_box(S.X, S.C, s);
    for (int64_t m = 0; m < M.n_el; ++m)
      if (boxes_touch(sb, mb[m], delta)) { os.push_back((int32_t)s); om.push_back((int32_t)m); }
  }
}

// Cartesian binning (Alg. 2 restricted to one process).  Minimal bin size:
// the longest slave element edge (the paper's rule with no motion term),
// raised to the largest element box extent plus delta so that overlapping
// boxes always have centres in the same or adjacent bins; a relative margin
// of 2^-20 keeps that argument valid under rounding.  The bounding box of all
// nodes is expanded by the minimal bin size on every side, and each axis gets
// max(1, floor(L / beta_min)) bins.  A slave element scans its own bin and
// its 26 neighbours.
void search_binned(const MeshView& S, const MeshView& M, double delta,
                   std::vector<int32_t>& os, std::vector<int32_t>& om) {
  std::vector<Box> sb(S.n_el), mb(M.n_el);
  double emax = 0.0, edge = 0.0;
  for (int64_t e = 0; e < S.n_el; ++e) {
    sb[e] = element_box(S.X, S.C, e);
    for (int d = 0; d < 3; ++d) emax = std::max(emax, sb[e].hi[d] - sb[e].lo[d]);
    for (int k = 0; k < 4; ++k) {
      const double* a = S.X + 3 * S.C[4 * e + k];
      const double* b = S.X + 3 * S.C[4 * e + (k + 1) % 4];
      const double l = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                                 (b[2] - a[2]) * (b[2] - a[2]));
      edge = std::max(edge, l);
    }
  }
  for (int64_t e = 0; e < M.n_el; ++e) {
    mb[e] = element_box(M.X, M.C, e);
    for (int d = 0; d < 3; ++d) emax = std::max(emax, mb[e].hi[d] - mb[e].lo[d]);
  }
  double beta_min = std::max(edge, emax + delta) * (1.0 + std::ldexp(1.0, -20));
  if (!(beta_min > 0.0)) beta_min = 1.0;
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) { lo[d] = INFINITY; hi[d] = -INFINITY; }
  for (const MeshView* mv : {&S, &M})
    for (int64_t i = 0; i < mv->n_nodes; ++i)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], mv->X[3 * i + d]);
        hi[d] = std::max(hi[d], mv->X[3 * i + d]);
      }
  int64_t nb[3];
  double beta[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] -= beta_min;
    hi[d] += beta_min;
    const double L = hi[d] - lo[d];
    nb[d] = std::max<int64_t>(1, (int64_t)std::floor(L / beta_min));
    nb[d] = std::min<int64_t>(nb[d], 1024);  // a coarser grid stays complete
    beta[d] = L / (double)nb[d];
  }
  auto bin_of = [&](const Box& b, int64_t ix[3]) {
    for (int d = 0; d < 3; ++d) {
      const double c = 0.5 * (b.lo[d] + b.hi[d]);
      int64_t i = (int64_t)std::floor((c - lo[d]) / beta[d]);
      ix[d] = std::min<int64_t>(nb[d] - 1, std::max<int64_t>(0, i));
    }
  };
  const int64_t nbins = nb[0] * nb[1] * nb[2];
  std::vector<std::vector<int32_t>> bins(nbins);
  for (int64_t e = 0; e < M.n_el; ++e) {
    int64_t ix[3];
    bin_of(mb[e], ix);
    bins[ix[0] + nb[0] * (ix[1] + nb[1] * ix[2])].push_back((int32_t)e);
  }
  std::vector<int32_t> found;
  for (int64_t s = 0; s < S.n_el; ++s) {
    int64_t ix[3];
    bin_of(sb[s], ix);
    found.clear();
    for (int64_t dz = -1; dz <= 1; ++dz)
      for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dx = -1; dx <= 1; ++dx) {
          const int64_t x = ix[0] + dx, y = ix[1] + dy, z = ix[2] + dz;
          if (x < 0 || y < 0 || z < 0 || x >= nb[0] || y >= nb[1] || z >= nb[2]) continue;
          for (int32_t m : bins[x + nb[0] * (y + nb[1] * z)])
            if (boxes_touch(sb[s], mb[m], delta)) found.push_back(m);
        }
    std::sort(found.begin(), found.end());
    for (int32_t m : found) { os.push_back((int32_t)s); om.push_back(m); }
  }
}

template <class T>
void load_pair(const MeshView& S, const MeshView& M, int32_t s, int32_t m, T Xs[4][3], T Xm[4][3]) {
  for (int k = 0; k < 4; ++k)
    for (int d = 0; d < 3; ++d) {
      Xs[k][d] = S.X[3 * S.C[4 * s + k] + d];
      Xm[k][d] = M.X[3 * M.C[4 * m + k] + d];
    }
}

// Continuous normal field of the slave side (Sec. "Discretization": the
// projections between the two sides usually rest on a continuous field of
// slave normals; the paper does not define it).  Our reading: the nodal
// normal n_a is the normalised sum of the unit corner normals of the elements
// around node a, added in ascending element order; an element's
// auxiliary-plane normal is the normalised sum of its four nodal normals in
// node order (the interpolated field at the element centre, normalised).
void nodal_normals(const MeshView& S, std::vector<double>& nn) {
  nn.assign(3 * S.n_nodes, 0.0);
  for (int64_t e = 0; e < S.n_el; ++e) {
    double X[4][3];
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) X[k][d] = S.X[3 * S.C[4 * e + k] + d];
    for (int k = 0; k < 4; ++k) {
      double v[3];
      corner_normal(X, k, v);
      const int64_t a = S.C[4 * e + k];
      for (int d = 0; d < 3; ++d) nn[3 * a + d] = nn[3 * a + d] + v[d];
    }
  }
  for (int64_t a = 0; a < S.n_nodes; ++a) {
    double* u = &nn[3 * a];
    const double l = std::sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
    if (l > 0.0)
      for (int d = 0; d < 3; ++d) u[d] = u[d] / l;
  }
}

void element_normals(const MeshView& S, const std::vector<double>& nn, std::vector<double>& ne) {
  ne.assign(3 * S.n_el, 0.0);
  for (int64_t e = 0; e < S.n_el; ++e) {
    const int32_t* c = S.C + 4 * e;
    double v[3];
    for (int d = 0; d < 3; ++d) v[d] = ((nn[3 * c[0] + d] + nn[3 * c[1] + d]) + nn[3 * c[2] + d]) + nn[3 * c[3] + d];
    const double l = std::sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    for (int d = 0; d < 3; ++d) ne[3 * e + d] = v[d] / l;
  }
}

// Element normals of the slave side when the parameters ask for the nodal
// field, else empty.
std::vector<double> frame_normals(const MeshView& S, const Params& prm) {
  std::vector<double> nn, ne;
  if (prm.normals) {
    nodal_normals(S, nn);
    element_normals(S, nn, ne);
  }
  return ne;
}

}  // namespace

// ================================================================== C API

extern "C" {

struct OrParams {
  double delta;
  int32_t dual;
  int32_t rule;
  double eps_d;
  double eps_a;
  double newton_tol;
  int32_t newton_maxit;
  int32_t normals;
};

static Params to_params(const OrParams* p) {
  Params q;
  q.delta = p->delta; q.dual = p->dual; q.rule = p->rule; q.eps_d = p->eps_d;
  q.eps_a = p->eps_a; q.newton_tol = p->newton_tol; q.newton_maxit = p->newton_maxit;
  q.normals = p->normals;
  return q;
}

int or_capacity() { return OR_MAX_VERTICES; }

// Candidate pairs sorted by (slave, master).  method 0: brute force over all
// pairs; method 1: binning.  Returns 0, or 1 when `cap` is too small (then
// *n_out holds the required count and nothing is written).
int or_search(int method, int64_t ns_nodes, const double* Xs, int64_t ns_el, const int32_t* Cs,
              int64_t nm_nodes, const double* Xm, int64_t nm_el, const int32_t* Cm,
              double delta, int64_t cap, int32_t* out_s, int32_t* out_m, int64_t* n_out) {
  MeshView S{ns_nodes, Xs, ns_el, Cs}, M{nm_nodes, Xm, nm_el, Cm};
  std::vector<int32_t> os, om;
  if (method == 0) search_brute(S, M, delta, os, om);
  else search_binned(S, M, delta, os, om);
  *n_out = (int64_t)os.size();
  if ((int64_t)os.size() > cap) return 1;
  std::copy(os.begin(), os.end(), out_s);
  std::copy(om.begin(), om.end(), out_m);
  return 0;
}

// Per candidate: vertex count of the cleaned clip polygon (0 = not a pair),
// status bits, and (when blocks != NULL) the local blocks
// [D 4x4 row-major | M 4x4 row-major | g 4] = 36 doubles per candidate.
int or_eval_candidates(int64_t ns_nodes, const double* Xs, int64_t ns_el, const int32_t* Cs,
                       int64_t nm_nodes, const double* Xm, int64_t nm_el, const int32_t* Cm,
                       const OrParams* op, int64_t n, const int32_t* cs, const int32_t* cm,
                       uint8_t* nverts, double* blocks, int32_t* status) {
  MeshView S{ns_nodes, Xs, ns_el, Cs}, M{nm_nodes, Xm, nm_el, Cm};
  const Params prm = to_params(op);
  const Rule rule = make_rule(prm.rule);
  const std::vector<double> ne = frame_normals(S, prm);
  int any = 0;
  for (int64_t i = 0; i < n; ++i) {
    double xs[4][3], xm[4][3];
    load_pair(S, M, cs[i], cm[i], xs, xm);
    PairOut<double> o;
    eval_pair(xs, xm, prm, rule, blocks != nullptr, o, ne.empty() ? nullptr : &ne[3 * cs[i]]);
    nverts[i] = (uint8_t)o.nv;
    if (status) status[i] = o.status;
    any |= o.status;
    if (blocks) {
      double* b = blocks + 36 * i;
      for (int k = 0; k < 16; ++k) { b[k] = o.D[k]; b[16 + k] = o.M[k]; }
      for (int k = 0; k < 4; ++k) b[32 + k] = o.g[k];
    }
  }
  return any;
}

// Clip polygon of one candidate (cleaned), in slave auxiliary-plane
// coordinates; returns the vertex count.
int or_pair_polygon(const double* Xs4, const double* Xm4, const OrParams* op, double* pu, double* pv,
                    int32_t* status) {
  double xs[4][3], xm[4][3];
  for (int k = 0; k < 4; ++k)
    for (int d = 0; d < 3; ++d) { xs[k][d] = Xs4[3 * k + d]; xm[k][d] = Xm4[3 * k + d]; }
  const Params prm = to_params(op);
  PairOut<double> o;
  eval_pair(xs, xm, prm, make_rule(prm.rule), false, o);
  *status = o.status;
  if (o.nv > OR_MAX_VERTICES) return -1;
  for (int i = 0; i < o.nv; ++i) { pu[i] = o.poly[i].u; pv[i] = o.poly[i].v; }
  return o.nv;
}

// Plain 2-D clip of a subject polygon by a convex counter-clockwise clipper.
// Writes the raw Sutherland-Hodgman output and the cleaned polygon.
int or_clip2d(int ns, const double* su, const double* sv, int nc, const double* cu, const double* cv,
              double tol, double* raw_u, double* raw_v, int32_t* n_raw, double* out_u, double* out_v) {
  Poly<double> cur, nxt, C;
  for (int i = 0; i < ns; ++i) cur.push_back({su[i], sv[i]});
  for (int i = 0; i < nc; ++i) C.push_back({cu[i], cv[i]});
  for (int l = 0; l < nc && !cur.empty(); ++l) {
    clip_stage(cur, C[l], C[(l + 1) % nc], nxt);
    cur.swap(nxt);
  }
  if ((int)cur.size() > OR_MAX_VERTICES) return -2;
  *n_raw = (int32_t)cur.size();
  for (size_t i = 0; i < cur.size(); ++i) { raw_u[i] = cur[i].u; raw_v[i] = cur[i].v; }
  cleanup(cur, tol);
  for (size_t i = 0; i < cur.size(); ++i) { out_u[i] = cur[i].u; out_v[i] = cur[i].v; }
  return (int)cur.size();
}

// Quadrature points of the fan triangulation of a polygon: for triangle
// (v0, v_i, v_{i+1}), i = 1..n-2, the rule's points in rule order; weights
// include the triangle area.  Returns the number of points.
int or_fan_points(int n, const double* pu, const double* pv, int which, double* qu, double* qv, double* qw) {
  const Rule r = make_rule(which);
  int c = 0;
  for (int i = 1; i + 1 < n; ++i) {
    const double A = 0.5 * ((pu[i] - pu[0]) * (pv[i + 1] - pv[0]) - (pv[i] - pv[0]) * (pu[i + 1] - pu[0]));
    for (int q = 0; q < r.n; ++q) {
      qu[c] = (r.l[q][0] * pu[0] + r.l[q][1] * pu[i]) + r.l[q][2] * pu[i + 1];
      qv[c] = (r.l[q][0] * pv[0] + r.l[q][1] * pv[i]) + r.l[q][2] * pv[i + 1];
      qw[c] = r.w[q] * A;
      ++c;
    }
  }
  return c;
}

// Triangle rule table (barycentric coordinates and weights) for tests.
int or_rule(int which, double* l, double* w) {
  const Rule r = make_rule(which);
  for (int q = 0; q < r.n; ++q) { for (int i = 0; i < 3; ++i) l[3 * q + i] = r.l[q][i]; w[q] = r.w[q]; }
  return r.n;
}

// Inverse bilinear map of a 2-D quad (for tests).
int or_inverse_bilinear(const double* qu, const double* qv, double pu, double pv, const OrParams* op,
                        double* x1, double* x2) {
  P2<double> X[4];
  for (int k = 0; k < 4; ++k) X[k] = {qu[k], qv[k]};
  P2<double> p{pu, pv};
  return inverse_bilinear(X, p, to_params(op), *x1, *x2);
}

// Dual basis coefficients of one slave element given by its 4 nodes (4x3).
void or_dual_matrix(const double* Xs4, double* A) {
  double xs[4][3];
  for (int k = 0; k < 4; ++k)
    for (int d = 0; d < 3; ++d) xs[k][d] = Xs4[3 * k + d];
  double x0[3], n0[3], t1[3], t2[3];
  slave_frame(xs, (const double*)nullptr, x0, n0, t1, t2);
  P2<double> S[4];
  double h;
  for (int k = 0; k < 4; ++k) project(xs[k], x0, n0, t1, t2, S[k], h);
  dual_coefficients(S, A);
}

// Gradient of L_pair = <w, blocks> (w: 36 weights per pair laid out like the
// blocks) with respect to the 24 nodal coordinates of each pair:
// [slave node 0..3 (x,y,z) | master node 0..3 (x,y,z)], by forward-mode dual
// numbers through the whole pair evaluation.  Newton is iterated to
// convergence, so the tangent is the implicit-function derivative.
// With the nodal normal field (params.normals), the slave element's
// auxiliary-plane normal n0 is a further input: grads_n0 (optional) receives
// dL/dn0 per pair (3 values), to be taken to the coordinates by
// or_normal_chain.
int or_pair_grads(int64_t ns_nodes, const double* Xs, int64_t ns_el, const int32_t* Cs,
                  int64_t nm_nodes, const double* Xm, int64_t nm_el, const int32_t* Cm,
                  const OrParams* op, int64_t n, const int32_t* cs, const int32_t* cm,
                  const double* w, double* grads, double* grads_n0, int32_t* status) {
  using D27 = Dual<27>;
  MeshView S{ns_nodes, Xs, ns_el, Cs}, M{nm_nodes, Xm, nm_el, Cm};
  const Params prm = to_params(op);
  const Rule rule = make_rule(prm.rule);
  const std::vector<double> ne = frame_normals(S, prm);
  int any = 0;
  for (int64_t i = 0; i < n; ++i) {
    double xs[4][3], xm[4][3];
    load_pair(S, M, cs[i], cm[i], xs, xm);
    D27 Ds[4][3], Dm[4][3], Dn[3];
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) {
        Ds[k][d] = D27(xs[k][d]); Ds[k][d].d[3 * k + d] = 1.0;
        Dm[k][d] = D27(xm[k][d]); Dm[k][d].d[12 + 3 * k + d] = 1.0;
      }
    if (!ne.empty())
      for (int d = 0; d < 3; ++d) { Dn[d] = D27(ne[3 * cs[i] + d]); Dn[d].d[24 + d] = 1.0; }
    PairOut<D27> o;
    eval_pair(Ds, Dm, prm, rule, true, o, ne.empty() ? nullptr : Dn);
    D27 L(0.0);
    const double* wi = w + 36 * i;
    for (int k = 0; k < 16; ++k) L = L + wi[k] * o.D[k];
    for (int k = 0; k < 16; ++k) L = L + wi[16 + k] * o.M[k];
    for (int k = 0; k < 4; ++k) L = L + wi[32 + k] * o.g[k];
    for (int k = 0; k < 24; ++k) grads[24 * i + k] = L.d[k];
    if (grads_n0)
      for (int d = 0; d < 3; ++d) grads_n0[3 * i + d] = L.d[24 + d];
    if (status) status[i] = o.status;
    any |= o.status;
  }
  return any;
}

// Gradient with respect to the slave coordinates of sum_e <gn0[e], n0_e>,
// n0_e the element normals of the nodal normal field (element_normals), by
// forward-mode dual numbers over the coordinates of each element's patch
// (the nodes of all elements around its four nodes).  Adds to gX (3 per node).
// Returns 0, or 1 when a patch exceeds PMAX (48) nodes.
int or_normal_chain(int64_t ns_nodes, const double* Xs, int64_t ns_el, const int32_t* Cs, const double* gn0,
                    double* gX) {
  constexpr int PMAX = 48;
  using DP = Dual<3 * PMAX>;
  std::vector<std::vector<int32_t>> inc(ns_nodes);
  for (int64_t e = 0; e < ns_el; ++e)
    for (int k = 0; k < 4; ++k) inc[Cs[4 * e + k]].push_back((int32_t)e);
  for (int64_t e = 0; e < ns_el; ++e) {
    const double* g = gn0 + 3 * e;
    if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
    std::vector<int32_t> patch;
    for (int k = 0; k < 4; ++k)
      for (int32_t f : inc[Cs[4 * e + k]])
        for (int j = 0; j < 4; ++j)
          if (std::find(patch.begin(), patch.end(), Cs[4 * f + j]) == patch.end()) patch.push_back(Cs[4 * f + j]);
    if ((int)patch.size() > PMAX) return 1;
    auto slot = [&](int32_t node) { return (int)(std::find(patch.begin(), patch.end(), node) - patch.begin()); };
    auto coords = [&](int32_t f, DP X[4][3]) {
      for (int j = 0; j < 4; ++j) {
        const int32_t a = Cs[4 * f + j];
        const int sl = slot(a);
        for (int d = 0; d < 3; ++d) {
          X[j][d] = DP(Xs[3 * a + d]);
          X[j][d].d[3 * sl + d] = 1.0;
        }
      }
    };
    DP nrm[4][3];
    for (int k = 0; k < 4; ++k) {
      const int32_t a = Cs[4 * e + k];
      DP u[3] = {DP(0.0), DP(0.0), DP(0.0)};
      for (int32_t f : inc[a]) {  // ascending element order
        DP X[4][3];
        coords(f, X);
        int kk = 0;
        while (Cs[4 * f + kk] != a) ++kk;
        DP v[3];
        corner_normal(X, kk, v);
        for (int d = 0; d < 3; ++d) u[d] = u[d] + v[d];
      }
      const DP l = sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
      for (int d = 0; d < 3; ++d) nrm[k][d] = u[d] / l;
    }
    DP v[3];
    for (int d = 0; d < 3; ++d) v[d] = ((nrm[0][d] + nrm[1][d]) + nrm[2][d]) + nrm[3][d];
    const DP l = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    DP L(0.0);
    for (int d = 0; d < 3; ++d) L = L + g[d] * (v[d] / l);
    for (size_t j = 0; j < patch.size(); ++j)
      for (int d = 0; d < 3; ++d) gX[3 * patch[j] + d] += L.d[3 * j + d];
  }
  return 0;
}

// Nodal normals (3 per node) and element normals (3 per element) of a slave
// surface (for tests).
void or_nodal_normals(int64_t ns_nodes, const double* Xs, int64_t ns_el, const int32_t* Cs, double* nn_out,
                      double* ne_out) {
  MeshView S{ns_nodes, Xs, ns_el, Cs};
  std::vector<double> nn, ne;
  nodal_normals(S, nn);
  element_normals(S, nn, ne);
  std::copy(nn.begin(), nn.end(), nn_out);
  std::copy(ne.begin(), ne.end(), ne_out);
}

// Gauss-Legendre rule on [-1, 1] (for tests).
void or_gauss_legendre(int n, double* x, double* w) { gauss_legendre(n, x, w); }

// Element-based integration over the pairs (ps, pm), sorted by slave element:
// the element's pairs are taken together (eval_element) with an ng x ng rule,
// 1 <= ng <= 8.  Writes 36 values per pair (layout of or_eval_candidates);
// status (optional) per pair: the status bits of its slave element.
// Returns the union of the status bits, or -1 for a bad ng.
int or_eval_elements(int64_t ns_nodes, const double* Xs, int64_t ns_el, const int32_t* Cs,
                     int64_t nm_nodes, const double* Xm, int64_t nm_el, const int32_t* Cm,
                     const OrParams* op, int ng, int64_t n, const int32_t* ps, const int32_t* pm,
                     double* blocks, int32_t* status) {
  if (ng < 1 || ng > 8) return -1;
  MeshView S{ns_nodes, Xs, ns_el, Cs}, M{nm_nodes, Xm, nm_el, Cm};
  const Params prm = to_params(op);
  double gx[8], gw[8];
  gauss_legendre(ng, gx, gw);
  const std::vector<double> ne = frame_normals(S, prm);
  int any = 0;
  for (int64_t i0 = 0; i0 < n;) {
    int64_t i1 = i0;
    while (i1 < n && ps[i1] == ps[i0]) ++i1;
    const int K = (int)(i1 - i0);
    double xs[4][3];
    std::vector<double> xm(12 * K);
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) xs[k][d] = S.X[3 * S.C[4 * ps[i0] + k] + d];
    for (int i = 0; i < K; ++i)
      for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) xm[12 * i + 3 * k + d] = M.X[3 * M.C[4 * pm[i0 + i] + k] + d];
    const int st = eval_element(xs, K, xm.data(), prm, ng, gx, gw, blocks + 36 * i0,
                                ne.empty() ? nullptr : &ne[3 * ps[i0]]);
    if (status)
      for (int64_t i = i0; i < i1; ++i) status[i] = st;
    any |= st;
    i0 = i1;
  }
  return any;
}

// Counted floating-point operations of the element-based integration of the
// pairs (ps, pm), sorted by slave element, with an ng x ng rule.
uint64_t or_count_flops_elements(int64_t ns_nodes, const double* Xs, int64_t ns_el, const int32_t* Cs,
                                 int64_t nm_nodes, const double* Xm, int64_t nm_el, const int32_t* Cm,
                                 const OrParams* op, int ng, int64_t n, const int32_t* ps, const int32_t* pm) {
  if (ng < 1 || ng > 8) return 0;
  MeshView S{ns_nodes, Xs, ns_el, Cs}, M{nm_nodes, Xm, nm_el, Cm};
  const Params prm = to_params(op);
  double gx[8], gw[8];
  gauss_legendre(ng, gx, gw);
  g_flops = 0;
  for (int64_t i0 = 0; i0 < n;) {
    int64_t i1 = i0;
    while (i1 < n && ps[i1] == ps[i0]) ++i1;
    const int K = (int)(i1 - i0);
    Cnt xs[4][3];
    std::vector<Cnt> xm(12 * K), blk(36 * K);
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) xs[k][d] = S.X[3 * S.C[4 * ps[i0] + k] + d];
    for (int i = 0; i < K; ++i)
      for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) xm[12 * i + 3 * k + d] = M.X[3 * M.C[4 * pm[i0 + i] + k] + d];
    eval_element(xs, K, xm.data(), prm, ng, gx, gw, blk.data());
    i0 = i1;
  }
  return g_flops;
}

// Counted floating-point operations of the pair evaluation over a list of
// candidates: flops[0] = projection + clip + cleanup of every candidate (the
// candidate test pass), flops[1] = full evaluation (clip + integration) of
// every candidate that is a pair, flops[2] = reverse-mode adjoint flops of
// those pairs by the standard cost model (adjoint of an add or subtract: 2
// flops, multiply: 4, divide: 4, square root: 3) over every operation outside
// the inverse bilinear maps, flops[3] = number of inverse bilinear maps
// evaluated (each differentiated by the implicit-function theorem instead of
// through its iterations), flops[4] = the cost model applied to the
// candidate pass (frame, projection, clip, cleanup) of those pairs alone.
void or_count_flops(int64_t ns_nodes, const double* Xs, int64_t ns_el, const int32_t* Cs,
                    int64_t nm_nodes, const double* Xm, int64_t nm_el, const int32_t* Cm,
                    const OrParams* op, int64_t n, const int32_t* cs, const int32_t* cm, uint64_t* flops) {
  MeshView S{ns_nodes, Xs, ns_el, Cs}, M{nm_nodes, Xm, nm_el, Cm};
  const Params prm = to_params(op);
  const Rule rule = make_rule(prm.rule);
  for (int k = 0; k < 5; ++k) flops[k] = 0;
  for (int64_t i = 0; i < n; ++i) {
    Cnt xs[4][3], xm[4][3];
    load_pair(S, M, cs[i], cm[i], xs, xm);
    PairOut<Cnt> o;
    g_flops = 0;
    for (int k = 0; k < 4; ++k) g_kind[k] = 0;
    eval_pair(xs, xm, prm, rule, false, o);
    flops[0] += g_flops;
    if (o.nv >= 3) {
      flops[4] += 2 * g_kind[0] + 4 * g_kind[1] + 4 * g_kind[2] + 3 * g_kind[3];
      g_flops = 0;
      for (int k = 0; k < 4; ++k) g_kind[k] = 0;
      g_inverse_maps = 0;
      eval_pair(xs, xm, prm, rule, true, o);
      flops[1] += g_flops;
      flops[2] += 2 * g_kind[0] + 4 * g_kind[1] + 4 * g_kind[2] + 3 * g_kind[3];
      flops[3] += g_inverse_maps;
    }
  }
}

}  // extern "C"
