// Element-based integration, the alternative to the segments of Alg. 1 that
// Sec. "Evaluation of mortar integrals" names: no clipping or triangulation,
// an ng x ng Gauss-Legendre product rule on each whole slave element, in the
// parameter space of its projected quad (measure: area in the auxiliary
// plane, the measure of the segment integrals).  A rule point belongs to the
// first pair of its slave element (ascending master) whose counter-clockwise
// projected master quad contains it: inside the quad's closed bounding box
// and by the clip's side test on the closed half-planes of its four edges;
// points in no master are dropped.
// Integrands are those of the segment-based blocks.
//
// One thread per pair integrates the rule points of its slave element that
// its master takes and writes its blocks blk[c * stride + p] for the
// assembly.
#include <cmath>
#include <mutex>

#include "mt_pair_eval.h"

namespace mt {

namespace {

constexpr int BSE = 64;

struct GaussTab {
  double x[8];
  double w[8];
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Inverse bilinear map of p on one quad by Newton's method from xi = 0 (the
// first step from the precomputed Jacobian at 0); at most maxit steps.
__device__ __forceinline__ void inverse1(const QMap& B, double pu, double pv, double tol, int maxit, double& b1,
                                         double& b2, unsigned& noconv) {
#pragma clang fp contract(fast)
  const double dbu = pu - B.cu, dbv = pv - B.cv;
  b1 = (B.e2v * dbu - B.e2u * dbv) * B.r0;
  b2 = (B.e1u * dbv - B.e1v * dbu) * B.r0;
  bool cb = false;
  for (int it = 1; it < maxit && !cb; ++it) newton_step(B, dbu, dbv, tol, b1, b2, cb);
  noconv += cb ? 0u : 1u;
}

// Rule point of the auxiliary plane at (x1, x2): the bilinear map of the
// projected slave quad in monomial form ((c + e1 x1) + e2 x2) + f (x1 x2),
// evaluated in this order without fused multiply-add (P decides which
// master takes the point).
__device__ __forceinline__ V2 rule_point(const QMap& ms, double x1, double x2) {
  const double x12 = x1 * x2;
  V2 P;
  P.u = ((ms.cu + ms.e1u * x1) + ms.e2u * x2) + ms.fu * x12;
  P.v = ((ms.cv + ms.e1v * x1) + ms.e2v * x2) + ms.fv * x12;
  return P;
}

// Closed containment in a counter-clockwise quad: inside its bounding box and
// on the inner side of its four edges (the clip's side test).
struct OQuad {
  V2 q[4];
  double lu, hu, lv, hv;
};

__device__ __forceinline__ OQuad oquad(const V2 Mo[4]) {
  OQuad o;
#pragma unroll
  for (int k = 0; k < 4; ++k) o.q[k] = Mo[k];
  o.lu = fmin(fmin(Mo[0].u, Mo[1].u), fmin(Mo[2].u, Mo[3].u));
  o.hu = fmax(fmax(Mo[0].u, Mo[1].u), fmax(Mo[2].u, Mo[3].u));
  o.lv = fmin(fmin(Mo[0].v, Mo[1].v), fmin(Mo[2].v, Mo[3].v));
  o.hv = fmax(fmax(Mo[0].v, Mo[1].v), fmax(Mo[2].v, Mo[3].v));
  return o;
}

__device__ __forceinline__ bool in_box(const OQuad& o, V2 P) {
  return !(P.u < o.lu || P.u > o.hu || P.v < o.lv || P.v > o.hv);
}

__device__ __forceinline__ bool in_edges(const V2 Mo[4], V2 P) {
  bool in = true;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const V2 a = Mo[l], b = Mo[(l + 1) & 3];
    const double c = (b.u - a.u) * (P.v - a.v) - (b.v - a.v) * (P.u - a.u);
    in = in && (c >= 0.0);
  }
  return in;
}

// Oriented (counter-clockwise) projected master quad of master element m on
// the slave plane f; Mn keeps the node order.
__device__ __forceinline__ void master_quad(const MeshPtrs& M, int m, const double f[12], V2 Mo[4], V2 Mn[4]) {
  double Xm[4][3], hm[4];
  load_nodes(M.x, M.y, M.z, load_conn(M.conn, m), Xm);
#pragma unroll
  for (int k = 0; k < 4; ++k) project(Xm[k], f, Mn[k], hm[k]);
  const bool flip = quad_fan_area(Mn) < 0.0;
  Mo[0] = Mn[0];
  Mo[1] = flip ? Mn[3] : Mn[1];
  Mo[2] = Mn[2];
  Mo[3] = flip ? Mn[1] : Mn[3];
}

// One thread per pair p of slave element s.  A rule point of s inside p's
// master is integrated by p unless the master of an earlier pair of s
// (pair_off[s] .. p - 1) contains it too; the oriented master quads of the
// block's pairs are shared through LDS, those of earlier pairs outside the
// block are recomputed.
template <bool DUAL>
__global__ __launch_bounds__(BSE) __attribute__((amdgpu_waves_per_eu(3))) void k_elem_fwd(
    MeshPtrs S, MeshPtrs M, KParams kp, GaussTab gt, const int32_t* __restrict__ pair_s,
    const int32_t* __restrict__ pair_m, const int32_t* __restrict__ pair_off, const int32_t* __restrict__ n_dev,
    double* __restrict__ blk, int64_t stride, Counters* cnt) {
  __shared__ double sq[8][BSE];
  __shared__ double sg[8], sw[8];
  const int64_t n_pairs = *n_dev;
  const int64_t tile = dyn_tile(blockIdx.x, n_pairs, BSE);
  if (tile < 0) return;  // the whole block
  if (threadIdx.x < 8) {
    sg[threadIdx.x] = gt.x[threadIdx.x];
    sw[threadIdx.x] = gt.w[threadIdx.x];
  }
  const int64_t base = tile * BSE;
  const int64_t p = base + threadIdx.x;
  const bool valid = p < n_pairs;
  const int s = valid ? pair_s[p] : 0;
  QMap ms, mm;
  V2 Mo[4];
  if (valid) {
    double Xs[4][3], f[12];
    load_nodes(S.x, S.y, S.z, load_conn(S.conn, s), Xs);
    slave_frame_p(Xs, elem_nrm(S, s), f);
    V2 Sp[4], Mn[4];
    double hs[4], As, hmax;
    slave_setup(Xs, f, Sp, hs, As, hmax);
    ms = qmap(Sp);
    master_quad(M, pair_m[p], f, Mo, Mn);
    mm = qmap(Mn);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sq[2 * k][threadIdx.x] = Mo[k].u;
      sq[2 * k + 1][threadIdx.x] = Mo[k].v;
    }
  }
  __syncthreads();
  unsigned noconv = 0;
  if (valid) {
    const int pfirst = pair_off[s];
    const OQuad own = oquad(Mo);
    // det J of the slave map is linear in xi: d0 + d1 xi1 + d2 xi2
    double d0, d1, d2;
    {
#pragma clang fp contract(fast)
      d0 = ms.e1u * ms.e2v - ms.e2u * ms.e1v;
      d1 = ms.e1u * ms.fv - ms.fu * ms.e1v;
      d2 = ms.fu * ms.e2v - ms.e2u * ms.fv;
    }
    double mu[9], Mm[16];
#pragma unroll
    for (int k = 0; k < 9; ++k) mu[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) Mm[k] = 0.0;
    const int ng = kp.elem, nq = ng * ng;
    // points inside the own master (a loop uniform over the wave)
    unsigned long long mine = 0ull;
#pragma unroll 1
    for (int q = 0; q < nq; ++q) {
      const V2 P = rule_point(ms, gt.x[q % ng], gt.x[q / ng]);
      if (in_box(own, P) && in_edges(own.q, P)) mine |= 1ull << q;
    }
    // each lane walks its own points: the wave runs as many iterations as
    // its busiest lane has points, every active lane on a point of its own
#pragma unroll 1
    while (mine) {
      const int q = __builtin_ctzll(mine);
      mine &= mine - 1ull;
      const int a = q % ng, b = q / ng;
      const double x1 = sg[a], x2 = sg[b];
      const V2 P = rule_point(ms, x1, x2);
      bool earlier = false;
#pragma unroll 1
      for (int pp = pfirst; pp < (int)p && !earlier; ++pp) {
        V2 Eo[4];
        if (pp >= base) {
          const int t = pp - (int)base;
#pragma unroll
          for (int k = 0; k < 4; ++k) Eo[k] = V2{sq[2 * k][t], sq[2 * k + 1][t]};
        } else {
          // earlier pair outside the block: its quad from reloaded nodes
          double Xs2[4][3], f2[12];
          const int s2 = launder(s);
          load_nodes(S.x, S.y, S.z, load_conn(S.conn, s2), Xs2);
          slave_frame_p(Xs2, elem_nrm(S, s2), f2);
          V2 En[4];
          master_quad(M, pair_m[pp], f2, Eo, En);
        }
        earlier = in_box(oquad(Eo), P) && in_edges(Eo, P);
      }
      if (earlier) continue;
      double y1, y2;
      inverse1(mm, P.u, P.v, kp.newton_tol, kp.newton_maxit, y1, y2, noconv);
      {
#pragma clang fp contract(fast)
        const double wJ = (sw[a] * sw[b]) * (d0 + d1 * x1 + d2 * x2);
        const double t[4] = {wJ, wJ * x1, wJ * x2, wJ * x1 * x2};
        mu[0] += t[0];
        mu[1] += t[1];
        mu[2] += t[2];
        mu[3] += t[3];
        mu[4] += t[1] * x1;
        mu[5] += t[2] * x2;
        mu[6] += t[3] * x1;
        mu[7] += t[3] * x2;
        mu[8] += t[3] * (x1 * x2);
        const double y12 = y1 * y2;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          Mm[4 * r] += t[r];
          Mm[4 * r + 1] += t[r] * y1;
          Mm[4 * r + 2] += t[r] * y2;
          Mm[4 * r + 3] += t[r] * y12;
        }
      }
    }
    // heights from reloaded nodes rather than kept through the loop
    double D[16], Mv[16], g[4];
    {
      const int s2 = launder(s);
      const int4 cs = load_conn(S.conn, s2);
      const int4 cm = load_conn(M.conn, launder(pair_m[p]));
      double Xs2[4][3], Xm2[4][3], f2[12];
      load_nodes(S.x, S.y, S.z, cs, Xs2);
      load_nodes(M.x, M.y, M.z, cm, Xm2);
      slave_frame_p(Xs2, elem_nrm(S, s2), f2);
      V2 S2[4], M2[4];
      double hs[4], hm[4];
      pair_project(Xs2, Xm2, f2, S2, M2, hs, hm);
      moments_to_blocks<DUAL>(qmap(S2), mu, Mm, hs, hm, D, Mv, g);
    }
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

// Gauss-Legendre rule with n points on [-1, 1], ascending: the positive roots
// of the Legendre polynomial P_n by Newton's method from Tricomi's estimate
// (1 - 1/(8 n^2) + 1/(8 n^3)) cos(pi (4 i + 3) / (4 n + 2)), with P_n and
// P_n' = n (P_{n-1} - x P_n) / (1 - x^2) from Bonnet's recurrence; the
// negative roots by symmetry, 0 for odd n; weights 2 / ((1 - x^2) P_n'^2).
void gauss_table(int n, GaussTab& t) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < 8; ++i) t.x[i] = t.w[i] = 0.0;
  auto eval = [n](double x, double& pn, double& dpn) {
    double pm1 = 1.0, pk = x;  // P_0, P_1
    for (int k = 2; k <= n; ++k) {
      const double pk1 = ((2 * k - 1) * x * pk - (k - 1) * pm1) / k;
      pm1 = pk;
      pk = pk1;
    }
    pn = pk;
    dpn = n * (pm1 - x * pk) / (1.0 - x * x);
  };
  for (int i = 0; i < n / 2; ++i) {
    // i-th root from the top
    double x = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) * std::cos(pi * (4 * i + 3) / (4 * n + 2));
    double pn, dpn;
    for (int it = 0; it < 60; ++it) {
      eval(x, pn, dpn);
      const double dx = pn / dpn;
      x -= dx;
      if (std::fabs(dx) <= 1e-16) break;
    }
    eval(x, pn, dpn);
    const double w = 2.0 / ((1.0 - x * x) * dpn * dpn);
    t.x[n - 1 - i] = x;
    t.w[n - 1 - i] = w;
    t.x[i] = -x;
    t.w[i] = w;
  }
  if (n % 2 == 1) {
    double pn, dpn;
    eval(0.0, pn, dpn);
    t.x[n / 2] = 0.0;
    t.w[n / 2] = 2.0 / (dpn * dpn);
  }
}

}  // namespace

hipError_t launch_elem_fwd(const DeviceMesh& S, const DeviceMesh& M, const KParams& kp, const int32_t* pair_s,
                           const int32_t* pair_m, const int32_t* pair_off, const int32_t* n_pairs, int64_t cap,
                           double* blk, int64_t stride, Counters* cnt, hipStream_t s) {
  if (cap == 0) return hipSuccess;
  if (kp.elem < 1 || kp.elem > 8) return hipErrorInvalidValue;
  static GaussTab tabs[9];
  static std::once_flag once;
  std::call_once(once, [] {
    for (int n = 1; n <= 8; ++n) gauss_table(n, tabs[n]);
  });
  const MeshPtrs ms{S.x, S.y, S.z, S.conn, S.nrm}, mm{M.x, M.y, M.z, M.conn, nullptr};
  const unsigned nb = xcd_grid((unsigned)((cap + BSE - 1) / BSE));
  if (kp.dual)
    k_elem_fwd<true><<<nb, BSE, 0, s>>>(ms, mm, kp, tabs[kp.elem], pair_s, pair_m, pair_off, n_pairs, blk, stride, cnt);
  else
    k_elem_fwd<false><<<nb, BSE, 0, s>>>(ms, mm, kp, tabs[kp.elem], pair_s, pair_m, pair_off, n_pairs, blk, stride,
                                         cnt);
  return hipGetLastError();
}

}  // namespace mt
