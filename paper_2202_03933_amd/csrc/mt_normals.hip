// Continuous normal field of the slave side and its linearisation.  The
// paper bases the projections between the two sides on a continuous field of
// slave normals (Sec. "Discretization") without defining it; here the nodal
// normal n_a is the normalised sum of the unit corner normals of the elements
// around node a (ascending element order), and an element's auxiliary plane
// normal is the normalised sum of its four nodal normals (node order).  Every
// sum runs in that fixed order without fused multiply-add, so the planes, and
// with them the clip topology, are reproducible bit for bit.
//
// Backward: the pair kernels leave dL/dn0 per pair; the chain runs
// element (sum over its pairs, normalisation) -> node (sum over its elements,
// normalisation) -> element corners (cross product of the two edges) -> node
// coordinates, each stage one thread per owner, summing in a fixed order.
#include "mt_geometry.h"
#include "mt_internal.h"

namespace mt {

namespace {

constexpr int BSN = 256;

// Unit normal of element e at its corner k and the length it was normalised
// from; e1, e2 are the edges to the next and to the previous node.
__device__ __forceinline__ void corner_normal(const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, int4 c, int k, double e1[3],
                                              double e2[3], double v[3], double& l) {
  const int nd[4] = {c.x, c.y, c.z, c.w};
  const int a = nd[k], b = nd[(k + 1) & 3], p = nd[(k + 3) & 3];
  e1[0] = x[b] - x[a];
  e1[1] = y[b] - y[a];
  e1[2] = z[b] - z[a];
  e2[0] = x[p] - x[a];
  e2[1] = y[p] - y[a];
  e2[2] = z[p] - z[a];
  const double cx = e1[1] * e2[2] - e1[2] * e2[1];
  const double cy = e1[2] * e2[0] - e1[0] * e2[2];
  const double cz = e1[0] * e2[1] - e1[1] * e2[0];
  l = sqrt((cx * cx + cy * cy) + cz * cz);
  v[0] = cx / l;
  v[1] = cy / l;
  v[2] = cz / l;
}

__global__ __launch_bounds__(BSN) void k_node_normals(const double* __restrict__ x, const double* __restrict__ y,
                                                      const double* __restrict__ z, const int32_t* __restrict__ conn,
                                                      const int32_t* __restrict__ inc_off,
                                                      const int32_t* __restrict__ inc_list, int32_t n_nodes,
                                                      double* __restrict__ nn) {
  const int a = blockIdx.x * BSN + threadIdx.x;
  if (a >= n_nodes) return;
  double u[3] = {0.0, 0.0, 0.0};
  for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
    const int e = inc_list[i] >> 2, k = inc_list[i] & 3;
    double e1[3], e2[3], v[3], l;
    corner_normal(x, y, z, load_conn(conn, e), k, e1, e2, v, l);
    u[0] = u[0] + v[0];
    u[1] = u[1] + v[1];
    u[2] = u[2] + v[2];
  }
  const double l = sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  double4 o;
  o.x = l > 0.0 ? u[0] / l : u[0];
  o.y = l > 0.0 ? u[1] / l : u[1];
  o.z = l > 0.0 ? u[2] / l : u[2];
  o.w = l;
  reinterpret_cast<double4*>(nn)[a] = o;
}

__global__ __launch_bounds__(BSN) void k_elem_normals(const int32_t* __restrict__ conn, int32_t n_el,
                                                      const double* __restrict__ nn, double* __restrict__ ne) {
  const int e = blockIdx.x * BSN + threadIdx.x;
  if (e >= n_el) return;
  const int4 c = load_conn(conn, e);
  const double4* N = reinterpret_cast<const double4*>(nn);
  const double4 a = N[c.x], b = N[c.y], d = N[c.z], f = N[c.w];
  const double vx = ((a.x + b.x) + d.x) + f.x;
  const double vy = ((a.y + b.y) + d.y) + f.y;
  const double vz = ((a.z + b.z) + d.z) + f.z;
  const double l = sqrt((vx * vx + vy * vy) + vz * vz);
  reinterpret_cast<double4*>(ne)[e] = make_double4(vx / l, vy / l, vz / l, l);
}

// dL/ds of s = sum of the element's four nodal normals, from dL/dn0 of its
// pairs (pairs of element e: pair_off[e] .. pair_off[e + 1], in order).
__global__ __launch_bounds__(BSN) void k_elem_normal_adj(int32_t n_el, const int32_t* __restrict__ pair_off,
                                                         const double* __restrict__ gn0, int64_t stride,
                                                         const double* __restrict__ ne, double* __restrict__ sb) {
  const int e = blockIdx.x * BSN + threadIdx.x;
  if (e >= n_el) return;
  double g[3] = {0.0, 0.0, 0.0};
  for (int p = pair_off[e]; p < pair_off[e + 1]; ++p) {
    g[0] += gn0[p];
    g[1] += gn0[stride + p];
    g[2] += gn0[2 * stride + p];
  }
  const double4 n = reinterpret_cast<const double4*>(ne)[e];
  const double ng = n.x * g[0] + n.y * g[1] + n.z * g[2];
  const double r = 1.0 / n.w;
  reinterpret_cast<double4*>(sb)[e] =
      make_double4((g[0] - n.x * ng) * r, (g[1] - n.y * ng) * r, (g[2] - n.z * ng) * r, 0.0);
}

// dL/du of u = the sum of the corner normals at node a (before normalising).
__global__ __launch_bounds__(BSN) void k_node_normal_adj(int32_t n_nodes, const int32_t* __restrict__ inc_off,
                                                         const int32_t* __restrict__ inc_list,
                                                         const double* __restrict__ sb, const double* __restrict__ nn,
                                                         double* __restrict__ ub) {
  const int a = blockIdx.x * BSN + threadIdx.x;
  if (a >= n_nodes) return;
  double g[3] = {0.0, 0.0, 0.0};
  const double4* SB = reinterpret_cast<const double4*>(sb);
  for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
    const double4 v = SB[inc_list[i] >> 2];
    g[0] += v.x;
    g[1] += v.y;
    g[2] += v.z;
  }
  const double4 n = reinterpret_cast<const double4*>(nn)[a];
  const double ng = n.x * g[0] + n.y * g[1] + n.z * g[2];
  const double r = n.w > 0.0 ? 1.0 / n.w : 0.0;
  reinterpret_cast<double4*>(ub)[a] =
      make_double4((g[0] - n.x * ng) * r, (g[1] - n.y * ng) * r, (g[2] - n.z * ng) * r, 0.0);
}

// Per element: the coordinate gradient of its four corner normals, given
// dL/du of the nodes they were added to; cg[(3 j + d) * n_el + e] for local
// node j.  With S_at the coordinate arrays are read from device memory (see
// k_corner_gather).
__global__ __launch_bounds__(BSN) void k_corner_adj(const double* x, const double* y, const double* z,
                                                    const int32_t* __restrict__ conn, int32_t n_el,
                                                    const double* __restrict__ ub, double* __restrict__ cg,
                                                    const MeshPtrs* S_at) {
  const int e = blockIdx.x * BSN + threadIdx.x;
  if (e >= n_el) return;
  if (S_at) {
    x = S_at->x;
    y = S_at->y;
    z = S_at->z;
  }
  const int4 c = load_conn(conn, e);
  const int nd[4] = {c.x, c.y, c.z, c.w};
  double G[4][3];
#pragma unroll
  for (int j = 0; j < 4; ++j) G[j][0] = G[j][1] = G[j][2] = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double e1[3], e2[3], v[3], l;
    corner_normal(x, y, z, c, k, e1, e2, v, l);
    const double4 u = reinterpret_cast<const double4*>(ub)[nd[k]];
    const double vu = v[0] * u.x + v[1] * u.y + v[2] * u.z;
    const double r = 1.0 / l;
    const double cb[3] = {(u.x - v[0] * vu) * r, (u.y - v[1] * vu) * r, (u.z - v[2] * vu) * r};
    // c = e1 x e2: e1b = e2 x cb, e2b = cb x e1
    const double a1[3] = {e2[1] * cb[2] - e2[2] * cb[1], e2[2] * cb[0] - e2[0] * cb[2], e2[0] * cb[1] - e2[1] * cb[0]};
    const double a2[3] = {cb[1] * e1[2] - cb[2] * e1[1], cb[2] * e1[0] - cb[0] * e1[2], cb[0] * e1[1] - cb[1] * e1[0]};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      G[(k + 1) & 3][d] += a1[d];
      G[(k + 3) & 3][d] += a2[d];
      G[k][d] -= a1[d] + a2[d];
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int d = 0; d < 3; ++d) cg[(int64_t)(3 * j + d) * n_el + e] = G[j][d];
}

// gX[d * n + a] += sum over the elements around node a of their corner
// gradients at a.  With gX_at, the output pointer is read from device
// memory (a launch recorded in a graph then follows a table updated per call).
__global__ __launch_bounds__(BSN) void k_corner_gather(int32_t n_nodes, const int32_t* __restrict__ inc_off,
                                                       const int32_t* __restrict__ inc_list, int32_t n_el,
                                                       const double* __restrict__ cg, double* gX,
                                                       double* const* gX_at) {
  const int a = blockIdx.x * BSN + threadIdx.x;
  if (a >= n_nodes) return;
  if (gX_at) gX = *gX_at;
  double g[3] = {0.0, 0.0, 0.0};
  for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
    const int e = inc_list[i] >> 2, j = inc_list[i] & 3;
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] += cg[(int64_t)(3 * j + d) * n_el + e];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) gX[(int64_t)d * n_nodes + a] += g[d];
}

unsigned blocks(int64_t n) { return (unsigned)((n + BSN - 1) / BSN); }

}  // namespace

hipError_t launch_normals(const DeviceMesh& S, const int32_t* inc_off, const int32_t* inc_list, double* nn,
                          double* ne, hipStream_t s) {
  if (S.n_nodes > 0)
    k_node_normals<<<blocks(S.n_nodes), BSN, 0, s>>>(S.x, S.y, S.z, S.conn, inc_off, inc_list, S.n_nodes, nn);
  if (S.n_el > 0) k_elem_normals<<<blocks(S.n_el), BSN, 0, s>>>(S.conn, S.n_el, nn, ne);
  return hipGetLastError();
}

hipError_t launch_normal_chain(const DeviceMesh& S, const int32_t* inc_off, const int32_t* inc_list,
                               const int32_t* pair_off, const double* gn0, int64_t stride, const double* nn,
                               const double* ne, double* sb, double* ub, double* cg, double* gX,
                               double* const* gX_at, const MeshPtrs* S_at, hipStream_t s) {
  if (S.n_el == 0) return hipSuccess;
  k_elem_normal_adj<<<blocks(S.n_el), BSN, 0, s>>>(S.n_el, pair_off, gn0, stride, ne, sb);
  k_node_normal_adj<<<blocks(S.n_nodes), BSN, 0, s>>>(S.n_nodes, inc_off, inc_list, sb, nn, ub);
  k_corner_adj<<<blocks(S.n_el), BSN, 0, s>>>(S.x, S.y, S.z, S.conn, S.n_el, ub, cg, S_at);
  k_corner_gather<<<blocks(S.n_nodes), BSN, 0, s>>>(S.n_nodes, inc_off, inc_list, S.n_el, cg, gX, gX_at);
  return hipGetLastError();
}

}  // namespace mt
