// Contact search on the GPU: element preparation, Cartesian bins sorted by
// radix sort with bin ranges from segment heads, and the candidate lists of
// every slave element from its own bin and the 26 neighbouring bins
// (Alg. 2 and the bin-sizing rule of Sec. "Geometrically motivated binning").
#include <cmath>
#include <cstring>

#include "mt_geometry.h"
#include "mt_internal.h"

namespace mt {

namespace {

constexpr int BS = 256;

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

__global__ __launch_bounds__(BS) void k_prep(const double* __restrict__ x, const double* __restrict__ y,
                                              const double* __restrict__ z, const int32_t* __restrict__ conn,
                                              int32_t n_el, int32_t n_nodes, int slave,
                                              double* __restrict__ box, PrepReduce* red) {
  const int e = blockIdx.x * BS + threadIdx.x;
  const bool live = e < n_el;
  double ext = 0.0, edge = 0.0;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (live) {
    const int4 c = load_conn(conn, e);
    const bool ok = c.x >= 0 && c.y >= 0 && c.z >= 0 && c.w >= 0 && c.x < n_nodes && c.y < n_nodes &&
                    c.z < n_nodes && c.w < n_nodes;
    if (!ok) {
      atomicOr(&red->bad_index, 1);
    } else {
      double X[4][3];
      load_nodes(x, y, z, c, X);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(fmin(X[0][d], X[1][d]), fmin(X[2][d], X[3][d]));
        hi[d] = fmax(fmax(X[0][d], X[1][d]), fmax(X[2][d], X[3][d]));
        box[(int64_t)d * n_el + e] = lo[d];
        box[(int64_t)(3 + d) * n_el + e] = hi[d];
        ext = fmax(ext, hi[d] - lo[d]);
      }
      if (slave) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int k1 = (k + 1) & 3;
          const double a = X[k1][0] - X[k][0], b = X[k1][1] - X[k][1], cc = X[k1][2] - X[k][2];
          edge = fmax(edge, sqrt(a * a + b * b + cc * cc));
        }
      }
    }
  }
  ext = wave_max(ext);
  edge = wave_max(edge);
  double l3[3], h3[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    l3[d] = wave_min(lo[d]);
    h3[d] = wave_max(hi[d]);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&red->emax_bits, (unsigned long long)__double_as_longlong(ext));
    if (slave) atomicMax(&red->edge_bits, (unsigned long long)__double_as_longlong(edge));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (l3[d] <= h3[d]) {
        atomicMin(&red->lo_key[d], order_key(l3[d]));
        atomicMax(&red->hi_key[d], order_key(h3[d]));
      }
    }
  }
}

__global__ void k_init_reduce(PrepReduce* r) {
  r->emax_bits = 0;
  r->edge_bits = 0;
  for (int d = 0; d < 3; ++d) {
    r->lo_key[d] = ~0ull;
    r->hi_key[d] = 0ull;
  }
  r->bad_index = 0;
  r->pad = 0;
}

__device__ __forceinline__ int cell_coord(double c, double lo, double inv_beta, int n) {
  int i = (int)floor((c - lo) * inv_beta);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__global__ __launch_bounds__(BS) void k_master_keys(const double* __restrict__ box, int32_t n, Grid g,
                                                     uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int m = blockIdx.x * BS + threadIdx.x;
  if (m >= n) return;
  int ix[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double c = 0.5 * (box[(int64_t)d * n + m] + box[(int64_t)(3 + d) * n + m]);
    ix[d] = cell_coord(c, g.lo[d], g.inv_beta[d], g.n[d]);
  }
  keys[m] = (uint32_t)(ix[0] + g.n[0] * (ix[1] + g.n[1] * ix[2]));
  vals[m] = (uint32_t)m;
}

__global__ __launch_bounds__(BS) void k_cell_ranges(const uint32_t* __restrict__ keys, int32_t n,
                                                     int32_t* __restrict__ start, int32_t* __restrict__ end) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i];
  if (i == 0 || keys[i - 1] != k) start[k] = i;
  if (i == n - 1 || keys[i + 1] != k) end[k] = i + 1;
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
// master box on all three axes.
__device__ __forceinline__ bool touch(const SlaveBox& s, const double* __restrict__ box_m, int32_t n_m, int m,
                                      double delta) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double mlo = box_m[(int64_t)d * n_m + m];
    const double mhi = box_m[(int64_t)(3 + d) * n_m + m];
    if (!((s.lo[d] - delta) <= mhi && mlo <= (s.hi[d] + delta))) return false;
  }
  return true;
}

template <bool FILL>
__global__ __launch_bounds__(BS) void k_cand(const double* __restrict__ box_s, int32_t n_s,
                                              const double* __restrict__ box_m, int32_t n_m,
                                              const uint32_t* __restrict__ mvals, const int32_t* __restrict__ start,
                                              const int32_t* __restrict__ end, Grid g, double delta,
                                              int32_t* __restrict__ count, const int32_t* __restrict__ off,
                                              int32_t* __restrict__ cand_s, int32_t* __restrict__ cand_m) {
  const int s = blockIdx.x * BS + threadIdx.x;
  if (s >= n_s) return;
  const SlaveBox b = load_box(box_s, n_s, s);
  int ix[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) ix[d] = cell_coord(0.5 * (b.lo[d] + b.hi[d]), g.lo[d], g.inv_beta[d], g.n[d]);
  int c = 0;
  const int base = FILL ? off[s] : 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = ix[2] + dz;
    if (zz < 0 || zz >= g.n[2]) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = ix[1] + dy;
      if (yy < 0 || yy >= g.n[1]) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = ix[0] + dx;
        if (xx < 0 || xx >= g.n[0]) continue;
        const int64_t cell = xx + (int64_t)g.n[0] * (yy + (int64_t)g.n[1] * zz);
        const int i1 = end[cell];
        for (int i = start[cell]; i < i1; ++i) {
          const int m = (int)mvals[i];
          if (touch(b, box_m, n_m, m, delta)) {
            if (FILL) cand_m[base + c] = m;
            ++c;
          }
        }
      }
    }
  }
  if (!FILL) {
    count[s] = c;
    return;
  }
  // insertion sort of this slave's candidates by master index
  for (int i = 1; i < c; ++i) {
    const int v = cand_m[base + i];
    int j = i - 1;
    while (j >= 0 && cand_m[base + j] > v) {
      cand_m[base + j + 1] = cand_m[base + j];
      --j;
    }
    cand_m[base + j + 1] = v;
  }
  for (int i = 0; i < c; ++i) cand_s[base + i] = s;
}

}  // namespace

hipError_t launch_init_reduce(PrepReduce* red, hipStream_t s) {
  k_init_reduce<<<1, 1, 0, s>>>(red);
  return hipGetLastError();
}

hipError_t launch_prep(const DeviceMesh& m, bool slave, double* box, PrepReduce* red, hipStream_t s) {
  if (m.n_el == 0) return hipSuccess;
  k_prep<<<(m.n_el + BS - 1) / BS, BS, 0, s>>>(m.x, m.y, m.z, m.conn, m.n_el, m.n_nodes, slave ? 1 : 0, box, red);
  return hipGetLastError();
}

void grid_from_reduce(const PrepReduce& r, double delta, double bin_size, Grid& g) {
  double emax, edge;
  std::memcpy(&emax, &r.emax_bits, sizeof(double));
  std::memcpy(&edge, &r.edge_bits, sizeof(double));
  double beta_min = std::fmax(std::fmax(edge, emax + delta), bin_size) * (1.0 + std::ldexp(1.0, -20));
  if (!(beta_min > 0.0) || !std::isfinite(beta_min)) beta_min = 1.0;
  double L[3];
  int64_t n[3];
  for (int d = 0; d < 3; ++d) {
    double lo = from_order_key(r.lo_key[d]);
    double hi = from_order_key(r.hi_key[d]);
    if (!(lo <= hi)) { lo = 0.0; hi = 0.0; }
    g.lo[d] = lo - beta_min;
    L[d] = (hi + beta_min) - g.lo[d];
    n[d] = std::max<int64_t>(1, (int64_t)std::floor(L[d] / beta_min));
  }
  // Bound the dense cell table; coarser cells keep the search complete.
  const int64_t cap = int64_t(1) << 24;
  while (n[0] * n[1] * n[2] > cap) {
    const double f = std::cbrt((double)(n[0] * n[1] * n[2]) / (double)cap) * 1.01;
    for (int d = 0; d < 3; ++d) n[d] = std::max<int64_t>(1, (int64_t)std::floor((double)n[d] / f));
  }
  for (int d = 0; d < 3; ++d) {
    g.n[d] = (int32_t)n[d];
    g.beta[d] = L[d] / (double)n[d];
    g.inv_beta[d] = 1.0 / g.beta[d];
  }
  g.ncells = n[0] * n[1] * n[2];
}

hipError_t launch_master_keys(const double* box_m, int32_t n_m, Grid g, uint32_t* keys, uint32_t* vals,
                              hipStream_t s) {
  if (n_m == 0) return hipSuccess;
  k_master_keys<<<(n_m + BS - 1) / BS, BS, 0, s>>>(box_m, n_m, g, keys, vals);
  return hipGetLastError();
}

hipError_t launch_cell_ranges(const uint32_t* keys, int32_t n, int32_t* start, int32_t* end, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_cell_ranges<<<(n + BS - 1) / BS, BS, 0, s>>>(keys, n, start, end);
  return hipGetLastError();
}

hipError_t launch_cand_count(const double* box_s, int32_t n_s, const double* box_m, int32_t n_m,
                             const uint32_t* mvals, const int32_t* start, const int32_t* end, Grid g,
                             double delta, int32_t* count, hipStream_t s) {
  if (n_s == 0) return hipSuccess;
  k_cand<false><<<(n_s + BS - 1) / BS, BS, 0, s>>>(box_s, n_s, box_m, n_m, mvals, start, end, g, delta, count,
                                                   nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_cand_fill(const double* box_s, int32_t n_s, const double* box_m, int32_t n_m,
                            const uint32_t* mvals, const int32_t* start, const int32_t* end, Grid g,
                            double delta, const int32_t* off, int32_t* cand_s, int32_t* cand_m, hipStream_t s) {
  if (n_s == 0) return hipSuccess;
  k_cand<true><<<(n_s + BS - 1) / BS, BS, 0, s>>>(box_s, n_s, box_m, n_m, mvals, start, end, g, delta, nullptr,
                                                  off, cand_s, cand_m);
  return hipGetLastError();
}

}  // namespace mt
