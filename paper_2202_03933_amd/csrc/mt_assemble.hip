// Deterministic assembly of the mortar operators into CSR (the assembly of
// the nodal blocks of eq. (DiscreteWeakFormInterfaceFlux)) and of the nodal
// gradients, with no floating-point atomics: every output row (slave node)
// or gradient entry (node) is owned by one thread that sums its
// contributions in a fixed order (incident elements ascending, then pairs in
// (slave, master) order), so results are bitwise reproducible.
#include "mt_geometry.h"
#include "mt_internal.h"
#include "mt_rows.h"

namespace mt {

namespace {

constexpr int BS = 256;
constexpr int PB = 128;   // block of the pattern kernels
constexpr int PCAP = 32;  // per-thread LDS segment of the pattern kernels (ints)

__global__ __launch_bounds__(BS) void k_inc_count(const int32_t* __restrict__ conn, int32_t n_el, int32_t* cnt) {
  const int e = blockIdx.x * BS + threadIdx.x;
  if (e >= n_el) return;
  const int4 c = reinterpret_cast<const int4*>(conn)[e];
  atomicAdd(&cnt[c.x], 1);
  atomicAdd(&cnt[c.y], 1);
  atomicAdd(&cnt[c.z], 1);
  atomicAdd(&cnt[c.w], 1);
}

__global__ __launch_bounds__(BS) void k_inc_fill(const int32_t* __restrict__ conn, int32_t n_el,
                                                  const int32_t* __restrict__ off, int32_t* cur, int32_t* list) {
  const int e = blockIdx.x * BS + threadIdx.x;
  if (e >= n_el) return;
  const int4 c = reinterpret_cast<const int4*>(conn)[e];
  const int id[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = atomicAdd(&cur[id[j]], 1);
    list[off[id[j]] + k] = e * 4 + j;
  }
}

// Sort each node's incidence list ascending (element, then local index).
__global__ __launch_bounds__(BS) void k_inc_sort(const int32_t* __restrict__ off, int32_t n, int32_t* list) {
  const int a = blockIdx.x * BS + threadIdx.x;
  if (a >= n) return;
  const int b = off[a], e = off[a + 1];
  for (int i = b + 1; i < e; ++i) {
    const int v = list[i];
    int j = i - 1;
    while (j >= b && list[j] > v) {
      list[j + 1] = list[j];
      --j;
    }
    list[j + 1] = v;
  }
}

// Inserts x into the ascending, duplicate-free strided list v[0..u) unless
// it is already there; returns the new length, or -1 when the list holds cap
// entries and x is new.
__device__ __forceinline__ int insert_unique(int32_t* v, int u, int x, int stride, int cap) {
  int j = u - 1;
  while (j >= 0 && v[j * stride] > x) --j;
  if (j >= 0 && v[j * stride] == x) return u;
  if (u == cap) return -1;
  for (int k = u - 1; k > j; --k) v[(k + 1) * stride] = v[k * stride];
  v[(j + 1) * stride] = x;
  return u + 1;
}

// Sorted, duplicate-free columns of row a: for D the nodes of every incident
// slave element that has pairs, for M the master nodes of every pair of
// those elements.
template <bool MCOLS>
__device__ __forceinline__ int row_columns(int a, const int32_t* __restrict__ inc_off,
                                           const int32_t* __restrict__ inc_list,
                                           const int32_t* __restrict__ pair_off,
                                           const int32_t* __restrict__ pair_m, const int32_t* __restrict__ conn_s,
                                           const int32_t* __restrict__ conn_m, int32_t* v, int stride, int cap) {
  int u = 0;
  for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
    const int e = inc_list[i] >> 2;
    const int p0 = pair_off[e], p1 = pair_off[e + 1];
    if (p1 == p0) continue;
    for (int p = MCOLS ? p0 : 0; p < (MCOLS ? p1 : 1); ++p) {
      const int4 q = reinterpret_cast<const int4*>(MCOLS ? conn_m : conn_s)[MCOLS ? pair_m[p] : e];
      u = insert_unique(v, u, q.x, stride, cap);
      if (u >= 0) u = insert_unique(v, u, q.y, stride, cap);
      if (u >= 0) u = insert_unique(v, u, q.z, stride, cap);
      if (u >= 0) u = insert_unique(v, u, q.w, stride, cap);
      if (u < 0) return -1;
    }
  }
  return u;
}

// The same columns without any scratch, for rows that outgrow the LDS
// segment: the u-th column is the smallest candidate above the (u-1)-th, found
// by a pass over all candidates (raw x unique work, for rare long rows).  With
// col the columns are written there.
template <bool MCOLS>
__device__ __forceinline__ int row_columns_scan(int a, const int32_t* __restrict__ inc_off,
                                                const int32_t* __restrict__ inc_list,
                                                const int32_t* __restrict__ pair_off,
                                                const int32_t* __restrict__ pair_m,
                                                const int32_t* __restrict__ conn_s,
                                                const int32_t* __restrict__ conn_m, int32_t* col) {
  int u = 0, prev = -1;
  while (true) {
    int next = 0x7fffffff;
    for (int i = inc_off[a]; i < inc_off[a + 1]; ++i) {
      const int e = inc_list[i] >> 2;
      const int p0 = pair_off[e], p1 = pair_off[e + 1];
      if (p1 == p0) continue;
      for (int p = MCOLS ? p0 : 0; p < (MCOLS ? p1 : 1); ++p) {
        const int4 q = reinterpret_cast<const int4*>(MCOLS ? conn_m : conn_s)[MCOLS ? pair_m[p] : e];
        const int key[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int l = 0; l < 4; ++l) next = key[l] > prev && key[l] < next ? key[l] : next;
      }
    }
    if (next == 0x7fffffff) return u;
    if (col) col[u] = next;
    ++u;
    prev = next;
  }
}

// Sorted, duplicate-free master nodes of the pairs of each slave element
// (the element's contribution to the M rows of its four nodes), in the
// lane-interleaved list elist[k * n_el + e], k < ecnt[e]; ecnt[e] = -1 when
// there are more than EL of them.
constexpr int EL = 16;

__global__ __launch_bounds__(BS) void k_elem_mlist(int32_t n_el, const int32_t* __restrict__ pair_off,
                                                    const int32_t* __restrict__ pair_m,
                                                    const int32_t* __restrict__ conn_m, int32_t* __restrict__ ecnt,
                                                    int32_t* __restrict__ elist) {
  __shared__ int32_t lds[EL * BS];
  const int e = xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
  if (e >= n_el) return;
  int32_t* v = lds + threadIdx.x;
  int u = 0;
  for (int p = pair_off[e]; p < pair_off[e + 1] && u >= 0; ++p) {
    const int4 q = reinterpret_cast<const int4*>(conn_m)[pair_m[p]];
    u = insert_unique(v, u, q.x, BS, EL);
    if (u >= 0) u = insert_unique(v, u, q.y, BS, EL);
    if (u >= 0) u = insert_unique(v, u, q.z, BS, EL);
    if (u >= 0) u = insert_unique(v, u, q.w, BS, EL);
  }
  ecnt[e] = u;
  for (int k = 0; k < u; ++k) elist[(int64_t)k * n_el + e] = v[k * BS];
}

// M row of node a as the merge of the sorted lists of its (at most ROW_RUNS)
// incident elements: the row length, with the first kcap columns written to
// keep[i * n] (lane-interleaved).  Returns -1 (nothing written) when a list
// is missing (ecnt < 0) or the node has more than ROW_RUNS elements.
__device__ __forceinline__ int merge_mrow(int a, int32_t n, const int32_t* __restrict__ inc_off,
                                          const int32_t* __restrict__ inc_list, int32_t n_el,
                                          const int32_t* __restrict__ ecnt, const int32_t* __restrict__ elist,
                                          int32_t* keep, int kcap) {
  constexpr int NONE = 0x7fffffff;
  const int i0 = inc_off[a], ni = inc_off[a + 1] - i0;
  if (ni > ROW_RUNS) return -1;
  int el[ROW_RUNS], len[ROW_RUNS], cur[ROW_RUNS], head[ROW_RUNS];
#pragma unroll
  for (int t = 0; t < ROW_RUNS; ++t) {
    el[t] = t < ni ? inc_list[i0 + t] >> 2 : 0;
    len[t] = t < ni ? ecnt[el[t]] : 0;
  }
#pragma unroll
  for (int t = 0; t < ROW_RUNS; ++t)
    if (len[t] < 0) return -1;
#pragma unroll
  for (int t = 0; t < ROW_RUNS; ++t) {
    cur[t] = 0;
    head[t] = len[t] > 0 ? elist[el[t]] : NONE;
  }
  int u = 0;
  while (true) {
    const int m = min(min(head[0], head[1]), min(head[2], head[3]));
    if (m == NONE) return u;
    if (u < kcap) keep[(int64_t)u * n] = m;
    ++u;
#pragma unroll
    for (int t = 0; t < ROW_RUNS; ++t)
      if (head[t] == m) {
        ++cur[t];
        head[t] = cur[t] < len[t] ? elist[(int64_t)cur[t] * n_el + el[t]] : NONE;
      }
  }
}

// Row patterns of D and M.  Each thread builds its row's sorted column list
// in a lane-interleaved LDS segment of PCAP entries; a row that outgrows it
// is counted, and in the fill pass written, by row_columns_scan.  The count
// pass writes the row lengths and keeps rows of at most KD (D) / KM (M)
// columns in lane-interleaved scratch keep[i * n + a]; the fill pass copies
// those and recomputes the rest.  The CSR positions of the local blocks are
// found afterwards, pair by pair (k_positions).
constexpr int KD = 16;
constexpr int KM = 32;
static_assert(KD <= PCAP && KM <= PCAP, "kept rows fit the LDS segment");

template <bool FILL, bool MCOLS>
__device__ __forceinline__ void pattern_row(int a, int32_t n, int32_t* lds, const int32_t* __restrict__ inc_off,
                                            const int32_t* __restrict__ inc_list,
                                            const int32_t* __restrict__ pair_off,
                                            const int32_t* __restrict__ pair_m,
                                            const int32_t* __restrict__ conn_s,
                                            const int32_t* __restrict__ conn_m, int32_t* cnt,
                                            const int32_t* __restrict__ rowptr, int32_t* colv, int32_t* keep,
                                            int kcap) {
  const int u = row_columns<MCOLS>(a, inc_off, inc_list, pair_off, pair_m, conn_s, conn_m, lds, PB, PCAP);
  if (u >= 0) {
    if (!FILL) {
      cnt[a] = u;
      if (u <= kcap)
        for (int i = 0; i < u; ++i) keep[(int64_t)i * n] = lds[i * PB];
    } else {
      int32_t* col = colv + rowptr[a];
      for (int i = 0; i < u; ++i) col[i] = lds[i * PB];
    }
  } else if (!FILL) {
    cnt[a] = row_columns_scan<MCOLS>(a, inc_off, inc_list, pair_off, pair_m, conn_s, conn_m, nullptr);
  } else {
    row_columns_scan<MCOLS>(a, inc_off, inc_list, pair_off, pair_m, conn_s, conn_m, colv + rowptr[a]);
  }
}

// Kept rows of the fill pass: copied from the lane-interleaved scratch.
__device__ __forceinline__ void kept_row(int a, int32_t n, int u, const int32_t* __restrict__ keep,
                                         const int32_t* __restrict__ rowptr, int32_t* colv) {
  int32_t* col = colv + rowptr[a];
  for (int i = 0; i < u; ++i) col[i] = keep[(int64_t)i * n + a];
}

template <bool FILL>
__global__ __launch_bounds__(PB) void k_pattern_rows(const int32_t* __restrict__ inc_off,
                                                      const int32_t* __restrict__ inc_list, int32_t n,
                                                      const int32_t* __restrict__ pair_off,
                                                      const int32_t* __restrict__ pair_m,
                                                      const int32_t* __restrict__ conn_s,
                                                      const int32_t* __restrict__ conn_m, int32_t* D_cnt,
                                                      int32_t* M_cnt,
                                                      const int32_t* __restrict__ D_rowptr,
                                                      const int32_t* __restrict__ M_rowptr, int32_t* D_col,
                                                      int32_t* M_col, int32_t* keepD, int32_t* keepM, int32_t n_el,
                                                      const int32_t* __restrict__ ecnt,
                                                      const int32_t* __restrict__ elist) {
  __shared__ int32_t lds[PCAP * PB];
  const int a = xcd_tile(blockIdx.x, gridDim.x) * PB + threadIdx.x;
  if (a >= n) return;
  int32_t* seg = lds + threadIdx.x;
  // D row
  if (FILL && D_rowptr[a + 1] - D_rowptr[a] <= KD)
    kept_row(a, n, D_rowptr[a + 1] - D_rowptr[a], keepD, D_rowptr, D_col);
  else
    pattern_row<FILL, false>(a, n, seg, inc_off, inc_list, pair_off, pair_m, conn_s, conn_m, D_cnt, D_rowptr, D_col,
                             keepD + a, KD);
  // M row (count pass: merge of the element lists when they exist)
  if (!FILL && ecnt) {
    const int u = merge_mrow(a, n, inc_off, inc_list, n_el, ecnt, elist, keepM + a, KM);
    if (u >= 0) {
      M_cnt[a] = u;
      return;
    }
  }
  if (FILL && M_rowptr[a + 1] - M_rowptr[a] <= KM)
    kept_row(a, n, M_rowptr[a + 1] - M_rowptr[a], keepM, M_rowptr, M_col);
  else
    pattern_row<FILL, true>(a, n, seg, inc_off, inc_list, pair_off, pair_m, conn_s, conn_m, M_cnt, M_rowptr, M_col,
                            keepM + a, KM);
}

// Positions of four keys that all occur in the sorted row v[0..u): a
// branch-free lower bound in power-of-two steps from the largest power of
// two not above u (the position of a key is the number of smaller entries),
// the four keys' steps interleaved.
template <class P>
__device__ __forceinline__ void lower_bound4(P v, int u, const int key[4], int pos[4]) {
  pos[0] = pos[1] = pos[2] = pos[3] = 0;
  for (int st = u > 0 ? 1 << (31 - __clz(u)) : 0; st > 0; st >>= 1) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int q = pos[l] + st;
      if (q <= u && v[q - 1] < key[l]) pos[l] = q;
    }
  }
}

// CSR positions of the local blocks, one lane per pair (M) or slave element
// with pairs (D), for the four local nodes j in turn: for M, of the four
// master nodes of pair p in the row of slave node j of its element
// (posM[(4 j + l) * pstride + p]); for D, of the four nodes of element e in
// the row of its node j (posD[(4 j + k) * n_el + e]; elements without pairs
// are skipped, nothing reads their entries).  The rows a workgroup's lanes
// need for one j are neighbours in a mesh numbered row by row, so the
// workgroup stages the span of the column array from its smallest to its
// largest row in LDS with coalesced loads and each lane searches its row
// there; a span longer than POS_SPAN is searched in global memory.  Lanes
// write consecutive entries.
constexpr int POS_SPAN = 4096;

template <bool MCOLS>
__global__ __launch_bounds__(BS) void k_positions(int64_t n_items, const int32_t* __restrict__ n_dev,
                                                   const int32_t* __restrict__ pair_s,
                                                   const int32_t* __restrict__ pair_m,
                                                   const int32_t* __restrict__ pair_off,
                                                   const int32_t* __restrict__ conn_s,
                                                   const int32_t* __restrict__ conn_m,
                                                   const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col, int32_t* __restrict__ pos,
                                                   int64_t pstride) {
  __shared__ int32_t span[POS_SPAN];
  __shared__ int32_t red[2][BS / 64];
  const int64_t n = MCOLS ? (int64_t)*n_dev : n_items;
  // XCD-major tiles: neighbouring pairs (and the rows they stage) share an L2
  const int64_t tile = dyn_tile(blockIdx.x, n, BS);
  if (tile < 0) return;  // whole workgroups past the end
  const int64_t i = tile * BS + threadIdx.x;
  bool act = i < n;
  int4 cs = make_int4(0, 0, 0, 0), key4 = make_int4(0, 0, 0, 0);
  if (act) {
    const int e = MCOLS ? pair_s[i] : (int)i;
    if (!MCOLS) act = pair_off[e + 1] > pair_off[e];
    cs = reinterpret_cast<const int4*>(conn_s)[e];
    key4 = MCOLS ? reinterpret_cast<const int4*>(conn_m)[pair_m[i]] : cs;
  }
  const int key[4] = {key4.x, key4.y, key4.z, key4.w};
  const int w = threadIdx.x >> 6;
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {
    const int a = j == 0 ? cs.x : j == 1 ? cs.y : j == 2 ? cs.z : cs.w;
    int lo = act ? a : 0x7fffffff, hi = act ? a : -1;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      lo = min(lo, __shfl_xor(lo, d, 64));
      hi = max(hi, __shfl_xor(hi, d, 64));
    }
    __syncthreads();  // (the previous j's searches are done with the span)
    if ((threadIdx.x & 63) == 0) {
      red[0][w] = lo;
      red[1][w] = hi;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BS / 64; ++k) {
      lo = min(lo, red[0][k]);
      hi = max(hi, red[1][k]);
    }
    if (hi < 0) continue;  // no active lane (uniform across the workgroup)
    const int c0 = rowptr[lo], c1 = rowptr[hi + 1];
    const bool staged = c1 - c0 <= POS_SPAN;
    if (staged)
      for (int k = threadIdx.x; k < c1 - c0; k += BS) span[k] = col[c0 + k];
    __syncthreads();
    if (act) {
      const int r0 = rowptr[a], u = rowptr[a + 1] - r0;
      int ix[4];
      if (staged)
        lower_bound4(span + (r0 - c0), u, key, ix);
      else
        lower_bound4(col + r0, u, key, ix);
#pragma unroll
      for (int l = 0; l < 4; ++l) pos[(int64_t)(j * 4 + l) * pstride + i] = r0 + ix[l];
    }
  }
}

// One thread per slave node (row): the row is accumulated in a per-thread
// LDS segment (lane-interleaved) in a fixed order and written once.
constexpr int AB = 128;   // block of the assembly kernel
constexpr int ACAP = 32;  // per-thread accumulator entries (D + M of one row)

__global__ __launch_bounds__(AB) void k_assemble(const int32_t* __restrict__ inc_off,
                                                  const int32_t* __restrict__ inc_list, int32_t n,
                                                  const int32_t* __restrict__ pair_off,
                                                  const int32_t* __restrict__ D_rowptr,
                                                  const int32_t* __restrict__ M_rowptr,
                                                  const int32_t* __restrict__ posD, int32_t n_s_el,
                                                  const int32_t* __restrict__ posM, const double* __restrict__ blk,
                                                  int64_t stride, double* __restrict__ D_val,
                                                  double* __restrict__ M_val, double* __restrict__ gap) {
  __shared__ double acc[ACAP * AB];
  const int a = xcd_tile(blockIdx.x, gridDim.x) * AB + threadIdx.x;
  if (a >= n) return;
  assemble_row_acc(a, inc_off, inc_list, pair_off, D_rowptr, M_rowptr, posD, n_s_el, posM, blk, stride, D_val,
                   M_val, gap, acc + threadIdx.x, AB, ACAP);
}

__global__ __launch_bounds__(BS) void k_grad_slave(const int32_t* __restrict__ inc_off,
                                                    const int32_t* __restrict__ inc_list, int32_t n,
                                                    const int32_t* __restrict__ pair_off,
                                                    const double* __restrict__ gpair, int64_t stride,
                                                    double* __restrict__ gX) {
  const int a = xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
  if (a >= n) return;
  grad_slave_row(a, n, inc_off, inc_list, pair_off, gpair, stride, gX);
}

__global__ __launch_bounds__(BS) void k_grad_master(const int32_t* __restrict__ inc_off,
                                                     const int32_t* __restrict__ inc_list, int32_t n,
                                                     const int32_t* __restrict__ mstart,
                                                     const int32_t* __restrict__ mend,
                                                     const double* __restrict__ gpair, int64_t stride,
                                                     double* __restrict__ gX) {
  const int b = xcd_tile(blockIdx.x, gridDim.x) * BS + threadIdx.x;
  if (b >= n) return;
  grad_master_row(b, n, inc_off, inc_list, mstart, mend, gpair, stride, gX);
}

// Pairs by master element (the order the master-node gradient sums read):
// a counting sort -- pairs per master element (integer atomics), their
// exclusive scan, a scatter into each element's range -- then each range
// sorted ascending, so the order is the stable one (pair index within a
// master element) whatever order the atomics took; rank of each pair in it.
// A range of up to MS_SMALL pairs is sorted by one thread; a longer one (a
// master element much coarser than the slave elements it meets) goes on a
// list for a workgroup, which sorts runs of MS_RUN in LDS and merges them.
constexpr int MS_SMALL = 32;
constexpr int MS_RUN = 2048;
constexpr int MS_BLOCKS = 512;
constexpr unsigned MS_GRID = 2048;  // workgroups of the count and scatter passes

// (grid-stride over the live pairs with at most MS_GRID workgroups: these
// kernels run beside the pair quadrature on another stream)
__global__ __launch_bounds__(BS) void k_mcount(const int32_t* __restrict__ pair_m, const int32_t* __restrict__ n_dev,
                                                int32_t* __restrict__ cnt) {
  const int64_t n = *n_dev;
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS)
    atomicAdd(&cnt[pair_m[p]], 1);
}

__global__ __launch_bounds__(BS) void k_mscatter(const int32_t* __restrict__ pair_m, const int32_t* __restrict__ n_dev,
                                                  const int32_t* __restrict__ off, int32_t* __restrict__ cur,
                                                  uint32_t* __restrict__ vals) {
  const int64_t n = *n_dev;
  for (int64_t p = (int64_t)blockIdx.x * BS + threadIdx.x; p < n; p += (int64_t)gridDim.x * BS) {
    const int m = pair_m[p];
    vals[off[m] + atomicAdd(&cur[m], 1)] = (uint32_t)p;
  }
}

// Ranges of up to MS_REG values: held in registers (no LDS, so that the
// kernel finds room beside the LDS-heavy pattern kernels it runs with), each
// value placed at its rank, the number of smaller values in the range (the
// values, pair indices, are distinct), with its position recorded.  Up to
// MS_SMALL: an insertion sort in place.  Longer ranges: appended to `big`
// (its length in *n_big; the list order does not matter, each range is
// sorted on its own).
constexpr int MS_REG = 16;

__global__ __launch_bounds__(BS) void k_msort(const int32_t* __restrict__ off, int32_t n_m_el,
                                               uint32_t* __restrict__ vals, int32_t* __restrict__ mpos,
                                               int32_t* __restrict__ big, int32_t* __restrict__ n_big) {
  const int m = blockIdx.x * BS + threadIdx.x;
  if (m >= n_m_el) return;
  const int b = off[m], n = off[m + 1] - b;
  if (n > MS_SMALL) {
    big[atomicAdd(n_big, 1)] = m;
    return;
  }
  if (n <= MS_REG) {
    uint32_t v[MS_REG];
#pragma unroll
    for (int k = 0; k < MS_REG; ++k) v[k] = k < n ? vals[b + k] : 0xffffffffu;
#pragma unroll
    for (int k = 0; k < MS_REG; ++k) {
      if (k < n) {
        int rank = 0;
#pragma unroll
        for (int i = 0; i < MS_REG; ++i) rank += v[i] < v[k] ? 1 : 0;
        vals[b + rank] = v[k];
        mpos[v[k]] = b + rank;
      }
    }
    return;
  }
  for (int i = b + 1; i < b + n; ++i) {
    const uint32_t x = vals[i];
    int j = i - 1;
    while (j >= b && vals[j] > x) {
      vals[j + 1] = vals[j];
      --j;
    }
    vals[j + 1] = x;
  }
  for (int k = b; k < b + n; ++k) mpos[vals[k]] = k;
}

// Ascending bitonic sort of a[0..n) (n <= MS_RUN) through LDS, by the block.
__device__ void block_sort_run(uint32_t* __restrict__ a, int n, uint32_t* __restrict__ s) {
  int n2 = 2;
  while (n2 < n) n2 <<= 1;
  for (int t = threadIdx.x; t < n2; t += BS) s[t] = t < n ? a[t] : 0xffffffffu;
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (n2 >> 1); t += BS) {
        const int i = 2 * t - (t & (stride - 1));
        const int j = i + stride;
        const uint32_t x = s[i], y = s[j];
        if ((x > y) == ((i & size) == 0)) {
          s[i] = y;
          s[j] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < n; t += BS) a[t] = s[t];
  __syncthreads();
}

// Merge of the sorted runs x[0..nx) and y[0..ny) (distinct values) into
// out[0..nx+ny) by the block: each thread takes an equal share of the
// output and finds where it starts by a search along its diagonal.
__device__ void block_merge(const uint32_t* __restrict__ x, int nx, const uint32_t* __restrict__ y, int ny,
                            uint32_t* __restrict__ out) {
  const int n = nx + ny;
  const int seg = (n + BS - 1) / BS;
  const int d = min(n, (int)threadIdx.x * seg);
  const int end = min(n, d + seg);
  int lo = max(0, d - ny), hi = min(d, nx);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] < y[d - mid - 1])
      lo = mid + 1;
    else
      hi = mid;
  }
  int i = lo, j = d - lo;
  for (int o = d; o < end; ++o) out[o] = (j >= ny || (i < nx && x[i] < y[j])) ? x[i++] : y[j++];
}

__global__ __launch_bounds__(BS) void k_msort_big(const int32_t* __restrict__ off, const int32_t* __restrict__ big,
                                                   const int32_t* __restrict__ n_big, uint32_t* __restrict__ vals,
                                                   uint32_t* __restrict__ tmp, int32_t* __restrict__ mpos) {
  __shared__ uint32_t s[MS_RUN];
  const int nb = *n_big;
  for (int q = blockIdx.x; q < nb; q += gridDim.x) {
    const int m = big[q];
    const int b = off[m], k = off[m + 1] - b;
    for (int r = 0; r < k; r += MS_RUN) block_sort_run(vals + b + r, min(MS_RUN, k - r), s);
    uint32_t* src = vals + b;
    uint32_t* dst = tmp + b;
    for (int w = MS_RUN; w < k; w <<= 1) {
      for (int lo = 0; lo < k; lo += 2 * w) {
        const int mid = min(k, lo + w), hi = min(k, lo + 2 * w);
        block_merge(src + lo, mid - lo, src + mid, hi - mid, dst + lo);
      }
      __syncthreads();
      uint32_t* t = src;
      src = dst;
      dst = t;
    }
    for (int t = threadIdx.x; t < k; t += BS) {
      const uint32_t v = src[t];
      if (src != vals + b) vals[b + t] = v;
      mpos[v] = b + t;
    }
    __syncthreads();
  }
}

inline unsigned grid_of(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

}  // namespace

hipError_t launch_inc_count(const int32_t* conn, int32_t n_el, int32_t* cnt, hipStream_t s) {
  if (n_el == 0) return hipSuccess;
  k_inc_count<<<grid_of(n_el), BS, 0, s>>>(conn, n_el, cnt);
  return hipGetLastError();
}

hipError_t launch_inc_fill(const int32_t* conn, int32_t n_el, const int32_t* off, int32_t* cur, int32_t* list,
                           hipStream_t s) {
  if (n_el == 0) return hipSuccess;
  k_inc_fill<<<grid_of(n_el), BS, 0, s>>>(conn, n_el, off, cur, list);
  return hipGetLastError();
}

hipError_t launch_inc_sort(const int32_t* off, int32_t n_nodes, int32_t* list, hipStream_t s) {
  if (n_nodes == 0) return hipSuccess;
  k_inc_sort<<<grid_of(n_nodes), BS, 0, s>>>(off, n_nodes, list);
  return hipGetLastError();
}

hipError_t launch_pattern_rows(bool fill, const int32_t* inc_off, const int32_t* inc_list, int32_t n_nodes,
                               const int32_t* pair_off, const int32_t* pair_m, const int32_t* conn_s,
                               const int32_t* conn_m, int32_t* D_cnt, int32_t* M_cnt, const int32_t* D_rowptr,
                               const int32_t* M_rowptr, int32_t* D_col, int32_t* M_col, int32_t* keep,
                               int32_t n_s_el, int32_t* ecnt, int32_t* elist, hipStream_t s) {
  if (n_nodes == 0) return hipSuccess;
  const unsigned g = xcd_grid((unsigned)((n_nodes + PB - 1) / PB));
  int32_t* keepD = keep;
  int32_t* keepM = keep + (int64_t)KD * n_nodes;
  if (fill)
    k_pattern_rows<true><<<g, PB, 0, s>>>(inc_off, inc_list, n_nodes, pair_off, pair_m, conn_s, conn_m, D_cnt, M_cnt,
                                          D_rowptr, M_rowptr, D_col, M_col, keepD, keepM, n_s_el, nullptr, nullptr);
  else
    k_pattern_rows<false><<<g, PB, 0, s>>>(inc_off, inc_list, n_nodes, pair_off, pair_m, conn_s, conn_m, D_cnt,
                                           M_cnt, D_rowptr, M_rowptr, D_col, M_col, keepD, keepM, n_s_el, ecnt,
                                           elist);
  return hipGetLastError();
}

hipError_t launch_pattern_positions(const int32_t* pair_s, const int32_t* pair_m, const int32_t* n_pairs,
                                    int64_t cap, const int32_t* conn_s, const int32_t* conn_m, int32_t n_s_el,
                                    const int32_t* pair_off, const int32_t* D_rowptr, const int32_t* D_col,
                                    const int32_t* M_rowptr, const int32_t* M_col, int32_t* posD, int32_t* posM,
                                    hipStream_t s) {
  if (n_s_el > 0) {
    k_positions<false><<<xcd_grid(grid_of(n_s_el)), BS, 0, s>>>(n_s_el, nullptr, nullptr, nullptr, pair_off, conn_s, nullptr,
                                                      D_rowptr, D_col, posD, n_s_el);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (cap > 0)
    k_positions<true><<<xcd_grid(grid_of(cap)), BS, 0, s>>>(cap, n_pairs, pair_s, pair_m, nullptr, conn_s, conn_m, M_rowptr,
                                                  M_col, posM, cap);
  return hipGetLastError();
}

hipError_t launch_elem_mlist(int32_t n_s_el, const int32_t* pair_off, const int32_t* pair_m, const int32_t* conn_m,
                             int32_t* ecnt, int32_t* elist, hipStream_t s) {
  if (n_s_el == 0) return hipSuccess;
  k_elem_mlist<<<xcd_grid(grid_of(n_s_el)), BS, 0, s>>>(n_s_el, pair_off, pair_m, conn_m, ecnt, elist);
  return hipGetLastError();
}

int pattern_keep_per_row() { return KD + KM; }
int pattern_elem_list() { return EL; }

hipError_t launch_assemble(const int32_t* inc_off, const int32_t* inc_list, int32_t n_nodes, const int32_t* pair_off,
                           const int32_t* D_rowptr, const int32_t* M_rowptr, const int32_t* posD, int32_t n_s_el,
                           const int32_t* posM, const double* blk, int64_t stride, double* D_val, double* M_val,
                           double* gap, hipStream_t s) {
  if (n_nodes == 0) return hipSuccess;
  k_assemble<<<xcd_grid((unsigned)((n_nodes + AB - 1) / AB)), AB, 0, s>>>(inc_off, inc_list, n_nodes, pair_off, D_rowptr, M_rowptr, posD, n_s_el,
                                             posM, blk, stride, D_val, M_val, gap);
  return hipGetLastError();
}

hipError_t launch_grad_slave(const int32_t* inc_off, const int32_t* inc_list, int32_t n_nodes,
                             const int32_t* pair_off, const double* gpair, int64_t stride, double* gX,
                             hipStream_t s) {
  if (n_nodes == 0) return hipSuccess;
  k_grad_slave<<<xcd_grid(grid_of(n_nodes)), BS, 0, s>>>(inc_off, inc_list, n_nodes, pair_off, gpair, stride, gX);
  return hipGetLastError();
}

hipError_t launch_master_index(const int32_t* pair_m, const int32_t* n_pairs, int64_t cap, int32_t n_m_el,
                               int32_t* cnt, int32_t* cur, int32_t* off, uint32_t* vals, uint32_t* tmp, int32_t* mpos,
                               const Buf& scan_tmp, hipStream_t s) {
  if (n_m_el == 0) return hipSuccess;
  // cnt[n_m_el] counts the long ranges; cur, after the scatter, lists them
  hipError_t e = fill_i32(cnt, 0, (int64_t)n_m_el + 1, s);
  if (e == hipSuccess) e = fill_i32(cur, 0, (int64_t)n_m_el + 1, s);
  if (e != hipSuccess) return e;
  if (cap > 0) {
    k_mcount<<<std::min<unsigned>(grid_of(cap), MS_GRID), BS, 0, s>>>(pair_m, n_pairs, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = scan_exclusive(cnt, off, n_m_el, scan_tmp, s, SCAN_BLOCKS_BESIDE)) != hipSuccess) return e;
  if (cap > 0) {
    k_mscatter<<<std::min<unsigned>(grid_of(cap), MS_GRID), BS, 0, s>>>(pair_m, n_pairs, off, cur, vals);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  k_msort<<<grid_of(n_m_el), BS, 0, s>>>(off, n_m_el, vals, mpos, cur, cnt + n_m_el);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_msort_big<<<(unsigned)std::min<int64_t>(MS_BLOCKS, n_m_el), BS, 0, s>>>(off, cur, cnt + n_m_el, vals, tmp, mpos);
  return hipGetLastError();
}

hipError_t launch_grad_master(const int32_t* inc_off, const int32_t* inc_list, int32_t n_nodes,
                              const int32_t* mstart, const int32_t* mend, const double* gpair, int64_t stride,
                              double* gX, hipStream_t s) {
  if (n_nodes == 0) return hipSuccess;
  k_grad_master<<<xcd_grid(grid_of(n_nodes)), BS, 0, s>>>(inc_off, inc_list, n_nodes, mstart, mend, gpair, stride, gX);
  return hipGetLastError();
}

}  // namespace mt
