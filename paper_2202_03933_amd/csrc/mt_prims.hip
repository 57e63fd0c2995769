// Device-wide primitives: exclusive scan and a stable LSD radix sort of
// (uint32 key, uint32 value) pairs, written for 64-wide wavefronts.
#include "mt_internal.h"

namespace mt {

namespace {

constexpr int SCAN_BS = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IPT;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Inclusive scan of one value per lane across a wavefront.
template <class T>
__device__ __forceinline__ T wave_inclusive(T x) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane_id() >= d) x += y;
  }
  return x;
}

// Exclusive scan across the block of one value per thread; returns the
// exclusive prefix and writes the block total to *total.
template <class T>
__device__ __forceinline__ T block_exclusive(T x, T* total) {
  __shared__ T wsum[SCAN_BS / 64];
  const int w = threadIdx.x >> 6;
  T inc = wave_inclusive(x);
  if (lane_id() == 63) wsum[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_BS / 64; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - x;
}

// n_dev (optional): a count the device holds, at most n; entries from it on
// count as zero.
template <class T>
__device__ __forceinline__ int64_t live_count(int64_t n, const int32_t* n_dev) {
  if (!n_dev) return n;
  const int64_t m = *n_dev;
  return m < 0 ? 0 : (m < n ? m : n);
}

// Exclusive scan: per-tile sums, then each tile's scan with its offset.
// Up to SCAN_DIRECT tiles, every tile adds up the sums before it itself (no
// third launch; the sums are a few KB, read from L2); beyond, the sums are
// scanned recursively first.  No tile waits for another.
constexpr int64_t SCAN_DIRECT = 8192;

// The SCAN_IPT values of thread's slot (zero past `live`): two 16-byte loads
// when VEC (in 16-byte aligned) and the slot is whole.
template <bool VEC>
__device__ __forceinline__ void load_slot(const int32_t* __restrict__ in, int64_t base, int64_t live,
                                          int32_t v[SCAN_IPT]) {
  static_assert(SCAN_IPT == 8, "two 16-byte vectors per thread");
  if (VEC && base + SCAN_IPT <= live) {
    const int4 a = *reinterpret_cast<const int4*>(in + base);
    const int4 b = *reinterpret_cast<const int4*>(in + base + 4);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) v[i] = (base + i < live) ? in[base + i] : 0;
  }
}

// Each workgroup takes `per` consecutive tiles.  A launch with gridDim.y = 2
// scans a second array of the same length (in2 into out2, its workgroup sums
// after the first array's) in the same launches.
template <bool VEC>
__global__ __launch_bounds__(SCAN_BS) void k_tile_sums(const int32_t* __restrict__ in, const int32_t* __restrict__ in2,
                                                       int64_t n, const int32_t* n_dev, int32_t* __restrict__ sums,
                                                       int per) {
  if (blockIdx.y) {
    in = in2;
    sums += gridDim.x;
  }
  const int64_t live = live_count<int32_t>(n, n_dev);
  int32_t s = 0;
  for (int q = 0; q < per; ++q) {
    const int64_t base = ((int64_t)blockIdx.x * per + q) * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int32_t v[SCAN_IPT];
    load_slot<VEC>(in, base, live, v);
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) s += v[i];
  }
  int32_t tot;
  block_exclusive(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = offset of the workgroup + exclusive prefix of in within its
// tiles; the last workgroup also writes out[n] = grand total.  Offset of
// workgroup w: offs[w] (scanned), or with DIRECT the sum of sums[0..w) (raw
// workgroup sums), or 0.
template <bool VEC, bool DIRECT>
__global__ __launch_bounds__(SCAN_BS) void k_tile_scan(const int32_t* __restrict__ in, const int32_t* __restrict__ in2,
                                                       int64_t n, const int32_t* n_dev,
                                                       const int32_t* __restrict__ offs, int32_t* __restrict__ out,
                                                       int32_t* __restrict__ out2, int per) {
  if (blockIdx.y) {  // (the raw workgroup sums of the second array follow the first's)
    in = in2;
    out = out2;
    if (DIRECT) offs += gridDim.x;
  }
  const int64_t live = live_count<int32_t>(n, n_dev);
  const int64_t w = blockIdx.x;
  int32_t off = 0;
  if (DIRECT) {
    int32_t part = 0;
    for (int64_t i = threadIdx.x; i < w; i += SCAN_BS) part += offs[i];
    block_exclusive(part, &off);
  } else if (offs) {
    off = offs[w];
  }
  for (int q = 0; q < per; ++q) {
    const int64_t base = (w * per + q) * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int32_t v[SCAN_IPT];
    load_slot<VEC>(in, base, live, v);
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) s += v[i];
    int32_t tot;
    int32_t run = block_exclusive(s, &tot) + off;
    int32_t o[SCAN_IPT];
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) {
      o[i] = run;
      run += v[i];
    }
    if (VEC && base + SCAN_IPT <= n) {
      *reinterpret_cast<int4*>(out + base) = make_int4(o[0], o[1], o[2], o[3]);
      *reinterpret_cast<int4*>(out + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
      for (int i = 0; i < SCAN_IPT; ++i)
        if (base + i < n) out[base + i] = o[i];
    }
    off += tot;
  }
  if (w == (int64_t)gridDim.x - 1 && threadIdx.x == 0) out[n] = off;
}

// Exclusive scan of n values (of the first *n_dev when given; the rest count
// as zero) into out[0..n]; with in2, also of in2 into out2 (n_dev null) in
// the same launches while the workgroup sums of both fit the direct scheme.
// max_blocks > 0 caps the workgroups of each launch (several tiles each): a
// scan queued beside a long kernel on another stream then waits for few
// dispatch slots.  No memset: the launches can be captured in a graph.
hipError_t scan_impl(const int32_t* in, int32_t* out, int64_t n, const int32_t* n_dev, int32_t* tmp, hipStream_t s,
                     const int32_t* in2 = nullptr, int32_t* out2 = nullptr, int64_t max_blocks = 0) {
  const int64_t tiles = std::max<int64_t>(1, (n + SCAN_TILE - 1) / SCAN_TILE);
  const int per = max_blocks > 0 ? (int)((tiles + max_blocks - 1) / max_blocks) : 1;
  const int64_t blocks = (tiles + per - 1) / per;
  uintptr_t addr = reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out);
  if (in2) addr |= reinterpret_cast<uintptr_t>(in2) | reinterpret_cast<uintptr_t>(out2);
  const bool vec = (addr & 15) == 0;
  if (in2 && blocks > SCAN_DIRECT) {
    hipError_t e = scan_impl(in, out, n, n_dev, tmp, s, nullptr, nullptr, max_blocks);
    return e != hipSuccess ? e : scan_impl(in2, out2, n, nullptr, tmp, s, nullptr, nullptr, max_blocks);
  }
  const dim3 grid((unsigned)blocks, in2 ? 2u : 1u);
  if (blocks == 1) {
    auto* k = vec ? k_tile_scan<true, false> : k_tile_scan<false, false>;
    k<<<grid, SCAN_BS, 0, s>>>(in, in2, n, n_dev, nullptr, out, out2, per);
    return hipGetLastError();
  }
  int32_t* sums = tmp;  // blocks (2 blocks with in2) entries
  (vec ? k_tile_sums<true> : k_tile_sums<false>)<<<grid, SCAN_BS, 0, s>>>(in, in2, n, n_dev, sums, per);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (blocks <= SCAN_DIRECT) {
    auto* k = vec ? k_tile_scan<true, true> : k_tile_scan<false, true>;
    k<<<grid, SCAN_BS, 0, s>>>(in, in2, n, n_dev, sums, out, out2, per);
    return hipGetLastError();
  }
  int32_t* offs = tmp + blocks;  // blocks + 1 entries
  e = scan_impl(sums, offs, blocks, nullptr, offs + blocks + 1, s);
  if (e != hipSuccess) return e;
  auto* k = vec ? k_tile_scan<true, false> : k_tile_scan<false, false>;
  k<<<(unsigned)blocks, SCAN_BS, 0, s>>>(in, nullptr, n, n_dev, offs, out, nullptr, per);
  return hipGetLastError();
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) {
  // per level: the tile sums and their scan (tiles + 1), while recursing
  int64_t total = 0;
  while (true) {
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles <= 1) break;
    total += 2 * tiles + 1;
    if (tiles <= SCAN_DIRECT) break;
    n = tiles;
  }
  return total + 1;
}

namespace {

// ---- radix sort ------------------------------------------------------------

constexpr int RS_BS = 256;
constexpr int RS_IPT = 8;
constexpr int RS_TILE = RS_BS * RS_IPT;
constexpr int RS_RADIX = 256;

// Per tile digit histogram, stored digit-major: hist[d * tiles + tile].
__global__ __launch_bounds__(RS_BS) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                    const int32_t* n_dev, int shift, int32_t* __restrict__ hist,
                                                    int64_t tiles) {
  n = live_count<int32_t>(n, n_dev);
  __shared__ int32_t h[RS_RADIX];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int i = 0; i < RS_IPT; ++i) {
    const int64_t idx = base + (int64_t)i * RS_BS + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xff], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: keys of a tile are taken in rounds of RS_BS consecutive
// keys; a key's rank among equal digits is its rank within its wavefront
// (ballot match over the 8 digit bits), plus the counts of lower waves in
// the round, plus the count of earlier rounds.
__global__ __launch_bounds__(RS_BS) void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                       uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                       int64_t n, const int32_t* n_dev, int shift,
                                                       const int32_t* __restrict__ offs, int64_t tiles) {
  n = live_count<int32_t>(n, n_dev);
  __shared__ int32_t run[RS_RADIX];
  __shared__ int32_t wcnt[RS_BS / 64][RS_RADIX];
  run[threadIdx.x] = offs[(int64_t)threadIdx.x * tiles + blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_IPT; ++r) {
#pragma unroll
    for (int i = 0; i < RS_BS / 64; ++i) wcnt[i][threadIdx.x] = 0;
    __syncthreads();
    const int64_t idx = base + (int64_t)r * RS_BS + threadIdx.x;
    const bool valid = idx < n;
    uint32_t key = 0, val = 0;
    int d = 0;
    if (valid) {
      key = kin[idx];
      val = vin[idx];
      d = (key >> shift) & 0xff;
    }
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const int rank = __popcll(m & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(m);
    __syncthreads();
    // exclusive prefix over waves for digit threadIdx.x
    {
      int acc = 0;
#pragma unroll
      for (int i = 0; i < RS_BS / 64; ++i) {
        const int c = wcnt[i][threadIdx.x];
        wcnt[i][threadIdx.x] = acc;
        acc += c;
      }
      __syncthreads();
      if (valid) {
        const int64_t pos = (int64_t)run[d] + wcnt[w][d] + rank;
        kout[pos] = key;
        vout[pos] = val;
      }
      __syncthreads();
      run[threadIdx.x] += acc;
    }
    __syncthreads();
  }
}

// Grid-stride fill: at most FILL_BLOCKS workgroups, so that a fill queued
// beside a long kernel on another stream waits for few dispatch slots.
constexpr int64_t FILL_BLOCKS = 1024;
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_copy_u32(const uint32_t* __restrict__ a, uint32_t* __restrict__ b, int64_t n,
                           const int32_t* n_dev) {
  n = live_count<int32_t>(n, n_dev);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace

hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, const Buf& tmp, hipStream_t s,
                          int64_t max_blocks) {
  if ((int64_t)(tmp.bytes / sizeof(int32_t)) < scan_tmp_elems(n)) return hipErrorInvalidValue;
  return scan_impl(in, out, n, nullptr, tmp.as<int32_t>(), s, nullptr, nullptr, max_blocks);
}

hipError_t scan_exclusive2(const int32_t* in, int32_t* out, const int32_t* in2, int32_t* out2, int64_t n,
                           const Buf& tmp, hipStream_t s, int64_t max_blocks) {
  if ((int64_t)(tmp.bytes / sizeof(int32_t)) < scan_tmp_elems(n)) return hipErrorInvalidValue;
  return scan_impl(in, out, n, nullptr, tmp.as<int32_t>(), s, in2, out2, max_blocks);
}

hipError_t scan_exclusive_dev(const int32_t* in, int32_t* out, const int32_t* n_dev, int64_t cap, const Buf& tmp,
                              hipStream_t s) {
  if ((int64_t)(tmp.bytes / sizeof(int32_t)) < scan_tmp_elems(cap)) return hipErrorInvalidValue;
  return scan_impl(in, out, cap, n_dev, tmp.as<int32_t>(), s);
}

int64_t radix_hist_elems(int64_t n) { return 2 * ((n + RS_TILE - 1) / RS_TILE) * RS_RADIX + 1; }

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                            const int32_t* n_dev, int bits, const Buf& hist, const Buf& scan_tmp, hipStream_t s,
                            bool in_tmp) {
  if (in_tmp) {
    std::swap(keys, keys_tmp);
    std::swap(vals, vals_tmp);
  }
  // from here the input is in (keys, vals); the result goes to (keys, vals)
  // of the caller: the other pair when in_tmp
  uint32_t* const out_k = in_tmp ? keys_tmp : keys;
  uint32_t* const out_v = in_tmp ? vals_tmp : vals;
  if (n <= 1 || bits <= 0) {  // no pass: the input is the result
    if (in_tmp && n > 0) {
      const unsigned nb = (unsigned)((n + 255) / 256);
      k_copy_u32<<<nb, 256, 0, s>>>(keys, out_k, n, n_dev);
      k_copy_u32<<<nb, 256, 0, s>>>(vals, out_v, n, n_dev);
      return hipGetLastError();
    }
    return hipSuccess;
  }
  const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
  const int64_t hn = tiles * RS_RADIX;
  if ((int64_t)(hist.bytes / sizeof(int32_t)) < radix_hist_elems(n)) return hipErrorInvalidValue;
  int32_t* h = hist.as<int32_t>();
  int32_t* off = h + hn;
  hipError_t e;
  const int passes = radix_passes(bits);
  uint32_t *ki = keys, *vi = vals, *ko = keys_tmp, *vo = vals_tmp;
  for (int p = 0; p < passes; ++p) {
    k_rs_hist<<<(unsigned)tiles, RS_BS, 0, s>>>(ki, n, n_dev, 8 * p, h, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(h, off, hn, scan_tmp, s)) != hipSuccess) return e;
    k_rs_scatter<<<(unsigned)tiles, RS_BS, 0, s>>>(ki, vi, ko, vo, n, n_dev, 8 * p, off, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  if (ki != out_k) {
    const unsigned nb = (unsigned)((n + 255) / 256);
    k_copy_u32<<<nb, 256, 0, s>>>(ki, out_k, n, n_dev);
    k_copy_u32<<<nb, 256, 0, s>>>(vi, out_v, n, n_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<(unsigned)std::min<int64_t>((n + 255) / 256, FILL_BLOCKS), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_f64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

}  // namespace mt
