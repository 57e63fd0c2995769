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

template <class T>
__global__ __launch_bounds__(SCAN_BS) void k_tile_sums(const T* __restrict__ in, int64_t n, T* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i)
    if (base + i < n) s += in[base + i];
  T tot;
  block_exclusive(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = offs[tile] + exclusive prefix of in within the tile; the last
// tile also writes out[n] = grand total.
template <class T>
__global__ __launch_bounds__(SCAN_BS) void k_tile_scan(const T* __restrict__ in, int64_t n,
                                                       const T* __restrict__ offs, T* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
  T v[SCAN_IPT];
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    v[i] = (base + i < n) ? in[base + i] : T(0);
    s += v[i];
  }
  T tot;
  T run = block_exclusive(s, &tot) + (offs ? offs[blockIdx.x] : T(0));
#pragma unroll
  for (int i = 0; i < SCAN_IPT; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BS - 1) out[n] = run;
}

template <class T>
hipError_t scan_impl(const T* in, T* out, int64_t n, T* tmp, hipStream_t s) {
  const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (n == 0) return hipMemsetAsync(out, 0, sizeof(T), s);
  if (tiles == 1) {
    k_tile_scan<T><<<1, SCAN_BS, 0, s>>>(in, n, nullptr, out);
    return hipGetLastError();
  }
  T* sums = tmp;
  T* offs = tmp + tiles;  // tiles + 1 entries
  T* rest = offs + tiles + 1;
  k_tile_sums<T><<<(unsigned)tiles, SCAN_BS, 0, s>>>(in, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_impl<T>(sums, offs, tiles, rest, s);
  if (e != hipSuccess) return e;
  k_tile_scan<T><<<(unsigned)tiles, SCAN_BS, 0, s>>>(in, n, offs, out);
  return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) {
  int64_t total = 0;
  while (true) {
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles <= 1) break;
    total += 2 * tiles + 1;
    n = tiles;
  }
  return total + 1;
}

// ---- radix sort ------------------------------------------------------------

constexpr int RS_BS = 256;
constexpr int RS_IPT = 8;
constexpr int RS_TILE = RS_BS * RS_IPT;
constexpr int RS_RADIX = 256;

// Per tile digit histogram, stored digit-major: hist[d * tiles + tile].
__global__ __launch_bounds__(RS_BS) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                    int32_t* __restrict__ hist, int64_t tiles) {
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
                                                       int64_t n, int shift, const int32_t* __restrict__ offs,
                                                       int64_t tiles) {
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

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t scan_exclusive(const int32_t* in, int32_t* out, int64_t n, Buf& tmp, hipStream_t s) {
  hipError_t e = ensure(tmp, sizeof(int32_t) * (size_t)scan_tmp_elems(n));
  if (e != hipSuccess) return e;
  return scan_impl<int32_t>(in, out, n, tmp.as<int32_t>(), s);
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                            int bits, Buf& hist, Buf& scan_tmp, hipStream_t s) {
  if (n <= 1 || bits <= 0) return hipSuccess;
  const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
  const int64_t hn = tiles * RS_RADIX;
  hipError_t e = ensure(hist, sizeof(int32_t) * (size_t)(2 * hn + 1));
  if (e != hipSuccess) return e;
  int32_t* h = hist.as<int32_t>();
  int32_t* off = h + hn;
  int passes = (bits + 7) / 8;
  uint32_t *ki = keys, *vi = vals, *ko = keys_tmp, *vo = vals_tmp;
  for (int p = 0; p < passes; ++p) {
    k_rs_hist<<<(unsigned)tiles, RS_BS, 0, s>>>(ki, n, 8 * p, h, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive(h, off, hn, scan_tmp, s)) != hipSuccess) return e;
    k_rs_scatter<<<(unsigned)tiles, RS_BS, 0, s>>>(ki, vi, ko, vo, n, 8 * p, off, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  if (ki != keys) {
    if ((e = hipMemcpyAsync(keys, ki, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(vals, vi, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_f64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

}  // namespace mt
