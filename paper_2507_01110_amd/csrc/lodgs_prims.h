// Data-parallel primitives with device-resident element counts: exclusive
// scan and stable LSD radix sort of 32-bit keys with 32-bit values.  Every
// kernel runs a fixed grid whose blocks each own one contiguous segment of the
// input (segment = ceil(n / grid)), so launches need no host-side count and
// can be captured in a graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lodgs {

constexpr int kScanGrid = 512;    // blocks of the multi-block scan
constexpr int kSortGrid = 512;    // blocks of a radix pass
constexpr int kBlock = 256;
static_assert(kSortGrid % kBlock == 0, "a radix offsets workgroup scans a table row in whole chunks");

struct Segment {
  int64_t begin, end;
};

__device__ __forceinline__ Segment block_segment(int64_t n, int grid) {
  const int64_t per = (n + grid - 1) / grid;
  int64_t b = (int64_t)blockIdx.x * per;
  int64_t e = b + per;
  if (b > n) b = n;
  if (e > n) e = n;
  return {b, e};
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Exclusive scan of one value per thread over a block of kBlock threads.
// wave_tot must hold kBlock / 64 entries.  Returns the exclusive prefix and
// the block total in *total.  Contains barriers: call from all threads.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wave_tot, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wave_tot[wave] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    uint32_t t = wave_tot[w];
    base += w < wave ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// ---------------------------------------------------------------- scan
template <class Load>
__global__ void __launch_bounds__(kBlock) k_scan_reduce(Load load, const int32_t* d_n, int64_t cap,
                                                        uint32_t* block_sums) {
  __shared__ uint32_t wt[kBlock / 64];
  int64_t n = *d_n;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const Segment s = block_segment(n, kScanGrid);
  uint32_t acc = 0;
  for (int64_t i = s.begin + threadIdx.x; i < s.end; i += kBlock) acc += load(i);
  uint32_t tot;
  block_exclusive_scan(acc, wt, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Each block first sums the totals of the blocks before it (block 0 also
// sums all of them and writes the grand total to *d_total, if not null), then
// scans its own segment, handing each element's exclusive prefix to the
// store functor: store(i, prefix, value).
template <class Load, class Store>
__global__ void __launch_bounds__(kBlock) k_scan_down(Load load, const int32_t* d_n, int64_t cap,
                                                      const uint32_t* block_sums, Store store, int32_t* d_total) {
  __shared__ uint32_t wt[kBlock / 64];
  uint32_t before = 0, all = 0;
  for (int t = threadIdx.x; t < kScanGrid; t += kBlock) {
    const uint32_t x = block_sums[t];
    before += t < (int)blockIdx.x ? x : 0u;
    all += x;
  }
  uint32_t base;
  block_exclusive_scan(before, wt, &base);
  if (blockIdx.x == 0) {
    uint32_t grand;
    block_exclusive_scan(all, wt, &grand);
    if (threadIdx.x == 0 && d_total) *d_total = (int32_t)grand;
  }
  int64_t n = *d_n;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const Segment s = block_segment(n, kScanGrid);
  for (int64_t t0 = s.begin; t0 < s.end; t0 += kBlock * 4) {
    const int64_t i0 = t0 + (int64_t)threadIdx.x * 4;
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (i0 + k < s.end) ? load(i0 + k) : 0u;
    uint32_t tot;
    uint32_t run = base + block_exclusive_scan(v[0] + v[1] + v[2] + v[3], wt, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < s.end) store(i0 + k, run, v[k]);
      run += v[k];
    }
    base += tot;
  }
}

struct LoadArray {
  const uint32_t* a;
  __device__ uint32_t operator()(int64_t i) const { return a[i]; }
};

struct StoreArray {
  uint32_t* out;
  __device__ void operator()(int64_t i, uint32_t prefix, uint32_t) const { out[i] = prefix; }
};

// store(i, sum_{j < i} load(j), load(i)) for i < min(*d_n, cap); *d_total =
// sum (may be null).  block_sums: kScanGrid words of scratch.  The store may
// overwrite the array read by load at index i.  Two kernels: per-block
// totals, then per-block bases and the scan of each segment.
template <class Load, class Store>
inline void scan_exclusive(Load load, const int32_t* d_n, int64_t cap, uint32_t* block_sums, Store store,
                           int32_t* d_total, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_reduce<Load>, dim3(kScanGrid), dim3(kBlock), 0, st, load, d_n, cap, block_sums);
  hipLaunchKernelGGL((k_scan_down<Load, Store>), dim3(kScanGrid), dim3(kBlock), 0, st, load, d_n, cap, block_sums,
                     store, d_total);
}

template <class Load>
inline void scan_exclusive(Load load, const int32_t* d_n, int64_t cap, uint32_t* block_sums, uint32_t* out,
                           int32_t* d_total, hipStream_t st) {
  scan_exclusive(load, d_n, cap, block_sums, StoreArray{out}, d_total, st);
}

// ---------------------------------------------------------------- radix sort
// One pass = three kernels: per-block digit counts (digit-major table
// [256][kSortGrid]) together with each block's exclusive prefix over the
// digits (same layout, in below); the exclusive offsets of every (digit,
// block), one workgroup per digit (the sum of its row of below gives the
// count of all smaller digits, the scan of its row of counts the blocks
// before); the stable scatter.  Ranks inside a block come from wave ballots
// over the digit bits plus per-wave digit counts in LDS, so equal digits keep
// their input order.
__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint32_t* keys, const int32_t* d_n, int64_t cap,
                                                       int shift, uint32_t* table, uint32_t* below);
__global__ void __launch_bounds__(kBlock) k_radix_offsets(uint32_t* table, const uint32_t* below);
template <bool XTRA>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint32_t* kin, const uint32_t* vin,
                                                          uint32_t* kout, uint32_t* vout, const uint2* xin,
                                                          uint2* xout, const int32_t* d_n, int64_t cap, int shift,
                                                          const uint32_t* table);

// Workspace for sort_pairs: two tables of 256 * kSortGrid words.
struct SortScratch {
  uint32_t* table;
  uint32_t* below;
};

// Sorts (keys, vals) of length min(*d_n, cap) by the key bits [0, bits), stable.
// Uses (k2, v2) as ping-pong buffers; returns true if the result ended in
// (k2, v2), false if in (keys, vals).  With xtra non-null, an 8-byte payload
// per element moves with it (xtra / x2 ping-pong like keys / k2).
bool sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* k2, uint32_t* v2, const int32_t* d_n, int64_t cap,
                int bits, const SortScratch& ws, hipStream_t st, uint2* xtra = nullptr, uint2* x2 = nullptr);

}  // namespace lodgs
