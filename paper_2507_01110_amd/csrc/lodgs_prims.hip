// Scan and radix-sort kernels (see lodgs_prims.h).
#include "lodgs_prims.h"

namespace lodgs {

__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint32_t* keys, const int32_t* d_n, int64_t cap,
                                                       int shift, uint32_t* table, uint32_t* below) {
  __shared__ uint32_t h[256];
  __shared__ uint32_t wt[kBlock / 64];
  int64_t n = *d_n;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const Segment s = block_segment(n, kSortGrid);
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = s.begin + threadIdx.x; i < s.end; i += kBlock) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  const uint32_t c = h[threadIdx.x];
  uint32_t tot;
  const uint32_t pre = block_exclusive_scan(c, wt, &tot);  // thread = digit
  table[(int64_t)threadIdx.x * kSortGrid + blockIdx.x] = c;
  below[(int64_t)threadIdx.x * kSortGrid + blockIdx.x] = pre;
}

// One workgroup per digit d: offset(d, b) = (elements of all blocks with a
// digit below d) + (elements with digit d in the blocks before b).
__global__ void __launch_bounds__(kBlock) k_radix_offsets(uint32_t* table, const uint32_t* below) {
  __shared__ uint32_t wt[kBlock / 64];
  constexpr int per = kSortGrid / kBlock;  // row entries per thread
  const int64_t row0 = (int64_t)blockIdx.x * kSortGrid + threadIdx.x * per;
  uint32_t bsum = 0, v[per], sum = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    bsum += below[row0 + k];
    v[k] = table[row0 + k];
    sum += v[k];
  }
  uint32_t base;
  block_exclusive_scan(bsum, wt, &base);
  uint32_t tot;
  uint32_t run = base + block_exclusive_scan(sum, wt, &tot);
#pragma unroll
  for (int k = 0; k < per; ++k) {
    table[row0 + k] = run;
    run += v[k];
  }
}

__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint32_t* kin, const uint32_t* vin,
                                                          uint32_t* kout, uint32_t* vout, const int32_t* d_n,
                                                          int64_t cap, int shift, const uint32_t* table) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kBlock / 64][256];
  int64_t n = *d_n;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const Segment s = block_segment(n, kSortGrid);
  if (s.begin >= s.end) return;  // uniform across the block
  const int t = threadIdx.x, wave = t >> 6;
  base[t] = table[(int64_t)t * kSortGrid + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  for (int64_t r0 = s.begin; r0 < s.end; r0 += kBlock) {
    const int64_t i = r0 + t;
    const bool valid = i < s.end;
    const uint32_t key = valid ? kin[i] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bm = __ballot(bit);
      m &= bit ? bm : ~bm;
    }
    const uint32_t rank = (uint32_t)__popcll(m & lt);
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = vin[i];
    }
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      sum += wcnt[w][t];
      wcnt[w][t] = 0;
    }
    base[t] += sum;
    __syncthreads();
  }
}

bool sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* k2, uint32_t* v2, const int32_t* d_n, int64_t cap,
                int bits, const SortScratch& ws, hipStream_t st) {
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  bool swapped = false;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(kSortGrid), dim3(kBlock), 0, st, ka, d_n, cap, shift, ws.table,
                       ws.below);
    hipLaunchKernelGGL(k_radix_offsets, dim3(256), dim3(kBlock), 0, st, ws.table, ws.below);
    hipLaunchKernelGGL(k_radix_scatter, dim3(kSortGrid), dim3(kBlock), 0, st, ka, va, kb, vb, d_n, cap, shift,
                       ws.table);
    uint32_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
    swapped = !swapped;
  }
  return swapped;
}

}  // namespace lodgs
