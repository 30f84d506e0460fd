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

// Stable scatter of one radix pass.  The block's segment is taken in tiles of
// up to kScatterTile keys.  For each tile: (1) keys are ranked in order within
// their digit, 256 per round (one ballot per digit bit finds the lanes of a
// wave with the same digit, per-wave counts give the order across waves, a
// running count per digit the order across rounds); (2) the tile is staged in
// LDS in digit order; (3) consecutive threads write consecutive staged keys,
// so a digit's keys go to consecutive global positions.  With XTRA an 8-byte
// payload per key is read when the tile is staged (coalesced: input order)
// and staged and written with it.
constexpr int kScatterRounds = 16;
constexpr int kScatterTile = kScatterRounds * kBlock;

template <bool XTRA>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint32_t* kin, const uint32_t* vin,
                                                          uint32_t* kout, uint32_t* vout, const uint2* xin,
                                                          uint2* xout, const int32_t* d_n, int64_t cap, int shift,
                                                          const uint32_t* table) {
  __shared__ uint32_t base[256];   // global position of the digit's next key
  __shared__ uint32_t lcnt[256];   // keys of the digit in the tile (so far)
  __shared__ uint32_t lstart[256]; // first staged position of the digit
  __shared__ uint32_t wcnt[kBlock / 64][256];
  __shared__ uint32_t wt[kBlock / 64];
  __shared__ uint32_t sk[kScatterTile], sv[kScatterTile];
  __shared__ uint2 sx[XTRA ? kScatterTile : 1];
  int64_t n = *d_n;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const Segment s = block_segment(n, kSortGrid);
  if (s.begin >= s.end) return;  // uniform across the block
  const int t = threadIdx.x, wave = t >> 6;
  base[t] = table[(int64_t)t * kSortGrid + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) wcnt[w][t] = 0;
  const uint64_t lt = lanemask_lt();
  for (int64_t t0 = s.begin; t0 < s.end; t0 += kScatterTile) {  // block-uniform
    const int64_t tn = s.end - t0 < kScatterTile ? s.end - t0 : kScatterTile;
    lcnt[t] = 0;
    __syncthreads();
    uint32_t kr[kScatterRounds], vr[kScatterRounds], lr[kScatterRounds];
#pragma unroll
    for (int u = 0; u < kScatterRounds; ++u) {
      const int64_t j = (int64_t)u * kBlock + t;
      const bool valid = j < tn;
      kr[u] = valid ? kin[t0 + j] : 0u;
      vr[u] = valid ? vin[t0 + j] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kScatterRounds; ++u) {
      if ((int64_t)u * kBlock >= tn) break;  // block-uniform
      const bool valid = (int64_t)u * kBlock + t < tn;
      const uint32_t d = (kr[u] >> shift) & 255u;
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
      uint32_t r = lcnt[d] + rank;
      for (int w = 0; w < wave; ++w) r += wcnt[w][d];
      lr[u] = r;
      __syncthreads();
      uint32_t sum = 0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) {
        sum += wcnt[w][t];
        wcnt[w][t] = 0;
      }
      lcnt[t] += sum;
      __syncthreads();
    }
    uint32_t tot;
    lstart[t] = block_exclusive_scan(lcnt[t], wt, &tot);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kScatterRounds; ++u) {
      if ((int64_t)u * kBlock + t < tn) {
        const uint32_t d = (kr[u] >> shift) & 255u;
        const uint32_t pos = lstart[d] + lr[u];
        sk[pos] = kr[u];
        sv[pos] = vr[u];
        if (XTRA) sx[pos] = xin[t0 + (int64_t)u * kBlock + t];
      }
    }
    __syncthreads();
    for (int j = t; j < (int)tn; j += kBlock) {
      const uint32_t key = sk[j];
      const uint32_t d = (key >> shift) & 255u;
      const uint32_t g = base[d] + ((uint32_t)j - lstart[d]);
      kout[g] = key;
      vout[g] = sv[j];
      if (XTRA) xout[g] = sx[j];
    }
    __syncthreads();
    base[t] += lcnt[t];
    __syncthreads();
  }
}

bool sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* k2, uint32_t* v2, const int32_t* d_n, int64_t cap,
                int bits, const SortScratch& ws, hipStream_t st, uint2* xtra, uint2* x2) {
  uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
  uint2 *xa = xtra, *xb = x2;
  bool swapped = false;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(kSortGrid), dim3(kBlock), 0, st, ka, d_n, cap, shift, ws.table,
                       ws.below);
    hipLaunchKernelGGL(k_radix_offsets, dim3(256), dim3(kBlock), 0, st, ws.table, ws.below);
    if (xtra)
      hipLaunchKernelGGL(k_radix_scatter<true>, dim3(kSortGrid), dim3(kBlock), 0, st, ka, va, kb, vb, xa, xb, d_n,
                         cap, shift, ws.table);
    else
      hipLaunchKernelGGL(k_radix_scatter<false>, dim3(kSortGrid), dim3(kBlock), 0, st, ka, va, kb, vb,
                         (const uint2*)nullptr, (uint2*)nullptr, d_n, cap, shift, ws.table);
    uint32_t* tk = ka; ka = kb; kb = tk;
    uint32_t* tv = va; va = vb; vb = tv;
    uint2* tx = xa; xa = xb; xb = tx;
    swapped = !swapped;
  }
  return swapped;
}

}  // namespace lodgs
