// Device pool of the rows of cached SPT cuts (Sec. 4.4 "Caching on the GPU":
// the Gaussians of a cached cut stay in VRAM; Alg. 3: Load from RAM, cache
// insert, write-back of evicted entries).  The parameters live in pinned host
// memory; the upper hierarchy's rows are kept resident (Alg. 3 renders them
// every iteration); the rows of every SPT entry of an SPT-cut cache occupy
// pool slots, one per selected node of its cached cut, so a cache hit reads
// nothing over the host link.  After each lodgs_lod_select_cached, for every
// SPT: an entry that was dropped gives all its slots back; an entry that was
// cut afresh (a cache miss) gives back the slots of the nodes its new cut no
// longer holds (write-back of the rows lodgs_row_pool_store changed comes
// first); every node of a cached, visible entry that has no slot takes one,
// filled from host memory.  The rows handed to the render are then read from
// the resident upper rows, the pool, or host memory for what neither holds.
// The free-slot stack is pushed and popped one workgroup at a time: a
// workgroup counts, claims its total with one atomic, then writes at prefix
// counts of its ballots.
#include "lodgs_internal.h"

struct lodgs_row_pool {
  const lodgs_scene* scene;
  lodgs_cut_cache* cache;
  int32_t sh_degree, n_coef;
  int64_t capacity;
  uint32_t stamp;          // per gather call, marks the selected nodes
  const float* host[5];   // device-visible addresses of the host store
  float* pool;            // [capacity] records (see Groups)
  float* upper;           // [n_upper] records
  int32_t* node_slot;     // [n_nodes] pool slot of a node, -1
  uint32_t* mark;         // [n_nodes] stamp of the last call that selected the node
  int32_t* free_slots;    // [capacity] stack of free slots
  int2* fill;             // [capacity] (node, slot) taken by this call, in pop order
  uint8_t* dirty;         // [capacity] the slot's row was changed by lodgs_row_pool_store
  uint8_t* pooled;        // [n_spt] the SPT's cached cut is in the pool
  uint8_t* act;           // [n_spt] this call: bit 0 release all, bit 1 insert, bit 2 release the unselected
  int2* rel_chunks;       // 64-node chunks of the layout ranges of the SPTs with bit 0 or 2 this call
  int64_t max_chunks;     // chunks of all SPTs together
  unsigned long long* counters;  // see the enum below
};

namespace lodgs {
namespace {

constexpr int kGroups = 5;
// free-stack top (signed), host rows, slots taken, slots given back, pops
// that found the stack empty, rows written back, the top after the releases,
// rows filled this call, chunks listed for release this call
enum { kTop = 0, kHostRows, kInserted, kReleased, kFailed, kWritten, kTop0, kFill, kList, kCounters };

// A row in the pool (and a resident upper row) is one record of rec floats,
// read by 16 lanes as float4s: [SH (wsh floats, zero-padded to s4)]
// [quaternion] [mean x, y, z, log-scale 0] [log-scale 1, 2, opacity logit, 0].
// Host memory and the rows handed out keep one array per group.
struct Groups {
  const float* host[kGroups];
  float* hostw[kGroups];
  float* pool;
  float* upper;
  int32_t w[kGroups];
  int32_t s4, rec;
};

__host__ __device__ constexpr int rec_s4(int wsh) { return (wsh + 3) / 4 * 4; }
__host__ __device__ constexpr int rec_floats(int wsh) { return rec_s4(wsh) + 12; }

__device__ __forceinline__ void copy_row(const float* src, float* dst, int w) {
  for (int c = 0; c < w; ++c) dst[c] = src[c];
}

// One record to the host arrays of node / from them (one lane, rare paths).
__device__ void rec_to_host(const Groups& G, const float* r, int64_t node) {
  copy_row(r, G.hostw[4] + node * G.w[4], G.w[4]);
  copy_row(r + G.s4, G.hostw[2] + node * 4, 4);
  copy_row(r + G.s4 + 4, G.hostw[0] + node * 3, 3);
  G.hostw[1][node * 3] = r[G.s4 + 7];
  G.hostw[1][node * 3 + 1] = r[G.s4 + 8];
  G.hostw[1][node * 3 + 2] = r[G.s4 + 9];
  G.hostw[3][node] = r[G.s4 + 10];
}
__device__ void rec_from_host(const Groups& G, int64_t node, float* r) {
  for (int c = 0; c < G.s4; ++c) r[c] = c < G.w[4] ? G.host[4][node * G.w[4] + c] : 0.0f;
  copy_row(G.host[2] + node * 4, r + G.s4, 4);
  copy_row(G.host[0] + node * 3, r + G.s4 + 4, 3);
  r[G.s4 + 7] = G.host[1][node * 3];
  r[G.s4 + 8] = G.host[1][node * 3 + 1];
  r[G.s4 + 9] = G.host[1][node * 3 + 2];
  r[G.s4 + 10] = G.host[3][node];
  r[G.s4 + 11] = 0.0f;
}

// Lowest set lane of a non-zero mask.
__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

// Sum over the wave (every lane gets it).
__device__ __forceinline__ unsigned long long wave_total(unsigned long long v) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Stack and list positions are claimed with one atomic per workgroup of
// kClaimBlock threads over a grid of kClaimGrid: a workgroup counts what its
// waves will push or pop, claims the total, then does the work again and
// writes.  (Atomics on one address are serialised; a claim per wave or per
// small workgroup made them the cost of these kernels.)
constexpr int kClaimBlock = 1024, kClaimGrid = 256;

// Claims cnt (wave-uniform) entries for each wave of the block with a single
// atomic on *ctr (adding the block's total, or subtracting it with pop):
// returns the counter's old value and the counts of the lower waves.
// Contains barriers: call from every thread of the block.
struct Claim {
  unsigned long long old, below;
};
__device__ __forceinline__ Claim block_claim(unsigned long long* ctr, unsigned long long cnt, bool pop,
                                             unsigned long long* sh) {
  const int nwaves = (int)(blockDim.x >> 6), wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < nwaves; ++w) tot += sh[w];
    sh[nwaves] = tot ? atomicAdd(ctr, pop ? 0ull - tot : tot) : 0ull;
  }
  __syncthreads();
  Claim c{sh[nwaves], 0ull};
  for (int w = 0; w < wave; ++w) c.below += sh[w];
  return c;
}

// Adds the block's sum of v (wave-uniform) to *ctr with one atomic, if not
// zero.  Contains barriers: call from every thread of the block.
__device__ __forceinline__ void block_add(unsigned long long* ctr, unsigned long long v, unsigned long long* sh) {
  const int nwaves = (int)(blockDim.x >> 6);
  __syncthreads();  // sh may still be read by an earlier claim
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < nwaves; ++w) tot += sh[w];
    if (tot) atomicAdd(ctr, tot);
  }
}

// Exclusive prefix sum over the wave (lane order) and the wave's total.
__device__ __forceinline__ uint32_t wave_exclusive(uint32_t v, uint32_t* total) {
  const int lane = threadIdx.x & 63;
  uint32_t x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

// Per SPT: release all when pooled and no longer cached; release the nodes
// the new cut dropped and insert when pooled and cut afresh; insert when
// cached, visible and not pooled.  The 64-node chunks of the layout ranges of
// the SPTs to release are listed as (first node, length | 128 when all go).
__global__ void __launch_bounds__(kClaimBlock) k_pool_classify(int64_t n_spt, const int32_t* spt_begin,
                                                               const uint8_t* cached, const uint8_t* vstate,
                                                               uint8_t* pooled, uint8_t* act, int2* rel_chunks,
                                                               unsigned long long* counters) {
  __shared__ unsigned long long sh[kClaimBlock / 64 + 1];
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t w0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  unsigned long long cnt = 0;  // wave-uniform
  for (int64_t j0 = w0; j0 < n_spt; j0 += stride) {  // wave-uniform
    const int64_t j = j0 + lane;
    uint32_t nch = 0;
    if (j < n_spt) {
      const bool in = pooled[j] != 0, c = cached[j] != 0;
      const bool drop = in && !c, recut = in && c && vstate[j] == 2;
      const bool ins = c && vstate[j] != 0 && (!in || recut);
      act[j] = (uint8_t)((drop ? 1 : 0) | (ins ? 2 : 0) | (recut ? 4 : 0));
      pooled[j] = (uint8_t)(c && (in || ins) ? 1 : 0);
      if (drop || recut) nch = (uint32_t)((spt_begin[j + 1] - spt_begin[j] + 63) / 64);
    }
    uint32_t tot;
    wave_exclusive(nch, &tot);
    cnt += tot;
  }
  const Claim c = block_claim(&counters[kList], cnt, false, sh);
  unsigned long long pos = c.old + c.below;
  for (int64_t j0 = w0; j0 < n_spt; j0 += stride) {  // wave-uniform; this lane wrote act[j] above
    const int64_t j = j0 + lane;
    const uint8_t a = j < n_spt ? act[j] : 0;
    uint32_t nch = 0;
    int32_t beg = 0, end = 0;
    if (a & 5u) {
      beg = spt_begin[j];
      end = spt_begin[j + 1];
      nch = (uint32_t)((end - beg + 63) / 64);
    }
    uint32_t tot;
    const uint32_t off = wave_exclusive(nch, &tot);
    for (uint32_t q = 0; q < nch; ++q) {
      const int32_t b = beg + 64 * (int32_t)q;
      const int32_t len = end - b < 64 ? end - b : 64;
      rel_chunks[(int64_t)pos + off + q] = make_int2(b, len | ((a & 1u) ? 128 : 0));
    }
    pos += tot;
  }
}

// Stamps every selected node below the upper hierarchy.
__global__ void __launch_bounds__(kBlock) k_pool_mark(const int32_t* idx, const int32_t* d_count, int64_t cap,
                                                      int32_t n_upper, uint32_t* mark, uint32_t stamp) {
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t node = idx[k];
    if (node >= n_upper) mark[node] = stamp;
  }
}

// One wave per listed chunk (the list in turn): every slotted node of the
// chunk (an SPT dropped), or every one not stamped by this call (an SPT cut
// afresh), gives its slot back, a changed row written back to host memory
// first.
__global__ void __launch_bounds__(kClaimBlock) k_pool_release(const int2* rel_chunks, int32_t* node_slot,
                                                              const uint32_t* mark, uint32_t stamp,
                                                              int32_t* free_slots, uint8_t* dirty,
                                                              unsigned long long* counters, Groups G) {
  __shared__ unsigned long long sh[kClaimBlock / 64 + 1];
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  const int64_t n_list = (int64_t)counters[kList];
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  unsigned long long cnt = 0, wb = 0;  // wave-uniform
  for (int64_t l = w0; l < n_list; l += nw) {  // wave-uniform
    const int2 ch = rel_chunks[l];
    const int64_t node = (int64_t)ch.x + lane;
    const int32_t s = lane < (ch.y & 127) ? node_slot[node] : -1;
    cnt += (unsigned long long)__popcll(__ballot(s >= 0 && ((ch.y & 128) || mark[node] != stamp)));
  }
  const Claim c = block_claim(&counters[kTop], cnt, false, sh);
  unsigned long long pos = c.old + c.below;
  for (int64_t l = w0; l < n_list; l += nw) {  // wave-uniform
    const int2 ch = rel_chunks[l];
    const int64_t node = (int64_t)ch.x + lane;
    const int32_t s = lane < (ch.y & 127) ? node_slot[node] : -1;
    const bool f = s >= 0 && ((ch.y & 128) || mark[node] != stamp);
    const bool wr = f && dirty[s];
    if (wr) {
      rec_to_host(G, G.pool + (int64_t)s * G.rec, node);
      dirty[s] = 0;
    }
    wb += (unsigned long long)__popcll(__ballot(wr));
    const uint64_t m = __ballot(f);
    if (f) {
      node_slot[node] = -1;
      free_slots[(int64_t)pos + __popcll(m & lt)] = s;
    }
    pos += (unsigned long long)__popcll(m);
  }
  block_add(&counters[kReleased], cnt, sh);
  block_add(&counters[kWritten], wb, sh);
}

// The SPT holding layout position node (>= n_upper): the last j with
// spt_begin[j] <= node.
__device__ __forceinline__ int64_t spt_of(const int32_t* spt_begin, int64_t n_spt, int64_t node) {
  int64_t lo = 0, hi = n_spt;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (spt_begin[mid] <= node) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Every selected node of an SPT to insert that has no slot pops one; the
// (node, slot) pairs go to the fill list at (top after the releases) - 1 -
// (stack position), so the list is dense in pop order.  A pool without a free
// slot leaves the node out (counted; its row is read from host memory).
__device__ __forceinline__ bool wants_slot(const int32_t* idx, int64_t k, int64_t n, int32_t n_upper,
                                           const int32_t* spt_begin, int64_t n_spt, const uint8_t* act,
                                           const int32_t* node_slot, int64_t* node) {
  *node = k < n ? idx[k] : -1;
  if (*node < n_upper || node_slot[*node] >= 0) return false;  // most selected nodes hold a slot
  return (act[spt_of(spt_begin, n_spt, *node)] & 2u) != 0;
}

__global__ void __launch_bounds__(kClaimBlock) k_pool_insert(const int32_t* idx, const int32_t* d_count, int64_t cap,
                                                             int32_t n_upper, const int32_t* spt_begin, int64_t n_spt,
                                                             const uint8_t* act, int32_t* node_slot,
                                                             const int32_t* free_slots, uint8_t* dirty, int2* fill,
                                                             unsigned long long* counters) {
  __shared__ unsigned long long sh[kClaimBlock / 64 + 1];
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  const long long top0 = (long long)counters[kTop0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t w0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  unsigned long long cnt = 0, fail = 0;  // wave-uniform
  int64_t node;
  for (int64_t k0 = w0; k0 < n; k0 += stride)  // wave-uniform
    cnt += (unsigned long long)__popcll(
        __ballot(wants_slot(idx, k0 + lane, n, n_upper, spt_begin, n_spt, act, node_slot, &node)));
  const Claim c = block_claim(&counters[kTop], cnt, true, sh);
  long long p0 = (long long)c.old - 1 - (long long)c.below;  // this wave's first stack position
  for (int64_t k0 = w0; k0 < n; k0 += stride) {  // wave-uniform
    const bool want = wants_slot(idx, k0 + lane, n, n_upper, spt_begin, n_spt, act, node_slot, &node);
    const uint64_t m = __ballot(want);
    const long long p = p0 - __popcll(m & lt);
    if (want && p >= 0) {
      const int32_t s = free_slots[p];
      dirty[s] = 0;
      node_slot[node] = s;
      fill[top0 - 1 - p] = make_int2((int)node, s);
    }
    fail += (unsigned long long)__popcll(__ballot(want && p < 0));
    p0 -= __popcll(m);
  }
  block_add(&counters[kFailed], fail, sh);
}

// Phase 0: clears the per-call counters.  Phase 1 (after the releases): keeps
// the stack top.  Phase 2 (after the pops): clamps the top at 0 and counts the
// slots taken.
__global__ void k_pool_counters(unsigned long long* counters, int phase) {
  if (phase == 0) {
    counters[kHostRows] = 0;
    counters[kInserted] = 0;
    counters[kReleased] = 0;
    counters[kList] = 0;
  } else if (phase == 1) {
    counters[kTop0] = counters[kTop];
  } else {
    long long top = (long long)counters[kTop];
    if (top < 0) top = 0;
    counters[kTop] = (unsigned long long)top;
    counters[kFill] = counters[kTop0] - (unsigned long long)top;
    counters[kInserted] = counters[kFill];
    counters[kHostRows] = counters[kFill];
  }
}

// Float4 c of row `from` of the group arrays src, as the record lays it out.
template <int WSH, typename Src>
__device__ __forceinline__ float4 rec_chunk(int c, const Src& src, int64_t from) {
  constexpr int S = rec_s4(WSH) / 4;
  if (c < S) {
    if (WSH % 4 == 0) return reinterpret_cast<const float4*>(src[4] + from * WSH)[c];
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = 4 * c + i < WSH ? src[4][from * WSH + 4 * c + i] : 0.0f;
    return make_float4(v[0], v[1], v[2], v[3]);
  }
  if (c == S) return reinterpret_cast<const float4*>(src[2])[from];
  if (c == S + 1) return make_float4(src[0][from * 3], src[0][from * 3 + 1], src[0][from * 3 + 2], src[1][from * 3]);
  return make_float4(src[1][from * 3 + 1], src[1][from * 3 + 2], src[3][from], 0.0f);
}

// Float4 c of a record into row `to` of the group arrays dst.
template <int WSH, typename Dst>
__device__ __forceinline__ void rec_chunk_out(int c, float4 v, const Dst& dst, int64_t to) {
  constexpr int S = rec_s4(WSH) / 4;
  if (c < S) {
    if (WSH % 4 == 0) {
      reinterpret_cast<float4*>(dst[4] + to * WSH)[c] = v;
    } else {
      const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * c + i < WSH) dst[4][to * WSH + 4 * c + i] = x[i];
    }
  } else if (c == S) {
    reinterpret_cast<float4*>(dst[2])[to] = v;
  } else if (c == S + 1) {
    dst[0][to * 3] = v.x;
    dst[0][to * 3 + 1] = v.y;
    dst[0][to * 3 + 2] = v.z;
    dst[1][to * 3] = v.w;
  } else {
    dst[1][to * 3 + 1] = v.x;
    dst[1][to * 3 + 2] = v.y;
    dst[3][to] = v.z;
  }
}

// The slots taken this call, filled from host memory, 16 lanes per row.
template <int WSH>
__global__ void __launch_bounds__(kBlock) k_pool_fill(const int2* fill, const unsigned long long* counters, Groups G) {
  constexpr int Q = rec_floats(WSH) / 4;
  const int64_t n = (int64_t)counters[kFill];
  const int64_t stride = ((int64_t)gridDim.x * blockDim.x) >> 4;
  const int t = threadIdx.x & 15;
  for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4; k < n; k += stride) {
    const int2 ns = fill[k];
    float4* r = reinterpret_cast<float4*>(G.pool + (int64_t)ns.y * rec_floats(WSH));
    for (int c = t; c < Q; c += 16) r[c] = rec_chunk<WSH>(c, G.host, ns.x);
  }
}

// Row k of every group for selected node idx[k], 16 lanes per row: from the
// record of a resident upper row or of a pool slot (one float4 per lane), or
// from host memory (a node without a slot, counted).
template <int WSH>
__global__ void __launch_bounds__(kBlock) k_pool_assemble(const int32_t* idx, const int32_t* d_count, int64_t cap,
                                                          int32_t n_upper, const int32_t* node_slot, Groups G,
                                                          lodgs_grads rows, unsigned long long* counters) {
  constexpr int Q = rec_floats(WSH) / 4;
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  float* const dst[kGroups] = {rows.d_means, rows.d_log_scales, rows.d_quats, rows.d_opacity_logits, rows.d_sh};
  const int64_t stride = ((int64_t)gridDim.x * blockDim.x) >> 4;
  const int t = threadIdx.x & 15;
  unsigned long long from_host = 0;
  for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4; k < n; k += stride) {
    const int64_t node = idx[k];
    const int32_t s = node < n_upper ? -1 : node_slot[node];
    if (node < n_upper || s >= 0) {
      const float4* r = reinterpret_cast<const float4*>(node < n_upper ? G.upper + node * rec_floats(WSH)
                                                                       : G.pool + (int64_t)s * rec_floats(WSH));
      for (int c = t; c < Q; c += 16) rec_chunk_out<WSH>(c, r[c], dst, k);
    } else {
      for (int c = t; c < Q; c += 16) rec_chunk_out<WSH>(c, rec_chunk<WSH>(c, G.host, node), dst, k);
      from_host += t == 0;
    }
  }
  from_host = wave_total(from_host);
  if ((threadIdx.x & 63) == 0 && from_host) atomicAdd(&counters[kHostRows], from_host);
}

// Trained rows back, 16 lanes per row: to the pool slot (marked changed) of a
// pooled node, to the resident upper record and host memory of an upper node,
// to host memory otherwise.
template <int WSH>
__global__ void __launch_bounds__(kBlock) k_pool_store(const int32_t* idx, const int32_t* d_count, int64_t cap,
                                                       int32_t n_upper, const int32_t* node_slot, uint8_t* dirty,
                                                       Groups G, lodgs_grads rows) {
  constexpr int Q = rec_floats(WSH) / 4;
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const float* const src[kGroups] = {rows.d_means, rows.d_log_scales, rows.d_quats, rows.d_opacity_logits, rows.d_sh};
  const int64_t stride = ((int64_t)gridDim.x * blockDim.x) >> 4;
  const int t = threadIdx.x & 15;
  for (int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4; k < n; k += stride) {
    const int64_t node = idx[k];
    const int32_t s = node < n_upper ? -1 : node_slot[node];
    for (int c = t; c < Q; c += 16) {
      const float4 v = rec_chunk<WSH>(c, src, k);
      if (node < n_upper) {
        reinterpret_cast<float4*>(G.upper + node * rec_floats(WSH))[c] = v;
        rec_chunk_out<WSH>(c, v, G.hostw, node);
      } else if (s >= 0) {
        reinterpret_cast<float4*>(G.pool + (int64_t)s * rec_floats(WSH))[c] = v;
      } else {
        rec_chunk_out<WSH>(c, v, G.hostw, node);
      }
    }
    if (s >= 0 && t == 0) dirty[s] = 1;
  }
}

// Every changed pooled row back to host memory (the rows stay pooled, no
// longer marked changed): one thread per node below the upper hierarchy.
__global__ void __launch_bounds__(kBlock) k_pool_write_back(int64_t n_upper, int64_t n_nodes,
                                                            const int32_t* node_slot, uint8_t* dirty,
                                                            unsigned long long* counters, Groups G) {
  unsigned long long wb = 0;
  for (int64_t node = n_upper + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; node < n_nodes;
       node += (int64_t)gridDim.x * blockDim.x) {
    const int32_t s = node_slot[node];
    if (s < 0 || !dirty[s]) continue;
    rec_to_host(G, G.pool + (int64_t)s * G.rec, node);
    dirty[s] = 0;
    ++wb;
  }
  wb = wave_total(wb);
  if ((threadIdx.x & 63) == 0 && wb) atomicAdd(&counters[kWritten], wb);
}

__global__ void __launch_bounds__(kBlock) k_pool_init(int32_t* node_slot, uint32_t* mark, int64_t n_nodes,
                                                      int32_t* free_slots, uint8_t* dirty, int64_t capacity) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes; i += stride) {
    node_slot[i] = -1;
    mark[i] = 0;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < capacity; i += stride) {
    free_slots[i] = (int32_t)(capacity - 1 - i);
    dirty[i] = 0;
  }
}

// The upper hierarchy's records (layout positions below n_upper), from host memory.
__global__ void __launch_bounds__(kBlock) k_pool_upper(int64_t n_upper, Groups G) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n_upper; u += (int64_t)gridDim.x * blockDim.x)
    rec_from_host(G, u, G.upper + u * G.rec);
}

int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

Groups groups_of(const lodgs_row_pool* p) {
  Groups G;
  const int32_t w[kGroups] = {3, 3, 4, 1, p->n_coef};
  for (int g = 0; g < kGroups; ++g) {
    G.host[g] = p->host[g];
    G.hostw[g] = const_cast<float*>(p->host[g]);
    G.w[g] = w[g];
  }
  G.pool = p->pool;
  G.upper = p->upper;
  G.s4 = rec_s4(p->n_coef);
  G.rec = rec_floats(p->n_coef);
  return G;
}

void free_pool(lodgs_row_pool* p) {
  if (!p) return;
  void* ptrs[] = {p->pool, p->upper, p->node_slot, p->mark, p->free_slots, p->fill, p->dirty, p->pooled, p->act, p->rel_chunks,
                  p->counters};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
}

const float* pinned_device_address(const float* h) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, h) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
  return static_cast<const float*>(a.devicePointer);
}

// Every group present, and the groups read as float4s (quaternions, SH rows)
// 16-byte aligned.
bool rows_ok(const lodgs_grads* r) {
  const float* m[kGroups] = {r->d_means, r->d_log_scales, r->d_quats, r->d_opacity_logits, r->d_sh};
  for (const float* q : m)
    if (!q) return false;
  return ((reinterpret_cast<uintptr_t>(r->d_quats) | reinterpret_cast<uintptr_t>(r->d_sh)) & 15u) == 0;
}

}  // namespace
}  // namespace lodgs

using lodgs::hip_fail;
using lodgs::set_error;

extern "C" {

int lodgs_row_pool_create(lodgs_cut_cache* cache, const lodgs_grads* host, int32_t sh_degree, int64_t capacity,
                          lodgs_row_pool** out) {
  using namespace lodgs;
  if (!cache || !host || !out) return set_error(LODGS_E_INVALID, "lodgs_row_pool_create: null argument");
  *out = nullptr;
  const lodgs_scene* scene = cache->scene;
  if (sh_degree != scene->dev.sh_degree) return set_error(LODGS_E_INVALID, "lodgs_row_pool_create: sh_degree");
  if (capacity < cache->prm.max_nodes || capacity > (int64_t)INT32_MAX)
    return set_error(LODGS_E_INVALID,
                     "lodgs_row_pool_create: capacity must hold the cache's max_nodes (and fit int32)");
  if (!rows_ok(host))
    return set_error(LODGS_E_INVALID, "lodgs_row_pool_create: every parameter group is needed, 16-byte aligned");
  lodgs_row_pool* p = new (std::nothrow) lodgs_row_pool();
  if (!p) return set_error(LODGS_E_OOM, "lodgs_row_pool_create: out of host memory");
  p->scene = scene;
  p->cache = cache;
  p->sh_degree = sh_degree;
  p->n_coef = scene->dev.n_coef;
  p->capacity = capacity;
  const float* src[kGroups] = {host->d_means, host->d_log_scales, host->d_quats, host->d_opacity_logits, host->d_sh};
  for (int g = 0; g < kGroups; ++g) {
    p->host[g] = pinned_device_address(src[g]);
    if (!p->host[g]) {
      free_pool(p);
      return set_error(LODGS_E_INVALID, "lodgs_row_pool_create: a host array is not pinned host memory");
    }
  }
  if (((reinterpret_cast<uintptr_t>(p->host[2]) | reinterpret_cast<uintptr_t>(p->host[4])) & 15u) != 0) {
    free_pool(p);
    return set_error(LODGS_E_INVALID, "lodgs_row_pool_create: quaternion and SH arrays must be 16-byte aligned");
  }
  const size_t n_nodes = (size_t)scene->dev.n_nodes, n_spt = (size_t)scene->dev.n_spt;
  const size_t n_up = (size_t)scene->dev.n_upper;
  const size_t rec = sizeof(float) * (size_t)rec_floats(p->n_coef);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->pool), rec * (size_t)(capacity > 0 ? capacity : 1));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->upper), rec * (n_up > 0 ? n_up : 1));
  const size_t cap1 = (size_t)(capacity > 0 ? capacity : 1);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->node_slot), sizeof(int32_t) * n_nodes);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->mark), sizeof(uint32_t) * n_nodes);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->free_slots), sizeof(int32_t) * cap1);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->fill), sizeof(int2) * cap1);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->dirty), cap1);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->pooled), n_spt);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->act), n_spt);
  // every SPT's chunks: at most (layout range)/64 + 1 each
  p->max_chunks = (int64_t)((n_nodes - n_up) / 64 + n_spt + 1);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->rel_chunks), sizeof(int2) * (size_t)p->max_chunks);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->counters), sizeof(unsigned long long) * kCounters);
  if (e != hipSuccess) {
    free_pool(p);
    (void)hipGetLastError();
    return set_error(LODGS_E_OOM, "lodgs_row_pool_create: device allocation failed");
  }
  unsigned long long c0[kCounters] = {(unsigned long long)capacity};
  e = hipMemcpy(p->counters, c0, sizeof c0, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p->pooled, 0, n_spt);
  if (e == hipSuccess) {
    const Groups G = groups_of(p);
    hipLaunchKernelGGL(k_pool_init, dim3(grid_for((int64_t)n_nodes)), dim3(kBlock), 0, 0, p->node_slot, p->mark,
                       (int64_t)n_nodes, p->free_slots, p->dirty, capacity);
    hipLaunchKernelGGL(k_pool_upper, dim3(grid_for((int64_t)n_up)), dim3(kBlock), 0, 0, (int64_t)n_up, G);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    free_pool(p);
    return hip_fail(e, "lodgs_row_pool_create");
  }
  *out = p;
  return LODGS_OK;
}

void lodgs_row_pool_destroy(lodgs_row_pool* p) { lodgs::free_pool(p); }

int lodgs_gather_rows_pooled(lodgs_row_pool* p, const int32_t* d_idx, const int32_t* d_count, const lodgs_grads* rows,
                             int64_t capacity, lodgs_stream stream) {
  using namespace lodgs;
  if (!p || !d_idx || !d_count || !rows || !rows_ok(rows))
    return set_error(LODGS_E_INVALID, "lodgs_gather_rows_pooled: null argument or misaligned rows");
  if (capacity < 0) return set_error(LODGS_E_INVALID, "lodgs_gather_rows_pooled: capacity");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const SceneDev& S = p->scene->dev;
  const Groups G = groups_of(p);
  const int64_t n_spt = S.n_spt;
  if (++p->stamp == 0) {  // the stamps wrapped: no node may carry a live one
    const hipError_t e = hipMemsetAsync(p->mark, 0, sizeof(uint32_t) * (size_t)S.n_nodes, st);
    if (e != hipSuccess) return hip_fail(e, "lodgs_gather_rows_pooled");
    p->stamp = 1;
  }
  const uint32_t stamp = p->stamp;
  hipLaunchKernelGGL(k_pool_counters, dim3(1), dim3(1), 0, st, p->counters, 0);
  hipLaunchKernelGGL(k_pool_classify, dim3(kClaimGrid), dim3(kClaimBlock), 0, st, n_spt, S.spt_begin,
                     p->cache->cached, p->cache->vstate, p->pooled, p->act, p->rel_chunks, p->counters);
  hipLaunchKernelGGL(k_pool_mark, dim3(grid_for(capacity)), dim3(kBlock), 0, st, d_idx, d_count, capacity, S.n_upper,
                     p->mark, stamp);
  hipLaunchKernelGGL(k_pool_release, dim3(kClaimGrid), dim3(kClaimBlock), 0, st, p->rel_chunks, p->node_slot,
                     p->mark, stamp, p->free_slots, p->dirty, p->counters, G);
  hipLaunchKernelGGL(k_pool_counters, dim3(1), dim3(1), 0, st, p->counters, 1);
  hipLaunchKernelGGL(k_pool_insert, dim3(kClaimGrid), dim3(kClaimBlock), 0, st, d_idx, d_count, capacity,
                     S.n_upper, S.spt_begin, n_spt, p->act, p->node_slot, p->free_slots, p->dirty, p->fill,
                     p->counters);
  hipLaunchKernelGGL(k_pool_counters, dim3(1), dim3(1), 0, st, p->counters, 2);
  // 16 lanes per row; the fill's grid sized for every slot one call can take
  const int64_t fill_max = p->capacity < capacity ? p->capacity : capacity;
#define LODGS_POOL(WSH)                                                                                              \
  hipLaunchKernelGGL(k_pool_fill<WSH>, dim3(grid_for(16 * fill_max)), dim3(kBlock), 0, st, p->fill, p->counters, G); \
  hipLaunchKernelGGL(k_pool_assemble<WSH>, dim3(grid_for(16 * capacity)), dim3(kBlock), 0, st, d_idx, d_count,       \
                     capacity, S.n_upper, p->node_slot, G, *rows, p->counters)
  switch (p->n_coef) {  // floats per SH row: 3 (sh_degree + 1)^2
    case 3: LODGS_POOL(3); break;
    case 12: LODGS_POOL(12); break;
    case 27: LODGS_POOL(27); break;
    default: LODGS_POOL(48); break;
  }
#undef LODGS_POOL
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_gather_rows_pooled");
}

int lodgs_row_pool_store(lodgs_row_pool* p, const int32_t* d_idx, const int32_t* d_count, const lodgs_grads* rows,
                         int64_t capacity, lodgs_stream stream) {
  using namespace lodgs;
  if (!p || !d_idx || !d_count || !rows || !rows_ok(rows))
    return set_error(LODGS_E_INVALID, "lodgs_row_pool_store: null argument or misaligned rows");
  if (capacity < 0) return set_error(LODGS_E_INVALID, "lodgs_row_pool_store: capacity");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const lodgs_scene* sc = p->scene;
  const Groups G = groups_of(p);
#define LODGS_STORE(WSH)                                                                                         \
  hipLaunchKernelGGL(k_pool_store<WSH>, dim3(grid_for(16 * capacity)), dim3(kBlock), 0, st, d_idx, d_count,    \
                     capacity, sc->dev.n_upper, p->node_slot, p->dirty, G, *rows)
  switch (p->n_coef) {  // floats per SH row: 3 (sh_degree + 1)^2
    case 3: LODGS_STORE(3); break;
    case 12: LODGS_STORE(12); break;
    case 27: LODGS_STORE(27); break;
    default: LODGS_STORE(48); break;
  }
#undef LODGS_STORE
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_row_pool_store");
}

int lodgs_row_pool_write_back(lodgs_row_pool* p, lodgs_stream stream) {
  using namespace lodgs;
  if (!p) return set_error(LODGS_E_INVALID, "lodgs_row_pool_write_back: null argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const SceneDev& S = p->scene->dev;
  hipLaunchKernelGGL(k_pool_write_back, dim3(4096), dim3(kBlock), 0, st, (int64_t)S.n_upper, (int64_t)S.n_nodes,
                     p->node_slot, p->dirty, p->counters, groups_of(p));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_row_pool_write_back");
}

int lodgs_row_pool_stats_read(lodgs_row_pool* p, lodgs_row_pool_stats* out, int32_t* d_node_slot_copy,
                              lodgs_stream stream) {
  using namespace lodgs;
  if (!p || !out) return set_error(LODGS_E_INVALID, "lodgs_row_pool_stats_read: null argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unsigned long long c[kCounters];
  hipError_t e = hipMemcpyAsync(c, p->counters, sizeof c, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && d_node_slot_copy)
    e = hipMemcpyAsync(d_node_slot_copy, p->node_slot, sizeof(int32_t) * (size_t)p->scene->dev.n_nodes,
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "lodgs_row_pool_stats_read");
  out->capacity = p->capacity;
  out->pooled_rows = p->capacity - (int64_t)c[kTop];
  out->host_rows = (int64_t)c[kHostRows];
  out->inserted = (int64_t)c[kInserted];
  out->released = (int64_t)c[kReleased];
  out->insert_failures = (int64_t)c[kFailed];
  out->written_back = (int64_t)c[kWritten];
  return LODGS_OK;
}

}  // extern "C"
