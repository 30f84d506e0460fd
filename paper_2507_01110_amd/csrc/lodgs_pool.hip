// Device pool of the rows of cached SPT cuts (Sec. 4.4 "Caching on the GPU":
// the Gaussians of a cached cut stay in VRAM; Alg. 3: Load from RAM, cache
// insert, write-back of evicted entries).  The parameters live in pinned host
// memory; the upper hierarchy's rows are kept resident (Alg. 3 renders them
// every iteration); the rows of every SPT entry of an SPT-cut cache occupy
// pool slots, one per selected node of its cached cut, so a cache hit reads
// nothing over the host link.  After each lodgs_lod_select_cached, for every
// SPT: an entry that was reloaded (a cache miss) or dropped gives its slots
// back (writing back the rows that lodgs_row_pool_store changed); a cached
// entry that is visible and not pooled takes slots for its selected nodes,
// filled from host memory.  The rows handed to the render are then read from
// the resident upper rows, the pool, or host memory for what neither holds.
#include "lodgs_internal.h"

struct lodgs_row_pool {
  const lodgs_scene* scene;
  lodgs_cut_cache* cache;
  int32_t sh_degree, n_coef;
  int64_t capacity;
  const float* host[5];   // device-visible addresses of the host store
  float* pool[5];         // [capacity][w]
  float* upper[5];        // [n_upper][w]
  int32_t* node_slot;     // [n_nodes] pool slot of a node, -1
  int32_t* free_slots;    // [capacity] stack of free slots
  uint8_t* dirty;         // [capacity] the slot's row was changed by lodgs_row_pool_store
  uint8_t* fresh;         // [capacity] the slot was taken this view and is filled by the assembly
  uint8_t* pooled;        // [n_spt] the SPT's cached cut is in the pool
  uint8_t* act;           // [n_spt] this view: bit 0 release, bit 1 insert
  unsigned long long* counters;  // free-stack top (signed), host rows, inserted, released, insert failures,
                                 // written back
};

namespace lodgs {
namespace {

constexpr int kGroups = 5;
enum { kTop = 0, kHostRows = 1, kInserted = 2, kReleased = 3, kFailed = 4, kWritten = 5, kCounters = 6 };

struct Groups {
  const float* host[kGroups];
  float* hostw[kGroups];
  float* pool[kGroups];
  float* upper[kGroups];
  int32_t w[kGroups];
};

__device__ __forceinline__ void copy_row(const float* src, float* dst, int w) {
  for (int c = 0; c < w; ++c) dst[c] = src[c];
}

// Per SPT: release when pooled and reloaded or no longer cached; insert when
// cached, visible and not (still) pooled.
__global__ void __launch_bounds__(kBlock) k_pool_classify(int64_t n_spt, const uint8_t* cached, const uint8_t* vstate,
                                                          uint8_t* pooled, uint8_t* act) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_spt; j += (int64_t)gridDim.x * blockDim.x) {
    const bool in = pooled[j] != 0, c = cached[j] != 0;
    const bool rel = in && (!c || vstate[j] == 2);
    const bool keep = in && !rel;
    const bool ins = c && vstate[j] != 0 && !keep;
    act[j] = (uint8_t)((rel ? 1 : 0) | (ins ? 2 : 0));
    pooled[j] = (uint8_t)(keep || ins ? 1 : 0);
  }
}

// One wave per SPT to release: every pooled node of its layout range gives
// its slot back (changed rows written back to host memory first).
__global__ void __launch_bounds__(kBlock) k_pool_release(int64_t n_spt, const uint8_t* act, const int32_t* spt_begin,
                                                         int32_t* node_slot, int32_t* free_slots, uint8_t* dirty,
                                                         unsigned long long* counters, Groups G) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  unsigned long long rel = 0, wb = 0;
  for (int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; j < n_spt; j += nw) {  // wave-uniform
    if (!(act[j] & 1u)) continue;
    for (int64_t node = spt_begin[j] + lane; node < spt_begin[j + 1]; node += 64) {
      const int32_t s = node_slot[node];
      if (s < 0) continue;
      if (dirty[s]) {
        for (int g = 0; g < kGroups; ++g)
          copy_row(G.pool[g] + (int64_t)s * G.w[g], G.hostw[g] + node * G.w[g], G.w[g]);
        dirty[s] = 0;
        ++wb;
      }
      node_slot[node] = -1;
      free_slots[(int64_t)atomicAdd(&counters[kTop], 1ull)] = s;
      ++rel;
    }
  }
  if (rel) atomicAdd(&counters[kReleased], rel);
  if (wb) atomicAdd(&counters[kWritten], wb);
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

// Per selected node of an SPT to insert: a slot from the free stack (the
// assembly fills it from host memory).  A pool without a free slot leaves the
// node out (counted).
__global__ void __launch_bounds__(kBlock) k_pool_insert(const int32_t* idx, const int32_t* d_count, int64_t cap,
                                                        int32_t n_upper, const int32_t* spt_begin, int64_t n_spt,
                                                        const uint8_t* act, int32_t* node_slot,
                                                        const int32_t* free_slots, uint8_t* dirty, uint8_t* fresh,
                                                        unsigned long long* counters) {
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  unsigned long long ins = 0, fail = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = idx[k];
    if (node < n_upper) continue;
    const int64_t j = spt_of(spt_begin, n_spt, node);
    if (!(act[j] & 2u) || node_slot[node] >= 0) continue;
    const int64_t p = (int64_t)atomicAdd(&counters[kTop], ~0ull) - 1;  // pop (the top is signed)
    if (p < 0) {
      ++fail;
      continue;
    }
    const int32_t s = free_slots[p];
    dirty[s] = 0;
    fresh[s] = 1;
    node_slot[node] = s;
    ++ins;
  }
  if (ins) atomicAdd(&counters[kInserted], ins);
  if (fail) atomicAdd(&counters[kFailed], fail);
}

// Clamps the stack top at 0 after pops that found it empty; clears the
// per-view counters first when `begin`.
__global__ void k_pool_counters(unsigned long long* counters, int begin) {
  if (begin) {
    counters[kHostRows] = 0;
    counters[kInserted] = 0;
    counters[kReleased] = 0;
  } else if ((long long)counters[kTop] < 0) {
    counters[kTop] = 0;
  }
}

// Row k of one group (W floats) for selected node idx[k], one thread per
// (row, chunk) so that neighbouring threads read neighbouring bytes: from the
// resident upper rows, the pool, or host memory (a node without a slot, or
// whose slot was taken this view: then the slot is filled too).  Group 0
// counts the rows read from host memory.
template <int W>
__global__ void __launch_bounds__(kBlock) k_pool_assemble(const int32_t* idx, const int32_t* d_count, int64_t cap,
                                                          int32_t n_upper, const int32_t* node_slot,
                                                          const uint8_t* fresh, const float* host, float* pool,
                                                          const float* upper, float* dst,
                                                          unsigned long long* counters) {
  constexpr int V = W % 4 == 0 ? 4 : 1, C = W / V;
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  unsigned long long from_host = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * C; e += stride) {
    const int64_t k = e / C;
    const int c = (int)(e - k * C);
    const int64_t node = idx[k];
    const int32_t s = node < n_upper ? -1 : node_slot[node];
    const bool up = node < n_upper, hot = s >= 0 && !fresh[s];
    const float* src = up ? upper + node * W : (hot ? pool + (int64_t)s * W : host + node * W);
    if (V == 4) {
      const float4 x = reinterpret_cast<const float4*>(src)[c];
      reinterpret_cast<float4*>(dst + k * W)[c] = x;
      if (s >= 0 && !hot) reinterpret_cast<float4*>(pool + (int64_t)s * W)[c] = x;
    } else {
      const float x = src[c];
      dst[k * W + c] = x;
      if (s >= 0 && !hot) pool[(int64_t)s * W + c] = x;
    }
    if (counters && c == 0 && !up && !hot) ++from_host;
  }
  if (from_host) atomicAdd(&counters[kHostRows], from_host);
}

// After the assembly: the slots taken this view hold their rows.
__global__ void __launch_bounds__(kBlock) k_pool_settle(const int32_t* idx, const int32_t* d_count, int64_t cap,
                                                        int32_t n_upper, const int32_t* node_slot, uint8_t* fresh) {
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = idx[k];
    if (node < n_upper) continue;
    const int32_t s = node_slot[node];
    if (s >= 0) fresh[s] = 0;
  }
}

// Trained rows back: to the pool slot (marked changed) of a pooled node, to
// the resident upper rows and host memory of an upper node, to host memory
// otherwise.
__global__ void __launch_bounds__(kBlock) k_pool_store(const int32_t* idx, const int32_t* d_count, int64_t cap,
                                                       int32_t n_upper, const int32_t* node_slot, uint8_t* dirty,
                                                       Groups G, lodgs_grads rows) {
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const float* const src[kGroups] = {rows.d_means, rows.d_log_scales, rows.d_quats, rows.d_opacity_logits, rows.d_sh};
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = idx[k];
    const int32_t s = node < n_upper ? -1 : node_slot[node];
    for (int g = 0; g < kGroups; ++g) {
      const float* r = src[g] + k * G.w[g];
      if (node < n_upper) {
        copy_row(r, G.upper[g] + node * G.w[g], G.w[g]);
        copy_row(r, G.hostw[g] + node * G.w[g], G.w[g]);
      } else if (s >= 0) {
        copy_row(r, G.pool[g] + (int64_t)s * G.w[g], G.w[g]);
      } else {
        copy_row(r, G.hostw[g] + node * G.w[g], G.w[g]);
      }
    }
    if (s >= 0) dirty[s] = 1;
  }
}

__global__ void __launch_bounds__(kBlock) k_pool_init(int32_t* node_slot, int64_t n_nodes, int32_t* free_slots,
                                                      uint8_t* dirty, uint8_t* fresh, int64_t capacity) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes; i += stride) node_slot[i] = -1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < capacity; i += stride) {
    free_slots[i] = (int32_t)(capacity - 1 - i);
    dirty[i] = 0;
    fresh[i] = 0;
  }
}

// The upper hierarchy's rows (layout positions below n_upper), from host memory.
__global__ void __launch_bounds__(kBlock) k_pool_upper(int64_t n_upper, Groups G) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n_upper; u += (int64_t)gridDim.x * blockDim.x)
    for (int g = 0; g < kGroups; ++g) copy_row(G.host[g] + u * G.w[g], G.upper[g] + u * G.w[g], G.w[g]);
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
    G.pool[g] = p->pool[g];
    G.upper[g] = p->upper[g];
    G.w[g] = w[g];
  }
  return G;
}

void free_pool(lodgs_row_pool* p) {
  if (!p) return;
  for (int g = 0; g < kGroups; ++g) {
    if (p->pool[g]) (void)hipFree(p->pool[g]);
    if (p->upper[g]) (void)hipFree(p->upper[g]);
  }
  void* ptrs[] = {p->node_slot, p->free_slots, p->dirty, p->fresh, p->pooled, p->act, p->counters};
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
  const int32_t w[kGroups] = {3, 3, 4, 1, p->n_coef};
  const size_t n_nodes = (size_t)scene->dev.n_nodes, n_spt = (size_t)scene->dev.n_spt;
  const size_t n_up = (size_t)scene->dev.n_upper;
  hipError_t e = hipSuccess;
  for (int g = 0; g < kGroups && e == hipSuccess; ++g) {
    e = hipMalloc(reinterpret_cast<void**>(&p->pool[g]), sizeof(float) * w[g] * (size_t)(capacity > 0 ? capacity : 1));
    if (e == hipSuccess)
      e = hipMalloc(reinterpret_cast<void**>(&p->upper[g]), sizeof(float) * w[g] * (n_up > 0 ? n_up : 1));
  }
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->node_slot), sizeof(int32_t) * n_nodes);
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void**>(&p->free_slots), sizeof(int32_t) * (size_t)(capacity > 0 ? capacity : 1));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->dirty), (size_t)(capacity > 0 ? capacity : 1));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->fresh), (size_t)(capacity > 0 ? capacity : 1));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->pooled), n_spt);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->act), n_spt);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->counters), sizeof(unsigned long long) * kCounters);
  if (e != hipSuccess) {
    free_pool(p);
    (void)hipGetLastError();
    return set_error(LODGS_E_OOM, "lodgs_row_pool_create: device allocation failed");
  }
  unsigned long long c0[kCounters] = {(unsigned long long)capacity, 0, 0, 0, 0, 0};
  e = hipMemcpy(p->counters, c0, sizeof c0, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p->pooled, 0, n_spt);
  if (e == hipSuccess) {
    const Groups G = groups_of(p);
    hipLaunchKernelGGL(k_pool_init, dim3(grid_for((int64_t)n_nodes)), dim3(kBlock), 0, 0, p->node_slot,
                       (int64_t)n_nodes, p->free_slots, p->dirty, p->fresh, capacity);
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
  hipLaunchKernelGGL(k_pool_counters, dim3(1), dim3(1), 0, st, p->counters, 1);
  hipLaunchKernelGGL(k_pool_classify, dim3(grid_for(n_spt)), dim3(kBlock), 0, st, n_spt, p->cache->cached,
                     p->cache->vstate, p->pooled, p->act);
  hipLaunchKernelGGL(k_pool_release, dim3(grid_for(64 * n_spt)), dim3(kBlock), 0, st, n_spt, p->act, S.spt_begin,
                     p->node_slot, p->free_slots, p->dirty, p->counters, G);
  hipLaunchKernelGGL(k_pool_insert, dim3(grid_for(capacity)), dim3(kBlock), 0, st, d_idx, d_count, capacity,
                     S.n_upper, S.spt_begin, n_spt, p->act, p->node_slot, p->free_slots, p->dirty, p->fresh,
                     p->counters);
  hipLaunchKernelGGL(k_pool_counters, dim3(1), dim3(1), 0, st, p->counters, 0);
  float* const dst[kGroups] = {rows->d_means, rows->d_log_scales, rows->d_quats, rows->d_opacity_logits, rows->d_sh};
  for (int g = 0; g < kGroups; ++g) {
    unsigned long long* cnt = g == 0 ? p->counters : nullptr;
#define LODGS_ASM(W)                                                                                                 \
  hipLaunchKernelGGL(k_pool_assemble<W>, dim3(grid_for(capacity * (W % 4 == 0 ? W / 4 : W))), dim3(kBlock), 0, st, \
                     d_idx, d_count, capacity, S.n_upper, p->node_slot, p->fresh, G.host[g], G.pool[g], G.upper[g],  \
                     dst[g], cnt)
    switch (G.w[g]) {
      case 1: LODGS_ASM(1); break;
      case 3: LODGS_ASM(3); break;
      case 4: LODGS_ASM(4); break;
      case 12: LODGS_ASM(12); break;
      case 27: LODGS_ASM(27); break;
      default: LODGS_ASM(48); break;
    }
#undef LODGS_ASM
  }
  hipLaunchKernelGGL(k_pool_settle, dim3(grid_for(capacity)), dim3(kBlock), 0, st, d_idx, d_count, capacity,
                     S.n_upper, p->node_slot, p->fresh);
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
  hipLaunchKernelGGL(k_pool_store, dim3(grid_for(capacity)), dim3(kBlock), 0, st, d_idx, d_count, capacity,
                     p->scene->dev.n_upper, p->node_slot, p->dirty, groups_of(p), *rows);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_row_pool_store");
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
