// The GPU cache of SPT cuts (Sec. 4.4 "Caching on the GPU", Eq. 7; the
// training loop of Alg. 3).  Per SPT the cache keeps whether an entry exists,
// the root distance and X it was cut at, its node count and its last use.
// The cut kernels take the ratio test (CacheDev); after the cut one thread per
// SPT enters the loaded SPTs and stamps the visible ones, a stable radix sort
// of (last use, SPT) orders the entries oldest first, a scan of their node
// counts in that order gives what would be left after dropping each prefix,
// and every entry whose remainder still exceeds the budget is dropped.
#include "lodgs_internal.h"


namespace lodgs {
namespace {

__global__ void __launch_bounds__(kBlock) k_cache_flush(uint8_t* cached, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    cached[j] = 0;
}

__device__ __forceinline__ void block_add(unsigned long long* dst, unsigned long long x) {
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  if ((threadIdx.x & 63) == 0 && x) atomicAdd(dst, x);
}

// Enters the loaded SPTs, stamps every visible one with iteration t, counts
// hits and loads, and writes the sort keys (last use <= t; absent entries
// t + 1, so they sort last and the keys need only the bits of t + 1).
__global__ void __launch_bounds__(kBlock) k_cache_update(int64_t n, uint32_t t, const uint8_t* vstate,
                                                         const float* dcur, const float* spt_X,
                                                         const uint32_t* spt_sel, uint8_t* cached, float* dc,
                                                         float* Xc, uint32_t* size, uint32_t* last_use,
                                                         uint32_t* keys, uint32_t* vals,
                                                         unsigned long long* counters) {
  unsigned long long hits = 0, loads = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); j0 < n; j0 += stride) {
    const int64_t j = j0 + (threadIdx.x & 63);  // wave-uniform loop for the sums
    if (j < n) {
      const uint8_t s = vstate[j];
      if (s == 2) {
        cached[j] = 1;
        dc[j] = dcur[j];
        Xc[j] = spt_X[j];
        size[j] = spt_sel[j];
        ++loads;
      } else if (s == 1) {
        ++hits;
      }
      if (s) last_use[j] = t;
      keys[j] = cached[j] ? last_use[j] : t + 1u;
      vals[j] = (uint32_t)j;
    }
  }
  block_add(&counters[0], hits);
  block_add(&counters[1], loads);
}

struct LoadSortedSize {
  const uint32_t* order;
  const uint8_t* cached;
  const uint32_t* size;
  __device__ uint32_t operator()(int64_t p) const {
    const uint32_t j = order[p];
    return cached[j] ? size[j] : 0u;
  }
};

// Oldest first: entry p is dropped while the entries from p on still hold
// more than the budget.
__global__ void __launch_bounds__(kBlock) k_cache_evict(int64_t n, const uint32_t* order, const uint32_t* prefix,
                                                        const int32_t* total, int64_t max_nodes, uint8_t* cached,
                                                        unsigned long long* counters) {
  unsigned long long ev = 0;
  const int64_t all = (uint32_t)*total;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); p0 < n; p0 += stride) {
    const int64_t p = p0 + (threadIdx.x & 63);
    if (p < n) {
      const uint32_t j = order[p];
      if (cached[j] && all - (int64_t)prefix[p] > max_nodes) {
        cached[j] = 0;
        ++ev;
      }
    }
  }
  block_add(&counters[2], ev);
}

__global__ void __launch_bounds__(kBlock) k_cache_count(int64_t n, const uint8_t* cached, const uint32_t* size,
                                                        unsigned long long* counters) {
  unsigned long long c = 0, nodes = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); j0 < n; j0 += stride) {
    const int64_t j = j0 + (threadIdx.x & 63);
    if (j < n && cached[j]) {
      ++c;
      nodes += size[j];
    }
  }
  block_add(&counters[3], c);
  block_add(&counters[4], nodes);
}

int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

void free_cache(lodgs_cut_cache* c) {
  void* ptrs[] = {c->cached, c->dc, c->Xc, c->size, c->last_use, c->vstate, c->dcur, c->spt_sel, c->keys[0],
                  c->keys[1], c->vals[0], c->vals[1], c->prefix, c->counters, c->total};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
}

template <class T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count ? count : 1));
}

}  // namespace
}  // namespace lodgs

namespace lodgs {

int cache_select(lodgs_frame* f, lodgs_cut_cache* c, const ViewConst& v, uint32_t flags, int32_t* d_idx,
                 int64_t capacity, int32_t* d_count, hipStream_t st) {
  if (f->scene != c->scene) return set_error(LODGS_E_INVALID, "lodgs_lod_select_cached: frame and cache of different scenes");
  if (c->iteration >= (int64_t)0xFFFFFFFEll)
    return set_error(LODGS_E_INVALID, "lodgs_lod_select_cached: iteration count exhausted");
  const int64_t n = c->scene->dev.n_spt;
  const uint32_t t = (uint32_t)++c->iteration;
  if (c->prm.flush_every > 0 && t % (uint32_t)c->prm.flush_every == 0)
    hipLaunchKernelGGL(k_cache_flush, dim3(grid_for(n)), dim3(kBlock), 0, st, c->cached, n);
  const CacheDev cd{c->cached, c->dc, c->Xc, c->prm.d_min, c->prm.d_max, c->vstate, c->dcur, c->spt_sel};
  launch_select(f, v, flags, d_idx, capacity, d_count, st, &cd);
  hipLaunchKernelGGL(k_cache_update, dim3(grid_for(n)), dim3(kBlock), 0, st, n, t, c->vstate, c->dcur, f->spt_X,
                     c->spt_sel, c->cached, c->dc, c->Xc, c->size, c->last_use, c->keys[0], c->vals[0], c->counters);
  const SortScratch ws{f->sort_table, f->sort_below};
  int bits = 8;  // whole 8-bit digits covering t + 1
  while (bits < 32 && ((uint64_t)t + 1u) >> bits) bits += 8;
  const bool in2 = sort_pairs(c->keys[0], c->vals[0], c->keys[1], c->vals[1], &f->ctr->spt_count, n, bits, ws, st);
  const uint32_t* order = in2 ? c->vals[1] : c->vals[0];
  scan_exclusive(LoadSortedSize{order, c->cached, c->size}, &f->ctr->spt_count, n, f->block_sums, c->prefix, c->total,
                 st);
  hipLaunchKernelGGL(k_cache_evict, dim3(grid_for(n)), dim3(kBlock), 0, st, n, order, c->prefix, c->total,
                     c->prm.max_nodes, c->cached, c->counters);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_lod_select_cached");
}

}  // namespace lodgs

using lodgs::hip_fail;
using lodgs::set_error;

extern "C" {

int lodgs_cut_cache_create(const lodgs_scene* scene, const lodgs_cut_cache_params* prm, lodgs_cut_cache** out) {
  if (!scene || !prm || !out) return set_error(LODGS_E_INVALID, "lodgs_cut_cache_create: null argument");
  *out = nullptr;
  if (prm->max_nodes < 0 || !(prm->d_min >= 0.0f) || !(prm->d_max >= prm->d_min) || prm->flush_every < 0)
    return set_error(LODGS_E_INVALID, "lodgs_cut_cache_create: parameters out of range");
  lodgs_cut_cache* c = new (std::nothrow) lodgs_cut_cache();
  if (!c) return set_error(LODGS_E_OOM, "lodgs_cut_cache_create: out of host memory");
  c->scene = scene;
  c->prm = *prm;
  c->iteration = 0;
  const size_t n = (size_t)scene->dev.n_spt;
  hipError_t e = hipSuccess;
#define A(ptr, cnt) if (e == hipSuccess) e = lodgs::dalloc(&c->ptr, cnt)
  A(cached, n);
  A(dc, n);
  A(Xc, n);
  A(size, n);
  A(last_use, n);
  A(vstate, n);
  A(dcur, n);
  A(spt_sel, n);
  A(keys[0], n);
  A(keys[1], n);
  A(vals[0], n);
  A(vals[1], n);
  A(prefix, n);
  A(counters, 5);
  A(total, 1);
#undef A
  if (e == hipSuccess) e = hipMemset(c->cached, 0, n);
  if (e == hipSuccess) e = hipMemset(c->last_use, 0, 4 * n);
  if (e == hipSuccess) e = hipMemset(c->counters, 0, 5 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    lodgs::free_cache(c);
    (void)hipGetLastError();
    return set_error(LODGS_E_OOM, "lodgs_cut_cache_create: device allocation failed");
  }
  *out = c;
  return LODGS_OK;
}

void lodgs_cut_cache_destroy(lodgs_cut_cache* c) {
  if (c) lodgs::free_cache(c);
}

int lodgs_cut_cache_stats_read(lodgs_cut_cache* c, lodgs_cut_cache_stats* out, lodgs_stream stream) {
  using namespace lodgs;
  if (!c || !out) return set_error(LODGS_E_INVALID, "lodgs_cut_cache_stats_read: null argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t n = c->scene->dev.n_spt;
  unsigned long long h[5] = {0, 0, 0, 0, 0};
  hipError_t e = hipMemsetAsync(c->counters + 3, 0, 2 * sizeof(unsigned long long), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_cache_count, dim3(grid_for(n)), dim3(kBlock), 0, st, n, c->cached, c->size, c->counters);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, c->counters, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "lodgs_cut_cache_stats_read");
  out->iterations = c->iteration;
  out->hits = (int64_t)h[0];
  out->loads = (int64_t)h[1];
  out->evictions = (int64_t)h[2];
  out->cached_spts = (int64_t)h[3];
  out->cached_nodes = (int64_t)h[4];
  return LODGS_OK;
}

}  // extern "C"
