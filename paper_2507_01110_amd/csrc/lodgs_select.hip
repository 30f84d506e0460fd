// LoD cut over the flattened HSPT (Sec. 4.3 two-step cut; Sec. 4.1 Eq. 4 and
// Alg. 2 for the SPTs) and order-preserving stream compaction of the result.
//
// Step 1 (k_cut_upper): one thread per upper node and per SPT root.  A node is
// reached when no upper ancestor "stops" the descent (stops = culled, or fine
// enough at its own distance); the ancestor chain of the balanced upper
// hierarchy is short, so every thread walks it instead of running a
// level-synchronous BFS.  Reached upper nodes that are not culled and fine
// enough are selected; reached SPT roots that are not culled make their SPT
// visible, and a binary search over the SPT's r_max (descending) gives the
// candidate prefix length high_j = #{r_max > X_j}.  X_j is taken at the root's
// distance times the view's LoD noise factor (1 outside noisy training; the
// upper nodes' own distances are never scaled).
// Step 2: the candidates (upper nodes, then the prefixes of the visible SPTs)
// are compacted in order with wave ballots, one wave per segment.
#include "lodgs_internal.h"

namespace lodgs {

namespace {

// Per upper node, the two view tests of the cut, evaluated once per view:
// bit 0 = culled (its sphere is outside the frustum, when culling), bit 1 =
// fine enough (r_min <= X at its own distance).  The descent stops at a node
// with either bit; an upper node is selected when it is reached, not culled
// and fine enough.
__global__ void __launch_bounds__(kBlock) k_upper_tests(SceneDev S, const ViewConst* __restrict__ vp, uint32_t flags,
                                                        uint8_t* utest) {
  const ViewConst v = *vp;
  const bool cull = (flags & LODGS_CULL) != 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < S.n_upper;
       u += (int64_t)gridDim.x * blockDim.x) {
    const float mx = S.means[3 * u], my = S.means[3 * u + 1], mz = S.means[3 * u + 2];
    const bool culled = cull && sphere_culled(v, mx, my, mz, S.rho[u]);
    const bool fine = S.r_min[u] <= view_distance(v, mx, my, mz) * v.k;
    utest[u] = (uint8_t)((culled ? 1u : 0u) | (fine ? 2u : 0u));
  }
}

// Longest ancestor chain a walk follows (a malformed parent array with a
// cycle then reads as "not reached" instead of looping).
constexpr int32_t kMaxWalk = 4096;

// Walk up from a (the first upper ancestor, -1 for none): reached iff no
// upper ancestor stops the descent.
__device__ __forceinline__ bool chain_reached(const SceneDev& S, const uint8_t* utest, int32_t a) {
  for (int32_t steps = 0; a >= 0; ++steps) {
    if (steps >= kMaxWalk || a >= S.n_upper) return false;
    if (utest[a]) return false;
    a = S.upper_parent[a];
  }
  return true;
}

// The same from the ancestor table of element e: sixteen ancestors' tests are
// requested together instead of one dependent load per level.
__device__ __forceinline__ bool table_reached(const SceneDev& S, const uint8_t* utest, int64_t e, int64_t total) {
  constexpr int W = 16;
  for (int32_t d0 = 0; d0 < S.anc_depth; d0 += W) {
    int32_t a[W];
#pragma unroll
    for (int k = 0; k < W; ++k) a[k] = d0 + k < S.anc_depth ? S.anc[(int64_t)(d0 + k) * total + e] : -1;
    uint32_t t[W];
#pragma unroll
    for (int k = 0; k < W; ++k) t[k] = utest[a[k] < 0 ? 0 : a[k]];  // node 0 stands in for missing entries
    bool stop = false, end = false;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      end = end || a[k] < 0;
      stop = stop || (!end && t[k] != 0u);
    }
    if (stop) return false;
    if (end) return true;
  }
  return true;
}

// high = #{i < m : r[i] > X} for r descending, by an 8-ary search: each
// round requests 8 evenly spaced samples together and keeps the interval
// between the last sample above X and the first one not above it.
__device__ __forceinline__ int32_t count_above(const float* r, int32_t m, float X) {
  int32_t lo = 0, hi = m;  // the answer lies in [lo, hi]
  while (hi - lo > 8) {
    const int32_t span = hi - lo;
    int32_t p[8];
    float rv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      p[k] = lo + (int32_t)(((int64_t)(k + 1) * span) / 9);
      rv[k] = r[p[k]];
    }
    int32_t c = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) c += rv[k] > X ? 1 : 0;
    const int32_t nlo = c > 0 ? p[c > 0 ? c - 1 : 0] + 1 : lo;
    const int32_t nhi = c < 8 ? p[c < 8 ? c : 7] : hi;
    lo = nlo;
    hi = nhi;
  }
  float rv[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) rv[k] = lo + k < hi ? r[lo + k] : 0.0f;
  int32_t c = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) c += (lo + k < hi && rv[k] > X) ? 1 : 0;
  return lo + c;
}

__device__ __forceinline__ bool reached(const SceneDev& S, const uint8_t* utest, int64_t e, int64_t total,
                                        int32_t first) {
  return S.anc ? table_reached(S, utest, e, total) : chain_reached(S, utest, first);
}

// Ancestor-table construction: chain lengths (the maximum, or kMaxAncDepth + 1
// for a chain that is too long or leaves the upper node range), then the rows.
__global__ void __launch_bounds__(kBlock) k_anc_depth(SceneDev S, int32_t* depth) {
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  int32_t dmax = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t a = e < S.n_upper ? S.upper_parent[e] : S.spt_parent[e - S.n_upper];
    int32_t d = 0;
    while (a >= 0 && d <= kMaxAncDepth) {
      if (a >= S.n_upper) {
        d = kMaxAncDepth + 1;
        break;
      }
      ++d;
      a = S.upper_parent[a];
    }
    dmax = d > dmax ? d : dmax;
  }
  if (dmax) atomicMax(depth, dmax);
}

__global__ void __launch_bounds__(kBlock) k_anc_fill(SceneDev S, int32_t D, int32_t* anc) {
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t a = e < S.n_upper ? S.upper_parent[e] : S.spt_parent[e - S.n_upper];
    for (int32_t d = 0; d < D; ++d) {
      anc[(int64_t)d * total + e] = a;
      if (a >= 0) a = S.upper_parent[a];
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_cut_upper(SceneDev S, const ViewConst* __restrict__ vp, uint32_t flags,
                                                      const uint8_t* utest, uint8_t* upper_sel, int32_t* spt_high,
                                                      float* spt_X, FrameCounters* ctr, CacheDev C) {
  const ViewConst v = *vp;
  const bool cull = (flags & LODGS_CULL) != 0;
  const bool conservative = (flags & LODGS_CONSERVATIVE) != 0 && S.spt_radius != nullptr;
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  int vis = 0, hsum = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < S.n_upper) {
      const int32_t u = (int32_t)e;
      upper_sel[u] = (utest[u] == 2u && reached(S, utest, e, total, S.upper_parent[u])) ? 1 : 0;
    } else {
      const int32_t j = (int32_t)(e - S.n_upper);
      const int32_t b = S.spt_begin[j], m = S.spt_begin[j + 1] - b;
      int32_t high = 0;
      float X = 0.0f;
      uint8_t vst = 0;
      if (reached(S, utest, e, total, S.spt_parent[j])) {
        const float mx = S.means[3 * (int64_t)b], my = S.means[3 * (int64_t)b + 1], mz = S.means[3 * (int64_t)b + 2];
        if (!(cull && sphere_culled(v, mx, my, mz, S.rho[b]))) {
          const float d = view_distance(v, mx, my, mz) * v.spt_scale;  // the LoD noise (1: none)
          X = conservative ? fmaxf(0.0f, d - S.spt_radius[j]) * v.k : d * v.k;
          if (C.cached) {  // the cache's ratio test (squared, FP32)
            vst = 2;
            if (C.cached[j]) {
              const float r = d / C.dc[j];
              const float r2 = r * r;
              if (C.d_min <= r2 && r2 <= C.d_max) {
                X = C.Xc[j];
                vst = 1;
              }
            }
            C.dcur[j] = d;
          }
          high = count_above(S.r_max + b, m, X);
          hsum += high;
          ++vis;
        }
      }
      if (C.cached) {
        C.vstate[j] = vst;
        C.spt_sel[j] = 0u;
      }
      spt_high[j] = high;
      spt_X[j] = X;
    }
  }
  // one pair of atomics per workgroup (same-address atomics serialise)
  __shared__ int wsum[kBlock / 64][2];
  for (int d = 32; d > 0; d >>= 1) {
    vis += __shfl_xor(vis, d, 64);
    hsum += __shfl_xor(hsum, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    wsum[threadIdx.x >> 6][0] = vis;
    wsum[threadIdx.x >> 6][1] = hsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      a += wsum[w][0];
      b += wsum[w][1];
    }
    if (a) {
      atomicAdd(&ctr->n_spt_visible, a);
      atomicAdd(&ctr->sum_high, b);
    }
  }
}

// Compaction by segments, one wave per segment: segments 0 .. n_up_chunks-1
// are 64-node chunks of the upper hierarchy (predicate: selected), the rest
// are chunks of at most kChunk candidates of the visible SPT prefixes
// (predicate: r_min <= X_j); an SPT contributes ceil(high_j / kChunk)
// chunks, located through the scan of those counts (which also writes the
// SPT of every chunk).  Pass 1 counts each
// segment with ballots, a scan turns the counts into output offsets, pass 2
// writes each segment's selected nodes in order with ballot ranks.  Segments
// follow the layout order, so the output is ascending.
constexpr int32_t kChunk = 512;

// The scan of the chunk counts stores each SPT's first chunk index and the
// owner table: owner[t] = the SPT whose prefix holds candidate chunk t.
struct StoreChunks {
  uint32_t* ch_off;
  uint32_t* owner;
  __device__ void operator()(int64_t j, uint32_t first, uint32_t count) const {
    ch_off[j] = first;
    for (uint32_t t = 0; t < count; ++t) owner[first + t] = (uint32_t)j;
  }
};

template <bool WRITE>
__global__ void __launch_bounds__(kBlock) k_segments(SceneDev S, const uint8_t* upper_sel, const int32_t* spt_high,
                                                     const float* spt_X, const uint32_t* ch_off,
                                                     const uint32_t* owner, int32_t n_up_chunks,
                                                     uint32_t* seg, int32_t* idx, int64_t capacity,
                                                     FrameCounters* ctr, int32_t* d_count, uint32_t* spt_sel) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  const int64_t nseg = (int64_t)n_up_chunks + ctr->n_chunks;
  const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
  if (!WRITE && blockIdx.x == 0 && threadIdx.x == 0) ctr->seg_total = (int32_t)nseg;
  uint32_t up_count = 0;
  for (int64_t sg = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); sg < nseg; sg += nw) {
    const uint32_t base = WRITE ? seg[sg] : 0u;
    uint32_t c = 0;
    if (sg < n_up_chunks) {
      const int64_t u = sg * 64 + lane;
      const bool p = u < S.n_upper && upper_sel[u] != 0;
      const uint64_t b = __ballot(p);
      if (WRITE && p) {
        const uint32_t pos = base + (uint32_t)__popcll(b & lt);
        if (pos < capacity) idx[pos] = (int32_t)u;
      }
      c = (uint32_t)__popcll(b);
      up_count += c;
    } else {
      const uint32_t t = (uint32_t)(sg - n_up_chunks);
      const int32_t j = (int32_t)owner[t];
      const int32_t h = spt_high[j];
      const int32_t e_begin = (int32_t)(t - ch_off[j]) * kChunk;
      const int32_t e_end = min(h, e_begin + kChunk);
      const float X = spt_X[j];
      const int32_t b0 = S.spt_begin[j];
      // the chunk's candidates (at most kChunk = 8 x 64) are requested together
      static_assert(kChunk == 8 * 64, "eight wave-wide loads per chunk");
      float rm[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int32_t e = e_begin + 64 * q + lane;
        rm[q] = e < e_end ? S.r_min[b0 + e] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int32_t e = e_begin + 64 * q + lane;
        const bool p = e < e_end && rm[q] <= X;
        const uint64_t b = __ballot(p);
        if (WRITE && p) {
          const uint32_t pos = base + c + (uint32_t)__popcll(b & lt);
          if (pos < capacity) idx[pos] = b0 + e;
        }
        c += (uint32_t)__popcll(b);
      }
      if (!WRITE && spt_sel && lane == 0 && c) atomicAdd(&spt_sel[j], c);
    }
    if (!WRITE && lane == 0) seg[sg] = c;
  }
  if (!WRITE) {  // one atomic per workgroup
    __shared__ uint32_t wup[kBlock / 64];
    if (lane == 0) wup[threadIdx.x >> 6] = up_count;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int w = 0; w < kBlock / 64; ++w) t += wup[w];
      if (t) atomicAdd(&ctr->n_upper_selected, (int)t);
    }
  } else if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int32_t n = ctr->n_selected;
    *d_count = n;
    if ((int64_t)n > capacity) ctr->status = LODGS_E_CAPACITY;
  }
}

struct LoadChunks {
  const int32_t* high;
  __device__ uint32_t operator()(int64_t j) const { return (uint32_t)((high[j] + kChunk - 1) / kChunk); }
};

}  // namespace

int build_ancestor_table(lodgs_scene* s) {
  SceneDev& S = s->dev;
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  if (S.n_upper <= 0 || total <= 0) return LODGS_OK;
  int32_t* d_depth = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&d_depth), sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(d_depth, 0, sizeof(int32_t));
  int grid = (int)((total + kBlock - 1) / kBlock);
  grid = grid > 4096 ? 4096 : grid;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_anc_depth, dim3(grid), dim3(kBlock), 0, 0, S, d_depth);
    e = hipGetLastError();
  }
  int32_t D = 0;
  if (e == hipSuccess) e = hipMemcpy(&D, d_depth, sizeof D, hipMemcpyDeviceToHost);
  if (d_depth) (void)hipFree(d_depth);
  if (e != hipSuccess) return hip_fail(e, "lodgs_scene_create: ancestor table");
  if (D <= 0 || D > kMaxAncDepth) return LODGS_OK;  // the cut walks the parent array instead
  int32_t* anc = nullptr;
  e = hipMalloc(reinterpret_cast<void**>(&anc), sizeof(int32_t) * (size_t)D * (size_t)total);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return LODGS_OK;  // no room: the cut walks the parent array instead
  }
  hipLaunchKernelGGL(k_anc_fill, dim3(grid), dim3(kBlock), 0, 0, S, D, anc);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(anc);
    return hip_fail(e, "lodgs_scene_create: ancestor table");
  }
  s->anc_owned = anc;
  S.anc = anc;
  S.anc_depth = D;
  return LODGS_OK;
}

// Radius of each SPT about its root's mean, for the CONSERVATIVE cut: the
// largest |mu_i - mu_root| over the SPT's members (its layout segment), in
// FP64 from the FP32 means (((dx dx + dy dy) + dz dz), correctly rounded
// square root), rounded once to FP32.  One wave per SPT; the maximum is exact,
// so the order does not matter.
__global__ void __launch_bounds__(kBlock) k_spt_radius(SceneDev S, float* radius) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t j = wave; j < S.n_spt; j += waves) {  // wave-uniform
    const int64_t b = S.spt_begin[j], e = S.spt_begin[j + 1];
    const double rx = S.means[3 * b], ry = S.means[3 * b + 1], rz = S.means[3 * b + 2];
    double r = 0.0;
    for (int64_t i = b + lane; i < e; i += 64) {
      const double dx = (double)S.means[3 * i] - rx, dy = (double)S.means[3 * i + 1] - ry,
                   dz = (double)S.means[3 * i + 2] - rz;
      r = fmax(r, __builtin_sqrt((dx * dx + dy * dy) + dz * dz));
    }
    for (int d = 32; d > 0; d >>= 1) r = fmax(r, __shfl_xor(r, d, 64));
    if (lane == 0) radius[j] = (float)r;
  }
}

int build_spt_radius(lodgs_scene* s) {
  SceneDev& S = s->dev;
  if (S.n_spt <= 0) return LODGS_OK;
  float* r = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&r), sizeof(float) * (size_t)S.n_spt);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(LODGS_E_OOM, "lodgs_scene_create: SPT radii");
  }
  int grid = (int)(((int64_t)S.n_spt * 64 + kBlock - 1) / kBlock);
  grid = grid > 4096 ? 4096 : grid;
  hipLaunchKernelGGL(k_spt_radius, dim3(grid), dim3(kBlock), 0, 0, S, r);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(r);
    return hip_fail(e, "lodgs_scene_create: SPT radii");
  }
  s->radius_owned = r;
  S.spt_radius = r;
  return LODGS_OK;
}

void launch_select(lodgs_frame* f, const ViewConst& v, uint32_t flags, int32_t* d_idx, int64_t capacity,
                   int32_t* d_count, hipStream_t st, const CacheDev* cache) {
  CacheDev C{};
  if (cache) C = *cache;
  const SceneDev& S = f->scene->dev;
  stage_begin(f, LODGS_STAGE_SELECT, st);
  launch_set_view(v, f->d_view_sel, f->ctr, kViewSelect, nullptr, 0, st);
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  int grid = (int)((total + kBlock - 1) / kBlock);
  grid = grid < 1 ? 1 : (grid > 4096 ? 4096 : grid);
  int ugrid = (int)((S.n_upper + kBlock - 1) / kBlock);
  ugrid = ugrid < 1 ? 1 : (ugrid > 4096 ? 4096 : ugrid);
  hipLaunchKernelGGL(k_upper_tests, dim3(ugrid), dim3(kBlock), 0, st, S, f->d_view_sel, flags, f->upper_test);
  hipLaunchKernelGGL(k_cut_upper, dim3(grid), dim3(kBlock), 0, st, S, f->d_view_sel, flags, f->upper_test,
                     f->upper_sel, f->spt_high, f->spt_X, f->ctr, C);
  const int32_t n_up_chunks = (S.n_upper + 63) / 64;
  // chunks per visible SPT prefix -> offsets, total -> n_chunks
  scan_exclusive(LoadChunks{f->spt_high}, &f->ctr->spt_count, (int64_t)S.n_spt, f->block_sums,
                 StoreChunks{f->spt_off, f->chunk_owner}, &f->ctr->n_chunks, st);
  const int sgrid = 4096;
  const int64_t seg_cap = (int64_t)n_up_chunks + S.n_spt + S.n_nodes / kChunk + 1;
  hipLaunchKernelGGL(k_segments<false>, dim3(sgrid), dim3(kBlock), 0, st, S, f->upper_sel, f->spt_high, f->spt_X,
                     f->spt_off, f->chunk_owner, n_up_chunks, f->seg, (int32_t*)nullptr, capacity, f->ctr, d_count,
                     C.spt_sel);
  scan_exclusive(LoadArray{f->seg}, &f->ctr->seg_total, seg_cap, f->block_sums, f->seg, &f->ctr->n_selected, st);
  hipLaunchKernelGGL(k_segments<true>, dim3(sgrid), dim3(kBlock), 0, st, S, f->upper_sel, f->spt_high, f->spt_X,
                     f->spt_off, f->chunk_owner, n_up_chunks, f->seg, d_idx, capacity, f->ctr, d_count,
                     (uint32_t*)nullptr);
  stage_end(f, st);
}

// ---------------------------------------------------------------- comparator cuts
// The two whole-hierarchy cuts the HSPT replaces (Sec. 4.3): the BFS cut and
// the parallel cut of Eq. 5.  Both mark the selected nodes in a bitmask (bit
// i % 32 of word i / 32); an exclusive scan of the words' popcounts then
// writes the ascending list, so the order of the marking does not matter.
namespace {

__device__ __forceinline__ bool node_fine(const SceneDev& S, const ViewConst& v, int64_t i, float mx, float my,
                                          float mz) {
  return S.r_min[i] <= view_distance(v, mx, my, mz) * v.k;
}

// Clears the bitmask and the BFS level counts (level 0 holds the root alone).
__global__ void __launch_bounds__(kBlock) k_cut_clear(uint32_t* bits, int64_t n_words, int32_t* level_count,
                                                      int32_t n_levels) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = t0; w < n_words; w += stride) bits[w] = 0u;
  if (level_count)
    for (int64_t l = t0; l < n_levels; l += stride) level_count[l] = l == 0 ? 1 : 0;
}

// Eq. 5 per node: fine at its own distance while its parent is not (the root
// has none); with culling, a node whose own sphere is outside the frustum is
// dropped.  One wave per 64 nodes writes their two bitmask words.
__global__ void __launch_bounds__(kBlock) k_parallel_cut(SceneDev S, const ViewConst* __restrict__ vp, uint32_t flags,
                                                         uint32_t* bits) {
  const ViewConst v = *vp;
  const bool cull = (flags & LODGS_CULL) != 0;
  const int lane = threadIdx.x & 63;
  const int64_t n_waves = (S.n_nodes + 63) / 64;
  for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < n_waves;
       w += ((int64_t)gridDim.x * blockDim.x) >> 6) {  // wave-uniform
    const int64_t i = w * 64 + lane;
    bool sel = false;
    if (i < S.n_nodes) {
      const float mx = S.means[3 * i], my = S.means[3 * i + 1], mz = S.means[3 * i + 2];
      sel = node_fine(S, v, i, mx, my, mz);
      if (sel) {
        const int64_t p = S.parent[i];
        if (p >= 0 && p < S.n_nodes)
          sel = !node_fine(S, v, p, S.means[3 * p], S.means[3 * p + 1], S.means[3 * p + 2]);
      }
      if (sel && cull) sel = !sphere_culled(v, mx, my, mz, S.rho[i]);
    }
    const uint64_t b = __ballot(sel);
    if (lane == 0) reinterpret_cast<uint2*>(bits)[w] = make_uint2((uint32_t)b, (uint32_t)(b >> 32));
  }
}

// One BFS level: every frontier node is dropped when culled, marked when fine
// at its own distance, else its two children join the next frontier (one
// atomic per wave for their slots).  Level 0 is the root, position 0.  Counts stay even past the root's level,
// and fcap is even, so a pair of children is written whole or not at all; a
// full queue records LODGS_E_CAPACITY and the next level reads only what was
// written.
__global__ void __launch_bounds__(kBlock) k_bfs_level(SceneDev S, const ViewConst* __restrict__ vp, uint32_t flags,
                                                      int32_t level, const int32_t* fin, int32_t* fout,
                                                      int32_t* level_count, int64_t fcap, uint32_t* bits,
                                                      FrameCounters* ctr) {
  const ViewConst v = *vp;
  const bool cull = (flags & LODGS_CULL) != 0;
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  int64_t n_in = level_count[level];
  n_in = level == 0 ? 1 : (n_in < fcap ? n_in : fcap);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); t0 < n_in; t0 += stride) {
    const int64_t t = t0 + lane;  // t0 is wave-aligned: the loop is wave-uniform
    bool push = false;
    int2 ch = make_int2(-1, -1);
    if (t < n_in) {
      const int64_t u = level == 0 ? 0 : fin[t];
      if (u >= 0 && u < S.n_nodes) {
        const float mx = S.means[3 * u], my = S.means[3 * u + 1], mz = S.means[3 * u + 2];
        if (!(cull && sphere_culled(v, mx, my, mz, S.rho[u]))) {
          if (node_fine(S, v, u, mx, my, mz)) {
            atomicOr(&bits[u >> 5], 1u << (u & 31));
          } else {
            ch = S.child[u];
            push = ch.x >= 0 && ch.x < S.n_nodes && ch.y >= 0 && ch.y < S.n_nodes;
          }
        }
      }
    }
    const uint64_t pb = __ballot(push);
    if (pb) {
      uint32_t base = 0;
      if (lane == 0) base = (uint32_t)atomicAdd(&level_count[level + 1], 2 * __popcll(pb));
      base = __shfl(base, 0, 64);
      if (push) {
        const int64_t pos = (int64_t)base + 2 * __popcll(pb & lt);
        if (pos < fcap) {
          fout[pos] = ch.x;
          fout[pos + 1] = ch.y;
        } else {
          ctr->status = LODGS_E_CAPACITY;
        }
      }
    }
  }
}

struct LoadPopc {
  const uint32_t* bits;
  __device__ uint32_t operator()(int64_t w) const { return (uint32_t)__popc(bits[w]); }
};

// Word w's set bits, lowest first, at idx[prefix ...].
struct StoreBits {
  const uint32_t* bits;
  int32_t* idx;
  int64_t cap;
  __device__ void operator()(int64_t w, uint32_t prefix, uint32_t) const {
    uint32_t b = bits[w];
    int64_t p = prefix;
    while (b) {
      const int k = __ffs(b) - 1;
      b &= b - 1u;
      if (p < cap) idx[p] = (int32_t)(w * 32 + k);
      ++p;
    }
  }
};

// The count, the capacity check and, for the BFS, the depth check: a
// frontier left after the last level means the hierarchy is deeper than its
// stated height.
__global__ void k_cut_finish(FrameCounters* ctr, int32_t* d_count, int64_t capacity, const int32_t* level_count,
                             int32_t height) {
  const int32_t n = ctr->n_selected;
  *d_count = n;
  if ((int64_t)n > capacity) ctr->status = LODGS_E_CAPACITY;
  if (level_count && level_count[height] > 0) ctr->status = LODGS_E_INVALID;
}

}  // namespace

void launch_select_full(lodgs_frame* f, const ViewConst& v, uint32_t flags, int32_t* d_idx, int64_t capacity,
                        int32_t* d_count, hipStream_t st) {
  const SceneDev& S = f->scene->dev;
  const bool bfs = (flags & LODGS_CUT_BFS) != 0;
  const int64_t n_words = cut_bit_words(S.n_nodes);
  stage_begin(f, LODGS_STAGE_SELECT, st);
  launch_set_view(v, f->d_view_sel, f->ctr, kViewSelect, nullptr, 0, st);
  int cgrid = (int)((n_words + kBlock - 1) / kBlock);
  cgrid = cgrid < 1 ? 1 : (cgrid > 2048 ? 2048 : cgrid);
  hipLaunchKernelGGL(k_cut_clear, dim3(cgrid), dim3(kBlock), 0, st, f->cut_bits, n_words,
                     bfs ? f->level_count : (int32_t*)nullptr, f->cut_height + 1);
  if (bfs) {
    const int64_t fcap = f->caps.max_selected & ~(int64_t)1;
    for (int32_t l = 0; l < f->cut_height; ++l)
      hipLaunchKernelGGL(k_bfs_level, dim3(1024), dim3(kBlock), 0, st, S, f->d_view_sel, flags, l,
                         f->frontier[l & 1], f->frontier[(l + 1) & 1], f->level_count, fcap, f->cut_bits, f->ctr);
  } else {
    int pgrid = (int)((S.n_nodes + kBlock - 1) / kBlock);
    pgrid = pgrid < 1 ? 1 : (pgrid > 8192 ? 8192 : pgrid);
    hipLaunchKernelGGL(k_parallel_cut, dim3(pgrid), dim3(kBlock), 0, st, S, f->d_view_sel, flags, f->cut_bits);
  }
  scan_exclusive(LoadPopc{f->cut_bits}, &f->ctr->n_bit_words, n_words, f->block_sums,
                 StoreBits{f->cut_bits, d_idx, capacity}, &f->ctr->n_selected, st);
  hipLaunchKernelGGL(k_cut_finish, dim3(1), dim3(1), 0, st, f->ctr, d_count, capacity,
                     bfs ? (const int32_t*)f->level_count : (const int32_t*)nullptr, f->cut_height);
  stage_end(f, st);
}

}  // namespace lodgs
