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
// candidate prefix length high_j = #{r_max > X_j}.
// Step 2: the candidate space (upper nodes, then the prefixes of the visible
// SPTs laid end to end) is compacted in order with wave ballots: per block
// counts, a scan of the counts, and an ordered write.
#include "lodgs_internal.h"

namespace lodgs {

namespace {

__device__ __forceinline__ bool upper_stops(const SceneDev& S, const ViewConst& v, bool cull, int32_t a) {
  const float mx = S.means[3 * (int64_t)a], my = S.means[3 * (int64_t)a + 1], mz = S.means[3 * (int64_t)a + 2];
  if (cull && sphere_culled(v, mx, my, mz, S.rho[a])) return true;
  return S.r_min[a] <= view_distance(v, mx, my, mz) * v.k;
}

__device__ __forceinline__ bool chain_reached(const SceneDev& S, const ViewConst& v, bool cull, int32_t a) {
  while (a >= 0) {
    if (upper_stops(S, v, cull, a)) return false;
    a = S.upper_parent[a];
  }
  return true;
}

__global__ void __launch_bounds__(kBlock) k_cut_upper(SceneDev S, ViewConst v, uint32_t flags,
                                                      uint8_t* upper_sel, int32_t* spt_high, float* spt_X,
                                                      FrameCounters* ctr) {
  const bool cull = (flags & LODGS_CULL) != 0;
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  int vis = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < S.n_upper) {
      const int32_t u = (int32_t)e;
      uint8_t sel = 0;
      if (chain_reached(S, v, cull, S.upper_parent[u])) {
        const float mx = S.means[3 * e], my = S.means[3 * e + 1], mz = S.means[3 * e + 2];
        const bool culled = cull && sphere_culled(v, mx, my, mz, S.rho[u]);
        sel = (!culled && S.r_min[u] <= view_distance(v, mx, my, mz) * v.k) ? 1 : 0;
      }
      upper_sel[u] = sel;
    } else {
      const int32_t j = (int32_t)(e - S.n_upper);
      const int32_t b = S.spt_begin[j], m = S.spt_begin[j + 1] - b;
      int32_t high = 0;
      float X = 0.0f;
      if (chain_reached(S, v, cull, S.spt_parent[j])) {
        const float mx = S.means[3 * (int64_t)b], my = S.means[3 * (int64_t)b + 1], mz = S.means[3 * (int64_t)b + 2];
        if (!(cull && sphere_culled(v, mx, my, mz, S.rho[b]))) {
          X = view_distance(v, mx, my, mz) * v.k;
          int32_t lo = 0, hi = m;
          while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (S.r_max[b + mid] > X) lo = mid + 1;
            else hi = mid;
          }
          high = lo;
          ++vis;
        }
      }
      spt_high[j] = high;
      spt_X[j] = X;
    }
  }
  // one atomic per wave
  for (int d = 32; d > 0; d >>= 1) vis += __shfl_xor(vis, d, 64);
  if ((threadIdx.x & 63) == 0 && vis) atomicAdd(&ctr->n_spt_visible, vis);
}

// Candidate e of the concatenated space: upper node e (e < n_upper), else
// element f = e - n_upper of the SPT prefixes.
struct Candidate {
  int32_t node;
  bool sel;
};

__device__ __forceinline__ Candidate candidate(const SceneDev& S, const uint8_t* upper_sel, const uint32_t* spt_off,
                                               const float* spt_X, int64_t e) {
  if (e < S.n_upper) return {(int32_t)e, upper_sel[e] != 0};
  const uint32_t f = (uint32_t)(e - S.n_upper);
  // largest j with spt_off[j] <= f
  int32_t lo = 0, hi = S.n_spt;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (spt_off[mid] <= f) lo = mid;
    else hi = mid;
  }
  const int32_t node = S.spt_begin[lo] + (int32_t)(f - spt_off[lo]);
  return {node, S.r_min[node] <= spt_X[lo]};
}

__global__ void k_set_candidates(FrameCounters* ctr, int32_t n_upper) {
  ctr->upper_plus_high = n_upper + ctr->sum_high;
}

__global__ void __launch_bounds__(kBlock) k_compact_count(SceneDev S, const uint8_t* upper_sel,
                                                          const uint32_t* spt_off, const float* spt_X,
                                                          const FrameCounters* ctr, uint32_t* chunk) {
  __shared__ uint32_t wt[kBlock / 64];
  const Segment s = block_segment(ctr->upper_plus_high, kScanGrid);
  uint32_t c = 0;
  for (int64_t e = s.begin + threadIdx.x; e < s.end; e += kBlock) c += candidate(S, upper_sel, spt_off, spt_X, e).sel;
  uint32_t tot;
  block_exclusive_scan(c, wt, &tot);
  if (threadIdx.x == 0) chunk[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_compact_write(SceneDev S, const uint8_t* upper_sel,
                                                          const uint32_t* spt_off, const float* spt_X,
                                                          FrameCounters* ctr, const uint32_t* chunk,
                                                          int32_t* idx, int64_t capacity, int32_t* d_count) {
  __shared__ uint32_t wt[kBlock / 64];
  const Segment s = block_segment(ctr->upper_plus_high, kScanGrid);
  uint32_t base = chunk[blockIdx.x];
  for (int64_t r0 = s.begin; r0 < s.end; r0 += kBlock) {
    const int64_t e = r0 + threadIdx.x;
    Candidate c{0, false};
    if (e < s.end) c = candidate(S, upper_sel, spt_off, spt_X, e);
    uint32_t tot;
    const uint32_t pos = base + block_exclusive_scan(c.sel ? 1u : 0u, wt, &tot);
    if (c.sel && pos < capacity) idx[pos] = c.node;
    base += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t n = chunk[kScanGrid];
    *d_count = (int32_t)n;
    ctr->n_selected = (int32_t)n;
    if ((int64_t)n > capacity) ctr->status = LODGS_E_CAPACITY;
  }
}

__global__ void __launch_bounds__(kBlock) k_count_upper(const uint8_t* upper_sel, int32_t n_upper,
                                                        FrameCounters* ctr) {
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_upper; i += (int64_t)gridDim.x * blockDim.x)
    c += upper_sel[i];
  for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(&ctr->n_upper_selected, c);
}

__global__ void k_reset_select(FrameCounters* ctr) {
  ctr->n_spt_visible = 0;
  ctr->n_upper_selected = 0;
}

struct LoadHigh {
  const int32_t* h;
  __device__ uint32_t operator()(int64_t i) const { return (uint32_t)h[i]; }
};

}  // namespace

void launch_select(lodgs_frame* f, const ViewConst& v, uint32_t flags, int32_t* d_idx, int64_t capacity,
                   int32_t* d_count, hipStream_t st) {
  const SceneDev& S = f->scene->dev;
  stage_begin(f, LODGS_STAGE_SELECT, st);
  hipLaunchKernelGGL(k_reset_select, dim3(1), dim3(1), 0, st, f->ctr);
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  int grid = (int)((total + kBlock - 1) / kBlock);
  grid = grid < 1 ? 1 : (grid > 4096 ? 4096 : grid);
  hipLaunchKernelGGL(k_cut_upper, dim3(grid), dim3(kBlock), 0, st, S, v, flags, f->upper_sel, f->spt_high, f->spt_X,
                     f->ctr);
  // exclusive scan of the prefix lengths; total -> sum_high
  scan_exclusive(LoadHigh{f->spt_high}, &f->ctr->spt_count, (int64_t)S.n_spt, f->block_sums, f->spt_off,
                 &f->ctr->sum_high, st);
  hipLaunchKernelGGL(k_set_candidates, dim3(1), dim3(1), 0, st, f->ctr, S.n_upper);
  hipLaunchKernelGGL(k_compact_count, dim3(kScanGrid), dim3(kBlock), 0, st, S, f->upper_sel, f->spt_off, f->spt_X,
                     f->ctr, f->chunk);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanGrid), 0, st, f->chunk, (int32_t*)nullptr);
  hipLaunchKernelGGL(k_compact_write, dim3(kScanGrid), dim3(kBlock), 0, st, S, f->upper_sel, f->spt_off, f->spt_X,
                     f->ctr, f->chunk, d_idx, capacity, d_count);
  if (S.n_upper > 0) {
    int g2 = (S.n_upper + kBlock - 1) / kBlock;
    g2 = g2 > 1024 ? 1024 : g2;
    hipLaunchKernelGGL(k_count_upper, dim3(g2), dim3(kBlock), 0, st, f->upper_sel, S.n_upper, f->ctr);
  }
  stage_end(f, st);
}

}  // namespace lodgs
