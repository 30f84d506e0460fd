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
// Step 2: the candidates (upper nodes, then the prefixes of the visible SPTs)
// are compacted in order with wave ballots, one wave per segment.
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

__global__ void __launch_bounds__(kBlock) k_cut_upper(SceneDev S, const ViewConst* __restrict__ vp, uint32_t flags,
                                                      uint8_t* upper_sel, int32_t* spt_high, float* spt_X,
                                                      FrameCounters* ctr) {
  const ViewConst v = *vp;
  const bool cull = (flags & LODGS_CULL) != 0;
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  int vis = 0, hsum = 0;
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
          hsum += lo;
          ++vis;
        }
      }
      spt_high[j] = high;
      spt_X[j] = X;
    }
  }
  // one atomic per wave
  for (int d = 32; d > 0; d >>= 1) {
    vis += __shfl_xor(vis, d, 64);
    hsum += __shfl_xor(hsum, d, 64);
  }
  if ((threadIdx.x & 63) == 0 && vis) {
    atomicAdd(&ctr->n_spt_visible, vis);
    atomicAdd(&ctr->sum_high, hsum);
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
                                                     FrameCounters* ctr, int32_t* d_count) {
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
      for (int32_t e0 = e_begin; e0 < e_end; e0 += 64) {
        const int32_t e = e0 + lane;
        const bool p = e < e_end && S.r_min[b0 + e] <= X;
        const uint64_t b = __ballot(p);
        if (WRITE && p) {
          const uint32_t pos = base + c + (uint32_t)__popcll(b & lt);
          if (pos < capacity) idx[pos] = b0 + e;
        }
        c += (uint32_t)__popcll(b);
      }
    }
    if (!WRITE && lane == 0) seg[sg] = c;
  }
  if (!WRITE) {
    if (lane == 0 && up_count) atomicAdd(&ctr->n_upper_selected, (int)up_count);
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

void launch_select(lodgs_frame* f, const ViewConst& v, uint32_t flags, int32_t* d_idx, int64_t capacity,
                   int32_t* d_count, hipStream_t st) {
  const SceneDev& S = f->scene->dev;
  stage_begin(f, LODGS_STAGE_SELECT, st);
  launch_set_view(v, f->d_view_sel, f->ctr, kViewSelect, nullptr, 0, st);
  const int64_t total = (int64_t)S.n_upper + S.n_spt;
  int grid = (int)((total + kBlock - 1) / kBlock);
  grid = grid < 1 ? 1 : (grid > 4096 ? 4096 : grid);
  hipLaunchKernelGGL(k_cut_upper, dim3(grid), dim3(kBlock), 0, st, S, f->d_view_sel, flags, f->upper_sel, f->spt_high, f->spt_X,
                     f->ctr);
  const int32_t n_up_chunks = (S.n_upper + 63) / 64;
  // chunks per visible SPT prefix -> offsets, total -> n_chunks
  scan_exclusive(LoadChunks{f->spt_high}, &f->ctr->spt_count, (int64_t)S.n_spt, f->block_sums,
                 StoreChunks{f->spt_off, f->chunk_owner}, &f->ctr->n_chunks, st);
  const int sgrid = 4096;
  const int64_t seg_cap = (int64_t)n_up_chunks + S.n_spt + S.n_nodes / kChunk + 1;
  hipLaunchKernelGGL(k_segments<false>, dim3(sgrid), dim3(kBlock), 0, st, S, f->upper_sel, f->spt_high, f->spt_X,
                     f->spt_off, f->chunk_owner, n_up_chunks, f->seg, (int32_t*)nullptr, capacity, f->ctr, d_count);
  scan_exclusive(LoadArray{f->seg}, &f->ctr->seg_total, seg_cap, f->block_sums, f->seg, &f->ctr->n_selected, st);
  hipLaunchKernelGGL(k_segments<true>, dim3(sgrid), dim3(kBlock), 0, st, S, f->upper_sel, f->spt_high, f->spt_X,
                     f->spt_off, f->chunk_owner, n_up_chunks, f->seg, d_idx, capacity, f->ctr, d_count);
  stage_end(f, st);
}

}  // namespace lodgs
