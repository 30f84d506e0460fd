// Forward render of a selected set (Sec. 3: EWA projection, SH colour, Eq. 1
// front-to-back compositing with Eq. 2's alpha), tiled 16x16.
//
//  k_project  one thread per selected node: camera transform, near-plane test,
//             covariance from (scale, rotation), EWA Jacobian, projected
//             covariance + 0.3 px^2, conic, square footprint, tile rectangle,
//             opacity, SH colour.  Writes a 64-byte Splat record, the depth key
//             and the tile count (0 for a splat that is not drawn).
//  sort       order-preserving compaction of the drawn splats, stable radix
//             sort of their FP32 depth bits, then (k_dup) one (tile, splat)
//             instance per covered tile emitted in depth order, then a stable
//             radix sort of the instances by tile: the result is the order of
//             the 64-bit key (tile << 32 | depth), ties by selection order, with
//             far less key traffic.
//  k_ranges   first/last instance of every tile.
//  k_blend    one workgroup per tile, PX pixels per lane; splat records are
//             staged in LDS one batch per workgroup size; each 16-lane row
//             (4x4 pixel blocks) replays only the splats whose alpha >= 1/255
//             ellipse reaches one of its blocks (elsewhere the result is known).
#include "lodgs_internal.h"
#include "lodgs_proj.h"

namespace lodgs {

// Projection of one node.  The per-splat chain runs in FP64 with a fixed
// operation order (scales from the FP32 exp, opacity as the FP32 sigmoid);
// its decisions (near plane, positive determinant, footprint radius, tile
// rectangle) are taken in FP64 and its outputs rounded to the FP32 record.
struct Proj {
  bool visible;
  float depth;
  Splat sp;
  int x0, x1, y0, y1;
};

__device__ __forceinline__ int tile_clamp(double v, int hi) {
  if (v < 0.0) return 0;
  if (v > (double)hi) return hi;
  return (int)v;
}

__device__ __forceinline__ Proj project_node(const SceneDev& S, const ViewConst& v, int32_t node) {
  Proj P;
  P.visible = false;
  P.x0 = P.x1 = P.y0 = P.y1 = 0;
  const int64_t n = node;
  // every parameter but the colour is requested up front, before the
  // near-plane test needs the mean
  const NodeGeom geo = load_geom(S.means, S.log_scales, S.quats, n);
  const float theta = S.opacity_logits[n];
  Proj64 G;
  const bool ok = proj_chain64(geo, v, G);
  P.depth = (float)G.c[2];
  if (!ok) return P;
  const double A = G.A, B = G.B, C = G.C, det = G.det;
  const double fx = v.fx, fy = v.fy, u = G.u, vv = G.v;
  const double mx = fx * u + (double)v.cx, my = fy * vv + (double)v.cy;
  const double mid = 0.5 * (A + C);
  const double disc = mid * mid - det;
  const double r = ceil(3.0 * __builtin_sqrt(mid + __builtin_sqrt(fmax(0.1, disc))));
  P.x0 = tile_clamp(floor((mx - r) * 0.0625), v.tiles_x);
  P.x1 = tile_clamp(floor((mx + r) * 0.0625) + 1.0, v.tiles_x);
  P.y0 = tile_clamp(floor((my - r) * 0.0625), v.tiles_y);
  P.y1 = tile_clamp(floor((my + r) * 0.0625) + 1.0, v.tiles_y);
  P.visible = P.x1 > P.x0 && P.y1 > P.y0;
  // principal axes of the projected covariance
  const double l1 = mid + __builtin_sqrt(fmax(0.0, disc));
  const double l2 = det / l1;
  double vx, vy;
  if (A >= C) {
    vx = l1 - C;
    vy = B;
  } else {
    vx = B;
    vy = l1 - A;
  }
  const double nn = __builtin_sqrt(vx * vx + vy * vy);
  double ce = 1.0, se = 0.0;
  if (nn > 0.0) {
    ce = vx / nn;
    se = vy / nn;
  }
  P.sp.mxh = (float)mx;
  P.sp.mxl = (float)(mx - (double)P.sp.mxh);
  P.sp.myh = (float)my;
  P.sp.myl = (float)(my - (double)P.sp.myh);
  P.sp.ce = (float)ce;
  P.sp.se = (float)se;
  P.sp.h1 = (float)(-0.5 / l1);
  P.sp.h2 = (float)(-0.5 / l2);
  P.sp.o = 1.0f / (1.0f + fexp(-theta));
  P.sp.rect_x = (uint32_t)P.x0 | ((uint32_t)P.x1 << 16);
  P.sp.rect_y = (uint32_t)P.y0 | ((uint32_t)P.y1 << 16);
  P.sp.pad0 = P.sp.pad1 = 0u;
  return P;
}

// SH colour for the view direction (mu - pos) / |mu - pos|; returns the
// unclamped value in raw[3] and, in J[3 c + a], the derivative of channel c
// with respect to component a of the unit direction (sum over the basis of
// coefficient times basis gradient), which the colour backward takes in place
// of the coefficients, and the unit direction and 1 / |mu - pos| it used.
template <int DEG>
__device__ __forceinline__ void sh_color(const SceneDev& S, const ViewConst& v, int64_t n, float* raw, float* J,
                                         float* dir, float& inv_len) {
  const float dx = S.means[3 * n] - v.pos[0], dy = S.means[3 * n + 1] - v.pos[1], dz = S.means[3 * n + 2] - v.pos[2];
  const float il = 1.0f / __builtin_sqrtf(dx * dx + dy * dy + dz * dz);
  dir[0] = dx * il;
  dir[1] = dy * il;
  dir[2] = dz * il;
  inv_len = il;
  float Y[16], dY[16][3];
  sh_basis(DEG, dir[0], dir[1], dir[2], Y);
  sh_basis_grad(DEG, dir[0], dir[1], dir[2], dY);
  constexpr int nb = (DEG + 1) * (DEG + 1), nc = 3 * nb;
  // the coefficient row, as float4s when its length allows (rows are 16-byte
  // aligned: the scene's array is, and a row is a multiple of 16 bytes)
  float c[nc];
  if (nc % 4 == 0) {
    const float4* c4 = reinterpret_cast<const float4*>(S.sh + (int64_t)nc * n);
#pragma unroll
    for (int q = 0; q < nc / 4; ++q) {
      const float4 x = c4[q];
      c[4 * q] = x.x;
      c[4 * q + 1] = x.y;
      c[4 * q + 2] = x.z;
      c[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int f = 0; f < nc; ++f) c[f] = S.sh[(int64_t)nc * n + f];
  }
  float r = 0.5f, g = 0.5f, b = 0.5f;
#pragma unroll
  for (int q = 0; q < 9; ++q) J[q] = 0.0f;
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    const float c0 = c[3 * k], c1 = c[3 * k + 1], c2 = c[3 * k + 2];
    r = __builtin_fmaf(c0, Y[k], r);
    g = __builtin_fmaf(c1, Y[k], g);
    b = __builtin_fmaf(c2, Y[k], b);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      J[a] = __builtin_fmaf(c0, dY[k][a], J[a]);
      J[3 + a] = __builtin_fmaf(c1, dY[k][a], J[3 + a]);
      J[6 + a] = __builtin_fmaf(c2, dY[k][a], J[6 + a]);
    }
  }
  raw[0] = r;
  raw[1] = g;
  raw[2] = b;
}

template <int DEG>
__global__ void __launch_bounds__(kBlock) k_project(SceneDev S, const ViewConst* __restrict__ vp, const int32_t* idx,
                                                    const int32_t* d_count, int64_t cap, Splat* splats,
                                                    uint32_t* depth_key, uint32_t* tiles, ushort4* rect,
                                                    float* dcol) {
  const ViewConst v = *vp;
  const int64_t n = clamp_count(d_count, cap);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t node = idx[i];
    Proj P = project_node(S, v, node);
    uint32_t t = 0;
    if (P.visible) {
      float raw[3], J[9], dir[3], il;
      sh_color<DEG>(S, v, node, raw, J, dir, il);
      P.sp.r = fmaxf(raw[0], 0.0f);
      P.sp.g = fmaxf(raw[1], 0.0f);
      P.sp.b = fmaxf(raw[2], 0.0f);
      const uint32_t clamp = (raw[0] < 0.0f ? 1u : 0u) | (raw[1] < 0.0f ? 2u : 0u) | (raw[2] < 0.0f ? 4u : 0u);
      // the colour backward's record: everything it needs but the gradients
      float4* rec = reinterpret_cast<float4*>(dcol + kColorRec * i);
      rec[0] = make_float4(J[0], J[1], J[2], J[3]);
      rec[1] = make_float4(J[4], J[5], J[6], J[7]);
      rec[2] = make_float4(J[8], dir[0], dir[1], dir[2]);
      rec[3] = make_float4(il, __uint_as_float(clamp), 0.0f, 0.0f);
      t = (uint32_t)((P.x1 - P.x0) * (P.y1 - P.y0));
      splats[i] = P.sp;
      depth_key[i] = __float_as_uint(P.depth);
      rect[i] = make_ushort4((unsigned short)P.x0, (unsigned short)P.x1, (unsigned short)P.y0, (unsigned short)P.y1);
    }
    tiles[i] = t;  // 0: not drawn
  }
}

struct LoadDrawn {
  const uint32_t* tiles;
  __device__ uint32_t operator()(int64_t i) const { return tiles[i] != 0u ? 1u : 0u; }
};

// Order-preserving compaction of the drawn splats, done by the scan of their
// flags: the drawn splat at selection position i has rank = its prefix among
// the drawn ones; (depth key, i) go to that rank (the sort's input), and so
// does i in the list of drawn selection positions (kept for the backward).
struct StoreDrawn {
  const uint32_t* depth_key;
  uint32_t* key_out;
  uint32_t* val_out;
  uint32_t* list;
  __device__ void operator()(int64_t i, uint32_t prefix, uint32_t drawn) const {
    if (!drawn) return;
    key_out[prefix] = depth_key[i];
    val_out[prefix] = (uint32_t)i;
    list[prefix] = (uint32_t)i;
  }
};

struct LoadTilesInOrder {
  const uint32_t* tiles;
  const uint32_t* order;
  __device__ uint32_t operator()(int64_t r) const { return tiles[order[r]]; }
};

// Instance emission, load-balanced over the instances: the instances (splat,
// tile) in depth order of their splats are cut into chunks of 64 and each
// wave takes a contiguous run of chunks.  The drawn splats whose instances
// meet a chunk (at most 64, as every drawn splat has one) are found from the
// instance offsets (the scan of the tile counts in depth order): a 64-ary
// search for the wave's first chunk, then one comparison per chunk.  Lane l
// loads the l-th of them (splat, rectangle, 64-byte record and the per-splat
// part of the block mask) into LDS; lane l then emits instance k0 + l, whose
// splat is the last one starting at or before it (a binary search over the
// chunk's splats in LDS).  An instance is its tile key (tile row-major in the
// rectangle), its emission index (the tile sort carries it) and the (splat,
// block mask) word: the 4x4 blocks of the tile that the splat's alpha >=
// 1/255 ellipse can reach (splat_block_mask).  The chunk holding a splat's
// first instance also writes the splat's record for the projection backward
// (rank_info) and lists it when it has more than kLongSegment instances.  The
// instance count is clamped to the capacity here (block 0 publishes the
// clamped count and flags an overflow); only instances below it are emitted,
// so only splats whose first instance is emitted get a record or a place on
// the list.
constexpr int kDupWaves = kBlock / 64;

__global__ void __launch_bounds__(kBlock) k_dup(FrameCounters* ctr, const uint32_t* order, const uint32_t* inst_off,
                                                int32_t tiles_x, int64_t cap, uint32_t* ikey, uint32_t* ival,
                                                uint2* inst_info, uint32_t* long_list,
                                                const Splat* __restrict__ splats, uint4* rank_info) {
  __shared__ Splat rec[kDupWaves][64];
  __shared__ MaskSetup msk[kDupWaves][64];
  __shared__ uint4 own[kDupWaves][64];  // (splat, instance offset, rectangle width, x0 | y0 << 16)
  const uint32_t total = (uint32_t)ctr->n_instances;  // the scan's 32-bit sum
  const int64_t n = (int64_t)total > cap ? cap : (int64_t)total;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctr->n_inst_clamped = (int32_t)n;
    if ((int64_t)total > cap) ctr->status = LODGS_E_CAPACITY;
  }
  const int64_t nd = ctr->n_drawn;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nchunks = (n + 63) / 64, nw = (int64_t)gridDim.x * kDupWaves;
  const int64_t per = (nchunks + nw - 1) / nw;
  const int64_t c0 = ((int64_t)blockIdx.x * kDupWaves + wv) * per;
  const int64_t c1 = c0 + per < nchunks ? c0 + per : nchunks;
  if (c0 >= c1) return;  // wave-uniform; no block barrier below
  // rf = the last drawn splat with inst_off[rf] <= 64 c0 (inst_off[0] = 0,
  // offsets strictly increase): 64 samples of [lo, hi) per step, the answer
  // stays in [lo, hi)
  int64_t lo = 0, hi = nd;
  {
    const uint32_t k0 = (uint32_t)(64 * c0);
    while (hi - lo > 1) {  // wave-uniform
      const int64_t span = hi - lo;
      const bool le = inst_off[lo + span * lane / 64] <= k0;  // a prefix of the lanes (lane 0 always)
      const int m = 63 - __builtin_clzll(__ballot(le));
      const int64_t nlo = lo + span * m / 64;
      hi = m == 63 ? hi : lo + span * (m + 1) / 64;
      lo = nlo;
    }
  }
  int64_t rf = lo;
  for (int64_t c = c0; c < c1; ++c) {  // wave-uniform
    const int64_t k0 = 64 * c, k1 = k0 + 64 < n ? k0 + 64 : n;
    // the splats rf .. rf + cnt - 1 start before k1
    const int64_t r = rf + lane;
    const uint32_t off = r < nd ? inst_off[r] : 0xFFFFFFFFu;
    const bool in = r < nd && (int64_t)off < k1;  // a prefix of the lanes (lane 0 always)
    const int cnt = __popcll(__ballot(in));
    if (in) {
      const uint32_t i = order[r];
      const Splat sp = splats[i];  // the one random read per splat (the record holds the rectangle)
      const uint32_t x0 = sp.rect_x & 0xFFFFu, y0 = sp.rect_y & 0xFFFFu;
      const uint32_t w = (sp.rect_x >> 16) - x0, h = (sp.rect_y >> 16) - y0;
      rec[wv][lane] = sp;
      msk[wv][lane] = block_mask_setup(sp);
      own[wv][lane] = make_uint4(i, off, w, x0 | (y0 << 16));
      if ((int64_t)off >= k0) {  // the splat's first instance is in this chunk
        rank_info[2 * r] = make_uint4(i, 0u, sp.rect_x, sp.rect_y);
        rank_info[2 * r + 1] = make_uint4(__float_as_uint(sp.mxh), __float_as_uint(sp.mxl), __float_as_uint(sp.myh),
                                          __float_as_uint(sp.myl));
        if (w * h > kLongSegment) long_list[atomicAdd(&ctr->n_long, 1)] = (uint32_t)r;
      }
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t k = k0 + lane;
    if (k < k1) {
      int o = 0;  // the last of the chunk's splats starting at or before k
#pragma unroll
      for (int step = 32; step > 0; step >>= 1)
        if (o + step < cnt && (int64_t)own[wv][o + step].y <= k) o += step;
      const uint4 ow = own[wv][o];
      const uint32_t l = (uint32_t)(k - ow.y);
      const uint32_t ty = (ow.w >> 16) + l / ow.z, tx = (ow.w & 0xFFFFu) + l % ow.z;
      ikey[k] = ty * (uint32_t)tiles_x + tx;
      ival[k] = (uint32_t)k;  // the tile sort carries the emission index
      inst_info[k] = make_uint2(ow.x, splat_block_mask(rec[wv][o], msk[wv][o], (int)tx, (int)ty));
    }
    __builtin_amdgcn_wave_barrier();  // rec, msk and own are rewritten by the next chunk
    // the next chunk's first splat: the last one starting at or before k1
    const int64_t rn = rf + cnt;
    const uint32_t offn = rn < nd ? inst_off[rn] : 0xFFFFFFFFu;
    rf = (int64_t)offn == k1 ? rn : rn - 1;
  }
}

// Tile ranges from the tile-sorted keys, one thread per boundary k in
// [0, n]: between the keys t0 = key[k - 1] and t1 = key[k] (-1 before the
// first, ntiles after the last; keys >= ntiles, which only an instance
// overflow produces, count as ntiles) tile t0 ends at k, tile t1 starts at k,
// and every tile strictly between them is empty (k, k).
__global__ void __launch_bounds__(kBlock) k_ranges(const FrameCounters* ctr, const uint32_t* key, uint2* ranges,
                                                   uint32_t ntiles) {
  const int64_t n = ctr->n_inst_clamped;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t0 = k > 0 ? (int64_t)min(key[k - 1], ntiles) : -1;
    const int64_t t1 = k < n ? (int64_t)min(key[k], ntiles) : (int64_t)ntiles;
    if (t0 == t1) continue;
    if (t0 >= 0 && t0 < ntiles) ranges[t0].y = (uint32_t)k;
    if (t1 < ntiles) ranges[t1].x = (uint32_t)k;
    for (int64_t t = t0 + 1; t < t1; ++t) ranges[t] = make_uint2((uint32_t)k, (uint32_t)k);
  }
}

// Workgroup order of the blend kernels: tiles by descending class of their
// instance count n (the bit length of n and the two bits below its leading
// one, so classes are a quarter octave wide), so the longest workgroups start
// early; results do not depend on the order of the tiles.  Workgroup b orders
// the chunk of kOrderChunk tiles starting at b * kOrderChunk (a 1080p frame
// has one chunk): each tile takes its rank within its class from an LDS
// counter, and a scan over the classes gives each class its start.  The
// order within a class is whatever the LDS atomics give.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBatch = 8;  // tiles per thread
constexpr int32_t kOrderChunk = kOrderThreads * kOrderBatch;
static_assert(kTileClasses == 128, "one thread per class in waves 0 and 1");

__device__ __forceinline__ int tile_class(uint2 r) {
  const uint32_t n = r.y - r.x;
  const int bl = min(31, 32 - __clz((int)n));  // 0 for an empty tile
  const int sub = bl >= 3 ? (int)((n >> (bl - 3)) & 3u) : 0;
  return bl * 4 + sub;  // < kTileClasses
}

__global__ void __launch_bounds__(kOrderThreads) k_tile_order(const uint2* ranges, int32_t ntiles, uint32_t* order) {
  __shared__ uint32_t cnt[kTileClasses];
  __shared__ uint32_t half[2];
  const int32_t lo = blockIdx.x * kOrderChunk;
  const int32_t n = min(kOrderChunk, ntiles - lo);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint2 r[kOrderBatch];
#pragma unroll
  for (int k = 0; k < kOrderBatch; ++k) {
    const int32_t t = k * kOrderThreads + (int32_t)threadIdx.x;
    r[k] = t < n ? ranges[lo + t] : make_uint2(0u, 0u);
  }
  if (threadIdx.x < kTileClasses) cnt[threadIdx.x] = 0;
  __syncthreads();
  uint32_t key[kOrderBatch];  // class << 16 | rank within the class (rank < kOrderChunk)
#pragma unroll
  for (int k = 0; k < kOrderBatch; ++k) {
    const int32_t t = k * kOrderThreads + (int32_t)threadIdx.x;
    key[k] = 0;
    if (t < n) {
      const int c = tile_class(r[k]);
      key[k] = ((uint32_t)c << 16) | atomicAdd(&cnt[c], 1u);
    }
  }
  __syncthreads();
  // cnt[c] becomes the tiles of all classes above c (waves 0 and 1, whole waves)
  const int c = threadIdx.x;
  uint32_t incl = 0;
  if (c < kTileClasses) {
    incl = cnt[c];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) half[wv] = incl;
  }
  __syncthreads();
  if (c < kTileClasses) cnt[c] = half[0] + half[1] - (incl + (wv == 1 ? half[0] : 0u));
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kOrderBatch; ++k) {
    const int32_t t = k * kOrderThreads + (int32_t)threadIdx.x;
    if (t < n) order[lo + cnt[key[k] >> 16] + (key[k] & 0xFFFFu)] = (uint32_t)(lo + t);
  }
}

// One workgroup per tile with 4/PX waves, PX pixels per lane; each 16-lane
// row of a wave covers 4x4 pixel blocks (blend_pixel).  Per batch of
// instances, every row lists the instances whose block mask (k_dup) meets
// its blocks and replays only those, in order: elsewhere alpha < 1/255 at
// every pixel.  The rows of a wave step through their lists together, each on
// its own splat.  For every instance that it replays, the forward records in
// event[k] the blocks where some pixel blended the splat or stopped on it;
// elsewhere the splat changed nothing, which lets the backward skip it there.
// alpha = min(0.99, o e^power), skipped below 1/255; a pixel stops before its
// transmittance would drop below 1e-4.  Splat records are staged in LDS one
// batch per workgroup size and read into registers one list entry ahead; the
// per-pixel steps are written with selects, so the only branches are
// wave-uniform.  The counting variant lists every instance in every row (the
// algorithmic evaluation count: every splat of the tile up to termination).
template <bool COUNT, int PX>
__global__ void __launch_bounds__(256 / PX) k_blend(const ViewConst* __restrict__ vp, const uint2* __restrict__ ranges,
                                                    const uint2* __restrict__ info_k,
                                                    const Splat* __restrict__ splats, const FrameCounters* ctr,
                                                    const uint32_t* __restrict__ tile_order, float bg0, float bg1,
                                                    float bg2, float* rgb, uint32_t* event, unsigned long long* work) {
  constexpr int NT = 256 / PX, NW = 4 / PX;
  const ViewConst v = *vp;
  __shared__ Splat batch[NT];
  __shared__ uint32_t ev[NT];
  __shared__ uint32_t bm[NT];
  __shared__ uint8_t hits[NW][4][NT];  // per row of each wave: the batch slots it replays, in order
  const int tile = (int)tile_order[blockIdx.x];
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4;
  int px, pys[PX];
  float fy[PX], T[PX], cr[PX], cg[PX], cb[PX];
  uint32_t pbit[PX];
  bool inside[PX], live[PX];
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    blend_pixel<PX>(tx, ty, wv, lane, p, px, pys[p]);
    pbit[p] = blend_pixel_block<PX>(wv, g, p);
    fy[p] = (float)pys[p] + 0.5f;
    inside[p] = px < v.width && pys[p] < v.height;
    live[p] = inside[p];
    T[p] = 1.0f;
    cr[p] = cg[p] = cb[p] = 0.0f;
  }
  const float fx = (float)px + 0.5f;
  const uint2 rg = ranges[tile];
  const uint32_t nr = (uint32_t)ctr->n_render;
  const float thr = 1.0f / 255.0f;
  unsigned long long n_eval = 0, n_contrib = 0;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += NT) {
    bool active = false;
#pragma unroll
    for (int p = 0; p < PX; ++p) active = active || live[p];
    if (__syncthreads_count(active) == 0) break;
    const uint32_t k = b0 + threadIdx.x;
    ev[threadIdx.x] = 0u;
    if (k < rg.y) {
      const uint2 w = info_k[k];
      const uint32_t i = w.x;
      bm[threadIdx.x] = w.y;
      if (i < nr) {
        batch[threadIdx.x] = splats[i];
      } else {  // only reachable if the instance count overflowed (its block mask is 0)
        batch[threadIdx.x].o = 0.0f;
      }
    }
    __syncthreads();
    const int m = (int)min((uint32_t)NT, rg.y - b0);
    int nh[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) nh[r] = wave_hit_list<NT, COUNT>(m, blend_row_blocks<PX>(wv, r), bm, hits[wv][r]);
    __syncthreads();
    const int n = g == 0 ? nh[0] : (g == 1 ? nh[1] : (g == 2 ? nh[2] : nh[3]));  // this row's list
    const int nmax = max(max(nh[0], nh[1]), max(nh[2], nh[3]));
    // one splat (batch slot j of this row's list; has = false past its end)
    // against the row's pixels; true when every pixel of the wave has stopped
    auto step = [&](const Splat& s, int j, bool has) -> bool {
      bool act = false;
      uint32_t eb = 0u;
#pragma unroll
      for (int p = 0; p < PX; ++p) {
        float dx, dy, u1, u2;
        const float power = splat_power(s, fx, fy[p], dx, dy, u1, u2);
        const float alpha = fminf(0.99f, s.o * fexp(power));
        const float tt = T[p] * (1.0f - alpha);
        const bool in = live[p] & has;
        const bool hit = in & (alpha >= thr);
        const bool stop = hit & (tt < 0.0001f);
        const bool con = hit & !stop;
        if (COUNT) {
          n_eval += in ? 1 : 0;
          n_contrib += con ? 1 : 0;
        }
        live[p] = live[p] & !stop;
        const float w = alpha * T[p];
        cr[p] = con ? __builtin_fmaf(s.r, w, cr[p]) : cr[p];
        cg[p] = con ? __builtin_fmaf(s.g, w, cg[p]) : cg[p];
        cb[p] = con ? __builtin_fmaf(s.b, w, cb[p]) : cb[p];
        T[p] = con ? tt : T[p];
        act = act | live[p];
        if (!COUNT && ((__ballot(hit) >> (lane & 48)) & 0xFFFFull) != 0ull) eb |= pbit[p];
      }
      if (!COUNT && (lane & 15) == 0 && eb != 0u) atomicOr(&ev[j], eb);
      return !__any(act);
    };
    if (__any(active) && nmax > 0) {  // wave-uniform
      // two register sets, each loaded one list entry ahead of its use
      const uint8_t* hl = hits[wv][g];
      // (an entry is read unconditionally, within the row's 64 bytes, and
      // replaced by 0 past the list's end, so every read is a plain LDS load)
      auto slot = [&](int t) -> int {
        const int e = (int)hl[t & 63];
        return t < n ? e : 0;
      };
      Splat sa = batch[slot(0)], sb;
      for (int t = 0;;) {
        const int ja = slot(t);
        const bool ha = t < n;
        sb = batch[slot(t + 1)];
        if (step(sa, ja, ha) || ++t >= nmax) break;
        const int jb = slot(t);
        const bool hb = t < n;
        sa = batch[slot(t + 1)];
        if (step(sb, jb, hb) || ++t >= nmax) break;
      }
    }
    if (!COUNT) {
      __syncthreads();
      if ((int)threadIdx.x < m) event[b0 + threadIdx.x] = event_word(ev[threadIdx.x]);
    }
  }
  if (COUNT) {
    for (int d = 32; d > 0; d >>= 1) {
      n_eval += __shfl_xor(n_eval, d, 64);
      n_contrib += __shfl_xor(n_contrib, d, 64);
    }
    if (lane == 0) {
      atomicAdd(work, n_eval);
      atomicAdd(work + 1, n_contrib);
    }
    return;
  }
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    if (!inside[p]) continue;
    float* o = rgb + 3 * ((int64_t)pys[p] * v.width + px);
    o[0] = __builtin_fmaf(T[p], bg0, cr[p]);
    o[1] = __builtin_fmaf(T[p], bg1, cg[p]);
    o[2] = __builtin_fmaf(T[p], bg2, cb[p]);
  }
}

// Forward blend with one wave per 8x8 quarter of a tile (four single-wave
// workgroups per tile, tiles in the blend order): the wave's rows are the
// quarter's four 4x4 blocks (blend_pixel<1>), lane l its pixel.  The wave
// streams the tile's instances in batches of 64 and replays, row by row, the
// ones whose block mask meets the row's block, as k_blend does.  Instance
// words (owning splat, block mask, gathered in tile order) are loaded two
// batches ahead and the splat records of the instances that reach the quarter
// one batch ahead, into registers, so the loads overlap the blending; the
// waves of a tile never wait for each other, and each stops when its own
// pixels have.  Events: byte q of each instance's event word holds quarter q's
// (4-bit) events, written by quarter q's wave, zero for instances it never
// reached.
__global__ void __launch_bounds__(64) k_blend_q(const ViewConst* __restrict__ vp, const uint2* __restrict__ ranges,
                                                const uint2* __restrict__ info_k,
                                                const Splat* __restrict__ splats, const FrameCounters* ctr,
                                                const uint32_t* __restrict__ tile_order, float bg0, float bg1,
                                                float bg2, float* rgb, uint8_t* event8) {
  const ViewConst v = *vp;
  __shared__ float4 rec[3][64];     // the batch's records: (mx hi, lo, my hi, lo), (ce, se, h1, h2), (o, r, g, b)
  __shared__ uint8_t hits[4][64];   // per row: the batch slots it replays, in order
  __shared__ uint32_t evr[64];      // per slot: this quarter's event bits
  const int tile = (int)tile_order[blockIdx.x >> 2], q = (int)(blockIdx.x & 3u);
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int lane = threadIdx.x, g = lane >> 4;
  const uint64_t lt = lanemask_lt();
  int px, py;
  blend_pixel<1>(tx, ty, q, lane, 0, px, py);
  const uint32_t pbit = blend_pixel_block<1>(q, g, 0);
  const uint32_t qbits = 0xFu << (4 * q);
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const bool inside = px < v.width && py < v.height;
  bool live = inside;
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  const uint2 rg = ranges[tile];
  const uint32_t nr = (uint32_t)ctr->n_render;
  const float thr = 1.0f / 255.0f;
  // pipeline: words of batches b and b + 64, the record of batch b (this lane's slot)
  uint32_t sk0 = 0u, bk0 = 0u, sk1 = 0u, bk1 = 0u;
  if (rg.x + lane < rg.y) {
    const uint2 w = info_k[rg.x + lane];
    sk0 = w.x;
    bk0 = w.y;
  }
  if (rg.x + 64 + lane < rg.y) {
    const uint2 w = info_k[rg.x + 64 + lane];
    sk1 = w.x;
    bk1 = w.y;
  }
  float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra, rc = ra;
  if (rg.x + lane < rg.y && sk0 < nr && (bk0 & qbits) != 0u) {
    const float4* r = reinterpret_cast<const float4*>(splats + sk0);
    ra = r[0];
    rb = r[1];
    rc = r[2];
  }
  uint32_t b0 = rg.x;
  for (; b0 < rg.y; b0 += 64) {
    if (!__any(live)) break;  // wave-uniform
    const int m = (int)min(64u, rg.y - b0);
    const bool mine = lane < m && sk0 < nr;
    rec[0][lane] = ra;
    rec[1][lane] = rb;
    rec[2][lane] = rc;
    evr[lane] = 0u;
    int nh[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool h = mine && (bk0 & blend_row_blocks<1>(q, r)) != 0u;
      const uint64_t hb = __ballot(h);
      if (h) hits[r][__popcll(hb & lt)] = (uint8_t)lane;
      nh[r] = __popcll(hb);
    }
    __syncthreads();
    // prefetch: the records of the next batch, the words of the one after
    ra = rb = rc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (b0 + 64 + lane < rg.y && sk1 < nr && (bk1 & qbits) != 0u) {
      const float4* r = reinterpret_cast<const float4*>(splats + sk1);
      ra = r[0];
      rb = r[1];
      rc = r[2];
    }
    uint32_t sk2 = 0u, bk2 = 0u;
    if (b0 + 128 + lane < rg.y) {
      const uint2 w = info_k[b0 + 128 + lane];
      sk2 = w.x;
      bk2 = w.y;
    }
    const int n = g == 0 ? nh[0] : (g == 1 ? nh[1] : (g == 2 ? nh[2] : nh[3]));  // this row's list
    const int nmax = max(max(nh[0], nh[1]), max(nh[2], nh[3]));
    auto load = [&](int j) -> Splat {
      Splat s;
      const float4 a = rec[0][j], b = rec[1][j], c = rec[2][j];
      s.mxh = a.x; s.mxl = a.y; s.myh = a.z; s.myl = a.w;
      s.ce = b.x; s.se = b.y; s.h1 = b.z; s.h2 = b.w;
      s.o = c.x; s.r = c.y; s.g = c.z; s.b = c.w;
      return s;
    };
    // one splat (slot j of this row's list; has = false past its end) against
    // the lane's pixel; true when every pixel of the wave has stopped
    auto step = [&](const Splat& s, int j, bool has) -> bool {
      float dx, dy, u1, u2;
      const float power = splat_power(s, fx, fy, dx, dy, u1, u2);
      const float alpha = fminf(0.99f, s.o * fexp(power));
      const float tt = T * (1.0f - alpha);
      const bool hit = live & has & (alpha >= thr);
      const bool stop = hit & (tt < 0.0001f);
      const bool con = hit & !stop;
      live = live & !stop;
      const float w = alpha * T;
      cr = con ? __builtin_fmaf(s.r, w, cr) : cr;
      cg = con ? __builtin_fmaf(s.g, w, cg) : cg;
      cb = con ? __builtin_fmaf(s.b, w, cb) : cb;
      T = con ? tt : T;
      const uint64_t hb = __ballot(hit);  // all lanes
      if ((lane & 15) == 0 && ((hb >> lane) & 0xFFFFull) != 0ull) atomicOr(&evr[j], pbit);
      return !__any(live);
    };
    if (nmax > 0) {
      const uint8_t* hl = hits[g];
      // (an entry is read unconditionally, within the row's 64 bytes, and
      // replaced by 0 past the list's end, so every read is a plain LDS load)
      auto slot = [&](int t) -> int {
        const int e = (int)hl[t & 63];
        return t < n ? e : 0;
      };
      // records one entry ahead of their use, list entries two ahead (so a
      // record's LDS read never waits for the read of its slot index)
      int ja = slot(0), jb = slot(1);
      Splat sa = load(ja), sb;
      for (int t = 0;;) {
        const int jc = slot(t + 2);
        sb = load(jb);
        if (step(sa, ja, t < n) || ++t >= nmax) break;
        const int jd = slot(t + 2);
        sa = load(jc);
        if (step(sb, jb, t < n) || ++t >= nmax) break;
        ja = jc;
        jb = jd;
      }
    }
    __syncthreads();
    if (lane < m) event8[4 * (int64_t)(b0 + lane) + q] = (uint8_t)((evr[lane] >> (4 * q)) & 0xFu);
    __syncthreads();
    sk0 = sk1;
    bk0 = bk1;
    sk1 = sk2;
    bk1 = bk2;
  }
  // instances of the tile that this quarter never reached
  for (uint32_t k = b0 + lane; k < rg.y; k += 64) event8[4 * (int64_t)k + q] = 0;
  if (inside) {
    float* o = rgb + 3 * ((int64_t)py * v.width + px);
    o[0] = __builtin_fmaf(T, bg0, cr);
    o[1] = __builtin_fmaf(T, bg1, cg);
    o[2] = __builtin_fmaf(T, bg2, cb);
  }
}

template <bool COUNT>
static void launch_blend(lodgs_frame* f, const ViewConst& v, const float bg[3], float* d_rgb, hipStream_t st) {
  const int ntiles = v.tiles_x * v.tiles_y;
  unsigned long long* work = COUNT ? f->work : nullptr;
  uint32_t* event = COUNT ? nullptr : f->inst_event;
  if (!COUNT && f->blend_px_fwd == 1) {
    hipLaunchKernelGGL(k_blend_q, dim3(4 * ntiles), dim3(64), 0, st, f->d_view_ren, f->ranges, f->sorted_info,
                       f->splats, f->ctr, f->tile_order, bg[0], bg[1], bg[2], d_rgb,
                       reinterpret_cast<uint8_t*>(event));
    return;
  }
  switch (f->blend_px_fwd) {
    case 1:
      hipLaunchKernelGGL((k_blend<COUNT, 1>), dim3(ntiles), dim3(256), 0, st, f->d_view_ren, f->ranges,
                         f->sorted_info, f->splats, f->ctr, f->tile_order, bg[0], bg[1], bg[2],
                         d_rgb, event, work);
      break;
    case 4:
      hipLaunchKernelGGL((k_blend<COUNT, 4>), dim3(ntiles), dim3(64), 0, st, f->d_view_ren, f->ranges,
                         f->sorted_info, f->splats, f->ctr, f->tile_order, bg[0], bg[1], bg[2],
                         d_rgb, event, work);
      break;
    default:
      hipLaunchKernelGGL((k_blend<COUNT, 2>), dim3(ntiles), dim3(128), 0, st, f->d_view_ren, f->ranges,
                         f->sorted_info, f->splats, f->ctr, f->tile_order, bg[0], bg[1], bg[2],
                         d_rgb, event, work);
      break;
  }
}

int blend_output_arg(const void* func, int* n_args) {
  // k_blend_q (..., bg2, rgb, event8) and k_blend<false, PX> (..., bg2, rgb, event, work)
  if (func == reinterpret_cast<const void*>(&k_blend_q)) {
    *n_args = 11;
    return 9;
  }
  if (func == reinterpret_cast<const void*>(&k_blend<false, 1>) ||
      func == reinterpret_cast<const void*>(&k_blend<false, 2>) ||
      func == reinterpret_cast<const void*>(&k_blend<false, 4>)) {
    *n_args = 12;
    return 9;
  }
  return -1;
}

void launch_render(lodgs_frame* f, const int32_t* d_idx, const int32_t* d_count, const ViewConst& v,
                   const float bg[3], float* d_rgb, hipStream_t st) {
  const SceneDev& S = render_params(f);
  const int64_t cap = f->caps.max_selected, icap = f->caps.max_instances;
  stage_begin(f, LODGS_STAGE_PROJECT, st);
  launch_set_view(v, f->d_view_ren, f->ctr, kViewRender, d_count, cap, st);
  const int pgrid = 2048;
  switch (S.sh_degree) {
#define LODGS_PROJECT(D)                                                                                         \
  hipLaunchKernelGGL(k_project<D>, dim3(pgrid), dim3(kBlock), 0, st, S, f->d_view_ren, d_idx, d_count, cap,   \
                     f->splats, f->depth_key, f->tiles, f->rect, f->dcol)
    case 0: LODGS_PROJECT(0); break;
    case 1: LODGS_PROJECT(1); break;
    case 2: LODGS_PROJECT(2); break;
    default: LODGS_PROJECT(3); break;
#undef LODGS_PROJECT
  }
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_DEPTH_SORT, st);
  // drawn splats only: ranks among them in selection order, then a stable
  // sort of their depth keys, ties in selection order
  scan_exclusive(LoadDrawn{f->tiles}, &f->ctr->n_render, cap, f->block_sums,
                 StoreDrawn{f->depth_key, f->depth_key2, f->order, f->drawn_list}, &f->ctr->n_drawn,
                 st);
  SortScratch ws{f->sort_table, f->sort_below};
  const bool sw = sort_pairs(f->depth_key2, f->order, f->depth_key, f->order2, &f->ctr->n_drawn, cap, 32, ws, st);
  const uint32_t* order = sw ? f->order2 : f->order;
  f->sorted_order = order;
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_DUPLICATE, st);
  scan_exclusive(LoadTilesInOrder{f->tiles, order}, &f->ctr->n_drawn, cap, f->block_sums, f->inst_off,
                 &f->ctr->n_instances, st);
  hipLaunchKernelGGL(k_dup, dim3(pgrid), dim3(kBlock), 0, st, f->ctr, order, f->inst_off, v.tiles_x, icap, f->ikey,
                     f->ival, f->inst_info, f->long_list, f->splats, f->rank_info);
  stage_end(f, st);
  const int ntiles = v.tiles_x * v.tiles_y;
  int tbits = 8;
  while ((1 << tbits) < ntiles) tbits += 8;
  stage_begin(f, LODGS_STAGE_TILE_SORT, st);
  // the (splat, block mask) word of each instance moves with it (read in
  // emission order, so coalesced)
  const bool sw2 = sort_pairs(f->ikey, f->ival, f->ikey2, f->ival2, &f->ctr->n_inst_clamped, icap, tbits, ws, st,
                              f->inst_info, f->info_k);
  f->sorted_ikey = sw2 ? f->ikey2 : f->ikey;
  f->sorted_ival = sw2 ? f->ival2 : f->ival;
  f->sorted_info = sw2 ? f->info_k : f->inst_info;
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_RANGES, st);
  hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(kBlock), 0, st, f->ctr, f->sorted_ikey, f->ranges, (uint32_t)ntiles);
  if (ntiles > 0)
    hipLaunchKernelGGL(k_tile_order, dim3((ntiles + kOrderChunk - 1) / kOrderChunk), dim3(kOrderThreads), 0, st,
                       f->ranges, ntiles, f->tile_order);
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_BLEND, st);
  launch_blend<false>(f, v, bg, d_rgb, st);
  stage_end(f, st);
}

__global__ void k_zero_work(unsigned long long* w) {
  w[0] = 0;
  w[1] = 0;
}

void launch_blend_count(lodgs_frame* f, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_work, dim3(1), dim3(1), 0, st, f->work);
  const float zero[3] = {0.0f, 0.0f, 0.0f};
  launch_blend<true>(f, f->view, zero, nullptr, st);
}

}  // namespace lodgs
