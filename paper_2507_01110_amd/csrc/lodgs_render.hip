// Forward render of a selected set (Sec. 3: EWA projection, SH colour, Eq. 1
// front-to-back compositing with Eq. 2's alpha), tiled 16x16.
//
//  k_project  one thread per selected node: camera transform, near-plane test,
//             covariance from (scale, rotation), EWA Jacobian, projected
//             covariance + 0.3 px^2, conic, square footprint, tile rectangle,
//             opacity, SH colour.  Writes a 64-byte Splat record, the depth key
//             and the tile count.
//  sort       stable radix sort of the selected splats by FP32 depth bits, then
//             (k_dup) one (tile, splat) instance per covered tile emitted in
//             depth order, then a stable radix sort of the instances by tile:
//             the result is the order of the 64-bit key (tile << 32 | depth),
//             ties by selection order, with far less key traffic.
//  k_ranges   first/last instance of every tile.
//  k_blend    one workgroup per tile, one lane per pixel; splat records are
//             staged in LDS in batches of 256; a wave skips a splat whose
//             alpha >= 1/255 box misses its 16x4 pixels (known result).
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
  Proj64 G;
  const bool ok = proj_chain64(S.means, S.log_scales, S.quats, v, n, G);
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
  const float theta = S.opacity_logits[n];
  P.sp.o = 1.0f / (1.0f + fexp(-theta));
  P.sp.radius = (float)r;
  P.sp.pad = 0.0f;
  // Box outside which alpha < 1/255 is certain: alpha >= 1/255 needs
  // q = x^T Sigma'^-1 x <= 2 ln(255 o), hence |x| <= sqrt(q_max Sigma'_00) per
  // axis.  Margins cover the FP32 evaluation of the power.
  const float lo = 255.0f * P.sp.o;
  if (lo < 1.0f) {
    P.sp.ex = -1.0f;
    P.sp.ey = -1.0f;
  } else {
    const double qmax = 1.05 * (2.0 * (double)__logf(lo) + 0.01);
    P.sp.ex = (float)(__builtin_sqrt(qmax * A) * 1.001 + 1.0);
    P.sp.ey = (float)(__builtin_sqrt(qmax * C) * 1.001 + 1.0);
  }
  return P;
}

// SH colour for the view direction (mu - pos) / |mu - pos|; returns the
// unclamped value in raw[3].
__device__ __forceinline__ void sh_color(const SceneDev& S, const ViewConst& v, int64_t n, float* raw) {
  const float dx = S.means[3 * n] - v.pos[0], dy = S.means[3 * n + 1] - v.pos[1], dz = S.means[3 * n + 2] - v.pos[2];
  const float il = 1.0f / __builtin_sqrtf(dx * dx + dy * dy + dz * dz);
  float Y[16];
  sh_basis(S.sh_degree, dx * il, dy * il, dz * il, Y);
  const int nb = (S.sh_degree + 1) * (S.sh_degree + 1);
  const float* c = S.sh + (int64_t)S.n_coef * n;
  float r = 0.5f, g = 0.5f, b = 0.5f;
  for (int k = 0; k < nb; ++k) {
    r = __builtin_fmaf(c[3 * k], Y[k], r);
    g = __builtin_fmaf(c[3 * k + 1], Y[k], g);
    b = __builtin_fmaf(c[3 * k + 2], Y[k], b);
  }
  raw[0] = r;
  raw[1] = g;
  raw[2] = b;
}

__global__ void __launch_bounds__(kBlock) k_project(SceneDev S, const ViewConst* __restrict__ vp, const int32_t* idx,
                                                    const int32_t* d_count, int64_t cap, Splat* splats,
                                                    uint32_t* depth_key, uint32_t* order, uint32_t* tiles,
                                                    ushort4* rect, FrameCounters* ctr) {
  const ViewConst v = *vp;
  const int64_t n = clamp_count(d_count, cap);
  int drawn = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t node = idx[i];
    Proj P = project_node(S, v, node);
    uint32_t t = 0;
    if (P.visible) {
      float raw[3];
      sh_color(S, v, node, raw);
      P.sp.r = fmaxf(raw[0], 0.0f);
      P.sp.g = fmaxf(raw[1], 0.0f);
      P.sp.b = fmaxf(raw[2], 0.0f);
      t = (uint32_t)((P.x1 - P.x0) * (P.y1 - P.y0));
      splats[i] = P.sp;
      ++drawn;
    }
    depth_key[i] = P.visible ? __float_as_uint(P.depth) : 0xFFFFFFFFu;
    order[i] = (uint32_t)i;
    tiles[i] = t;
    rect[i] = make_ushort4((unsigned short)P.x0, (unsigned short)P.x1, (unsigned short)P.y0, (unsigned short)P.y1);
  }
  for (int d = 32; d > 0; d >>= 1) drawn += __shfl_xor(drawn, d, 64);
  if ((threadIdx.x & 63) == 0 && drawn) atomicAdd(&ctr->n_drawn, drawn);
}

__global__ void k_render_begin(FrameCounters* ctr, const int32_t* d_count, int64_t cap) {
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  ctr->n_render = (int32_t)n;
  ctr->n_drawn = 0;
}

struct LoadTilesInOrder {
  const uint32_t* tiles;
  const uint32_t* order;
  __device__ uint32_t operator()(int64_t r) const { return tiles[order[r]]; }
};

__global__ void k_inst_count(FrameCounters* ctr, int64_t cap) {
  const int32_t n = ctr->n_instances;
  ctr->n_inst_clamped = n > cap ? (int32_t)cap : n;
  if (n > cap) ctr->status = LODGS_E_CAPACITY;
}

// One thread per (splat, tile) instance: the owning splat is found by binary
// search over the instance offsets of the drawn splats (which lead the depth
// order), so splats covering thousands of tiles cost no more than small ones.
__global__ void __launch_bounds__(kBlock) k_dup(const FrameCounters* ctr, const uint32_t* order,
                                                const uint32_t* inst_off, const ushort4* rect, int32_t tiles_x,
                                                uint32_t* ikey, uint32_t* ival) {
  const int64_t n = ctr->n_inst_clamped;
  const int32_t nd = ctr->n_drawn;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = nd;  // largest r < nd with inst_off[r] <= k
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (inst_off[mid] <= (uint32_t)k) lo = mid;
      else hi = mid;
    }
    const uint32_t i = order[lo];
    const uint32_t l = (uint32_t)k - inst_off[lo];
    const ushort4 q = rect[i];
    const uint32_t w = (uint32_t)(q.y - q.x);
    if (w == 0) {  // only reachable if the instance count overflowed
      ikey[k] = 0xFFFFFFFFu;
      ival[k] = i;
      continue;
    }
    const uint32_t ty = q.z + l / w, tx = q.x + l % w;
    ikey[k] = ty * (uint32_t)tiles_x + tx;
    ival[k] = i;
  }
}

__global__ void __launch_bounds__(kBlock) k_zero_ranges(uint2* ranges, int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) ranges[i] = make_uint2(0, 0);
}

__global__ void __launch_bounds__(kBlock) k_ranges(const FrameCounters* ctr, const uint32_t* key, uint2* ranges,
                                                   uint32_t ntiles) {
  const int64_t n = ctr->n_inst_clamped;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t t = key[k];
    if (t >= ntiles) continue;  // only reachable if the instance count overflowed
    if (k == 0 || key[k - 1] != t) ranges[t].x = (uint32_t)k;
    if (k == n - 1 || key[k + 1] != t) ranges[t].y = (uint32_t)(k + 1);
  }
}

// One workgroup per tile, one lane per pixel.  alpha = min(0.99, o e^power),
// skipped below 1/255; stop before the transmittance would drop below 1e-4.
template <bool COUNT>
__global__ void __launch_bounds__(256) k_blend(const ViewConst* __restrict__ vp, const uint2* ranges, const uint32_t* ival,
                                               const Splat* splats, const FrameCounters* ctr, float bg0, float bg1,
                                               float bg2, float* rgb, unsigned long long* work) {
  const ViewConst v = *vp;
  __shared__ Splat batch[256];
  const int tile = blockIdx.x;
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < v.width && py < v.height;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  // pixel-centre rectangle of this wave (16 x 4 pixels)
  const float wx0 = (float)(tx * kTile) + 0.5f, wx1 = wx0 + 15.0f;
  const float wy0 = (float)(ty * kTile + 4 * (threadIdx.x >> 6)) + 0.5f, wy1 = wy0 + 3.0f;
  const uint2 rg = ranges[tile];
  const uint32_t nr = (uint32_t)ctr->n_render;
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  bool done = !inside;
  const float thr = 1.0f / 255.0f;
  unsigned long long n_eval = 0, n_contrib = 0;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += 256) {
    if (__syncthreads_count(done) == 256) break;
    const uint32_t k = b0 + threadIdx.x;
    if (k < rg.y) {
      const uint32_t i = ival[k];
      if (i < nr) {
        batch[threadIdx.x] = splats[i];
      } else {  // only reachable if the instance count overflowed
        batch[threadIdx.x].o = 0.0f;
        batch[threadIdx.x].ex = -1.0f;
      }
    }
    __syncthreads();
    const int m = (int)min(256u, rg.y - b0);
    for (int j = 0; j < m && !done; ++j) {
      const Splat& s = batch[j];
      if (COUNT) ++n_eval;
      else if (splat_misses(s, wx0, wx1, wy0, wy1)) continue;
      float dx, dy, u1, u2;
      const float power = splat_power(s, fx, fy, dx, dy, u1, u2);
      const float alpha = fminf(0.99f, s.o * fexp(power));
      if (alpha < thr) continue;
      const float tt = T * (1.0f - alpha);
      if (tt < 0.0001f) {
        done = true;
        break;
      }
      const float w = alpha * T;
      cr = __builtin_fmaf(s.r, w, cr);
      cg = __builtin_fmaf(s.g, w, cg);
      cb = __builtin_fmaf(s.b, w, cb);
      T = tt;
      if (COUNT) ++n_contrib;
    }
  }
  if (COUNT) {
    for (int d = 32; d > 0; d >>= 1) {
      n_eval += __shfl_xor(n_eval, d, 64);
      n_contrib += __shfl_xor(n_contrib, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(work, n_eval);
      atomicAdd(work + 1, n_contrib);
    }
    return;
  }
  if (inside) {
    float* o = rgb + 3 * ((int64_t)py * v.width + px);
    o[0] = __builtin_fmaf(T, bg0, cr);
    o[1] = __builtin_fmaf(T, bg1, cg);
    o[2] = __builtin_fmaf(T, bg2, cb);
  }
}

void launch_render(lodgs_frame* f, const int32_t* d_idx, const int32_t* d_count, const ViewConst& v,
                   const float bg[3], float* d_rgb, hipStream_t st) {
  const SceneDev& S = f->scene->dev;
  const int64_t cap = f->caps.max_selected, icap = f->caps.max_instances;
  stage_begin(f, LODGS_STAGE_PROJECT, st);
  launch_set_view(v, f->d_view_ren, st);
  hipLaunchKernelGGL(k_render_begin, dim3(1), dim3(1), 0, st, f->ctr, d_count, cap);
  const int pgrid = 2048;
  hipLaunchKernelGGL(k_project, dim3(pgrid), dim3(kBlock), 0, st, S, f->d_view_ren, d_idx, d_count, cap, f->splats, f->depth_key,
                     f->order, f->tiles, f->rect, f->ctr);
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_DEPTH_SORT, st);
  SortScratch ws{f->sort_table, f->block_sums, &f->ctr->sort_table_n};
  const bool sw = sort_pairs(f->depth_key, f->order, f->depth_key2, f->order2, &f->ctr->n_render, cap, 32, ws, st);
  const uint32_t* order = sw ? f->order2 : f->order;
  f->sorted_order = order;
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_DUPLICATE, st);
  scan_exclusive(LoadTilesInOrder{f->tiles, order}, &f->ctr->n_render, cap, f->block_sums, f->inst_off,
                 &f->ctr->n_instances, st);
  hipLaunchKernelGGL(k_inst_count, dim3(1), dim3(1), 0, st, f->ctr, icap);
  hipLaunchKernelGGL(k_dup, dim3(pgrid), dim3(kBlock), 0, st, f->ctr, order, f->inst_off, f->rect, v.tiles_x,
                     f->ikey, f->ival);
  stage_end(f, st);
  const int ntiles = v.tiles_x * v.tiles_y;
  int tbits = 8;
  while ((1 << tbits) < ntiles) tbits += 8;
  stage_begin(f, LODGS_STAGE_TILE_SORT, st);
  const bool sw2 = sort_pairs(f->ikey, f->ival, f->ikey2, f->ival2, &f->ctr->n_inst_clamped, icap, tbits, ws, st);
  f->sorted_ikey = sw2 ? f->ikey2 : f->ikey;
  f->sorted_ival = sw2 ? f->ival2 : f->ival;
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_RANGES, st);
  hipLaunchKernelGGL(k_zero_ranges, dim3((ntiles + kBlock - 1) / kBlock), dim3(kBlock), 0, st, f->ranges, ntiles);
  hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(kBlock), 0, st, f->ctr, f->sorted_ikey, f->ranges, (uint32_t)ntiles);
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_BLEND, st);
  hipLaunchKernelGGL(k_blend<false>, dim3(ntiles), dim3(256), 0, st, f->d_view_ren, f->ranges, f->sorted_ival, f->splats, f->ctr,
                     bg[0], bg[1], bg[2], d_rgb, (unsigned long long*)nullptr);
  stage_end(f, st);
}

__global__ void k_zero_work(unsigned long long* w) {
  w[0] = 0;
  w[1] = 0;
}

void launch_blend_count(lodgs_frame* f, hipStream_t st) {
  const ViewConst& v = f->view;
  const int ntiles = v.tiles_x * v.tiles_y;
  hipLaunchKernelGGL(k_zero_work, dim3(1), dim3(1), 0, st, f->work);
  hipLaunchKernelGGL(k_blend<true>, dim3(ntiles), dim3(256), 0, st, f->d_view_ren, f->ranges, f->sorted_ival, f->splats, f->ctr,
                     0.0f, 0.0f, 0.0f, (float*)nullptr, f->work);
}

}  // namespace lodgs
