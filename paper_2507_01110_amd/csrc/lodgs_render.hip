// Forward render of a selected set (Sec. 3: EWA projection, SH colour, Eq. 1
// front-to-back compositing with Eq. 2's alpha), tiled 16x16.
//
//  k_project  one thread per selected node: camera transform, near-plane test,
//             covariance from (scale, rotation), EWA Jacobian, projected
//             covariance + 0.3 px^2, conic, square footprint, tile rectangle,
//             opacity, SH colour.  Writes a 48-byte Splat record, the depth key
//             and the tile count.
//  sort       stable radix sort of the selected splats by FP32 depth bits, then
//             (k_dup) one (tile, splat) instance per covered tile emitted in
//             depth order, then a stable radix sort of the instances by tile:
//             the result is the order of the 64-bit key (tile << 32 | depth),
//             ties by selection order, with far less key traffic.
//  k_ranges   first/last instance of every tile.
//  k_blend    one workgroup per tile, one lane per pixel; splat records are
//             staged in LDS in batches of 256.
#include "lodgs_internal.h"

namespace lodgs {

// FP32 projection of one node (the decisions of the path are taken here).
struct Proj {
  bool visible;
  float depth;
  Splat sp;
  int x0, x1, y0, y1;
};

__device__ __forceinline__ int tile_clamp(float v, int hi) {
  if (v < 0.0f) return 0;
  if (v > (float)hi) return hi;
  return (int)v;
}

__device__ __forceinline__ Proj project_node(const SceneDev& S, const ViewConst& v, int32_t node) {
  Proj P;
  P.visible = false;
  P.x0 = P.x1 = P.y0 = P.y1 = 0;
  const int64_t n = node;
  const float mx = S.means[3 * n], my = S.means[3 * n + 1], mz = S.means[3 * n + 2];
  float cx, cy, cz;
  to_camera(v, mx, my, mz, cx, cy, cz);
  P.depth = cz;
  if (!(cz > v.z_near)) return P;
  const float s0 = fexp(S.log_scales[3 * n]), s1 = fexp(S.log_scales[3 * n + 1]), s2 = fexp(S.log_scales[3 * n + 2]);
  const float4 q = *reinterpret_cast<const float4*>(S.quats + 4 * n);
  float qq = q.x * q.x;
  qq = qq + q.y * q.y;
  qq = qq + q.z * q.z;
  qq = qq + q.w * q.w;
  const float ql = __builtin_sqrtf(qq);
  const float w = q.x / ql, x = q.y / ql, y = q.z / ql, z = q.w / ql;
  const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  const float r00 = 1.0f - 2.0f * (yy + zz), r01 = 2.0f * (xy - wz), r02 = 2.0f * (xz + wy);
  const float r10 = 2.0f * (xy + wz), r11 = 1.0f - 2.0f * (xx + zz), r12 = 2.0f * (yz - wx);
  const float r20 = 2.0f * (xz - wy), r21 = 2.0f * (yz + wx), r22 = 1.0f - 2.0f * (xx + yy);
  const float m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
  const float m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
  const float m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
  const float S00 = (m00 * m00 + m01 * m01) + m02 * m02;
  const float S01 = (m00 * m10 + m01 * m11) + m02 * m12;
  const float S02 = (m00 * m20 + m01 * m21) + m02 * m22;
  const float S11 = (m10 * m10 + m11 * m11) + m12 * m12;
  const float S12 = (m10 * m20 + m11 * m21) + m12 * m22;
  const float S22 = (m20 * m20 + m21 * m21) + m22 * m22;
  const float u = cx / cz, vv = cy / cz;
  const float jx = v.fx / cz, jy = v.fy / cz;
  const float jxz = -(jx * u), jyz = -(jy * vv);
  const float* W = v.R;
  const float T00 = jx * W[0] + jxz * W[6], T01 = jx * W[1] + jxz * W[7], T02 = jx * W[2] + jxz * W[8];
  const float T10 = jy * W[3] + jyz * W[6], T11 = jy * W[4] + jyz * W[7], T12 = jy * W[5] + jyz * W[8];
  const float U00 = (T00 * S00 + T01 * S01) + T02 * S02;
  const float U01 = (T00 * S01 + T01 * S11) + T02 * S12;
  const float U02 = (T00 * S02 + T01 * S12) + T02 * S22;
  const float U10 = (T10 * S00 + T11 * S01) + T12 * S02;
  const float U11 = (T10 * S01 + T11 * S11) + T12 * S12;
  const float U12 = (T10 * S02 + T11 * S12) + T12 * S22;
  const float A = ((U00 * T00 + U01 * T01) + U02 * T02) + 0.3f;
  const float B = (U00 * T10 + U01 * T11) + U02 * T12;
  const float C = ((U10 * T10 + U11 * T11) + U12 * T12) + 0.3f;
  const float det = A * C - B * B;
  if (!(det > 0.0f)) return P;
  P.sp.na = -0.5f * (C / det);
  P.sp.nb = B / det;
  P.sp.nc = -0.5f * (A / det);
  P.sp.mx = v.fx * u + v.cx;
  P.sp.my = v.fy * vv + v.cy;
  const float mid = 0.5f * (A + C);
  const float disc = mid * mid - det;
  const float sq = __builtin_sqrtf(fmaxf(0.1f, disc));
  const float l1 = mid + sq;
  const float r = ceilf(3.0f * __builtin_sqrtf(l1));
  P.x0 = tile_clamp(floorf((P.sp.mx - r) * 0.0625f), v.tiles_x);
  P.x1 = tile_clamp(floorf((P.sp.mx + r) * 0.0625f) + 1.0f, v.tiles_x);
  P.y0 = tile_clamp(floorf((P.sp.my - r) * 0.0625f), v.tiles_y);
  P.y1 = tile_clamp(floorf((P.sp.my + r) * 0.0625f) + 1.0f, v.tiles_y);
  P.visible = P.x1 > P.x0 && P.y1 > P.y0;
  const float theta = S.opacity_logits[n];
  P.sp.o = 1.0f / (1.0f + fexp(-theta));
  // Box outside which alpha < 1/255 is certain: alpha >= 1/255 needs
  // q = x^T Sigma'^-1 x <= 2 ln(255 o); |x| <= sqrt(q_max Sigma'_00) per axis.
  // Margins cover FP32 rounding of the power; very anisotropic splats get no box.
  const float l2 = mid - sq;
  const float lo = 255.0f * P.sp.o;
  if (lo < 1.0f) {
    P.sp.ex = -1.0f;
    P.sp.ey = -1.0f;
  } else if (l2 > 0.0f && l1 < 1e5f * l2) {
    const float qmax = 1.1f * (2.0f * __logf(lo) + 0.01f);
    P.sp.ex = __builtin_sqrtf(qmax * A) + 2.0f;
    P.sp.ey = __builtin_sqrtf(qmax * C) + 2.0f;
  } else {
    P.sp.ex = 3.0e38f;
    P.sp.ey = 3.0e38f;
  }
  P.sp.pad = r;
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

__global__ void __launch_bounds__(kBlock) k_project(SceneDev S, ViewConst v, const int32_t* idx,
                                                    const int32_t* d_count, int64_t cap, Splat* splats,
                                                    uint32_t* depth_key, uint32_t* order, uint32_t* tiles,
                                                    ushort4* rect, FrameCounters* ctr) {
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

__global__ void __launch_bounds__(kBlock) k_dup(const FrameCounters* ctr, const uint32_t* order,
                                                const uint32_t* tiles, const uint32_t* inst_off,
                                                const ushort4* rect, int32_t tiles_x, int64_t cap,
                                                uint32_t* ikey, uint32_t* ival) {
  const int64_t n = ctr->n_render;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t i = order[r];
    if (tiles[i] == 0) continue;
    int64_t o = inst_off[r];
    const ushort4 q = rect[i];
    for (int ty = q.z; ty < q.w; ++ty)
      for (int tx = q.x; tx < q.y; ++tx) {
        if (o < cap) {
          ikey[o] = (uint32_t)(ty * tiles_x + tx);
          ival[o] = i;
        }
        ++o;
      }
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
__global__ void __launch_bounds__(256) k_blend(ViewConst v, const uint2* ranges, const uint32_t* ival,
                                               const Splat* splats, const FrameCounters* ctr, float bg0, float bg1,
                                               float bg2, float* rgb) {
  __shared__ Splat batch[256];
  const int tile = blockIdx.x;
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < v.width && py < v.height;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const uint32_t nr = (uint32_t)ctr->n_render;
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  bool done = !inside;
  const float thr = 1.0f / 255.0f;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += 256) {
    if (__syncthreads_count(done) == 256) break;
    const uint32_t k = b0 + threadIdx.x;
    if (k < rg.y) {
      const uint32_t i = ival[k];
      if (i < nr) batch[threadIdx.x] = splats[i];
      else batch[threadIdx.x].o = 0.0f;  // only reachable if the instance count overflowed
    }
    __syncthreads();
    const int m = (int)min(256u, rg.y - b0);
    for (int j = 0; j < m && !done; ++j) {
      const Splat& s = batch[j];
      const float dx = fx - s.mx, dy = fy - s.my;
      float t1 = s.na * dx;
      t1 = __builtin_fmaf(s.nb, dy, t1);
      float u = s.nc * dy;
      u = u * dy;
      const float power = __builtin_fmaf(t1, dx, u);
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
    }
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
  hipLaunchKernelGGL(k_render_begin, dim3(1), dim3(1), 0, st, f->ctr, d_count, cap);
  const int pgrid = 2048;
  hipLaunchKernelGGL(k_project, dim3(pgrid), dim3(kBlock), 0, st, S, v, d_idx, d_count, cap, f->splats, f->depth_key,
                     f->order, f->tiles, f->rect, f->ctr);
  SortScratch ws{f->sort_table, f->block_sums, &f->ctr->sort_table_n};
  const bool sw = sort_pairs(f->depth_key, f->order, f->depth_key2, f->order2, &f->ctr->n_render, cap, 32, ws, st);
  const uint32_t* order = sw ? f->order2 : f->order;
  scan_exclusive(LoadTilesInOrder{f->tiles, order}, &f->ctr->n_render, cap, f->block_sums, f->inst_off,
                 &f->ctr->n_instances, st);
  hipLaunchKernelGGL(k_inst_count, dim3(1), dim3(1), 0, st, f->ctr, icap);
  hipLaunchKernelGGL(k_dup, dim3(pgrid), dim3(kBlock), 0, st, f->ctr, order, f->tiles, f->inst_off, f->rect,
                     v.tiles_x, icap, f->ikey, f->ival);
  const int ntiles = v.tiles_x * v.tiles_y;
  int tbits = 8;
  while ((1 << tbits) < ntiles) tbits += 8;
  const bool sw2 = sort_pairs(f->ikey, f->ival, f->ikey2, f->ival2, &f->ctr->n_inst_clamped, icap, tbits, ws, st);
  f->sorted_ikey = sw2 ? f->ikey2 : f->ikey;
  f->sorted_ival = sw2 ? f->ival2 : f->ival;
  hipLaunchKernelGGL(k_zero_ranges, dim3((ntiles + kBlock - 1) / kBlock), dim3(kBlock), 0, st, f->ranges, ntiles);
  hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(kBlock), 0, st, f->ctr, f->sorted_ikey, f->ranges, (uint32_t)ntiles);
  hipLaunchKernelGGL(k_blend, dim3(ntiles), dim3(256), 0, st, v, f->ranges, f->sorted_ival, f->splats, f->ctr, bg[0],
                     bg[1], bg[2], d_rgb);
}

}  // namespace lodgs
