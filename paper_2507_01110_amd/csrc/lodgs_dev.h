// Device-side definitions shared by the library's kernels (gfx950).
//
// FP32 arithmetic here follows fixed operation orders: every discrete
// decision of the path (LoD test, frustum test, near-plane test, tile
// rectangle, depth key, alpha skip/clamp, early termination) must be
// reproducible bit for bit.  The library is compiled with -ffp-contract=off,
// correctly rounded FP32 division and square root, and FP32 denormals kept;
// fused multiply-adds appear only where written as __builtin_fmaf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lodgs.h"

namespace lodgs {

constexpr int kTile = 16;
constexpr int kWave = 64;

// Camera plus per-view constants derived on the host in FP32.
struct ViewConst {
  float R[9], t[3], pos[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float z_near;
  // LoD: X = d * k, k = tau / fx
  float k;
  // LoD noise: the distance to an SPT root is multiplied by spt_scale before
  // that SPT's cut and the cut cache's ratio test (1: no noise); upper nodes
  // keep their own distance
  float spt_scale;
  // frustum side planes x/z <= hr, -x/z <= hl, y/z <= hb, -y/z <= ht, with
  // normalisers n* = sqrt(1 + h*^2)
  float hl, hr, ht, hb, nl, nr, nt, nb;
  int32_t tiles_x, tiles_y;
};

ViewConst make_view(const lodgs_camera& c, float tau);

// e^x for the FP32 path: Cody-Waite reduction x = n ln2 + r (ln2 split in a
// high part with trailing zero bits and a low part), degree-7 Taylor
// polynomial of e^r by Horner with fused multiply-adds, scaling by 2^n.
// Returns 0 below -87 and for NaN; clamps the argument at 88.
// Written with selects rather than branches (same arithmetic on live lanes).
__device__ __forceinline__ float fexp(float x) {
  const bool live = x >= -87.0f;  // false for NaN
  x = x > 88.0f ? 88.0f : x;
  x = live ? x : 0.0f;
  const float n = __builtin_rintf(x * 1.44269502f);
  float r = __builtin_fmaf(-n, 0.693145752f, x);
  r = __builtin_fmaf(-n, 1.42860677e-06f, r);
  float p = 1.98412701e-04f;
  p = __builtin_fmaf(p, r, 1.38888892e-03f);
  p = __builtin_fmaf(p, r, 8.33333377e-03f);
  p = __builtin_fmaf(p, r, 4.16666679e-02f);
  p = __builtin_fmaf(p, r, 1.66666672e-01f);
  p = __builtin_fmaf(p, r, 0.5f);
  p = __builtin_fmaf(p, r, 1.0f);
  p = __builtin_fmaf(p, r, 1.0f);
  return live ? __builtin_ldexpf(p, (int)n) : 0.0f;
}

// |mu - pos| as sqrt((dx*dx + dy*dy) + dz*dz).
__device__ __forceinline__ float view_distance(const ViewConst& v, float mx, float my, float mz) {
  const float dx = mx - v.pos[0], dy = my - v.pos[1], dz = mz - v.pos[2];
  float s = dx * dx;
  s = s + dy * dy;
  s = s + dz * dz;
  return __builtin_sqrtf(s);
}

// x_cam row r = ((R[r0] mx + R[r1] my) + R[r2] mz) + t[r].
__device__ __forceinline__ void to_camera(const ViewConst& v, float mx, float my, float mz, float& cx, float& cy,
                                          float& cz) {
  float a = v.R[0] * mx;
  a = a + v.R[1] * my;
  a = a + v.R[2] * mz;
  cx = a + v.t[0];
  float b = v.R[3] * mx;
  b = b + v.R[4] * my;
  b = b + v.R[5] * mz;
  cy = b + v.t[1];
  float c = v.R[6] * mx;
  c = c + v.R[7] * my;
  c = c + v.R[8] * mz;
  cz = c + v.t[2];
}

// Sphere (mu, rho) entirely outside the near plane or one of the side planes.
__device__ __forceinline__ bool sphere_culled(const ViewConst& v, float mx, float my, float mz, float rho) {
  float cx, cy, cz;
  to_camera(v, mx, my, mz, cx, cy, cz);
  if (cz + rho < v.z_near) return true;
  if (cx - v.hr * cz > rho * v.nr) return true;
  if (-cx - v.hl * cz > rho * v.nl) return true;
  if (cy - v.hb * cz > rho * v.nb) return true;
  if (-cy - v.ht * cz > rho * v.nt) return true;
  return false;
}

// Per-splat record read by the blend kernels (64 bytes, 16-byte aligned):
// the projected mean as hi/lo float pairs, the principal axis (ce, se) of the
// projected covariance and the power coefficients h1 = -1/(2 l1),
// h2 = -1/(2 l2) of its eigenvalues (power = h1 u1^2 + h2 u2^2 in that
// basis), opacity, colour, footprint radius and the colour clamp decisions.
struct alignas(16) Splat {
  float mxh, mxl, myh, myl;
  float ce, se, h1, h2;
  float o, r, g, b;
  uint32_t rect_x;  // tile rectangle: x0 | x1 << 16 (columns [x0, x1))
  uint32_t rect_y;  // y0 | y1 << 16 (rows [y0, y1))
  uint32_t pad0, pad1;
};

// Power of a splat at the pixel centre (px, py), FP32, fixed operation order.
__device__ __forceinline__ float splat_power(const Splat& s, float px, float py, float& dx, float& dy, float& u1,
                                             float& u2) {
  dx = (px - s.mxh) - s.mxl;
  dy = (py - s.myh) - s.myl;
  u1 = s.ce * dx;
  u1 = __builtin_fmaf(s.se, dy, u1);
  u2 = s.ce * dy;
  u2 = __builtin_fmaf(-s.se, dx, u2);
  float a2 = s.h2 * u2;
  a2 = a2 * u2;
  return __builtin_fmaf(s.h1 * u1, u1, a2);
}

// Real SH basis constants, l <= 3 (3DGS sign convention).
constexpr float kSH0 = 0.28209479177387814f;
constexpr float kSH1 = 0.4886025119029199f;
constexpr float kSH2_0 = 1.0925484305920792f, kSH2_1 = -1.0925484305920792f, kSH2_2 = 0.31539156525252005f,
                kSH2_3 = -1.0925484305920792f, kSH2_4 = 0.5462742152960396f;
constexpr float kSH3_0 = -0.5900435899266435f, kSH3_1 = 2.890611442640554f, kSH3_2 = -0.4570457994644658f,
                kSH3_3 = 0.3731763325901154f, kSH3_4 = -0.4570457994644658f, kSH3_5 = 1.445305721320277f,
                kSH3_6 = -0.5900435899266435f;

// Fills Y[0 .. (deg+1)^2) for the unit direction (x, y, z).
__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
  Y[0] = kSH0;
  if (deg < 1) return;
  Y[1] = -kSH1 * y;
  Y[2] = kSH1 * z;
  Y[3] = -kSH1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kSH2_0 * x * y;
  Y[5] = kSH2_1 * y * z;
  Y[6] = kSH2_2 * (2.0f * zz - xx - yy);
  Y[7] = kSH2_3 * x * z;
  Y[8] = kSH2_4 * (xx - yy);
  if (deg < 3) return;
  Y[9] = kSH3_0 * y * (3.0f * xx - yy);
  Y[10] = kSH3_1 * x * y * z;
  Y[11] = kSH3_2 * y * (4.0f * zz - xx - yy);
  Y[12] = kSH3_3 * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = kSH3_4 * x * (4.0f * zz - xx - yy);
  Y[14] = kSH3_5 * z * (xx - yy);
  Y[15] = kSH3_6 * x * (xx - 3.0f * yy);
}

// Gradient of the basis polynomials with respect to (x, y, z): dY[k][3].
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, float (*dY)[3]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) dY[k][0] = dY[k][1] = dY[k][2] = 0.0f;
  if (deg < 1) return;
  dY[1][1] = -kSH1;
  dY[2][2] = kSH1;
  dY[3][0] = -kSH1;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  dY[4][0] = kSH2_0 * y; dY[4][1] = kSH2_0 * x;
  dY[5][1] = kSH2_1 * z; dY[5][2] = kSH2_1 * y;
  dY[6][0] = -2.0f * kSH2_2 * x; dY[6][1] = -2.0f * kSH2_2 * y; dY[6][2] = 4.0f * kSH2_2 * z;
  dY[7][0] = kSH2_3 * z; dY[7][2] = kSH2_3 * x;
  dY[8][0] = 2.0f * kSH2_4 * x; dY[8][1] = -2.0f * kSH2_4 * y;
  if (deg < 3) return;
  dY[9][0] = 6.0f * kSH3_0 * x * y; dY[9][1] = kSH3_0 * (3.0f * xx - 3.0f * yy);
  dY[10][0] = kSH3_1 * y * z; dY[10][1] = kSH3_1 * x * z; dY[10][2] = kSH3_1 * x * y;
  dY[11][0] = -2.0f * kSH3_2 * x * y; dY[11][1] = kSH3_2 * (4.0f * zz - xx - 3.0f * yy);
  dY[11][2] = 8.0f * kSH3_2 * y * z;
  dY[12][0] = -6.0f * kSH3_3 * x * z; dY[12][1] = -6.0f * kSH3_3 * y * z;
  dY[12][2] = kSH3_3 * (6.0f * zz - 3.0f * xx - 3.0f * yy);
  dY[13][0] = kSH3_4 * (4.0f * zz - 3.0f * xx - yy); dY[13][1] = -2.0f * kSH3_4 * x * y;
  dY[13][2] = 8.0f * kSH3_4 * x * z;
  dY[14][0] = 2.0f * kSH3_5 * x * z; dY[14][1] = -2.0f * kSH3_5 * y * z; dY[14][2] = kSH3_5 * (xx - yy);
  dY[15][0] = kSH3_6 * (3.0f * xx - 3.0f * yy); dY[15][1] = -6.0f * kSH3_6 * x * y;
}

// Smallest value of -power = a1 u1^2 + a2 u2^2 (a = -h > 0, u the splat's
// eigenbasis coordinates of the offset from its mean) over the pixel-centre
// rectangle [x0, x1] x [y0, y1]: zero when the mean lies inside, otherwise
// the smallest of the four edge minima (a convex quadratic on a segment).
__device__ __forceinline__ float splat_rect_min(const Splat& s, float x0, float x1, float y0, float y1) {
  const float a1 = -s.h1, a2 = -s.h2;
  const float mx = s.mxh + s.mxl, my = s.myh + s.myl;
  if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.0f;
  float best = 3.0e38f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // edges: bottom/top (along x) and left/right (along y)
    const bool along_x = k < 2;
    const float px = (k == 3) ? x1 : x0, py = (k == 1) ? y1 : y0;
    const float len = along_x ? x1 - x0 : y1 - y0;
    const float dx = (px - s.mxh) - s.mxl, dy = (py - s.myh) - s.myl;
    const float c1 = __builtin_fmaf(s.se, dy, s.ce * dx), c2 = __builtin_fmaf(-s.se, dx, s.ce * dy);
    const float e1 = along_x ? s.ce : s.se, e2 = along_x ? -s.se : s.ce;
    const float den = __builtin_fmaf(a1 * e1, e1, a2 * e2 * e2);
    float t = den > 0.0f ? -__builtin_fmaf(a1 * c1, e1, a2 * c2 * e2) / den : 0.0f;
    t = fminf(fmaxf(t, 0.0f), len);
    const float u1 = __builtin_fmaf(t, e1, c1), u2 = __builtin_fmaf(t, e2, c2);
    best = fminf(best, __builtin_fmaf(a1 * u1, u1, a2 * u2 * u2));
  }
  return best;
}

// Bit of the 4x4 block (bx, by) of a 16x16 tile in block masks and events:
// quarter-major, 4 q + b with q = (bx >> 1) + 2 (by >> 1) the 8x8 quarter and
// b = (bx & 1) + 2 (by & 1) the block inside it, so the bits of quarter q are
// nibble q.
__device__ __forceinline__ uint32_t block_bit(int bx, int by) {
  return 1u << (4 * ((bx >> 1) + 2 * (by >> 1)) + ((bx & 1) + 2 * (by & 1)));
}

// The per-splat part of splat_block_mask: the bound K, the bounding box's
// half-widths and the mean (ok = false: alpha < 1/255 everywhere).
struct MaskSetup {
  float K, hx, hy, mx, my;
  bool ok;
};

__device__ __forceinline__ MaskSetup block_mask_setup(const Splat& s) {
  MaskSetup m;
  const float lo = 255.0f * s.o;
  m.ok = lo >= 1.0f;
  const float L = __logf(m.ok ? lo : 1.0f);
  m.K = __builtin_fmaf(0.01f, L, L) + 0.02f;
  const float i1 = -1.0f / s.h1, i2 = -1.0f / s.h2;  // 1 / a1, 1 / a2
  const float cc = s.ce * s.ce, ss = s.se * s.se;
  float hx = 1.0001f * __builtin_sqrtf(m.K * __builtin_fmaf(cc, i1, ss * i2)) + 1e-3f;
  float hy = 1.0001f * __builtin_sqrtf(m.K * __builtin_fmaf(ss, i1, cc * i2)) + 1e-3f;
  m.hx = hx == hx ? hx : __builtin_inff();  // no box from a NaN: every block
  m.hy = hy == hy ? hy : __builtin_inff();
  m.mx = s.mxh + s.mxl;
  m.my = s.myh + s.myl;
  return m;
}

// Bit block_bit(bx, by) (the 4x4 block (bx, by) of the 16x16 tile at (tx, ty))
// is set unless alpha < 1/255 is certain at every pixel centre of that block.
// alpha >= 1/255 needs -power = a1 u1^2 + a2 u2^2 <= ln(255 o) (a = -h), an
// ellipse; the mask keeps the blocks that both of two supersets of it reach:
// the 8x8 quarters whose minimum of -power does not exceed the bound, and the
// blocks that meet the ellipse's axis-aligned bounding box (half-widths
// sqrt(K (ce^2 / a1 + se^2 / a2)) and sqrt(K (se^2 / a1 + ce^2 / a2)), sums of
// positive terms).  The bound K carries a margin (1% + 0.02) far above the
// FP32 evaluation error of the power, and the box a further 1e-4 relative +
// 1e-3 px, so a cleared bit only skips known results.
__device__ __forceinline__ uint32_t splat_block_mask(const Splat& s, const MaskSetup& ms, int tx, int ty) {
  if (!ms.ok) return 0u;
  uint32_t quarters = 0u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float x0 = (float)(tx * kTile + 8 * (q & 1)) + 0.5f, y0 = (float)(ty * kTile + 8 * (q >> 1)) + 0.5f;
    if (splat_rect_min(s, x0, x0 + 7.0f, y0, y0 + 7.0f) <= ms.K) quarters |= 1u << q;
  }
  if (quarters == 0u) return 0u;
  uint32_t cols = 0u, rows = 0u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float x0 = (float)(tx * kTile + 4 * k) + 0.5f, y0 = (float)(ty * kTile + 4 * k) + 0.5f;
    if (x0 <= ms.mx + ms.hx && x0 + 3.0f >= ms.mx - ms.hx) cols |= 1u << k;
    if (y0 <= ms.my + ms.hy && y0 + 3.0f >= ms.my - ms.hy) rows |= 1u << k;
  }
  uint32_t m = 0u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!((quarters >> q) & 1u)) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int bx = 2 * (q & 1) + (b & 1), by = 2 * (q >> 1) + (b >> 1);
      if (((cols >> bx) & 1u) && ((rows >> by) & 1u)) m |= 1u << (4 * q + b);
    }
  }
  return m;
}

// Pixel layout of the blend kernels: a 16x16 tile is one workgroup of 4/PX
// waves, PX pixels per lane, and each 16-lane row g of a wave covers 4x4
// pixel blocks (lane l its pixel (l & 3, (l >> 2) & 3) of the block): block
// column bx and, for pixel p, block row by, with
//   PX = 1: wave w on the 8x8 quarter (w & 1, w >> 1): bx = 2 (w & 1) + (g & 1),
//           by = 2 (w >> 1) + (g >> 1); or, SPREAD, bx = g, by = (w + g) & 3,
//           so that every wave has one block in each block row and column (a
//           band of heavy blocks, such as a horizon, spreads over the waves,
//           which meet at every batch);
//   PX = 2: wave w on rows [8 w, 8 w + 8): bx = g, by = 2 w + p;
//   PX = 4: one wave: bx = g, by = p.
// Block bits are block_bit(bx, by), as in splat_block_mask, whatever the
// layout.
template <int PX, bool SPREAD = false>
__device__ __forceinline__ void blend_block(int wv, int g, int p, int& bx, int& by) {
  if (PX == 1 && SPREAD) {
    bx = g;
    by = (wv + g) & 3;
  } else if (PX == 1) {
    bx = 2 * (wv & 1) + (g & 1);
    by = 2 * (wv >> 1) + (g >> 1);
  } else if (PX == 2) {
    bx = g;
    by = 2 * wv + p;
  } else {
    bx = g;
    by = p;
  }
}

template <int PX, bool SPREAD = false>
__device__ __forceinline__ void blend_pixel(int tx, int ty, int wv, int lane, int p, int& x, int& y) {
  int bx, by;
  blend_block<PX, SPREAD>(wv, lane >> 4, p, bx, by);
  x = tx * kTile + 4 * bx + (lane & 3);
  y = ty * kTile + 4 * by + ((lane >> 2) & 3);
}

// Block bit of pixel p of row g of wave w.
template <int PX, bool SPREAD = false>
__device__ __forceinline__ uint32_t blend_pixel_block(int wv, int g, int p) {
  int bx, by;
  blend_block<PX, SPREAD>(wv, g, p, bx, by);
  return block_bit(bx, by);
}

// Forward events of one instance: byte q holds the (4-bit) events of quarter
// q, written by that quarter's wave; as a 16-bit block mask and back.
__device__ __forceinline__ uint32_t event_blocks(uint32_t w) {
  return (w & 0xFu) | ((w >> 4) & 0xF0u) | ((w >> 8) & 0xF00u) | ((w >> 12) & 0xF000u);
}
__device__ __forceinline__ uint32_t event_word(uint32_t m) {
  return (m & 0xFu) | ((m & 0xF0u) << 4) | ((m & 0xF00u) << 8) | ((m & 0xF000u) << 12);
}

// The blocks that row g of wave w covers.
template <int PX, bool SPREAD = false>
__device__ __forceinline__ uint32_t blend_row_blocks(int wv, int g) {
  uint32_t m = 0u;
#pragma unroll
  for (int p = 0; p < PX; ++p) m |= blend_pixel_block<PX, SPREAD>(wv, g, p);
  return m;
}

// Sum over the 64 lanes of a wave with DPP lane moves, result in lane 63:
// swaps inside quads, row rotations by 4 and 8 (every lane then holds its
// 16-lane row's sum), then the row broadcasts 15 and 31 fold the rows into
// the last one.  Lanes that do not take part must pass 0.
#define LODGS_DPP(x, ctrl, row_mask) \
  __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, row_mask, 0xf, false))
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += LODGS_DPP(v, 0xB1, 0xf);   // quad_perm [1,0,3,2]
  v += LODGS_DPP(v, 0x4E, 0xf);   // quad_perm [2,3,0,1]
  v += LODGS_DPP(v, 0x124, 0xf);  // row_ror 4
  v += LODGS_DPP(v, 0x128, 0xf);  // row_ror 8
  v += LODGS_DPP(v, 0x142, 0xa);  // row_bcast 15 into rows 1 and 3
  v += LODGS_DPP(v, 0x143, 0xc);  // row_bcast 31 into rows 2 and 3
  return v;
}
#undef LODGS_DPP

// Grid-stride bounds for kernels whose element count lives in device memory.
__device__ __forceinline__ int64_t clamp_count(const int32_t* d_n, int64_t cap) {
  int64_t n = *d_n;
  if (n < 0) n = 0;
  return n < cap ? n : cap;
}

}  // namespace lodgs
