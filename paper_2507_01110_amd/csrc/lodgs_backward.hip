// Backward of the render (recompute-based): per tile, the forward
// front-to-back pass is replayed with identical FP32 decisions and the
// gradient of every contributing (splat, pixel) pair is formed on the fly,
// using the final pixel colour to obtain the colour behind each splat
// (S_i = C_final - C_prefix_i - c_i alpha_i T_i).  Per-splat sums over the
// tile's pixels are gathered in LDS for each batch of 256 splats (LDS atomics
// from the contributing lanes when a wave has at most four of them, else a
// DPP reduction across the wave and one LDS atomic) and flushed with one
// global atomic per splat, tile and value.  A wave skips
// a splat whose alpha >= 1/255 box misses the wave's 16x4 pixels (its result
// there is known to be "skip").  Then one thread per rendered node carries
// the 2D gradients through the conic inverse, the EWA Jacobian, the camera
// transform, the covariance factorisation, the quaternion normalisation, the
// sigmoid and the SH basis to the raw parameters.
#include "lodgs_internal.h"
#include "lodgs_proj.h"

namespace lodgs {

// Reduce-scatter of 9 per-lane values over a wave (all lanes active): four
// DPP exchange steps inside each 16-lane row pair lane l with l^1, l^2, l^7
// and l^15; at each step a lane keeps half of its remaining values (chosen by
// b0^b2, b1^b2, b2^b3 and b3 of l & 15) and adds its partner's copy of that
// half.  Lane l then holds its row's sum of value
// slot(l) = (b0^b2) + 2 (b1^b2) + 4 (b2^b3) + 8 b3 (slots 9..15 are zero);
// in the wave form two cross-row exchanges complete the sums over the wave.
#define LODGS_DPP(x, ctrl) __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xf, 0xf, false))
#define LODGS_RS_PAIR(out, a, b, k, ctrl)       \
  do {                                          \
    const float keep_ = (k) ? (b) : (a);        \
    const float send_ = (k) ? (a) : (b);        \
    (out) = keep_ + LODGS_DPP(send_, ctrl);     \
  } while (0)

__device__ __forceinline__ float row_reduce_scatter9(const float* g, int lane, int& slot) {
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  const bool k1 = (b0 ^ b2) != 0, k2 = (b1 ^ b2) != 0, k3 = (b2 ^ b3) != 0, k4 = b3 != 0;
  float h0, h1, h2, h3, h4;
  LODGS_RS_PAIR(h0, g[0], g[1], k1, 0xB1);  // quad_perm [1,0,3,2]: l^1
  LODGS_RS_PAIR(h1, g[2], g[3], k1, 0xB1);
  LODGS_RS_PAIR(h2, g[4], g[5], k1, 0xB1);
  LODGS_RS_PAIR(h3, g[6], g[7], k1, 0xB1);
  LODGS_RS_PAIR(h4, g[8], 0.0f, k1, 0xB1);
  float q0, q1, q2;
  LODGS_RS_PAIR(q0, h0, h1, k2, 0x4E);  // quad_perm [2,3,0,1]: l^2
  LODGS_RS_PAIR(q1, h2, h3, k2, 0x4E);
  LODGS_RS_PAIR(q2, h4, 0.0f, k2, 0x4E);
  float r0, r1;
  LODGS_RS_PAIR(r0, q0, q1, k3, 0x141);  // row_half_mirror: l^7
  LODGS_RS_PAIR(r1, q2, 0.0f, k3, 0x141);
  float z;
  LODGS_RS_PAIR(z, r0, r1, k4, 0x140);  // row_mirror: l^15
  slot = (int)k1 + 2 * (int)k2 + 4 * (int)k3 + 8 * (int)k4;
  return z;
}

__device__ __forceinline__ float wave_reduce_scatter9(const float* g, int lane, int& slot) {
  float z = row_reduce_scatter9(g, lane, slot);
  z += __shfl_xor(z, 16, 64);
  z += __shfl_xor(z, 32, 64);
  return z;
}
#undef LODGS_RS_PAIR
#undef LODGS_DPP

// Backward of the blend, same layout and decisions as the forward.  Per
// batch, each wave reduces the 9 gradient values of a splat over its lanes
// (only when some lane contributes) and stores them in its own LDS row; the
// workgroup then sums the rows in wave order and writes one 9-float partial
// per (splat, tile) instance at the instance's emission index, with zeros for
// instances that no pixel reached.  No atomics: the result is deterministic.
template <int PX>
__global__ void __launch_bounds__(256 / PX) k_blend_bwd(const ViewConst* __restrict__ vp,
                                                        const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ ival,
                                                        const uint32_t* __restrict__ inst_splat,
                                                        const Splat* __restrict__ splats, const FrameCounters* ctr,
                                                        const float* __restrict__ rgb, const float* __restrict__ dL,
                                                        float* __restrict__ partial) {
  constexpr int NT = 256 / PX, NW = 4 / PX;
  const ViewConst v = *vp;
  __shared__ Splat batch[NT];
  __shared__ uint32_t bid[NT];
  __shared__ float acc[NW][9][NT];
  const int tile = blockIdx.x;
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int px = tx * kTile + (lane & 15);
  const int py0 = ty * kTile + 4 * PX * wv + (lane >> 4);
  const float fx = (float)px + 0.5f;
  float fy[PX], T[PX], P0[PX], P1[PX], P2[PX], C0[PX], C1[PX], C2[PX], G0[PX], G1[PX], G2[PX];
  bool live[PX];
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    const int py = py0 + 4 * p;
    fy[p] = (float)py + 0.5f;
    live[p] = px < v.width && py < v.height;
    T[p] = 1.0f;
    P0[p] = P1[p] = P2[p] = 0.0f;
    C0[p] = C1[p] = C2[p] = G0[p] = G1[p] = G2[p] = 0.0f;
    if (live[p]) {
      const int64_t o = 3 * ((int64_t)py * v.width + px);
      C0[p] = rgb[o];
      C1[p] = rgb[o + 1];
      C2[p] = rgb[o + 2];
      G0[p] = dL[o];
      G1[p] = dL[o + 1];
      G2[p] = dL[o + 2];
    }
  }
  const float wx0 = (float)(tx * kTile) + 0.5f, wx1 = wx0 + 15.0f;
  const float wy0 = (float)(ty * kTile + 4 * PX * wv) + 0.5f, wy1 = wy0 + (float)(4 * PX - 1);
  const uint2 rg = ranges[tile];
  const uint32_t nr = (uint32_t)ctr->n_render;
  const float thr = 1.0f / 255.0f;
  for (int t = threadIdx.x; t < NW * 9 * NT; t += NT) (&acc[0][0][0])[t] = 0.0f;
  uint32_t b0 = rg.x;
  for (; b0 < rg.y; b0 += NT) {
    bool active = false;
#pragma unroll
    for (int p = 0; p < PX; ++p) active = active || live[p];
    if (__syncthreads_count(active) == 0) break;
    const uint32_t k = b0 + threadIdx.x;
    if (k < rg.y) {
      const uint32_t e = ival[k];
      const uint32_t i = inst_splat[e];
      bid[threadIdx.x] = e;
      if (i < nr) {
        batch[threadIdx.x] = splats[i];
      } else {  // only reachable if the instance count overflowed
        batch[threadIdx.x].o = 0.0f;
        batch[threadIdx.x].ex = -1.0f;
      }
    }
    __syncthreads();
    const int m = (int)min((uint32_t)NT, rg.y - b0);
    if (__any(active)) {  // wave-uniform
      // one splat (batch slot j) against the wave's pixels; true when every
      // pixel has stopped
      auto step = [&](const Splat& s, int j) -> bool {
        if (splat_misses(s, wx0, wx1, wy0, wy1)) return false;  // wave-uniform
        float dxs[PX], dys[PX], u1s[PX], u2s[PX], es[PX], oes[PX], als[PX], tts[PX];
        bool cons[PX];
        bool any_con = false, act = false;
#pragma unroll
        for (int p = 0; p < PX; ++p) {
          const float power = splat_power(s, fx, fy[p], dxs[p], dys[p], u1s[p], u2s[p]);
          es[p] = fexp(power);
          oes[p] = s.o * es[p];
          als[p] = fminf(0.99f, oes[p]);
          tts[p] = T[p] * (1.0f - als[p]);
          const bool hit = live[p] & (als[p] >= thr);
          const bool stop = hit & (tts[p] < 0.0001f);
          cons[p] = hit & !stop;
          live[p] = live[p] & !stop;
          any_con = any_con | cons[p];
          act = act | live[p];
        }
        if (__any(any_con)) {  // wave-uniform
          float g[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int p = 0; p < PX; ++p) {
            const float alpha = als[p], Tp = T[p];
            const float w = alpha * Tp;
            const float q0 = __builtin_fmaf(s.r, w, P0[p]);
            const float q1 = __builtin_fmaf(s.g, w, P1[p]);
            const float q2 = __builtin_fmaf(s.b, w, P2[p]);
            const float ia = __builtin_amdgcn_rcpf(1.0f - alpha);  // gradient values only
            float dA = G0[p] * (s.r * Tp - (C0[p] - q0) * ia);
            dA = __builtin_fmaf(G1[p], s.g * Tp - (C1[p] - q1) * ia, dA);
            dA = __builtin_fmaf(G2[p], s.b * Tp - (C2[p] - q2) * ia, dA);
            const bool con = cons[p];
            const bool unclamped = con & (oes[p] <= 0.99f);
            const float dpow = dA * alpha;
            // d power / d mean2D = -2 (h1 u1 e1 + h2 u2 e2), e1 = (ce, se), e2 = (-se, ce)
            const float k1 = -2.0f * s.h1 * u1s[p], k2 = -2.0f * s.h2 * u2s[p];
            const float dx = dxs[p], dy = dys[p];
            g[0] += unclamped ? dpow * (k1 * s.ce - k2 * s.se) : 0.0f;
            g[1] += unclamped ? dpow * (k1 * s.se + k2 * s.ce) : 0.0f;
            g[2] += unclamped ? dpow * (-0.5f * dx * dx) : 0.0f;
            g[3] += unclamped ? dpow * (-dx * dy) : 0.0f;
            g[4] += unclamped ? dpow * (-0.5f * dy * dy) : 0.0f;
            g[5] += unclamped ? dA * es[p] : 0.0f;
            g[6] += con ? G0[p] * w : 0.0f;
            g[7] += con ? G1[p] * w : 0.0f;
            g[8] += con ? G2[p] * w : 0.0f;
            P0[p] = con ? q0 : P0[p];
            P1[p] = con ? q1 : P1[p];
            P2[p] = con ? q2 : P2[p];
            T[p] = con ? tts[p] : Tp;
          }
          int slot;
          const float r = wave_reduce_scatter9(g, lane, slot);
          if (lane < 16 && slot < 9) acc[wv][slot][j] = r;
        }
        return !__any(act);
      };
      // two register sets, each loaded one splat ahead of its use
      Splat sa = batch[0], sb;
      for (int j = 0;;) {
        sb = batch[j + 1 < m ? j + 1 : j];
        if (step(sa, j) || ++j >= m) break;
        sa = batch[j + 1 < m ? j + 1 : j];
        if (step(sb, j) || ++j >= m) break;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      float* dst = partial + 9 * (int64_t)bid[threadIdx.x];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        float r = acc[0][c][threadIdx.x];
        acc[0][c][threadIdx.x] = 0.0f;
#pragma unroll
        for (int w = 1; w < NW; ++w) {
          r += acc[w][c][threadIdx.x];
          acc[w][c][threadIdx.x] = 0.0f;
        }
        dst[c] = r;
      }
    }
  }
  // instances that no pixel of the tile reached
  for (uint32_t k = b0 + threadIdx.x; k < rg.y; k += NT) {
    float* dst = partial + 9 * (int64_t)ival[k];
#pragma unroll
    for (int c = 0; c < 9; ++c) dst[c] = 0.0f;
  }
}

// Projection backward, FP64 (per splat): the forward chain is replayed and the
// 2D gradients (mean2D, conic, opacity, colour) are carried to the raw
// parameters.
// Zeroes the per-selection gradient rows (splats that were not drawn keep 0).
__global__ void __launch_bounds__(kBlock) k_zero_sel(const FrameCounters* ctr, int nc, lodgs_grads sel) {
  const int64_t n = ctr->n_render;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (sel.d_means) for (int k = 0; k < 3; ++k) sel.d_means[3 * i + k] = 0.0f;
    if (sel.d_log_scales) for (int k = 0; k < 3; ++k) sel.d_log_scales[3 * i + k] = 0.0f;
    if (sel.d_quats) for (int k = 0; k < 4; ++k) sel.d_quats[4 * i + k] = 0.0f;
    if (sel.d_opacity_logits) sel.d_opacity_logits[i] = 0.0f;
    if (sel.d_sh) for (int k = 0; k < nc; ++k) sel.d_sh[(int64_t)nc * i + k] = 0.0f;
  }
}

// Per drawn splat (rank r in depth order), the sum of its instance partials,
// which are contiguous in emission order: 16 lanes per splat stride over the
// range, then the in-row reduce-scatter leaves each of the 9 sums in one lane.
// Fixed order, so deterministic; long ranges (splats covering many tiles) are
// spread over 16 lanes instead of one thread.
__global__ void __launch_bounds__(kBlock) k_sum_partials(const FrameCounters* ctr, const uint32_t* inst_off,
                                                         const float* __restrict__ partial, float* grad2d) {
  const int64_t n = ctr->n_drawn;
  const int64_t n_inst = (uint32_t)ctr->n_instances, n_cl = ctr->n_inst_clamped;
  const int lane = threadIdx.x & 63, sub = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r0 = wave * 4; r0 < n; r0 += waves * 4) {  // wave-uniform
    const int64_t r = r0 + (lane >> 4);
    float g[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (r < n) {
      int64_t a = inst_off[r], b = r + 1 < n ? (int64_t)inst_off[r + 1] : n_inst;
      a = a < n_cl ? a : n_cl;
      b = b < n_cl ? b : n_cl;
      for (int64_t q = a + sub; q < b; q += 16) {
#pragma unroll
        for (int c = 0; c < 9; ++c) g[c] += partial[9 * q + c];
      }
    }
    int slot;
    const float z = row_reduce_scatter9(g, lane, slot);  // all lanes active
    if (r < n && slot < 9) grad2d[9 * r + slot] = z;
  }
}

// Colour backward for one splat: dL/dRGB (zero where the forward's FP32
// colour was clamped at 0) to the SH coefficients (written to the optional
// per-selection row and added to the optional node row) and to the view
// direction; returns dL/dmean from the direction term.  DEG is the SH degree,
// so the basis lives in registers.
template <int DEG>
__device__ __forceinline__ void sh_backward(const SceneDev& S, const ViewConst& v, int64_t node, const float* g2,
                                            float* sel_sh, float* node_sh, double* gdir) {
  constexpr int nb = (DEG + 1) * (DEG + 1);
  const float* shc = S.sh + (int64_t)(3 * nb) * node;
  const double mx = S.means[3 * node], my = S.means[3 * node + 1], mz = S.means[3 * node + 2];
  const double dx = mx - (double)v.pos[0], dy = my - (double)v.pos[1], dz = mz - (double)v.pos[2];
  // the forward's FP32 colour decides the clamp at 0
  float raw[3] = {0.5f, 0.5f, 0.5f};
  {
    const float il = 1.0f / __builtin_sqrtf((float)dx * (float)dx + (float)dy * (float)dy + (float)dz * (float)dz);
    float Yf[16];
    sh_basis(DEG, (float)dx * il, (float)dy * il, (float)dz * il, Yf);
#pragma unroll
    for (int k = 0; k < nb; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) raw[c] = __builtin_fmaf(shc[3 * k + c], Yf[k], raw[c]);
  }
  double dRGB[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) dRGB[c] = raw[c] < 0.0f ? 0.0 : (double)g2[6 + c];
  const double dl = __builtin_sqrt(dx * dx + dy * dy + dz * dz);
  const double d0 = dx / dl, d1 = dy / dl, d2 = dz / dl;
  float Y[16], dY[16][3];
  sh_basis(DEG, (float)d0, (float)d1, (float)d2, Y);
  sh_basis_grad(DEG, (float)d0, (float)d1, (float)d2, dY);
  double dd[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < nb; ++k) {
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float gk = (float)(dRGB[c] * (double)Y[k]);
      if (sel_sh) sel_sh[3 * k + c] = gk;
      if (node_sh) node_sh[3 * k + c] += gk;
      a += dRGB[c] * (double)shc[3 * k + c];
    }
    dd[0] += a * (double)dY[k][0];
    dd[1] += a * (double)dY[k][1];
    dd[2] += a * (double)dY[k][2];
  }
  const double dot = dd[0] * d0 + dd[1] * d1 + dd[2] * d2;
  gdir[0] = (dd[0] - d0 * dot) / dl;
  gdir[1] = (dd[1] - d1 * dot) / dl;
  gdir[2] = (dd[2] - d2 * dot) / dl;
}

// One thread per drawn splat: order[0 .. n_drawn) lists exactly the drawn
// splats in depth order (no lanes idle on culled ones).
// The colour part runs first so that its registers are free before the FP64
// geometry chain is replayed.
template <int DEG>
__global__ void __launch_bounds__(kBlock) k_project_bwd(SceneDev S, const ViewConst* __restrict__ vp, const int32_t* idx,
                                                        const FrameCounters* ctr, const uint32_t* order,
                                                        const float* grad2d, lodgs_grads sel, lodgs_grads nodes) {
  const ViewConst v = *vp;
  const int64_t n = ctr->n_drawn;
  constexpr int nc = 3 * (DEG + 1) * (DEG + 1);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = order[r];
    const int64_t node = idx[i];
    float g2[9];  // 2D gradients of the splat (rank r)
#pragma unroll
    for (int c = 0; c < 9; ++c) g2[c] = grad2d[9 * r + c];
    double gdir[3];
    sh_backward<DEG>(S, v, node, g2, sel.d_sh ? sel.d_sh + nc * i : nullptr,
                     nodes.d_sh ? nodes.d_sh + nc * node : nullptr, gdir);
    double gm[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0;
    Proj64 P;
    const bool visible = proj_chain64(S.means, S.log_scales, S.quats, v, node, P);
    if (visible) {
      // opacity
      const double o = 1.0 / (1.0 + (double)fexp(-S.opacity_logits[node]));
      go = (double)g2[5] * o * (1.0 - o);
      // conic -> projected covariance: GS = -Q GQ Q
      const double ca = P.C / P.det, cb = -P.B / P.det, cc = P.A / P.det;
      const double gq00 = g2[2], gq01 = 0.5 * (double)g2[3], gq11 = g2[4];
      const double qg00 = ca * gq00 + cb * gq01, qg01 = ca * gq01 + cb * gq11;
      const double qg10 = cb * gq00 + cc * gq01, qg11 = cb * gq01 + cc * gq11;
      const double GS00 = -(qg00 * ca + qg01 * cb), GS01 = -(qg00 * cb + qg01 * cc);
      const double GS11 = -(qg10 * cb + qg11 * cc);
      // Sigma' = T Sigma T^T: dL/dT = 2 GS T Sigma, dL/dSigma = T^T GS T
      const double* Tm = P.T;
      const double* Sg = P.Sg;
      double TS[6];
      for (int r = 0; r < 2; ++r) {
        TS[3 * r + 0] = Tm[3 * r] * Sg[0] + Tm[3 * r + 1] * Sg[1] + Tm[3 * r + 2] * Sg[2];
        TS[3 * r + 1] = Tm[3 * r] * Sg[1] + Tm[3 * r + 1] * Sg[3] + Tm[3 * r + 2] * Sg[4];
        TS[3 * r + 2] = Tm[3 * r] * Sg[2] + Tm[3 * r + 1] * Sg[4] + Tm[3 * r + 2] * Sg[5];
      }
      double dT[6];
      for (int c = 0; c < 3; ++c) {
        dT[c] = 2.0 * (GS00 * TS[c] + GS01 * TS[3 + c]);
        dT[3 + c] = 2.0 * (GS01 * TS[c] + GS11 * TS[3 + c]);
      }
      double dS[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          dS[3 * a + b] = Tm[a] * (GS00 * Tm[b] + GS01 * Tm[3 + b]) + Tm[3 + a] * (GS01 * Tm[b] + GS11 * Tm[3 + b]);
      // T = J W
      double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
      for (int c = 0; c < 3; ++c) {
        dJ00 += dT[c] * (double)v.R[c];
        dJ02 += dT[c] * (double)v.R[6 + c];
        dJ11 += dT[3 + c] * (double)v.R[3 + c];
        dJ12 += dT[3 + c] * (double)v.R[6 + c];
      }
      const double cx = P.c[0], cy = P.c[1], cz = P.c[2];
      const double fx = v.fx, fy = v.fy;
      const double iz = 1.0 / cz, iz2 = iz * iz, iz3 = iz2 * iz;
      const double dcx = dJ02 * (-fx * iz2) + (double)g2[0] * fx * iz;
      const double dcy = dJ12 * (-fy * iz2) + (double)g2[1] * fy * iz;
      const double dcz = dJ00 * (-fx * iz2) + dJ02 * (2.0 * fx * cx * iz3) + dJ11 * (-fy * iz2) +
                         dJ12 * (2.0 * fy * cy * iz3) + (double)g2[0] * (-fx * cx * iz2) +
                         (double)g2[1] * (-fy * cy * iz2);
      for (int a = 0; a < 3; ++a)
        gm[a] = (double)v.R[a] * dcx + (double)v.R[3 + a] * dcy + (double)v.R[6 + a] * dcz + gdir[a];
      // Sigma = M M^T, M = Rq diag(s)
      double dRq[9];
      for (int c = 0; c < 3; ++c) {
        double ds = 0.0;
        for (int r = 0; r < 3; ++r) {
          const double dm = 2.0 * (dS[3 * r] * P.M[c] + dS[3 * r + 1] * P.M[3 + c] + dS[3 * r + 2] * P.M[6 + c]);
          ds += dm * P.Rq[3 * r + c];
          dRq[3 * r + c] = dm * P.s[c];
        }
        gls[c] = ds * P.s[c];
      }
      const double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
      double dq[4];
      dq[0] = 2.0 * (-z * dRq[1] + y * dRq[2] + z * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
      dq[1] = 2.0 * (y * dRq[1] + z * dRq[2] + y * dRq[3] - 2.0 * x * dRq[4] - w * dRq[5] + z * dRq[6] +
                     w * dRq[7] - 2.0 * x * dRq[8]);
      dq[2] = 2.0 * (-2.0 * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + z * dRq[5] - w * dRq[6] +
                     z * dRq[7] - 2.0 * y * dRq[8]);
      dq[3] = 2.0 * (-2.0 * z * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - 2.0 * z * dRq[4] + y * dRq[5] +
                     x * dRq[6] + y * dRq[7]);
      const double qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
      for (int k = 0; k < 4; ++k) gq[k] = (dq[k] - P.qn[k] * qd) / P.ql;
    }
    if (sel.d_means) for (int k = 0; k < 3; ++k) sel.d_means[3 * i + k] = (float)gm[k];
    if (sel.d_log_scales) for (int k = 0; k < 3; ++k) sel.d_log_scales[3 * i + k] = (float)gls[k];
    if (sel.d_quats) for (int k = 0; k < 4; ++k) sel.d_quats[4 * i + k] = (float)gq[k];
    if (sel.d_opacity_logits) sel.d_opacity_logits[i] = (float)go;
    if (!visible) continue;
    if (nodes.d_means) for (int k = 0; k < 3; ++k) nodes.d_means[3 * node + k] += (float)gm[k];
    if (nodes.d_log_scales) for (int k = 0; k < 3; ++k) nodes.d_log_scales[3 * node + k] += (float)gls[k];
    if (nodes.d_quats) for (int k = 0; k < 4; ++k) nodes.d_quats[4 * node + k] += (float)gq[k];
    if (nodes.d_opacity_logits) nodes.d_opacity_logits[node] += (float)go;
  }
}

template <int DEG>
static void launch_project_bwd_deg(const SceneDev& S, lodgs_frame* f, const lodgs_grads& sel,
                                   const lodgs_grads& nodes, hipStream_t st) {
  hipLaunchKernelGGL(k_project_bwd<DEG>, dim3(1024), dim3(kBlock), 0, st, S, f->d_view_ren, f->r_idx, f->ctr,
                     f->sorted_order, f->grad2d, sel, nodes);
}

void launch_backward(lodgs_frame* f, const float* d_dL, const lodgs_grads* sel, const lodgs_grads* nodes,
                     hipStream_t st) {
  const SceneDev& S = f->scene->dev;
  const ViewConst& v = f->view;
  stage_begin(f, LODGS_STAGE_BLEND_BWD, st);
  const int ntiles = v.tiles_x * v.tiles_y;
  switch (f->blend_px_bwd) {
    case 1:
      hipLaunchKernelGGL(k_blend_bwd<1>, dim3(ntiles), dim3(256), 0, st, f->d_view_ren, f->ranges, f->sorted_ival,
                         f->inst_splat, f->splats, f->ctr, f->r_rgb, d_dL, f->inst_grad);
      break;
    case 4:
      hipLaunchKernelGGL(k_blend_bwd<4>, dim3(ntiles), dim3(64), 0, st, f->d_view_ren, f->ranges, f->sorted_ival,
                         f->inst_splat, f->splats, f->ctr, f->r_rgb, d_dL, f->inst_grad);
      break;
    default:
      hipLaunchKernelGGL(k_blend_bwd<2>, dim3(ntiles), dim3(128), 0, st, f->d_view_ren, f->ranges, f->sorted_ival,
                         f->inst_splat, f->splats, f->ctr, f->r_rgb, d_dL, f->inst_grad);
      break;
  }
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_PROJECT_BWD, st);
  hipLaunchKernelGGL(k_sum_partials, dim3(2048), dim3(kBlock), 0, st, f->ctr, f->inst_off, f->inst_grad, f->grad2d);
  lodgs_grads none{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (sel) hipLaunchKernelGGL(k_zero_sel, dim3(1024), dim3(kBlock), 0, st, f->ctr, S.n_coef, *sel);
  const lodgs_grads gs = sel ? *sel : none, gn = nodes ? *nodes : none;
  switch (S.sh_degree) {
    case 0: launch_project_bwd_deg<0>(S, f, gs, gn, st); break;
    case 1: launch_project_bwd_deg<1>(S, f, gs, gn, st); break;
    case 2: launch_project_bwd_deg<2>(S, f, gs, gn, st); break;
    default: launch_project_bwd_deg<3>(S, f, gs, gn, st); break;
  }
  stage_end(f, st);
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// L1 loss: grad = sign(img - target) / n, loss = sum |img - target| / n.
__global__ void __launch_bounds__(kBlock) k_l1(const float* img, const float* tgt, int64_t n, float* grad,
                                               float* loss) {
  const float inv = 1.0f / (float)n;
  float acc = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = img[i] - tgt[i];
    grad[i] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
    acc += fabsf(d);
  }
  if (!loss) return;
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, acc * inv);
}

__global__ void k_zero_one(float* p) { *p = 0.0f; }

void launch_l1_loss(const float* img, const float* target, int64_t n, float* grad, float* loss, hipStream_t st) {
  if (loss) hipLaunchKernelGGL(k_zero_one, dim3(1), dim3(1), 0, st, loss);
  int64_t g = (n + kBlock - 1) / kBlock;
  g = g > 4096 ? 4096 : g;
  hipLaunchKernelGGL(k_l1, dim3((int)g), dim3(kBlock), 0, st, img, target, n, grad, loss);
}

}  // namespace lodgs
