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

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__global__ void __launch_bounds__(256) k_blend_bwd(const ViewConst* __restrict__ vp, const uint2* ranges, const uint32_t* ival,
                                                   const Splat* splats, const FrameCounters* ctr, const float* rgb,
                                                   const float* dL, float* grad2d) {
  const ViewConst v = *vp;
  __shared__ Splat batch[256];
  __shared__ uint32_t bid[256];
  __shared__ float acc[9][256];
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
  float Cf[3] = {0.0f, 0.0f, 0.0f}, G[3] = {0.0f, 0.0f, 0.0f};
  if (inside) {
    const int64_t p = 3 * ((int64_t)py * v.width + px);
    for (int c = 0; c < 3; ++c) {
      Cf[c] = rgb[p + c];
      G[c] = dL[p + c];
    }
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c][threadIdx.x] = 0.0f;
  float T = 1.0f, P0 = 0.0f, P1 = 0.0f, P2 = 0.0f;
  bool done = !inside;
  const float thr = 1.0f / 255.0f;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += 256) {
    if (__syncthreads_count(done) == 256) break;
    const uint32_t k = b0 + threadIdx.x;
    if (k < rg.y) {
      const uint32_t i = ival[k];
      if (i < nr) {
        bid[threadIdx.x] = i;
        batch[threadIdx.x] = splats[i];
      } else {  // only reachable if the instance count overflowed
        bid[threadIdx.x] = 0;
        batch[threadIdx.x].o = 0.0f;
        batch[threadIdx.x].ex = -1.0f;
      }
    }
    __syncthreads();
    const int m = (int)min(256u, rg.y - b0);
    for (int j = 0; j < m; ++j) {
      if (__all(done)) break;  // wave-uniform
      const Splat& s = batch[j];
      if (splat_misses(s, wx0, wx1, wy0, wy1)) continue;  // wave-uniform
      float g[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      bool contrib = false;
      if (!done) {
        float dx, dy, u1, u2;
        const float power = splat_power(s, fx, fy, dx, dy, u1, u2);
        const float e = fexp(power);
        const float oe = s.o * e;
        const float alpha = fminf(0.99f, oe);
        if (alpha >= thr) {
          const float tt = T * (1.0f - alpha);
          if (tt < 0.0001f) {
            done = true;
          } else {
            contrib = true;
            const float w = alpha * T;
            g[6] = G[0] * w;
            g[7] = G[1] * w;
            g[8] = G[2] * w;
            P0 = __builtin_fmaf(s.r, w, P0);
            P1 = __builtin_fmaf(s.g, w, P1);
            P2 = __builtin_fmaf(s.b, w, P2);
            const float ia = __builtin_amdgcn_rcpf(1.0f - alpha);  // gradient values only
            float dA = G[0] * (s.r * T - (Cf[0] - P0) * ia);
            dA = __builtin_fmaf(G[1], s.g * T - (Cf[1] - P1) * ia, dA);
            dA = __builtin_fmaf(G[2], s.b * T - (Cf[2] - P2) * ia, dA);
            if (oe <= 0.99f) {
              const float dpow = dA * alpha;
              // d power / d mean2D = Sigma'^-1 (x - mean) = -2 (h1 u1 e1 + h2 u2 e2)
              const float k1 = -2.0f * s.h1 * u1, k2 = -2.0f * s.h2 * u2;
              g[0] = dpow * (k1 * s.ce - k2 * s.se);
              g[1] = dpow * (k1 * s.se + k2 * s.ce);
              g[2] = dpow * (-0.5f * dx * dx);
              g[3] = dpow * (-dx * dy);
              g[4] = dpow * (-0.5f * dy * dy);
              g[5] = dA * e;
            }
            T = tt;
          }
        }
      }
      const uint64_t who = __ballot(contrib);
      if (who == 0ull) continue;
      if (__popcll(who) <= 4) {  // few lanes: LDS atomics, little contention
        if (contrib) {
#pragma unroll
          for (int c = 0; c < 9; ++c) atomicAdd(&acc[c][j], g[c]);
        }
      } else {  // many lanes: DPP reduction, one LDS atomic per value
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const float r = wave_sum_to_lane63(g[c]);
          if ((threadIdx.x & 63) == 63) atomicAdd(&acc[c][j], r);
        }
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      float* dst = grad2d + 9 * (int64_t)bid[threadIdx.x];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const float r = acc[c][threadIdx.x];
        if (r != 0.0f) {
          atomicAdd(dst + c, r);
          acc[c][threadIdx.x] = 0.0f;
        }
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_zero_grad2d(float* p, const FrameCounters* ctr) {
  const int64_t n = (int64_t)9 * ctr->n_render;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
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

// One thread per drawn splat: the drawn splats lead the depth order, so
// order[0 .. n_drawn) lists exactly them (no lanes idle on culled ones).
__global__ void __launch_bounds__(kBlock) k_project_bwd(SceneDev S, const ViewConst* __restrict__ vp, const int32_t* idx,
                                                        const FrameCounters* ctr, const uint32_t* order,
                                                        const float* grad2d, lodgs_grads sel, lodgs_grads nodes) {
  const ViewConst v = *vp;
  const int64_t n = ctr->n_drawn;
  const int nc = S.n_coef;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = order[r];
    const int64_t node = idx[i];
    double gm[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0;
    Proj64 P;
    const bool visible = proj_chain64(S.means, S.log_scales, S.quats, v, node, P);
    const float* g2 = grad2d + 9 * i;
    float* sel_sh = sel.d_sh ? sel.d_sh + (int64_t)nc * i : nullptr;
    float* node_sh = nodes.d_sh ? nodes.d_sh + (int64_t)nc * node : nullptr;
    if (visible) {
      // colour -> SH coefficients and view direction
      const double mx = S.means[3 * node], my = S.means[3 * node + 1], mz = S.means[3 * node + 2];
      const double dx = mx - (double)v.pos[0], dy = my - (double)v.pos[1], dz = mz - (double)v.pos[2];
      const double dl = __builtin_sqrt(dx * dx + dy * dy + dz * dz);
      const double d0 = dx / dl, d1 = dy / dl, d2 = dz / dl;
      float Y[16], dY[16][3];
      sh_basis(S.sh_degree, (float)d0, (float)d1, (float)d2, Y);
      sh_basis_grad(S.sh_degree, (float)d0, (float)d1, (float)d2, dY);
      const int nb = nc / 3;
      const float* shc = S.sh + (int64_t)nc * node;
      // the forward's FP32 colour decides the clamp at 0
      const float il = 1.0f / __builtin_sqrtf((float)dx * (float)dx + (float)dy * (float)dy + (float)dz * (float)dz);
      float Yf[16];
      sh_basis(S.sh_degree, (float)dx * il, (float)dy * il, (float)dz * il, Yf);
      float raw[3] = {0.5f, 0.5f, 0.5f};
      for (int k = 0; k < nb; ++k)
        for (int c = 0; c < 3; ++c) raw[c] = __builtin_fmaf(shc[3 * k + c], Yf[k], raw[c]);
      double dRGB[3];
      for (int c = 0; c < 3; ++c) dRGB[c] = raw[c] < 0.0f ? 0.0 : (double)g2[6 + c];
      double dd[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < nb; ++k) {
        double a = 0.0;
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
      const double gdir[3] = {(dd[0] - d0 * dot) / dl, (dd[1] - d1 * dot) / dl, (dd[2] - d2 * dot) / dl};
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

void launch_backward(lodgs_frame* f, const float* d_dL, const lodgs_grads* sel, const lodgs_grads* nodes,
                     hipStream_t st) {
  const SceneDev& S = f->scene->dev;
  const ViewConst& v = f->view;
  stage_begin(f, LODGS_STAGE_BLEND_BWD, st);
  hipLaunchKernelGGL(k_zero_grad2d, dim3(2048), dim3(kBlock), 0, st, f->grad2d, f->ctr);
  const int ntiles = v.tiles_x * v.tiles_y;
  hipLaunchKernelGGL(k_blend_bwd, dim3(ntiles), dim3(256), 0, st, f->d_view_ren, f->ranges, f->sorted_ival, f->splats, f->ctr,
                     f->r_rgb, d_dL, f->grad2d);
  stage_end(f, st);
  stage_begin(f, LODGS_STAGE_PROJECT_BWD, st);
  lodgs_grads none{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (sel) hipLaunchKernelGGL(k_zero_sel, dim3(1024), dim3(kBlock), 0, st, f->ctr, S.n_coef, *sel);
  hipLaunchKernelGGL(k_project_bwd, dim3(1024), dim3(kBlock), 0, st, S, f->d_view_ren, f->r_idx, f->ctr,
                     f->sorted_order, f->grad2d, sel ? *sel : none, nodes ? *nodes : none);
  stage_end(f, st);
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
