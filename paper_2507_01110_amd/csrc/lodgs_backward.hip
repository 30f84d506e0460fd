// Backward of the render (recompute-based): per tile, the forward
// front-to-back pass is replayed with identical FP32 decisions and the
// gradient of every contributing (splat, pixel) pair is formed on the fly,
// using the final pixel colour to obtain the colour behind each splat
// (S_i = C_final - C_prefix_i - c_i alpha_i T_i).  Per-splat sums over the
// pixels of a wave are reduced with lane shuffles and added with one atomic
// per wave and value.  Then one thread per rendered node carries the 2D
// gradients through the conic inverse, the EWA Jacobian, the camera
// transform, the covariance factorisation, the quaternion normalisation, the
// sigmoid and the SH basis to the raw parameters.
#include "lodgs_internal.h"

namespace lodgs {

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__global__ void __launch_bounds__(256) k_blend_bwd(ViewConst v, const uint2* ranges, const uint32_t* ival,
                                                   const Splat* splats, const FrameCounters* ctr, const float* rgb,
                                                   const float* dL, float* grad2d) {
  __shared__ Splat batch[256];
  __shared__ uint32_t bid[256];
  const int tile = blockIdx.x;
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < v.width && py < v.height;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
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
      }
    }
    __syncthreads();
    const int m = (int)min(256u, rg.y - b0);
    for (int j = 0; j < m; ++j) {
      if (__all(done)) break;  // wave-uniform
      const Splat& s = batch[j];
      float g[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      bool contrib = false;
      if (!done) {
        const float dx = fx - s.mx, dy = fy - s.my;
        float t1 = s.na * dx;
        t1 = __builtin_fmaf(s.nb, dy, t1);
        float u = s.nc * dy;
        u = u * dy;
        const float power = __builtin_fmaf(t1, dx, u);
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
            const float ia = 1.0f / (1.0f - alpha);
            float dA = G[0] * (s.r * T - (Cf[0] - P0) * ia);
            dA = __builtin_fmaf(G[1], s.g * T - (Cf[1] - P1) * ia, dA);
            dA = __builtin_fmaf(G[2], s.b * T - (Cf[2] - P2) * ia, dA);
            if (oe <= 0.99f) {
              const float dpow = dA * alpha;
              g[5] = dA * e;
              // conic (a, b, c) = (-2 na, -nb, -2 nc)
              g[0] = dpow * (-2.0f * s.na * dx - s.nb * dy);
              g[1] = dpow * (-s.nb * dx - 2.0f * s.nc * dy);
              g[2] = dpow * (-0.5f * dx * dx);
              g[3] = dpow * (-dx * dy);
              g[4] = dpow * (-0.5f * dy * dy);
            }
            T = tt;
          }
        }
      }
      if (__ballot(contrib) == 0ull) continue;
      float* dst = grad2d + 9 * (int64_t)bid[j];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const float r = wave_sum(g[c]);
        if ((threadIdx.x & 63) == 0 && r != 0.0f) atomicAdd(dst + c, r);
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_zero_f32(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

__global__ void __launch_bounds__(kBlock) k_project_bwd(SceneDev S, ViewConst v, const int32_t* idx,
                                                        const FrameCounters* ctr, const float* grad2d,
                                                        lodgs_grads sel, lodgs_grads nodes) {
  const int64_t n = ctr->n_render;
  const int nc = S.n_coef;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = idx[i];
    float gm[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0f;
    float gsh[48];
    for (int k = 0; k < nc; ++k) gsh[k] = 0.0f;
    // Replay the forward FP32 projection (decisions and values).
    const float mx = S.means[3 * node], my = S.means[3 * node + 1], mz = S.means[3 * node + 2];
    float cx, cy, cz;
    to_camera(v, mx, my, mz, cx, cy, cz);
    bool visible = false;
    float s[3], qn[4], ql = 1.0f, Rq[9], M[9], Sg[6], Tm[6], Ac = 0, Bc = 0, Cc = 0, det = 1.0f;
    if (cz > v.z_near) {
      for (int k = 0; k < 3; ++k) s[k] = fexp(S.log_scales[3 * node + k]);
      const float4 q = *reinterpret_cast<const float4*>(S.quats + 4 * node);
      float qq = q.x * q.x;
      qq = qq + q.y * q.y;
      qq = qq + q.z * q.z;
      qq = qq + q.w * q.w;
      ql = __builtin_sqrtf(qq);
      qn[0] = q.x / ql; qn[1] = q.y / ql; qn[2] = q.z / ql; qn[3] = q.w / ql;
      const float w = qn[0], x = qn[1], y = qn[2], z = qn[3];
      const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
      const float wx = w * x, wy = w * y, wz = w * z;
      Rq[0] = 1.0f - 2.0f * (yy + zz); Rq[1] = 2.0f * (xy - wz); Rq[2] = 2.0f * (xz + wy);
      Rq[3] = 2.0f * (xy + wz); Rq[4] = 1.0f - 2.0f * (xx + zz); Rq[5] = 2.0f * (yz - wx);
      Rq[6] = 2.0f * (xz - wy); Rq[7] = 2.0f * (yz + wx); Rq[8] = 1.0f - 2.0f * (xx + yy);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * s[c];
      Sg[0] = (M[0] * M[0] + M[1] * M[1]) + M[2] * M[2];
      Sg[1] = (M[0] * M[3] + M[1] * M[4]) + M[2] * M[5];
      Sg[2] = (M[0] * M[6] + M[1] * M[7]) + M[2] * M[8];
      Sg[3] = (M[3] * M[3] + M[4] * M[4]) + M[5] * M[5];
      Sg[4] = (M[3] * M[6] + M[4] * M[7]) + M[5] * M[8];
      Sg[5] = (M[6] * M[6] + M[7] * M[7]) + M[8] * M[8];
      const float u = cx / cz, vv = cy / cz;
      const float jx = v.fx / cz, jy = v.fy / cz;
      const float jxz = -(jx * u), jyz = -(jy * vv);
      const float* W = v.R;
      Tm[0] = jx * W[0] + jxz * W[6]; Tm[1] = jx * W[1] + jxz * W[7]; Tm[2] = jx * W[2] + jxz * W[8];
      Tm[3] = jy * W[3] + jyz * W[6]; Tm[4] = jy * W[4] + jyz * W[7]; Tm[5] = jy * W[5] + jyz * W[8];
      const float U00 = (Tm[0] * Sg[0] + Tm[1] * Sg[1]) + Tm[2] * Sg[2];
      const float U01 = (Tm[0] * Sg[1] + Tm[1] * Sg[3]) + Tm[2] * Sg[4];
      const float U02 = (Tm[0] * Sg[2] + Tm[1] * Sg[4]) + Tm[2] * Sg[5];
      const float U10 = (Tm[3] * Sg[0] + Tm[4] * Sg[1]) + Tm[5] * Sg[2];
      const float U11 = (Tm[3] * Sg[1] + Tm[4] * Sg[3]) + Tm[5] * Sg[4];
      const float U12 = (Tm[3] * Sg[2] + Tm[4] * Sg[4]) + Tm[5] * Sg[5];
      Ac = ((U00 * Tm[0] + U01 * Tm[1]) + U02 * Tm[2]) + 0.3f;
      Bc = (U00 * Tm[3] + U01 * Tm[4]) + U02 * Tm[5];
      Cc = ((U10 * Tm[3] + U11 * Tm[4]) + U12 * Tm[5]) + 0.3f;
      det = Ac * Cc - Bc * Bc;
      visible = det > 0.0f;
    }
    const float* g2 = grad2d + 9 * i;
    if (visible) {
      // colour -> SH coefficients and view direction
      const float dx = mx - v.pos[0], dy = my - v.pos[1], dz = mz - v.pos[2];
      const float dl = __builtin_sqrtf(dx * dx + dy * dy + dz * dz);
      const float d0 = dx / dl, d1 = dy / dl, d2 = dz / dl;
      float Y[16], dY[16][3];
      sh_basis(S.sh_degree, d0, d1, d2, Y);
      sh_basis_grad(S.sh_degree, d0, d1, d2, dY);
      const int nb = nc / 3;
      const float* shc = S.sh + (int64_t)nc * node;
      float raw[3] = {0.5f, 0.5f, 0.5f};
      for (int k = 0; k < nb; ++k)
        for (int c = 0; c < 3; ++c) raw[c] = __builtin_fmaf(shc[3 * k + c], Y[k], raw[c]);
      float dRGB[3];
      for (int c = 0; c < 3; ++c) dRGB[c] = raw[c] < 0.0f ? 0.0f : g2[6 + c];
      float dd[3] = {0.0f, 0.0f, 0.0f};
      for (int k = 0; k < nb; ++k) {
        float a = 0.0f;
        for (int c = 0; c < 3; ++c) {
          gsh[3 * k + c] = dRGB[c] * Y[k];
          a = __builtin_fmaf(dRGB[c], shc[3 * k + c], a);
        }
        dd[0] = __builtin_fmaf(a, dY[k][0], dd[0]);
        dd[1] = __builtin_fmaf(a, dY[k][1], dd[1]);
        dd[2] = __builtin_fmaf(a, dY[k][2], dd[2]);
      }
      const float dot = dd[0] * d0 + dd[1] * d1 + dd[2] * d2;
      const float gdir[3] = {(dd[0] - d0 * dot) / dl, (dd[1] - d1 * dot) / dl, (dd[2] - d2 * dot) / dl};
      // opacity
      const float o = 1.0f / (1.0f + fexp(-S.opacity_logits[node]));
      go = g2[5] * o * (1.0f - o);
      // conic -> projected covariance: GS = -Q GQ Q
      const float ca = Cc / det, cb = -Bc / det, cc = Ac / det;
      const float gq00 = g2[2], gq01 = 0.5f * g2[3], gq11 = g2[4];
      const float qg00 = ca * gq00 + cb * gq01, qg01 = ca * gq01 + cb * gq11;
      const float qg10 = cb * gq00 + cc * gq01, qg11 = cb * gq01 + cc * gq11;
      const float GS00 = -(qg00 * ca + qg01 * cb), GS01 = -(qg00 * cb + qg01 * cc);
      const float GS11 = -(qg10 * cb + qg11 * cc);
      // Sigma' = T Sigma T^T
      float TS[6];
      for (int r = 0; r < 2; ++r) {
        TS[3 * r + 0] = Tm[3 * r] * Sg[0] + Tm[3 * r + 1] * Sg[1] + Tm[3 * r + 2] * Sg[2];
        TS[3 * r + 1] = Tm[3 * r] * Sg[1] + Tm[3 * r + 1] * Sg[3] + Tm[3 * r + 2] * Sg[4];
        TS[3 * r + 2] = Tm[3 * r] * Sg[2] + Tm[3 * r + 1] * Sg[4] + Tm[3 * r + 2] * Sg[5];
      }
      float dT[6];
      for (int c = 0; c < 3; ++c) {
        dT[c] = 2.0f * (GS00 * TS[c] + GS01 * TS[3 + c]);
        dT[3 + c] = 2.0f * (GS01 * TS[c] + GS11 * TS[3 + c]);
      }
      float dS[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          dS[3 * a + b] = Tm[a] * (GS00 * Tm[b] + GS01 * Tm[3 + b]) + Tm[3 + a] * (GS01 * Tm[b] + GS11 * Tm[3 + b]);
      // T = J W
      const float* W = v.R;
      float dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
      for (int c = 0; c < 3; ++c) {
        dJ00 += dT[c] * W[c];
        dJ02 += dT[c] * W[6 + c];
        dJ11 += dT[3 + c] * W[3 + c];
        dJ12 += dT[3 + c] * W[6 + c];
      }
      const float iz = 1.0f / cz, iz2 = iz * iz, iz3 = iz2 * iz;
      const float dcx = dJ02 * (-v.fx * iz2) + g2[0] * v.fx * iz;
      const float dcy = dJ12 * (-v.fy * iz2) + g2[1] * v.fy * iz;
      const float dcz = dJ00 * (-v.fx * iz2) + dJ02 * (2.0f * v.fx * cx * iz3) + dJ11 * (-v.fy * iz2) +
                        dJ12 * (2.0f * v.fy * cy * iz3) + g2[0] * (-v.fx * cx * iz2) + g2[1] * (-v.fy * cy * iz2);
      for (int a = 0; a < 3; ++a) gm[a] = W[a] * dcx + W[3 + a] * dcy + W[6 + a] * dcz + gdir[a];
      // Sigma = M M^T, M = Rq diag(s)
      float dRq[9];
      for (int c = 0; c < 3; ++c) {
        float ds = 0.0f;
        for (int r = 0; r < 3; ++r) {
          const float dm = 2.0f * (dS[3 * r] * M[c] + dS[3 * r + 1] * M[3 + c] + dS[3 * r + 2] * M[6 + c]);
          ds += dm * Rq[3 * r + c];
          dRq[3 * r + c] = dm * s[c];
        }
        gls[c] = ds * s[c];
      }
      const float w = qn[0], x = qn[1], y = qn[2], z = qn[3];
      float dq[4];
      dq[0] = 2.0f * (-z * dRq[1] + y * dRq[2] + z * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
      dq[1] = 2.0f * (y * dRq[1] + z * dRq[2] + y * dRq[3] - 2.0f * x * dRq[4] - w * dRq[5] + z * dRq[6] +
                      w * dRq[7] - 2.0f * x * dRq[8]);
      dq[2] = 2.0f * (-2.0f * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + z * dRq[5] - w * dRq[6] +
                      z * dRq[7] - 2.0f * y * dRq[8]);
      dq[3] = 2.0f * (-2.0f * z * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - 2.0f * z * dRq[4] +
                      y * dRq[5] + x * dRq[6] + y * dRq[7]);
      const float qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
      for (int k = 0; k < 4; ++k) gq[k] = (dq[k] - qn[k] * qd) / ql;
    }
    if (sel.d_means) for (int k = 0; k < 3; ++k) sel.d_means[3 * i + k] = gm[k];
    if (sel.d_log_scales) for (int k = 0; k < 3; ++k) sel.d_log_scales[3 * i + k] = gls[k];
    if (sel.d_quats) for (int k = 0; k < 4; ++k) sel.d_quats[4 * i + k] = gq[k];
    if (sel.d_opacity_logits) sel.d_opacity_logits[i] = go;
    if (sel.d_sh) for (int k = 0; k < nc; ++k) sel.d_sh[(int64_t)nc * i + k] = gsh[k];
    if (!visible) continue;
    if (nodes.d_means) for (int k = 0; k < 3; ++k) nodes.d_means[3 * node + k] += gm[k];
    if (nodes.d_log_scales) for (int k = 0; k < 3; ++k) nodes.d_log_scales[3 * node + k] += gls[k];
    if (nodes.d_quats) for (int k = 0; k < 4; ++k) nodes.d_quats[4 * node + k] += gq[k];
    if (nodes.d_opacity_logits) nodes.d_opacity_logits[node] += go;
    if (nodes.d_sh) for (int k = 0; k < nc; ++k) nodes.d_sh[(int64_t)nc * node + k] += gsh[k];
  }
}

void launch_backward(lodgs_frame* f, const float* d_dL, const lodgs_grads* sel, const lodgs_grads* nodes,
                     hipStream_t st) {
  const SceneDev& S = f->scene->dev;
  const ViewConst& v = f->view;
  hipLaunchKernelGGL(k_zero_f32, dim3(2048), dim3(kBlock), 0, st, f->grad2d, (int64_t)9 * f->caps.max_selected);
  const int ntiles = v.tiles_x * v.tiles_y;
  hipLaunchKernelGGL(k_blend_bwd, dim3(ntiles), dim3(256), 0, st, v, f->ranges, f->sorted_ival, f->splats, f->ctr,
                     f->r_rgb, d_dL, f->grad2d);
  lodgs_grads none{nullptr, nullptr, nullptr, nullptr, nullptr};
  hipLaunchKernelGGL(k_project_bwd, dim3(2048), dim3(kBlock), 0, st, S, v, f->r_idx, f->ctr, f->grad2d,
                     sel ? *sel : none, nodes ? *nodes : none);
}

}  // namespace lodgs
