// Per-splat EWA projection chain in FP64 (Sec. 3), shared by the forward
// projection (which takes the path's per-splat decisions from it) and the
// projection backward (which replays it).  Fixed operation order; scales from
// the FP32 exp, quaternion (w, x, y, z) normalised in FP64.
#pragma once

#include "lodgs_dev.h"

namespace lodgs {

struct Proj64 {
  double c[3];           // camera-space mean
  double s[3];           // scales
  double qn[4], ql;      // normalised quaternion and the raw quaternion's length
  double Rq[9], M[9];    // rotation, M = Rq diag(s)
  double Sg[6];          // Sigma = M M^T (00, 01, 02, 11, 12, 22)
  double T[6];           // J W (2 x 3)
  double A, B, C, det;   // projected covariance + 0.3 I and its determinant
  double u, v;           // c.x / c.z, c.y / c.z
};

// Camera-space position: ((R[r0] m0 + R[r1] m1) + R[r2] m2) + t[r].
__device__ __forceinline__ void to_camera64(const ViewConst& v, double m0, double m1, double m2, double* c) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    c[r] = (((double)v.R[3 * r] * m0 + (double)v.R[3 * r + 1] * m1) + (double)v.R[3 * r + 2] * m2) + (double)v.t[r];
}

// The raw parameters of one node, loaded together (independent loads).
struct NodeGeom {
  float m[3], ls[3];
  float4 q;
};

__device__ __forceinline__ NodeGeom load_geom(const float* means, const float* log_scales, const float* quats,
                                              int64_t n) {
  NodeGeom g;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g.m[k] = means[3 * n + k];
    g.ls[k] = log_scales[3 * n + k];
  }
  g.q = *reinterpret_cast<const float4*>(quats + 4 * n);
  return g;
}

// Returns false when the splat is not drawn (depth <= z_near or a
// non-positive determinant); P is then only partly filled.
__device__ __forceinline__ bool proj_chain64(const NodeGeom& g, const ViewConst& v, Proj64& P) {
  to_camera64(v, g.m[0], g.m[1], g.m[2], P.c);
  if (!(P.c[2] > (double)v.z_near)) return false;
#pragma unroll
  for (int k = 0; k < 3; ++k) P.s[k] = fexp(g.ls[k]);
  const float4 qf = g.q;
  const double q0 = qf.x, q1 = qf.y, q2 = qf.z, q3 = qf.w;
  const double qq = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
  P.ql = __builtin_sqrt(qq);
  const double w = q0 / P.ql, x = q1 / P.ql, y = q2 / P.ql, z = q3 / P.ql;
  P.qn[0] = w; P.qn[1] = x; P.qn[2] = y; P.qn[3] = z;
  const double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const double wx = w * x, wy = w * y, wz = w * z;
  double* R = P.Rq;
  R[0] = 1.0 - 2.0 * (yy + zz); R[1] = 2.0 * (xy - wz); R[2] = 2.0 * (xz + wy);
  R[3] = 2.0 * (xy + wz); R[4] = 1.0 - 2.0 * (xx + zz); R[5] = 2.0 * (yz - wx);
  R[6] = 2.0 * (xz - wy); R[7] = 2.0 * (yz + wx); R[8] = 1.0 - 2.0 * (xx + yy);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) P.M[3 * r + k] = R[3 * r + k] * P.s[k];
  const double* M = P.M;
  P.Sg[0] = (M[0] * M[0] + M[1] * M[1]) + M[2] * M[2];
  P.Sg[1] = (M[0] * M[3] + M[1] * M[4]) + M[2] * M[5];
  P.Sg[2] = (M[0] * M[6] + M[1] * M[7]) + M[2] * M[8];
  P.Sg[3] = (M[3] * M[3] + M[4] * M[4]) + M[5] * M[5];
  P.Sg[4] = (M[3] * M[6] + M[4] * M[7]) + M[5] * M[8];
  P.Sg[5] = (M[6] * M[6] + M[7] * M[7]) + M[8] * M[8];
  const double fx = v.fx, fy = v.fy;
  P.u = P.c[0] / P.c[2];
  P.v = P.c[1] / P.c[2];
  const double jx = fx / P.c[2], jy = fy / P.c[2];
  const double jxz = -(jx * P.u), jyz = -(jy * P.v);
  const double W0 = v.R[0], W1 = v.R[1], W2 = v.R[2], W3 = v.R[3], W4 = v.R[4], W5 = v.R[5];
  const double W6 = v.R[6], W7 = v.R[7], W8 = v.R[8];
  double* T = P.T;
  T[0] = jx * W0 + jxz * W6; T[1] = jx * W1 + jxz * W7; T[2] = jx * W2 + jxz * W8;
  T[3] = jy * W3 + jyz * W6; T[4] = jy * W4 + jyz * W7; T[5] = jy * W5 + jyz * W8;
  const double* S = P.Sg;
  const double U00 = (T[0] * S[0] + T[1] * S[1]) + T[2] * S[2];
  const double U01 = (T[0] * S[1] + T[1] * S[3]) + T[2] * S[4];
  const double U02 = (T[0] * S[2] + T[1] * S[4]) + T[2] * S[5];
  const double U10 = (T[3] * S[0] + T[4] * S[1]) + T[5] * S[2];
  const double U11 = (T[3] * S[1] + T[4] * S[3]) + T[5] * S[4];
  const double U12 = (T[3] * S[2] + T[4] * S[4]) + T[5] * S[5];
  P.A = ((U00 * T[0] + U01 * T[1]) + U02 * T[2]) + 0.3;
  P.B = (U00 * T[3] + U01 * T[4]) + U02 * T[5];
  P.C = ((U10 * T[3] + U11 * T[4]) + U12 * T[5]) + 0.3;
  P.det = P.A * P.C - P.B * P.B;
  return P.det > 0.0;
}

__device__ __forceinline__ bool proj_chain64(const float* means, const float* log_scales, const float* quats,
                                             const ViewConst& v, int64_t n, Proj64& P) {
  return proj_chain64(load_geom(means, log_scales, quats, n), v, P);
}

}  // namespace lodgs
