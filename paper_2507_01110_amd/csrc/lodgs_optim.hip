// Adam step on the cut set (init/training appendix: a view updates only the
// parameters of its cut set).  One launch per parameter group, one thread per
// (selected node, chunk) with chunks of 4 floats for rows of a multiple of 4
// floats (quaternions, SH of degree 1 and 3) and of 1 float otherwise: the
// gradient rows are read by selection position (coalesced), the parameter
// and its two moments by node row; d_idx holds every node at most once, so
// no two threads touch one element.
#include "lodgs_internal.h"

#include <cmath>

namespace lodgs {
namespace {

struct AdamGroup {
  float* p;
  const float* g;
  float* m;
  float* v;
  int32_t w;
  float step_size;  // lr / (1 - beta1^step)
};

struct AdamConst {
  float b1, b2, eps, bc2_sqrt;  // bc2_sqrt = sqrt(1 - beta2^step)
};

__device__ __forceinline__ void adam_element(const AdamConst& a, float step_size, float g, float& p, float& m,
                                             float& v) {
  m = a.b1 * m + (1.0f - a.b1) * g;
  v = a.b2 * v + (1.0f - a.b2) * (g * g);
  p = p - step_size * m / (__builtin_sqrtf(v) / a.bc2_sqrt + a.eps);
}

template <int W>
__global__ void __launch_bounds__(kBlock) k_adam_cut(AdamGroup G, AdamConst a, const int32_t* idx,
                                                     const int32_t* d_count, int64_t cap, int64_t n_nodes) {
  constexpr int V = W % 4 == 0 ? 4 : 1, C = W / V;
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = t0; e < n * C; e += stride) {
    const int64_t i = e / C;
    const int c = (int)(e - i * C);
    const int64_t node = idx[i];
    if (node < 0 || node >= n_nodes) continue;
    if (V == 4) {
      const float4 g = reinterpret_cast<const float4*>(G.g + i * W)[c];
      float4* pp = reinterpret_cast<float4*>(G.p + node * W) + c;
      float4* mp = reinterpret_cast<float4*>(G.m + node * W) + c;
      float4* vp = reinterpret_cast<float4*>(G.v + node * W) + c;
      float4 p = *pp, m = *mp, v = *vp;
      adam_element(a, G.step_size, g.x, p.x, m.x, v.x);
      adam_element(a, G.step_size, g.y, p.y, m.y, v.y);
      adam_element(a, G.step_size, g.z, p.z, m.z, v.z);
      adam_element(a, G.step_size, g.w, p.w, m.w, v.w);
      *mp = m;
      *vp = v;
      *pp = p;
    } else {
      const int64_t o = node * W + c;
      float p = G.p[o], m = G.m[o], v = G.v[o];
      adam_element(a, G.step_size, G.g[i * W + c], p, m, v);
      G.m[o] = m;
      G.v[o] = v;
      G.p[o] = p;
    }
  }
}

template <int W>
void launch_adam(const AdamGroup& G, const AdamConst& a, const int32_t* idx, const int32_t* d_count, int64_t cap,
                 int64_t n_nodes, hipStream_t st) {
  constexpr int C = W % 4 == 0 ? W / 4 : W;
  int64_t blocks = (cap * C + kBlock - 1) / kBlock;
  blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
  hipLaunchKernelGGL(k_adam_cut<W>, dim3((unsigned)blocks), dim3(kBlock), 0, st, G, a, idx, d_count, cap, n_nodes);
}

}  // namespace
}  // namespace lodgs

extern "C" int lodgs_adam_cut(const lodgs_grads* params, const lodgs_grads* grads, const lodgs_grads* exp_avg,
                              const lodgs_grads* exp_avg_sq, const lodgs_adam* hp, const int32_t* d_idx,
                              const int32_t* d_count, int64_t capacity, int64_t n_nodes, lodgs_stream stream) {
  using namespace lodgs;
  if (!params || !grads || !exp_avg || !exp_avg_sq || !hp || !d_idx || !d_count)
    return set_error(LODGS_E_INVALID, "lodgs_adam_cut: null argument");
  if (hp->step < 1 || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) || !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) ||
      !(hp->eps >= 0.0f) || hp->sh_degree < 0 || hp->sh_degree > 3 || capacity < 0 || n_nodes < 0)
    return set_error(LODGS_E_INVALID, "lodgs_adam_cut: hyper-parameters out of range");
  float* const lodgs_grads::*members[5] = {&lodgs_grads::d_means, &lodgs_grads::d_log_scales, &lodgs_grads::d_quats,
                                          &lodgs_grads::d_opacity_logits, &lodgs_grads::d_sh};
  const int32_t widths[5] = {3, 3, 4, 1, 3 * (hp->sh_degree + 1) * (hp->sh_degree + 1)};
  const double bc1 = 1.0 - std::pow((double)hp->beta1, (double)hp->step);
  const double bc2 = 1.0 - std::pow((double)hp->beta2, (double)hp->step);
  AdamGroup grp[5];
  int n_groups = 0;
  for (int k = 0; k < 5; ++k) {
    float* p = params->*members[k];
    if (!p) continue;
    const float* g = grads->*members[k];
    float* m = exp_avg->*members[k];
    float* v = exp_avg_sq->*members[k];
    if (!g || !m || !v)
      return set_error(LODGS_E_INVALID, "lodgs_adam_cut: a group has parameters but no gradient or moments");
    if (widths[k] % 4 == 0 && ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(g) |
                                reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15u))
      return set_error(LODGS_E_INVALID, "lodgs_adam_cut: quaternion and SH arrays must be 16-byte aligned");
    grp[n_groups++] = AdamGroup{p, g, m, v, widths[k], (float)((double)hp->lr[k] / bc1)};
  }
  const AdamConst a{hp->beta1, hp->beta2, hp->eps, (float)std::sqrt(bc2)};
  if (n_groups == 0 || capacity == 0) return LODGS_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int k = 0; k < n_groups; ++k) {
    const AdamGroup& G = grp[k];
    switch (G.w) {
      case 1: launch_adam<1>(G, a, d_idx, d_count, capacity, n_nodes, st); break;
      case 3: launch_adam<3>(G, a, d_idx, d_count, capacity, n_nodes, st); break;
      case 4: launch_adam<4>(G, a, d_idx, d_count, capacity, n_nodes, st); break;
      case 12: launch_adam<12>(G, a, d_idx, d_count, capacity, n_nodes, st); break;
      case 27: launch_adam<27>(G, a, d_idx, d_count, capacity, n_nodes, st); break;
      default: launch_adam<48>(G, a, d_idx, d_count, capacity, n_nodes, st); break;
    }
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_adam_cut");
}
