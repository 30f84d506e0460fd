// Adam step on the cut set (init/training appendix: a view updates only the
// parameters of its cut set).  One thread per (selected node, element) of a
// parameter group: the gradient row is read by selection position
// (coalesced), the parameter and its two moments by node row; d_idx holds
// every node at most once, so no two threads touch one element.
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

struct AdamArgs {
  AdamGroup grp[5];
  int32_t n_groups;
  float b1, b2, eps, bc2_sqrt;  // bc2_sqrt = sqrt(1 - beta2^step)
};

__global__ void __launch_bounds__(kBlock) k_adam_cut(AdamArgs a, const int32_t* idx, const int32_t* d_count,
                                                     int64_t cap, int64_t n_nodes) {
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  for (int gi = 0; gi < a.n_groups; ++gi) {
    const AdamGroup G = a.grp[gi];
    const int64_t total = n * G.w;
    for (int64_t e = t0; e < total; e += stride) {
      const int64_t i = e / G.w;
      const int64_t node = idx[i];
      if (node < 0 || node >= n_nodes) continue;
      const int64_t o = node * G.w + (e - i * G.w);
      const float g = G.g[e];
      const float m = a.b1 * G.m[o] + (1.0f - a.b1) * g;
      const float v = a.b2 * G.v[o] + (1.0f - a.b2) * (g * g);
      G.m[o] = m;
      G.v[o] = v;
      G.p[o] = G.p[o] - G.step_size * m / (__builtin_sqrtf(v) / a.bc2_sqrt + a.eps);
    }
  }
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
  AdamArgs a;
  a.n_groups = 0;
  const double bc1 = 1.0 - std::pow((double)hp->beta1, (double)hp->step);
  const double bc2 = 1.0 - std::pow((double)hp->beta2, (double)hp->step);
  for (int k = 0; k < 5; ++k) {
    float* p = params->*members[k];
    if (!p) continue;
    if (!(grads->*members[k]) || !(exp_avg->*members[k]) || !(exp_avg_sq->*members[k]))
      return set_error(LODGS_E_INVALID, "lodgs_adam_cut: a group has parameters but no gradient or moments");
    AdamGroup& G = a.grp[a.n_groups++];
    G.p = p;
    G.g = grads->*members[k];
    G.m = exp_avg->*members[k];
    G.v = exp_avg_sq->*members[k];
    G.w = widths[k];
    G.step_size = (float)((double)hp->lr[k] / bc1);
  }
  a.b1 = hp->beta1;
  a.b2 = hp->beta2;
  a.eps = hp->eps;
  a.bc2_sqrt = (float)std::sqrt(bc2);
  if (a.n_groups == 0 || capacity == 0) return LODGS_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_adam_cut, dim3(8192), dim3(kBlock), 0, st, a, d_idx, d_count, capacity, n_nodes);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_adam_cut");
}
