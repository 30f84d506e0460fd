// Out-of-core parameters (Sec. 4.4: the Gaussians of a cut are loaded from
// RAM): one kernel gathers the selected nodes' parameter rows from pinned
// host memory, read by the GPU over the host link, into device row arrays,
// row k for the k-th selected node.  One thread per (row, chunk) of a group:
// chunks are float4s for rows of 4, 12 or 48 floats and single floats
// otherwise, so consecutive threads read consecutive bytes of a row.
#include "lodgs_internal.h"

namespace lodgs {
namespace {

struct GatherGroup {
  const float* src;  // device-visible address of the host array
  float* dst;
  int32_t w;
};

template <int W>
__global__ void __launch_bounds__(kBlock) k_gather_rows(GatherGroup G, const int32_t* idx, const int32_t* d_count,
                                                        int64_t cap, int64_t n_nodes) {
  constexpr int V = W % 4 == 0 ? 4 : 1, C = W / V;
  int64_t n = *d_count;
  n = n < 0 ? 0 : (n > cap ? cap : n);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * C; e += stride) {
    const int64_t k = e / C;
    const int c = (int)(e - k * C);
    const int64_t node = idx[k];
    if (node < 0 || node >= n_nodes) continue;
    if (V == 4)
      reinterpret_cast<float4*>(G.dst + k * W)[c] = reinterpret_cast<const float4*>(G.src + node * W)[c];
    else
      G.dst[k * W + c] = G.src[node * W + c];
  }
}

template <int W>
void launch_gather(const GatherGroup& G, const int32_t* idx, const int32_t* d_count, int64_t cap, int64_t n_nodes,
                   hipStream_t st) {
  constexpr int C = W % 4 == 0 ? W / 4 : W;
  int64_t blocks = (cap * C + kBlock - 1) / kBlock;
  blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
  hipLaunchKernelGGL(k_gather_rows<W>, dim3((unsigned)blocks), dim3(kBlock), 0, st, G, idx, d_count, cap, n_nodes);
}

// The device-visible address of pinned host memory, or nullptr.
const float* host_device_address(const float* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
  return static_cast<const float*>(a.devicePointer);
}

bool is_device_memory(const float* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

}  // namespace
}  // namespace lodgs

extern "C" int lodgs_gather_rows(const lodgs_grads* host, const lodgs_grads* rows, int32_t sh_degree,
                                 const int32_t* d_idx, const int32_t* d_count, int64_t capacity, int64_t n_nodes,
                                 lodgs_stream stream) {
  using namespace lodgs;
  if (!host || !rows || !d_idx || !d_count) return set_error(LODGS_E_INVALID, "lodgs_gather_rows: null argument");
  if (sh_degree < 0 || sh_degree > 3 || capacity < 0 || n_nodes < 0)
    return set_error(LODGS_E_INVALID, "lodgs_gather_rows: sh_degree 0..3, capacity and n_nodes >= 0");
  float* const lodgs_grads::*members[5] = {&lodgs_grads::d_means, &lodgs_grads::d_log_scales, &lodgs_grads::d_quats,
                                          &lodgs_grads::d_opacity_logits, &lodgs_grads::d_sh};
  const int32_t widths[5] = {3, 3, 4, 1, 3 * (sh_degree + 1) * (sh_degree + 1)};
  GatherGroup grp[5];
  for (int g = 0; g < 5; ++g) {
    const float* src = host->*members[g];
    float* dst = rows->*members[g];
    if (!src || !dst) return set_error(LODGS_E_INVALID, "lodgs_gather_rows: every parameter group is needed");
    const float* dsrc = host_device_address(src);
    if (!dsrc) return set_error(LODGS_E_INVALID, "lodgs_gather_rows: a host array is not pinned host memory");
    if (!is_device_memory(dst)) return set_error(LODGS_E_INVALID, "lodgs_gather_rows: a rows array is not device memory");
    if (widths[g] % 4 == 0 && ((reinterpret_cast<uintptr_t>(dsrc) | reinterpret_cast<uintptr_t>(dst)) & 15u))
      return set_error(LODGS_E_INVALID, "lodgs_gather_rows: quaternion and SH arrays must be 16-byte aligned");
    grp[g] = GatherGroup{dsrc, dst, widths[g]};
  }
  if (capacity == 0) return LODGS_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  launch_gather<3>(grp[0], d_idx, d_count, capacity, n_nodes, st);
  launch_gather<3>(grp[1], d_idx, d_count, capacity, n_nodes, st);
  launch_gather<4>(grp[2], d_idx, d_count, capacity, n_nodes, st);
  launch_gather<1>(grp[3], d_idx, d_count, capacity, n_nodes, st);
  switch (grp[4].w) {
    case 3: launch_gather<3>(grp[4], d_idx, d_count, capacity, n_nodes, st); break;
    case 12: launch_gather<12>(grp[4], d_idx, d_count, capacity, n_nodes, st); break;
    case 27: launch_gather<27>(grp[4], d_idx, d_count, capacity, n_nodes, st); break;
    default: launch_gather<48>(grp[4], d_idx, d_count, capacity, n_nodes, st); break;
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_gather_rows");
}
