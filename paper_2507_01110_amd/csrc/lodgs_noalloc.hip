// lodgs_lod_select_noalloc: the HSPT cut of lodgs_lod_select for callers that
// cannot allocate device memory.  The select stage's workspace (counters,
// view constants, scan block sums, per-upper-node and per-SPT arrays, the
// compaction segments) lives in one file-scope device array instead of a
// frame; the kernels are those of lodgs_lod_select.
//
// A __device__ array's name in host code is only a host-side handle, so the
// array's device address is looked up once per device with
// hipGetSymbolAddress and that address is what the kernels receive.  Every
// call on one device shares the array: calls that overlap on a device race,
// and each call clears the counters it reads before the cut runs.
#include <cmath>
#include <mutex>

#include "lodgs_internal.h"

namespace {

constexpr size_t kScratchBytes = LODGS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
  std::once_flag once;
  hipError_t err = hipSuccess;
  unsigned char* ptr = nullptr;
};
DeviceScratch g_dev[kMaxDevices];

// Device address of this device's copy of the array (looked up on the first
// call made with the device current).
hipError_t scratch_address(int dev, unsigned char** out) {
  DeviceScratch& d = g_dev[dev];
  std::call_once(d.once, [&d] {
    void* p = nullptr;
    d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    d.ptr = static_cast<unsigned char*>(p);
  });
  *out = d.ptr;
  return d.err;
}

// Carves the select workspace out of a base address; with base == nullptr it
// only measures (returns the bytes needed).
struct Carve {
  unsigned char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count > 0 ? count : 1);
    return p;
  }
};

size_t layout(const SceneDev& S, unsigned char* base, lodgs_frame* f) {
  Carve c{base};
  lodgs_frame tmp{};
  lodgs_frame& g = f ? *f : tmp;
  g.ctr = c.take<FrameCounters>(1);
  g.d_view_sel = c.take<lodgs::ViewConst>(1);
  g.block_sums = c.take<uint32_t>(lodgs::kScanGrid + 1);
  g.upper_sel = c.take<uint8_t>((size_t)S.n_upper);
  g.upper_test = c.take<uint8_t>((size_t)S.n_upper);
  g.spt_high = c.take<int32_t>((size_t)S.n_spt);
  g.spt_X = c.take<float>((size_t)S.n_spt);
  g.spt_off = c.take<uint32_t>((size_t)S.n_spt);
  // the same lengths lodgs_frame_create gives these two
  g.seg = c.take<uint32_t>((size_t)(S.n_upper + 63) / 64 + (size_t)S.n_spt + (size_t)S.n_nodes / 512 + 1);
  g.chunk_owner = c.take<uint32_t>((size_t)S.n_spt + (size_t)S.n_nodes / 512 + 1);
  return c.off;
}

// Every counter the cut reads starts from a known value (a kernel, not a
// memset, so the call can sit in a captured graph).
__global__ void k_noalloc_counters(FrameCounters* c, int32_t n_spt) {
  FrameCounters z{};
  z.status = LODGS_OK;
  z.spt_count = n_spt;
  *c = z;
}

}  // namespace

extern "C" int lodgs_lod_select_noalloc(const lodgs_scene* scene, const lodgs_camera* cam, float tau, uint32_t flags,
                                        int32_t* d_idx, int64_t capacity, int32_t* d_count, lodgs_stream stream) {
  if (!scene || !d_idx || !d_count) return lodgs::set_error(LODGS_E_INVALID, "lodgs_lod_select_noalloc: null argument");
  if (!lodgs::camera_ok(cam)) return lodgs::set_error(LODGS_E_INVALID, "lodgs_lod_select_noalloc: bad camera");
  if (!std::isfinite(tau) || tau < 0.0f)
    return lodgs::set_error(LODGS_E_INVALID, "lodgs_lod_select_noalloc: tau must be finite, >= 0");
  if (capacity < 0 || capacity > (int64_t)INT32_MAX)
    return lodgs::set_error(LODGS_E_INVALID, "lodgs_lod_select_noalloc: capacity");
  if (flags & ~(LODGS_CULL | LODGS_CONSERVATIVE))
    return lodgs::set_error(LODGS_E_INVALID, "lodgs_lod_select_noalloc: only LODGS_CULL and LODGS_CONSERVATIVE");
  const size_t need = layout(scene->dev, nullptr, nullptr);
  if (need > kScratchBytes)
    return lodgs::set_error(LODGS_E_CAPACITY,
                            "lodgs_lod_select_noalloc: the scene's select workspace exceeds the static scratch "
                            "(LODGS_NOALLOC_SCRATCH_BYTES)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lodgs::hip_fail(e, "lodgs_lod_select_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return lodgs::set_error(LODGS_E_INVALID, "lodgs_lod_select_noalloc: device id");
  unsigned char* base = nullptr;
  e = scratch_address(dev, &base);
  if (e != hipSuccess || !base) return lodgs::hip_fail(e, "lodgs_lod_select_noalloc: hipGetSymbolAddress(scratch)");
  lodgs_frame f{};  // host-side view of the workspace: no allocation, timing off
  f.scene = scene;
  f.timing = false;
  f.open_event = nullptr;
  layout(scene->dev, base, &f);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_noalloc_counters, dim3(1), dim3(1), 0, st, f.ctr, scene->dev.n_spt);
  lodgs::launch_select(&f, lodgs::make_view(*cam, tau), flags, d_idx, capacity, d_count, st);
  e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : lodgs::hip_fail(e, "lodgs_lod_select_noalloc");
}
