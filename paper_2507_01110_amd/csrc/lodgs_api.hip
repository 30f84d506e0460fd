// C ABI: error reporting, scene and frame objects, argument checks and the
// per-view constants.  The stage kernels live in lodgs_select.hip,
// lodgs_render.hip and lodgs_backward.hip.
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>

#include "lodgs_internal.h"

namespace {
thread_local char g_err[512] = "";
}

namespace lodgs {

int set_error(int code, const char* msg) {
  std::snprintf(g_err, sizeof g_err, "%s", msg);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  std::snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
  return LODGS_E_HIP;
}

int blend_pixels_per_lane(bool backward) {
  const char* e = std::getenv(backward ? "LODGS_BLEND_PX_BWD" : "LODGS_BLEND_PX_FWD");
  if (e && (e[0] == '1' || e[0] == '2' || e[0] == '4') && e[1] == 0) return e[0] - '0';
  return 1;
}

// Per-view constants, FP32 on the host (IEEE single, correctly rounded / and
// sqrt), identical for every kernel of the view.
ViewConst make_view(const lodgs_camera& c, float tau) {
  ViewConst v;
  std::memcpy(v.R, c.R, sizeof v.R);
  std::memcpy(v.t, c.t, sizeof v.t);
  std::memcpy(v.pos, c.pos, sizeof v.pos);
  v.fx = c.fx;
  v.fy = c.fy;
  v.cx = c.cx;
  v.cy = c.cy;
  v.width = c.width;
  v.height = c.height;
  v.z_near = c.z_near;
  v.k = tau / c.fx;
  v.spt_scale = 1.0f;
  v.hl = c.cx / c.fx;
  v.hr = ((float)c.width - c.cx) / c.fx;
  v.ht = c.cy / c.fy;
  v.hb = ((float)c.height - c.cy) / c.fy;
  v.nl = std::sqrt(1.0f + v.hl * v.hl);
  v.nr = std::sqrt(1.0f + v.hr * v.hr);
  v.nt = std::sqrt(1.0f + v.ht * v.ht);
  v.nb = std::sqrt(1.0f + v.hb * v.hb);
  v.tiles_x = (c.width + kTile - 1) / kTile;
  v.tiles_y = (c.height + kTile - 1) / kTile;
  return v;
}

void stage_begin(lodgs_frame* f, int stage, hipStream_t st) {
  if (!f || !f->timing) return;
  hipEvent_t a;
  if (hipEventCreate(&a) != hipSuccess) return;
  (void)hipEventRecord(a, st);
  f->open_stage = stage;
  f->open_event = a;
}

void stage_end(lodgs_frame* f, hipStream_t st) {
  if (!f || !f->timing || !f->open_event) return;
  hipEvent_t b;
  if (hipEventCreate(&b) != hipSuccess) return;
  (void)hipEventRecord(b, st);
  f->timed.push_back({f->open_stage, f->open_event, b});
  f->open_event = nullptr;
}

namespace {
__global__ void k_set_view(ViewConst v, ViewConst* dst, FrameCounters* ctr, int mode, const int32_t* d_count,
                           int64_t cap) {
  *dst = v;
  if (mode == kViewSelect) {
    ctr->n_spt_visible = 0;
    ctr->n_upper_selected = 0;
    ctr->sum_high = 0;
  } else if (mode == kViewRender) {
    int64_t n = *d_count;
    n = n < 0 ? 0 : (n > cap ? cap : n);
    ctr->n_render = (int32_t)n;
    ctr->n_drawn = 0;
    ctr->n_long = 0;
  }
}
}  // namespace

void launch_set_view(const ViewConst& v, ViewConst* dst, FrameCounters* ctr, int mode, const int32_t* d_count,
                     int64_t cap, hipStream_t st) {
  hipLaunchKernelGGL(k_set_view, dim3(1), dim3(1), 0, st, v, dst, ctr, mode, d_count, cap);
}

void launch_blend_count(lodgs_frame* f, hipStream_t st);
void launch_l1_loss(const float* img, const float* target, int64_t n, float* grad, float* loss, hipStream_t st);

}  // namespace lodgs

using lodgs::hip_fail;
using lodgs::set_error;

namespace {

__global__ void k_clear_status(FrameCounters* c) { c->status = LODGS_OK; }

__global__ void k_selftest(const float* in32, const double* in64, int64_t n, float* out32, double* out64) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float a = in32[2 * i], b = in32[2 * i + 1];
    out32[3 * i] = a / b;
    out32[3 * i + 1] = __builtin_sqrtf(fabsf(a));
    out32[3 * i + 2] = lodgs::fexp(a);
    const double c = in64[2 * i], d = in64[2 * i + 1];
    out64[2 * i] = c / d;
    out64[2 * i + 1] = __builtin_sqrt(fabs(c));
  }
}

}  // namespace

namespace lodgs {

bool camera_ok(const lodgs_camera* c) {
  if (!c) return false;
  if (c->width <= 0 || c->height <= 0 || c->width > 16384 || c->height > 16384) return false;
  if (!(c->fx > 0.0f) || !(c->fy > 0.0f) || !std::isfinite(c->fx) || !std::isfinite(c->fy)) return false;
  if (!std::isfinite(c->cx) || !std::isfinite(c->cy) || !std::isfinite(c->z_near) || !(c->z_near > 0.0f))
    return false;
  for (float x : c->R)
    if (!std::isfinite(x)) return false;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(c->t[k]) || !std::isfinite(c->pos[k])) return false;
  return true;
}

}  // namespace lodgs

using lodgs::camera_ok;

namespace {

template <class T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (count > 0 ? count : 1));
}

void free_frame(lodgs_frame* f) {
  if (!f) return;
  for (auto& r : f->timed) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (f->open_event) (void)hipEventDestroy(f->open_event);
  // the arrays frame_create allocated (the same visitor; null ones skipped)
  if (f->scene)
    lodgs::frame_arrays(f, f->scene->dev, f->caps, [](auto*& ptr, size_t) {
      if (ptr) (void)hipFree(ptr);
      ptr = nullptr;
    });
  delete f;
}

__global__ void k_iota(int32_t* a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (int32_t)i;
}

}  // namespace

namespace lodgs {

size_t frame_bytes(const lodgs_scene* scene, const lodgs_frame_caps& caps) {
  lodgs_frame f{};
  size_t total = 0;
  frame_arrays(&f, scene->dev, caps, [&total](auto*& ptr, size_t cnt) {
    const size_t b = sizeof(*ptr) * (cnt > 0 ? cnt : 1);
    total += (b + 255) / 256 * 256;  // hipMalloc's granularity at least
  });
  return total;
}

}  // namespace lodgs

namespace {

// Selection position of each instance in tile order.
__global__ void k_instance_positions(const uint2* info_k, int64_t m, int32_t* pos) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
    pos[k] = (int32_t)info_k[k].x;
}

}  // namespace

extern "C" {

const char* lodgs_last_error(void) { return g_err; }

int lodgs_scene_create(const lodgs_scene_desc* d, lodgs_scene** out) {
  if (!d || !out) return set_error(LODGS_E_INVALID, "lodgs_scene_create: null argument");
  *out = nullptr;
  if (d->n_nodes <= 0 || d->n_nodes > (int64_t)INT32_MAX - 1)
    return set_error(LODGS_E_INVALID, "lodgs_scene_create: n_nodes out of range");
  if (d->n_upper < 0 || d->n_spt <= 0 || (int64_t)d->n_upper + d->n_spt > d->n_nodes)
    return set_error(LODGS_E_INVALID, "lodgs_scene_create: bad n_upper / n_spt");
  if (d->sh_degree < 0 || d->sh_degree > 3) return set_error(LODGS_E_INVALID, "lodgs_scene_create: sh_degree 0..3");
  if (!d->d_means || !d->d_log_scales || !d->d_quats || !d->d_opacity_logits || !d->d_sh || !d->d_r_min ||
      !d->d_r_max || !d->d_rho || (!d->d_upper_parent && d->n_upper > 0) || !d->d_spt_begin || !d->d_spt_parent)
    return set_error(LODGS_E_INVALID, "lodgs_scene_create: null device array");
  if ((reinterpret_cast<uintptr_t>(d->d_quats) & 15u) != 0 || (reinterpret_cast<uintptr_t>(d->d_sh) & 15u) != 0)
    return set_error(LODGS_E_INVALID, "lodgs_scene_create: quats and sh must be 16-byte aligned");
  lodgs_scene* s = new (std::nothrow) lodgs_scene;
  if (!s) return set_error(LODGS_E_OOM, "lodgs_scene_create: out of host memory");
  SceneDev& v = s->dev;
  v.n_nodes = d->n_nodes;
  v.n_upper = d->n_upper;
  v.n_spt = d->n_spt;
  v.sh_degree = d->sh_degree;
  v.n_coef = 3 * (d->sh_degree + 1) * (d->sh_degree + 1);
  v.means = d->d_means;
  v.log_scales = d->d_log_scales;
  v.quats = d->d_quats;
  v.opacity_logits = d->d_opacity_logits;
  v.sh = d->d_sh;
  v.r_min = d->d_r_min;
  v.r_max = d->d_r_max;
  v.rho = d->d_rho;
  v.upper_parent = d->d_upper_parent;
  v.spt_begin = d->d_spt_begin;
  v.spt_parent = d->d_spt_parent;
  v.anc = nullptr;
  v.anc_depth = 0;
  v.spt_radius = nullptr;
  v.parent = nullptr;
  v.child = nullptr;
  v.height = 0;
  s->anc_owned = nullptr;
  s->radius_owned = nullptr;
  int rc = lodgs::build_ancestor_table(s);
  if (rc == LODGS_OK) rc = lodgs::build_spt_radius(s);
  if (rc != LODGS_OK) {
    if (s->anc_owned) (void)hipFree(s->anc_owned);
    if (s->radius_owned) (void)hipFree(s->radius_owned);
    delete s;
    return rc;
  }
  *out = s;
  return LODGS_OK;
}

int lodgs_scene_set_hierarchy(lodgs_scene* s, const int32_t* d_parent, const int32_t* d_child, int32_t height) {
  if (!s || !d_parent || !d_child) return set_error(LODGS_E_INVALID, "lodgs_scene_set_hierarchy: null argument");
  if (height < 1 || height > 4096) return set_error(LODGS_E_INVALID, "lodgs_scene_set_hierarchy: height 1..4096");
  if ((reinterpret_cast<uintptr_t>(d_child) & 7u) != 0)
    return set_error(LODGS_E_INVALID, "lodgs_scene_set_hierarchy: d_child must be 8-byte aligned");
  int32_t p0 = 0;
  hipError_t e = hipMemcpy(&p0, d_parent, sizeof p0, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "lodgs_scene_set_hierarchy");
  if (p0 != -1) return set_error(LODGS_E_INVALID, "lodgs_scene_set_hierarchy: position 0 must be the root");
  s->dev.parent = d_parent;
  s->dev.child = reinterpret_cast<const int2*>(d_child);
  s->dev.height = height;
  return LODGS_OK;
}

void lodgs_scene_destroy(lodgs_scene* s) {
  if (!s) return;
  if (s->anc_owned) (void)hipFree(s->anc_owned);
  if (s->radius_owned) (void)hipFree(s->radius_owned);
  delete s;
}

int lodgs_frame_create(const lodgs_scene* scene, const lodgs_frame_caps* caps, lodgs_frame** out) {
  if (!scene || !caps || !out) return set_error(LODGS_E_INVALID, "lodgs_frame_create: null argument");
  *out = nullptr;
  if (caps->max_selected <= 0 || caps->max_selected > (int64_t)INT32_MAX / 16 || caps->max_instances <= 0 ||
      caps->max_instances > (int64_t)INT32_MAX - 1 || caps->max_width <= 0 || caps->max_height <= 0 ||
      caps->max_width > 16384 || caps->max_height > 16384)
    return set_error(LODGS_E_INVALID, "lodgs_frame_create: capacities out of range");
  lodgs_frame* f = new (std::nothrow) lodgs_frame();
  if (!f) return set_error(LODGS_E_OOM, "lodgs_frame_create: out of host memory");
  f->scene = scene;
  f->caps = *caps;
  f->spt_scale = 1.0f;
  f->blend_px_fwd = lodgs::blend_pixels_per_lane(false);
  f->blend_px_bwd = lodgs::blend_pixels_per_lane(true);
  hipError_t e = hipSuccess;
  // LODGS_FAIL_FRAME_ALLOC=k (a test of the failure path): the k-th device
  // allocation of this call reports out of memory instead of allocating
  const char* fail_env = std::getenv("LODGS_FAIL_FRAME_ALLOC");
  const long fail_at = fail_env ? std::strtol(fail_env, nullptr, 10) : 0;
  long n_alloc = 0;
  lodgs::frame_arrays(f, scene->dev, *caps, [&e, &n_alloc, fail_at](auto*& ptr, size_t cnt) {
    if (e != hipSuccess) return;
    e = ++n_alloc == fail_at ? hipErrorOutOfMemory : dalloc(&ptr, cnt);
  });
  if (scene->dev.parent) f->cut_height = scene->dev.height;
  if (e != hipSuccess) {
    free_frame(f);
    (void)hipGetLastError();
    return set_error(LODGS_E_OOM, "lodgs_frame_create: device allocation failed");
  }
  const SceneDev& S = scene->dev;
  const size_t ns = (size_t)caps->max_selected;
  FrameCounters c;
  std::memset(&c, 0, sizeof c);
  c.spt_count = S.n_spt;
  c.n_bit_words = (int32_t)lodgs::cut_bit_words(S.n_nodes);
  e = hipMemcpy(f->ctr, &c, sizeof c, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_iota, dim3(1024), dim3(256), 0, 0, f->iota, (int64_t)ns);
    e = hipGetLastError();
    // the null stream only: work in flight on other (non-blocking) streams,
    // such as a server's other slots, is not waited for
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  }
  if (e != hipSuccess) {
    free_frame(f);
    return hip_fail(e, "lodgs_frame_create");
  }
  *out = f;
  return LODGS_OK;
}

void lodgs_frame_destroy(lodgs_frame* f) { free_frame(f); }

int lodgs_lod_select(lodgs_frame* f, const lodgs_camera* cam, float tau, uint32_t flags, int32_t* d_idx,
                     int64_t capacity, int32_t* d_count, lodgs_stream stream) {
  if (!f || !d_idx || !d_count) return set_error(LODGS_E_INVALID, "lodgs_lod_select: null argument");
  if (!camera_ok(cam)) return set_error(LODGS_E_INVALID, "lodgs_lod_select: bad camera");
  if (!std::isfinite(tau) || tau < 0.0f) return set_error(LODGS_E_INVALID, "lodgs_lod_select: tau must be finite, >= 0");
  if (capacity < 0 || capacity > (int64_t)INT32_MAX) return set_error(LODGS_E_INVALID, "lodgs_lod_select: capacity");
  if (flags & ~(LODGS_CULL | LODGS_CONSERVATIVE | LODGS_CUT_BFS | LODGS_CUT_PARALLEL))
    return set_error(LODGS_E_INVALID, "lodgs_lod_select: unknown flag");
  const uint32_t full = flags & (LODGS_CUT_BFS | LODGS_CUT_PARALLEL);
  if (full && (full == (LODGS_CUT_BFS | LODGS_CUT_PARALLEL) || (flags & LODGS_CONSERVATIVE)))
    return set_error(LODGS_E_INVALID, "lodgs_lod_select: LODGS_CUT_BFS, LODGS_CUT_PARALLEL and LODGS_CONSERVATIVE exclude each other");
  if (full && !f->cut_bits)
    return set_error(LODGS_E_STATE, "lodgs_lod_select: the frame was created before lodgs_scene_set_hierarchy");
  lodgs::ViewConst v = lodgs::make_view(*cam, tau);
  v.spt_scale = f->spt_scale;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (full) lodgs::launch_select_full(f, v, flags, d_idx, capacity, d_count, st);
  else lodgs::launch_select(f, v, flags, d_idx, capacity, d_count, st);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_lod_select");
}

int lodgs_lod_select_cached(lodgs_frame* f, lodgs_cut_cache* c, const lodgs_camera* cam, float tau, uint32_t flags,
                            int32_t* d_idx, int64_t capacity, int32_t* d_count, lodgs_stream stream) {
  if (!f || !c || !d_idx || !d_count) return set_error(LODGS_E_INVALID, "lodgs_lod_select_cached: null argument");
  if (!camera_ok(cam)) return set_error(LODGS_E_INVALID, "lodgs_lod_select_cached: bad camera");
  if (!std::isfinite(tau) || tau < 0.0f)
    return set_error(LODGS_E_INVALID, "lodgs_lod_select_cached: tau must be finite, >= 0");
  if (capacity < 0 || capacity > (int64_t)INT32_MAX)
    return set_error(LODGS_E_INVALID, "lodgs_lod_select_cached: capacity");
  if (flags & ~LODGS_CULL) return set_error(LODGS_E_INVALID, "lodgs_lod_select_cached: only LODGS_CULL is allowed");
  lodgs::ViewConst v = lodgs::make_view(*cam, tau);
  v.spt_scale = f->spt_scale;
  return lodgs::cache_select(f, c, v, flags, d_idx, capacity, d_count, reinterpret_cast<hipStream_t>(stream));
}

int lodgs_render(lodgs_frame* f, const int32_t* d_idx, const int32_t* d_count, const lodgs_camera* cam,
                 const float bg[3], float* d_rgb, lodgs_stream stream) {
  if (!f || !d_idx || !d_count || !d_rgb) return set_error(LODGS_E_INVALID, "lodgs_render: null argument");
  if (!camera_ok(cam)) return set_error(LODGS_E_INVALID, "lodgs_render: bad camera");
  if (cam->width > f->caps.max_width || cam->height > f->caps.max_height)
    return set_error(LODGS_E_CAPACITY, "lodgs_render: image larger than the frame's capacity");
  const lodgs::ViewConst v = lodgs::make_view(*cam, 0.0f);
  float b[3] = {0.0f, 0.0f, 0.0f};
  if (bg)
    for (int k = 0; k < 3; ++k) b[k] = bg[k];
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  f->rows_mode = false;
  lodgs::launch_render(f, d_idx, d_count, v, b, d_rgb, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "lodgs_render");
  f->rendered = true;
  f->partials_ready = false;
  f->r_idx = d_idx;
  f->r_count = d_count;
  f->r_rgb = d_rgb;
  std::memcpy(f->bg, b, sizeof b);
  f->view = v;
  return LODGS_OK;
}

int lodgs_render_rows(lodgs_frame* f, const lodgs_grads* rows, const int32_t* d_count, const lodgs_camera* cam,
                      const float bg[3], float* d_rgb, lodgs_stream stream) {
  if (!f || !rows || !d_count || !d_rgb) return set_error(LODGS_E_INVALID, "lodgs_render_rows: null argument");
  if (!rows->d_means || !rows->d_log_scales || !rows->d_quats || !rows->d_opacity_logits || !rows->d_sh)
    return set_error(LODGS_E_INVALID, "lodgs_render_rows: every parameter group is needed");
  if ((reinterpret_cast<uintptr_t>(rows->d_quats) | reinterpret_cast<uintptr_t>(rows->d_sh)) & 15u)
    return set_error(LODGS_E_INVALID, "lodgs_render_rows: quaternion and SH rows must be 16-byte aligned");
  if (!camera_ok(cam)) return set_error(LODGS_E_INVALID, "lodgs_render_rows: bad camera");
  if (cam->width > f->caps.max_width || cam->height > f->caps.max_height)
    return set_error(LODGS_E_CAPACITY, "lodgs_render_rows: image larger than the frame's capacity");
  const lodgs::ViewConst v = lodgs::make_view(*cam, 0.0f);
  float b[3] = {0.0f, 0.0f, 0.0f};
  if (bg)
    for (int k = 0; k < 3; ++k) b[k] = bg[k];
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  f->rows_dev = f->scene->dev;
  f->rows_dev.means = rows->d_means;
  f->rows_dev.log_scales = rows->d_log_scales;
  f->rows_dev.quats = rows->d_quats;
  f->rows_dev.opacity_logits = rows->d_opacity_logits;
  f->rows_dev.sh = rows->d_sh;
  f->rows_mode = true;
  lodgs::launch_render(f, f->iota, d_count, v, b, d_rgb, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "lodgs_render_rows");
  f->rendered = true;
  f->partials_ready = false;
  f->r_idx = f->iota;
  f->r_count = d_count;
  f->r_rgb = d_rgb;
  std::memcpy(f->bg, b, sizeof b);
  f->view = v;
  return LODGS_OK;
}

int lodgs_render_backward_phases(lodgs_frame* f, const float* d_dL_drgb, const lodgs_grads* sel,
                                 const lodgs_grads* nodes, uint32_t phases, lodgs_stream stream) {
  const bool part = (phases & LODGS_BWD_PARTIALS) != 0, scat = (phases & LODGS_BWD_SCATTER) != 0;
  if (!f || (part && !d_dL_drgb) || (phases & ~(uint32_t)(LODGS_BWD_PARTIALS | LODGS_BWD_SCATTER)) != 0)
    return set_error(LODGS_E_INVALID, "lodgs_render_backward: null argument or unknown phase");
  if (!f->rendered) return set_error(LODGS_E_STATE, "lodgs_render_backward: no render on this frame");
  if (scat && !part && !f->partials_ready)
    return set_error(LODGS_E_STATE, "lodgs_render_backward: the scatter half needs the partials of the last render");
  if (scat && f->rows_mode && nodes)
    return set_error(LODGS_E_INVALID, "lodgs_render_backward: after lodgs_render_rows only sel gradients are written");
  if (scat &&
      ((sel && (reinterpret_cast<uintptr_t>(sel->d_sh) & 15u)) || (nodes && (reinterpret_cast<uintptr_t>(nodes->d_sh) & 15u))))
    return set_error(LODGS_E_INVALID, "lodgs_render_backward: SH gradient arrays must be 16-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  lodgs::launch_backward(f, d_dL_drgb, sel, nodes, phases, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "lodgs_render_backward");
  if (part) f->partials_ready = true;
  return LODGS_OK;
}

int lodgs_render_backward(lodgs_frame* f, const float* d_dL_drgb, const lodgs_grads* sel, const lodgs_grads* nodes,
                          lodgs_stream stream) {
  return lodgs_render_backward_phases(f, d_dL_drgb, sel, nodes, LODGS_BWD_PARTIALS | LODGS_BWD_SCATTER, stream);
}

int lodgs_frame_stats(lodgs_frame* f, lodgs_stats* out, lodgs_stream stream) {
  if (!f || !out) return set_error(LODGS_E_INVALID, "lodgs_frame_stats: null argument");
  FrameCounters c;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&c, f->ctr, sizeof c, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "lodgs_frame_stats");
  out->status = c.status;
  out->n_selected = c.n_selected;
  out->n_upper_selected = c.n_upper_selected;
  out->n_spt_visible = c.n_spt_visible;
  out->n_spt_candidates = c.sum_high;
  out->n_rendered = c.n_render;
  out->n_drawn = c.n_drawn;
  out->n_instances = c.n_instances;
  return LODGS_OK;
}

int lodgs_frame_read_instances(lodgs_frame* f, int32_t* d_tile, int32_t* d_pos, int64_t capacity, int64_t* n_out,
                               lodgs_stream stream) {
  if (!f || !d_tile || !d_pos || !n_out || capacity < 0)
    return set_error(LODGS_E_INVALID, "lodgs_frame_read_instances: bad argument");
  if (!f->rendered) return set_error(LODGS_E_STATE, "lodgs_frame_read_instances: no render on this frame");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  FrameCounters c;
  hipError_t e = hipMemcpyAsync(&c, f->ctr, sizeof c, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "lodgs_frame_read_instances");
  *n_out = c.n_instances;
  int64_t m = c.n_inst_clamped < capacity ? c.n_inst_clamped : capacity;
  if (m > 0) {
    e = hipMemcpyAsync(d_tile, f->sorted_ikey, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
      const int64_t g = (m + lodgs::kBlock - 1) / lodgs::kBlock;
      hipLaunchKernelGGL(k_instance_positions, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(lodgs::kBlock), 0, st,
                         f->sorted_info, m, d_pos);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "lodgs_frame_read_instances");
  }
  return LODGS_OK;
}

int lodgs_frame_set_timing(lodgs_frame* f, int enable) {
  if (!f) return set_error(LODGS_E_INVALID, "lodgs_frame_set_timing: null frame");
  f->timing = enable != 0;
  return LODGS_OK;
}

int lodgs_frame_timings(lodgs_frame* f, lodgs_timings* out) {
  if (!f || !out) return set_error(LODGS_E_INVALID, "lodgs_frame_timings: null argument");
  std::memset(out, 0, sizeof *out);
  int rc = LODGS_OK;
  for (auto& r : f->timed) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && rc == LODGS_OK) rc = hip_fail(e, "lodgs_frame_timings");
    if (r.stage >= 0 && r.stage < LODGS_N_STAGES) {
      out->ms[r.stage] += ms;
      out->calls[r.stage] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  f->timed.clear();
  return rc;
}

int lodgs_frame_blend_work(lodgs_frame* f, int64_t* evaluations, int64_t* contributions, lodgs_stream stream) {
  if (!f || !evaluations || !contributions) return set_error(LODGS_E_INVALID, "lodgs_frame_blend_work: null argument");
  if (!f->rendered) return set_error(LODGS_E_STATE, "lodgs_frame_blend_work: no render on this frame");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  lodgs::launch_blend_count(f, st);
  unsigned long long w[2] = {0, 0};
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(w, f->work, sizeof w, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "lodgs_frame_blend_work");
  *evaluations = (int64_t)w[0];
  *contributions = (int64_t)w[1];
  return LODGS_OK;
}

int lodgs_l1_loss(lodgs_frame* f, const float* d_img, const float* d_target, int64_t n, float* d_grad, float* d_loss,
                  lodgs_stream stream) {
  if (!d_img || !d_target || !d_grad || n <= 0) return set_error(LODGS_E_INVALID, "lodgs_l1_loss: bad argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  lodgs::stage_begin(f, LODGS_STAGE_LOSS, st);
  lodgs::launch_l1_loss(d_img, d_target, n, d_grad, d_loss, st);
  lodgs::stage_end(f, st);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_l1_loss");
}

int lodgs_selftest_arith(const float* d_in32, const double* d_in64, int64_t n, float* d_out32, double* d_out64,
                         lodgs_stream stream) {
  if (!d_in32 || !d_in64 || !d_out32 || !d_out64 || n < 0)
    return set_error(LODGS_E_INVALID, "lodgs_selftest_arith: bad argument");
  if (n == 0) return LODGS_OK;
  int64_t g = (n + 255) / 256;
  g = g > 1024 ? 1024 : g;
  hipLaunchKernelGGL(k_selftest, dim3((int)g), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), d_in32, d_in64, n,
                     d_out32, d_out64);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_selftest_arith");
}

}  // extern "C"

struct lodgs_graph {
  lodgs_frame* frame;
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipGraphNode_t node_sel, node_ren;
  hipKernelNodeParams p_sel, p_ren;
  // the captured arguments of the two k_set_view nodes other than the view
  lodgs::ViewConst* dst_sel;
  lodgs::ViewConst* dst_ren;
  FrameCounters* ctr_sel;
  FrameCounters* ctr_ren;
  int mode_sel, mode_ren;
  const int32_t* count_sel;
  const int32_t* count_ren;
  int64_t cap_sel, cap_ren;
  int32_t width, height;
  // the forward blend node: its output image argument is replaced when a
  // replay writes to another image
  hipGraphNode_t node_blend;
  hipKernelNodeParams p_blend;
  int blend_arg, blend_nargs;
  // a training step's loss node (nullptr in a view graph): its target image
  // argument is replaced when a replay takes another target
  hipGraphNode_t node_l1;
  hipKernelNodeParams p_l1;
  int l1_arg, l1_nargs;
};

namespace lodgs {

// Replaces argument `arg` of a captured kernel node (nargs arguments) by the
// pointer value v.
static hipError_t set_pointer_arg(hipGraphExec_t exec, hipGraphNode_t node, const hipKernelNodeParams& p, int arg,
                                  int nargs, const void* v) {
  void* args[16];
  if (nargs > 16) return hipErrorInvalidValue;
  for (int k = 0; k < nargs; ++k) args[k] = p.kernelParams[k];
  args[arg] = &v;
  hipKernelNodeParams q = p;
  q.kernelParams = args;
  return hipGraphExecKernelNodeSetParams(exec, node, &q);
}

int graph_launch(lodgs_graph* g, const lodgs_camera* cam, float tau, float* d_rgb, hipStream_t st) {
  if (!g || !camera_ok(cam)) return set_error(LODGS_E_INVALID, "lodgs_graph_launch: bad argument");
  if (cam->width != g->width || cam->height != g->height)
    return set_error(LODGS_E_INVALID, "lodgs_graph_launch: image size differs from the captured one");
  if (!std::isfinite(tau) || tau < 0.0f) return set_error(LODGS_E_INVALID, "lodgs_graph_launch: bad tau");
  ViewConst vs = make_view(*cam, tau), vr = make_view(*cam, 0.0f);
  vs.spt_scale = g->frame->spt_scale;  // the frame's LoD noise at this launch
  void* args_s[6] = {&vs, &g->dst_sel, &g->ctr_sel, &g->mode_sel, &g->count_sel, &g->cap_sel};
  void* args_r[6] = {&vr, &g->dst_ren, &g->ctr_ren, &g->mode_ren, &g->count_ren, &g->cap_ren};
  hipKernelNodeParams ps = g->p_sel, pr = g->p_ren;
  ps.kernelParams = args_s;
  pr.kernelParams = args_r;
  hipError_t e = hipGraphExecKernelNodeSetParams(g->exec, g->node_sel, &ps);
  if (e == hipSuccess) e = hipGraphExecKernelNodeSetParams(g->exec, g->node_ren, &pr);
  if (e == hipSuccess && d_rgb) {
    if (g->node_l1) return set_error(LODGS_E_INVALID, "lodgs_graph_launch: a training step keeps its image");
    e = set_pointer_arg(g->exec, g->node_blend, g->p_blend, g->blend_arg, g->blend_nargs, d_rgb);
  }
  if (e == hipSuccess) e = hipGraphLaunch(g->exec, st);
  if (e != hipSuccess) return hip_fail(e, "lodgs_graph_launch");
  g->frame->view = vr;
  if (d_rgb) g->frame->r_rgb = d_rgb;
  return LODGS_OK;
}

// Captures what launch() enqueues on st into g, finds the nodes a replay
// updates (the two view-constant nodes, the forward blend, the loss if any)
// and instantiates the graph.
template <class Launch>
static int capture(lodgs_graph* g, hipStream_t st, const char* who, Launch launch) {
  lodgs_frame* f = g->frame;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, who);
  launch();
  e = hipStreamEndCapture(st, &g->graph);
  if (e != hipSuccess) return hip_fail(e, who);
  size_t nn = 0;
  e = hipGraphGetNodes(g->graph, nullptr, &nn);
  std::vector<hipGraphNode_t> nodes(nn);
  if (e == hipSuccess && nn) e = hipGraphGetNodes(g->graph, nodes.data(), &nn);
  for (size_t k = 0; e == hipSuccess && k < nn; ++k) {
    hipGraphNodeType ty;
    if (hipGraphNodeGetType(nodes[k], &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams p;
    if (hipGraphKernelNodeGetParams(nodes[k], &p) != hipSuccess) continue;
    int nargs = 0;
    int a = blend_output_arg(p.func, &nargs);
    if (a >= 0) {
      g->node_blend = nodes[k];
      g->p_blend = p;
      g->blend_arg = a;
      g->blend_nargs = nargs;
      continue;
    }
    a = l1_target_arg(p.func, &nargs);
    if (a >= 0) {
      g->node_l1 = nodes[k];
      g->p_l1 = p;
      g->l1_arg = a;
      g->l1_nargs = nargs;
      continue;
    }
    if (p.func != reinterpret_cast<void*>(&k_set_view)) continue;
    ViewConst* dst = *reinterpret_cast<ViewConst**>(p.kernelParams[1]);
    FrameCounters* ctr = *reinterpret_cast<FrameCounters**>(p.kernelParams[2]);
    const int mode = *reinterpret_cast<int*>(p.kernelParams[3]);
    const int32_t* cnt = *reinterpret_cast<const int32_t**>(p.kernelParams[4]);
    const int64_t cap = *reinterpret_cast<int64_t*>(p.kernelParams[5]);
    if (dst == f->d_view_sel) {
      g->node_sel = nodes[k];
      g->p_sel = p;
      g->dst_sel = dst;
      g->ctr_sel = ctr;
      g->mode_sel = mode;
      g->count_sel = cnt;
      g->cap_sel = cap;
    } else if (dst == f->d_view_ren) {
      g->node_ren = nodes[k];
      g->p_ren = p;
      g->dst_ren = dst;
      g->ctr_ren = ctr;
      g->mode_ren = mode;
      g->count_ren = cnt;
      g->cap_ren = cap;
    }
  }
  if (e != hipSuccess) return hip_fail(e, who);
  if (!g->node_sel || !g->node_ren || !g->node_blend)
    return set_error(LODGS_E_STATE, "graph capture: view nodes not found in the captured graph");
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  return e == hipSuccess ? LODGS_OK : hip_fail(e, who);
}

// Argument checks shared by the two captures.
static int capture_args_ok(lodgs_frame* f, const lodgs_camera* cam, float tau, uint32_t flags, int64_t capacity,
                           const char* who) {
  if (!camera_ok(cam)) return set_error(LODGS_E_INVALID, who);
  if (!std::isfinite(tau) || tau < 0.0f) return set_error(LODGS_E_INVALID, who);
  if (capacity < 0 || capacity > (int64_t)INT32_MAX || (flags & ~(LODGS_CULL | LODGS_CONSERVATIVE)))
    return set_error(LODGS_E_INVALID, who);
  if (cam->width > f->caps.max_width || cam->height > f->caps.max_height)
    return set_error(LODGS_E_CAPACITY, who);
  if (f->timing) return set_error(LODGS_E_STATE, who);
  return LODGS_OK;
}

}  // namespace lodgs

extern "C" {

void lodgs_graph_destroy(lodgs_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

int lodgs_graph_capture_view(lodgs_frame* f, const lodgs_camera* cam, float tau, uint32_t flags, int32_t* d_idx,
                             int64_t capacity, int32_t* d_count, const float bg[3], float* d_rgb,
                             lodgs_stream stream, lodgs_graph** out) {
  if (!f || !d_idx || !d_count || !d_rgb || !out || !stream)
    return set_error(LODGS_E_INVALID, "lodgs_graph_capture_view: null argument (a non-default stream is required)");
  *out = nullptr;
  int rc = lodgs::capture_args_ok(f, cam, tau, flags, capacity,
                                  "lodgs_graph_capture_view: bad camera, tau, capacity or flags, an image larger "
                                  "than the frame's, or a frame in timing mode");
  if (rc != LODGS_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  lodgs_graph* g = new (std::nothrow) lodgs_graph();
  if (!g) return set_error(LODGS_E_OOM, "lodgs_graph_capture_view: out of host memory");
  g->frame = f;
  g->width = cam->width;
  g->height = cam->height;
  float b[3] = {0.0f, 0.0f, 0.0f};
  if (bg)
    for (int k = 0; k < 3; ++k) b[k] = bg[k];
  lodgs::ViewConst vs = lodgs::make_view(*cam, tau);
  vs.spt_scale = f->spt_scale;
  const lodgs::ViewConst vr = lodgs::make_view(*cam, 0.0f);
  rc = lodgs::capture(g, st, "lodgs_graph_capture_view", [&] {
    lodgs::launch_select(f, vs, flags, d_idx, capacity, d_count, st);
    f->rows_mode = false;
    lodgs::launch_render(f, d_idx, d_count, vr, b, d_rgb, st);
  });
  if (rc != LODGS_OK) {
    lodgs_graph_destroy(g);
    return rc;
  }
  f->rendered = true;
  f->partials_ready = false;
  f->r_idx = d_idx;
  f->r_count = d_count;
  f->r_rgb = d_rgb;
  std::memcpy(f->bg, b, sizeof b);
  f->view = vr;
  *out = g;
  return LODGS_OK;
}

int lodgs_graph_capture_step(lodgs_frame* f, const lodgs_camera* cam, float tau, uint32_t flags, int32_t* d_idx,
                             int64_t capacity, int32_t* d_count, const float bg[3], float* d_rgb,
                             const float* d_target, float* d_dL, float* d_loss, const lodgs_grads* sel,
                             const lodgs_grads* nodes, lodgs_stream stream, lodgs_graph** out) {
  if (!f || !d_idx || !d_count || !d_rgb || !d_target || !d_dL || !out || !stream)
    return set_error(LODGS_E_INVALID, "lodgs_graph_capture_step: null argument (a non-default stream is required)");
  *out = nullptr;
  int rc = lodgs::capture_args_ok(f, cam, tau, flags, capacity,
                                  "lodgs_graph_capture_step: bad camera, tau, capacity or flags, an image larger "
                                  "than the frame's, or a frame in timing mode");
  if (rc != LODGS_OK) return rc;
  if (nodes && sel) return set_error(LODGS_E_INVALID, "lodgs_graph_capture_step: give sel or nodes, not both");
  if ((sel && sel->d_sh && (reinterpret_cast<uintptr_t>(sel->d_sh) & 15u)) ||
      (nodes && nodes->d_sh && (reinterpret_cast<uintptr_t>(nodes->d_sh) & 15u)))
    return set_error(LODGS_E_INVALID, "lodgs_graph_capture_step: d_sh must be 16-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  lodgs_graph* g = new (std::nothrow) lodgs_graph();
  if (!g) return set_error(LODGS_E_OOM, "lodgs_graph_capture_step: out of host memory");
  g->frame = f;
  g->width = cam->width;
  g->height = cam->height;
  float b[3] = {0.0f, 0.0f, 0.0f};
  if (bg)
    for (int k = 0; k < 3; ++k) b[k] = bg[k];
  lodgs::ViewConst vs = lodgs::make_view(*cam, tau);
  vs.spt_scale = f->spt_scale;
  const lodgs::ViewConst vr = lodgs::make_view(*cam, 0.0f);
  const int64_t npx = 3 * (int64_t)cam->width * cam->height;
  rc = lodgs::capture(g, st, "lodgs_graph_capture_step", [&] {
    lodgs::launch_select(f, vs, flags, d_idx, capacity, d_count, st);
    f->rows_mode = false;
    lodgs::launch_render(f, d_idx, d_count, vr, b, d_rgb, st);
    // the state the backward's launches read, as lodgs_render leaves it
    f->r_idx = d_idx;
    f->r_count = d_count;
    f->r_rgb = d_rgb;
    f->view = vr;
    lodgs::launch_l1_loss(d_rgb, d_target, npx, d_dL, d_loss, st);
    lodgs::launch_backward(f, d_dL, sel, nodes, LODGS_BWD_PARTIALS | LODGS_BWD_SCATTER, st);
  });
  if (rc == LODGS_OK && !g->node_l1) rc = set_error(LODGS_E_STATE, "lodgs_graph_capture_step: loss node not found");
  if (rc != LODGS_OK) {
    lodgs_graph_destroy(g);
    return rc;
  }
  f->rendered = true;
  f->partials_ready = false;
  f->r_idx = d_idx;
  f->r_count = d_count;
  f->r_rgb = d_rgb;
  std::memcpy(f->bg, b, sizeof b);
  f->view = vr;
  *out = g;
  return LODGS_OK;
}

int lodgs_graph_launch(lodgs_graph* g, const lodgs_camera* cam, float tau, lodgs_stream stream) {
  return lodgs::graph_launch(g, cam, tau, nullptr, reinterpret_cast<hipStream_t>(stream));
}

int lodgs_graph_launch_step(lodgs_graph* g, const lodgs_camera* cam, float tau, const float* d_target,
                            lodgs_stream stream) {
  if (!g || !g->node_l1 || !d_target)
    return set_error(LODGS_E_INVALID, "lodgs_graph_launch_step: not a training-step graph, or no target");
  const hipError_t e = lodgs::set_pointer_arg(g->exec, g->node_l1, g->p_l1, g->l1_arg, g->l1_nargs, d_target);
  if (e != hipSuccess) return hip_fail(e, "lodgs_graph_launch_step");
  return lodgs::graph_launch(g, cam, tau, nullptr, reinterpret_cast<hipStream_t>(stream));
}

int lodgs_frame_set_contrib_stats(lodgs_frame* f, int32_t* d_last, int32_t* d_count, const int32_t* d_iteration) {
  if (!f) return set_error(LODGS_E_INVALID, "lodgs_frame_set_contrib_stats: null frame");
  if (d_last && !d_iteration)
    return set_error(LODGS_E_INVALID, "lodgs_frame_set_contrib_stats: d_iteration is required with d_last");
  f->last_contrib = d_last;
  f->contrib_count = d_last ? d_count : nullptr;
  f->contrib_iteration = d_last ? d_iteration : nullptr;
  return LODGS_OK;
}

int lodgs_frame_set_lod_noise(lodgs_frame* f, float factor) {
  if (!f) return set_error(LODGS_E_INVALID, "lodgs_frame_set_lod_noise: null frame");
  if (!std::isfinite(factor) || !(factor > 0.0f))
    return set_error(LODGS_E_INVALID, "lodgs_frame_set_lod_noise: the factor must be finite and > 0");
  f->spt_scale = factor;
  return LODGS_OK;
}

int lodgs_frame_set_densify_stats(lodgs_frame* f, float* d_max_grad2d) {
  if (!f) return set_error(LODGS_E_INVALID, "lodgs_frame_set_densify_stats: null frame");
  f->max_grad2d = d_max_grad2d;
  return LODGS_OK;
}

int lodgs_frame_clear_status(lodgs_frame* f, lodgs_stream stream) {
  if (!f) return set_error(LODGS_E_INVALID, "lodgs_frame_clear_status: null argument");
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, reinterpret_cast<hipStream_t>(stream), f->ctr);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? LODGS_OK : hip_fail(e, "lodgs_frame_clear_status");
}

}  // extern "C"
