// Continuous-batching render server (forward only): requests of different
// image sizes, cameras and tau share the device through slots.  A slot owns
// a frame (the render workspace), a stream, a selection buffer, one captured
// view graph per image-size class, a completion event and a small record in
// mapped host memory through which its requests report their counters.
//
// Requests wait in a queue until a slot can take them: the largest idle slot
// whose capacities cover the request, or a new slot when fewer than max_slots exist
// and free HBM (hipMemGetInfo) covers the slot's bytes plus the caller's
// reserve.  A launch updates the graph's view constants and output image and
// replays it on the slot's stream, so the views of different slots overlap on
// the device while the host only queues, launches and polls events.
//
// A request whose selection or instance list outgrew its slot (the frame
// records LODGS_E_CAPACITY) is queued again at the front with the counts it
// reported as its new minimum capacities, and runs again on a slot large
// enough (made when free HBM allows, evicting idle slots that are too small
// if needed).  When no slot can ever take it (none busy, none large enough,
// none can be made) it completes with LODGS_E_CAPACITY: rejected.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <new>
#include <vector>

#include "lodgs_internal.h"

namespace {

constexpr int kMaxAttempts = 6;  // launches of one request (1 + capacity retries)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// What a finished request reports (written by the device into mapped host
// memory after the view's kernels).
struct Published {
  int32_t status;
  int32_t n_selected;
  int32_t n_drawn;
  int32_t pad;
  int64_t n_instances;
};

__global__ void k_publish(FrameCounters* ctr, Published* out) {
  Published p;
  p.status = ctr->status;
  p.n_selected = ctr->n_selected;
  p.n_drawn = ctr->n_drawn;
  p.pad = 0;
  p.n_instances = (int64_t)(uint32_t)ctr->n_instances;  // the scan's 32-bit full count
  *out = p;
  ctr->status = LODGS_OK;  // the next request on the slot starts clean
}

struct Job {
  uint64_t ticket, user;
  lodgs_camera cam;
  float tau;
  float* d_rgb;
  int size_class;
  int attempts;
  int64_t need_sel, need_inst;  // minimum capacities (from an earlier overflow)
  double t_submit, t_admit;
};

struct Slot {
  lodgs_frame* f = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  int32_t* idx = nullptr;
  int32_t* cnt = nullptr;
  Published* h_pub = nullptr;  // mapped host memory
  Published* d_pub = nullptr;  // its device address
  lodgs_graph* g[LODGS_SERVER_MAX_SIZES] = {};
  int64_t cap_sel = 0, cap_inst = 0;
  size_t bytes = 0;
  bool busy = false;
  Job job{};
};

}  // namespace

struct lodgs_server {
  const lodgs_scene* scene;
  lodgs_server_caps caps;
  int32_t max_w, max_h;
  std::vector<Slot*> slots;
  std::deque<Job> queue;
  std::deque<lodgs_completion> done;
  uint64_t next_ticket;
  int64_t n_retries, n_rejected, n_evicted;
};

namespace {

using lodgs::hip_fail;
using lodgs::set_error;

void destroy_slot(Slot* s) {
  if (!s) return;
  if (s->st) (void)hipStreamSynchronize(s->st);
  for (lodgs_graph*& g : s->g)
    if (g) lodgs_graph_destroy(g);
  if (s->f) lodgs_frame_destroy(s->f);
  if (s->idx) (void)hipFree(s->idx);
  if (s->cnt) (void)hipFree(s->cnt);
  if (s->h_pub) (void)hipHostFree(s->h_pub);
  if (s->ev) (void)hipEventDestroy(s->ev);
  if (s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

lodgs_frame_caps slot_caps(const lodgs_server* sv, int64_t sel, int64_t inst) {
  lodgs_frame_caps c;
  c.max_selected = sel;
  c.max_instances = inst;
  c.max_width = sv->max_w;
  c.max_height = sv->max_h;
  return c;
}

size_t slot_bytes(const lodgs_server* sv, int64_t sel, int64_t inst) {
  // frame + selection buffer and count (256-byte granules)
  const size_t idx = ((size_t)sel * 4 + 255) / 256 * 256 + 256;
  return lodgs::frame_bytes(sv->scene, slot_caps(sv, sel, inst)) + idx;
}

// A camera of the given size for the capture (the graph's view constants are
// replaced at every launch).
lodgs_camera capture_camera(int32_t w, int32_t h) {
  lodgs_camera c{};
  c.R[0] = c.R[4] = c.R[8] = 1.0f;
  c.fx = c.fy = 0.5f * (float)w;
  c.cx = 0.5f * (float)w;
  c.cy = 0.5f * (float)h;
  c.width = w;
  c.height = h;
  c.z_near = 0.2f;
  return c;
}

int make_slot(lodgs_server* sv, int64_t sel, int64_t inst, Slot** out) {
  *out = nullptr;
  Slot* s = new (std::nothrow) Slot();
  if (!s) return set_error(LODGS_E_OOM, "lodgs_server: out of host memory");
  s->cap_sel = sel;
  s->cap_inst = inst;
  s->bytes = slot_bytes(sv, sel, inst);
  const lodgs_frame_caps fc = slot_caps(sv, sel, inst);
  int rc = lodgs_frame_create(sv->scene, &fc, &s->f);
  hipError_t e = hipSuccess;
  if (rc == LODGS_OK) {
    e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->idx), sizeof(int32_t) * (size_t)sel);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s->cnt), sizeof(int32_t));
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&s->h_pub), sizeof(Published), hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_pub), s->h_pub, 0);
    if (e != hipSuccess) rc = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? LODGS_E_OOM : LODGS_E_HIP;
  }
  // One graph per size class, captured with a placeholder output that every
  // launch replaces (graph_launch is always given the request's image).
  for (int k = 0; rc == LODGS_OK && k < sv->caps.n_sizes; ++k) {
    const lodgs_camera c = capture_camera(sv->caps.sizes[k][0], sv->caps.sizes[k][1]);
    rc = lodgs_graph_capture_view(s->f, &c, 1.0f, sv->caps.flags, s->idx, sel, s->cnt, sv->caps.bg,
                                  reinterpret_cast<float*>(s->h_pub), s->st, &s->g[k]);
  }
  if (rc != LODGS_OK) {
    (void)hipGetLastError();
    destroy_slot(s);
    return e != hipSuccess ? hip_fail(e, "lodgs_server: slot") : rc;
  }
  *out = s;
  return LODGS_OK;
}

bool fits(const Slot* s, const Job& j) { return s->cap_sel >= j.need_sel && s->cap_inst >= j.need_inst; }

bool any_busy(const lodgs_server* sv) {
  for (const Slot* s : sv->slots)
    if (s->busy) return true;
  return false;
}

// Drops the idle slot with the smallest capacities that does not fit j;
// false when there is none.
bool evict_one(lodgs_server* sv, const Job& j) {
  int best = -1;
  for (int k = 0; k < (int)sv->slots.size(); ++k) {
    const Slot* s = sv->slots[k];
    if (s->busy || fits(s, j)) continue;
    if (best < 0 || s->bytes < sv->slots[best]->bytes) best = k;
  }
  if (best < 0) return false;
  destroy_slot(sv->slots[best]);
  sv->slots.erase(sv->slots.begin() + best);
  ++sv->n_evicted;
  return true;
}

// A new slot for j if the slot limit and free HBM allow it, evicting idle
// slots too small for j to make room.  Returns nullptr when impossible now.
Slot* grow(lodgs_server* sv, const Job& j, int* rc) {
  *rc = LODGS_OK;
  const int64_t sel = std::max(j.need_sel, sv->caps.max_selected);
  const int64_t inst = std::max(j.need_inst, sv->caps.max_instances);
  const size_t need = slot_bytes(sv, sel, inst);
  for (;;) {
    bool room = (int)sv->slots.size() < sv->caps.max_slots;
    if (room) {
      size_t free_b = 0, total_b = 0;
      hipError_t e = hipMemGetInfo(&free_b, &total_b);
      if (e != hipSuccess) {
        *rc = hip_fail(e, "lodgs_server: hipMemGetInfo");
        return nullptr;
      }
      room = free_b >= need + (size_t)sv->caps.hbm_reserve;
    }
    if (room) {
      Slot* s = nullptr;
      const int r = make_slot(sv, sel, inst, &s);
      if (r == LODGS_OK) {
        sv->slots.push_back(s);
        return s;
      }
      if (r != LODGS_E_OOM) {
        *rc = r;
        return nullptr;
      }
    }
    if (!evict_one(sv, j)) return nullptr;
  }
}

void complete(lodgs_server* sv, const Job& j, int32_t status, const Published* p) {
  lodgs_completion c{};
  c.ticket = j.ticket;
  c.user = j.user;
  c.status = status;
  c.attempts = j.attempts;
  if (p) {
    c.n_selected = p->n_selected;
    c.n_drawn = p->n_drawn;
    c.n_instances = p->n_instances;
  }
  c.t_submit = j.t_submit;
  c.t_admit = j.t_admit;
  c.t_done = now_s();
  if (status != LODGS_OK) ++sv->n_rejected;
  sv->done.push_back(c);
}

int launch(lodgs_server* sv, Slot* s, Job& j) {
  j.attempts += 1;
  j.t_admit = now_s();
  s->job = j;
  s->busy = true;
  int rc = lodgs::graph_launch(s->g[j.size_class], &j.cam, j.tau, j.d_rgb, s->st);
  if (rc == LODGS_OK) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(1), 0, s->st, s->f->ctr, s->d_pub);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(s->ev, s->st);
    if (e != hipSuccess) rc = hip_fail(e, "lodgs_server: launch");
  }
  if (rc != LODGS_OK) s->busy = false;
  return rc;
}

// Admits queued requests into slots, in queue order, as far as slots and
// free HBM allow.
int pump(lodgs_server* sv) {
  for (auto it = sv->queue.begin(); it != sv->queue.end();) {
    Job& j = *it;
    Slot* best = nullptr;
    // the largest idle slot that fits: a request's size is known only after
    // its first run, so a heavy one overflows less often on a grown slot
    for (Slot* s : sv->slots)
      if (!s->busy && fits(s, j) && (!best || s->bytes > best->bytes)) best = s;
    int rc = LODGS_OK;
    if (!best) best = grow(sv, j, &rc);
    if (rc != LODGS_OK) return rc;
    if (!best) {
      bool larger = false;  // a busy slot that fits will come free
      for (const Slot* s : sv->slots) larger = larger || fits(s, j);
      if (!any_busy(sv) && !larger) {  // nothing will change: rejected
        complete(sv, j, LODGS_E_CAPACITY, nullptr);
        it = sv->queue.erase(it);
        continue;
      }
      ++it;
      continue;
    }
    rc = launch(sv, best, j);
    if (rc != LODGS_OK) return rc;
    it = sv->queue.erase(it);
  }
  return LODGS_OK;
}

int find_class(const lodgs_server* sv, int32_t w, int32_t h) {
  for (int k = 0; k < sv->caps.n_sizes; ++k)
    if (sv->caps.sizes[k][0] == w && sv->caps.sizes[k][1] == h) return k;
  return -1;
}

}  // namespace

extern "C" {

int lodgs_server_create(const lodgs_scene* scene, const lodgs_server_caps* caps, lodgs_server** out) {
  if (!scene || !caps || !out) return set_error(LODGS_E_INVALID, "lodgs_server_create: null argument");
  *out = nullptr;
  if (caps->n_sizes < 1 || caps->n_sizes > LODGS_SERVER_MAX_SIZES)
    return set_error(LODGS_E_INVALID, "lodgs_server_create: n_sizes 1..LODGS_SERVER_MAX_SIZES");
  if (caps->max_slots < 1 || caps->max_slots > 64) return set_error(LODGS_E_INVALID, "lodgs_server_create: max_slots 1..64");
  if (caps->max_selected <= 0 || caps->max_selected > (int64_t)INT32_MAX / 16 || caps->max_instances <= 0 ||
      caps->max_instances > (int64_t)INT32_MAX - 1 || caps->hbm_reserve < 0)
    return set_error(LODGS_E_INVALID, "lodgs_server_create: capacities out of range");
  if (caps->flags & ~(LODGS_CULL | LODGS_CONSERVATIVE))
    return set_error(LODGS_E_INVALID, "lodgs_server_create: flags");
  int32_t mw = 0, mh = 0;
  for (int k = 0; k < caps->n_sizes; ++k) {
    const int32_t w = caps->sizes[k][0], h = caps->sizes[k][1];
    if (w <= 0 || h <= 0 || w > 16384 || h > 16384) return set_error(LODGS_E_INVALID, "lodgs_server_create: size");
    mw = std::max(mw, w);
    mh = std::max(mh, h);
  }
  lodgs_server* sv = new (std::nothrow) lodgs_server();
  if (!sv) return set_error(LODGS_E_OOM, "lodgs_server_create: out of host memory");
  sv->scene = scene;
  sv->caps = *caps;
  sv->max_w = mw;
  sv->max_h = mh;
  sv->next_ticket = 1;
  sv->n_retries = sv->n_rejected = sv->n_evicted = 0;
  *out = sv;
  return LODGS_OK;
}

void lodgs_server_destroy(lodgs_server* sv) {
  if (!sv) return;
  for (Slot* s : sv->slots) destroy_slot(s);
  delete sv;
}

int lodgs_server_submit(lodgs_server* sv, const lodgs_request* r, uint64_t* ticket) {
  if (!sv || !r || !r->d_rgb) return set_error(LODGS_E_INVALID, "lodgs_server_submit: null argument");
  if (!lodgs::camera_ok(&r->cam)) return set_error(LODGS_E_INVALID, "lodgs_server_submit: bad camera");
  if (!std::isfinite(r->tau) || r->tau < 0.0f) return set_error(LODGS_E_INVALID, "lodgs_server_submit: bad tau");
  const int cls = find_class(sv, r->cam.width, r->cam.height);
  if (cls < 0) return set_error(LODGS_E_INVALID, "lodgs_server_submit: image size is not one of the server's classes");
  Job j{};
  j.ticket = sv->next_ticket++;
  j.user = r->user;
  j.cam = r->cam;
  j.tau = r->tau;
  j.d_rgb = r->d_rgb;
  j.size_class = cls;
  j.attempts = 0;
  j.need_sel = sv->caps.max_selected;
  j.need_inst = sv->caps.max_instances;
  j.t_submit = now_s();
  sv->queue.push_back(j);
  if (ticket) *ticket = j.ticket;
  return pump(sv);
}

int lodgs_server_poll(lodgs_server* sv, lodgs_completion* out, int32_t max, int32_t* n) {
  if (!sv || !n || max < 0 || (max > 0 && !out)) return set_error(LODGS_E_INVALID, "lodgs_server_poll: bad argument");
  *n = 0;
  for (Slot* s : sv->slots) {
    if (!s->busy) continue;
    const hipError_t q = hipEventQuery(s->ev);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return hip_fail(q, "lodgs_server_poll: event");
    const volatile Published* hp = s->h_pub;
    Published p;
    p.status = hp->status;
    p.n_selected = hp->n_selected;
    p.n_drawn = hp->n_drawn;
    p.pad = 0;
    p.n_instances = hp->n_instances;
    s->busy = false;
    Job j = s->job;
    if (p.status == LODGS_E_CAPACITY) {
      if (j.attempts >= kMaxAttempts) {
        complete(sv, j, LODGS_E_CAPACITY, &p);
        continue;
      }
      // the counts it reported (a cut-short selection under-reports its
      // instances; a further attempt then grows those)
      j.need_sel = std::max(j.need_sel, (int64_t)p.n_selected + p.n_selected / 4 + 1024);
      j.need_inst = std::max(j.need_inst, p.n_instances + p.n_instances / 4 + 1024);
      if (j.need_sel > (int64_t)INT32_MAX / 16) j.need_sel = (int64_t)INT32_MAX / 16;
      if (j.need_inst > (int64_t)INT32_MAX - 1) j.need_inst = (int64_t)INT32_MAX - 1;
      ++sv->n_retries;
      sv->queue.push_front(j);
      continue;
    }
    complete(sv, j, p.status, &p);
  }
  const int rc = pump(sv);
  while (*n < max && !sv->done.empty()) {
    out[(*n)++] = sv->done.front();
    sv->done.pop_front();
  }
  return rc;
}

int lodgs_server_stats_read(const lodgs_server* sv, lodgs_server_stats* out) {
  if (!sv || !out) return set_error(LODGS_E_INVALID, "lodgs_server_stats_read: null argument");
  lodgs_server_stats i{};
  i.slots = (int32_t)sv->slots.size();
  for (const Slot* s : sv->slots) {
    i.busy += s->busy ? 1 : 0;
    i.slot_bytes += (int64_t)s->bytes;
  }
  i.queued = (int32_t)sv->queue.size();
  i.unpolled = (int32_t)sv->done.size();
  i.base_slot_bytes = (int64_t)slot_bytes(sv, sv->caps.max_selected, sv->caps.max_instances);
  i.retries = sv->n_retries;
  i.rejected = sv->n_rejected;
  i.evicted = sv->n_evicted;
  *out = i;
  return LODGS_OK;
}

}  // extern "C"
