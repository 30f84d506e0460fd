// Host-side state of scenes and frames, and the per-stage launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "lodgs.h"
#include "lodgs_dev.h"
#include "lodgs_error.h"
#include "lodgs_prims.h"

#include <vector>

// Device pointers of a scene, passed to kernels by value.
struct SceneDev {
  int64_t n_nodes;
  int32_t n_upper, n_spt, sh_degree, n_coef;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh;
  const float* r_min;
  const float* r_max;
  const float* rho;
  const int32_t* upper_parent;
  const int32_t* spt_begin;
  const int32_t* spt_parent;
  // Ancestor table of the upper hierarchy (library-owned, built at scene
  // creation): row d (d < anc_depth) holds the d-th upper ancestor (the
  // parent first) of every upper node e and SPT root n_upper + j, -1 past the
  // root; nullptr when the hierarchy is deeper than kMaxAncDepth.
  const int32_t* anc;
  int32_t anc_depth;
  // Radius of each SPT about its root's mean (library-owned, built at scene
  // creation; the CONSERVATIVE cut).
  const float* spt_radius;
  // Whole hierarchy for the comparator cuts (borrowed; nullptr when not
  // attached): parent and two children per layout position, and the number of
  // levels.
  const int32_t* parent;
  const int2* child;
  int32_t height;
};

// SPT-cut cache state handed to the cut kernels (cached == nullptr: no cache).
struct CacheDev {
  const uint8_t* cached;  // [n_spt] entry present
  const float* dc;        // [n_spt] cached root distance
  const float* Xc;        // [n_spt] cached X
  float d_min, d_max;
  uint8_t* vstate;        // [n_spt] this view: 0 not visible, 1 hit, 2 loaded
  float* dcur;            // [n_spt] this view's root distance
  uint32_t* spt_sel;      // [n_spt] this view's selected nodes per SPT
};

// Pruning statistics handed to the projection backward (last == nullptr: off).
struct ContribStats {
  const int32_t* contrib;    // per selection position
  int32_t* last;             // node-indexed
  int32_t* count;            // node-indexed (optional)
  const int32_t* iteration;  // device word
};

// State of an SPT-cut cache (lodgs_cache.hip); per SPT unless noted.
struct lodgs_cut_cache {
  const lodgs_scene* scene;
  lodgs_cut_cache_params prm;
  int64_t iteration;
  uint8_t* cached;
  float* dc;
  float* Xc;
  uint32_t* size;
  uint32_t* last_use;
  uint8_t* vstate;
  float* dcur;
  uint32_t* spt_sel;
  uint32_t* keys[2];
  uint32_t* vals[2];
  uint32_t* prefix;
  unsigned long long* counters;  // hits, loads, evictions, cached SPTs, cached nodes
  int32_t* total;                // node count of the entries before the drop
};

struct lodgs_scene {
  SceneDev dev;
  int32_t* anc_owned;
  float* radius_owned;
};

namespace lodgs {
constexpr int32_t kMaxAncDepth = 64;
constexpr int kTileClasses = 128;  // blend tile-order classes (quarter octaves of the instance count)
// Builds the ancestor table (synchronous; scene creation only).
int build_ancestor_table(lodgs_scene* s);
int build_spt_radius(lodgs_scene* s);
}  // namespace lodgs

// Device counters of a frame (one struct in device memory).
struct FrameCounters {
  int32_t status;
  int32_t n_selected;
  int32_t n_upper_selected;
  int32_t n_spt_visible;
  int32_t sum_high;
  int32_t n_render;      // min(count, max_selected) of the last render
  int32_t n_drawn;
  int32_t n_instances;   // full count
  int32_t n_inst_clamped;
  int32_t n_bit_words;   // constant: words of the comparator cuts' node bitmask
  int32_t upper_plus_high;
  int32_t spt_count;     // constant n_spt
  int32_t n_chunks;      // SPT candidate chunks of the last select
  int32_t seg_total;     // compaction segments of the last select
  int32_t n_long;        // drawn splats with more than kLongSegment instances
  int32_t pad;
};

struct lodgs_frame {
  const lodgs_scene* scene;
  lodgs_frame_caps caps;
  // device workspace
  FrameCounters* ctr;
  uint32_t* block_sums;   // kScanGrid + 1
  uint32_t* sort_table;   // 256 * kSortGrid
  uint32_t* sort_below;   // 256 * kSortGrid
  // select
  uint8_t* upper_sel;     // [n_upper]
  uint8_t* upper_test;    // [n_upper] bit 0 culled, bit 1 fine enough
  int32_t* spt_high;      // [n_spt]
  float* spt_X;           // [n_spt]
  uint32_t* spt_off;      // [n_spt]
  uint32_t* seg;          // [ceil(n_upper/64) + n_spt + n_nodes/512 + 1]
  uint32_t* chunk_owner;  // [n_spt + n_nodes/512 + 1] SPT of each candidate chunk
  // comparator cuts (allocated when the scene has its hierarchy attached)
  uint32_t* cut_bits;     // [n_bit_words] one bit per node, selected
  int32_t* frontier[2];   // [max_selected] BFS frontiers (ping-pong)
  int32_t* level_count;   // [cut_height + 1] BFS frontier lengths
  int32_t cut_height;     // the scene's height when the frame was created
  // render
  lodgs::Splat* splats;   // [max_selected]
  uint32_t* depth_key;    // [max_selected]
  uint32_t* depth_key2;
  uint32_t* order;        // [max_selected]
  uint32_t* order2;
  uint32_t* tiles;        // [max_selected]
  uint32_t* inst_off;     // [max_selected] instance offsets of the drawn splats in depth order
  uint32_t* drawn_list;   // [max_selected] selection positions of the drawn splats (selection order)
  ushort4* rect;          // [max_selected]
  uint32_t* ikey;         // [max_instances]
  uint32_t* ival;
  uint32_t* ikey2;
  uint32_t* ival2;
  uint2* inst_info;       // [max_instances] (selection position of the splat, block mask) (emission order),
                          // then a ping-pong buffer of the tile sort's payload
  float* inst_grad;       // [max_instances][kPartial] per-instance partials (emission order)
  uint32_t* inst_event;   // [max_instances] forward events, byte q for quarter q's 4x4 blocks (tile order)
  uint2* info_k;          // [max_instances] the other ping-pong buffer of that payload
  uint4* rank_info;       // [max_selected][2] per depth rank: (splat, 0, rect x0|x1<<16, y0|y1<<16),
                          // (mean x hi, lo, y hi, lo); written with the splat's first instance
  double* grad2d;         // [max_selected][9] per-drawn-splat 2D sums (selection position)
  float* dcol;            // [max_selected][kColorRec] colour backward record of each drawn splat (selection
                          // position): d colour / d view direction (9), unit view direction (3), 1 / distance,
                          // clamp bits, 2 unused
  uint32_t* long_list;    // [max_selected] depth ranks of the splats with many instances
  uint2* ranges;          // [max tiles]
  uint32_t* tile_order;   // [max tiles] tiles, heaviest first
  float spt_scale;        // LoD noise factor on the distances to SPT roots (lodgs_frame_set_lod_noise)
  lodgs::ViewConst* d_view_sel;  // view constants of the last lod_select (device)
  lodgs::ViewConst* d_view_ren;  // view constants of the last render (device)
  // state of the last render
  bool rendered;
  bool partials_ready;  // a LODGS_BWD_PARTIALS pass ran since the last render
  int partials_np;      // the values per instance partial of that pass
  const int32_t* r_idx;
  const int32_t* r_count;
  const float* r_rgb;
  float bg[3];
  lodgs::ViewConst view;
  const uint32_t* sorted_ival;  // the buffer holding the final instance order
  const uint32_t* sorted_ikey;
  const uint2* sorted_info;     // the (splat, block mask) words in tile order (inst_info or info_k)
  const uint32_t* sorted_order;  // selection positions of the drawn splats in depth order
  // timing mode: one (stage, start, end) event pair per stage and call
  bool timing;
  struct TimedStage {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<TimedStage> timed;
  int open_stage;
  hipEvent_t open_event;
  unsigned long long* work;  // [2] evaluation / contribution counters (device)
  // rendering from gathered parameter rows (lodgs_render_rows)
  bool rows_mode;            // the last render read rows_dev, with node i at row i
  SceneDev rows_dev;         // the scene's view with the parameter pointers on the rows
  int32_t* iota;             // [max_selected] i at i
  float* max_grad2d;         // [n_nodes] densification statistic raised by each backward (borrowed; optional)
  int32_t* contrib;          // [max_selected] contributing pixels of each drawn splat (selection position)
  int32_t* last_contrib;     // [n_nodes] pruning statistic: iteration of the last contribution (borrowed; optional)
  int32_t* contrib_count;    // [n_nodes] contributing pixels, accumulated (borrowed; optional)
  const int32_t* contrib_iteration;  // the iteration stamped into last_contrib (borrowed device word)
  int blend_px_fwd;          // pixels per lane of the forward blend (1, 2 or 4)
  int blend_px_bwd;          // pixels per lane of the blend backward (1, 2 or 4)
};

namespace lodgs {

// A drawn splat with more instances than this has its instance partials
// summed by a whole workgroup in the backward (listed by the duplication).
constexpr uint32_t kLongSegment = 32;
// The wave's list of batch slots j < m whose mask bits meet `want` (every
// slot j < m if ALL), in slot order, written to list; returns its length
// (wave-uniform).  A blend wave replays only these: for the others its result
// is known.
template <int NT, bool ALL>
__device__ __forceinline__ int wave_hit_list(int m, uint32_t want, const uint32_t* mask, uint8_t* list) {
  static_assert(NT % 64 == 0 && NT <= 256, "whole waves, byte slot indices");
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  int nh = 0;
#pragma unroll
  for (int c = 0; c < NT / 64; ++c) {
    const int j = c * 64 + lane;
    const bool h = j < m && (ALL || (mask[j] & want) != 0u);
    const uint64_t hb = __ballot(h);
    if (h) list[nh + __popcll(hb & lt)] = (uint8_t)j;
    nh += __popcll(hb);
  }
  return nh;
}

// Per-instance partial of the blend backward: sum w, sum w e (2), sum w e e^T
// (3) about the tile centre, dL/do, dL/dRGB (3), and (only while the pruning
// statistic is attached) contributing pixels: at most kPartial floats.
constexpr int kPartial = 11;

// Floats of the colour backward's per-splat record (written by the forward).
constexpr int kColorRec = 16;

// Writes the per-view constants to the frame's device slot (one thread): the
// kernels of a stage read them from there, so a captured graph is replayed
// for another camera by updating this one node's argument.  The same thread
// starts the stage's counters: kViewSelect clears the select counters,
// kViewRender sets n_render = clamp(*d_count, 0, cap) and clears n_drawn.
constexpr int kViewOnly = 0, kViewSelect = 1, kViewRender = 2;
void launch_set_view(const ViewConst& v, ViewConst* dst, FrameCounters* ctr, int mode, const int32_t* d_count,
                     int64_t cap, hipStream_t st);

int hip_fail(hipError_t e, const char* what);

// A camera the kernels can take: positive sizes up to 16384, finite values,
// positive focal lengths and near plane.
bool camera_ok(const lodgs_camera* c);

// Pixels per lane of the forward blend and the blend backward (1), or
// LODGS_BLEND_PX_FWD / LODGS_BLEND_PX_BWD (1, 2 or 4) when set in the
// environment (a tuning knob: images are identical, gradients equal up to the
// order of their sums).
int blend_pixels_per_lane(bool backward);

// Timing mode: brackets a stage with events on the stream (no-op otherwise).
void stage_begin(lodgs_frame* f, int stage, hipStream_t st);
void stage_end(lodgs_frame* f, hipStream_t st);

// Stage launchers (all stream-ordered, no host synchronisation).
void launch_select(lodgs_frame* f, const ViewConst& v, uint32_t flags, int32_t* d_idx, int64_t capacity,
                   int32_t* d_count, hipStream_t st, const CacheDev* cache = nullptr);
// The parameters the last render read: the scene's, or the gathered rows.
inline const SceneDev& render_params(const lodgs_frame* f) { return f->rows_mode ? f->rows_dev : f->scene->dev; }
// lod_select through an SPT-cut cache (arguments validated by the caller).
int cache_select(lodgs_frame* f, lodgs_cut_cache* c, const ViewConst& v, uint32_t flags, int32_t* d_idx,
                 int64_t capacity, int32_t* d_count, hipStream_t st);
// The comparator cuts (LODGS_CUT_BFS / LODGS_CUT_PARALLEL in flags).
void launch_select_full(lodgs_frame* f, const ViewConst& v, uint32_t flags, int32_t* d_idx, int64_t capacity,
                        int32_t* d_count, hipStream_t st);
// Words of the node bitmask: whole 64-node waves.
inline int64_t cut_bit_words(int64_t n_nodes) { return 2 * ((n_nodes + 63) / 64); }
// Position of the target image among the arguments of the L1 loss kernel
// (the function of a captured kernel node) and its argument count, or -1.
int l1_target_arg(const void* func, int* n_args);
void launch_l1_loss(const float* img, const float* target, int64_t n, float* grad, float* loss, hipStream_t st);
// Replays a captured view for cam and tau on st, writing the image to d_rgb
// (the captured image when null).
int graph_launch(lodgs_graph* g, const lodgs_camera* cam, float tau, float* d_rgb, hipStream_t st);
// Position of the output image among the arguments of a forward blend kernel
// (the function of a captured kernel node) and its argument count in
// *n_args, or -1 when func is not one: a captured view is pointed at another
// image by updating that one argument.
int blend_output_arg(const void* func, int* n_args);
void launch_render(lodgs_frame* f, const int32_t* d_idx, const int32_t* d_count, const ViewConst& v,
                   const float bg[3], float* d_rgb, hipStream_t st);
void launch_backward(lodgs_frame* f, const float* d_dL, const lodgs_grads* sel, const lodgs_grads* nodes,
                     uint32_t phases, hipStream_t st);

}  // namespace lodgs

namespace lodgs {

// Every device array of a frame with its element count, in allocation order:
// fn(pointer member, count).  lodgs_frame_create allocates through it and
// frame_bytes sums it, so the two cannot disagree.
template <class Fn>
void frame_arrays(lodgs_frame* f, const SceneDev& S, const lodgs_frame_caps& caps, Fn&& fn) {
  const size_t ns = (size_t)caps.max_selected, ni = (size_t)caps.max_instances;
  const size_t nt = (size_t)((caps.max_width + 15) / 16) * ((caps.max_height + 15) / 16);
  fn(f->ctr, 1);
  fn(f->block_sums, kScanGrid + 1);
  fn(f->sort_table, (size_t)256 * kSortGrid);
  fn(f->sort_below, (size_t)256 * kSortGrid);
  fn(f->upper_sel, (size_t)S.n_upper);
  fn(f->upper_test, (size_t)S.n_upper);
  fn(f->spt_high, (size_t)S.n_spt);
  fn(f->spt_X, (size_t)S.n_spt);
  fn(f->spt_off, (size_t)S.n_spt);
  fn(f->seg, (size_t)(S.n_upper + 63) / 64 + (size_t)S.n_spt + (size_t)S.n_nodes / 512 + 1);
  fn(f->chunk_owner, (size_t)S.n_spt + (size_t)S.n_nodes / 512 + 1);
  fn(f->splats, ns);
  fn(f->depth_key, ns);
  fn(f->depth_key2, ns);
  fn(f->order, ns);
  fn(f->order2, ns);
  fn(f->tiles, ns);
  fn(f->inst_off, ns);
  fn(f->drawn_list, ns);
  fn(f->rect, ns);
  fn(f->ikey, ni);
  fn(f->ival, ni);
  fn(f->ikey2, ni);
  fn(f->ival2, ni);
  fn(f->inst_info, ni);
  fn(f->inst_grad, (size_t)kPartial * ni);
  fn(f->inst_event, ni);
  fn(f->info_k, ni);
  fn(f->rank_info, 2 * ns);
  fn(f->grad2d, 9 * ns);
  fn(f->contrib, ns);
  fn(f->dcol, (size_t)kColorRec * ns);
  fn(f->long_list, ns);
  fn(f->ranges, nt);
  fn(f->tile_order, nt);
  fn(f->work, 2);
  fn(f->d_view_sel, 1);
  fn(f->d_view_ren, 1);
  fn(f->iota, ns);
  if (S.parent) {
    fn(f->cut_bits, (size_t)cut_bit_words(S.n_nodes));
    fn(f->frontier[0], ns);
    fn(f->frontier[1], ns);
    fn(f->level_count, (size_t)S.height + 1);
  }
}

// Device bytes lodgs_frame_create allocates for these capacities.
size_t frame_bytes(const lodgs_scene* scene, const lodgs_frame_caps& caps);

}  // namespace lodgs
