/*
 * lodgs.h -- C ABI of the MI355X LoD-select + Gaussian-splat library
 * (liblodgs.so).  The calls follow the paper's statement of the per-view
 * problem ("A LoD of Gaussians", arXiv 2507.01110, Sec. 4 and Alg. 3): cut the
 * hierarchy for a camera into a set of Gaussian indices, render that set, and
 * differentiate the rendering.
 *
 * Conventions
 *  - Every pointer named d_* is device memory on the current HIP device; all
 *    others are host memory.  The caller owns every array it passes in; the
 *    library owns only the opaque handles and their internal workspaces.
 *  - Calls that take a stream are asynchronous and stream-ordered (stream may
 *    be NULL for the default stream).  Nothing blocks except
 *    lodgs_frame_stats and the host-only builder.
 *  - Every call returns a status code (0 on success, one of LODGS_E_* on
 *    failure); lodgs_last_error() returns a thread-local message for the last
 *    failure.  No exception crosses the ABI.
 *  - Device errors found while a kernel runs (a capacity overflow) are
 *    recorded in the frame and reported by lodgs_frame_stats; the outputs of
 *    the call that overflowed are then incomplete.
 *  - Node parameters are the raw ones, FP32, indexed by layout position:
 *    means [n][3], log_scales [n][3], quats [n][4] as (w, x, y, z), not
 *    necessarily normalised, opacity_logits [n], sh [n][(deg+1)^2][3].
 *  - Images are float32 [height][width][3], row-major.
 */
#ifndef LODGS_H_
#define LODGS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LODGS_OK 0
#define LODGS_E_INVALID (-1)  /* bad argument                                     */
#define LODGS_E_CAPACITY (-2) /* an output or workspace is too small               */
#define LODGS_E_HIP (-3)      /* a HIP runtime call failed                         */
#define LODGS_E_OOM (-4)      /* device or host allocation failed                  */
#define LODGS_E_STATE (-5)    /* call out of order (backward without a forward)    */

/* lod_select flags */
#define LODGS_CULL 1u         /* frustum-cull upper nodes and SPT roots (Sec. 4.3) */
#define LODGS_CONSERVATIVE 2u /* cut each SPT at X = max(0, d - R) tau / fx, R the SPT's
                                 radius about its root (the conservative distance of
                                 Sec. 4.1): no member is cut coarser than its own
                                 distance allows.  Default: X = d tau / fx (Alg. 2). */
/* Comparator cuts over the whole hierarchy (Sec. 4.3, the two approaches the
 * HSPT replaces); both need lodgs_scene_set_hierarchy and exclude each other
 * and LODGS_CONSERVATIVE.  A node is fine at its own distance when
 * r_min <= X = d tau / fx (leaves, r_min = 0, always are). */
#define LODGS_CUT_BFS 4u      /* descent from the root: a reached node is dropped with its
                                 subtree when culled (if LODGS_CULL), selected when fine,
                                 else both children are reached */
#define LODGS_CUT_PARALLEL 8u /* the per-node test of Eq. 5: selected when fine and its
                                 parent (if any) is not; with LODGS_CULL a node whose own
                                 sphere is culled is dropped.  A proper cut only when
                                 fineness passes from parents to children. */

typedef void* lodgs_stream; /* a hipStream_t */

/* Pinhole camera.  x_cam = R x_world + t with R row-major and OpenCV axes
 * (x right, y down, z forward); pos is the camera centre in world space (used
 * for LoD distances and SH view directions); (cx, cy) the principal point in
 * pixels; pixels are sampled at their centres (x + 0.5, y + 0.5); splats with
 * camera depth <= z_near are not drawn and spheres entirely in front of the
 * near plane are culled. */
typedef struct lodgs_camera {
  float R[9];
  float t[3];
  float pos[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float z_near;
} lodgs_camera;

/* ---------------------------------------------------------------- HSPT build
 * Hierarchical SPT construction (Sec. 4.3 "The Hierarchical SPT
 * Datastructure"; Sec. 4.1 for the SPT arrays).  Host only, OpenMP.
 *
 * Input: a binary hierarchy of n_nodes nodes given by left/right child ids (-1
 * for leaves) and root, the nodes' FP32 log-scales [n_nodes][3], and the
 * volume threshold as log(size) (double).  The BFS split puts node i in the
 * cut set when it is a leaf or when ((double)ls0 + (double)ls1) + (double)ls2
 * < log_size; cut nodes root SPTs, nodes above them form the upper hierarchy.
 *
 * Outputs (caller-allocated host arrays; sizes in brackets):
 *   perm [n_nodes]          layout position -> tree node id.  Layout: upper
 *                           nodes in left-first DFS preorder, then one segment
 *                           per SPT in the order that DFS meets the SPT roots;
 *                           inside a segment nodes are sorted by r_max
 *                           descending, then r_min descending, then tree id.
 *   r_min, r_max [n_nodes]  in layout order.  Size metric g = sqrt(s1 s2 + s1 s3
 *                           + s2 s3) (Eq. 6's surface measure), evaluated in FP64
 *                           and rounded once to FP32.  Upper nodes: r_min = g,
 *                           r_max = +inf.  SPT members: r_min = g (0 for leaves),
 *                           r_max = +inf for the SPT root, else the minimum of g
 *                           over the node's ancestors inside its SPT.
 *   rho [n_nodes]           3 * max_j s_j (the cull-sphere radius), layout order.
 *   upper_parent [n_nodes]  first n_upper entries: layout position of the parent
 *                           (-1 for the root).
 *   spt_begin [n_nodes + 1] first n_spt + 1 entries: segment boundaries.
 *   spt_parent [n_nodes]    first n_spt entries: layout position of the upper
 *                           parent of each SPT root (-1 if it is the hierarchy
 *                           root).
 *   n_upper, n_spt          counts.
 * Errors: LODGS_E_INVALID for a malformed tree (cycle, missing child, n_nodes >
 * 2^31 - 2), LODGS_E_OOM if host memory runs out. */
int lodgs_hspt_build(int64_t n_nodes, const int32_t* left, const int32_t* right, int32_t root,
                     const float* log_scales, double log_size, int32_t* perm, float* r_min, float* r_max,
                     float* rho, int32_t* upper_parent, int32_t* spt_begin, int32_t* spt_parent,
                     int32_t* n_upper, int32_t* n_spt);

/* ---------------------------------------------------------------- scene
 * A scene borrows device arrays in layout order (the outputs of
 * lodgs_hspt_build, uploaded, plus the node parameters permuted by perm).  The
 * arrays must outlive the scene handle.  rho is indexed by layout position.
 * sh_degree is 0..3.  d_quats and d_sh must be 16-byte aligned (rows are read
 * as float4s), else LODGS_E_INVALID. */
typedef struct lodgs_scene_desc {
  int64_t n_nodes;
  int32_t n_upper, n_spt, sh_degree;
  const float* d_means;
  const float* d_log_scales;
  const float* d_quats;
  const float* d_opacity_logits;
  const float* d_sh;
  const float* d_r_min;
  const float* d_r_max;
  const float* d_rho;
  const int32_t* d_upper_parent; /* [n_upper] */
  const int32_t* d_spt_begin;    /* [n_spt + 1] */
  const int32_t* d_spt_parent;   /* [n_spt] */
} lodgs_scene_desc;

typedef struct lodgs_scene lodgs_scene;

/* Validates sizes (host-side checks only) and stores the descriptor. */
int lodgs_scene_create(const lodgs_scene_desc* desc, lodgs_scene** out);
void lodgs_scene_destroy(lodgs_scene* scene);

/* Attaches the whole binary hierarchy for the comparator cuts LODGS_CUT_BFS
 * and LODGS_CUT_PARALLEL (Sec. 4.3: the BFS cut, and the parallel cut of
 * Eq. 5).  Borrowed device arrays in layout order (they must outlive the
 * scene): d_parent [n_nodes] the layout position of each node's parent, -1
 * for the root, which must be position 0; d_child [n_nodes][2] the layout
 * positions of the two children, (-1, -1) for a leaf.  height = the number of
 * levels (1 for a lone root), at most 4096: the BFS runs one pass per level.
 * Frames created after this call hold the comparators' workspace (a bit per
 * node and two frontier queues of max_selected entries) and run height BFS
 * passes, the height at their creation; a BFS that still has a frontier after
 * them records LODGS_E_INVALID in the frame's status.  Synchronous; checks
 * that position 0 is the root.  Errors: LODGS_E_INVALID (null array, height
 * out of range, position 0 has a parent). */
int lodgs_scene_set_hierarchy(lodgs_scene* scene, const int32_t* d_parent, const int32_t* d_child, int32_t height);

/* ---------------------------------------------------------------- frame
 * A frame owns the device workspace of one view in flight: the LoD-cut
 * scratch, the per-splat projections, the sorted instance lists, the tile
 * ranges and the 2D gradients.  Capacities bound the selected-node count, the
 * (splat, tile) instance count and the image size.  A frame is used by one
 * stream at a time; frames on different streams may overlap. */
typedef struct lodgs_frame_caps {
  int64_t max_selected;
  int64_t max_instances;
  int32_t max_width, max_height;
} lodgs_frame_caps;

typedef struct lodgs_frame lodgs_frame;

/* Errors: LODGS_E_INVALID for capacities out of range, LODGS_E_OOM when a
 * device allocation fails (everything the call allocated is freed first).
 * LODGS_FAIL_FRAME_ALLOC=k in the environment makes the k-th device
 * allocation of the call report out of memory (a test of that path). */
int lodgs_frame_create(const lodgs_scene* scene, const lodgs_frame_caps* caps, lodgs_frame** out);
void lodgs_frame_destroy(lodgs_frame* frame);

/* ---------------------------------------------------------------- calls
 * lod_select (Sec. 4.3, two-step HSPT cut; Eq. 4 for the SPTs; Alg. 2).
 * With X = d * tau / fx (the focal-normalised distance of the implementation
 * appendix; d = |mu - pos| in FP32):
 *   - an upper node is dropped with its subtree when culled (if LODGS_CULL),
 *     selected when r_min (= g) <= X at its own distance, else descended;
 *   - a reached SPT root that is not culled makes its SPT visible; the SPT is
 *     cut at the root's X: a binary search gives the prefix with r_max > X and
 *     every prefix node with r_min <= X is selected.
 * Writes the selected layout positions in ascending order to d_idx[0 ..
 * min(count, capacity)) and the full count to *d_count (device int32).  If
 * count > capacity the frame records LODGS_E_CAPACITY (see lodgs_frame_stats).
 * tau must be finite and >= 0.  With LODGS_CUT_BFS or LODGS_CUT_PARALLEL the
 * comparator cut replaces the HSPT cut (same output contract; the frame must
 * have been created after lodgs_scene_set_hierarchy, else LODGS_E_STATE); a
 * BFS frontier longer than max_selected records LODGS_E_CAPACITY. */
int lodgs_lod_select(lodgs_frame* frame, const lodgs_camera* cam, float tau, uint32_t flags, int32_t* d_idx,
                     int64_t capacity, int32_t* d_count, lodgs_stream stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the HSPT cut of
 * lodgs_lod_select with no frame.  Its workspace (counters, view constants,
 * scan sums, 2 bytes per upper node, 12 per SPT and the compaction segments,
 * about 30 bytes per 512 nodes) lives in one static device array of
 * LODGS_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; the call
 * allocates nothing.  Same arguments and output contract as lodgs_lod_select
 * (selected positions ascending in d_idx, the full count in *d_count, a
 * count above capacity meaning the list was cut short), with the scene in
 * place of the frame and flags limited to LODGS_CULL | LODGS_CONSERVATIVE
 * (else LODGS_E_INVALID).  A scene whose workspace exceeds the array returns
 * LODGS_E_CAPACITY before any launch.  Every call on one GPU shares the
 * array, which keeps the last call's contents (each call resets the counters
 * it reads): calls that overlap on one GPU race, so keep them stream-ordered. */
#define LODGS_NOALLOC_SCRATCH_BYTES (32u << 20)
int lodgs_lod_select_noalloc(const lodgs_scene* scene, const lodgs_camera* cam, float tau, uint32_t flags,
                             int32_t* d_idx, int64_t capacity, int32_t* d_count, lodgs_stream stream);

/* ---------------------------------------------------------------- SPT-cut cache
 * The GPU cache of SPT cuts (Sec. 4.4 "Caching on the GPU", Eq. 7, and the
 * training loop of Alg. 3).  Here the scene is resident, so a cache entry
 * holds what decides the cut, the root distance d_c and the X_c an SPT was
 * cut at, and its node count; a hit reuses the cached cut, which makes the
 * level of detail depend on the cache state as the paper describes.
 * Iteration t = 1, 2, ... of lodgs_lod_select_cached on a cache: when
 * flush_every > 0 and t is a multiple of it, every entry is dropped first.  A
 * visible SPT (reached and not culled) at root distance d (FP32, as the cut
 * computes it) with an entry is a hit when d_min <= r * r <= d_max, r = d / d_c
 * in FP32 (Alg. 3 compares squared ratios), and is cut at X_c; otherwise it
 * is loaded: cut at X = d tau / fx like lodgs_lod_select, then entered with
 * (d, X) and its number of selected nodes.  Every visible SPT's last use
 * becomes t.  Then, oldest last use first (ties by SPT index), entries are
 * dropped while the node counts of those left exceed max_nodes (the LRU
 * write-back).  Flags: LODGS_CULL only.  One cache per scene, which must
 * outlive it; calls on one cache must be stream-ordered (they use the
 * frame's scratch and the cache's state in order). */
typedef struct lodgs_cut_cache_params {
  int64_t max_nodes;   /* budget of cached SPT-cut nodes, >= 0 */
  float d_min, d_max;  /* the window of squared distance ratios, 0 <= d_min <= d_max */
  int32_t flush_every; /* drop everything at multiples of this iteration count (0: never) */
} lodgs_cut_cache_params;

typedef struct lodgs_cut_cache lodgs_cut_cache;

typedef struct lodgs_cut_cache_stats {
  int64_t iterations, hits, loads, evictions; /* totals since creation */
  int64_t cached_spts, cached_nodes;          /* entries now */
} lodgs_cut_cache_stats;

int lodgs_cut_cache_create(const lodgs_scene* scene, const lodgs_cut_cache_params* params, lodgs_cut_cache** out);
void lodgs_cut_cache_destroy(lodgs_cut_cache* cache);
/* lodgs_lod_select through the cache (same output contract).  The frame must
 * belong to the cache's scene. */
int lodgs_lod_select_cached(lodgs_frame* frame, lodgs_cut_cache* cache, const lodgs_camera* cam, float tau,
                            uint32_t flags, int32_t* d_idx, int64_t capacity, int32_t* d_count, lodgs_stream stream);
/* Blocks on the stream. */
int lodgs_cut_cache_stats_read(lodgs_cut_cache* cache, lodgs_cut_cache_stats* out, lodgs_stream stream);

/* render (Sec. 3, Eq. 1 front-to-back compositing with Eq. 2 alpha over the
 * EWA projection; the rasterizer conventions the paper reuses): projects the
 * d_idx[0 .. *d_count) nodes (count clamped to the frame's max_selected),
 * evaluates SH colour, sorts (tile, depth) instances over 16x16 tiles and
 * blends front to back into d_rgb [height][width][3] with background bg (3
 * floats, host).  alpha = min(0.99, o exp(power)); alpha < 1/255 is skipped;
 * blending stops before the transmittance would fall below 1e-4.  The frame
 * keeps d_idx, d_count and d_rgb for render_backward, which reads them: they
 * must stay unchanged until then. */
int lodgs_render(lodgs_frame* frame, const int32_t* d_idx, const int32_t* d_count, const lodgs_camera* cam,
                 const float bg[3], float* d_rgb, lodgs_stream stream);

/* Gradient destinations, one array per parameter group, same layouts as the
 * parameters.  Any member may be NULL to skip that group.  (The same struct
 * carries parameter arrays where a call says so.) */
typedef struct lodgs_grads {
  float* d_means;
  float* d_log_scales;
  float* d_quats;
  float* d_opacity_logits;
  float* d_sh;
} lodgs_grads;

/* ---------------------------------------------------------------- out-of-core parameters
 * Rendering a cut whose parameters live in host memory (Sec. 4.4: the cut's
 * Gaussians are loaded from RAM).  lodgs_gather_rows copies, with one kernel
 * reading host memory over the host link, the parameter rows of the selected
 * nodes: row k of every group of rows receives node d_idx[k]'s parameters,
 * k < min(*d_count, capacity).  host: the five parameter groups in layout
 * order (the scene's layouts; sh of sh_degree), in pinned host memory from
 * hipHostMalloc (or torch's pin_memory); rows: device arrays of capacity rows
 * each.  Rows of 4 or 12 / 48 floats move as float4s: all arrays 16-byte
 * aligned.  Errors: LODGS_E_INVALID (a NULL member, a host array that is not
 * pinned host memory, a rows array that is not device memory, misalignment,
 * sh_degree outside 0..3). */
int lodgs_gather_rows(const lodgs_grads* host, const lodgs_grads* rows, int32_t sh_degree, const int32_t* d_idx,
                      const int32_t* d_count, int64_t capacity, int64_t n_nodes, lodgs_stream stream);

/* A device pool of the rows of cached SPT cuts (Sec. 4.4 "Caching on the
 * GPU": a cached cut's Gaussians stay in VRAM; Alg. 3: load from RAM, cache
 * insert, write-back of evicted entries), over an SPT-cut cache and a host
 * store in pinned memory (the layout of lodgs_gather_rows).  The upper
 * hierarchy's rows are kept resident.  lodgs_gather_rows_pooled, called after
 * a lodgs_lod_select_cached on the pool's cache with that call's d_idx and
 * d_count, first gives back the slots of every entry that the select dropped,
 * and those of the nodes that the new cut of an entry it cut afresh (a miss of
 * the ratio test) no longer holds, writing back to host memory the rows that
 * lodgs_row_pool_store changed; then every selected node of a cached, visible
 * entry that has no slot takes one, filled from host memory; then writes row
 * k of rows (k < min(*d_count, capacity)) for node d_idx[k] from the resident
 * upper rows, the pool, or host memory (a node without a slot): a cache hit
 * reads nothing over the host link, a re-cut entry only its new nodes.  The
 * selection marks carry a per-call 32-bit stamp; when it wraps the marks are
 * cleared with hipMemsetAsync, so this call is not for graph capture.
 * lodgs_row_pool_store writes trained rows back: to the pool
 * for pooled nodes (written to host memory when their entry leaves), to the
 * resident upper rows and host memory for upper nodes, to host memory
 * otherwise.  The pool's capacity (slots) must be at least the cache's
 * max_nodes, so an entry always finds its slots.  One pool per cache; calls
 * are stream-ordered after the select they follow.  Errors: LODGS_E_INVALID
 * for a null or unpinned host array, a wrong sh_degree or a capacity below
 * max_nodes; LODGS_E_OOM. */
typedef struct lodgs_row_pool lodgs_row_pool;
typedef struct lodgs_row_pool_stats {
  int64_t capacity;         /* slots                                            */
  int64_t pooled_rows;      /* slots in use                                     */
  int64_t host_rows;        /* rows of the last gather read from host memory    */
  int64_t inserted;         /* slots taken (and filled) by the last gather      */
  int64_t released;         /* slots given back by the last gather              */
  int64_t insert_failures;  /* nodes left without a slot (total; 0 by design)   */
  int64_t written_back;     /* changed rows written back on release (total)     */
} lodgs_row_pool_stats;

int lodgs_row_pool_create(lodgs_cut_cache* cache, const lodgs_grads* host, int32_t sh_degree, int64_t capacity,
                          lodgs_row_pool** out);
void lodgs_row_pool_destroy(lodgs_row_pool* pool);
int lodgs_gather_rows_pooled(lodgs_row_pool* pool, const int32_t* d_idx, const int32_t* d_count,
                             const lodgs_grads* rows, int64_t capacity, lodgs_stream stream);
int lodgs_row_pool_store(lodgs_row_pool* pool, const int32_t* d_idx, const int32_t* d_count, const lodgs_grads* rows,
                         int64_t capacity, lodgs_stream stream);
/* Writes every changed pooled row back to host memory now (the rows stay
 * pooled): at the end of training, or before lodgs_row_pool_destroy, which
 * drops the pool without writing anything back.  Stream-ordered. */
int lodgs_row_pool_write_back(lodgs_row_pool* pool, lodgs_stream stream);
/* Counters (blocks on the stream); with d_node_slot (device int32 [n_nodes])
 * not NULL, also copies each node's slot (-1: not pooled). */
int lodgs_row_pool_stats_read(lodgs_row_pool* pool, lodgs_row_pool_stats* out, int32_t* d_node_slot,
                              lodgs_stream stream);

/* lodgs_render with the parameters of the i-th rendered node taken from row
 * i of rows (as lodgs_gather_rows writes them) instead of the scene: the
 * image, the instances and the frame state equal those of lodgs_render on
 * the same cut.  rows must hold at least min(*d_count, max_selected) rows.
 * lodgs_render_backward after it takes sel only (rows-indexed gradients;
 * nodes must be NULL).  rows must stay unchanged until then. */
int lodgs_render_rows(lodgs_frame* frame, const lodgs_grads* rows, const int32_t* d_count, const lodgs_camera* cam,
                      const float bg[3], float* d_rgb, lodgs_stream stream);

/* render_backward: given dL/dimage (d_dL_drgb, [height][width][3]) for the
 * last render of this frame, computes the gradients of the raw parameters of
 * the rendered nodes.  Blending state is recomputed per tile (front to back,
 * using the final colour), nothing per pixel is stored by the forward.
 *   sel (optional):   written for positions i < count: gradient of node
 *                     d_idx[i] (zero for nodes that were not drawn);
 *   nodes (optional): accumulated (+=) into node-indexed arrays at d_idx[i].
 * The d_sh members must be 16-byte aligned (rows move as float4s).
 * Returns LODGS_E_STATE if the frame has not rendered, LODGS_E_INVALID for a
 * misaligned d_sh. */
int lodgs_render_backward(lodgs_frame* frame, const float* d_dL_drgb, const lodgs_grads* sel,
                          const lodgs_grads* nodes, lodgs_stream stream);

/* lodgs_render_backward in two halves, for callers that keep several views
 * in flight on several frames (Alg. 3 accumulating gradients over views):
 *   LODGS_BWD_PARTIALS: the blend backward and the per-splat 2D sums, which
 *                       write only this frame's state (d_dL_drgb needed;
 *                       sel and nodes ignored);
 *   LODGS_BWD_SCATTER:  the colour and projection backward into sel / nodes
 *                       and the attached node statistics (needs a PARTIALS
 *                       pass after the frame's last render; d_dL_drgb
 *                       ignored).
 * Both together equal lodgs_render_backward.  PARTIALS passes of different
 * frames may run concurrently on different streams; SCATTER passes that write
 * the same arrays must be ordered by the caller.  Errors: LODGS_E_INVALID for
 * an unknown phase bit or a missing d_dL_drgb, LODGS_E_STATE for a SCATTER
 * without its PARTIALS, and those of lodgs_render_backward. */
#define LODGS_BWD_PARTIALS 1u
#define LODGS_BWD_SCATTER 2u
int lodgs_render_backward_phases(lodgs_frame* frame, const float* d_dL_drgb, const lodgs_grads* sel,
                                 const lodgs_grads* nodes, uint32_t phases, lodgs_stream stream);

/* Counters of the last calls on this frame (blocks on the stream). */
typedef struct lodgs_stats {
  int32_t status;          /* LODGS_OK or LODGS_E_CAPACITY                  */
  int32_t n_selected;      /* full count of the last lod_select             */
  int32_t n_upper_selected;
  int32_t n_spt_visible;
  int64_t n_spt_candidates; /* sum over visible SPTs of the prefix length    */
  int32_t n_rendered;      /* nodes given to the last render                */
  int32_t n_drawn;         /* of which projected in front of z_near, on screen */
  int64_t n_instances;     /* (splat, tile) pairs of the last render        */
} lodgs_stats;

int lodgs_frame_stats(lodgs_frame* frame, lodgs_stats* out, lodgs_stream stream);

/* Copies the sorted instance list of the last render (blocks on the stream):
 * for k < min(n_instances, capacity), d_tile[k] = tile id (row-major over the
 * 16x16 tile grid) and d_pos[k] = position in d_idx of the splat, in blend
 * order (tile, FP32 depth bits, selection position).  *n_out (host) receives
 * the full instance count.  For parity tests and diagnostics. */
int lodgs_frame_read_instances(lodgs_frame* frame, int32_t* d_tile, int32_t* d_pos, int64_t capacity,
                               int64_t* n_out, lodgs_stream stream);

/* Clears the recorded device error of the frame. */
int lodgs_frame_clear_status(lodgs_frame* frame, lodgs_stream stream);

/* The varying level of detail of training (implementation appendix: the
 * distances to the SPT centres are multiplied by a random factor each
 * iteration, against overfitting Gaussians of one scale to views from one
 * distance): every later lodgs_lod_select and lodgs_lod_select_cached on this
 * frame, and every replay of a graph captured on it, multiplies the FP32
 * distance to each SPT root by factor before that SPT's cut (X = (d factor)
 * tau / fx; with LODGS_CONSERVATIVE, max(0, d factor - R) tau / fx) and
 * before the cut cache's ratio test, whose entries then hold that distance.
 * Upper-hierarchy nodes keep their own distance; the comparator cuts
 * (LODGS_CUT_BFS, LODGS_CUT_PARALLEL) have no SPTs and ignore it.  1 (the
 * default) is no noise.  factor must be finite and > 0 (else
 * LODGS_E_INVALID); the training loop draws 1 + 5 r^4, r ~ U(0, 1). */
int lodgs_frame_set_lod_noise(lodgs_frame* frame, float factor);

/* The densification criterion (Sec. 4.2: nodes are chosen for densification
 * by their largest screen-space gradient): with d_max_grad2d [n_nodes]
 * (device, node-indexed, borrowed) attached, every later
 * lodgs_render_backward on this frame raises d_max_grad2d[node] to the norm
 * of dL/d(projected mean) in pixels (FP64, rounded to FP32) of each drawn
 * node; NULL detaches it.  Not updated after lodgs_render_rows.  Frames that
 * share one array must not run backwards concurrently. */
int lodgs_frame_set_densify_stats(lodgs_frame* frame, float* d_max_grad2d);

/* The pruning statistic (appendix on densification details: the opacity of a
 * Gaussian that has not contributed for a number of iterations equal to
 * twice the training-set size is zeroed): with d_last attached, every later
 * lodgs_render_backward on this frame writes *d_iteration (a device int32 the
 * caller advances) into d_last[node] for each rendered node that contributed
 * to at least one pixel (composited with alpha >= 1/255 before its pixel
 * stopped, the forward's FP32 decisions), and, if d_count is not NULL, adds
 * that node's number of contributing pixels to d_count[node].  d_last and
 * d_count: node-indexed int32 device arrays (borrowed).  NULL d_last
 * detaches; d_iteration is required with it (else LODGS_E_INVALID).  Not
 * updated after lodgs_render_rows.  Frames that share the arrays must not
 * run backwards concurrently. */
int lodgs_frame_set_contrib_stats(lodgs_frame* frame, int32_t* d_last, int32_t* d_count, const int32_t* d_iteration);

/* ---------------------------------------------------------------- graphs
 * A forward view (lod_select + render) captured once into a HIP graph and
 * replayed for any camera of the same image size and any tau.  All counts
 * stay on the device, so the graph never needs the host between stages; a
 * replay updates only the two nodes that load the per-view constants.
 * Capture requires a non-default stream and a frame not in timing mode; the
 * graph reuses the frame, d_idx, d_count and d_rgb of the capture (they must
 * outlive it), so replays of one graph (or graphs of one frame) must not
 * overlap.  The serving loop keeps one frame, stream and graph set per slot. */
typedef struct lodgs_graph lodgs_graph;

int lodgs_graph_capture_view(lodgs_frame* frame, const lodgs_camera* cam, float tau, uint32_t flags,
                             int32_t* d_idx, int64_t capacity, int32_t* d_count, const float bg[3], float* d_rgb,
                             lodgs_stream stream, lodgs_graph** out);
/* Replays the graph for cam (same width and height as captured) and tau on
 * stream; LODGS_E_INVALID for another image size. */
int lodgs_graph_launch(lodgs_graph* graph, const lodgs_camera* cam, float tau, lodgs_stream stream);
void lodgs_graph_destroy(lodgs_graph* graph);
/* A training step captured into one graph: lod_select, render into d_rgb,
 * the L1 loss against d_target (d_dL receives dL/dimage, *d_loss the loss if
 * d_loss is not NULL) and render_backward into sel or nodes (one of them, or
 * neither; as lodgs_render_backward), the operations of Alg. 3's
 * render-and-optimise step without the optimizer.  Same rules as
 * lodgs_graph_capture_view; every buffer given here is reused by every
 * replay and must outlive the graph. */
int lodgs_graph_capture_step(lodgs_frame* frame, const lodgs_camera* cam, float tau, uint32_t flags,
                             int32_t* d_idx, int64_t capacity, int32_t* d_count, const float bg[3], float* d_rgb,
                             const float* d_target, float* d_dL, float* d_loss, const lodgs_grads* sel,
                             const lodgs_grads* nodes, lodgs_stream stream, lodgs_graph** out);
/* Replays a training-step graph for cam (the captured size), tau and the
 * target image d_target ([height][width][3], device). */
int lodgs_graph_launch_step(lodgs_graph* graph, const lodgs_camera* cam, float tau, const float* d_target,
                            lodgs_stream stream);

/* ---------------------------------------------------------------- serving
 * Continuous-batching render server, forward only (the renderer of Sec. 5
 * on the same LoD path: lodgs_lod_select then lodgs_render per request).
 * Requests of the declared image-size classes, any camera and any tau are
 * queued by lodgs_server_submit and admitted into slots as slots and memory
 * free up; each slot owns a frame, a stream and one captured view graph per
 * size class, so the requests of different slots overlap on the device.  The
 * scene and every per-request buffer stay on the device; the host only
 * queues, launches and polls events.
 * Admission: the largest idle slot whose capacities cover the request takes
 * it (a request's size shows only after its first run);
 * otherwise a new slot is made if fewer than max_slots exist and free HBM
 * (hipMemGetInfo) is at least the slot's bytes plus hbm_reserve; otherwise
 * the request waits.  A request whose selection or instance list overflows
 * its slot's capacities runs again, first in the queue, with the counts it
 * reported as its minimum capacities (a larger slot is made, evicting idle
 * slots too small for it when memory or the slot limit requires).  A request
 * that no slot can ever take (no slot busy, none large enough, none can be
 * made) completes with LODGS_E_CAPACITY: rejected, its image unwritten.
 * A server is driven by one host thread; it must be destroyed before the
 * scene.  Making a slot synchronises the null stream. */
#define LODGS_SERVER_MAX_SIZES 8
typedef struct lodgs_server_caps {
  int32_t n_sizes;                         /* image-size classes, 1..LODGS_SERVER_MAX_SIZES  */
  int32_t sizes[LODGS_SERVER_MAX_SIZES][2]; /* width, height of each class                   */
  int32_t max_slots;                       /* requests in flight at most, 1..64              */
  int64_t max_selected;                    /* capacities of a slot as first made             */
  int64_t max_instances;
  int64_t hbm_reserve;                     /* free HBM bytes a new slot must leave           */
  uint32_t flags;                          /* LODGS_CULL | LODGS_CONSERVATIVE                 */
  float bg[3];                             /* background colour                              */
} lodgs_server_caps;

typedef struct lodgs_request {
  lodgs_camera cam;  /* width x height must be one of the size classes       */
  float tau;         /* pixel threshold of the cut, finite, >= 0              */
  float* d_rgb;      /* caller's device image [height][width][3] FP32, written
                        by the time the request completes; owned by the caller,
                        who keeps it until then                               */
  uint64_t user;     /* returned in the completion                            */
} lodgs_request;

typedef struct lodgs_completion {
  uint64_t ticket;      /* lodgs_server_submit's ticket                        */
  uint64_t user;
  int32_t status;       /* LODGS_OK, or LODGS_E_CAPACITY: rejected             */
  int32_t attempts;     /* launches it took (1 + capacity retries)             */
  int32_t n_selected;   /* counts of its final launch                          */
  int32_t n_drawn;
  int64_t n_instances;
  double t_submit;      /* host monotonic clock, seconds: queued, first        */
  double t_admit;       /* launch of the final attempt, seen complete by a poll */
  double t_done;
} lodgs_completion;

typedef struct lodgs_server_stats {
  int32_t slots, busy, queued, unpolled;
  int64_t slot_bytes;       /* device bytes held by the slots                   */
  int64_t base_slot_bytes;  /* bytes of one slot at the first capacities        */
  int64_t retries, rejected, evicted;
} lodgs_server_stats;

typedef struct lodgs_server lodgs_server;

int lodgs_server_create(const lodgs_scene* scene, const lodgs_server_caps* caps, lodgs_server** out);
void lodgs_server_destroy(lodgs_server* server);
/* Queues the request (LODGS_E_INVALID for a size outside the classes or a
 * bad camera / tau / null image) and admits what can be admitted; *ticket
 * identifies it in its completion. */
int lodgs_server_submit(lodgs_server* server, const lodgs_request* request, uint64_t* ticket);
/* Non-blocking: collects finished requests (re-queueing overflowed ones),
 * admits queued ones, and copies up to max completions, oldest first, to
 * out; *n receives their number. */
int lodgs_server_poll(lodgs_server* server, lodgs_completion* out, int32_t max, int32_t* n);
int lodgs_server_stats_read(const lodgs_server* server, lodgs_server_stats* out);

/* ---------------------------------------------------------------- timing
 * Timing mode brackets every stage of lod_select / render / render_backward
 * with HIP events on the call's stream.  lodgs_frame_timings blocks until
 * the recorded events complete, returns the summed milliseconds and call
 * counts per stage since the last read, and clears the record. */
#define LODGS_STAGE_SELECT 0      /* upper cut, SPT binary search, compaction */
#define LODGS_STAGE_PROJECT 1     /* gather + EWA + SH                          */
#define LODGS_STAGE_DEPTH_SORT 2  /* radix sort of splats by depth              */
#define LODGS_STAGE_DUPLICATE 3   /* tile-count scan + instance emission        */
#define LODGS_STAGE_TILE_SORT 4   /* radix sort of instances by tile            */
#define LODGS_STAGE_RANGES 5      /* per-tile ranges                            */
#define LODGS_STAGE_BLEND 6       /* forward blend                              */
#define LODGS_STAGE_BLEND_BWD 7   /* backward blend (2D gradients)              */
#define LODGS_STAGE_PROJECT_BWD 8 /* projection / SH backward + scatter         */
#define LODGS_STAGE_LOSS 9        /* lodgs_l1_loss                              */
#define LODGS_N_STAGES 10

typedef struct lodgs_timings {
  double ms[LODGS_N_STAGES];
  int64_t calls[LODGS_N_STAGES];
} lodgs_timings;

int lodgs_frame_set_timing(lodgs_frame* frame, int enable);
int lodgs_frame_timings(lodgs_frame* frame, lodgs_timings* out);

/* Work counts of the last render's blend (blocks on the stream): replays the
 * forward blend with counters and returns the number of (pixel, splat)
 * evaluations, i.e. splats visited by a pixel before it stopped, and of
 * contributing pairs.  Diagnostics for the roofline; does not change any
 * output. */
int lodgs_frame_blend_work(lodgs_frame* frame, int64_t* evaluations, int64_t* contributions,
                           lodgs_stream stream);

/* Device arithmetic self-test of the operations every decision of the path
 * relies on being exact (IEEE round-to-nearest FP32 and FP64 division and
 * square root) and of the FP32 exp of the decision path.  For i < n, with
 * (a, b) = (d_in32[2i], d_in32[2i+1]) and (c, d) = (d_in64[2i], d_in64[2i+1]):
 *   d_out32[3i] = a / b, d_out32[3i+1] = sqrt(|a|), d_out32[3i+2] = exp(a),
 *   d_out64[2i] = c / d, d_out64[2i+1] = sqrt(|c|). */
int lodgs_selftest_arith(const float* d_in32, const double* d_in64, int64_t n, float* d_out32, double* d_out64,
                         lodgs_stream stream);

/* ---------------------------------------------------------------- loss
 * L1 loss of an image against a target (the configs' training objective):
 * L = sum |img - target| / n and dL/dimg = sign(img - target) / n with
 * sign(0) = 0, n = number of floats.  d_grad [n] is written; d_loss (one
 * float, optional) receives L.  Frame-free; records LODGS_STAGE_LOSS when a
 * frame in timing mode is given (frame may be NULL). */
int lodgs_l1_loss(lodgs_frame* frame, const float* d_img, const float* d_target, int64_t n, float* d_grad,
                  float* d_loss, lodgs_stream stream);

/* ---------------------------------------------------------------- optimiser
 * Adam step on the cut set (init/training appendix: each view updates only
 * the parameters of its cut set; the optimiser is the 3DGS one, Adam).  For
 * every selected position i < min(*d_count, capacity) with node = d_idx[i] in
 * [0, n_nodes), and every parameter group whose member of params is not NULL
 * (widths 3, 3, 4, 1 and 3 (sh_degree + 1)^2), element by element with
 * g = grads.<group>[i][c] (selection-indexed: the sel output of
 * lodgs_render_backward) and p, m, v the node's elements in params, exp_avg
 * and exp_avg_sq (node-indexed, the parameters' layouts):
 *   m = beta1 m + (1 - beta1) g,   v = beta2 v + (1 - beta2) g^2,
 *   p = p - lr / (1 - beta1^step) * m / (sqrt(v) / sqrt(1 - beta2^step) + eps).
 * step >= 1 counts the optimiser's steps (one count for all nodes).  d_idx must
 * not repeat a node (lodgs_lod_select's output does not); nodes outside
 * [0, n_nodes) are skipped.  All arrays are device arrays; FP32 throughout.
 * The quaternion and SH arrays (rows of 4 and 12 or 48 floats, which move as
 * float4s) must be 16-byte aligned.  Errors: LODGS_E_INVALID (a NULL grads /
 * exp_avg / exp_avg_sq member where the params member is set, a misaligned
 * quaternion or SH array, step < 1, a beta outside [0, 1), eps < 0,
 * sh_degree outside 0..3). */
typedef struct lodgs_adam {
  float lr[5]; /* per group: means, log_scales, quats, opacity_logits, sh */
  float beta1, beta2, eps;
  int32_t step;
  int32_t sh_degree;
} lodgs_adam;

int lodgs_adam_cut(const lodgs_grads* params, const lodgs_grads* grads, const lodgs_grads* exp_avg,
                   const lodgs_grads* exp_avg_sq, const lodgs_adam* hp, const int32_t* d_idx, const int32_t* d_count,
                   int64_t capacity, int64_t n_nodes, lodgs_stream stream);

const char* lodgs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LODGS_H_ */
