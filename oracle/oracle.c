/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.  A plain, slow CPU reference of the
 * per-view LoD-select + Gaussian-splat path of "A LoD of Gaussians"
 * (arXiv 2507.01110).  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the product path never does.  It shares no source
 * with the HIP library.
 *
 * Precision: continuous values (projections, colours, alphas, gradients) are
 * FP64.  Every discrete decision (LoD test, frustum test, near-plane test,
 * tile rectangle, depth key, alpha skip, alpha clamp, early termination) is
 * taken by an FP32 "decision mirror" that evaluates the documented FP32
 * formula operation by operation (no contraction, correctly rounded
 * + - * / sqrt, fmaf only where the formula says so), so that the selected
 * set, the key order and the set of contributing splats are defined exactly.
 * Decisions that lie within one ulp of their threshold, or that FP64 would
 * take the other way, are counted in the frame statistics.
 *
 * Readings of the paper that this file fixes (the paper is silent or garbled
 * there) are marked READING.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CULL 1u
#define ORC_CONSERVATIVE 2u
#define ORC_TILE 16

typedef struct orc_camera {
  float R[9];    /* world -> camera rotation, row-major, OpenCV axes      */
  float t[3];    /* x_cam = R x_world + t                                  */
  float pos[3];  /* camera centre in world space                           */
  float fx, fy, ppx, ppy;
  int32_t width, height;
  float z_near;
} orc_camera;

/* ------------------------------------------------------------------------ */
/* Portable FP32 exp used by every FP32 decision (and by the GPU's FP32 path,
 * which implements the same definition separately): Cody-Waite range
 * reduction x = n ln2 + r with ln2 split into a 16-bit-exact high part and a
 * low part, then the degree-7 Taylor polynomial of e^r by Horner's rule with
 * fmaf, then scaling by 2^n.  Inputs below -87 (and NaN) give 0.            */
float orc_pexp(float x) {
  if (!(x >= -87.0f)) return 0.0f;
  if (x > 88.0f) x = 88.0f;
  float n = rintf(x * 1.44269502f);
  float r = fmaf(-n, 0.693145752f, x);
  r = fmaf(-n, 1.42860677e-06f, r);
  float p = 1.98412701e-04f;         /* 1/7! */
  p = fmaf(p, r, 1.38888892e-03f);   /* 1/6! */
  p = fmaf(p, r, 8.33333377e-03f);   /* 1/5! */
  p = fmaf(p, r, 4.16666679e-02f);   /* 1/4! */
  p = fmaf(p, r, 1.66666672e-01f);   /* 1/3! */
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  return ldexpf(p, (int)n);
}

/* ------------------------------------------------------------------------ */
/* Per-node size metric and cull radius (Sec. 4.3, Eq. 6 and "Frustum
 * Culling").  READING: Eq. 6 prints a *minimum distance* T/sqrt(area); a node
 * is fine enough when its projected size is below tau pixels, i.e. when
 * g <= d tau / f with g = sqrt(s1 s2 + s1 s3 + s2 s3) (the size domain form of
 * the same test).  g and rho = 3 max_j s_j are evaluated in FP64 from the FP32
 * log-scales with the C library's exp and rounded once to FP32.  lv is the
 * log-volume log(s1 s2 s3) used by the HSPT split.                          */
void orc_metrics(int64_t n, const float* ls, float* g, float* rho, double* lv) {
  for (int64_t i = 0; i < n; ++i) {
    double s0 = exp((double)ls[3 * i]), s1 = exp((double)ls[3 * i + 1]), s2 = exp((double)ls[3 * i + 2]);
    double a = s0 * s1 + s0 * s2 + s1 * s2;
    g[i] = (float)sqrt(a);
    double m = s0 > s1 ? s0 : s1;
    m = m > s2 ? m : s2;
    rho[i] = (float)(3.0 * m);
    lv[i] = ((double)ls[3 * i] + (double)ls[3 * i + 1]) + (double)ls[3 * i + 2];
  }
}

/* ------------------------------------------------------------------------ */
/* HSPT construction (Sec. 4.3 "Hierarchical SPT"): a BFS from the root on the
 * condition s1 s2 s3 < size (here lv < log_size) splits the hierarchy; the
 * cut set roots the SPTs, the nodes above it form the upper hierarchy.  A
 * leaf reached by the BFS is a cut node as it has no children.  Every cut
 * node roots an SPT (READING of "subtrees of sufficient size": size >= 1).
 *
 * SPT intervals (Sec. 4.1, Eq. 4, with the size-domain reading): inside an SPT
 * a node is selected iff r_min <= X < r_max, where
 *   r_min = g(node) for interior nodes and 0 for leaves (a reached leaf is
 *           always acceptable, READING so that every root-to-leaf path is
 *           covered),
 *   r_max = +inf for the SPT root, else min(g(parent), r_max(parent)), the
 *           prefix minimum over ancestors inside the SPT (READING of the
 *           "unreachable Gaussians" paragraph: a node whose ancestor is already
 *           fine enough is never selected, so cuts stay proper even when the
 *           heap condition fails).
 * role: 0 upper node, 1 SPT root, 2 other SPT member.  spt_of: tree id of the
 * SPT root for members and roots, -1 for upper nodes.                      */
int orc_hspt(int64_t n, const int32_t* left, const int32_t* right, int32_t root, const double* lv,
             double log_size, const float* g, int8_t* role, int32_t* spt_of, float* r_min, float* r_max) {
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue || !stack) { free(queue); free(stack); return -1; }
  for (int64_t i = 0; i < n; ++i) { role[i] = -1; spt_of[i] = -1; r_min[i] = NAN; r_max[i] = NAN; }
  int64_t qh = 0, qt = 0;
  queue[qt++] = root;
  while (qh < qt) {
    int32_t u = queue[qh++];
    int leaf = left[u] < 0;
    if (leaf || lv[u] < log_size) {
      /* u roots an SPT: walk its subtree, filling the intervals. */
      role[u] = 1;
      int64_t sp = 0;
      stack[sp++] = u;
      r_max[u] = INFINITY;
      while (sp > 0) {
        int32_t v = stack[--sp];
        spt_of[v] = u;
        if (v != u) role[v] = 2;
        if (left[v] < 0) {
          r_min[v] = 0.0f;
        } else {
          r_min[v] = g[v];
          float m = fminf(g[v], r_max[v]);
          r_max[left[v]] = m;
          r_max[right[v]] = m;
          stack[sp++] = left[v];
          stack[sp++] = right[v];
        }
      }
    } else {
      role[u] = 0;
      queue[qt++] = left[u];
      queue[qt++] = right[u];
    }
  }
  free(queue);
  free(stack);
  return 0;
}

/* Layout (the flattened order the device arrays use): upper nodes in DFS
 * preorder (left child first), then one contiguous segment per SPT, segments in
 * the order a left-first DFS of the upper hierarchy meets their roots, each
 * segment sorted by r_max descending (the sort of Sec. 4.1 that makes the
 * candidate set a prefix found by binary search), ties by r_min descending,
 * then tree id ascending.  pos_of[tree id] = layout position, perm = inverse. */
typedef struct { float rmax, rmin; int32_t id; } orc_sptkey;
static int cmp_sptkey(const void* a, const void* b) {
  const orc_sptkey* x = (const orc_sptkey*)a;
  const orc_sptkey* y = (const orc_sptkey*)b;
  if (x->rmax != y->rmax) return x->rmax > y->rmax ? -1 : 1;
  if (x->rmin != y->rmin) return x->rmin > y->rmin ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

int orc_layout(int64_t n, const int32_t* left, const int32_t* right, int32_t root, const int8_t* role,
               const int32_t* spt_of, const float* r_min, const float* r_max, int32_t* pos_of,
               int32_t* perm, int32_t* n_upper_out, int32_t* n_spt_out, int32_t* spt_begin) {
  int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* roots = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  if (!stack || !roots || !cnt) { free(stack); free(roots); free(cnt); return -1; }
  int64_t sp = 0, nu = 0, ns = 0;
  stack[sp++] = root;
  while (sp > 0) {
    int32_t u = stack[--sp];
    if (role[u] == 0) {
      pos_of[u] = (int32_t)nu;
      perm[nu++] = u;
      stack[sp++] = right[u];  /* pushed first so the left child pops first */
      stack[sp++] = left[u];
    } else {
      roots[ns++] = u;
    }
  }
  for (int64_t i = 0; i < n; ++i)
    if (role[i] != 0) cnt[spt_of[i]]++;
  int64_t off = nu;
  orc_sptkey* keys = NULL;
  int64_t kcap = 0;
  for (int64_t j = 0; j < ns; ++j) {
    int32_t rj = roots[j];
    spt_begin[j] = (int32_t)off;
    int64_t m = cnt[rj];
    if (m > kcap) {
      free(keys);
      kcap = m;
      keys = (orc_sptkey*)malloc(sizeof(orc_sptkey) * (size_t)kcap);
    }
    int64_t k = 0, tp = 0;
    stack[tp++] = rj;
    while (tp > 0) {
      int32_t v = stack[--tp];
      keys[k].rmax = r_max[v];
      keys[k].rmin = r_min[v];
      keys[k].id = v;
      ++k;
      if (left[v] >= 0) {
        stack[tp++] = left[v];
        stack[tp++] = right[v];
      }
    }
    qsort(keys, (size_t)k, sizeof(orc_sptkey), cmp_sptkey);
    for (int64_t e = 0; e < k; ++e) {
      pos_of[keys[e].id] = (int32_t)(off + e);
      perm[off + e] = keys[e].id;
    }
    off += k;
  }
  spt_begin[ns] = (int32_t)off;
  *n_upper_out = (int32_t)nu;
  *n_spt_out = (int32_t)ns;
  free(keys);
  free(stack);
  free(roots);
  free(cnt);
  return off == n ? 0 : -2;
}

/* ------------------------------------------------------------------------ */
/* FP32 decision mirror for the LoD cut.                                     */
static float dist32(const float* mu, const float* p) {
  float dx = mu[0] - p[0], dy = mu[1] - p[1], dz = mu[2] - p[2];
  float s = dx * dx;
  s = s + dy * dy;
  s = s + dz * dz;
  return sqrtf(s);
}

static void cam32(const orc_camera* C, const float* mu, float* c) {
  const float* R = C->R;
  for (int r = 0; r < 3; ++r) {
    float v = R[3 * r] * mu[0];
    v = v + R[3 * r + 1] * mu[1];
    v = v + R[3 * r + 2] * mu[2];
    c[r] = v + C->t[r];
  }
}

/* Frustum test of the sphere (mu, rho) (Sec. 4.3 "Frustum Culling").  READING:
 * the frustum is the four side planes through the camera centre and the near
 * plane z = z_near, no far plane; a sphere is culled when it lies entirely
 * outside one of them.  Side plane normals are normalised by sqrt(1 + h^2). */
typedef struct { float hl, hr, ht, hb, nl, nr, nt, nb; } orc_frustum;
static orc_frustum frustum32(const orc_camera* C) {
  orc_frustum F;
  F.hl = C->ppx / C->fx;
  F.hr = ((float)C->width - C->ppx) / C->fx;
  F.ht = C->ppy / C->fy;
  F.hb = ((float)C->height - C->ppy) / C->fy;
  F.nl = sqrtf(1.0f + F.hl * F.hl);
  F.nr = sqrtf(1.0f + F.hr * F.hr);
  F.nt = sqrtf(1.0f + F.ht * F.ht);
  F.nb = sqrtf(1.0f + F.hb * F.hb);
  return F;
}

static int culled32(const orc_camera* C, const orc_frustum* F, const float* mu, float rho) {
  float c[3];
  cam32(C, mu, c);
  if (c[2] + rho < C->z_near) return 1;
  if (c[0] - F->hr * c[2] > rho * F->nr) return 1;
  if (-c[0] - F->hl * c[2] > rho * F->nl) return 1;
  if (c[1] - F->hb * c[2] > rho * F->nb) return 1;
  if (-c[1] - F->ht * c[2] > rho * F->nt) return 1;
  return 0;
}

typedef struct orc_select_stats {
  int64_t upper_tested, upper_selected, spt_visible, spt_culled, spt_nodes_tested, spt_selected;
  int64_t ties_exact, ties_1ulp;
} orc_select_stats;

static void tie_log(float a, float X, orc_select_stats* st) {
  if (a == X) st->ties_exact++;
  else if (isfinite(a) && fabsf(a - X) <= fabsf(nextafterf(X, INFINITY) - X)) st->ties_1ulp++;
}

static const int32_t* g_sort_pos;
static int cmp_by_pos(const void* a, const void* b) {
  int32_t x = g_sort_pos[*(const int32_t*)a], y = g_sort_pos[*(const int32_t*)b];
  return (x > y) - (x < y);
}

/* The HSPT cut (Sec. 4.3, two steps; Alg. 1 semantics for the BFS, Eq. 4 for
 * the SPTs), written as a recursive descent:
 *  - an upper node u is dropped with its subtree when culled, selected when
 *    fine enough at its own distance (g_u <= d_u tau / fx), else both children
 *    are visited;
 *  - an SPT root j is dropped with its SPT when culled, otherwise its SPT is
 *    cut at the root's distance X_j = d_j tau / fx: descending from j, the
 *    first node on each path with g <= X_j is selected, and a reached leaf is
 *    always selected.
 * READING (Alg. 3): culled upper nodes and culled SPTs are not rendered; the
 * focal normalisation of the implementation appendix is X = d tau / fx with
 * each camera's own fx.
 * mode 0: SPT cut by descent; mode 1: SPT cut by the linear scan of Alg. 2
 * (every member tested with r_min <= X_j < r_max).  Output: tree ids sorted
 * by layout position pos_of.                                                */
/* Radius of the SPT rooted at u about the root's mean: the largest
 * |mu_v - mu_u| over the nodes v of u's subtree (the SPT's members), in FP64
 * from the FP32 means (((dx dx + dy dy) + dz dz), correctly rounded square
 * root), rounded once to FP32.  READING (Sec. 4.1, the conservative M_d, as
 * printed camera-dependent): the CONSERVATIVE variant cuts SPT u at
 * X = max(0, d_u - R_u) tau / fx, a distance no member can be closer than
 * (triangle inequality), so no member is cut coarser than its own distance
 * allows; X stays one per SPT, so Eq. 4's sorted intervals still apply. */
static float spt_radius(const int32_t* left, const int32_t* right, const float* means, int32_t u,
                        int32_t* stack) {
  const double rx = means[3 * (int64_t)u], ry = means[3 * (int64_t)u + 1], rz = means[3 * (int64_t)u + 2];
  double r = 0.0;
  int64_t sp = 0;
  stack[sp++] = u;
  while (sp > 0) {
    const int32_t v = stack[--sp];
    const double dx = (double)means[3 * (int64_t)v] - rx, dy = (double)means[3 * (int64_t)v + 1] - ry,
                 dz = (double)means[3 * (int64_t)v + 2] - rz;
    const double d = sqrt((dx * dx + dy * dy) + dz * dz);
    if (d > r) r = d;
    if (left[v] >= 0) {
      stack[sp++] = left[v];
      stack[sp++] = right[v];
    }
  }
  return (float)r;
}

/* spt_X (optional, [n] by tree id): a value that is not NaN at a visible SPT
 * root replaces that SPT's X (the SPT-cut cache reuses a cached cut this
 * way); spt_visible (optional, [n]): set to 1 at every visible SPT root.
 * spt_scale: the varying level of detail of the implementation appendix
 * multiplies the distances to the SPT centres by a per-iteration factor; the
 * FP32 distance to an SPT root is multiplied by spt_scale (1: no noise)
 * before it enters that SPT's cut, upper nodes keep their own distance. */
int orc_select(int64_t n, const int32_t* left, const int32_t* right, int32_t root, const float* means,
               const float* g, const float* rho, const int8_t* role, const int32_t* spt_of,
               const float* r_min, const float* r_max, const int32_t* pos_of, const orc_camera* C,
               float tau, float spt_scale, uint32_t flags, int mode, int32_t* out, int64_t cap, int64_t* n_out,
               orc_select_stats* st_out, const float* spt_X, uint8_t* spt_visible) {
  orc_select_stats st;
  memset(&st, 0, sizeof st);
  const float k = tau / C->fx;
  const orc_frustum F = frustum32(C);
  const int cull = (flags & ORC_CULL) != 0;
  int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* stk2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!stack || !stk2) { free(stack); free(stk2); return -1; }
  int64_t cnt = 0, sp = 0;
  int overflow = 0;
#define EMIT(v) do { if (cnt < cap) out[cnt] = (v); else overflow = 1; cnt++; } while (0)
  stack[sp++] = root;
  while (sp > 0) {
    int32_t u = stack[--sp];
    const float* mu = means + 3 * (int64_t)u;
    if (role[u] == 0) {
      st.upper_tested++;
      if (cull && culled32(C, &F, mu, rho[u])) continue;
      float X = dist32(mu, C->pos) * k;
      tie_log(g[u], X, &st);
      if (g[u] <= X) {
        st.upper_selected++;
        EMIT(u);
      } else {
        stack[sp++] = left[u];
        stack[sp++] = right[u];
      }
      continue;
    }
    /* u is an SPT root */
    if (cull && culled32(C, &F, mu, rho[u])) { st.spt_culled++; continue; }
    st.spt_visible++;
    if (spt_visible) spt_visible[u] = 1;
    const float d = dist32(mu, C->pos) * spt_scale;
    float X = d * k;
    if (flags & ORC_CONSERVATIVE) X = fmaxf(0.0f, d - spt_radius(left, right, means, u, stk2)) * k;
    if (spt_X && !isnan(spt_X[u])) X = spt_X[u];
    int64_t tp = 0;
    stk2[tp++] = u;
    while (tp > 0) {
      int32_t v = stk2[--tp];
      st.spt_nodes_tested++;
      if (mode == 0) {
        int leaf = left[v] < 0;
        if (!leaf) tie_log(g[v], X, &st);
        if (leaf || g[v] <= X) {
          st.spt_selected++;
          EMIT(v);
        } else {
          stk2[tp++] = left[v];
          stk2[tp++] = right[v];
        }
      } else {
        tie_log(r_min[v], X, &st);
        tie_log(r_max[v], X, &st);
        if (r_min[v] <= X && X < r_max[v]) {
          st.spt_selected++;
          EMIT(v);
        }
        if (left[v] >= 0) {  /* the scan visits every member */
          stk2[tp++] = left[v];
          stk2[tp++] = right[v];
        }
      }
    }
  }
#undef EMIT
  free(stack);
  free(stk2);
  *n_out = cnt;
  if (st_out) *st_out = st;
  if (overflow) return -2;
  g_sort_pos = pos_of;
  qsort(out, (size_t)cnt, sizeof(int32_t), cmp_by_pos);
  (void)spt_of;
  return 0;
}

/* The two whole-hierarchy cuts that the HSPT replaces (Sec. 4.3, "BFS" and
 * "Parallel Cut"), for comparison.  Every node is tested at its own distance,
 * X_i = d_i tau / fx, with the size test read as for the HSPT cut: fine(i)
 * when i is a leaf or g_i <= X_i.
 *  - BFS cut: the descent of Alg. 1 over the whole hierarchy, in breadth-first
 *    order from the root: a reached node is dropped with its subtree when
 *    culled, selected when fine, else its two children are reached.
 *  - Parallel cut (Eq. 5, with the same reading of its size test): node i is
 *    selected when fine(i) and, unless it is the root, its parent is not
 *    fine; with culling, a node whose own sphere is culled is dropped.
 * Output: tree ids sorted by layout position pos_of; -2 when more than cap. */
static int finish_cut(int32_t* out, int64_t cnt, int64_t cap, const int32_t* pos_of, int64_t* n_out) {
  *n_out = cnt;
  if (cnt > cap) return -2;
  g_sort_pos = pos_of;
  qsort(out, (size_t)cnt, sizeof(int32_t), cmp_by_pos);
  return 0;
}

static int fine32(const int32_t* left, const float* means, const float* g, int32_t v, const float* pos, float k) {
  return left[v] < 0 || g[v] <= dist32(means + 3 * (int64_t)v, pos) * k;
}

int orc_select_bfs(int64_t n, const int32_t* left, const int32_t* right, int32_t root, const float* means,
                   const float* g, const float* rho, const int32_t* pos_of, const orc_camera* C, float tau,
                   uint32_t flags, int32_t* out, int64_t cap, int64_t* n_out) {
  const float k = tau / C->fx;
  const orc_frustum F = frustum32(C);
  const int cull = (flags & ORC_CULL) != 0;
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!queue) return -1;
  int64_t head = 0, tail = 0, cnt = 0;
  queue[tail++] = root;
  while (head < tail) {
    const int32_t u = queue[head++];
    if (cull && culled32(C, &F, means + 3 * (int64_t)u, rho[u])) continue;
    if (fine32(left, means, g, u, C->pos, k)) {
      if (cnt < cap) out[cnt] = u;
      cnt++;
    } else {
      queue[tail++] = left[u];
      queue[tail++] = right[u];
    }
  }
  free(queue);
  return finish_cut(out, cnt, cap, pos_of, n_out);
}

int orc_select_parallel(int64_t n, const int32_t* left, const int32_t* right, int32_t root, const float* means,
                        const float* g, const float* rho, const int32_t* pos_of, const orc_camera* C, float tau,
                        uint32_t flags, int32_t* out, int64_t cap, int64_t* n_out) {
  const float k = tau / C->fx;
  const orc_frustum F = frustum32(C);
  const int cull = (flags & ORC_CULL) != 0;
  int32_t* parent = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!parent) return -1;
  for (int64_t v = 0; v < n; ++v) parent[v] = -1;
  for (int64_t v = 0; v < n; ++v)
    if (left[v] >= 0) {
      parent[left[v]] = (int32_t)v;
      parent[right[v]] = (int32_t)v;
    }
  int64_t cnt = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int32_t i = (int32_t)v;
    if (!fine32(left, means, g, i, C->pos, k)) continue;
    if (i != root && parent[i] >= 0 && fine32(left, means, g, parent[i], C->pos, k)) continue;
    if (cull && culled32(C, &F, means + 3 * v, rho[i])) continue;
    if (cnt < cap) out[cnt] = i;
    cnt++;
  }
  free(parent);
  return finish_cut(out, cnt, cap, pos_of, n_out);
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics up to degree 3 (Sec. 3: view-dependent colour from
 * SH coefficients), index k = l^2 + l + m, Condon-Shortley signs folded in
 * as in the 3DGS convention.  The constants are the normalisation factors of
 * the real SH basis, sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the
 * polynomial scale for each (l, m).                                         */
static const double SHC0 = 0.28209479177387814;
static const double SHC1 = 0.4886025119029199;
static const double SHC2[5] = {1.0925484305920792, -1.0925484305920792, 0.31539156525252005,
                               -1.0925484305920792, 0.5462742152960396};
static const double SHC3[7] = {-0.5900435899266435, 2.890611442640554, -0.4570457994644658,
                               0.3731763325901154, -0.4570457994644658, 1.445305721320277,
                               -0.5900435899266435};

void orc_sh_basis(const double* d, double* Y, double* dY /* [16][3] or NULL */) {
  double x = d[0], y = d[1], z = d[2];
  double xx = x * x, yy = y * y, zz = z * z;
  Y[0] = SHC0;
  Y[1] = -SHC1 * y; Y[2] = SHC1 * z; Y[3] = -SHC1 * x;
  Y[4] = SHC2[0] * x * y; Y[5] = SHC2[1] * y * z; Y[6] = SHC2[2] * (2 * zz - xx - yy);
  Y[7] = SHC2[3] * x * z; Y[8] = SHC2[4] * (xx - yy);
  Y[9] = SHC3[0] * y * (3 * xx - yy); Y[10] = SHC3[1] * x * y * z;
  Y[11] = SHC3[2] * y * (4 * zz - xx - yy); Y[12] = SHC3[3] * z * (2 * zz - 3 * xx - 3 * yy);
  Y[13] = SHC3[4] * x * (4 * zz - xx - yy); Y[14] = SHC3[5] * z * (xx - yy);
  Y[15] = SHC3[6] * x * (xx - 3 * yy);
  if (!dY) return;
  memset(dY, 0, sizeof(double) * 48);
#define D(k, a, b, c) do { dY[3 * (k)] = (a); dY[3 * (k) + 1] = (b); dY[3 * (k) + 2] = (c); } while (0)
  D(1, 0, -SHC1, 0); D(2, 0, 0, SHC1); D(3, -SHC1, 0, 0);
  D(4, SHC2[0] * y, SHC2[0] * x, 0);
  D(5, 0, SHC2[1] * z, SHC2[1] * y);
  D(6, -2 * SHC2[2] * x, -2 * SHC2[2] * y, 4 * SHC2[2] * z);
  D(7, SHC2[3] * z, 0, SHC2[3] * x);
  D(8, 2 * SHC2[4] * x, -2 * SHC2[4] * y, 0);
  D(9, 6 * SHC3[0] * x * y, SHC3[0] * (3 * xx - 3 * yy), 0);
  D(10, SHC3[1] * y * z, SHC3[1] * x * z, SHC3[1] * x * y);
  D(11, -2 * SHC3[2] * x * y, SHC3[2] * (4 * zz - xx - 3 * yy), 8 * SHC3[2] * y * z);
  D(12, -6 * SHC3[3] * x * z, -6 * SHC3[3] * y * z, SHC3[3] * (6 * zz - 3 * xx - 3 * yy));
  D(13, SHC3[4] * (4 * zz - 3 * xx - yy), -2 * SHC3[4] * x * y, 8 * SHC3[4] * x * z);
  D(14, 2 * SHC3[5] * x * z, -2 * SHC3[5] * y * z, SHC3[5] * (xx - yy));
  D(15, SHC3[6] * (3 * xx - 3 * yy), -6 * SHC3[6] * x * y, 0);
#undef D
}

/* ------------------------------------------------------------------------ */
/* Projection (Sec. 3: EWA affine approximation of the projective transform,
 * Eq. 2 read with the inverse projected covariance).  READING: a 0.3 px^2
 * low-pass is added to the diagonal of the projected covariance; splats with
 * camera depth <= z_near are not drawn; the tile footprint is the square of
 * half-width ceil(3 sqrt(lambda_max)) around the projected mean, 16x16 tiles.
 *
 * Decision mirror of the projection: the per-splat chain is evaluated in FP64
 * with a fixed operation order (scales from the FP32 portable exp, opacity as
 * the FP32 sigmoid), and its results are rounded to the FP32 record that the
 * per-pixel FP32 alpha uses: the projected mean as a hi/lo pair of floats,
 * the principal axis (ce, se) of the projected covariance and the power
 * coefficients h1 = -1/(2 l1), h2 = -1/(2 l2) of its eigenvalues, so that
 * power = h1 u1^2 + h2 u2^2 with (u1, u2) the pixel offset in that basis. */
typedef struct {
  int32_t visible, tiles, x0, x1, y0, y1;
  float depth, mxh, mxl, myh, myl, ce, se, h1, h2, o, radius;
} orc_g32;

static int clamp_tile_d(double v, int hi) {
  if (v < 0.0) return 0;
  if (v > (double)hi) return hi;
  return (int)v;
}

void orc_project32(const float* mu, const float* ls, const float* q, float theta, const orc_camera* C,
                   int TX, int TY, orc_g32* G) {
  memset(G, 0, sizeof *G);
  double W[9], t[3];
  for (int k = 0; k < 9; ++k) W[k] = (double)C->R[k];
  for (int k = 0; k < 3; ++k) t[k] = (double)C->t[k];
  const double m0 = mu[0], m1 = mu[1], m2 = mu[2];
  double c[3];
  for (int r = 0; r < 3; ++r) c[r] = ((W[3 * r] * m0 + W[3 * r + 1] * m1) + W[3 * r + 2] * m2) + t[r];
  G->depth = (float)c[2];
  if (!(c[2] > (double)C->z_near)) return;
  const double s0 = (double)orc_pexp(ls[0]), s1 = (double)orc_pexp(ls[1]), s2 = (double)orc_pexp(ls[2]);
  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  const double qq = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
  const double qn = sqrt(qq);
  const double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
  const double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  const double wx = w * x, wy = w * y, wz = w * z;
  const double r00 = 1.0 - 2.0 * (yy + zz), r01 = 2.0 * (xy - wz), r02 = 2.0 * (xz + wy);
  const double r10 = 2.0 * (xy + wz), r11 = 1.0 - 2.0 * (xx + zz), r12 = 2.0 * (yz - wx);
  const double r20 = 2.0 * (xz - wy), r21 = 2.0 * (yz + wx), r22 = 1.0 - 2.0 * (xx + yy);
  const double m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
  const double m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
  const double m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
  const double S00 = (m00 * m00 + m01 * m01) + m02 * m02;
  const double S01 = (m00 * m10 + m01 * m11) + m02 * m12;
  const double S02 = (m00 * m20 + m01 * m21) + m02 * m22;
  const double S11 = (m10 * m10 + m11 * m11) + m12 * m12;
  const double S12 = (m10 * m20 + m11 * m21) + m12 * m22;
  const double S22 = (m20 * m20 + m21 * m21) + m22 * m22;
  const double fx = C->fx, fy = C->fy;
  const double u = c[0] / c[2], v = c[1] / c[2];
  const double jx = fx / c[2], jy = fy / c[2];
  const double jxz = -(jx * u), jyz = -(jy * v);
  const double T00 = jx * W[0] + jxz * W[6], T01 = jx * W[1] + jxz * W[7], T02 = jx * W[2] + jxz * W[8];
  const double T10 = jy * W[3] + jyz * W[6], T11 = jy * W[4] + jyz * W[7], T12 = jy * W[5] + jyz * W[8];
  const double U00 = (T00 * S00 + T01 * S01) + T02 * S02;
  const double U01 = (T00 * S01 + T01 * S11) + T02 * S12;
  const double U02 = (T00 * S02 + T01 * S12) + T02 * S22;
  const double U10 = (T10 * S00 + T11 * S01) + T12 * S02;
  const double U11 = (T10 * S01 + T11 * S11) + T12 * S12;
  const double U12 = (T10 * S02 + T11 * S12) + T12 * S22;
  const double A = ((U00 * T00 + U01 * T01) + U02 * T02) + 0.3;
  const double B = (U00 * T10 + U01 * T11) + U02 * T12;
  const double Cc = ((U10 * T10 + U11 * T11) + U12 * T12) + 0.3;
  const double det = A * Cc - B * B;
  if (!(det > 0.0)) return;
  const double mx = fx * u + (double)C->ppx, my = fy * v + (double)C->ppy;
  const double mid = 0.5 * (A + Cc);
  const double disc = mid * mid - det;
  const double r = ceil(3.0 * sqrt(mid + sqrt(fmax(0.1, disc))));
  G->radius = (float)r;
  G->x0 = clamp_tile_d(floor((mx - r) * 0.0625), TX);
  G->x1 = clamp_tile_d(floor((mx + r) * 0.0625) + 1.0, TX);
  G->y0 = clamp_tile_d(floor((my - r) * 0.0625), TY);
  G->y1 = clamp_tile_d(floor((my + r) * 0.0625) + 1.0, TY);
  G->tiles = (G->x1 > G->x0 && G->y1 > G->y0) ? (G->x1 - G->x0) * (G->y1 - G->y0) : 0;
  G->visible = G->tiles > 0;
  /* principal axes of the projected covariance */
  const double l1 = mid + sqrt(fmax(0.0, disc));
  const double l2 = det / l1;
  double vx, vy;
  if (A >= Cc) {
    vx = l1 - Cc;
    vy = B;
  } else {
    vx = B;
    vy = l1 - A;
  }
  const double nn = sqrt(vx * vx + vy * vy);
  double ce = 1.0, se = 0.0;
  if (nn > 0.0) {
    ce = vx / nn;
    se = vy / nn;
  }
  G->mxh = (float)mx;
  G->mxl = (float)(mx - (double)G->mxh);
  G->myh = (float)my;
  G->myl = (float)(my - (double)G->myh);
  G->ce = (float)ce;
  G->se = (float)se;
  G->h1 = (float)(-0.5 / l1);
  G->h2 = (float)(-0.5 / l2);
  G->o = 1.0f / (1.0f + orc_pexp(-theta));
}

/* FP64 values of one splat.  Parameter vector layout (per Gaussian):
 * [mu 3 | log-scale 3 | quaternion (w,x,y,z) 4 | opacity logit 1 | SH n_coef]. */
typedef struct {
  double c[3];        /* camera-space mean                      */
  double s[3], qn[4], qlen, Rq[9], M[9], Sig[6];
  double T[6];        /* J W, 2x3                               */
  double A, B, Cc, det, ca, cb, cc;
  double mx, my, o;
  double dir[3], dlen, Y[16], rgb[3];
  int clamp[3];
} orc_g64;

void orc_project64(const double* P, int n_coef, const orc_camera* C, orc_g64* G) {
  const double* mu = P;
  const double* W = NULL;
  double Wd[9];
  for (int i = 0; i < 9; ++i) Wd[i] = C->R[i];
  W = Wd;
  for (int r = 0; r < 3; ++r) G->c[r] = W[3 * r] * mu[0] + W[3 * r + 1] * mu[1] + W[3 * r + 2] * mu[2] + (double)C->t[r];
  for (int k = 0; k < 3; ++k) G->s[k] = exp(P[3 + k]);
  const double* q = P + 6;
  G->qlen = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) G->qn[k] = q[k] / G->qlen;
  double w = G->qn[0], x = G->qn[1], y = G->qn[2], z = G->qn[3];
  double* Rq = G->Rq;
  Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z); Rq[2] = 2 * (x * z + w * y);
  Rq[3] = 2 * (x * y + w * z); Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
  Rq[6] = 2 * (x * z - w * y); Rq[7] = 2 * (y * z + w * x); Rq[8] = 1 - 2 * (x * x + y * y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) G->M[3 * i + j] = Rq[3 * i + j] * G->s[j];
  static const int IJ[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  for (int e = 0; e < 6; ++e) {
    int i = IJ[e][0], j = IJ[e][1];
    G->Sig[e] = G->M[3 * i] * G->M[3 * j] + G->M[3 * i + 1] * G->M[3 * j + 1] + G->M[3 * i + 2] * G->M[3 * j + 2];
  }
  double cz = G->c[2];
  double J00 = C->fx / cz, J02 = -C->fx * G->c[0] / (cz * cz);
  double J11 = C->fy / cz, J12 = -C->fy * G->c[1] / (cz * cz);
  for (int j = 0; j < 3; ++j) {
    G->T[j] = J00 * W[j] + J02 * W[6 + j];
    G->T[3 + j] = J11 * W[3 + j] + J12 * W[6 + j];
  }
  double S[3][3] = {{G->Sig[0], G->Sig[1], G->Sig[2]}, {G->Sig[1], G->Sig[3], G->Sig[4]}, {G->Sig[2], G->Sig[4], G->Sig[5]}};
  double U[2][3];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) U[i][j] = G->T[3 * i] * S[0][j] + G->T[3 * i + 1] * S[1][j] + G->T[3 * i + 2] * S[2][j];
  G->A = U[0][0] * G->T[0] + U[0][1] * G->T[1] + U[0][2] * G->T[2] + 0.3;
  G->B = U[0][0] * G->T[3] + U[0][1] * G->T[4] + U[0][2] * G->T[5];
  G->Cc = U[1][0] * G->T[3] + U[1][1] * G->T[4] + U[1][2] * G->T[5] + 0.3;
  G->det = G->A * G->Cc - G->B * G->B;
  G->ca = G->Cc / G->det;
  G->cb = -G->B / G->det;
  G->cc = G->A / G->det;
  G->mx = C->fx * G->c[0] / cz + C->ppx;
  G->my = C->fy * G->c[1] / cz + C->ppy;
  G->o = 1.0 / (1.0 + exp(-P[10]));
  for (int k = 0; k < 3; ++k) G->dir[k] = mu[k] - (double)C->pos[k];
  G->dlen = sqrt(G->dir[0] * G->dir[0] + G->dir[1] * G->dir[1] + G->dir[2] * G->dir[2]);
  double d[3] = {G->dir[0] / G->dlen, G->dir[1] / G->dlen, G->dir[2] / G->dlen};
  orc_sh_basis(d, G->Y, NULL);
  int nb = n_coef / 3;
  const double* sh = P + 11;
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
    for (int k = 0; k < nb; ++k) acc += sh[3 * k + ch] * G->Y[k];
    acc += 0.5;
    G->clamp[ch] = acc < 0.0;
    G->rgb[ch] = acc < 0.0 ? 0.0 : acc;
  }
}

/* ------------------------------------------------------------------------ */
/* Render (Sec. 3, Eq. 1 front-to-back compositing; Eq. 2 alpha).  READING,
 * following the rasterizer the paper reuses: alpha = min(0.99, o exp(power)),
 * a splat with alpha < 1/255 is skipped at that pixel, compositing stops
 * *before* a splat that would bring the transmittance below 1e-4, and the
 * background (black unless given) fills the remaining transmittance.  Pixel
 * (x, y) is sampled at (x + 0.5, y + 0.5).  Splats are drawn per tile in the
 * order of the key (tile, FP32 depth bits), ties by selection order.       */
typedef struct orc_frame {
  int64_t n;
  int n_coef, W, H, TX, TY;
  orc_camera cam;
  double bg[3];
  double* P;          /* [n][11 + n_coef] FP64 parameters */
  orc_g32* g32;
  int64_t n_inst;
  int32_t* inst_tile;
  int32_t* inst_pos;  /* sorted instance -> selection position */
  int64_t* tile_start;
  int64_t* pix_off;   /* [W*H + 1] */
  int32_t* pix_list;
  uint8_t* pix_clamp;
  /* decision log: FP32 decisions within one ulp of their threshold, and
   * decisions that the FP64 evaluation of the same test takes the other way
   * (skip: alpha < 1/255; clamp: o e^power > 0.99; stop: T (1 - alpha) <
   * 1e-4 with T the FP64 transmittance along the FP32 decisions) */
  int64_t skip_1ulp, stop_1ulp, skip_flip64, stop_flip64, clamp_flip64;
  double* v64;        /* [n][6] FP64 mx, my, conic a, b, c, opacity (visible splats; the log pass only) */
  /* lazily built for directional finite differences */
  orc_g64* g64;       /* [n] FP64 values of the unperturbed splats */
  int64_t* gpix_off;  /* [n + 1] pixels each splat contributes to (CSR) */
  int64_t* gpix;
} orc_frame;

typedef struct { uint32_t tile, depth; int32_t pos; } orc_inst;
static int cmp_inst(const void* a, const void* b) {
  const orc_inst* x = (const orc_inst*)a;
  const orc_inst* y = (const orc_inst*)b;
  if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
  if (x->depth != y->depth) return x->depth < y->depth ? -1 : 1;
  return (x->pos > y->pos) - (x->pos < y->pos);
}

static uint32_t fbits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

/* FP32 mirror of one pixel's compositing decisions; returns the number of
 * contributing splats and, when list != NULL, their selection positions and
 * whether their alpha was clamped at 0.99.  The power of a splat at the
 * pixel centre (px, py) is evaluated from its FP32 record as
 *   dx = (px - mxh) - mxl;  dy = (py - myh) - myl;
 *   u1 = fmaf(se, dy, ce*dx);  u2 = fmaf(-se, dx, ce*dy);
 *   power = fmaf(h1*u1, u1, (h2*u2)*u2). */
static int64_t pixel32(const orc_frame* F, int px, int py, int32_t* list, uint8_t* clampf, int64_t* log5) {
  int tile = (py / ORC_TILE) * F->TX + px / ORC_TILE;
  float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  float T = 1.0f;
  double T64 = 1.0;
  int64_t cnt = 0;
  const float thr = 1.0f / 255.0f;
  for (int64_t k = F->tile_start[tile]; k < F->tile_start[tile + 1]; ++k) {
    int32_t i = F->inst_pos[k];
    const orc_g32* G = F->g32 + i;
    float dx = (fx - G->mxh) - G->mxl, dy = (fy - G->myh) - G->myl;
    float u1 = G->ce * dx;
    u1 = fmaf(G->se, dy, u1);
    float u2 = G->ce * dy;
    u2 = fmaf(-G->se, dx, u2);
    float a2 = G->h2 * u2;
    a2 = a2 * u2;
    float power = fmaf(G->h1 * u1, u1, a2);
    float oe = G->o * orc_pexp(power);
    float alpha = fminf(0.99f, oe);
    /* the FP64 evaluation of the same tests (log pass only) */
    double oe64 = 0.0, a64 = 0.0;
    if (log5) {
      if (fabsf(alpha - thr) <= fabsf(nextafterf(thr, 1.0f) - thr)) log5[0]++;
      const double* V = F->v64 + 6 * (int64_t)i;
      const double ddx = ((double)px + 0.5) - V[0], ddy = ((double)py + 0.5) - V[1];
      oe64 = V[5] * exp(-0.5 * (V[2] * ddx * ddx + V[4] * ddy * ddy) - V[3] * ddx * ddy);
      a64 = oe64 < 0.99 ? oe64 : 0.99;
      if ((a64 < 1.0 / 255.0) != (alpha < thr)) log5[2]++;
    }
    if (alpha < thr) continue;
    float tt = T * (1.0f - alpha);
    if (log5) {
      if (fabsf(tt - 0.0001f) <= fabsf(nextafterf(0.0001f, 1.0f) - 0.0001f)) log5[1]++;
      if ((oe64 > 0.99) != (oe > 0.99f)) log5[4]++;
      if ((T64 * (1.0 - a64) < 1e-4) != (tt < 0.0001f)) log5[3]++;
      /* the FP64 transmittance follows the FP32 decisions (the FP64 image's) */
      T64 *= 1.0 - (oe > 0.99f ? 0.99 : oe64);
    }
    if (tt < 0.0001f) break;
    if (list) {
      list[cnt] = i;
      clampf[cnt] = oe > 0.99f;
    }
    cnt++;
    T = tt;
  }
  return cnt;
}

void orc_frame_free(orc_frame* F) {
  if (!F) return;
  free(F->P); free(F->g32); free(F->inst_tile); free(F->inst_pos); free(F->tile_start);
  free(F->pix_off); free(F->pix_list); free(F->pix_clamp);
  free(F->g64); free(F->gpix_off); free(F->gpix); free(F->v64);
  free(F);
}

static void eval64(const orc_frame* F, const double* P, double* image, orc_g64* Gs);

/* Decide (FP32 mirror) and evaluate (FP64).  ids: tree ids in selection
 * order; parameter arrays are indexed by tree id.  image: [H][W][3] FP64. */
orc_frame* orc_render(int64_t n, const int32_t* ids, const float* means, const float* ls, const float* quats,
                      const float* op, const float* sh, int n_coef, const orc_camera* C, const float* bg,
                      double* image) {
  orc_frame* F = (orc_frame*)calloc(1, sizeof(orc_frame));
  if (!F) return NULL;
  F->n = n; F->n_coef = n_coef; F->cam = *C;
  F->W = C->width; F->H = C->height;
  F->TX = (C->width + ORC_TILE - 1) / ORC_TILE;
  F->TY = (C->height + ORC_TILE - 1) / ORC_TILE;
  for (int k = 0; k < 3; ++k) F->bg[k] = bg ? (double)bg[k] : 0.0;
  const int np = 11 + n_coef;
  F->P = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * np);
  F->g32 = (orc_g32*)calloc((size_t)(n > 0 ? n : 1), sizeof(orc_g32));
  if (!F->P || !F->g32) { orc_frame_free(F); return NULL; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t id = ids[i];
    double* p = F->P + i * np;
    for (int k = 0; k < 3; ++k) p[k] = means[3 * id + k];
    for (int k = 0; k < 3; ++k) p[3 + k] = ls[3 * id + k];
    for (int k = 0; k < 4; ++k) p[6 + k] = quats[4 * id + k];
    p[10] = op[id];
    for (int k = 0; k < n_coef; ++k) p[11 + k] = sh[(int64_t)n_coef * id + k];
    orc_project32(means + 3 * id, ls + 3 * id, quats + 4 * id, op[id], C, F->TX, F->TY, F->g32 + i);
  }
  int64_t ni = 0;
  for (int64_t i = 0; i < n; ++i) ni += F->g32[i].tiles;
  F->n_inst = ni;
  orc_inst* inst = (orc_inst*)malloc(sizeof(orc_inst) * (size_t)(ni > 0 ? ni : 1));
  F->inst_tile = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ni > 0 ? ni : 1));
  F->inst_pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ni > 0 ? ni : 1));
  F->tile_start = (int64_t*)calloc((size_t)F->TX * F->TY + 1, sizeof(int64_t));
  if (!inst || !F->inst_tile || !F->inst_pos || !F->tile_start) { free(inst); orc_frame_free(F); return NULL; }
  /* instances emitted in selection order, tiles row-major, then sorted by
   * (tile, depth bits, selection position): the order of a stable sort of
   * the 64-bit key tile << 32 | depth bits. */
  int64_t e = 0;
  for (int64_t i = 0; i < n; ++i) {
    const orc_g32* G = F->g32 + i;
    if (!G->visible) continue;
    for (int ty = G->y0; ty < G->y1; ++ty)
      for (int tx = G->x0; tx < G->x1; ++tx) {
        inst[e].tile = (uint32_t)(ty * F->TX + tx);
        inst[e].depth = fbits(G->depth);
        inst[e].pos = (int32_t)i;
        ++e;
      }
  }
  qsort(inst, (size_t)ni, sizeof(orc_inst), cmp_inst);
  for (int64_t k = 0; k < ni; ++k) {
    F->inst_tile[k] = (int32_t)inst[k].tile;
    F->inst_pos[k] = inst[k].pos;
    F->tile_start[inst[k].tile + 1]++;
  }
  free(inst);
  for (int64_t t = 0; t < (int64_t)F->TX * F->TY; ++t) F->tile_start[t + 1] += F->tile_start[t];
  /* FP64 values of the visible splats for the decision log */
  F->v64 = (double*)calloc((size_t)(n > 0 ? n : 1) * 6, sizeof(double));
  if (!F->v64) { orc_frame_free(F); return NULL; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (!F->g32[i].visible) continue;
    orc_g64 G;
    orc_project64(F->P + i * np, n_coef, C, &G);
    double* V = F->v64 + 6 * i;
    V[0] = G.mx; V[1] = G.my; V[2] = G.ca; V[3] = G.cb; V[4] = G.cc; V[5] = G.o;
  }
  /* per-pixel contributor lists (CSR) */
  const int64_t npx = (int64_t)F->W * F->H;
  F->pix_off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(npx + 1));
  if (!F->pix_off) { orc_frame_free(F); return NULL; }
  int64_t l1 = 0, l2 = 0, l3 = 0, l4 = 0, l5 = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : l1, l2, l3, l4, l5)
  for (int64_t p = 0; p < npx; ++p) {
    int64_t lg[5] = {0, 0, 0, 0, 0};
    F->pix_off[p + 1] = pixel32(F, (int)(p % F->W), (int)(p / F->W), NULL, NULL, lg);
    l1 += lg[0];
    l2 += lg[1];
    l3 += lg[2];
    l4 += lg[3];
    l5 += lg[4];
  }
  F->skip_1ulp = l1;
  F->stop_1ulp = l2;
  F->skip_flip64 = l3;
  F->stop_flip64 = l4;
  F->clamp_flip64 = l5;
  free(F->v64);
  F->v64 = NULL;
  F->pix_off[0] = 0;
  for (int64_t p = 0; p < npx; ++p) F->pix_off[p + 1] += F->pix_off[p];
  int64_t tot = F->pix_off[npx];
  F->pix_list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
  F->pix_clamp = (uint8_t*)malloc((size_t)(tot > 0 ? tot : 1));
  if (!F->pix_list || !F->pix_clamp) { orc_frame_free(F); return NULL; }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < npx; ++p)
    pixel32(F, (int)(p % F->W), (int)(p / F->W), F->pix_list + F->pix_off[p], F->pix_clamp + F->pix_off[p], NULL);
  if (image) eval64(F, F->P, image, NULL);
  return F;
}

/* FP64 evaluation of the image with the frame's decisions frozen (the
 * contributor lists, alpha clamps and colour clamps of the FP32 mirror /
 * the unperturbed FP64 projection). */
static void eval64(const orc_frame* F, const double* P, double* image, orc_g64* Gs_out) {
  const int np = 11 + F->n_coef;
  orc_g64* Gs = Gs_out ? Gs_out : (orc_g64*)malloc(sizeof(orc_g64) * (size_t)(F->n > 0 ? F->n : 1));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < F->n; ++i)
    if (F->g32[i].visible) orc_project64(P + i * np, F->n_coef, &F->cam, Gs + i);
  const int64_t npx = (int64_t)F->W * F->H;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < npx; ++p) {
    double px = (double)(p % F->W) + 0.5, py = (double)(p / F->W) + 0.5;
    double T = 1.0, C[3] = {0, 0, 0};
    for (int64_t e = F->pix_off[p]; e < F->pix_off[p + 1]; ++e) {
      const orc_g64* G = Gs + F->pix_list[e];
      double dx = px - G->mx, dy = py - G->my;
      double power = -0.5 * (G->ca * dx * dx + G->cc * dy * dy) - G->cb * dx * dy;
      double alpha = F->pix_clamp[e] ? 0.99 : G->o * exp(power);
      for (int ch = 0; ch < 3; ++ch) C[ch] += G->rgb[ch] * alpha * T;
      T *= 1.0 - alpha;
    }
    for (int ch = 0; ch < 3; ++ch) image[3 * p + ch] = C[ch] + T * F->bg[ch];
  }
  if (!Gs_out) free(Gs);
}

/* Re-evaluate with perturbed FP64 parameters P ([n][11 + n_coef]) and the
 * frame's decisions frozen; colour clamps are re-derived from P. */
int orc_eval_frozen(const orc_frame* F, const double* P, double* image) {
  eval64(F, P, image, NULL);
  return 0;
}

/* Directional central difference of f(P) = sum(W * image(P)) along v for the
 * parameters of selected splat i only, decisions frozen, in FP64:
 *   (f(P + h v) - f(P - h v)) / (2 h).
 * Only the pixels that splat i contributes to change, so only those are
 * recomposited.  W: [H][W][3]; v: [11 + n_coef]. */
static int build_fd_index(orc_frame* F) {
  const int np = 11 + F->n_coef;
  const int64_t npx = (int64_t)F->W * F->H, tot = F->pix_off[npx];
  F->g64 = (orc_g64*)malloc(sizeof(orc_g64) * (size_t)(F->n > 0 ? F->n : 1));
  F->gpix_off = (int64_t*)calloc((size_t)F->n + 1, sizeof(int64_t));
  F->gpix = (int64_t*)malloc(sizeof(int64_t) * (size_t)(tot > 0 ? tot : 1));
  if (!F->g64 || !F->gpix_off || !F->gpix) return -1;
  for (int64_t i = 0; i < F->n; ++i)
    if (F->g32[i].visible) orc_project64(F->P + i * np, F->n_coef, &F->cam, F->g64 + i);
  for (int64_t e = 0; e < tot; ++e) F->gpix_off[F->pix_list[e] + 1]++;
  for (int64_t i = 0; i < F->n; ++i) F->gpix_off[i + 1] += F->gpix_off[i];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(F->n > 0 ? F->n : 1));
  if (!fill) return -1;
  memcpy(fill, F->gpix_off, sizeof(int64_t) * (size_t)F->n);
  for (int64_t p = 0; p < npx; ++p)
    for (int64_t e = F->pix_off[p]; e < F->pix_off[p + 1]; ++e) F->gpix[fill[F->pix_list[e]]++] = p;
  free(fill);
  return 0;
}

static double pixel_dot(const orc_frame* F, int64_t p, int64_t i, const orc_g64* Gi, const double* W) {
  double px = (double)(p % F->W) + 0.5, py = (double)(p / F->W) + 0.5;
  double T = 1.0, C[3] = {0, 0, 0};
  for (int64_t e = F->pix_off[p]; e < F->pix_off[p + 1]; ++e) {
    const orc_g64* G = F->pix_list[e] == i ? Gi : F->g64 + F->pix_list[e];
    double dx = px - G->mx, dy = py - G->my;
    double power = -0.5 * (G->ca * dx * dx + G->cc * dy * dy) - G->cb * dx * dy;
    double alpha = F->pix_clamp[e] ? 0.99 : G->o * exp(power);
    for (int ch = 0; ch < 3; ++ch) C[ch] += G->rgb[ch] * alpha * T;
    T *= 1.0 - alpha;
  }
  double acc = 0.0;
  for (int ch = 0; ch < 3; ++ch) acc += W[3 * p + ch] * (C[ch] + T * F->bg[ch]);
  return acc;
}

int orc_fd_directional(orc_frame* F, const double* W, int64_t i, const double* v, double h, double* out) {
  if (i < 0 || i >= F->n) return -1;
  if (!F->g64 && build_fd_index(F) != 0) return -2;
  *out = 0.0;
  if (!F->g32[i].visible) return 0;
  const int np = 11 + F->n_coef;
  double* P = (double*)malloc(sizeof(double) * (size_t)np);
  if (!P) return -2;
  orc_g64 Gp, Gm;
  for (int k = 0; k < np; ++k) P[k] = F->P[i * np + k] + h * v[k];
  orc_project64(P, F->n_coef, &F->cam, &Gp);
  for (int k = 0; k < np; ++k) P[k] = F->P[i * np + k] - h * v[k];
  orc_project64(P, F->n_coef, &F->cam, &Gm);
  free(P);
  double acc = 0.0;
  for (int64_t e = F->gpix_off[i]; e < F->gpix_off[i + 1]; ++e) {
    const int64_t p = F->gpix[e];
    acc += pixel_dot(F, p, i, &Gp, W) - pixel_dot(F, p, i, &Gm, W);
  }
  *out = acc / (2.0 * h);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Backward of the render (FP64, decisions frozen).  dL_dimg: [H][W][3].
 * grad2d: [n][9] = dL/d(mean2D x, y, conic a, b, c, opacity, r, g, b).
 * grad:   [n][11 + n_coef] = dL/d(mu, log-scale, raw quaternion, opacity
 * logit, SH), the raw parameters.  Either output may be NULL.  Per pixel,
 * walking the contributors back to front with the suffix colour S:
 *   dC/drgb_i = alpha_i T_i,  dC/dalpha_i = rgb_i T_i - S_i / (1 - alpha_i),
 * alpha clamped at 0.99 passes no gradient; otherwise dalpha/do = e and
 * dalpha/dpower = alpha.  The chain continues through the conic inverse, the
 * EWA Jacobian, the camera transform, the covariance factors, the quaternion
 * normalisation, the sigmoid and the SH basis (with the view-direction term). */
int orc_backward(const orc_frame* F, const double* dL_dimg, double* grad2d_out, double* grad_out) {
  const int np = 11 + F->n_coef;
  const int64_t n = F->n;
  orc_g64* Gs = (orc_g64*)malloc(sizeof(orc_g64) * (size_t)(n > 0 ? n : 1));
  double* g2 = (double*)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
  if (!Gs || !g2) { free(Gs); free(g2); return -1; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    if (F->g32[i].visible) orc_project64(F->P + i * np, F->n_coef, &F->cam, Gs + i);
  const int64_t npx = (int64_t)F->W * F->H;
  /* pixel loop; per-Gaussian accumulation is serialised per thread chunk by
   * an atomic update, which keeps the arithmetic exact to FP64 rounding. */
#pragma omp parallel
  {
    int64_t cap = 64;
    double* Tl = (double*)malloc(sizeof(double) * cap);
    double* Al = (double*)malloc(sizeof(double) * cap);
    double* El = (double*)malloc(sizeof(double) * cap);
#pragma omp for schedule(dynamic, 64)
    for (int64_t p = 0; p < npx; ++p) {
      int64_t b = F->pix_off[p], m = F->pix_off[p + 1] - b;
      if (m == 0) continue;
      if (m > cap) {
        cap = m * 2;
        Tl = (double*)realloc(Tl, sizeof(double) * cap);
        Al = (double*)realloc(Al, sizeof(double) * cap);
        El = (double*)realloc(El, sizeof(double) * cap);
      }
      double px = (double)(p % F->W) + 0.5, py = (double)(p / F->W) + 0.5;
      double T = 1.0;
      for (int64_t e = 0; e < m; ++e) {
        const orc_g64* G = Gs + F->pix_list[b + e];
        double dx = px - G->mx, dy = py - G->my;
        double power = -0.5 * (G->ca * dx * dx + G->cc * dy * dy) - G->cb * dx * dy;
        El[e] = exp(power);
        Al[e] = F->pix_clamp[b + e] ? 0.99 : G->o * El[e];
        Tl[e] = T;
        T *= 1.0 - Al[e];
      }
      const double* dC = dL_dimg + 3 * p;
      double S[3] = {T * F->bg[0], T * F->bg[1], T * F->bg[2]};
      for (int64_t e = m - 1; e >= 0; --e) {
        int32_t i = F->pix_list[b + e];
        const orc_g64* G = Gs + i;
        double a = Al[e], Ti = Tl[e];
        double dA = 0.0, gr[9];
        for (int ch = 0; ch < 3; ++ch) {
          gr[6 + ch] = dC[ch] * a * Ti;
          dA += dC[ch] * (G->rgb[ch] * Ti - S[ch] / (1.0 - a));
          S[ch] += G->rgb[ch] * a * Ti;
        }
        double dx = px - G->mx, dy = py - G->my;
        if (F->pix_clamp[b + e]) {
          gr[0] = gr[1] = gr[2] = gr[3] = gr[4] = gr[5] = 0.0;
        } else {
          double dpow = dA * a;  /* d alpha / d power = alpha */
          gr[5] = dA * El[e];    /* d alpha / d o = e          */
          gr[0] = dpow * (G->ca * dx + G->cb * dy);
          gr[1] = dpow * (G->cb * dx + G->cc * dy);
          gr[2] = dpow * (-0.5 * dx * dx);
          gr[3] = dpow * (-dx * dy);
          gr[4] = dpow * (-0.5 * dy * dy);
        }
        for (int k = 0; k < 9; ++k) {
#pragma omp atomic
          g2[9 * i + k] += gr[k];
        }
      }
    }
    free(Tl); free(Al); free(El);
  }
  if (grad2d_out) memcpy(grad2d_out, g2, sizeof(double) * 9 * (size_t)n);
  if (grad_out) {
    const orc_camera* C = &F->cam;
    double W[9];
    for (int i = 0; i < 9; ++i) W[i] = C->R[i];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double* out = grad_out + i * np;
      memset(out, 0, sizeof(double) * np);
      if (!F->g32[i].visible) continue;
      const orc_g64* G = Gs + i;
      const double* gg = g2 + 9 * i;
      const double* P = F->P + i * np;
      /* colour -> SH and view direction */
      double dRGB[3];
      for (int ch = 0; ch < 3; ++ch) dRGB[ch] = G->clamp[ch] ? 0.0 : gg[6 + ch];
      int nb = F->n_coef / 3;
      double d[3] = {G->dir[0] / G->dlen, G->dir[1] / G->dlen, G->dir[2] / G->dlen};
      double Y[16], dY[48];
      orc_sh_basis(d, Y, dY);
      double dd[3] = {0, 0, 0};
      for (int k = 0; k < nb; ++k)
        for (int ch = 0; ch < 3; ++ch) {
          out[11 + 3 * k + ch] = dRGB[ch] * Y[k];
          for (int a = 0; a < 3; ++a) dd[a] += dRGB[ch] * P[11 + 3 * k + ch] * dY[3 * k + a];
        }
      double dot = dd[0] * d[0] + dd[1] * d[1] + dd[2] * d[2];
      double dmu[3];
      for (int a = 0; a < 3; ++a) dmu[a] = (dd[a] - d[a] * dot) / G->dlen;
      /* opacity */
      out[10] = gg[5] * G->o * (1.0 - G->o);
      /* conic -> projected covariance: dSigma' = -Q G_Q Q */
      double Q[2][2] = {{G->ca, G->cb}, {G->cb, G->cc}};
      double GQ[2][2] = {{gg[2], 0.5 * gg[3]}, {0.5 * gg[3], gg[4]}};
      double QG[2][2], GS[2][2];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) QG[r][c] = Q[r][0] * GQ[0][c] + Q[r][1] * GQ[1][c];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) GS[r][c] = -(QG[r][0] * Q[0][c] + QG[r][1] * Q[1][c]);
      /* Sigma' = T Sigma T^T:  dL/dT = 2 GS T Sigma,  dL/dSigma = T^T GS T */
      double S3[3][3] = {{G->Sig[0], G->Sig[1], G->Sig[2]}, {G->Sig[1], G->Sig[3], G->Sig[4]}, {G->Sig[2], G->Sig[4], G->Sig[5]}};
      const double* T = G->T;
      double TS[2][3], dT[2][3], dSig[3][3];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) TS[r][c] = T[3 * r] * S3[0][c] + T[3 * r + 1] * S3[1][c] + T[3 * r + 2] * S3[2][c];
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) dT[r][c] = 2.0 * (GS[r][0] * TS[0][c] + GS[r][1] * TS[1][c]);
      for (int a = 0; a < 3; ++a)
        for (int b2 = 0; b2 < 3; ++b2) {
          double acc = 0.0;
          for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) acc += T[3 * r + a] * GS[r][c] * T[3 * c + b2];
          dSig[a][b2] = acc;
        }
      /* T = J W: dL/dJ = dT W^T (only J00, J02, J11, J12 vary) */
      double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
      for (int c = 0; c < 3; ++c) {
        dJ00 += dT[0][c] * W[c];
        dJ02 += dT[0][c] * W[6 + c];
        dJ11 += dT[1][c] * W[3 + c];
        dJ12 += dT[1][c] * W[6 + c];
      }
      double cx = G->c[0], cy = G->c[1], cz = G->c[2];
      double fx = C->fx, fy = C->fy, iz = 1.0 / cz, iz2 = iz * iz, iz3 = iz2 * iz;
      double dc[3];
      dc[0] = dJ02 * (-fx * iz2) + gg[0] * fx * iz;
      dc[1] = dJ12 * (-fy * iz2) + gg[1] * fy * iz;
      dc[2] = dJ00 * (-fx * iz2) + dJ02 * (2.0 * fx * cx * iz3) + dJ11 * (-fy * iz2) +
              dJ12 * (2.0 * fy * cy * iz3) + gg[0] * (-fx * cx * iz2) + gg[1] * (-fy * cy * iz2);
      for (int a = 0; a < 3; ++a) out[a] = W[a] * dc[0] + W[3 + a] * dc[1] + W[6 + a] * dc[2] + dmu[a];
      /* Sigma = M M^T, M = Rq diag(s) */
      double dM[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          dM[r][c] = 2.0 * (dSig[r][0] * G->M[c] + dSig[r][1] * G->M[3 + c] + dSig[r][2] * G->M[6 + c]);
      double dRq[9];
      for (int c = 0; c < 3; ++c) {
        double ds = 0.0;
        for (int r = 0; r < 3; ++r) {
          ds += dM[r][c] * G->Rq[3 * r + c];
          dRq[3 * r + c] = dM[r][c] * G->s[c];
        }
        out[3 + c] = ds * G->s[c];
      }
      double w = G->qn[0], x = G->qn[1], y = G->qn[2], z = G->qn[3];
      double dqn[4];
      dqn[0] = 2 * (-z * dRq[1] + y * dRq[2] + z * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
      dqn[1] = 2 * (y * dRq[1] + z * dRq[2] + y * dRq[3] - 2 * x * dRq[4] - w * dRq[5] + z * dRq[6] +
                    w * dRq[7] - 2 * x * dRq[8]);
      dqn[2] = 2 * (-2 * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + z * dRq[5] - w * dRq[6] +
                    z * dRq[7] - 2 * y * dRq[8]);
      dqn[3] = 2 * (-2 * z * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - 2 * z * dRq[4] + y * dRq[5] +
                    x * dRq[6] + y * dRq[7]);
      double qd = dqn[0] * G->qn[0] + dqn[1] * G->qn[1] + dqn[2] * G->qn[2] + dqn[3] * G->qn[3];
      for (int k = 0; k < 4; ++k) out[6 + k] = (dqn[k] - G->qn[k] * qd) / G->qlen;
    }
  }
  free(Gs);
  free(g2);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Accessors for tests. */
typedef struct orc_frame_info {
  int64_t n, n_inst, n_visible, n_contrib;
  int32_t TX, TY;
  int64_t skip_1ulp, stop_1ulp, skip_flip64, stop_flip64, clamp_flip64;
} orc_frame_info;

void orc_frame_get_info(const orc_frame* F, orc_frame_info* I) {
  I->n = F->n;
  I->n_inst = F->n_inst;
  int64_t v = 0;
  for (int64_t i = 0; i < F->n; ++i) v += F->g32[i].visible;
  I->n_visible = v;
  I->n_contrib = F->pix_off[(int64_t)F->W * F->H];
  I->TX = F->TX;
  I->TY = F->TY;
  I->skip_1ulp = F->skip_1ulp;
  I->stop_1ulp = F->stop_1ulp;
  I->skip_flip64 = F->skip_flip64;
  I->stop_flip64 = F->stop_flip64;
  I->clamp_flip64 = F->clamp_flip64;
}

/* Per-splat mirror outputs: depth bits, tiles, rect [x0,x1,y0,y1] and the
 * FP32 record [mxh, mxl, myh, myl, ce, se, h1, h2, o, radius]. */
void orc_frame_get_splats(const orc_frame* F, uint32_t* depth_bits, int32_t* tiles, int32_t* rect,
                          float* f32x10) {
  for (int64_t i = 0; i < F->n; ++i) {
    const orc_g32* G = F->g32 + i;
    if (depth_bits) depth_bits[i] = fbits(G->depth);
    if (tiles) tiles[i] = G->tiles;
    if (rect) { rect[4 * i] = G->x0; rect[4 * i + 1] = G->x1; rect[4 * i + 2] = G->y0; rect[4 * i + 3] = G->y1; }
    if (f32x10) {
      float* o = f32x10 + 10 * i;
      o[0] = G->mxh; o[1] = G->mxl; o[2] = G->myh; o[3] = G->myl; o[4] = G->ce;
      o[5] = G->se; o[6] = G->h1; o[7] = G->h2; o[8] = G->o; o[9] = G->radius;
    }
  }
}

void orc_frame_get_instances(const orc_frame* F, int32_t* tile, int32_t* pos) {
  for (int64_t k = 0; k < F->n_inst; ++k) {
    if (tile) tile[k] = F->inst_tile[k];
    if (pos) pos[k] = F->inst_pos[k];
  }
}

/* Per-pixel contributor count and final transmittance of the FP32 mirror. */
void orc_frame_get_pixel_counts(const orc_frame* F, int32_t* counts) {
  const int64_t npx = (int64_t)F->W * F->H;
  for (int64_t p = 0; p < npx; ++p) counts[p] = (int32_t)(F->pix_off[p + 1] - F->pix_off[p]);
}

/* Pixels each splat is composited into (the pruning statistic of the
 * appendix on densification details: a Gaussian that has not contributed for
 * long has its opacity zeroed): counts[i] = the number of pixels whose
 * contributor list holds selection position i. */
void orc_frame_get_splat_contrib(const orc_frame* F, int32_t* counts) {
  for (int64_t i = 0; i < F->n; ++i) counts[i] = 0;
  const int64_t m = F->pix_off[(int64_t)F->W * F->H];
  for (int64_t k = 0; k < m; ++k) counts[F->pix_list[k]]++;
}

/* FP64 per-splat values: mean2D, conic (a, b, c), opacity, rgb, depth. */
void orc_frame_get_values64(const orc_frame* F, double* out9) {
  const int np = 11 + F->n_coef;
  for (int64_t i = 0; i < F->n; ++i) {
    double* o = out9 + 9 * i;
    if (!F->g32[i].visible) { memset(o, 0, sizeof(double) * 9); continue; }
    orc_g64 G;
    orc_project64(F->P + i * np, F->n_coef, &F->cam, &G);
    o[0] = G.mx; o[1] = G.my; o[2] = G.ca; o[3] = G.cb; o[4] = G.cc; o[5] = G.o;
    o[6] = G.rgb[0]; o[7] = G.rgb[1]; o[8] = G.rgb[2];
  }
}

/* One splat's FP64 projection, for closed-form pins. out: [mx, my, A, B, C,
 * ca, cb, cc, o, rgb0, rgb1, rgb2, cz]. */
void orc_project64_one(const double* P, int n_coef, const orc_camera* C, double* out) {
  orc_g64 G;
  orc_project64(P, n_coef, C, &G);
  double v[13] = {G.mx, G.my, G.A, G.B, G.Cc, G.ca, G.cb, G.cc, G.o, G.rgb[0], G.rgb[1], G.rgb[2], G.c[2]};
  memcpy(out, v, sizeof v);
}

