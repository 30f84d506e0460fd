// Seeded synthetic inputs for the LoD-select + splat path.
//
// This module is the only code shared by the product path and the oracle.  It
// produces *data*: leaf Gaussians drawn from the workload distributions, a
// binary Gaussian hierarchy over them (median split, parents merged by moment
// matching, as the hierarchy creator that the paper reuses does, Sec. 3
// "Gaussian Hierarchies" and the initialisation appendix), and a volume
// threshold for the HSPT split (the per-scene `size` of Sec. 4.3).  It holds
// none of the per-view arithmetic (no LoD test, projection, sorting or
// blending).
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11), counter = (index, stream, draw),
// key = seed.  Every draw is addressable, so generation is parallel and the
// output does not depend on the thread count.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

struct P4 {
  uint32_t v[4];
};

inline P4 philox4x32_10(P4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * c.v[0];
    uint64_t p1 = (uint64_t)M1 * c.v[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    P4 n = {{hi1 ^ c.v[1] ^ k0, lo1, hi0 ^ c.v[3] ^ k1, lo0}};
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Uniform double in (0, 1): 53 random bits plus half an ulp.
inline double uni(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t j) {
  P4 c = {{(uint32_t)idx, (uint32_t)(idx >> 32), stream, j >> 1}};
  P4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  uint32_t a = r.v[(j & 1) * 2], b = r.v[(j & 1) * 2 + 1];
  uint64_t u = ((((uint64_t)a) << 32) | b) >> 11;
  return ((double)u + 0.5) * (1.0 / 9007199254740992.0);
}

// Standard normal by Box-Muller (cosine branch) from draws 2j, 2j+1.
inline double nrm(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t j) {
  double u1 = uni(seed, stream, idx, 2 * j), u2 = uni(seed, stream, idx, 2 * j + 1);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

enum : uint32_t { S_POS = 1, S_LS = 2, S_Q = 3, S_OP = 4, S_SH = 5, S_BOX = 7 };

}  // namespace

extern "C" {

// Leaf distribution.  kind 0: means uniform in [-half_extent, half_extent]^3.
// kind 1 (city): a fraction plane_frac of the leaves on the plane z = 0 with
// N(0, plane_sigma) jitter and xy uniform over the square extent, the rest
// uniform inside n_boxes axis-aligned boxes resting on z = 0 whose centres are
// uniform over the extent; footprint side U(side_lo, side_hi) per axis and
// height U(height_lo, height_hi), or cubes of one side U(side_lo, side_hi) when
// height_lo < 0.  Every leaf: log-scales N(ls_mean, ls_sd) per axis, rotation
// the normalised N(0, I4) quaternion (w, x, y, z), opacity logit N(0, op_sd),
// n_coef SH coefficients N(0, sh_sd) (layout [coef][rgb], coef-major).
typedef struct sg_leaf_params {
  int32_t kind;
  int32_t n_coef;  // 3 * (degree + 1)^2
  double half_extent;
  double plane_frac;
  double plane_sigma;
  int64_t n_boxes;
  double side_lo, side_hi, height_lo, height_hi;
  double ls_mean, ls_sd, sh_sd, op_sd;
} sg_leaf_params;

// Known-answer hook for the generator (tests check it against the published
// Philox4x32-10 test vector).
void sg_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  P4 c = {{ctr[0], ctr[1], ctr[2], ctr[3]}};
  P4 r = philox4x32_10(c, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = r.v[i];
}

double sg_uniform(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t j) {
  return uni(seed, stream, idx, j);
}

int sg_leaves(int64_t n, uint64_t seed, const sg_leaf_params* p, float* means, float* log_scales,
              float* quats, float* opacity_logits, float* sh) {
  if (n <= 0 || !p || p->n_coef < 3 || p->n_coef % 3) return -1;
  const int64_t n_plane = p->kind == 1 ? (int64_t)std::llround(p->plane_frac * (double)n) : 0;
  const double E = p->half_extent;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double x, y, z;
    if (p->kind == 0) {
      x = -E + 2.0 * E * uni(seed, S_POS, i, 0);
      y = -E + 2.0 * E * uni(seed, S_POS, i, 1);
      z = -E + 2.0 * E * uni(seed, S_POS, i, 2);
    } else if (i < n_plane || p->n_boxes <= 0) {
      x = -E + 2.0 * E * uni(seed, S_POS, i, 0);
      y = -E + 2.0 * E * uni(seed, S_POS, i, 1);
      z = p->plane_sigma * nrm(seed, S_POS, i, 2);
    } else {
      int64_t b = (int64_t)(uni(seed, S_POS, i, 0) * (double)p->n_boxes);
      if (b >= p->n_boxes) b = p->n_boxes - 1;
      double bx = -E + 2.0 * E * uni(seed, S_BOX, b, 0);
      double by = -E + 2.0 * E * uni(seed, S_BOX, b, 1);
      double sx, sy, h;
      if (p->height_lo < 0) {
        sx = sy = h = p->side_lo + (p->side_hi - p->side_lo) * uni(seed, S_BOX, b, 2);
      } else {
        sx = p->side_lo + (p->side_hi - p->side_lo) * uni(seed, S_BOX, b, 2);
        sy = p->side_lo + (p->side_hi - p->side_lo) * uni(seed, S_BOX, b, 3);
        h = p->height_lo + (p->height_hi - p->height_lo) * uni(seed, S_BOX, b, 4);
      }
      x = bx + (uni(seed, S_POS, i, 1) - 0.5) * sx;
      y = by + (uni(seed, S_POS, i, 2) - 0.5) * sy;
      z = uni(seed, S_POS, i, 3) * h;
    }
    means[3 * i + 0] = (float)x;
    means[3 * i + 1] = (float)y;
    means[3 * i + 2] = (float)z;
    for (int k = 0; k < 3; ++k) log_scales[3 * i + k] = (float)(p->ls_mean + p->ls_sd * nrm(seed, S_LS, i, k));
    double q[4], qn = 0.0;
    for (int k = 0; k < 4; ++k) {
      q[k] = nrm(seed, S_Q, i, k);
      qn += q[k] * q[k];
    }
    qn = std::sqrt(qn);
    if (!(qn > 0.0)) {
      q[0] = 1.0;
      q[1] = q[2] = q[3] = 0.0;
      qn = 1.0;
    }
    for (int k = 0; k < 4; ++k) quats[4 * i + k] = (float)(q[k] / qn);
    opacity_logits[i] = (float)(p->op_sd * nrm(seed, S_OP, i, 0));
    for (int k = 0; k < p->n_coef; ++k) sh[(int64_t)p->n_coef * i + k] = (float)(p->sh_sd * nrm(seed, S_SH, i, k));
  }
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Hierarchy: recursive median split of the leaf means on the longest AABB axis
// (left child = the floor(n/2) lowest by (coordinate, leaf id)), parents by
// moment matching with weights opacity x volume.
namespace {

struct Pt {
  float c[3];
  int32_t id;
};

struct Builder {
  int n_coef;
  float *means, *ls, *q, *op, *sh;
  int32_t *left, *right, *parent;
};

void sym_eig3(const double A_in[6], double lam[3], double V[9]) {
  // Cyclic Jacobi on a symmetric 3x3 (A stored as 00,01,02,11,12,22).
  double a[3][3] = {{A_in[0], A_in[1], A_in[2]}, {A_in[1], A_in[3], A_in[4]}, {A_in[2], A_in[4], A_in[5]}};
  double v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= 1e-36 * dia || off == 0.0) break;
    static const int PQ[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int k = 0; k < 3; ++k) {
      int p = PQ[k][0], r = PQ[k][1];
      double apq = a[p][r];
      if (apq == 0.0) continue;
      double theta = (a[r][r] - a[p][p]) / (2.0 * apq);
      double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
      double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
      for (int m = 0; m < 3; ++m) {  // A <- A G  (columns p, r)
        double amp = a[m][p], amr = a[m][r];
        a[m][p] = c * amp - s * amr;
        a[m][r] = s * amp + c * amr;
      }
      for (int m = 0; m < 3; ++m) {  // A <- G^T A (rows p, r)
        double apm = a[p][m], arm = a[r][m];
        a[p][m] = c * apm - s * arm;
        a[r][m] = s * apm + c * arm;
      }
      a[p][r] = a[r][p] = 0.0;
      for (int m = 0; m < 3; ++m) {
        double vmp = v[m][p], vmr = v[m][r];
        v[m][p] = c * vmp - s * vmr;
        v[m][r] = s * vmp + c * vmr;
      }
    }
  }
  int ord[3] = {0, 1, 2};
  std::sort(ord, ord + 3, [&](int i, int j) { return a[i][i] > a[j][j] || (a[i][i] == a[j][j] && i < j); });
  for (int k = 0; k < 3; ++k) {
    lam[k] = a[ord[k]][ord[k]];
    for (int m = 0; m < 3; ++m) V[3 * m + k] = v[m][ord[k]];  // column k
  }
  double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
               V[2] * (V[3] * V[7] - V[4] * V[6]);
  if (det < 0)
    for (int m = 0; m < 3; ++m) V[3 * m + 2] = -V[3 * m + 2];
}

void quat_to_rot(const double qin[4], double R[9]) {
  double n = std::sqrt(qin[0] * qin[0] + qin[1] * qin[1] + qin[2] * qin[2] + qin[3] * qin[3]);
  double w = qin[0] / n, x = qin[1] / n, y = qin[2] / n, z = qin[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

void rot_to_quat(const double m[9], double q[4]) {
  double tr = m[0] + m[4] + m[8], w, x, y, z;
  if (tr > 0) {
    double S = std::sqrt(tr + 1.0) * 2;
    w = 0.25 * S; x = (m[7] - m[5]) / S; y = (m[2] - m[6]) / S; z = (m[3] - m[1]) / S;
  } else if (m[0] > m[4] && m[0] > m[8]) {
    double S = std::sqrt(1.0 + m[0] - m[4] - m[8]) * 2;
    w = (m[7] - m[5]) / S; x = 0.25 * S; y = (m[1] + m[3]) / S; z = (m[2] + m[6]) / S;
  } else if (m[4] > m[8]) {
    double S = std::sqrt(1.0 + m[4] - m[0] - m[8]) * 2;
    w = (m[2] - m[6]) / S; x = (m[1] + m[3]) / S; y = 0.25 * S; z = (m[5] + m[7]) / S;
  } else {
    double S = std::sqrt(1.0 + m[8] - m[0] - m[4]) * 2;
    w = (m[3] - m[1]) / S; x = (m[2] + m[6]) / S; y = (m[5] + m[7]) / S; z = 0.25 * S;
  }
  double n = std::sqrt(w * w + x * x + y * y + z * z);
  double sg = w < 0 ? -1.0 : 1.0;
  q[0] = sg * w / n; q[1] = sg * x / n; q[2] = sg * y / n; q[3] = sg * z / n;
}

struct Moments {
  double w, mu[3], cov[6], o;
};

Moments node_moments(const Builder& B, int32_t i) {
  Moments M;
  double s[3], qd[4], R[9];
  for (int k = 0; k < 3; ++k) s[k] = std::exp((double)B.ls[3 * (int64_t)i + k]);
  for (int k = 0; k < 4; ++k) qd[k] = B.q[4 * (int64_t)i + k];
  quat_to_rot(qd, R);
  M.o = 1.0 / (1.0 + std::exp(-(double)B.op[i]));
  M.w = M.o * s[0] * s[1] * s[2];
  for (int k = 0; k < 3; ++k) M.mu[k] = B.means[3 * (int64_t)i + k];
  static const int IJ[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  for (int e = 0; e < 6; ++e) {
    int a = IJ[e][0], b = IJ[e][1];
    double acc = 0;
    for (int k = 0; k < 3; ++k) acc += R[3 * a + k] * s[k] * s[k] * R[3 * b + k];
    M.cov[e] = acc;
  }
  return M;
}

void merge(const Builder& B, int32_t p, int32_t a, int32_t b) {
  Moments A = node_moments(B, a), C = node_moments(B, b);
  double wa = A.w, wb = C.w;
  if (!(wa + wb > 0)) wa = wb = 1.0;
  double W = wa + wb;
  double mu[3], cov[6];
  for (int k = 0; k < 3; ++k) mu[k] = (wa * A.mu[k] + wb * C.mu[k]) / W;
  static const int IJ[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  double da[3], db[3];
  for (int k = 0; k < 3; ++k) {
    da[k] = A.mu[k] - mu[k];
    db[k] = C.mu[k] - mu[k];
  }
  for (int e = 0; e < 6; ++e) {
    int i = IJ[e][0], j = IJ[e][1];
    cov[e] = (wa * (A.cov[e] + da[i] * da[j]) + wb * (C.cov[e] + db[i] * db[j])) / W;
  }
  double lam[3], V[9], q[4];
  sym_eig3(cov, lam, V);
  rot_to_quat(V, q);
  for (int k = 0; k < 3; ++k) {
    B.means[3 * (int64_t)p + k] = (float)mu[k];
    double l = lam[k] > 1e-24 ? lam[k] : 1e-24;
    B.ls[3 * (int64_t)p + k] = (float)(0.5 * std::log(l));
  }
  for (int k = 0; k < 4; ++k) B.q[4 * (int64_t)p + k] = (float)q[k];
  double o = (wa * A.o + wb * C.o) / W;
  o = std::min(std::max(o, 1e-7), 1.0 - 1e-7);
  B.op[p] = (float)std::log(o / (1.0 - o));
  for (int k = 0; k < B.n_coef; ++k)
    B.sh[(int64_t)B.n_coef * p + k] =
        (float)((wa * B.sh[(int64_t)B.n_coef * a + k] + wb * B.sh[(int64_t)B.n_coef * b + k]) / W);
}

// Builds the subtree over pts[lo, hi); internal nodes take ids base, base+1, ...
// in preorder.  Returns the subtree's root id.
int32_t build(const Builder& B, Pt* pts, int64_t lo, int64_t hi, int32_t base) {
  if (hi - lo == 1) return pts[lo].id;
  float mn[3] = {pts[lo].c[0], pts[lo].c[1], pts[lo].c[2]}, mx[3] = {mn[0], mn[1], mn[2]};
  for (int64_t i = lo + 1; i < hi; ++i)
    for (int k = 0; k < 3; ++k) {
      mn[k] = std::min(mn[k], pts[i].c[k]);
      mx[k] = std::max(mx[k], pts[i].c[k]);
    }
  int ax = 0;
  double ext = (double)mx[0] - (double)mn[0];
  for (int k = 1; k < 3; ++k)
    if ((double)mx[k] - (double)mn[k] > ext) {
      ext = (double)mx[k] - (double)mn[k];
      ax = k;
    }
  int64_t m = lo + (hi - lo) / 2;
  std::nth_element(pts + lo, pts + m, pts + hi, [ax](const Pt& u, const Pt& v) {
    return u.c[ax] < v.c[ax] || (u.c[ax] == v.c[ax] && u.id < v.id);
  });
  int32_t node = base;
  int32_t lbase = base + 1, rbase = base + (int32_t)(m - lo);
  int32_t l, r;
  if (hi - lo > (1 << 15)) {
#pragma omp task shared(l)
    l = build(B, pts, lo, m, lbase);
#pragma omp task shared(r)
    r = build(B, pts, m, hi, rbase);
#pragma omp taskwait
  } else {
    l = build(B, pts, lo, m, lbase);
    r = build(B, pts, m, hi, rbase);
  }
  B.left[node] = l;
  B.right[node] = r;
  B.parent[l] = node;
  B.parent[r] = node;
  merge(B, node, l, r);
  return node;
}

}  // namespace

extern "C" {

// Arrays hold 2n-1 nodes.  Leaves occupy ids [0, n) and must be filled on
// entry; internal nodes get ids [n, 2n-1) in preorder (root = n when n > 1).
// left/right are -1 for leaves, parent is -1 for the root.
int sg_build_hierarchy(int64_t n, int32_t n_coef, float* means, float* log_scales, float* quats,
                       float* opacity_logits, float* sh, int32_t* left, int32_t* right, int32_t* parent,
                       int32_t* root) {
  if (n <= 0 || 2 * n - 1 > INT32_MAX || n_coef < 3) return -1;
  Builder B{n_coef, means, log_scales, quats, opacity_logits, sh, left, right, parent};
  const int64_t nn = 2 * n - 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nn; ++i) {
    left[i] = right[i] = parent[i] = -1;
  }
  std::vector<Pt> pts((size_t)n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) pts[i].c[k] = means[3 * i + k];
    pts[i].id = (int32_t)i;
  }
  int32_t r = 0;
#pragma omp parallel
#pragma omp single
  r = build(B, pts.data(), 0, n, (int32_t)n);
  *root = r;
  return 0;
}

// The k-th largest (k >= 1) node log-volume, log(s1 s2 s3) evaluated as
// ((double)ls0 + (double)ls1) + (double)ls2.  Used to pick the HSPT volume
// threshold so that about k nodes lie above it.
double sg_log_volume_kth_largest(int64_t n, const float* log_scales, int64_t k) {
  if (n <= 0) return 0.0;
  if (k < 1) k = 1;
  if (k > n) k = n;
  std::vector<double> lv((size_t)n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    lv[i] = ((double)log_scales[3 * i] + (double)log_scales[3 * i + 1]) + (double)log_scales[3 * i + 2];
  std::nth_element(lv.begin(), lv.begin() + (k - 1), lv.end(), std::greater<double>());
  return lv[(size_t)(k - 1)];
}

}  // extern "C"
