// Host-side Hierarchical SPT construction (Sec. 4.3, "The Hierarchical SPT
// Datastructure"; SPT arrays of Sec. 4.1).  Builds the flattened layout that
// the device cut reads: the upper hierarchy in DFS preorder, then one segment
// per SPT sorted by r_max descending so that each view's candidate set is a
// prefix found by binary search.  The paper rebuilds this structure only after
// densification, on the CPU; here it runs once per scene.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "lodgs.h"
#include "lodgs_error.h"

namespace {

struct SptKey {
  float rmax, rmin;
  int32_t id;
  bool operator<(const SptKey& o) const {
    if (rmax != o.rmax) return rmax > o.rmax;
    if (rmin != o.rmin) return rmin > o.rmin;
    return id < o.id;
  }
};

}  // namespace

extern "C" int lodgs_hspt_build(int64_t n, const int32_t* left, const int32_t* right, int32_t root,
                                const float* ls, double log_size, int32_t* perm, float* r_min, float* r_max,
                                float* rho, int32_t* upper_parent, int32_t* spt_begin, int32_t* spt_parent,
                                int32_t* n_upper_out, int32_t* n_spt_out) {
  using lodgs::set_error;
  if (n <= 0 || n > (int64_t)INT32_MAX - 1 || !left || !right || !ls || !perm || !r_min || !r_max || !rho ||
      !upper_parent || !spt_begin || !spt_parent || !n_upper_out || !n_spt_out)
    return set_error(LODGS_E_INVALID, "lodgs_hspt_build: bad arguments");
  if (root < 0 || root >= n) return set_error(LODGS_E_INVALID, "lodgs_hspt_build: root out of range");
  try {
    // Tree sanity: children in range, each node has at most one parent.
    std::vector<int32_t> par((size_t)n, -1);
    for (int64_t i = 0; i < n; ++i) {
      int32_t a = left[i], b = right[i];
      if ((a < 0) != (b < 0)) return set_error(LODGS_E_INVALID, "lodgs_hspt_build: node with one child");
      if (a < 0) continue;
      if (a >= n || b >= n || a == b) return set_error(LODGS_E_INVALID, "lodgs_hspt_build: child out of range");
      if (par[a] >= 0 || par[b] >= 0) return set_error(LODGS_E_INVALID, "lodgs_hspt_build: node with two parents");
      par[a] = (int32_t)i;
      par[b] = (int32_t)i;
    }
    if (par[root] >= 0) return set_error(LODGS_E_INVALID, "lodgs_hspt_build: root has a parent");

    // Size metric g (Eq. 6's surface measure) and cull radius, FP64 -> FP32 once.
    std::vector<float> g((size_t)n), rh((size_t)n);
    std::vector<uint8_t> is_cut((size_t)n, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double s0 = std::exp((double)ls[3 * i]), s1 = std::exp((double)ls[3 * i + 1]),
             s2 = std::exp((double)ls[3 * i + 2]);
      double a = s0 * s1 + s0 * s2 + s1 * s2;
      g[i] = (float)std::sqrt(a);
      double m = s0 > s1 ? s0 : s1;
      m = m > s2 ? m : s2;
      rh[i] = (float)(3.0 * m);
    }

    // Left-first DFS of the upper hierarchy: upper nodes in preorder, SPT roots
    // in the order they are met (the volume BFS of Sec. 4.3 selects the same
    // cut set; the traversal order only fixes the layout).
    std::vector<int32_t> upper, roots, up_par_tree, root_par_tree;
    std::vector<int32_t> stack;
    std::vector<int32_t> stack_par;
    stack.push_back(root);
    stack_par.push_back(-1);
    int64_t visited = 0;
    while (!stack.empty()) {
      int32_t u = stack.back(), pu = stack_par.back();
      stack.pop_back();
      stack_par.pop_back();
      if (++visited > n) return set_error(LODGS_E_INVALID, "lodgs_hspt_build: cycle in the hierarchy");
      bool leaf = left[u] < 0;
      double lv = ((double)ls[3 * (int64_t)u] + (double)ls[3 * (int64_t)u + 1]) + (double)ls[3 * (int64_t)u + 2];
      if (leaf || lv < log_size) {
        is_cut[u] = 1;
        roots.push_back(u);
        root_par_tree.push_back(pu);
      } else {
        upper.push_back(u);
        up_par_tree.push_back(pu);
        stack.push_back(right[u]);
        stack_par.push_back(u);
        stack.push_back(left[u]);
        stack_par.push_back(u);
      }
    }
    const int64_t nu = (int64_t)upper.size(), ns = (int64_t)roots.size();

    // SPT sizes, then offsets.
    std::vector<int64_t> size((size_t)ns);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < ns; ++j) {
      std::vector<int32_t> st{roots[j]};
      int64_t k = 0;
      while (!st.empty()) {
        int32_t v = st.back();
        st.pop_back();
        ++k;
        if (left[v] >= 0) {
          st.push_back(left[v]);
          st.push_back(right[v]);
        }
      }
      size[j] = k;
    }
    std::vector<int64_t> off((size_t)ns + 1);
    off[0] = nu;
    for (int64_t j = 0; j < ns; ++j) off[j + 1] = off[j] + size[j];
    if (off[ns] != n) return set_error(LODGS_E_INVALID, "lodgs_hspt_build: nodes unreachable from the root");

    // Tree id -> layout position for the upper nodes (parents of roots and uppers).
    std::vector<int32_t> upos((size_t)n, -1);
    for (int64_t i = 0; i < nu; ++i) upos[upper[i]] = (int32_t)i;
    for (int64_t i = 0; i < nu; ++i) {
      perm[i] = upper[i];
      r_min[i] = g[upper[i]];
      r_max[i] = std::numeric_limits<float>::infinity();
      rho[i] = rh[upper[i]];
      upper_parent[i] = up_par_tree[i] < 0 ? -1 : upos[up_par_tree[i]];
    }
    for (int64_t j = 0; j <= ns; ++j) spt_begin[j] = (int32_t)off[j];
    for (int64_t j = 0; j < ns; ++j) spt_parent[j] = root_par_tree[j] < 0 ? -1 : upos[root_par_tree[j]];

    // Per SPT: intervals (r_min = g, 0 for leaves; r_max = prefix minimum of
    // the ancestors' g inside the SPT, +inf at the root), then the sort.
#pragma omp parallel
    {
      std::vector<SptKey> keys;
      std::vector<int32_t> st;
      std::vector<float> stm;
#pragma omp for schedule(dynamic, 16)
      for (int64_t j = 0; j < ns; ++j) {
        keys.clear();
        st.assign(1, roots[j]);
        stm.assign(1, std::numeric_limits<float>::infinity());
        while (!st.empty()) {
          int32_t v = st.back();
          float m = stm.back();
          st.pop_back();
          stm.pop_back();
          bool leaf = left[v] < 0;
          keys.push_back(SptKey{m, leaf ? 0.0f : g[v], v});
          if (!leaf) {
            float mc = std::fmin(g[v], m);
            st.push_back(left[v]);
            stm.push_back(mc);
            st.push_back(right[v]);
            stm.push_back(mc);
          }
        }
        std::sort(keys.begin(), keys.end());
        int64_t b = off[j];
        for (size_t e = 0; e < keys.size(); ++e) {
          perm[b + e] = keys[e].id;
          r_min[b + e] = keys[e].rmin;
          r_max[b + e] = keys[e].rmax;
          rho[b + e] = rh[keys[e].id];
        }
      }
    }
    *n_upper_out = (int32_t)nu;
    *n_spt_out = (int32_t)ns;
    return LODGS_OK;
  } catch (const std::bad_alloc&) {
    return set_error(LODGS_E_OOM, "lodgs_hspt_build: out of host memory");
  }
}
