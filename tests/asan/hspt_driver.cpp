// Host-only driver for the HSPT builder under AddressSanitizer and
// UndefinedBehaviorSanitizer: random valid hierarchies (all output arrays
// checked for their own invariants) and malformed ones (which must be
// rejected), built with g++ alone.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lodgs.h"

namespace lodgs {
int set_error(int code, const char*) { return code; }
}  // namespace lodgs

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double next_unit() { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

struct Tree {
  int64_t n;
  int32_t root;
  std::vector<int32_t> left, right;
  std::vector<float> ls;
};

// Random topology by repeated merges of two random roots.
static Tree random_tree(int leaves) {
  Tree t;
  t.n = 2 * (int64_t)leaves - 1;
  t.left.assign(t.n, -1);
  t.right.assign(t.n, -1);
  t.ls.resize(3 * t.n);
  for (auto& x : t.ls) x = (float)(next_unit() * 4.0 - 3.0);
  std::vector<int32_t> roots;
  for (int i = 0; i < leaves; ++i) roots.push_back(i);
  int32_t nxt = leaves;
  while (roots.size() > 1) {
    size_t a = next_u64() % roots.size();
    int32_t ra = roots[a];
    roots.erase(roots.begin() + a);
    size_t b = next_u64() % roots.size();
    int32_t rb = roots[b];
    roots.erase(roots.begin() + b);
    t.left[nxt] = ra;
    t.right[nxt] = rb;
    roots.push_back(nxt++);
  }
  t.root = roots[0];
  return t;
}

static int build(const Tree& t, double thr, int32_t* nu_out, int32_t* ns_out, std::vector<int32_t>& perm) {
  const size_t n = (size_t)t.n;
  perm.assign(n, -1);
  std::vector<float> rmin(n), rmax(n), rho(n);
  std::vector<int32_t> up(n), sb(n + 1), sp(n);
  return lodgs_hspt_build(t.n, t.left.data(), t.right.data(), t.root, t.ls.data(), thr, perm.data(), rmin.data(),
                          rmax.data(), rho.data(), up.data(), sb.data(), sp.data(), nu_out, ns_out);
}

int main() {
  int failures = 0;
  for (int it = 0; it < 300; ++it) {
    const int leaves = 1 + (int)(next_u64() % 200);
    Tree t = random_tree(leaves);
    const double thr = next_unit() * 6.0 - 9.0;
    int32_t nu = 0, ns = 0;
    std::vector<int32_t> perm;
    if (build(t, thr, &nu, &ns, perm) != LODGS_OK) {
      std::printf("valid tree %d rejected\n", it);
      ++failures;
      continue;
    }
    std::vector<char> seen(t.n, 0);  // perm is a permutation
    for (int32_t p : perm) {
      if (p < 0 || p >= t.n || seen[p]) {
        std::printf("tree %d: perm is not a permutation\n", it);
        ++failures;
        break;
      }
      seen[p] = 1;
    }
    if (nu < 0 || ns < 1 || (int64_t)nu + ns > t.n) {
      std::printf("tree %d: counts %d %d\n", it, nu, ns);
      ++failures;
    }
    // malformed variants: each must be rejected without touching memory out of range
    if (t.n >= 3) {
      Tree m = t;
      m.right[m.root] = -1;  // a node with one child
      if (build(m, thr, &nu, &ns, perm) == LODGS_OK) ++failures;
      m = t;
      m.left[m.root] = (int32_t)(t.n + 5);  // a child out of range
      if (build(m, thr, &nu, &ns, perm) == LODGS_OK) ++failures;
      m = t;
      m.left[m.root] = m.root;  // a cycle through the root
      if (build(m, thr, &nu, &ns, perm) == LODGS_OK) ++failures;
    }
  }
  std::printf("%s\n", failures ? "FAIL" : "ok");
  return failures ? 1 : 0;
}
