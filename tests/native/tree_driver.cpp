// Host-only driver of the tree builder's C ABI, built with the address and undefined-behaviour
// sanitizers by tests/test_tree_sanitized.py: valid cuboids, graphs, whole-face trees, custom
// trees, merges, forests, bonds and exports, and malformed inputs that must be rejected.  Prints
// "ok" and exits 0 when every call returns what it should.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/hsc.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s (%s)\n", what, hsc_last_error());
    ++failures;
  }
}

struct Dev {
  int64_t n = 0;
  std::vector<int64_t> indptr;
  std::vector<int32_t> indices;
  std::vector<double> values;   // (re, im) pairs
  std::vector<int32_t> coords;  // [n][3]
  std::vector<int64_t> left, right;
};

// 7-point cuboid, on-site values from a seeded generator, contacts on x = 0 and x = nx - 1
Dev cuboid(int nx, int ny, int nz, unsigned seed) {
  Dev d;
  d.n = (int64_t)nx * ny * nz;
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> u(-0.5, 0.5);
  d.indptr.push_back(0);
  for (int64_t i = 0; i < d.n; ++i) {
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    d.coords.insert(d.coords.end(), {x, y, z});
    std::vector<std::pair<int64_t, double>> row{{i, u(rng)}};
    const int64_t st[3] = {1, nx, (int64_t)nx * ny};
    const int c[3] = {x, y, z}, sz[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      if (c[a] > 0) row.push_back({i - st[a], -1.0});
      if (c[a] < sz[a] - 1) row.push_back({i + st[a], -1.0});
    }
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      d.indices.push_back((int32_t)e.first);
      d.values.push_back(e.second);
      d.values.push_back(0.0);
    }
    d.indptr.push_back((int64_t)d.indices.size());
    if (x == 0) d.left.push_back(i);
    if (x == nx - 1) d.right.push_back(i);
  }
  return d;
}

hsc_status build(const Dev& d, int method, int leaf, int dense, hsc_tree** t, int mask = 7) {
  hsc_contact c[2] = {{(int64_t)d.left.size(), d.left.data(), 0.0, -1.0, -1.0},
                      {(int64_t)d.right.size(), d.right.data(), 0.0, -1.0, -1.0}};
  hsc_tree_opts o{};
  o.coords = method == 0 ? d.coords.data() : nullptr;
  o.split_mask = mask;
  o.leaf_side = leaf;
  o.method = method;
  o.dense_contacts = dense;
  return hsc_tree_build(d.n, d.indptr.data(), d.indices.data(), d.values.data(), 2, c, &o, t);
}

void inspect(hsc_tree* t) {
  hsc_tree_stats s{};
  expect(hsc_tree_stats_get(t, &s) == HSC_OK, "stats");
  std::vector<int64_t> perm(s.n_sites);
  std::vector<int32_t> par(s.n_clusters), first(s.n_clusters), size(s.n_clusters);
  std::vector<int64_t> fptr(s.n_clusters + 1);
  expect(hsc_tree_export(t, perm.data(), par.data(), first.data(), size.data(), fptr.data(), nullptr) == HSC_OK,
         "export");
  std::vector<int64_t> fs((size_t)fptr[s.n_clusters]);
  expect(hsc_tree_export(t, nullptr, nullptr, nullptr, nullptr, nullptr, fs.data()) == HSC_OK, "export fronts");
  std::vector<char> seen(s.n_sites, 0);
  for (int64_t p : perm) {
    expect(p >= 0 && p < s.n_sites && !seen[p], "perm is a permutation");
    if (p >= 0 && p < s.n_sites) seen[p] = 1;
  }
  int64_t cnt = 0;
  expect(hsc_tree_bonds(t, nullptr, &cnt) == HSC_OK && cnt > 0, "bond count");
  std::vector<int64_t> pairs(2 * cnt);
  int64_t cap = cnt;
  expect(hsc_tree_bonds(t, pairs.data(), &cap) == HSC_OK && cap == cnt, "bonds");
  int64_t small = cnt - 1;
  if (cnt > 1) expect(hsc_tree_bonds(t, pairs.data(), &small) == HSC_E_ARG, "bonds: capacity too small");
}

}  // namespace

int main() {
  // geometric and graph trees, whole-face trees, odd shapes
  const int shapes[][4] = {{6, 5, 4, 2}, {9, 3, 2, 3}, {2, 1, 11, 2}, {12, 1, 1, 2}, {8, 8, 8, 4}, {5, 7, 3, 2}};
  std::vector<hsc_tree*> keep;
  for (auto& sh : shapes) {
    const Dev d = cuboid(sh[0], sh[1], sh[2], (unsigned)(sh[0] * 100 + sh[1]));
    for (int method = 0; method < 2; ++method) {
      hsc_tree* t = nullptr;
      expect(build(d, method, sh[3], 0, &t) == HSC_OK, "build");
      if (t) {
        inspect(t);
        keep.push_back(t);
      }
    }
    if (sh[0] >= 2) {
      hsc_tree* t = nullptr;
      expect(build(d, 0, sh[3], 1, &t) == HSC_OK, "whole-face build");
      if (t) {
        inspect(t);
        hsc_tree* m = nullptr;
        expect(hsc_tree_merge(t, 0, nullptr, &m) == HSC_E_ARG || m == nullptr || hsc_tree_destroy(m) == HSC_OK,
               "merge of a whole-face tree");
        hsc_tree_destroy(t);
      }
    }
  }
  // merges and forests
  if (keep.size() >= 2) {
    hsc_tree_stats s{};
    hsc_tree_stats_get(keep[0], &s);
    std::vector<int32_t> ids;
    for (int c = 0; c + 1 < s.n_clusters; c += 2) ids.push_back(c);
    hsc_tree* m = nullptr;
    expect(hsc_tree_merge(keep[0], (int32_t)ids.size(), ids.data(), &m) == HSC_OK, "merge");
    if (m) { inspect(m); hsc_tree_destroy(m); }
    const int32_t root = s.n_clusters - 1;
    expect(hsc_tree_merge(keep[0], 1, &root, &m) == HSC_E_ARG, "merging the root is refused");
    const int32_t bad = s.n_clusters + 5;
    expect(hsc_tree_merge(keep[0], 1, &bad, &m) == HSC_E_ARG, "merging a missing cluster is refused");
    hsc_tree* f = nullptr;
    expect(hsc_tree_concat((int32_t)keep.size(), keep.data(), &f) == HSC_OK, "concat");
    if (f) { inspect(f); hsc_tree_destroy(f); }
  }
  for (hsc_tree* t : keep) hsc_tree_destroy(t);

  // custom trees: a chain of x slabs (valid), and partitions that do not separate (refused)
  {
    const Dev d = cuboid(6, 3, 2, 7);
    std::vector<int32_t> cl(d.n), parent(6);
    for (int64_t i = 0; i < d.n; ++i) cl[i] = (int32_t)(i % 6);
    for (int c = 0; c < 6; ++c) parent[c] = c + 1 < 6 ? c + 1 : -1;
    hsc_contact c[2] = {{(int64_t)d.left.size(), d.left.data(), 0.0, -1.0, -1.0},
                        {(int64_t)d.right.size(), d.right.data(), 0.0, -1.0, -1.0}};
    hsc_tree* t = nullptr;
    expect(hsc_tree_build_custom(d.n, d.indptr.data(), d.indices.data(), d.values.data(), 2, c, 6, cl.data(),
                                 parent.data(), &t) == HSC_OK, "custom chain");
    if (t) { inspect(t); hsc_tree_destroy(t); }
    std::vector<int32_t> p2 = {2, 2, -1, 2, 2, 2};   // slabs 3..5 hang off the root beside slabs 0, 1
    expect(hsc_tree_build_custom(d.n, d.indptr.data(), d.indices.data(), d.values.data(), 2, c, 6, cl.data(),
                                 p2.data(), &t) == HSC_E_ARG, "non-separating partition refused");
    std::vector<int32_t> p3 = {1, 2, 0, 4, 5, -1};    // a cycle
    expect(hsc_tree_build_custom(d.n, d.indptr.data(), d.indices.data(), d.values.data(), 2, c, 6, cl.data(),
                                 p3.data(), &t) == HSC_E_ARG, "cyclic parents refused");
    std::vector<int32_t> cl2 = cl;
    cl2[3] = 9;
    expect(hsc_tree_build_custom(d.n, d.indptr.data(), d.indices.data(), d.values.data(), 2, c, 6, cl2.data(),
                                 parent.data(), &t) == HSC_E_ARG, "cluster id out of range refused");
  }

  // malformed inputs
  {
    Dev d = cuboid(4, 3, 3, 3);
    hsc_tree* t = nullptr;
    Dev e = d;
    e.indices[5] = (int32_t)d.n + 3;
    expect(build(e, 0, 2, 0, &t) == HSC_E_ARG, "column index out of range");
    e = d;
    e.indptr[7] = e.indptr[6] - 1;
    expect(build(e, 0, 2, 0, &t) == HSC_E_ARG, "decreasing indptr");
    e = d;
    e.values[2 * 4] = std::nan("");
    expect(build(e, 0, 2, 0, &t) == HSC_E_NONFINITE, "non-finite value");
    e = d;
    for (size_t q = 0; q < e.indices.size(); ++q)
      if (e.indices[q] != 0 && q < (size_t)e.indptr[1]) { e.values[2 * q] = -0.7; break; }
    expect(build(e, 0, 2, 0, &t) == HSC_E_NOT_SYMMETRIC, "non-symmetric H");
    e = d;
    e.left.push_back(e.right[0]);
    expect(build(e, 0, 2, 0, &t) == HSC_E_ARG, "site in both contacts");
    e = d;
    e.left[0] = -4;
    expect(build(e, 0, 2, 0, &t) == HSC_E_ARG, "contact site out of range");
    expect(build(d, 0, 0, 0, &t) == HSC_E_ARG, "leaf side 0");
    expect(build(d, 2, 2, 0, &t) == HSC_E_ARG, "unknown method");
    Dev f = cuboid(5, 4, 4, 4);
    f.left.pop_back();   // a face with a hole is not a whole face
    expect(build(f, 0, 2, 1, &t) == HSC_E_ARG, "whole-face contact that is not a full face");
    expect(hsc_tree_build(-1, nullptr, nullptr, nullptr, 2, nullptr, nullptr, &t) == HSC_E_ARG, "negative n");
  }
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
