// Host-side cluster tree: geometric multilevel nested dissection (Section 2.2),
// point-level fronts, relative index maps, and the per-energy operation count.
#include <algorithm>
#include <climits>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "hsc_internal.h"

namespace hsc {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

static std::atomic<uint64_t> g_uid{1};

namespace {

// Recursive bisection.  A cluster whose box still has a splittable axis becomes
// a separator (the one-site plane) with up to two children; otherwise a leaf.
struct NDBuilder {
  const hsc_tree* t;
  std::vector<std::vector<int64_t>> sites_of;
  std::vector<std::vector<int>> kids_of;

  int rec(std::vector<int64_t>& sites) {
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int64_t s : sites)
      for (int a = 0; a < 3; ++a) {
        int32_t c = t->coords[3 * s + a];
        lo[a] = std::min(lo[a], c);
        hi[a] = std::max(hi[a], c);
      }
    int best = -1;
    int64_t best_ext = 0;
    for (int a = 0; a < 3; ++a) {
      if (!((t->split_mask >> a) & 1)) continue;
      int64_t ext = (int64_t)hi[a] - lo[a] + 1;
      if (ext <= t->leaf_side || ext < 3) continue;
      if (ext > best_ext) { best_ext = ext; best = a; }
    }
    std::vector<int> kids;
    std::vector<int64_t> mine;
    if (best >= 0) {
      int32_t cut = lo[best] + (int32_t)(best_ext / 2);
      std::vector<int64_t> left, right;
      for (int64_t s : sites) {
        int32_t c = t->coords[3 * s + best];
        if (c < cut) left.push_back(s);
        else if (c > cut) right.push_back(s);
        else mine.push_back(s);
      }
      if (mine.empty()) {          // no plane there: keep the box whole
        mine.swap(sites);
      } else {
        std::vector<int64_t>().swap(sites);
        if (!left.empty()) kids.push_back(rec(left));
        if (!right.empty()) kids.push_back(rec(right));
      }
    } else {
      mine.swap(sites);
    }
    sites_of.push_back(std::move(mine));
    kids_of.push_back(std::move(kids));
    return (int)sites_of.size() - 1;
  }
};

// Graph nested dissection (for H without usable coordinates): bisect a site set by breadth-first
// level sets of its graph.  From a pseudo-peripheral site (the last site reached from the set's
// first site, then the last one reached from it) the levels L_0, L_1, ... of the set's component
// are formed; the separator is the level that best balances the sites below and above it (every
// path between the two sides crosses it), sites of other components join the lower side (no
// edge reaches them).  Stop at sets of at most `leaf` sites, or when no level separates.
struct GraphND {
  const hsc_tree* t;
  int64_t leaf;
  std::vector<std::vector<int64_t>> sites_of;
  std::vector<std::vector<int>> kids_of;
  std::vector<int32_t> mark, level;
  int32_t stamp = 0;
  GraphND(const hsc_tree* t_, int64_t leaf_) : t(t_), leaf(leaf_), mark(t_->n, 0), level(t_->n, -1) {}

  // levels from src inside the current mark; returns the sites in visiting order
  std::vector<int64_t> bfs(int64_t src) {
    std::vector<int64_t> order{src};
    level[src] = 0;
    for (size_t h = 0; h < order.size(); ++h) {
      const int64_t r = order[h];
      for (int64_t q = t->indptr[r]; q < t->indptr[r + 1]; ++q) {
        const int64_t c = t->indices[q];
        if (mark[c] != stamp || level[c] >= 0) continue;
        level[c] = level[r] + 1;
        order.push_back(c);
      }
    }
    return order;
  }

  int leaf_of(std::vector<int64_t>& sites) {
    sites_of.push_back(std::move(sites));
    kids_of.push_back({});
    return (int)sites_of.size() - 1;
  }

  int rec(std::vector<int64_t>& sites) {
    if ((int64_t)sites.size() <= leaf) return leaf_of(sites);
    ++stamp;
    for (int64_t s : sites) { mark[s] = stamp; level[s] = -1; }
    std::vector<int64_t> order = bfs(sites[0]);
    for (int pass = 0; pass < 2; ++pass) {
      const int64_t far = order.back();
      for (int64_t s : order) level[s] = -1;
      order = bfs(far);
    }
    const int depth = level[order.back()];
    if (depth < 2) {   // no level has sites on both sides
      for (int64_t s : sites) level[s] = -1;
      return leaf_of(sites);
    }
    std::vector<int64_t> count(depth + 1, 0);
    for (int64_t s : order) count[level[s]]++;
    const int64_t others = (int64_t)sites.size() - (int64_t)order.size();
    int best = 1;
    int64_t best_cost = INT64_MAX, below = others + count[0];
    for (int m = 1; m < depth; ++m) {
      const int64_t above = (int64_t)sites.size() - below - count[m];
      const int64_t cost = std::max(below, above) + count[m];
      if (cost < best_cost) { best_cost = cost; best = m; }
      below += count[m];
    }
    std::vector<int64_t> lo, hi, sep;
    for (int64_t s : sites) {
      const int l = level[s];
      if (l == best) sep.push_back(s);
      else if (l > best) hi.push_back(s);
      else lo.push_back(s);   // lower levels and the unreached components
      level[s] = -1;
    }
    std::vector<int64_t>().swap(sites);
    std::vector<int> kids;
    if (!lo.empty()) kids.push_back(rec(lo));
    if (!hi.empty()) kids.push_back(rec(hi));
    sites_of.push_back(std::move(sep));
    kids_of.push_back(std::move(kids));
    return (int)sites_of.size() - 1;
  }
};

// Whole-face contacts (dense self-energy blocks): each face must sit inside one cluster that is an
// ancestor of every cluster touching it, or the dense block would couple sibling clusters.  With
// d(s) the distance of site s from the left face along the normal axis and N planes in all:
//   N >= 4: root = plane d = N/2; its children are the two faces, each the parent of the nested
//           dissection of the planes between it and the root (the right face is a leaf when no
//           plane lies between them);
//   N = 2, 3: the left face is the root of a chain (middle plane, if any, then the right face).
// The left face is never a leaf, so its full diagonal block of every lesser channel is formed.
void build_dense(hsc_tree* t, NDBuilder& b) {
  const int64_t n = t->n;
  auto crd = [&](int64_t s, int a) { return t->coords[3 * s + a]; };
  int ax = -1;
  for (int a = 0; a < 3 && ax < 0; ++a) {
    bool flat = true;
    for (int k = 0; k < 2 && flat; ++k) {
      const auto& v = t->contact[k].sites;
      for (int64_t s : v) flat = flat && crd(s, a) == crd(v[0], a);
    }
    if (flat && crd(t->contact[0].sites[0], a) != crd(t->contact[1].sites[0], a)) ax = a;
  }
  if (ax < 0) throw std::string("dense contacts: the two contacts are not parallel faces");
  const int32_t x0 = crd(t->contact[0].sites[0], ax), x1 = crd(t->contact[1].sites[0], ax);
  const int32_t sgn = x1 > x0 ? 1 : -1;
  const int64_t planes = (int64_t)(x1 - x0) * sgn + 1;
  std::vector<int32_t> dist(n);
  std::vector<int64_t> per_plane(planes, 0);
  for (int64_t s = 0; s < n; ++s) {
    const int64_t d = (int64_t)(crd(s, ax) - x0) * sgn;
    if (d < 0 || d >= planes) throw std::string("dense contacts: a site lies outside the slab between the faces");
    dist[s] = (int32_t)d;
    per_plane[d]++;
  }
  for (int k = 0; k < 2; ++k) {
    const auto& v = t->contact[k].sites;
    FaceInfo& f = t->face[k];
    int q = 0;
    for (int a = 0; a < 3; ++a)
      if (a != ax) f.ax[q++] = a;
    int32_t hi[2];
    for (int q2 = 0; q2 < 2; ++q2) {
      f.lo[q2] = INT32_MAX;
      hi[q2] = INT32_MIN;
      for (int64_t s : v) {
        f.lo[q2] = std::min(f.lo[q2], crd(s, f.ax[q2]));
        hi[q2] = std::max(hi[q2], crd(s, f.ax[q2]));
      }
      f.dim[q2] = hi[q2] - f.lo[q2] + 1;
    }
    if ((int64_t)f.dim[0] * f.dim[1] != (int64_t)v.size() || per_plane[k == 0 ? 0 : planes - 1] != (int64_t)v.size())
      throw std::string("dense contacts: a contact is not a whole rectangular end plane of the device");
    std::vector<char> seen((size_t)f.dim[0] * f.dim[1], 0);
    for (int64_t s : v) {
      char& c = seen[(size_t)(crd(s, f.ax[0]) - f.lo[0]) * f.dim[1] + (crd(s, f.ax[1]) - f.lo[1])];
      if (c) throw std::string("dense contacts: two sites of a face share a position");
      c = 1;
    }
  }
  auto slab = [&](int64_t a, int64_t bnd) {   // sites with a <= d < bnd
    std::vector<int64_t> v;
    for (int64_t s = 0; s < n; ++s)
      if (dist[s] >= a && dist[s] < bnd) v.push_back(s);
    return v;
  };
  auto push = [&](std::vector<int64_t> sites, std::vector<int> kids) {
    b.sites_of.push_back(std::move(sites));
    b.kids_of.push_back(std::move(kids));
    return (int)b.sites_of.size() - 1;
  };
  if (planes <= 3) {
    const int r = push(slab(planes - 1, planes), {});
    t->face[1].cluster = r;
    int top = r;
    if (planes == 3) top = push(slab(1, 2), {r});
    t->face[0].cluster = push(slab(0, 1), {top});
    return;
  }
  const int64_t cut = planes / 2;
  std::vector<int64_t> inner = slab(1, cut);
  const int li = b.rec(inner);
  t->face[0].cluster = push(slab(0, 1), {li});
  std::vector<int> rk;
  if (cut + 1 < planes - 1) {
    std::vector<int64_t> rin = slab(cut + 1, planes - 1);
    rk.push_back(b.rec(rin));
  }
  t->face[1].cluster = push(slab(planes - 1, planes), rk);
  push(slab(cut, cut + 1), {t->face[0].cluster, t->face[1].cluster});
}

}  // namespace

int finalize_tree(hsc_tree* t, std::vector<std::vector<int64_t>>& sites_of) {
  const int nc = (int)t->cl.size();
  const int64_t n = t->n;
  // parents, depth, subtree ranges
  for (int i = 0; i < nc; ++i) t->cl[i].parent = -1;
  for (int i = 0; i < nc; ++i)
    for (int k : t->cl[i].children) t->cl[k].parent = i;
  for (int i = 0; i < nc; ++i) {
    int lo = i;
    for (int k : t->cl[i].children) lo = std::min(lo, t->cl[k].lo);
    t->cl[i].lo = lo;
  }
  t->depth = 0;
  for (int i = nc - 1; i >= 0; --i) {
    int p = t->cl[i].parent;
    t->cl[i].depth = p < 0 ? 0 : t->cl[p].depth + 1;
    t->depth = std::max(t->depth, t->cl[i].depth + 1);
  }
  // within a cluster: left-contact sites, right-contact sites, then the rest
  t->owner.assign(n, -1);
  t->perm.clear();
  t->perm.reserve(n);
  for (int i = 0; i < nc; ++i) {
    auto& v = sites_of[i];
    std::sort(v.begin(), v.end(), [&](int64_t a, int64_t b) {
      int ka = t->side[a] < 0 ? 2 : t->side[a], kb = t->side[b] < 0 ? 2 : t->side[b];
      return ka != kb ? ka < kb : a < b;
    });
    Cluster& c = t->cl[i];
    c.first = (int64_t)t->perm.size();
    c.n = (int)v.size();
    c.n_left = c.n_right = 0;
    for (int64_t s : v) {
      if (t->owner[s] >= 0) { set_error("internal: site in two clusters"); return HSC_E_ARG; }
      t->owner[s] = i;
      t->perm.push_back(s);
      if (t->side[s] == 0) c.n_left++;
      if (t->side[s] == 1) c.n_right++;
    }
  }
  if ((int64_t)t->perm.size() != n) { set_error("internal: sites lost in the tree"); return HSC_E_ARG; }
  t->pos.assign(n, 0);
  for (int64_t p = 0; p < n; ++p) t->pos[t->perm[p]] = p;
  // separation check: every edge joins a cluster and one of its ancestors/descendants
  for (int64_t r = 0; r < n; ++r)
    for (int64_t q = t->indptr[r]; q < t->indptr[r + 1]; ++q) {
      int64_t c = t->indices[q];
      int a = t->owner[r], b = t->owner[c];
      if (a == b) continue;
      int lo_ = std::min(a, b), hi_ = std::max(a, b);
      if (!(t->cl[hi_].lo <= lo_)) {
        set_error("the clusters do not separate the graph of H (edge " + std::to_string(r) + "-" +
                  std::to_string(c) + " crosses a separator)");
        return HSC_E_ARG;
      }
    }
  // contact paths
  for (int i = 0; i < nc; ++i) {
    Cluster& c = t->cl[i];
    c.lpath = c.n_left > 0;
    c.rpath = c.n_right > 0;
    for (int k : c.children) {
      c.lpath = c.lpath || t->cl[k].lpath;
      c.rpath = c.rpath || t->cl[k].rpath;
    }
  }
  // point-level fronts, bottom-up: ancestor sites adjacent to the subtree
  std::vector<int64_t> stamp(n, -1);
  for (int i = 0; i < nc; ++i) {
    Cluster& c = t->cl[i];
    std::vector<int64_t> cand;
    auto consider = [&](int64_t s) {
      int o = t->owner[s];
      if (o >= c.lo && o <= i) return;        // inside the subtree
      if (stamp[s] == i) return;
      stamp[s] = i;
      cand.push_back(s);
    };
    for (int64_t p = c.first; p < c.first + c.n; ++p) {
      int64_t r = t->perm[p];
      for (int64_t q = t->indptr[r]; q < t->indptr[r + 1]; ++q) consider(t->indices[q]);
    }
    for (int k : c.children)
      for (int64_t s : t->cl[k].front) consider(s);
    std::sort(cand.begin(), cand.end(), [&](int64_t a, int64_t b) { return t->pos[a] < t->pos[b]; });
    c.front.swap(cand);
  }
  // relative maps
  std::vector<int32_t> fidx(n, -1);
  for (int i = 0; i < nc; ++i) {
    Cluster& c = t->cl[i];
    c.rel.assign(c.front.size(), -1);
    c.frontpos.assign(c.front.size(), -1);
    // offsets of each ancestor in the list (parent, grandparent, ..., root)
    std::vector<std::pair<int, int64_t>> anc;
    int64_t off = 0;
    for (int p = c.parent; p >= 0; p = t->cl[p].parent) {
      anc.push_back({p, off});
      off += t->cl[p].n;
    }
    c.n_anc = off;
    if (c.parent < 0) {
      if (!c.front.empty()) { set_error("internal: root has a front"); return HSC_E_ARG; }
      continue;
    }
    const Cluster& pc = t->cl[c.parent];
    for (size_t k = 0; k < pc.front.size(); ++k) fidx[pc.front[k]] = (int32_t)k;
    for (size_t k = 0; k < c.front.size(); ++k) {
      int64_t s = c.front[k];
      int o = t->owner[s];
      if (o == c.parent) c.rel[k] = (int32_t)(t->pos[s] - pc.first);
      else if (fidx[s] >= 0) c.rel[k] = pc.n + fidx[s];
      for (auto& a : anc)
        if (a.first == o) c.frontpos[k] = (int32_t)(a.second + (t->pos[s] - t->cl[o].first));
      if (c.rel[k] < 0 || c.frontpos[k] < 0) {
        set_error("internal: front site outside the parent's frontal set");
        return HSC_E_ARG;
      }
    }
    for (size_t k = 0; k < pc.front.size(); ++k) fidx[pc.front[k]] = -1;
  }
  t->uid = g_uid.fetch_add(1);
  return HSC_OK;
}

// Real flops of one energy (complex FMA = 8 real flops), following the steps
// the solver executes for the requested outputs.
double flops_per_energy(const hsc_tree* t, uint32_t want) {
  double fl = 0;
  const bool need_gl = want & (HSC_DIAG_GL | HSC_TRANS | HSC_SPECTRAL_LR | HSC_BOND_GL);
  for (const auto& c : t->cl) {
    double n = c.n, f = c.f(), P = (double)c.n_anc;
    bool leaf = c.children.empty();
    double nc = c.n_left + c.n_right;
    fl += 8 * n * n * n + 8 * n * n * f + 8 * f * f * n;          // fold
    if (c.parent < 0) continue;
    if (need_gl && c.cpath()) {
      if (leaf) fl += 8 * n * f * f + 8 * n * f + 8 * nc * f * P + 8 * nc * f * n;
      else fl += 8 * n * f * P + 8 * n * n * f;
    } else {
      fl += leaf ? 8 * n * f * f + 8 * n * f : 8 * n * f * f + 8 * n * n * f;
    }
  }
  if (t->dense)
    for (int k = 0; k < 2; ++k) {
      // dense face self-energy in two separable mode sums (5 flops per term: one real product of
      // two sine factors, then a real-times-complex multiply-add)
      const double d1 = t->face[k].dim[0], d2 = t->face[k].dim[1], F = d1 * d2;
      fl += 5 * d1 * d2 * d2 * d2 + 5 * F * F * d1;
      // Gamma times the face's G rows, once per energy for every lesser channel
      const Cluster& c = t->cl[t->face[k].cluster];
      if (need_gl) fl += 8 * F * F * (c.n + (double)c.n_anc);
    }
  if (!need_gl) return fl;
  // channels: (fold-set, extract-set) as chosen by the solver
  struct Ch { int fold; int extract; };   // 0 = both sides, 1 = left, 2 = right, 3 = none
  std::vector<Ch> chans;
  if (want & HSC_SPECTRAL_LR) {
    chans.push_back({1, 0});
    chans.push_back({2, 0});
    if (want & HSC_BOND_GL) chans.push_back({0, 0});
  } else {
    if (want & (HSC_DIAG_GL | HSC_BOND_GL)) chans.push_back({0, 0});
    if (want & HSC_TRANS) chans.push_back({2, 1});
  }
  for (auto ch : chans)
    for (const auto& c : t->cl) {
      double n = c.n, f = c.f(), P = (double)c.n_anc;
      bool leaf = c.children.empty();
      bool in_fold = ch.fold == 0 ? c.cpath() : ch.fold == 1 ? c.lpath : c.rpath;
      bool in_ext = ch.extract == 0 ? true : c.lpath;
      if (in_fold) {
        double rows = leaf ? (ch.fold == 0 ? c.n_left + c.n_right : ch.fold == 1 ? c.n_left : c.n_right) : n;
        fl += 8 * f * rows * P + 8 * n * rows * (n + f);
      }
      if (in_ext && c.parent >= 0) fl += leaf ? 8 * n * f * f + 8 * n * f : 8 * n * f * f + 8 * n * n * f;
    }
  return fl;
}

std::vector<int64_t> tree_bonds(const hsc_tree* t) {
  std::vector<int64_t> out;
  std::vector<int32_t> cols;
  for (int64_t r = 0; r < t->n; ++r) {
    cols.clear();
    for (int64_t q = t->indptr[r]; q < t->indptr[r + 1]; ++q)
      if (t->indices[q] > r) cols.push_back(t->indices[q]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    for (int32_t c : cols) {
      out.push_back(r);
      out.push_back(c);
    }
  }
  return out;
}

double bytes_per_energy(const hsc_tree* t, uint32_t want) {
  double b = 0;
  const bool need_gl = want & (HSC_DIAG_GL | HSC_TRANS | HSC_SPECTRAL_LR | HSC_BOND_GL);
  for (const auto& c : t->cl) {
    double n = c.n, f = c.f(), P = (double)c.n_anc;
    b += 16 * ((n + f) * (n + f) + n * n + n * f);               // frontal, inverse, Psi
    if (!c.children.empty()) b += 16 * (n + f) * (n + (need_gl && c.cpath() ? P : f));
    if (need_gl && c.cpath()) b += 16 * 2 * ((n + f) * (n + P) + n * (n + f));
    if (need_gl && !c.children.empty()) b += 16 * 2 * (n + f) * (n + f);
  }
  return b;
}

}  // namespace hsc

using namespace hsc;

extern "C" {

const char* hsc_version(void) { return "hsc-mi355x 0.1"; }
const char* hsc_last_error(void) { return hsc::last_error(); }
const char* hsc_ctx_last_error(const hsc_ctx*) { return hsc::last_error(); }

// H (CSR, checked: indices in range, finite, exactly symmetric) and the contacts into t; argument
// errors throw a message, the other failures return their status
static int ingest(hsc_tree* t, int64_t n, const int64_t* indptr, const int32_t* indices, const double* values_ri,
                  int32_t n_contacts, const hsc_contact* contacts) {
  if (n_contacts != 2) throw std::string("exactly two contacts are required");
  t->n = n;
  if (indptr[0] != 0) throw std::string("indptr[0] != 0");
  for (int64_t r = 0; r < n; ++r)
    if (indptr[r + 1] < indptr[r]) throw std::string("indptr not monotone");
  int64_t nnz = indptr[n];
  t->indptr.assign(indptr, indptr + n + 1);
  t->indices.assign(indices, indices + nnz);
  t->values.assign(values_ri, values_ri + 2 * nnz);
  for (int64_t q = 0; q < nnz; ++q) {
    if (indices[q] < 0 || indices[q] >= n) throw std::string("column index out of range");
    if (!std::isfinite(values_ri[2 * q]) || !std::isfinite(values_ri[2 * q + 1])) {
      set_error("non-finite value in H");
      return HSC_E_NONFINITE;
    }
  }
  // symmetry H^T == H (exact): sort each row's (col, value) pairs
  {
    std::vector<int64_t> ord(nnz);
    for (int64_t r = 0; r < n; ++r) {
      for (int64_t q = indptr[r]; q < indptr[r + 1]; ++q) ord[q] = q;
      std::sort(ord.begin() + indptr[r], ord.begin() + indptr[r + 1],
                [&](int64_t a, int64_t b) { return indices[a] < indices[b]; });
    }
    auto find = [&](int64_t r, int32_t c, double* re, double* im) {
      int64_t a = indptr[r], b = indptr[r + 1];
      double sr = 0, si = 0;
      bool hit = false;
      auto it = std::lower_bound(ord.begin() + a, ord.begin() + b, c,
                                 [&](int64_t q, int32_t v) { return indices[q] < v; });
      for (; it != ord.begin() + b && indices[*it] == c; ++it) {
        sr += values_ri[2 * *it];
        si += values_ri[2 * *it + 1];
        hit = true;
      }
      *re = sr; *im = si;
      return hit;
    };
    for (int64_t r = 0; r < n; ++r)
      for (int64_t q = indptr[r]; q < indptr[r + 1]; ++q) {
        int32_t c = indices[q];
        double ar, ai, br, bi;
        find(r, c, &ar, &ai);
        bool ok = find(c, (int32_t)r, &br, &bi);
        if (!ok || ar != br || ai != bi) {
          set_error("H is not symmetric at (" + std::to_string(r) + "," + std::to_string(c) + ")");
          return HSC_E_NOT_SYMMETRIC;
        }
      }
  }
  t->side.assign(n, -1);
  for (int k = 0; k < 2; ++k) {
    const hsc_contact& c = contacts[k];
    if (c.n_sites <= 0 || !c.sites) throw std::string("empty contact");
    if (!(c.lead_hopping != 0.0) || !std::isfinite(c.lead_hopping) || !std::isfinite(c.coupling) ||
        !std::isfinite(c.lead_onsite))
      throw std::string("bad lead parameters");
    t->contact[k].sites.assign(c.sites, c.sites + c.n_sites);
    t->contact[k].lead_onsite = c.lead_onsite;
    t->contact[k].lead_hopping = c.lead_hopping;
    t->contact[k].coupling = c.coupling;
    for (int64_t j = 0; j < c.n_sites; ++j) {
      int64_t s = c.sites[j];
      if (s < 0 || s >= n) throw std::string("contact site out of range");
      if (t->side[s] >= 0) throw std::string("site listed in two contacts (or twice)");
      t->side[s] = (int8_t)k;
    }
  }
  return HSC_OK;
}

hsc_status hsc_tree_build(int64_t n, const int64_t* indptr, const int32_t* indices,
                          const double* values_ri, int32_t n_contacts,
                          const hsc_contact* contacts, const hsc_tree_opts* opts,
                          hsc_tree** out) {
  if (!out) { set_error("out is NULL"); return HSC_E_ARG; }
  *out = nullptr;
  if (n <= 0 || !indptr || !indices || !values_ri || !contacts || !opts) {
    set_error("null or empty argument to hsc_tree_build");
    return HSC_E_ARG;
  }
  if (opts->method != 0 && opts->method != 1) { set_error("method must be 0 (geometric) or 1 (graph)"); return HSC_E_ARG; }
  if (opts->method == 0 && !opts->coords) { set_error("geometric nested dissection needs coordinates"); return HSC_E_ARG; }
  if (opts->method == 1 && opts->dense_contacts) {
    set_error("whole-face contacts need the geometric dissection (coordinates)");
    return HSC_E_ARG;
  }
  if (opts->leaf_side < 1 || (opts->method == 0 && (opts->split_mask & 7) == 0)) {
    set_error("bad tree options");
    return HSC_E_ARG;
  }
  hsc_tree* t = new (std::nothrow) hsc_tree();
  if (!t) { set_error("host allocation failed"); return HSC_E_OOM; }
  try {
    const int rc = ingest(t, n, indptr, indices, values_ri, n_contacts, contacts);
    if (rc != HSC_OK) { delete t; return (hsc_status)rc; }
    if (opts->coords) t->coords.assign(opts->coords, opts->coords + 3 * n);
    else t->coords.assign(3 * n, 0);
    t->split_mask = opts->split_mask & 7;
    t->leaf_side = opts->leaf_side;
    if (opts->method == 1) {
      GraphND g(t, opts->leaf_side);
      std::vector<int64_t> all(n);
      for (int64_t s = 0; s < n; ++s) all[s] = s;
      g.rec(all);
      t->cl.resize(g.sites_of.size());
      for (size_t i = 0; i < g.sites_of.size(); ++i) t->cl[i].children = g.kids_of[i];
      int st = finalize_tree(t, g.sites_of);
      if (st != HSC_OK) { delete t; return (hsc_status)st; }
      t->seg_site = {0, n};
      t->seg_left = {0, (int64_t)t->contact[0].sites.size()};
      *out = t;
      return HSC_OK;
    }
    NDBuilder b{t, {}, {}};
    if (opts->dense_contacts != 0 && opts->dense_contacts != 1) throw std::string("dense_contacts must be 0 or 1");
    t->dense = opts->dense_contacts;
    if (t->dense) {
      build_dense(t, b);
    } else {
      std::vector<int64_t> all(n);
      for (int64_t s = 0; s < n; ++s) all[s] = s;
      b.rec(all);
    }
    t->cl.resize(b.sites_of.size());
    for (size_t i = 0; i < b.sites_of.size(); ++i) t->cl[i].children = b.kids_of[i];
    int st = finalize_tree(t, b.sites_of);
    if (st != HSC_OK) { delete t; return (hsc_status)st; }
    t->seg_site = {0, n};
    t->seg_left = {0, (int64_t)t->contact[0].sites.size()};
  } catch (const std::string& msg) {
    delete t;
    set_error(msg);
    return HSC_E_ARG;
  } catch (const std::bad_alloc&) {
    delete t;
    set_error("host allocation failed");
    return HSC_E_OOM;
  }
  *out = t;
  return HSC_OK;
}

hsc_status hsc_tree_build_custom(int64_t n, const int64_t* indptr, const int32_t* indices,
                                 const double* values_ri, int32_t n_contacts, const hsc_contact* contacts,
                                 int32_t n_clusters, const int32_t* cluster_of_site, const int32_t* parent,
                                 hsc_tree** out) {
  if (!out) { set_error("out is NULL"); return HSC_E_ARG; }
  *out = nullptr;
  if (n <= 0 || !indptr || !indices || !values_ri || !contacts || n_clusters < 1 || !cluster_of_site || !parent) {
    set_error("null or empty argument to hsc_tree_build_custom");
    return HSC_E_ARG;
  }
  hsc_tree* t = new (std::nothrow) hsc_tree();
  if (!t) { set_error("host allocation failed"); return HSC_E_OOM; }
  try {
    const int rc = ingest(t, n, indptr, indices, values_ri, n_contacts, contacts);
    if (rc != HSC_OK) { delete t; return (hsc_status)rc; }
    t->coords.assign(3 * n, 0);
    std::vector<std::vector<int64_t>> members(n_clusters);
    for (int64_t s = 0; s < n; ++s) {
      const int32_t c = cluster_of_site[s];
      if (c < 0 || c >= n_clusters) throw std::string("cluster_of_site out of range");
      members[c].push_back(s);
    }
    int root = -1;
    std::vector<std::vector<int>> kids(n_clusters);
    for (int c = 0; c < n_clusters; ++c) {
      if (members[c].empty()) throw std::string("empty cluster " + std::to_string(c));
      const int p = parent[c];
      if (p < -1 || p >= n_clusters || p == c) throw std::string("bad parent of cluster " + std::to_string(c));
      if (p < 0) {
        if (root >= 0) throw std::string("more than one root");
        root = c;
      } else {
        kids[p].push_back(c);
      }
    }
    if (root < 0) throw std::string("no root");
    // children-first numbering from the root (children in increasing given id); a cluster not
    // reached lies on a cycle
    std::vector<std::vector<int64_t>> sites_of;
    std::vector<std::vector<int>> kids_of;
    std::vector<int> newid(n_clusters, -1);
    std::vector<std::pair<int, size_t>> stack{{root, 0}};
    while (!stack.empty()) {
      auto& top = stack.back();
      if (top.second < kids[top.first].size()) {
        const int k = kids[top.first][top.second++];
        stack.push_back({k, 0});
        continue;
      }
      const int c = top.first;
      std::vector<int> ch;
      for (int k : kids[c]) ch.push_back(newid[k]);
      newid[c] = (int)sites_of.size();
      sites_of.push_back(members[c]);
      kids_of.push_back(ch);
      stack.pop_back();
    }
    if ((int)sites_of.size() != n_clusters) throw std::string("the parent links do not form one tree");
    t->cl.resize(sites_of.size());
    for (size_t i = 0; i < sites_of.size(); ++i) t->cl[i].children = kids_of[i];
    const int st = finalize_tree(t, sites_of);
    if (st != HSC_OK) { delete t; return (hsc_status)st; }
    t->seg_site = {0, n};
    t->seg_left = {0, (int64_t)t->contact[0].sites.size()};
  } catch (const std::string& msg) {
    delete t;
    set_error(msg);
    return HSC_E_ARG;
  } catch (const std::bad_alloc&) {
    delete t;
    set_error("host allocation failed");
    return HSC_E_OOM;
  }
  *out = t;
  return HSC_OK;
}

hsc_status hsc_tree_bonds(const hsc_tree* tree, int64_t* pairs, int64_t* count) {
  if (!tree || !count) { set_error("bad arguments to hsc_tree_bonds"); return HSC_E_ARG; }
  const std::vector<int64_t> b = tree_bonds(tree);
  const int64_t nb = (int64_t)b.size() / 2;
  if (pairs) {
    if (*count < nb) { set_error("hsc_tree_bonds: capacity below the number of bonds"); return HSC_E_ARG; }
    std::copy(b.begin(), b.end(), pairs);
  }
  *count = nb;
  return HSC_OK;
}

hsc_status hsc_tree_merge(const hsc_tree* src, int32_t n_ids, const int32_t* ids, hsc_tree** out) {
  if (!src || !out || n_ids < 0 || (n_ids > 0 && !ids)) { set_error("bad arguments to hsc_tree_merge"); return HSC_E_ARG; }
  *out = nullptr;
  if (src->dense) { set_error("trees with whole-face contacts cannot be merged"); return HSC_E_ARG; }
  const int nc = (int)src->cl.size();
  std::vector<char> gone(nc, 0);
  for (int k = 0; k < n_ids; ++k) {
    if (ids[k] < 0 || ids[k] >= nc || src->cl[ids[k]].parent < 0) {
      set_error("cluster id out of range (a root cannot be merged)");
      return HSC_E_ARG;
    }
    gone[ids[k]] = 1;
  }
  hsc_tree* t = new (std::nothrow) hsc_tree(*src);
  if (!t) { set_error("host allocation failed"); return HSC_E_OOM; }
  // target of each cluster: itself, or the nearest surviving ancestor
  std::vector<int> tgt(nc);
  for (int i = nc - 1; i >= 0; --i) tgt[i] = gone[i] ? tgt[src->cl[i].parent] : i;
  std::vector<std::vector<int64_t>> sites(nc);
  std::vector<std::vector<int>> kids(nc);
  for (int i = 0; i < nc; ++i) {
    const Cluster& c = src->cl[i];
    for (int64_t p = c.first; p < c.first + c.n; ++p) sites[tgt[i]].push_back(src->perm[p]);
    if (!gone[i] && c.parent >= 0) kids[tgt[c.parent]].push_back(i);
  }
  // renumber survivors in post-order (children keep their relative order)
  std::vector<int> newid(nc, -1);
  std::vector<Cluster> ncl;
  std::vector<std::vector<int64_t>> nsites;
  std::function<int(int)> walk = [&](int i) -> int {
    std::vector<int> ch;
    std::vector<int> order = kids[i];
    std::sort(order.begin(), order.end());
    for (int k : order) ch.push_back(walk(k));
    Cluster c;
    c.children = ch;
    ncl.push_back(c);
    nsites.push_back(sites[i]);
    newid[i] = (int)ncl.size() - 1;
    return newid[i];
  };
  for (int i = 0; i < nc; ++i)
    if (src->cl[i].parent < 0) walk(i);
  t->cl = ncl;
  int st = finalize_tree(t, nsites);
  if (st != HSC_OK) { delete t; return (hsc_status)st; }
  *out = t;
  return HSC_OK;
}

hsc_status hsc_tree_concat(int32_t n_trees, const hsc_tree* const* trees, hsc_tree** out) {
  if (!out || n_trees < 1 || !trees) { set_error("bad arguments to hsc_tree_concat"); return HSC_E_ARG; }
  *out = nullptr;
  for (int d = 0; d < n_trees; ++d) {
    if (!trees[d]) { set_error("null tree in hsc_tree_concat"); return HSC_E_ARG; }
    if (trees[d]->dense) { set_error("hsc_tree_concat: trees with whole-face contacts cannot form a forest"); return HSC_E_ARG; }
  }
  for (int d = 1; d < n_trees; ++d)
    for (int k = 0; k < 2; ++k) {
      const ContactInfo &a = trees[0]->contact[k], &b = trees[d]->contact[k];
      if (a.lead_onsite != b.lead_onsite || a.lead_hopping != b.lead_hopping || a.coupling != b.coupling) {
        set_error("hsc_tree_concat: devices differ in their lead model");
        return HSC_E_ARG;
      }
    }
  int64_t ntot = 0;
  for (int d = 0; d < n_trees; ++d) ntot += trees[d]->n;
  if (ntot > INT32_MAX) { set_error("hsc_tree_concat: more than 2^31 - 1 sites"); return HSC_E_ARG; }
  hsc_tree* t = new (std::nothrow) hsc_tree();
  if (!t) { set_error("host allocation failed"); return HSC_E_OOM; }
  try {
    t->n = ntot;
    t->split_mask = trees[0]->split_mask;
    t->leaf_side = trees[0]->leaf_side;
    t->indptr.assign(1, 0);
    for (int k = 0; k < 2; ++k) t->contact[k] = trees[0]->contact[k], t->contact[k].sites.clear();
    std::vector<std::vector<int64_t>> sites_of;
    std::vector<std::vector<int>> kids;
    int64_t s0 = 0;
    t->seg_site.assign(1, 0);
    t->seg_left.assign(1, 0);
    for (int d = 0; d < n_trees; ++d) {
      const hsc_tree* u = trees[d];
      const int64_t nnz0 = t->indptr.back();
      for (int64_t r = 0; r < u->n; ++r) t->indptr.push_back(nnz0 + u->indptr[r + 1]);
      for (int32_t c : u->indices) t->indices.push_back((int32_t)(c + s0));
      t->values.insert(t->values.end(), u->values.begin(), u->values.end());
      t->coords.insert(t->coords.end(), u->coords.begin(), u->coords.end());
      t->side.insert(t->side.end(), u->side.begin(), u->side.end());
      for (int k = 0; k < 2; ++k)
        for (int64_t x : u->contact[k].sites) t->contact[k].sites.push_back(x + s0);
      const int c0 = (int)kids.size();
      for (const Cluster& c : u->cl) {
        std::vector<int> ch;
        for (int k : c.children) ch.push_back(k + c0);
        kids.push_back(ch);
        std::vector<int64_t> v;
        for (int64_t p = c.first; p < c.first + c.n; ++p) v.push_back(u->perm[p] + s0);
        sites_of.push_back(v);
      }
      s0 += u->n;
      t->seg_site.push_back(s0);
      t->seg_left.push_back((int64_t)t->contact[0].sites.size());
    }
    t->cl.resize(kids.size());
    for (size_t i = 0; i < kids.size(); ++i) t->cl[i].children = kids[i];
    int st = finalize_tree(t, sites_of);
    if (st != HSC_OK) { delete t; return (hsc_status)st; }
  } catch (const std::bad_alloc&) {
    delete t;
    set_error("host allocation failed");
    return HSC_E_OOM;
  }
  *out = t;
  return HSC_OK;
}

hsc_status hsc_tree_stats_get(const hsc_tree* t, hsc_tree_stats* out) {
  if (!t || !out) { set_error("null argument"); return HSC_E_ARG; }
  std::memset(out, 0, sizeof(*out));
  out->n_sites = t->n;
  out->n_clusters = (int32_t)t->cl.size();
  out->depth = t->depth;
  for (const auto& c : t->cl) {
    out->max_cluster = std::max(out->max_cluster, c.n);
    out->max_front = std::max(out->max_front, c.f());
    if (c.cpath()) out->max_ancestors = std::max(out->max_ancestors, (int32_t)c.n_anc);
    if (c.children.empty()) out->n_leaves++;
  }
  uint32_t want = HSC_DIAG_GR | HSC_DIAG_GL | HSC_TRANS;
  out->flops_per_energy = flops_per_energy(t, want);
  out->bytes_per_energy = bytes_per_energy(t, want);
  return HSC_OK;
}

hsc_status hsc_tree_export(const hsc_tree* t, int64_t* perm, int32_t* cl_parent, int32_t* cl_first,
                           int32_t* cl_size, int64_t* front_ptr, int64_t* front_sites) {
  if (!t) { set_error("null tree"); return HSC_E_ARG; }
  const int nc = (int)t->cl.size();
  if (perm) std::copy(t->perm.begin(), t->perm.end(), perm);
  int64_t off = 0;
  for (int i = 0; i < nc; ++i) {
    const Cluster& c = t->cl[i];
    if (cl_parent) cl_parent[i] = c.parent;
    if (cl_first) cl_first[i] = (int32_t)c.first;
    if (cl_size) cl_size[i] = c.n;
    if (front_ptr) front_ptr[i] = off;
    if (front_sites) std::copy(c.front.begin(), c.front.end(), front_sites + off);
    off += (int64_t)c.front.size();
  }
  if (front_ptr) front_ptr[nc] = off;
  return HSC_OK;
}

hsc_status hsc_tree_destroy(hsc_tree* t) {
  delete t;
  return HSC_OK;
}

}  // extern "C"
