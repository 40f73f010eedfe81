// Internal structures shared by the host tree builder and the device solver.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hsc.h"

namespace hsc {

void set_error(const std::string& msg);

// the device index and HIP stream (hipStream_t, may be null) of a context
int ctx_device(const hsc_ctx* ctx);
void* ctx_stream(const hsc_ctx* ctx);

struct ContactInfo {
  std::vector<int64_t> sites;
  double lead_onsite = 0, lead_hopping = -1, coupling = -1;
};

// A whole-face contact (dense self-energy): transverse axes, the face's lowest coordinate and
// extent on each, and the cluster that holds exactly the face's sites.
struct FaceInfo {
  int32_t ax[2] = {1, 2};
  int32_t lo[2] = {0, 0};
  int32_t dim[2] = {1, 1};
  int cluster = -1;
};

// One cluster of the binary tree (Section 2.2: clusters organised in a binary
// tree; P_i = ancestors).  Ids are post-order: children before parents, the
// root is the last cluster, and the subtree of i is the id range [lo, i].
struct Cluster {
  int parent = -1;
  std::vector<int> children;
  int lo = 0;                      // smallest id in the subtree
  int depth = 0;                   // root = 0
  int64_t first = 0;               // first position in the cluster ordering
  int n = 0;                       // n_i
  int n_left = 0, n_right = 0;     // contact sites of this cluster (stored first: left, then right)
  bool lpath = false, rpath = false;  // subtree holds left / right contact sites
  std::vector<int64_t> front;      // point-level front (original site ids), position order
  // relative maps
  std::vector<int32_t> rel;        // front site k -> index in parent's frontal set (parent sites, parent front)
  std::vector<int32_t> frontpos;   // front site k -> column in the ancestor list (parent, grandparent, ... root)
  int64_t n_anc = 0;               // |P_i| in sites
  bool cpath() const { return lpath || rpath; }
  int f() const { return (int)front.size(); }
};

}  // namespace hsc

struct hsc_tree {
  int64_t n = 0;
  std::vector<int64_t> indptr;
  std::vector<int32_t> indices;
  std::vector<double> values;      // interleaved re, im
  std::vector<int32_t> coords;     // [n][3]
  int32_t split_mask = 7, leaf_side = 8;
  hsc::ContactInfo contact[2];
  int32_t dense = 0;               // whole-face contacts with dense self-energy blocks
  hsc::FaceInfo face[2];
  std::vector<int8_t> side;        // -1 none, 0 left, 1 right
  std::vector<hsc::Cluster> cl;    // post-order
  std::vector<int64_t> perm;       // position -> site
  std::vector<int64_t> pos;        // site -> position
  std::vector<int32_t> owner;      // site -> cluster
  int depth = 0;                   // number of levels
  uint64_t uid = 0;                // identity for device-side caches
  // devices of a forest (hsc_tree_concat); one segment for an ordinary tree:
  // device d owns sites [seg_site[d], seg_site[d+1]) and left-contact entries
  // [seg_left[d], seg_left[d+1]) of contact[0].sites
  std::vector<int64_t> seg_site, seg_left;
};

namespace hsc {
// Finish a tree whose clusters carry (children, sites): order, fronts, maps.
// `sites_of[i]` are the original site ids of cluster i (any order).
int finalize_tree(hsc_tree* t, std::vector<std::vector<int64_t>>& sites_of);
double flops_per_energy(const hsc_tree* t, uint32_t want);
// bonds of H: pairs (i, j), i < j, with a stored H_ij, by i then j, duplicates once
std::vector<int64_t> tree_bonds(const hsc_tree* t);
double bytes_per_energy(const hsc_tree* t, uint32_t want);
}  // namespace hsc
