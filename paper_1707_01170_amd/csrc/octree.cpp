// Host construction of the element octree for dyadic meshes (Sec. 3.2, the
// octree look-up structure; its GPU layout is described in Sec. 3.2.2).
//
// Knots that are multiples of 2^-L let the domain be cut into octree cells
// whose faces never cross an element face below level L.  A cell met by a
// single element (with positive volume) is a leaf holding that element;
// otherwise it is split into its eight children.  An element with unequal
// sides spans several leaves.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

struct lr_octree_host {
  uint32_t root = 0;
  std::vector<uint32_t> nodes;      // [n_nodes][8]
  lr_forest_stats stats{};
};

namespace {

constexpr int kLevels = 24;         // knots must be multiples of 2^-24

struct OctBuilder {
  const std::vector<int64_t>& box;  // [n][6], integer coordinates at level kLevels
  std::vector<uint32_t>& nodes;
  std::vector<int32_t> leaf_depth;
  bool gap = false, overlap = false, full = false;

  OctBuilder(const std::vector<int64_t>& b, std::vector<uint32_t>& n) : box(b), nodes(n) {}

  // Cell of side 2^(kLevels - level) at integer corner c; els are the
  // elements meeting the parent cell.  Pre-order: a node's eight children
  // are stored contiguously at 8 * index.
  uint32_t build(const int64_t c[3], int level, const std::vector<int32_t>& parent) {
    const int64_t side = (int64_t)1 << (kLevels - level);
    std::vector<int32_t> els;
    for (int32_t e : parent) {
      bool meets = true;
      for (int d = 0; d < 3 && meets; ++d) meets = box[6 * e + d] < c[d] + side && c[d] < box[6 * e + 3 + d];
      if (meets) els.push_back(e);
    }
    if (els.empty()) {
      gap = true;
      return LR_LEAF;
    }
    if (els.size() == 1) {
      leaf_depth.push_back(level);
      return LR_LEAF | (uint32_t)els[0];
    }
    if (level == kLevels) {
      overlap = true;
      return LR_LEAF;
    }
    if (nodes.size() / 8 + 1 >= (size_t)LR_LEAF) {
      full = true;
      return LR_LEAF;
    }
    const uint32_t idx = (uint32_t)(nodes.size() / 8);
    nodes.resize(nodes.size() + 8, LR_LEAF);
    const int64_t h = side / 2;
    for (int k = 0; k < 8; ++k) {
      const int64_t cc[3] = {c[0] + ((k & 1) ? h : 0), c[1] + ((k & 2) ? h : 0), c[2] + ((k & 4) ? h : 0)};
      const uint32_t r = build(cc, level + 1, els);
      nodes[8 * (size_t)idx + k] = r;
      if (gap || overlap || full) return LR_LEAF;
    }
    return idx;
  }
};

}  // namespace

using lrvr::fail;

LR_API lr_status lr_build_octree(const double* elem_box, int64_t n_elem, lr_octree_host** out, lr_forest_stats* stats) {
  if (!elem_box || !out || n_elem <= 0) return fail(LR_EINVAL, "lr_build_octree: null pointer or n_elem <= 0");
  if (n_elem >= (int64_t)LR_LEAF) return fail(LR_EINVAL, "lr_build_octree: too many elements");
  *out = nullptr;
  const double scale = std::ldexp(1.0, kLevels);
  std::vector<int64_t> box((size_t)n_elem * 6);
  double vol = 0.0;
  for (int64_t e = 0; e < n_elem; ++e) {
    vol += (elem_box[6 * e + 3] - elem_box[6 * e]) * (elem_box[6 * e + 4] - elem_box[6 * e + 1]) *
           (elem_box[6 * e + 5] - elem_box[6 * e + 2]);
    for (int d = 0; d < 3; ++d) {
      const double lo = elem_box[6 * e + d], hi = elem_box[6 * e + 3 + d];
      if (!(0.0 <= lo && lo < hi && hi <= 1.0))
        return fail(LR_EPARTITION, "lr_build_octree: element %lld is empty or leaves [0,1]^3", (long long)e);
      const double a = lo * scale, b = hi * scale;
      if (a != std::floor(a) || b != std::floor(b))
        return fail(LR_EKNOT, "lr_build_octree: element %lld has a knot that is not a multiple of 2^-%d",
                    (long long)e, kLevels);
      box[6 * e + d] = (int64_t)a;
      box[6 * e + 3 + d] = (int64_t)b;
    }
  }
  // With the volumes summing to one, a gap implies an overlap, which the
  // descent below finds (two elements still meeting a cell at the finest level).
  if (std::fabs(vol - 1.0) > 1e-9) return fail(LR_EPARTITION, "lr_build_octree: element volumes sum to %.17g", vol);
  auto* o = new lr_octree_host();
  OctBuilder b(box, o->nodes);
  std::vector<int32_t> all((size_t)n_elem);
  for (int64_t e = 0; e < n_elem; ++e) all[e] = (int32_t)e;
  const int64_t c0[3] = {0, 0, 0};
  o->root = b.build(c0, 0, all);
  if (b.gap || b.overlap || b.full) {
    delete o;
    if (b.full) return fail(LR_ECAPACITY, "lr_build_octree: more than 2^31 nodes");
    return fail(LR_EPARTITION, "lr_build_octree: the elements %s", b.gap ? "leave a gap" : "overlap");
  }
  lr_forest_stats& st = o->stats;
  st.n_heads = 1;
  st.n_nodes = (int64_t)(o->nodes.size() / 8);
  st.n_direct = (o->root & LR_LEAF) ? 1 : 0;
  const auto& ld = b.leaf_depth;
  st.min_depth = *std::min_element(ld.begin(), ld.end());
  st.max_depth = *std::max_element(ld.begin(), ld.end());
  double m = 0.0;
  for (int32_t d : ld) m += d;
  m /= (double)ld.size();
  double var = 0.0;
  for (int32_t d : ld) var += (d - m) * (d - m);
  st.mean_depth = m;
  st.var_depth = var / (double)ld.size();
  if (stats) *stats = st;
  *out = o;
  return LR_OK;
}

LR_API lr_status lr_octree_export(const lr_octree_host* o, uint32_t* root, uint32_t* nodes) {
  if (!o) return fail(LR_EINVAL, "lr_octree_export: null octree");
  if (root) *root = o->root;
  if (nodes && !o->nodes.empty()) std::memcpy(nodes, o->nodes.data(), o->nodes.size() * sizeof(uint32_t));
  return LR_OK;
}

LR_API void lr_octree_free(lr_octree_host* o) { delete o; }
