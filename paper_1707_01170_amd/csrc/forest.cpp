// Host construction of the k-d forest (Sec. 3.2.1): regular blocks, one
// depth-balanced k-d tree per block over the elements meeting it, a block met
// by a single element storing that element directly.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

struct lr_forest_host {
  int32_t blocks[3];
  std::vector<uint32_t> heads;
  std::vector<lr_kdnode> nodes;
  lr_forest_stats stats;
};

namespace {

constexpr int kMaxDepth = 255;

struct Builder {
  const std::vector<float>& box;   // [n][6]
  std::vector<lr_kdnode>& nodes;
  std::vector<double> faces;
  bool too_deep = false;
  bool stuck = false;

  Builder(const std::vector<float>& b, std::vector<lr_kdnode>& n) : box(b), nodes(n) {}

  // Chooses the split of a node (Sec. 3.2.1: count the elements left and
  // right of the mean split value in each direction).  Returns false if no
  // element face lies strictly inside the region.
  bool choose(const double rlo[3], const double rhi[3], const std::vector<int32_t>& els, int& axis,
              double& split) {
    bool found = false;
    size_t best_score = 0;
    double best_ext = 0.0;
    for (int d = 0; d < 3; ++d) {
      faces.clear();
      for (int32_t e : els) {
        const double f[2] = {box[6 * e + d], box[6 * e + 3 + d]};
        for (double x : f)
          if (rlo[d] < x && x < rhi[d]) faces.push_back(x);
      }
      if (faces.empty()) continue;
      std::sort(faces.begin(), faces.end());
      faces.erase(std::unique(faces.begin(), faces.end()), faces.end());
      double mean = 0.0;
      for (double x : faces) mean += x;
      mean /= (double)faces.size();
      double s = faces[0];
      for (double x : faces)
        if (std::fabs(x - mean) < std::fabs(s - mean)) s = x;   // ties keep the smaller
      size_t nl = 0, nr = 0;
      for (int32_t e : els) {
        nl += box[6 * e + d] < s;
        nr += box[6 * e + 3 + d] > s;
      }
      const size_t score = std::max(nl, nr);
      const double ext = rhi[d] - rlo[d];
      if (!found || score < best_score || (score == best_score && ext > best_ext)) {
        found = true;
        best_score = score;
        best_ext = ext;
        axis = d;
        split = s;
      }
    }
    return found;
  }

  // Pre-order layout; returns a child reference.
  uint32_t build(double rlo[3], double rhi[3], std::vector<int32_t>& els, int depth, int& maxd) {
    if (els.size() == 1) {
      maxd = std::max(maxd, depth);
      return LR_LEAF | (uint32_t)els[0];
    }
    if (depth >= kMaxDepth) {
      too_deep = true;
      return LR_LEAF;
    }
    int axis = 0;
    double s = 0.0;
    if (!choose(rlo, rhi, els, axis, s)) {
      stuck = true;
      return LR_LEAF;
    }
    const uint32_t idx = (uint32_t)nodes.size();
    nodes.push_back(lr_kdnode{0, 0, (float)s, (uint32_t)axis});
    std::vector<int32_t> left, right;
    for (int32_t e : els) {
      if (box[6 * e + axis] < s) left.push_back(e);
      if (box[6 * e + 3 + axis] > s) right.push_back(e);
    }
    const double keep_hi = rhi[axis], keep_lo = rlo[axis];
    rhi[axis] = s;
    const uint32_t lo = build(rlo, rhi, left, depth + 1, maxd);
    rhi[axis] = keep_hi;
    rlo[axis] = s;
    const uint32_t hi = build(rlo, rhi, right, depth + 1, maxd);
    rlo[axis] = keep_lo;
    nodes[idx].lo = lo;
    nodes[idx].hi = hi;
    return idx;
  }
};

}  // namespace

using lrvr::fail;

LR_API lr_status lr_build_forest(const double* elem_box, int64_t n_elem, const int32_t blocks[3],
                                 lr_forest_host** out, lr_forest_stats* stats) {
  if (!elem_box || !blocks || !out || n_elem <= 0) return fail(LR_EINVAL, "lr_build_forest: null pointer or n_elem <= 0");
  if (n_elem >= (int64_t)LR_LEAF) return fail(LR_EINVAL, "lr_build_forest: too many elements");
  *out = nullptr;
  for (int d = 0; d < 3; ++d)
    if (!lrvr::is_pow2(blocks[d]) || blocks[d] > 512)
      return fail(LR_ENOTPOW2, "lr_build_forest: blocks[%d] = %d is not a power of two in [1,512]", d, blocks[d]);
  std::vector<float> box((size_t)n_elem * 6);
  double vol = 0.0;
  for (int64_t e = 0; e < n_elem; ++e) {
    double v = 1.0;
    for (int d = 0; d < 3; ++d) {
      const double lo = elem_box[6 * e + d], hi = elem_box[6 * e + 3 + d];
      if (!lrvr::fp32_exact(lo) || !lrvr::fp32_exact(hi))
        return fail(LR_EKNOT, "lr_build_forest: element %lld has a coordinate not exact in FP32", (long long)e);
      if (!(0.0 <= lo && lo < hi && hi <= 1.0))
        return fail(LR_EPARTITION, "lr_build_forest: element %lld is empty or leaves [0,1]^3", (long long)e);
      box[6 * e + d] = (float)lo;
      box[6 * e + 3 + d] = (float)hi;
      v *= hi - lo;
    }
    vol += v;
  }
  if (std::fabs(vol - 1.0) > 1e-9) return fail(LR_EPARTITION, "lr_build_forest: element volumes sum to %.17g", vol);

  const int32_t B[3] = {blocks[0], blocks[1], blocks[2]};
  const int64_t nb = (int64_t)B[0] * B[1] * B[2];
  // Bin elements into the blocks they meet with positive volume.
  std::vector<int64_t> cnt(nb + 1, 0);
  auto brange = [&](int64_t e, int d, int64_t& a, int64_t& b) {
    a = (int64_t)std::floor((double)box[6 * e + d] * B[d]);
    b = (int64_t)std::ceil((double)box[6 * e + 3 + d] * B[d]) - 1;
    a = std::max<int64_t>(0, a);
    b = std::min<int64_t>(B[d] - 1, b);
  };
  for (int64_t e = 0; e < n_elem; ++e) {
    int64_t r[3][2];
    for (int d = 0; d < 3; ++d) brange(e, d, r[d][0], r[d][1]);
    for (int64_t k = r[2][0]; k <= r[2][1]; ++k)
      for (int64_t j = r[1][0]; j <= r[1][1]; ++j)
        for (int64_t i = r[0][0]; i <= r[0][1]; ++i) ++cnt[(k * B[1] + j) * B[0] + i + 1];
  }
  for (int64_t b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
  std::vector<int32_t> members((size_t)cnt[nb]);
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < n_elem; ++e) {
      int64_t r[3][2];
      for (int d = 0; d < 3; ++d) brange(e, d, r[d][0], r[d][1]);
      for (int64_t k = r[2][0]; k <= r[2][1]; ++k)
        for (int64_t j = r[1][0]; j <= r[1][1]; ++j)
          for (int64_t i = r[0][0]; i <= r[0][1]; ++i) members[pos[(k * B[1] + j) * B[0] + i]++] = (int32_t)e;
    }
  }

  auto* f = new lr_forest_host();
  std::memcpy(f->blocks, B, sizeof B);
  f->heads.assign((size_t)nb, 0u);
  Builder bld(box, f->nodes);
  std::vector<int32_t> depth((size_t)nb, 0);
  std::vector<int32_t> els;
  int64_t n_direct = 0;
  for (int64_t k = 0; k < B[2]; ++k)
    for (int64_t j = 0; j < B[1]; ++j)
      for (int64_t i = 0; i < B[0]; ++i) {
        const int64_t b = (k * B[1] + j) * B[0] + i;
        double rlo[3] = {(double)i / B[0], (double)j / B[1], (double)k / B[2]};
        double rhi[3] = {(double)(i + 1) / B[0], (double)(j + 1) / B[1], (double)(k + 1) / B[2]};
        els.assign(members.begin() + cnt[b], members.begin() + cnt[b + 1]);
        // The elements meeting a block must tile it.
        double v = 0.0;
        for (int32_t e : els) {
          double w = 1.0;
          for (int d = 0; d < 3; ++d)
            w *= std::min<double>(box[6 * e + 3 + d], rhi[d]) - std::max<double>(box[6 * e + d], rlo[d]);
          v += w;
        }
        const double bv = (rhi[0] - rlo[0]) * (rhi[1] - rlo[1]) * (rhi[2] - rlo[2]);
        if (els.empty() || std::fabs(v - bv) > 1e-9 * bv) {
          delete f;
          return fail(LR_EPARTITION, "lr_build_forest: elements do not tile block (%lld,%lld,%lld)",
                      (long long)i, (long long)j, (long long)k);
        }
        if (els.size() == 1) {
          f->heads[b] = LR_LEAF | (uint32_t)els[0];
          ++n_direct;
          continue;
        }
        int maxd = 0;
        const uint32_t root = bld.build(rlo, rhi, els, 0, maxd);
        if (bld.too_deep || bld.stuck || f->nodes.size() >= (size_t)LR_LEAF) {
          delete f;
          return fail(bld.stuck ? LR_EPARTITION : LR_ECAPACITY,
                      "lr_build_forest: cannot build the tree of block (%lld,%lld,%lld)%s", (long long)i,
                      (long long)j, (long long)k, bld.stuck ? " (overlapping elements)" : " (deeper than 255)");
        }
        f->heads[b] = root;
        depth[b] = maxd;
      }
  lr_forest_stats& st = f->stats;
  st.n_heads = nb;
  st.n_nodes = (int64_t)f->nodes.size();
  st.n_direct = n_direct;
  st.min_depth = *std::min_element(depth.begin(), depth.end());
  st.max_depth = *std::max_element(depth.begin(), depth.end());
  double m = 0.0;
  for (int32_t d : depth) m += d;
  m /= (double)nb;
  double var = 0.0;
  for (int32_t d : depth) var += (d - m) * (d - m);
  st.mean_depth = m;
  st.var_depth = var / (double)nb;
  if (stats) *stats = st;
  *out = f;
  return LR_OK;
}

LR_API lr_status lr_forest_export(const lr_forest_host* f, uint32_t* heads, lr_kdnode* nodes) {
  if (!f) return fail(LR_EINVAL, "lr_forest_export: null forest");
  if (heads) std::memcpy(heads, f->heads.data(), f->heads.size() * sizeof(uint32_t));
  if (nodes && !f->nodes.empty()) std::memcpy(nodes, f->nodes.data(), f->nodes.size() * sizeof(lr_kdnode));
  return LR_OK;
}

LR_API void lr_forest_free(lr_forest_host* f) { delete f; }
