// Host-side builders of the C ABI (support CSR, k-d forest, octree) and the
// look-up descents the kernels run (lookup.h, compiled here for the host) run
// under AddressSanitizer and UndefinedBehaviorSanitizer.  Built by
// tests/test_host_sanitize.py with g++ from the library's host sources only.  Input file: int32 p[3], int64 n_bspl, int32 kstride,
// double knots[n_bspl][3][kstride], int64 n_elem, double elem_box[n_elem][6],
// int32 dyadic.  Prints one line per check and exits non-zero on a failure.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lrvr.h"
#include "../paper_1707_01170_amd/csrc/lookup.h"
#include "../paper_1707_01170_amd/csrc/schedule.h"

namespace {

int g_fail = 0;

void check(bool ok, const char* what) {
  std::printf("%s %s\n", ok ? "ok" : "FAIL", what);
  if (!ok) {
    std::printf("  last error: %s\n", lr_last_error());
    g_fail = 1;
  }
}

template <class T>
bool read(FILE* f, T* dst, size_t n) {
  return std::fread(dst, sizeof(T), n, f) == n;
}

bool contains(const double* b, const double* x) {
  for (int a = 0; a < 3; ++a) {
    const bool upper = b[3 + a] == 1.0 ? x[a] <= 1.0 : x[a] < b[3 + a];
    if (!(b[a] <= x[a] && upper)) return false;
  }
  return true;
}

// Descent of Alg. 1 over exported forest arrays, written out here so that
// the check does not reuse the library's device code.
int64_t forest_find(const std::vector<uint32_t>& heads, const std::vector<lr_kdnode>& nodes, const int32_t blk[3],
                    const double* x) {
  int64_t b[3];
  for (int a = 0; a < 3; ++a) {
    int64_t i = (int64_t)std::floor((float)x[a] * (float)blk[a]);
    b[a] = i < blk[a] - 1 ? (i < 0 ? 0 : i) : blk[a] - 1;
  }
  uint32_t r = heads[(size_t)((b[2] * blk[1] + b[1]) * blk[0] + b[0])];
  for (int guard = 0; !(r & LR_LEAF); ++guard) {
    if (guard > 64 || r >= nodes.size()) return -1;
    const lr_kdnode& n = nodes[r];
    r = (float)x[n.axis] < n.split ? n.lo : n.hi;
  }
  return r & ~LR_LEAF;
}

int64_t octree_find(uint32_t root, const std::vector<uint32_t>& nodes, const double* x) {
  uint32_t r = root;
  for (int l = 0; !(r & LR_LEAF); ++l) {
    if (l > 30 || (size_t)r * 8 >= nodes.size()) return -1;
    const double s = std::ldexp(1.0, l + 1);
    int k = 0;
    for (int a = 0; a < 3; ++a) {
      double c = std::floor(x[a] * s);
      if (c > s - 1) c = s - 1;
      k |= ((int64_t)c & 1) << a;
    }
    r = nodes[(size_t)r * 8 + k];
  }
  return r & ~LR_LEAF;
}

// Points of the look-up checks: element centres, lower corners, upper corners
// (in [0,1]) and face centres, as FP32 values.
std::vector<float> probe_points(const std::vector<double>& box, int64_t n_elem) {
  std::vector<float> pts;
  for (int64_t e = 0; e < n_elem; ++e) {
    const double* b = &box[6 * e];
    for (int k = 0; k < 5; ++k)
      for (int a = 0; a < 3; ++a) {
        const double m = 0.5 * (b[a] + b[3 + a]);
        const double v = k == 0 ? m : k == 1 ? b[a] : k == 2 ? b[3 + a] : (k == 3 ? (a == 0 ? b[0] : m) : (a == 1 ? b[4] : m));
        pts.push_back((float)v);
      }
  }
  return pts;
}

// The kernels' descent (lookup.h) on the exported arrays: every probe point
// finds the element holding it, and references made corrupt (a node index
// beyond the nodes, an element id beyond the elements, a node that is its
// own child) give kBadRef without reading outside the arrays.
void check_kernel_forest(const std::vector<uint32_t>& heads, std::vector<lr_kdnode> nodes, const int32_t blk[3],
                         const std::vector<double>& box, int64_t n_elem, const char* what) {
  const std::vector<float> pts = probe_points(box, n_elem);
  const int64_t nn = (int64_t)nodes.size();
  const lr_kdnode* np = nn ? nodes.data() : nullptr;
  bool ok = true;
  for (size_t i = 0; i < pts.size() && ok; i += 3) {
    const float* p = &pts[i];
    const int32_t e = lrvr::forest_lookup(heads.data(), np, nn, n_elem, blk[0], blk[1], blk[2], (float)blk[0],
                                          (float)blk[1], (float)blk[2], p);
    const double x[3] = {p[0], p[1], p[2]};
    ok = e >= 0 && e < n_elem && contains(&box[6 * e], x) && e == forest_find(heads, nodes, blk, x);
  }
  char msg[192];
  std::snprintf(msg, sizeof msg, "%s: the kernels' descent finds the element of every probe point", what);
  check(ok, msg);
  if (nn == 0) return;
  // corrupt references: count points whose descent reports kBadRef
  auto bad_count = [&](const std::vector<lr_kdnode>& nd, int64_t n_el) {
    int64_t n = 0;
    for (size_t i = 0; i < pts.size(); i += 3)
      n += lrvr::forest_lookup(heads.data(), nd.data(), nn, n_el, blk[0], blk[1], blk[2], (float)blk[0],
                               (float)blk[1], (float)blk[2], &pts[i]) == lrvr::kBadRef;
    return n;
  };
  std::vector<lr_kdnode> c1(nodes), c2(nodes);
  c1[0].lo = (uint32_t)nn + 5;          // node index beyond the node array
  c1[0].hi = 0xfffffffu;
  c2[0].lo = 0;                         // node 0 is its own child: no leaf is ever reached
  c2[0].hi = 0;
  const bool caught = bad_count(c1, n_elem) > 0 && bad_count(c2, n_elem) > 0 && bad_count(nodes, 1) > 0;
  std::snprintf(msg, sizeof msg, "%s: corrupt references are reported, not followed", what);
  check(caught, msg);
}

void check_kernel_octree(uint32_t root, std::vector<uint32_t> nodes, const std::vector<double>& box, int64_t n_elem) {
  const std::vector<float> pts = probe_points(box, n_elem);
  const int64_t nn = (int64_t)nodes.size() / 8;
  bool ok = true;
  for (size_t i = 0; i < pts.size() && ok; i += 3) {
    const float* p = &pts[i];
    const int32_t e = lrvr::octree_lookup(&root, nn ? nodes.data() : nullptr, nn, n_elem, p);
    const double x[3] = {p[0], p[1], p[2]};
    ok = e >= 0 && e < n_elem && contains(&box[6 * e], x) && e == octree_find(root, nodes, x);
  }
  check(ok, "octree: the kernels' descent finds the element of every probe point");
  if (nn == 0) return;
  int64_t n_bad = 0;
  std::vector<uint32_t> c1(nodes);
  for (int k = 0; k < 8; ++k) c1[k] = (uint32_t)nn + 3;          // children beyond the nodes
  for (size_t i = 0; i < pts.size(); i += 3) n_bad += lrvr::octree_lookup(&root, c1.data(), nn, n_elem, &pts[i]) < 0;
  std::vector<uint32_t> c2(nodes);
  for (int k = 0; k < 8; ++k) c2[k] = 0;                           // root is its own child
  int64_t n_loop = 0;
  for (size_t i = 0; i < pts.size(); i += 3) n_loop += lrvr::octree_lookup(&root, c2.data(), nn, n_elem, &pts[i]) < 0;
  check(n_bad > 0 && n_loop > 0, "octree: corrupt references are reported, not followed");
}

// The render launch's dispatch order (ring_cell) visits every cell of a
// grid exactly once, first the middle one.
void check_ring_order() {
  bool ok = true;
  std::vector<int> seen;
  auto grid = [&](int w, int h) {
    seen.assign((size_t)w * h, 0);
    for (int64_t k = 0; k < (int64_t)w * h && ok; ++k) {
      int x = -1, y = -1;
      lrvr::ring_cell(k, w, h, x, y);
      ok = x >= 0 && x < w && y >= 0 && y < h && seen[(size_t)y * w + x]++ == 0;
      if (k == 0) ok = ok && x == (w - 1) / 2 && y == (h - 1) / 2;
    }
  };
  for (int w = 1; w <= 48 && ok; ++w)
    for (int h = 1; h <= 48 && ok; ++h) grid(w, h);
  const int shapes[][2] = {{120, 68}, {68, 120}, {256, 256}, {1024, 3}, {3, 1024}};
  for (const auto& s : shapes)
    if (ok) grid(s[0], s[1]);
  check(ok, "ring order: a bijection onto the grid, starting in the middle");
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  check_ring_order();
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t p[3], kstride, dyadic;
  int64_t n_bspl, n_elem;
  if (!read(f, p, 3) || !read(f, &n_bspl, 1) || !read(f, &kstride, 1)) return 2;
  std::vector<double> knots((size_t)n_bspl * 3 * kstride);
  if (!read(f, knots.data(), knots.size()) || !read(f, &n_elem, 1)) return 2;
  std::vector<double> box((size_t)n_elem * 6);
  if (!read(f, box.data(), box.size()) || !read(f, &dyadic, 1)) return 2;
  std::fclose(f);

  // support CSR, sized then filled
  std::vector<int64_t> ptr((size_t)n_elem + 1);
  int64_t nnz = 0;
  lr_status st = lr_build_support(knots.data(), n_bspl, kstride, p, box.data(), n_elem, ptr.data(), nullptr, 0, &nnz);
  check(st == LR_ECAPACITY || st == LR_OK, "support sizing call");
  std::vector<int32_t> idx((size_t)nnz);
  st = lr_build_support(knots.data(), n_bspl, kstride, p, box.data(), n_elem, ptr.data(), idx.data(), nnz, &nnz);
  check(st == LR_OK, "support fill");
  const int64_t nb = (int64_t)(p[0] + 1) * (p[1] + 1) * (p[2] + 1);
  bool csr_ok = ptr[0] == 0 && ptr[n_elem] == nnz;
  for (int64_t e = 0; e < n_elem && csr_ok; ++e) {
    csr_ok = ptr[e + 1] - ptr[e] >= nb;
    for (int64_t q = ptr[e] + 1; q < ptr[e + 1] && csr_ok; ++q) csr_ok = idx[q - 1] < idx[q];
  }
  check(csr_ok, "support CSR: at least (p+1)^3 B-splines per element, ascending");

  // forests of several shapes; every element centre descends to its element
  const int32_t shapes[][3] = {{1, 1, 1}, {4, 4, 4}, {16, 16, 16}, {64, 64, 64}, {2, 8, 4}};
  for (const auto& blk : shapes) {
    lr_forest_host* h = nullptr;
    lr_forest_stats stats;
    st = lr_build_forest(box.data(), n_elem, blk, &h, &stats);
    char what[128];
    std::snprintf(what, sizeof what, "forest %dx%dx%d build", blk[0], blk[1], blk[2]);
    check(st == LR_OK && h != nullptr, what);
    if (st != LR_OK) continue;
    std::vector<uint32_t> heads((size_t)stats.n_heads);
    std::vector<lr_kdnode> nodes((size_t)stats.n_nodes);
    check(lr_forest_export(h, heads.data(), nodes.data()) == LR_OK, "forest export");
    bool found = true;
    for (int64_t e = 0; e < n_elem && found; ++e) {
      double c[3];
      for (int a = 0; a < 3; ++a) c[a] = 0.5 * (box[6 * e + a] + box[6 * e + 3 + a]);
      const int64_t g = forest_find(heads, nodes, blk, c);
      found = g >= 0 && g < n_elem && contains(&box[6 * g], c);
    }
    std::snprintf(what, sizeof what, "forest %dx%dx%d: every element centre finds its element", blk[0], blk[1], blk[2]);
    check(found, what);
    std::snprintf(what, sizeof what, "forest %dx%dx%d", blk[0], blk[1], blk[2]);
    check_kernel_forest(heads, nodes, blk, box, n_elem, what);
    lr_forest_free(h);
  }

  if (dyadic) {
    lr_octree_host* o = nullptr;
    lr_forest_stats stats;
    st = lr_build_octree(box.data(), n_elem, &o, &stats);
    check(st == LR_OK && o != nullptr, "octree build");
    if (st == LR_OK) {
      uint32_t root = 0;
      std::vector<uint32_t> nodes((size_t)stats.n_nodes * 8);
      check(lr_octree_export(o, &root, nodes.data()) == LR_OK, "octree export");
      bool found = true;
      for (int64_t e = 0; e < n_elem && found; ++e) {
        double c[3];
        for (int a = 0; a < 3; ++a) c[a] = 0.5 * (box[6 * e + a] + box[6 * e + 3 + a]);
        const int64_t g = octree_find(root, nodes, c);
        found = g >= 0 && g < n_elem && contains(&box[6 * g], c);
      }
      check(found, "octree: every element centre finds its element");
      check_kernel_octree(root, nodes, box, n_elem);
      lr_octree_free(o);
    }
  }

  // error paths
  {
    lr_forest_host* h = nullptr;
    const int32_t bad[3] = {3, 4, 4};
    check(lr_build_forest(box.data(), n_elem, bad, &h, nullptr) == LR_ENOTPOW2, "forest rejects 3 blocks");
    const int32_t one[3] = {4, 4, 4};
    std::vector<double> gap(box.begin() + 6, box.end());   // drop the first element
    check(lr_build_forest(gap.data(), n_elem - 1, one, &h, nullptr) == LR_EPARTITION, "forest rejects a gap");
    std::vector<double> dup(box);
    dup.insert(dup.end(), box.begin(), box.begin() + 6);   // the first element twice
    check(lr_build_forest(dup.data(), n_elem + 1, one, &h, nullptr) == LR_EPARTITION, "forest rejects an overlap");
    std::vector<double> inexact(box);
    inexact[3] = 1.0 / 3.0;
    check(lr_build_forest(inexact.data(), n_elem, one, &h, nullptr) == LR_EKNOT, "forest rejects a non-FP32 knot");
    check(lr_build_forest(nullptr, n_elem, one, &h, nullptr) == LR_EINVAL, "forest rejects NULL boxes");
    lr_octree_host* o = nullptr;
    check(lr_build_octree(gap.data(), n_elem - 1, &o, nullptr) != LR_OK, "octree rejects a gap");
    check(lr_build_support(knots.data(), n_bspl, kstride, p, box.data(), n_elem, nullptr, nullptr, 0, &nnz) ==
              LR_EINVAL,
          "support rejects NULL csr_ptr");
  }
  std::printf("%s\n", g_fail ? "FAILED" : "ALL OK");
  return g_fail;
}
