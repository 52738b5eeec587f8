// Host-side builders of the C ABI (support CSR, k-d forest, octree) run
// under AddressSanitizer and UndefinedBehaviorSanitizer.  Built by
// tests/test_host_sanitize.py with g++ from the library's host sources only
// (no device code).  Input file: int32 p[3], int64 n_bspl, int32 kstride,
// double knots[n_bspl][3][kstride], int64 n_elem, double elem_box[n_elem][6],
// int32 dyadic.  Prints one line per check and exits non-zero on a failure.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lrvr.h"

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

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) return 2;
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
