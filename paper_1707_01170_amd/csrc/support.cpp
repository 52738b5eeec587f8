// Host construction of the element -> B-spline incidence (which LR B-splines
// are non-zero on which element, Eq. 2), the input of the Bezier extraction.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

using lrvr::fail;

LR_API lr_status lr_build_support(const double* knots, int64_t n_bspl, int32_t kstride, const int32_t p[3],
                                  const double* elem_box, int64_t n_elem, int64_t* csr_ptr,
                                  int32_t* csr_idx, int64_t idx_cap, int64_t* nnz) {
  if (!knots || !p || !elem_box || !csr_ptr || !nnz || n_bspl <= 0 || n_elem <= 0)
    return fail(LR_EINVAL, "lr_build_support: null pointer or empty input");
  if (n_bspl >= (int64_t)1 << 31) return fail(LR_EINVAL, "lr_build_support: too many B-splines");
  int pmax = 0;
  for (int d = 0; d < 3; ++d) {
    if (p[d] < 1 || p[d] > 3) return fail(LR_EINVAL, "lr_build_support: degree %d out of [1,3]", p[d]);
    pmax = std::max(pmax, p[d]);
  }
  if (kstride < pmax + 2) return fail(LR_EINVAL, "lr_build_support: kstride %d < max(p)+2", kstride);
  const size_t need = (size_t)(p[0] + 1) * (p[1] + 1) * (p[2] + 1);

  // Support boxes.
  std::vector<double> slo((size_t)n_bspl * 3), shi((size_t)n_bspl * 3), sides((size_t)n_bspl);
  for (int64_t b = 0; b < n_bspl; ++b) {
    for (int d = 0; d < 3; ++d) {
      slo[3 * b + d] = knots[(b * 3 + d) * kstride];
      shi[3 * b + d] = knots[(b * 3 + d) * kstride + p[d] + 1];
      if (!(slo[3 * b + d] < shi[3 * b + d]))
        return fail(LR_EINVAL, "lr_build_support: B-spline %lld has an empty support", (long long)b);
    }
    sides[b] = shi[3 * b] - slo[3 * b];
  }
  // Uniform bucket grid, about two cells per typical support side; every
  // B-spline is listed in each cell its support overlaps.
  std::nth_element(sides.begin(), sides.begin() + sides.size() / 2, sides.end());
  int G = 1;
  while (G < 64 && (double)G * sides[sides.size() / 2] < 2.0) G *= 2;
  auto cell = [&](double x) { return std::min(std::max((int)std::floor(x * G), 0), G - 1); };
  auto hi_cell = [&](double x) { return std::min(std::max((int)std::ceil(x * G) - 1, 0), G - 1); };
  const size_t ncell = (size_t)G * G * G;
  std::vector<int64_t> cstart(ncell + 1, 0);
  for (int64_t b = 0; b < n_bspl; ++b) {
    const int i0 = cell(slo[3 * b]), i1 = hi_cell(shi[3 * b]);
    const int j0 = cell(slo[3 * b + 1]), j1 = hi_cell(shi[3 * b + 1]);
    const int k0 = cell(slo[3 * b + 2]), k1 = hi_cell(shi[3 * b + 2]);
    for (int k = k0; k <= k1; ++k)
      for (int j = j0; j <= j1; ++j)
        for (int i = i0; i <= i1; ++i) ++cstart[((size_t)k * G + j) * G + i + 1];
  }
  for (size_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  std::vector<int32_t> cids((size_t)cstart[ncell]);
  {
    std::vector<int64_t> pos(cstart.begin(), cstart.end() - 1);
    for (int64_t b = 0; b < n_bspl; ++b) {
      const int i0 = cell(slo[3 * b]), i1 = hi_cell(shi[3 * b]);
      const int j0 = cell(slo[3 * b + 1]), j1 = hi_cell(shi[3 * b + 1]);
      const int k0 = cell(slo[3 * b + 2]), k1 = hi_cell(shi[3 * b + 2]);
      for (int k = k0; k <= k1; ++k)
        for (int j = j0; j <= j1; ++j)
          for (int i = i0; i <= i1; ++i) cids[pos[((size_t)k * G + j) * G + i]++] = (int32_t)b;
    }
  }
  // Per element: the B-splines of the bucket of its centre whose support
  // contains the whole element, ascending.
  std::vector<int32_t> all;
  std::vector<int32_t> hit;
  csr_ptr[0] = 0;
  for (int64_t e = 0; e < n_elem; ++e) {
    const double* eb = elem_box + 6 * e;
    const size_t c = ((size_t)cell(0.5 * (eb[2] + eb[5])) * G + cell(0.5 * (eb[1] + eb[4]))) * G +
                     cell(0.5 * (eb[0] + eb[3]));
    hit.clear();
    for (int64_t q = cstart[c]; q < cstart[c + 1]; ++q) {
      const int32_t b = cids[q];
      bool in = true;
      for (int d = 0; d < 3; ++d) in = in && slo[3 * b + d] <= eb[d] && eb[3 + d] <= shi[3 * b + d];
      if (in) hit.push_back(b);
    }
    if (hit.size() < need)
      return fail(LR_EPARTITION, "lr_build_support: element %lld is covered by %zu B-splines (< %zu)",
                  (long long)e, hit.size(), need);
    std::sort(hit.begin(), hit.end());
    all.insert(all.end(), hit.begin(), hit.end());
    csr_ptr[e + 1] = (int64_t)all.size();
  }
  *nnz = (int64_t)all.size();
  if (csr_idx) {
    if (idx_cap < *nnz)
      return fail(LR_ECAPACITY, "lr_build_support: csr_idx holds %lld entries, %lld needed", (long long)idx_cap,
                  (long long)*nnz);
    std::copy(all.begin(), all.end(), csr_idx);
  }
  return LR_OK;
}
