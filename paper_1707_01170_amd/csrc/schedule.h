// Order in which a render launch deals a view's blocks of tiles: from the
// middle of the view outwards.  Plain C++ so that a host build (the sanitizer
// driver) checks exactly this code; hipcc compiles it for both sides.
#pragma once

#include <cmath>
#include <cstdint>

#include "lookup.h"   // LR_HD

namespace lrvr {

// Index r (0-based) of [0, n) counted from the middle outwards: the middle,
// then alternately one to the right and one to the left.
LR_HD inline int center_out(int r, int n) {
  const int c0 = (n - 1) >> 1;
  return (r & 1) ? c0 + ((r + 1) >> 1) : c0 - (r >> 1);
}

// Cell of rank k in a w x h grid ordered by square rings around the middle:
// with columns and rows ranked by center_out, ring m holds the cells whose
// larger rank is m, so the first m * m cells (m <= min(w, h)) fill a centred
// m x m square; past the shorter side the rings are whole columns (or rows).
// A bijection of [0, w h) onto the grid.
LR_HD inline void ring_cell(int64_t k, int w, int h, int& x, int& y) {
  const int sq = w < h ? w : h;
  int rx, ry;
  if (k < (int64_t)sq * sq) {
    int m = (int)sqrtf((float)k);
    while ((int64_t)m * m > k) --m;
    while ((int64_t)(m + 1) * (m + 1) <= k) ++m;
    const int o = (int)(k - (int64_t)m * m);
    if (o <= m) {
      rx = m;
      ry = o;
    } else {
      rx = o - m - 1;
      ry = m;
    }
  } else if (w > h) {
    const int64_t kk = k - (int64_t)sq * sq;
    rx = sq + (int)(kk / h);
    ry = (int)(kk % h);
  } else {
    const int64_t kk = k - (int64_t)sq * sq;
    ry = sq + (int)(kk / w);
    rx = (int)(kk % w);
  }
  x = center_out(rx, w);
  y = center_out(ry, h);
}

}  // namespace lrvr
