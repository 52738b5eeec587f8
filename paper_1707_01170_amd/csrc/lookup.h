// Element look-up descents shared by the kernels and by host checks: the
// k-d forest of Alg. 1 (Sec. 3.2.1) and the octree of a dyadic mesh
// (Sec. 3.2, Sec. 3.2.2).  Plain C++ so that a host build (the sanitizer
// driver) runs exactly this code; hipcc compiles it for both sides.
//
// Both return the element id, or kBadRef when the structure is corrupt: a
// reference to a node beyond n_nodes, an element id >= n_elem, or a descent
// deeper than any valid tree.  The caller reports it (a NaN pixel, -1 in a
// look-up result) instead of reading an element that does not exist.
#pragma once

#include <cstdint>
#include <cstring>

#include "../../include/lrvr.h"

#if defined(__HIPCC__)
#define LR_HD __host__ __device__
#else
#define LR_HD
#endif

namespace lrvr {

constexpr int32_t kBadRef = -1;
constexpr int kMaxForestDepth = 256;   // a depth-balanced tree over < 2^31 elements is far shallower
constexpr int kMaxOctreeDepth = 24;    // knots are multiples of 2^-24

// A forest node as four 32-bit words, 16-byte aligned so that a kernel reads
// it with one 16-byte load: child for p[axis] < split, child otherwise, split
// (FP32 bits), axis.
struct alignas(16) NodeWords {
  uint32_t lo, hi, split, axis;
};

LR_HD inline float bits_to_float(uint32_t u) {
  float f;
  memcpy(&f, &u, sizeof f);
  return f;
}

LR_HD inline int32_t leaf_or_bad(uint32_t r, int64_t n_elem) {
  if (!(r & LR_LEAF)) return kBadRef;
  const int64_t e = (int64_t)(r & ~LR_LEAF);
  return e < n_elem ? (int32_t)e : kBadRef;
}

// Alg. 1: block b = min(floor(p * B), B - 1) per axis, then head -> leaf.
LR_HD inline int32_t forest_lookup(const uint32_t* __restrict__ heads, const lr_kdnode* __restrict__ nodes,
                                   int64_t n_nodes, int64_t n_elem, int32_t bx, int32_t by, int32_t bz, float fbx,
                                   float fby, float fbz, const float p[3]) {
  int ix = (int)(p[0] * fbx), iy = (int)(p[1] * fby), iz = (int)(p[2] * fbz);
  ix = ix < bx - 1 ? ix : bx - 1;
  iy = iy < by - 1 ? iy : by - 1;
  iz = iz < bz - 1 ? iz : bz - 1;
  uint32_t r = heads[((int64_t)iz * by + iy) * bx + ix];
  for (int depth = 0; !(r & LR_LEAF); ++depth) {
    if (depth >= kMaxForestDepth || (int64_t)r >= n_nodes) return kBadRef;
    const NodeWords nd = reinterpret_cast<const NodeWords*>(nodes)[r];
    const float v = nd.axis == 0 ? p[0] : (nd.axis == 1 ? p[1] : p[2]);
    r = v < bits_to_float(nd.split) ? nd.lo : nd.hi;
  }
  return leaf_or_bad(r, n_elem);
}

// Octree descent: one 4-byte child reference per level; the child of a
// level-l cell is picked by bit l+1 of floor(p * 2^(l+1)) per axis (exact in
// FP32: p is scaled by a power of two), clamped at p = 1.
LR_HD inline int32_t octree_lookup(const uint32_t* __restrict__ root, const uint32_t* __restrict__ nodes,
                                   int64_t n_nodes, int64_t n_elem, const float p[3]) {
  uint32_t r = root[0];
  float scale = 2.0f;
  int lim = 1;
  for (int level = 0; !(r & LR_LEAF); ++level) {
    if (level >= kMaxOctreeDepth || (int64_t)r >= n_nodes) return kBadRef;
    int cx = (int)(p[0] * scale), cy = (int)(p[1] * scale), cz = (int)(p[2] * scale);
    cx = (cx < lim ? cx : lim) & 1;
    cy = (cy < lim ? cy : lim) & 1;
    cz = (cz < lim ? cz : lim) & 1;
    r = nodes[8 * (int64_t)r + (cx | (cy << 1) | (cz << 2))];
    scale *= 2.0f;
    lim = 2 * lim + 1;
  }
  return leaf_or_bad(r, n_elem);
}

}  // namespace lrvr
