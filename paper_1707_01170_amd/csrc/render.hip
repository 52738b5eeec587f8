// Ray casting of LR-spline volumes on gfx950 (Sec. 4): forward render,
// adjoint, single-ray traces and the forest look-up kernel.
//
// Mapping: one workgroup of one 64-lane wavefront renders an 8x8 pixel tile;
// 2x2 blocks of tiles are dealt to the eight XCDs in turn (see locate), which
// spreads the uneven per-pixel work evenly over them, and single-wave
// workgroups let every CU refill at wave granularity.
//
// Per lane the ray keeps its current element (box, step and Bezier block in
// registers) and only descends the k-d forest (Alg. 1) when a sample leaves
// it; since elements are half-open and tile the domain, a sample inside the
// cached box has that element, so the element sequence equals the look-up's.
//
// The library is compiled without floating-point contraction, so sample
// positions are exact sequences of IEEE FP32 operations (the documented ray
// model); evaluation, transfer function and compositing use explicit fmaf.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"
#include "eval.h"
#include "schedule.h"

namespace {

using namespace lrvr;

constexpr int kGroup = 8;             // pixels per workgroup side (one 8x8 tile)
constexpr int kQuad = 2;              // workgroups per side of a block kept on one XCD
constexpr int kThreads = 64;
constexpr int kMaxViews = LR_MAX_VIEWS_PER_LAUNCH;

struct SceneK {
  const float* box;
  const void* bez;
  const uint32_t* heads;
  const void* nodes;        // lr_kdnode (forest) or uint32[8] (octree) records
  const float4* lut;
  int64_t n_elem;
  int64_t n_nodes;
  int64_t stride;           // Bezier row length in coefficients
  int32_t bx, by, bz;
  float fbx, fby, fbz;
  float vmin, inv_range, inv_xi, alpha_clamp, t_term;
  int32_t n_fixed, max_samples;
  int32_t lookup;           // LR_LOOKUP_FOREST or LR_LOOKUP_OCTREE
  int32_t shading;          // LR_SHADE_*
  float light[3];           // unit vector towards a directional light
};

struct ViewsK {
  lr_view v[kMaxViews];
  int64_t quad_base[kMaxViews + 1];    // prefix sums of kQuad x kQuad blocks of tiles
  int32_t quads_x[kMaxViews];
  int32_t n;
  const int32_t* order;                // the dealing order (see locate); null: ring order
  int64_t slot_base[kMaxViews + 1];    // prefix sums of the order's slots per view (see quad_order_kernel)
};

struct Ray {
  float o[3], d[3];
  float t0, t1;
  bool hit;
};

// ---------------------------------------------------------------- ray model
__device__ inline Ray make_ray(const lr_view& v, int i, int j) {
  // Built with -ffp-contract=off: each operator below is one IEEE FP32
  // operation rounded to nearest, / and sqrt correctly rounded.
  Ray r;
  const float W = (float)v.width, H = (float)v.height;
  const float fi = (float)(2 * i + 1), fj = (float)(2 * j + 1);
  const float sx = (fi / W - 1.0f) * v.tx;
  const float sy = (1.0f - fj / H) * v.ty;
  if (v.proj == LR_PERSP) {
    float dp[3];
    for (int a = 0; a < 3; ++a) dp[a] = (v.fwd[a] + sx * v.right[a]) + sy * v.up[a];
    const float n = __builtin_sqrtf((dp[0] * dp[0] + dp[1] * dp[1]) + dp[2] * dp[2]);
    for (int a = 0; a < 3; ++a) {
      r.d[a] = dp[a] / n;
      r.o[a] = v.eye[a];
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      r.o[a] = (v.eye[a] + sx * v.right[a]) + sy * v.up[a];
      r.d[a] = v.fwd[a];
    }
  }
  float t0 = 0.0f, t1 = INFINITY;
  bool hit = true;
  for (int a = 0; a < 3; ++a) {
    if (r.d[a] != 0.0f) {
      const float ta = (0.0f - r.o[a]) / r.d[a];
      const float tb = (1.0f - r.o[a]) / r.d[a];
      t0 = fmaxf(t0, fminf(ta, tb));
      t1 = fminf(t1, fmaxf(ta, tb));
    } else {
      hit = hit && r.o[a] >= 0.0f && r.o[a] <= 1.0f;
    }
  }
  r.t0 = t0;
  r.t1 = t1;
  r.hit = hit && t0 < t1;
  return r;
}

__device__ inline void position(const Ray& r, float t, float p[3]) {
  for (int a = 0; a < 3; ++a) p[a] = fminf(fmaxf(r.o[a] + t * r.d[a], 0.0f), 1.0f);
}

template <int LK>
__device__ inline int32_t find_element(const SceneK& s, const float p[3]) {
  if constexpr (LK == LR_LOOKUP_OCTREE)
    return octree_lookup(s.heads, static_cast<const uint32_t*>(s.nodes), s.n_nodes, s.n_elem, p);
  else
    return forest_lookup(s.heads, static_cast<const lr_kdnode*>(s.nodes), s.n_nodes, s.n_elem, s.bx, s.by, s.bz,
                         s.fbx, s.fby, s.fbz, p);
}

// ---------------------------------------------------------------- transfer function
struct TF {
  float4 rgba;
  float s;       // table position in [0, 255]
  int i0, i1;
  float w;
  bool inside;   // value strictly inside (vmin, vmax): d s / d v != 0
};

__device__ inline TF transfer(const float4* lut, float v, float vmin, float inv_range) {
  TF t;
  float x = (v - vmin) * inv_range;
  t.inside = x > 0.0f && x < 1.0f;
  x = fminf(fmaxf(x, 0.0f), 1.0f);
  t.s = x * 255.0f;
  t.i0 = min((int)t.s, 255);
  t.i1 = min(t.i0 + 1, 255);
  t.w = t.s - (float)t.i0;
  const float4 a = lut[t.i0], b = lut[t.i1];
  t.rgba.x = fmaf(t.w, b.x - a.x, a.x);
  t.rgba.y = fmaf(t.w, b.y - a.y, a.y);
  t.rgba.z = fmaf(t.w, b.z - a.z, a.z);
  t.rgba.w = fmaf(t.w, b.w - a.w, a.w);
  return t;
}

// RGB of hue h in [0,1) at full saturation and value.
// (The hexcone's six sectors written as clamped distances from the sector
// centres of each primary: branch-free.)
__device__ inline void hsv_full(float h, float rgb[3]) {
  const float h6 = h * 6.0f;
  rgb[0] = fminf(fmaxf(fabsf(h6 - 3.0f) - 1.0f, 0.0f), 1.0f);
  rgb[1] = fminf(fmaxf(2.0f - fabsf(h6 - 2.0f), 0.0f), 1.0f);
  rgb[2] = fminf(fmaxf(2.0f - fabsf(h6 - 4.0f), 0.0f), 1.0f);
}

// atan(t) for t in [0, 1] as t * P(t^2), degree 15, coefficients fitted by
// iteratively reweighted least squares on Chebyshev nodes (max error 1.1e-7).
__device__ inline float atan01(float t) {
  const float t2 = t * t;
  float p = -0.004054551012814045f;
  p = fmaf(p, t2, 0.02186291106045246f);
  p = fmaf(p, t2, -0.055912282317876816f);
  p = fmaf(p, t2, 0.09642196446657181f);
  p = fmaf(p, t2, -0.1390863060951233f);
  p = fmaf(p, t2, 0.19946566224098206f);
  p = fmaf(p, t2, -0.33329862356185913f);
  p = fmaf(p, t2, 0.9999993443489075f);
  return t * p;
}

// Hue in [0,1): atan2(fy, fx) / 2pi mod 1, 0 when fx = fy = 0.
__device__ inline float hue_of(float fx, float fy) {
  const float ax = fabsf(fx), ay = fabsf(fy);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  if (mx == 0.0f) return 0.0f;
  float r = atan01(mn * __builtin_amdgcn_rcpf(mx));        // [0, pi/4]
  if (ay > ax) r = 1.5707963267948966f - r;
  if (fx < 0.0f) r = 3.141592653589793f - r;
  float h = r * 0.15915494309189535f;                        // [0, 1/2]
  if (fy < 0.0f) h = 1.0f - h;
  return h >= 1.0f ? 0.0f : h;
}

// a = 1 - (1 - alpha)^r for alpha in [0, 1 - 2^-16], r >= 0, to ~5e-7 relative:
// ln(1 - alpha) by its series below 1/32, else by the hardware log2 with the
// rounding of 1 - alpha corrected by alpha / (1 - u); then -expm1(r ln(1 - alpha))
// by its Taylor polynomial for |.| < 1/8, else by the hardware exp2.
__device__ inline float opacity_of(float alpha, float r) {
  float s = 1.0f / 6.0f;
  s = fmaf(s, alpha, 0.2f);
  s = fmaf(s, alpha, 0.25f);
  s = fmaf(s, alpha, 1.0f / 3.0f);
  s = fmaf(s, alpha, 0.5f);
  s = fmaf(s, alpha, 1.0f);
  const float ser = -alpha * s;
  const float u = 1.0f - alpha;
  const float d = u - 1.0f;
  const float lu = __builtin_amdgcn_logf(u) * 0.6931471805599453f * (alpha * __builtin_amdgcn_rcpf(-d));
  const float L = (alpha < 0.03125f ? ser : lu) * r;
  float e = 1.0f / 5040.0f;
  e = fmaf(e, L, 1.0f / 720.0f);
  e = fmaf(e, L, 1.0f / 120.0f);
  e = fmaf(e, L, 1.0f / 24.0f);
  e = fmaf(e, L, 1.0f / 6.0f);
  e = fmaf(e, L, 0.5f);
  e = fmaf(e, L, 1.0f);
  e *= L;
  const float big = __builtin_amdgcn_exp2f(L * 1.4426950408889634f) - 1.0f;
  return -(L > -0.125f ? e : big);
}

// opacity_of, bit for bit, evaluating the logarithm and the exponential only
// when a lane of the wave needs them (with r = ds / xi small, the series
// cover most waves).  The illuminated degree-2 vector kernel, short of
// registers, runs 4 % faster with it (1080p frame 1.36 -> 1.30 ms, FP16
// blocks 1.31 -> 1.27); the illuminated scalar kernels run 3-11 % slower and
// the unlit ones as fast or slightly slower, so they keep opacity_of.
__device__ inline float opacity_of_uniform(float alpha, float r) {
  float s = 1.0f / 6.0f;
  s = fmaf(s, alpha, 0.2f);
  s = fmaf(s, alpha, 0.25f);
  s = fmaf(s, alpha, 1.0f / 3.0f);
  s = fmaf(s, alpha, 0.5f);
  s = fmaf(s, alpha, 1.0f);
  const float ser = -alpha * s;
  float ln = ser;
  if (__ballot(!(alpha < 0.03125f)) != 0) {
    const float u = 1.0f - alpha;
    const float d = u - 1.0f;
    const float lu = __builtin_amdgcn_logf(u) * 0.6931471805599453f * (alpha * __builtin_amdgcn_rcpf(-d));
    ln = alpha < 0.03125f ? ser : lu;
  }
  const float L = ln * r;
  float e = 1.0f / 5040.0f;
  e = fmaf(e, L, 1.0f / 720.0f);
  e = fmaf(e, L, 1.0f / 120.0f);
  e = fmaf(e, L, 1.0f / 24.0f);
  e = fmaf(e, L, 1.0f / 6.0f);
  e = fmaf(e, L, 0.5f);
  e = fmaf(e, L, 1.0f);
  e *= L;
  if (__ballot(!(L > -0.125f)) != 0) {
    const float big = __builtin_amdgcn_exp2f(L * 1.4426950408889634f) - 1.0f;
    e = L > -0.125f ? e : big;
  }
  return -e;
}

// ---------------------------------------------------------------- the march
// Everything a sample produced that a visitor may need.
template <int P>
struct Sample {
  int32_t e;
  float t, ds;            // sample parameter and composited segment length
  float bx[P + 1], by[P + 1], bz[P + 1];
  float csrc[3];
  float alpha;            // after the clamp
  bool clamped;
  TF tf;
};

// Deferred reloads (DF > 0).  A 16-byte wave load costs the CU's address and
// data units about the same however few lanes it serves, and in most steps
// of a wave some lane enters a new element, so nearly every step paid the
// whole block's loads for a third of the lanes.  With DF > 0 a lane that
// needs a new block waits (takes no sample this step) until at least 1/DF of
// the active lanes need one, or some lane has waited kDeferWait steps; then
// they all load in the same instructions.  Each lane still takes its own
// samples in order, so the results are unchanged.  The visitor hears of each
// step a lane skips (vis.wait()): the adjoint's lanes are inactive in any
// table spill meanwhile.
constexpr int kDeferWait = 3;

template <int P, int NCOMP, typename CT, int MODE, int COLOR, int LK = LR_LOOKUP_FOREST, int SH = 0, int DF = 0,
          class Visitor>
__device__ inline void march(const SceneK& s, const Ray& r, const float4* lut, Visitor& vis) {
  constexpr int NB = (P + 1) * (P + 1) * (P + 1);
  constexpr int NCF = NCOMP * NB;
  using CF = Coef<NCF, CT>;
  typename CF::Reg c[CF::kRegs];
  float lo[3] = {2.0f, 2.0f, 2.0f}, hi[3] = {-1.0f, -1.0f, -1.0f}, inv[3] = {0.0f, 0.0f, 0.0f};
  float ds_e = 0.0f;
  int32_t e = -1;
  const float step_scale = 1.0f / (float)(1 << P);
  float dsf = 0.0f;
  if (MODE == LR_STEP_FIXED) dsf = (r.t1 - r.t0) / (float)s.n_fixed;
  float t = r.t0;
  int n = 0;
  int waited = 0;
  for (;;) {
    float ts;
    if (MODE == LR_STEP_FIXED) {
      if (n >= s.n_fixed) break;
      ts = r.t0 + ((float)n + 0.5f) * dsf;
    } else {
      ts = t;
    }
    float p[3];
    position(r, ts, p);
    // Half-open containment; hi is stored as 2 where the box is closed at 1
    // (positions are clamped to [0,1]), so one comparison per bound suffices.
    const bool need = !(lo[0] <= p[0] && p[0] < hi[0] && lo[1] <= p[1] && p[1] < hi[1] && lo[2] <= p[2] && p[2] < hi[2]);
    if constexpr (DF > 0) {
      const uint64_t m = __ballot(need);
      const uint64_t act = __ballot(1);
      const bool go = __popcll(m) * DF >= __popcll(act) || __ballot(need && waited >= kDeferWait) != 0;
      if (!go && need) {
        ++waited;
        vis.wait();
        continue;
      }
      if (need) waited = 0;
    }
    if (need) {
      e = find_element<LK>(s, p);
      if (e < 0) {           // corrupt look-up structure: the visitor reports it
        vis.corrupt(ts);
        break;
      }
      const float2* b2 = reinterpret_cast<const float2*>(s.box + 6 * (int64_t)e);
      const float2 b01 = b2[0], b23 = b2[1], b45 = b2[2];
      lo[0] = b01.x; lo[1] = b01.y; lo[2] = b23.x;
      hi[0] = b23.y; hi[1] = b45.x; hi[2] = b45.y;
      const float side = fminf(fminf(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
      ds_e = side * step_scale;
      for (int a = 0; a < 3; ++a) inv[a] = __builtin_amdgcn_rcpf(hi[a] - lo[a]);
      for (int a = 0; a < 3; ++a) hi[a] = hi[a] == 1.0f ? 2.0f : hi[a];
      CF::load(s.bez, s.stride, e, c);
    }
    Sample<P> sm;
    sm.e = e;
    sm.t = ts;
    float ds;
    if (MODE == LR_STEP_FIXED) {
      ds = dsf;
      sm.ds = dsf;
    } else {
      ds = ds_e;
      sm.ds = fminf(ds_e, r.t1 - ts);
    }
    const float ux = fminf(fmaxf((p[0] - lo[0]) * inv[0], 0.0f), 1.0f);
    const float uy = fminf(fmaxf((p[1] - lo[1]) * inv[1], 0.0f), 1.0f);
    const float uz = fminf(fmaxf((p[2] - lo[2]) * inv[2], 0.0f), 1.0f);
    if constexpr (SH) {
      // Local illumination (Sec. 4.1): value and gradient from the same block;
      // world gradient = local gradient / element side.
      float dx[P + 1], dy[P + 1], dz[P + 1];
      bernstein_d<P>(ux, sm.bx, dx);
      bernstein_d<P>(uy, sm.by, dy);
      bernstein_d<P>(uz, sm.bz, dz);
      float f[NCOMP], g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < NCOMP; ++q) {
        float o[4];
        contract_grad<P, CF>(c, q * NB, sm.bx, sm.by, sm.bz, dx, dy, dz, o);
        f[q] = o[0];
        const float w = NCOMP == 1 ? 1.0f : o[0];      // grad |f| is parallel to sum_q f_q grad f_q
#pragma unroll
        for (int a = 0; a < 3; ++a) g[a] = fmaf(w, o[1 + a] * inv[a], g[a]);
      }
      const float l[3] = {s.shading == LR_SHADE_HEADLIGHT ? r.d[0] : s.light[0],
                          s.shading == LR_SHADE_HEADLIGHT ? r.d[1] : s.light[1],
                          s.shading == LR_SHADE_HEADLIGHT ? r.d[2] : s.light[2]};
      const float I = diffuse(l, g);
      if constexpr (COLOR == LR_COLOR_HUE) {
        const float vm = __builtin_amdgcn_sqrtf(fmaf(f[0], f[0], fmaf(f[1], f[1], f[2] * f[2])));
        sm.tf = transfer(lut, vm, s.vmin, s.inv_range);
        hsv_full(hue_of(f[0], f[1]), sm.csrc);
      } else {
        sm.tf = transfer(lut, f[0], s.vmin, s.inv_range);
        sm.csrc[0] = sm.tf.rgba.x;
        sm.csrc[1] = sm.tf.rgba.y;
        sm.csrc[2] = sm.tf.rgba.z;
      }
      sm.csrc[0] *= I;
      sm.csrc[1] *= I;
      sm.csrc[2] *= I;
    } else if constexpr (COLOR == LR_COLOR_HUE) {
      bernstein<P>(ux, sm.bx);
      bernstein<P>(uy, sm.by);
      bernstein<P>(uz, sm.bz);
      const float fx = contract<P, CF>(c, 0, sm.bx, sm.by, sm.bz);
      const float fy = contract<P, CF>(c, NB, sm.bx, sm.by, sm.bz);
      const float fz = contract<P, CF>(c, 2 * NB, sm.bx, sm.by, sm.bz);
      const float vm = __builtin_amdgcn_sqrtf(fmaf(fx, fx, fmaf(fy, fy, fz * fz)));
      sm.tf = transfer(lut, vm, s.vmin, s.inv_range);
      hsv_full(hue_of(fx, fy), sm.csrc);
    } else {
      bernstein<P>(ux, sm.bx);
      bernstein<P>(uy, sm.by);
      bernstein<P>(uz, sm.bz);
      const float v = contract<P, CF>(c, 0, sm.bx, sm.by, sm.bz);
      sm.tf = transfer(lut, v, s.vmin, s.inv_range);
      sm.csrc[0] = sm.tf.rgba.x;
      sm.csrc[1] = sm.tf.rgba.y;
      sm.csrc[2] = sm.tf.rgba.z;
    }
    sm.clamped = sm.tf.rgba.w > s.alpha_clamp;
    sm.alpha = fminf(sm.tf.rgba.w, s.alpha_clamp);
    ++n;
    const bool stop = vis.sample(s, sm);
    if (stop || n >= s.max_samples) break;
    if (MODE == LR_STEP_ADAPTIVE) {
      t = ts + ds;
      if (!(t < r.t1)) break;
    }
  }
  vis.finish(n);
}

// Alg. 2 with the transmittance carried multiplicatively:
// a = 1 - (1 - alpha)^(ds/xi), C += T a C_src, T *= 1 - a.  UNIFORM picks
// opacity_of_uniform (the same values).
template <bool UNIFORM = false>
struct CompositeT {
  float C[3] = {0.0f, 0.0f, 0.0f};
  float T = 1.0f;
  bool bad = false;          // the look-up met a corrupt reference
  __device__ inline void corrupt(float) { bad = true; }
  __device__ inline void wait() {}
  __device__ inline float opacity(const SceneK& s, float alpha, float ds) const {
    return UNIFORM ? opacity_of_uniform(alpha, ds * s.inv_xi) : opacity_of(alpha, ds * s.inv_xi);
  }
  template <int P>
  __device__ inline bool sample(const SceneK& s, const Sample<P>& sm) {
    const float a = opacity(s, sm.alpha, sm.ds);
    const float w = T * a;
    C[0] = fmaf(w, sm.csrc[0], C[0]);
    C[1] = fmaf(w, sm.csrc[1], C[1]);
    C[2] = fmaf(w, sm.csrc[2], C[2]);
    T = fmaf(-T, a, T);
    return T <= s.t_term;
  }
  __device__ inline void finish(int) {}
};
using Composite = CompositeT<>;

struct TraceVisitor : Composite {
  float* t_out;
  int32_t* e_out;
  float* ds_out;
  int32_t max_out;
  int32_t k = 0;
  template <int P>
  __device__ inline bool sample(const SceneK& s, const Sample<P>& sm) {
    if (k < max_out) {
      t_out[k] = sm.t;
      e_out[k] = sm.e;
      ds_out[k] = sm.ds;
    }
    ++k;
    return Composite::sample<P>(s, sm);
  }
  // the sample whose look-up failed is recorded with element -1
  __device__ inline void corrupt(float t) {
    bad = true;
    if (k < max_out) {
      t_out[k] = t;
      e_out[k] = kBadRef;
      ds_out[k] = 0.0f;
    }
    ++k;
  }
};

// Work distribution.  The hardware deals consecutive workgroups to the
// eight XCDs in turn: workgroup b runs on XCD b mod 8.  The tiles are grouped
// in blocks of kQuad x kQuad; XCD x renders the blocks x, x + 8, x + 16, ...
// of a view, one workgroup per tile, so a block's rays, which share
// elements, meet in one XCD's L2, while every XCD gets blocks from all over
// the image.  The work per pixel is very uneven (rays through dense regions
// take several times more samples): giving each XCD one contiguous band of
// the image instead left the busiest XCD with ~1.9x the mean work.  Blocks
// are dealt from the middle of the view outwards (ring_cell), because the
// rays through the middle of the volume are the long ones: dispatched first,
// they no longer finish alone at the end of the launch (1080p vector frame
// 1.00 -> 0.88 ms, degree-3 blob view 0.71 -> 0.61, illuminated 1.66 ->
// 1.51, images unchanged; dealt row by row, a one-view launch took 20 %
// longer per view than a launch of four copies of it).  b -> (block, tile)
// is a bijection onto the blocks padded to a multiple of 8; tiles outside
// the image do nothing.  With a dealing order (quad_order_kernel), q indexes
// its slots instead: slot q holds a block of the view, or -1 (nothing).
__device__ inline bool locate(const ViewsK& vk, int64_t b, int& v, int& px, int& py) {
  constexpr int QQ = kQuad * kQuad;
  const int64_t k = b >> 3;
  const int64_t q = (b & 7) + 8 * (k / QQ);
  const int w = (int)(k % QQ);
  v = 0;
  int qx, qy, qw;
  if (vk.order) {
    if (q >= vk.slot_base[vk.n]) return false;
    while (v + 1 < vk.n && q >= vk.slot_base[v + 1]) ++v;
    const int32_t o = vk.order[q];
    if (o < 0) return false;
    qw = vk.quads_x[v];
    qx = o % qw;
    qy = o / qw;
  } else {
    if (q >= vk.quad_base[vk.n]) return false;
    while (v + 1 < vk.n && q >= vk.quad_base[v + 1]) ++v;
    const int64_t lq = q - vk.quad_base[v];
    qw = vk.quads_x[v];
    const int qh = (int)((vk.quad_base[v + 1] - vk.quad_base[v]) / qw);
    ring_cell(lq, qw, qh, qx, qy);
  }
  const int gx = qx * kQuad + w % kQuad;
  const int gy = qy * kQuad + w / kQuad;
  const int lane = threadIdx.x & 63;
  px = gx * kGroup + (lane & 7);
  py = gy * kGroup + (lane >> 3);
  return px < vk.v[v].width && py < vk.v[v].height;
}

// Occupancy of the FP16 vector and degree-3 kernels.  Their registers would
// let 6 waves share a SIMD; at 4, compiled for 4, they run 8-12 % faster.  The
// transfer-table array is padded to 10 KB, so a CU's 160 KB of LDS hold 16
// single-wave workgroups and the compiler sees that bound.  (Reserving the
// same LDS only at launch gives the occupancy without the gain.)  The other
// kernels are limited by their registers or run fastest at full occupancy.
template <int P, int NCOMP, typename CT>
constexpr int lut_rows() {
  return (sizeof(CT) == 2 && (P == 3 || NCOMP == 3)) ? (160 * 1024 / 16) / (int)sizeof(float4) : 256;
}

// Deferral of the forward kernels (see march): reload once half the active
// lanes need a block, with FP32 blocks (1080p vector frame 1.24 -> 0.99 ms,
// degree-3 blob volume 0.80 -> 0.71, through the octree 1.46 -> 0.92,
// degree-2 scalar 0.33 -> 0.31; fixed counts of 8 to 48 lanes and waits of 2
// to 8 steps were no better).  Off where idle lanes cost more than the loads
// saved: FP16 blocks
// are half as many loads (vector frame 0.99 -> 1.16; the serving mix of
// degree-3 scalar views saturates at 2.19e9 instead of 2.47e9 px/s, a 2048^2
// view 1.78 -> 2.00 ms; small degree-3 scalar launches are the exception, see
// render_gathered_f16_kernel), and the illuminated kernels carry the gradient
// contraction as well (1.66 -> 1.78).
template <int P, int NCOMP, typename CT, int SH>
constexpr int defer_divisor() {
  return (SH || !std::is_same<CT, float>::value) ? 0 : 2;
}

__device__ __forceinline__ void load_lut(const SceneK& s, float4* lut) {
  for (int i = threadIdx.x; i < 256; i += kThreads) lut[i] = s.lut[i];
  __syncthreads();
}

// Renders the tile of workgroup index b (see locate), one pixel per lane,
// gathering reloads by DF (see march).
template <int P, int NCOMP, typename CT, int MODE, int COLOR, int LK, int SH, int DF>
__device__ __forceinline__ void render_block(const SceneK& s, const ViewsK& vk, int64_t b, float4* __restrict__ rgba,
                                             uint32_t* __restrict__ nsamples, float4* lut) {
  int v, px, py;
  if (!locate(vk, b, v, px, py)) return;
  const lr_view& view = vk.v[v];
  const int64_t o = view.out_offset + (int64_t)py * view.width + px;
  const Ray r = make_ray(view, px, py);
  struct Counter : CompositeT<SH != 0 && P == 2 && NCOMP == 3> {
    int n = 0;
    __device__ inline void finish(int k) { n = k; }
  } vis;
  if (r.hit) march<P, NCOMP, CT, MODE, COLOR, LK, SH, DF>(s, r, lut, vis);
  rgba[o] = vis.bad ? make_float4(NAN, NAN, NAN, NAN) : make_float4(vis.C[0], vis.C[1], vis.C[2], 1.0f - vis.T);
  if (nsamples) nsamples[o] = (uint32_t)vis.n;
}

template <int P, int NCOMP, typename CT, int MODE, int COLOR, int LK, int SH>
__global__ __launch_bounds__(kThreads) void render_kernel(const SceneK s, const ViewsK vk, float4* __restrict__ rgba,
                                                         uint32_t* __restrict__ nsamples) {
  __shared__ float4 lut[lut_rows<P, NCOMP, CT>()];   // rows beyond 256 are reserved, never touched
  load_lut(s, lut);
  render_block<P, NCOMP, CT, MODE, COLOR, LK, SH, defer_divisor<P, NCOMP, CT, SH>()>(s, vk, blockIdx.x, rgba,
                                                                                     nsamples, lut);
}

// Degree-3 scalar fields from FP16 blocks in launches that do not fill the
// GPU (at most kGatherTiles workgroups): the chain of the longest rays then
// bounds the launch, and gathering the reloads, as the FP32 kernels do,
// shortens it (blob views of 512^2-1280^2 0.80-0.84 -> 0.69-0.71 ms), where
// in fuller launches it costs more than it saves (1448^2 0.85 -> 0.88 ms,
// 2048^2 1.52 -> 1.69, four 1024^2 views in one launch 2.00 -> 2.05).  The
// same image bit for bit.  (Degree-2 scalar views gain nothing from it.)
constexpr int64_t kGatherTiles = 28672;

template <int MODE, int LK>
__global__ __launch_bounds__(kThreads) void render_gathered_f16_kernel(const SceneK s, const ViewsK vk,
                                                                      float4* __restrict__ rgba,
                                                                      uint32_t* __restrict__ nsamples) {
  __shared__ float4 lut[lut_rows<3, 1, _Float16>()];
  load_lut(s, lut);
  render_block<3, 1, _Float16, MODE, LR_COLOR_LUT, LK, 0, 2>(s, vk, blockIdx.x, rgba, nsamples, lut);
}

// Persistent form of the same launch, kept to compare work queues with the
// hardware's dispatch (which is faster here): a grid of resident single-wave
// workgroups takes workgroup indices b from atomic counters and renders tile
// b as workgroup b of render_kernel would, so the image is the same bit for
// bit.  With one counter the indices go out in order to whichever workgroup
// asks; with one counter per XCD, the workgroups g with g mod 8 = x (those the
// hardware deals to XCD x) share the indices b = x, x + 8, ..., the tiles
// workgroup b of render_kernel would render on that XCD.  Counters are 32
// bytes apart and zero at launch; each wave leaves once its counter has passed
// its last index, so the grid drains whatever its size (at least 8 with one
// counter per XCD, so that every counter has workgroups).  The loop holds a
// few more registers; the degree-2 vector kernel is held to render_kernel's 4
// waves per SIMD (128 VGPRs) so that the two differ in dispatch alone.
template <int P, int NCOMP, typename CT>
constexpr int queue_waves() {
  return (P == 2 && NCOMP == 3 && sizeof(CT) == 4) ? 4 : 1;
}

template <int P, int NCOMP, typename CT, int MODE, int COLOR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(queue_waves<P, NCOMP, CT>())))
void render_queue_kernel(const SceneK s, const ViewsK vk, float4* __restrict__ rgba, uint32_t* __restrict__ nsamples,
                         uint32_t* __restrict__ queue, int per_xcd, uint32_t nblk) {
  __shared__ float4 lut[lut_rows<P, NCOMP, CT>()];
  load_lut(s, lut);
  const uint32_t x = per_xcd ? blockIdx.x & 7u : 0u;
  const uint32_t stride = per_xcd ? 8u : 1u;
  const uint32_t items = nblk / stride;   // nblk is a multiple of 8
  for (;;) {
    uint32_t item = 0;
    if (threadIdx.x == 0) item = atomicAdd(&queue[8 * x], 1u);
    item = __shfl(item, 0);
    if (item >= items) break;
    render_block<P, NCOMP, CT, MODE, COLOR, LR_LOOKUP_FOREST, 0, defer_divisor<P, NCOMP, CT, 0>()>(
        s, vk, (int64_t)item * stride + x, rgba, nsamples, lut);
  }
}

__global__ __launch_bounds__(64) void queue_reset_kernel(uint32_t* __restrict__ queue) { queue[threadIdx.x] = 0u; }

// The illuminated degree-2 vector kernel keeps the block, the value and three
// derivatives of each component live: 173-175 VGPRs, 2 waves per SIMD.
// Compiled for 3 waves (168 VGPRs, at most 16 bytes spilled) it runs ~10 %
// faster.  With the registers capped, FP16 blocks are widened to FP32 when
// loaded (F16Widened: 1.89 -> 1.68 ms per 1080p frame against widening in
// every multiply-add).  The degree-3 vector kernel would spill most of its
// block at 3 waves and keeps the plain wrapper.
template <typename CT> struct LitStorage { using type = CT; };
template <> struct LitStorage<_Float16> { using type = F16Widened; };

template <typename CS, int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
void render_lit_vector2_kernel(const SceneK s, const ViewsK vk, float4* __restrict__ rgba,
                               uint32_t* __restrict__ nsamples) {
  __shared__ float4 lut[256];
  load_lut(s, lut);
  render_block<2, 3, CS, MODE, LR_COLOR_HUE, LR_LOOKUP_FOREST, 1, 0>(s, vk, blockIdx.x, rgba, nsamples, lut);
}

template <int P, int NCOMP, typename CT, int MODE, int COLOR, int LK, int SH>
__global__ __launch_bounds__(64) void trace_kernel(const SceneK s, const lr_view view, const int32_t* __restrict__ pix,
                                                   int64_t n, int32_t max_out, float* t_out, int32_t* e_out,
                                                   float* ds_out, int32_t* count) {
  __shared__ float4 lut[256];
  for (int i = threadIdx.x; i < 256; i += 64) lut[i] = s.lut[i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (k >= n) return;
  const int i = pix[2 * k], j = pix[2 * k + 1];
  TraceVisitor vis;
  vis.t_out = t_out + k * max_out;
  vis.e_out = e_out + k * max_out;
  vis.ds_out = ds_out + k * max_out;
  vis.max_out = max_out;
  int taken = 0;
  if (i >= 0 && j >= 0 && i < view.width && j < view.height) {
    const Ray r = make_ray(view, i, j);
    if (r.hit) march<P, NCOMP, CT, MODE, COLOR, LK, SH>(s, r, lut, vis);
    taken = vis.k;
  }
  count[k] = taken;
}

__global__ void lookup_kernel(const uint32_t* __restrict__ heads, const lr_kdnode* __restrict__ nodes, int64_t n_nodes,
                              int64_t n_elem, int32_t bx, int32_t by, int32_t bz, const float* __restrict__ pts, int64_t n,
                              int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float p[3];
  for (int a = 0; a < 3; ++a) p[a] = fminf(fmaxf(pts[3 * k + a], 0.0f), 1.0f);
  out[k] = forest_lookup(heads, nodes, n_nodes, n_elem, bx, by, bz, (float)bx, (float)by, (float)bz, p);
}

__global__ void lookup_octree_kernel(const uint32_t* __restrict__ root, const uint32_t* __restrict__ nodes,
                                     int64_t n_nodes, int64_t n_elem, const float* __restrict__ pts, int64_t n,
                                     int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float p[3];
  for (int a = 0; a < 3; ++a) p[a] = fminf(fmaxf(pts[3 * k + a], 0.0f), 1.0f);
  out[k] = octree_lookup(root, nodes, n_nodes, n_elem, p);
}

// ---------------------------------------------------------------- dispatch order
// The samples a ray takes follow from the element sizes along it (Eq. 4), so
// a block's cost is estimated before the render: half a wavefront per block of
// tiles, 32 points evenly spaced along the block's centre ray, each adding
// its stretch of the ray divided by the smallest side of the element there.
// quad_order_kernel then deals the blocks: groups of 2 x 2 neighbouring
// blocks (32 x 32 pixels, whose rays share elements) go whole to one XCD and
// its L2, ranked by their summed estimates and dealt in snake order (0..7,
// 7..0, ...), so the XCDs get the same number of groups of similar total
// cost; each XCD then takes its blocks longest first.  The order changes no
// pixel; blocks of one level are ordered arbitrarily.
template <int LK>
__global__ __launch_bounds__(64) void quad_cost_kernel(const SceneK s, const ViewsK vk, int fixed,
                                                       float* __restrict__ cost) {
  const int half = threadIdx.x >> 5, lane = threadIdx.x & 31;
  const int64_t q = 2 * (int64_t)blockIdx.x + half;
  const bool valid = q < vk.quad_base[vk.n];
  float c = 0.0f;
  if (valid) {
    int v = 0;
    while (v + 1 < vk.n && q >= vk.quad_base[v + 1]) ++v;
    const int64_t lq = q - vk.quad_base[v];
    const int qw = vk.quads_x[v];
    const int qx = (int)(lq % qw), qy = (int)(lq / qw);
    const lr_view& view = vk.v[v];
    constexpr int kSpan = kQuad * kGroup;
    const int px = min(qx * kSpan + kSpan / 2, view.width - 1);
    const int py = min(qy * kSpan + kSpan / 2, view.height - 1);
    const Ray r = make_ray(view, px, py);
    if (r.hit) {
      const float len = r.t1 - r.t0;
      if (fixed) {
        c = lane == 0 ? (float)s.n_fixed : 0.0f;
      } else {
        float p[3];
        position(r, r.t0 + ((float)lane + 0.5f) * (len * (1.0f / 32.0f)), p);
        const int32_t e = find_element<LK>(s, p);
        if (e >= 0) {
          const float* b = s.box + 6 * (int64_t)e;
          const float side = fminf(fminf(b[3] - b[0], b[4] - b[1]), b[5] - b[2]);
          c = side > 0.0f ? len * (1.0f / 32.0f) / side : 0.0f;
        }
      }
    }
  }
  for (int off = 16; off > 0; off >>= 1) c += __shfl_xor(c, off);   // within each half
  if (valid && lane == 0) cost[q] = c >= 0.0f ? c : 0.0f;
}

constexpr int kOrderThreads = 1024;
constexpr int kOrderLevels = 64;
// Blocks per side of a dealing group.  On the 1080p vector frame: L2-to-
// fabric reads 902 MB per frame when single blocks were dealt to the XCDs by
// rank, 506 MB with 2 x 2 groups (0.784 -> 0.778 ms), 323 MB with 4 x 4
// groups (0.790 ms, small views 1-2 % slower: coarser groups balance worse).
constexpr int kGS = 2;

// One workgroup per view, in two passes over counting sorts on 64 levels.
// First the kGS x kGS groups of blocks are ranked by their summed estimates and
// dealt to the XCDs in snake order, rank r to XCD x(r) (0..7, 7..0, ...),
// recorded in xmap (one entry per group).  Then each XCD's blocks are ranked
// by their own estimates, and block rank k of XCD x goes to slot x + 8 k of
// the view (from vk.slot_base[v]), the index locate gives to the k-th
// block-worth of workgroups the hardware deals to XCD x.  An XCD holds at
// most kGS^2 ceil(groups / 8) blocks, so the slots, 8 kGS^2 ceil(groups / 8)
// per view, suffice; those without a block hold -1.
__global__ __launch_bounds__(kOrderThreads) void quad_order_kernel(const ViewsK vk, const float* __restrict__ cost,
                                                                   int8_t* __restrict__ xmap,
                                                                   int32_t* __restrict__ order) {
  __shared__ float wmax[kOrderThreads / 64];
  __shared__ int32_t first[8][kOrderLevels];
  const int v = blockIdx.x, tid = threadIdx.x;
  const int64_t base = vk.quad_base[v];
  const int qw = vk.quads_x[v];
  const int nq = (int)(vk.quad_base[v + 1] - base);
  const int qh = nq / qw;
  const int gw = (qw + kGS - 1) / kGS, gh = (qh + kGS - 1) / kGS, ng = gw * gh;
  int32_t* const slots = order + vk.slot_base[v];
  int8_t* const xm = xmap + vk.slot_base[v] / (kGS * kGS);   // 8 ceil(ng / 8) >= ng entries per view
  const int nslots = (int)(vk.slot_base[v + 1] - vk.slot_base[v]);
  auto group_cost = [&](int g) {   // the same sum, in the same order, every time
    const int gx = g % gw, gy = g / gw;
    float c = 0.0f;
    for (int j = 0; j < kGS * kGS; ++j) {
      const int qx = kGS * gx + j % kGS, qy = kGS * gy + j / kGS;
      if (qx < qw && qy < qh) c += cost[base + (int64_t)qy * qw + qx];
    }
    return c;
  };
  auto block_max = [&](float m) {   // the workgroup's maximum of m
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((tid & 63) == 0) wmax[tid >> 6] = m;
    __syncthreads();
    float mx = 0.0f;
    for (int w = 0; w < kOrderThreads / 64; ++w) mx = fmaxf(mx, wmax[w]);
    __syncthreads();
    return mx;
  };
  auto level_of = [](float c, float scale) {   // 0 for the costliest
    int l = (int)(c * scale);
    l = l < 0 ? 0 : (l > kOrderLevels - 1 ? kOrderLevels - 1 : l);
    return kOrderLevels - 1 - l;
  };
  auto scan = [&](int rows) {   // exclusive scans of first[0..rows-1][], one wavefront per row
    const int w = tid >> 6, l = tid & 63;
    if (w < rows) {
      const int own = first[w][l];
      int x = own;
      for (int off = 1; off < kOrderLevels; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (l >= off) x += y;
      }
      first[w][l] = x - own;
    }
    __syncthreads();
  };
  for (int i = tid; i < nslots; i += kOrderThreads) slots[i] = -1;
  if (tid < 8 * kOrderLevels) first[tid / kOrderLevels][tid % kOrderLevels] = 0;
  // groups -> XCDs
  float m = 0.0f;
  for (int g = tid; g < ng; g += kOrderThreads) m = fmaxf(m, group_cost(g));
  const float mg = block_max(m);
  const float gscale = mg > 0.0f ? (float)(kOrderLevels - 1) / mg : 0.0f;
  for (int g = tid; g < ng; g += kOrderThreads) atomicAdd(&first[0][level_of(group_cost(g), gscale)], 1);
  __syncthreads();
  scan(1);
  for (int g = tid; g < ng; g += kOrderThreads) {
    const int r = atomicAdd(&first[0][level_of(group_cost(g), gscale)], 1);
    const int round = r >> 3, pos = r & 7;
    xm[g] = (int8_t)((round & 1) ? 7 - pos : pos);
  }
  __syncthreads();   // xm visible to the workgroup; the -1 fill ordered before the writes below
  if (tid < kOrderLevels) first[0][tid] = 0;
  // each XCD's blocks by their own estimates
  m = 0.0f;
  for (int i = tid; i < nq; i += kOrderThreads) m = fmaxf(m, cost[base + i]);
  const float mb = block_max(m);
  const float bscale = mb > 0.0f ? (float)(kOrderLevels - 1) / mb : 0.0f;
  auto xcd_of = [&](int i) { return (int)xm[((i / qw) / kGS) * gw + (i % qw) / kGS]; };
  for (int i = tid; i < nq; i += kOrderThreads) atomicAdd(&first[xcd_of(i)][level_of(cost[base + i], bscale)], 1);
  __syncthreads();
  scan(8);
  for (int i = tid; i < nq; i += kOrderThreads) {
    const int x = xcd_of(i);
    const int k = atomicAdd(&first[x][level_of(cost[base + i], bscale)], 1);
    slots[x + 8 * k] = i;
  }
}

// ---------------------------------------------------------------- adjoint
// Per sample i with T_i the transmittance before it, a_i its opacity and
// C_i = C after it:  dL/dC_src = g_C T_i a_i;
// dL/da_i = g_C . (T_i C_src - (C_final - C_i)/(1 - a_i)) + g_alpha T_final/(1 - a_i);
// da/dalpha = (ds/xi)(1 - a)/(1 - alpha) (0 if clamped); then through the table
// interpolation (LUT rows i0, i1) and s = 255 (v - vmin)/(vmax - vmin) into the
// Bezier coefficients of the sample's element (dv/dC_j = B_j(u)).
//
// Accumulation: a lane sums the gradient of consecutive samples of one
// element in registers; on element change it adds the sums into a small hash
// table in LDS (the 64 rays of an 8x8 tile share most elements): a slot is
// claimed for an element by compare-and-swap on its tag when the lane enters
// the element (its result is read when the lane leaves it; on a collision the
// lane probes on then, linearly), and values are added with LDS FP64 atomics.
// The table has four copies, lane l using copy l mod 4, so that neighbouring
// rays leaving the same element in the same step add to different addresses
// (same-address atomics of one instruction are serialised).  When a lane
// finds its copy full, the wave writes the whole table to global memory with
// atomics, clears it, claims the slots of its current elements again and goes
// on; at the end the workgroup writes what is left.  The table is small so
// that several waves share a SIMD: at one wave per SIMD the ray march's load
// latencies are exposed.  Table-row gradients are summed in registers while
// the row stays the same, then added into an LDS copy of the table (FP64).
// The transfer table itself is read from global memory (L1-resident): an LDS
// read would wait behind the wave's queued atomics.  On gfx950 an LDS FP64
// atomic add to distinct addresses issues ~20x faster than an FP32 one
// (measured ~11 against ~195 CU cycles per wavefront instruction).
//
// The re-march gathers reloads as the forward kernels do (march, DF = 2), so
// the lanes that leave their elements in one step also deposit their sums in
// one set of table atomics (backward 1.85 -> 1.70 ms on the 4 x 512^2 scalar
// step; a third or a quarter of the lanes, or all of them: 1.74 / 1.76 /
// 1.72).  A waiting lane is inactive in any spill meanwhile, so it claims
// its slot again when it deposits (march tells the visitor when a lane
// waits).  A count of spills in LDS, read every step, did the same job but
// cost a wait for the step's queued LDS atomics (1.60 against 1.59 ms);
// spilling at the top of the next step, where every marching lane is
// active, sent the failing lanes' sums to global atomics (2.06 ms).
constexpr int kAdjointDefer = 2;

// Position of table-gradient entry (row, ch) in the LDS array.  Rows are 32
// bytes, so at a plain [row][4] layout the lanes adding channel ch of
// different rows meet in only four bank groups; the channel is XOR-ed with
// bits 2-3 of the row so that 16 consecutive rows use 16 different groups
// (backward 1.59 -> 1.45 ms; bits 3-4 or 4-5: 1.46 / 1.48; a channel-major
// [4][256] layout 1.96).
__device__ inline int lut_grad_index(int row, int ch) { return 4 * row + (ch ^ ((row >> 2) & 3)); }

template <int P>
struct GradTable {
  static constexpr int NB = (P + 1) * (P + 1) * (P + 1);
  static constexpr int kLog2Slots = 3;
  static constexpr int kSlots = 1 << kLog2Slots;   // per copy
  static constexpr int kProbes = kSlots;
  static constexpr int kCopies = 4;                // lane l uses copy l mod 4
};

// The active lanes write every non-zero entry of the element table to the
// global gradient (FP32 atomics), clear the table and count the spill.  The wave's LDS
// operations complete in order, so every tag is read before it is cleared.
template <int NB, int S>
__device__ inline void spill_table(float* __restrict__ gbez, int64_t stride, int32_t* htag, double* hval) {
  const uint64_t act = __ballot(1);
  const int na = __popcll(act);
  const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
  for (int i = rank; i < S * NB; i += na) {
    const int32_t t = htag[i / NB];
    const double v = hval[i];
    if (t >= 0 && v != 0.0) unsafeAtomicAdd(gbez + (int64_t)t * stride + (i % NB), (float)v);
    hval[i] = 0.0;
  }
  for (int i = rank; i < S; i += na) htag[i] = -1;
}

template <int P>
struct Adjoint : Composite {
  static constexpr int NB = GradTable<P>::NB;
  static constexpr int kSlots = GradTable<P>::kSlots;
  float Cfin[3];
  float Tfin;
  float gC[3];
  float gA;
  float* gbez;
  int64_t stride;
  double* glut_s;             // LDS [256][4], channels swizzled (lut_grad_index)
  int32_t* htag;              // LDS [kSlots]: element id or -1
  double* hval;               // LDS [kSlots][NB]
  bool waited = false;        // the lane skipped a step since its last claim
  float range_scale;          // 255 / (vmax - vmin)
  const float4* lut;
  int32_t cur = -1;
  uint32_t h_cur = 0;         // hash slot of cur
  int32_t claim = -1;         // what the claim of h_cur found (-1: free, now cur's)
  float acc[NB];
  int32_t row = -1;           // table row i0 being accumulated
  float g0[4], g1[4];         // sums for rows i0 and min(i0 + 1, 255)

  __device__ inline void flush_row() {
    if (row >= 0) {
      const int r1 = row < 255 ? row + 1 : 255;
      for (int ch = 0; ch < 4; ++ch) {
        atomicAdd(&glut_s[lut_grad_index(row, ch)], (double)g0[ch]);
        atomicAdd(&glut_s[lut_grad_index(r1, ch)], (double)g1[ch]);
      }
    }
  }

  // Slot of cur: the one claimed on entry, else by linear probing; -1 if the
  // table is full.
  __device__ inline int32_t resolve() {
    if (claim == -1 || claim == cur) return (int32_t)h_cur;
    const uint32_t base = h_cur & ~(uint32_t)(kSlots - 1);
    uint32_t h = (h_cur + 1) & (kSlots - 1);
    for (int probe = 1; probe < GradTable<P>::kProbes; ++probe) {
      const int32_t t = atomicCAS(&htag[base + h], -1, cur);
      if (t == -1 || t == cur) return (int32_t)(base + h);
      h = (h + 1) & (kSlots - 1);
    }
    return -1;
  }

  // Adds the sums of the element the lane leaves (cur) into the table.  Every
  // active lane calls it (with cur < 0 if it has nothing to add), so that a
  // full table can be spilled by the whole wave.  A lane that waited for a
  // gathered reload step was inactive in any spill meanwhile, so its entry
  // claim may be stale: it claims again.
  __device__ inline void deposit(bool want) {
    if (want && waited) claim = atomicCAS(&htag[h_cur], -1, cur);
    int32_t ref = want ? resolve() : 0;
    if (__ballot(want && ref < 0)) {
      spill_table<NB, kSlots * GradTable<P>::kCopies>(gbez, stride, htag, hval);
      if (cur >= 0) claim = atomicCAS(&htag[h_cur], -1, cur);
      if (want) ref = resolve();
    }
    if (!want) return;
    if (ref >= 0) {
      double* v = hval + ref * NB;
#pragma unroll
      for (int j = 0; j < NB; ++j) atomicAdd(v + j, (double)acc[j]);   // straight-line, no per-value branches
      return;
    }
    float* out = gbez + (int64_t)cur * stride;             // still no slot: straight to global memory
#pragma unroll
    for (int j = 0; j < NB; ++j)
      if (acc[j] != 0.0f) unsafeAtomicAdd(out + j, acc[j]);
  }
  __device__ inline void wait() { waited = true; }

  __device__ inline bool sample(const SceneK& s, const Sample<P>& sm) {
    const float a = opacity(s, sm.alpha, sm.ds);
    const float w = T * a;
    float Cn[3];
    for (int ch = 0; ch < 3; ++ch) Cn[ch] = fmaf(w, sm.csrc[ch], C[ch]);
    // om = 0: the opacity rounded to 1, T becomes 0 and the march ends at
    // this sample; nothing follows it (suffix 0, later transmittance 1), and
    // g_a only reaches the table through da/dalpha, which has the factor om.
    const float om = 1.0f - a;
    const bool live = om > 0.0f;
    // hardware reciprocals (~1 ulp) in place of correctly rounded divisions
    // (five of those cost ~60 instructions per sample; 1.72 -> 1.62 ms):
    // these values feed only the gradient, never the march
    const float inv_om = live ? __builtin_amdgcn_rcpf(om) : 0.0f;
    float g_a = live ? gA * Tfin * inv_om : gA * T;
    float g_x[4];
    for (int ch = 0; ch < 3; ++ch) {
      g_x[ch] = gC[ch] * w;
      g_a = fmaf(gC[ch], T * sm.csrc[ch] - (Cfin[ch] - Cn[ch]) * inv_om, g_a);
    }
    const float r = sm.ds * s.inv_xi;
    g_x[3] = sm.clamped ? 0.0f : g_a * r * om * __builtin_amdgcn_rcpf(1.0f - sm.alpha);
    // table rows
    if (sm.tf.i0 != row) {
      flush_row();
      row = sm.tf.i0;
      for (int ch = 0; ch < 4; ++ch) g0[ch] = g1[ch] = 0.0f;
    }
    const float w1 = sm.tf.w, w0 = 1.0f - sm.tf.w;
    for (int ch = 0; ch < 4; ++ch) {
      g0[ch] = fmaf(w0, g_x[ch], g0[ch]);
      g1[ch] = fmaf(w1, g_x[ch], g1[ch]);
    }
    const float4 l0 = lut[sm.tf.i0], l1 = lut[sm.tf.i1];
    float g_s = g_x[0] * (l1.x - l0.x);
    g_s = fmaf(g_x[1], l1.y - l0.y, g_s);
    g_s = fmaf(g_x[2], l1.z - l0.z, g_s);
    g_s = fmaf(g_x[3], l1.w - l0.w, g_s);
    const float g_v = sm.tf.inside ? g_s * range_scale : 0.0f;
    const bool enter = sm.e != cur;
    deposit(enter && cur >= 0);
    if (enter) {
      cur = sm.e;
      waited = false;
      // Claim the element's slot now; the result is first needed when the
      // lane leaves the element, so the compare-and-swap's latency is hidden
      // behind the element's samples.
      h_cur = (((uint32_t)cur * 2654435761u) >> (32 - GradTable<P>::kLog2Slots)) +
              (threadIdx.x & (GradTable<P>::kCopies - 1)) * kSlots;
      claim = atomicCAS(&htag[h_cur], -1, cur);
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[j] = 0.0f;
    }
    constexpr int Q = P + 1;
#pragma unroll
    for (int kz = 0; kz < Q; ++kz)
#pragma unroll
      for (int jy = 0; jy < Q; ++jy) {
        const float gyz = g_v * sm.by[jy] * sm.bz[kz];
#pragma unroll
        for (int ix = 0; ix < Q; ++ix) acc[(kz * Q + jy) * Q + ix] = fmaf(gyz, sm.bx[ix], acc[(kz * Q + jy) * Q + ix]);
      }
    C[0] = Cn[0];
    C[1] = Cn[1];
    C[2] = Cn[2];
    T = fmaf(-T, a, T);
    return T <= s.t_term;
  }
  __device__ inline void finish(int) {
    // A lane whose ray ended early waited here while the others marched on;
    // if they spilled the table meanwhile, its claim is stale: claim again.
    if (cur >= 0) claim = atomicCAS(&htag[h_cur], -1, cur);
    waited = false;
    deposit(cur >= 0);
    flush_row();
  }
};

template <int P, int MODE, int LK>
__global__ __launch_bounds__(kThreads) void backward_kernel(const SceneK s, const ViewsK vk, const float4* __restrict__ fwd,
                                                           const float4* __restrict__ grad, float* __restrict__ gbez,
                                                           float* __restrict__ glut) {
  constexpr int NB = GradTable<P>::NB, S = GradTable<P>::kSlots * GradTable<P>::kCopies;
  __shared__ double glut_s[1024];
  __shared__ int32_t htag[S];
  __shared__ double hval[S * NB];
  for (int i = threadIdx.x; i < 1024; i += kThreads) glut_s[i] = 0.0;
  for (int i = threadIdx.x; i < S; i += kThreads) htag[i] = -1;
  for (int i = threadIdx.x; i < S * NB; i += kThreads) hval[i] = 0.0;
  __syncthreads();
  int v, px, py;
  if (locate(vk, blockIdx.x, v, px, py)) {
    const lr_view& view = vk.v[v];
    const int64_t o = view.out_offset + (int64_t)py * view.width + px;
    const Ray r = make_ray(view, px, py);
    const float4 gr = grad[o];
    if (r.hit && (gr.x != 0.0f || gr.y != 0.0f || gr.z != 0.0f || gr.w != 0.0f)) {
      const float4 f = fwd[o];
      Adjoint<P> vis;
      vis.Cfin[0] = f.x;
      vis.Cfin[1] = f.y;
      vis.Cfin[2] = f.z;
      vis.Tfin = 1.0f - f.w;
      vis.gC[0] = gr.x;
      vis.gC[1] = gr.y;
      vis.gC[2] = gr.z;
      vis.gA = gr.w;
      vis.gbez = gbez;
      vis.stride = s.stride;
      vis.glut_s = glut_s;
      vis.htag = htag;
      vis.hval = hval;
      vis.range_scale = 255.0f * s.inv_range;
      vis.lut = s.lut;
      march<P, 1, float, MODE, LR_COLOR_LUT, LK, 0, kAdjointDefer>(s, r, s.lut, vis);
    }
  }
  __syncthreads();
  // write what is left of the block's element sums and its table gradient
  for (int i = threadIdx.x; i < S * NB; i += kThreads) {
    const int32_t t = htag[i / NB];
    if (t >= 0 && hval[i] != 0.0) unsafeAtomicAdd(gbez + (int64_t)t * s.stride + (i % NB), (float)hval[i]);
  }
  for (int i = threadIdx.x; i < 1024; i += kThreads) {
    const int row = i >> 2, ch = (i & 3) ^ ((row >> 2) & 3);   // the inverse of lut_grad_index
    if (glut_s[i] != 0.0) unsafeAtomicAdd(glut + 4 * row + ch, (float)glut_s[i]);
  }
}

// ---------------------------------------------------------------- host side
lr_status make_scene(const lr_scene* sc, SceneK& s, bool need_forest = true) {
  using lrvr::fail;
  if (!sc) return fail(LR_EINVAL, "null scene");
  const int P = sc->p[0];
  if (sc->p[1] != P || sc->p[2] != P || P < 1 || P > 3)
    return fail(LR_EINVAL, "render kernels take equal degrees p1 = p2 = p3 in [1,3]");
  if (!((sc->ncomp == 1 && sc->color_mode == LR_COLOR_LUT) || (sc->ncomp == 3 && sc->color_mode == LR_COLOR_HUE)))
    return fail(LR_EINVAL, "ncomp/color_mode must be 1/LR_COLOR_LUT or 3/LR_COLOR_HUE");
  if (sc->bezier_dtype != LR_F32 && sc->bezier_dtype != LR_F16)
    return fail(LR_EINVAL, "bezier_dtype must be LR_F32 or LR_F16");
  if (sc->step_mode != LR_STEP_FIXED && sc->step_mode != LR_STEP_ADAPTIVE) return fail(LR_EINVAL, "bad step_mode");
  if (sc->step_mode == LR_STEP_FIXED && sc->n_fixed_steps < 1) return fail(LR_EINVAL, "n_fixed_steps < 1");
  if (sc->max_samples < 1) return fail(LR_EINVAL, "max_samples < 1");
  if (!sc->elem_box || !sc->bezier || !sc->lut || (need_forest && (!sc->heads || (!sc->nodes && sc->n_nodes > 0))))
    return fail(LR_EINVAL, "null device array in the scene");
  if (sc->n_elem <= 0 || sc->n_elem >= (int64_t)LR_LEAF || sc->n_nodes < 0) return fail(LR_EINVAL, "bad n_elem / n_nodes");
  if (sc->lookup != LR_LOOKUP_FOREST && sc->lookup != LR_LOOKUP_OCTREE)
    return fail(LR_EINVAL, "lookup must be LR_LOOKUP_FOREST or LR_LOOKUP_OCTREE");
  if (sc->n_nodes >= (int64_t)LR_LEAF) return fail(LR_EINVAL, "too many look-up nodes");
  if (sc->shading != LR_SHADE_NONE && sc->shading != LR_SHADE_DIRECTIONAL && sc->shading != LR_SHADE_HEADLIGHT)
    return fail(LR_EINVAL, "shading must be LR_SHADE_NONE, LR_SHADE_DIRECTIONAL or LR_SHADE_HEADLIGHT");
  if (sc->shading != LR_SHADE_NONE && sc->lookup != LR_LOOKUP_FOREST)
    return fail(LR_EINVAL, "shading is implemented with the forest look-up");
  const double ln = std::sqrt((double)sc->light[0] * sc->light[0] + (double)sc->light[1] * sc->light[1] +
                              (double)sc->light[2] * sc->light[2]);
  if (sc->shading == LR_SHADE_DIRECTIONAL && !(ln > 0.0 && std::isfinite(ln)))
    return fail(LR_EINVAL, "directional shading needs a finite non-zero light vector");
  if (sc->lookup == LR_LOOKUP_FOREST)
    for (int d = 0; d < 3; ++d)
      if (!lrvr::is_pow2(sc->blocks[d]) || sc->blocks[d] > 512) return fail(LR_ENOTPOW2, "blocks must be powers of two <= 512");
  if (!(sc->vmax > sc->vmin) || !(sc->xi > 0.0f) || !(sc->alpha_clamp < 1.0f) || !(sc->alpha_clamp >= 0.0f) ||
      !(sc->term_alpha > 0.0f && sc->term_alpha <= 1.0f))
    return fail(LR_EINVAL, "need vmax > vmin, xi > 0, 0 <= alpha_clamp < 1, 0 < term_alpha <= 1");
  s.box = sc->elem_box;
  s.bez = sc->bezier;
  s.heads = sc->heads;
  s.nodes = sc->nodes;
  s.lut = reinterpret_cast<const float4*>(sc->lut);
  s.n_elem = sc->n_elem;
  s.n_nodes = sc->n_nodes;
  s.stride = lr_bezier_stride(sc->p, sc->ncomp, sc->bezier_dtype);
  s.lookup = sc->lookup;
  s.shading = sc->shading;
  for (int a = 0; a < 3; ++a) s.light[a] = sc->shading == LR_SHADE_DIRECTIONAL ? (float)(sc->light[a] / ln) : 0.0f;
  const bool oct = sc->lookup == LR_LOOKUP_OCTREE;
  s.bx = oct ? 1 : sc->blocks[0];
  s.by = oct ? 1 : sc->blocks[1];
  s.bz = oct ? 1 : sc->blocks[2];
  s.fbx = (float)s.bx;
  s.fby = (float)s.by;
  s.fbz = (float)s.bz;
  s.vmin = sc->vmin;
  s.inv_range = (float)(1.0 / ((double)sc->vmax - (double)sc->vmin));
  s.inv_xi = (float)(1.0 / (double)sc->xi);
  s.alpha_clamp = sc->alpha_clamp;
  s.t_term = (float)(1.0 - (double)sc->term_alpha);
  s.n_fixed = sc->n_fixed_steps;
  s.max_samples = sc->max_samples;
  return LR_OK;
}

lr_status check_view(const lr_view& v) {
  if (v.proj != LR_PERSP && v.proj != LR_ORTHO) return lrvr::fail(LR_EINVAL, "view: bad projection");
  if (v.width < 1 || v.height < 1 || v.width > (1 << 16) || v.height > (1 << 16) || v.out_offset < 0)
    return lrvr::fail(LR_EINVAL, "view: size must be 1..65536 and out_offset >= 0");
  const float* f = v.eye;
  for (int i = 0; i < 14; ++i)
    if (!std::isfinite(f[i])) return lrvr::fail(LR_EINVAL, "view: non-finite camera value");
  return LR_OK;
}

// Packs up to kMaxViews views; returns the number of workgroups.
int64_t pack_views(const lr_view* views, int32_t n, ViewsK& vk) {
  std::memset(&vk, 0, sizeof vk);
  vk.n = n;
  vk.quad_base[0] = 0;
  for (int i = 0; i < n; ++i) {
    vk.v[i] = views[i];
    const int64_t gx = (views[i].width + kGroup - 1) / kGroup, gy = (views[i].height + kGroup - 1) / kGroup;
    vk.quads_x[i] = (int32_t)((gx + kQuad - 1) / kQuad);
    const int64_t qh = (gy + kQuad - 1) / kQuad;
    vk.quad_base[i + 1] = vk.quad_base[i] + (int64_t)vk.quads_x[i] * qh;
    const int64_t groups = ((vk.quads_x[i] + kGS - 1) / kGS) * ((qh + kGS - 1) / kGS);   // kGS x kGS blocks each
    vk.slot_base[i + 1] = vk.slot_base[i] + 8 * kGS * kGS * ((groups + 7) / 8);
  }
  return 8 * ((vk.quad_base[n] + 7) / 8) * (int64_t)kQuad * kQuad;   // workgroups to launch in ring order
}

// Workgroups of a launch dealt by its dealing order: one per tile slot.
int64_t ordered_workgroups(const ViewsK& vk) { return vk.slot_base[vk.n] * kQuad * kQuad; }

template <int P, int NCOMP, typename CT, int MODE, int COLOR>
void launch_render(const SceneK& s, const ViewsK& vk, int64_t nblk, float* rgba, uint32_t* ns, hipStream_t st) {
  // Variants: forest or octree look-up without shading; forest with shading.
  float4* out = reinterpret_cast<float4*>(rgba);
  if (s.shading != LR_SHADE_NONE) {
    if constexpr (P == 2 && NCOMP == 3)
      hipLaunchKernelGGL((render_lit_vector2_kernel<typename LitStorage<CT>::type, MODE>), dim3((unsigned)nblk),
                         dim3(kThreads), 0, st, s, vk, out, ns);
    else
      hipLaunchKernelGGL((render_kernel<P, NCOMP, CT, MODE, COLOR, LR_LOOKUP_FOREST, 1>), dim3((unsigned)nblk),
                         dim3(kThreads), 0, st, s, vk, out, ns);
    return;
  }
  if constexpr (P == 3 && NCOMP == 1 && std::is_same<CT, _Float16>::value) {
    if (nblk <= kGatherTiles) {
      if (s.lookup == LR_LOOKUP_OCTREE)
        hipLaunchKernelGGL((render_gathered_f16_kernel<MODE, LR_LOOKUP_OCTREE>), dim3((unsigned)nblk), dim3(kThreads),
                           0, st, s, vk, out, ns);
      else
        hipLaunchKernelGGL((render_gathered_f16_kernel<MODE, LR_LOOKUP_FOREST>), dim3((unsigned)nblk), dim3(kThreads),
                           0, st, s, vk, out, ns);
      return;
    }
  }
  if (s.lookup == LR_LOOKUP_OCTREE)
    hipLaunchKernelGGL((render_kernel<P, NCOMP, CT, MODE, COLOR, LR_LOOKUP_OCTREE, 0>), dim3((unsigned)nblk),
                       dim3(kThreads), 0, st, s, vk, out, ns);
  else
    hipLaunchKernelGGL((render_kernel<P, NCOMP, CT, MODE, COLOR, LR_LOOKUP_FOREST, 0>), dim3((unsigned)nblk),
                       dim3(kThreads), 0, st, s, vk, out, ns);
}

template <int P, int NCOMP, int COLOR>
void dispatch_dtype_mode(const lr_scene* sc, const SceneK& s, const ViewsK& vk, int64_t nblk, float* rgba, uint32_t* ns,
                         hipStream_t st) {
  const bool f16 = sc->bezier_dtype == LR_F16;
  if (sc->step_mode == LR_STEP_FIXED) {
    if (f16) launch_render<P, NCOMP, _Float16, LR_STEP_FIXED, COLOR>(s, vk, nblk, rgba, ns, st);
    else launch_render<P, NCOMP, float, LR_STEP_FIXED, COLOR>(s, vk, nblk, rgba, ns, st);
  } else {
    if (f16) launch_render<P, NCOMP, _Float16, LR_STEP_ADAPTIVE, COLOR>(s, vk, nblk, rgba, ns, st);
    else launch_render<P, NCOMP, float, LR_STEP_ADAPTIVE, COLOR>(s, vk, nblk, rgba, ns, st);
  }
}

template <int P>
void dispatch_render(const lr_scene* sc, const SceneK& s, const ViewsK& vk, int64_t nblk, float* rgba, uint32_t* ns,
                     hipStream_t st) {
  if (sc->ncomp == 1) dispatch_dtype_mode<P, 1, LR_COLOR_LUT>(sc, s, vk, nblk, rgba, ns, st);
  else dispatch_dtype_mode<P, 3, LR_COLOR_HUE>(sc, s, vk, nblk, rgba, ns, st);
}

// Persistent launch: zeroes the counters, then starts `workgroups` resident
// workgroups (0: as many as the GPU holds at once), rounded up to a multiple
// of 8.
template <int P, int NCOMP, typename CT, int MODE, int COLOR>
hipError_t launch_queue(const SceneK& s, const ViewsK& vk, int64_t nblk, float* rgba, uint32_t* ns, uint32_t* queue,
                        int queues, int workgroups, hipStream_t st) {
  const auto kern = render_queue_kernel<P, NCOMP, CT, MODE, COLOR>;
  int grid = workgroups;
  if (grid <= 0) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, 0);
    if (e != hipSuccess) return e;
    grid = per_cu * cus;
  }
  grid = grid < 8 ? 8 : (grid + 7) / 8 * 8;
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, st, queue);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), 0, st, s, vk, reinterpret_cast<float4*>(rgba), ns,
                     queue, queues == 8 ? 1 : 0, (uint32_t)nblk);
  return hipSuccess;
}

template <int P, int NCOMP, int COLOR>
hipError_t queue_dtype_mode(const lr_scene* sc, const SceneK& s, const ViewsK& vk, int64_t nblk, float* rgba,
                            uint32_t* ns, uint32_t* queue, int queues, int workgroups, hipStream_t st) {
  const bool f16 = sc->bezier_dtype == LR_F16;
  if (sc->step_mode == LR_STEP_FIXED)
    return f16 ? launch_queue<P, NCOMP, _Float16, LR_STEP_FIXED, COLOR>(s, vk, nblk, rgba, ns, queue, queues, workgroups, st)
               : launch_queue<P, NCOMP, float, LR_STEP_FIXED, COLOR>(s, vk, nblk, rgba, ns, queue, queues, workgroups, st);
  return f16 ? launch_queue<P, NCOMP, _Float16, LR_STEP_ADAPTIVE, COLOR>(s, vk, nblk, rgba, ns, queue, queues, workgroups, st)
             : launch_queue<P, NCOMP, float, LR_STEP_ADAPTIVE, COLOR>(s, vk, nblk, rgba, ns, queue, queues, workgroups, st);
}

template <int P>
hipError_t dispatch_queue(const lr_scene* sc, const SceneK& s, const ViewsK& vk, int64_t nblk, float* rgba,
                          uint32_t* ns, uint32_t* queue, int queues, int workgroups, hipStream_t st) {
  if (sc->ncomp == 1)
    return queue_dtype_mode<P, 1, LR_COLOR_LUT>(sc, s, vk, nblk, rgba, ns, queue, queues, workgroups, st);
  return queue_dtype_mode<P, 3, LR_COLOR_HUE>(sc, s, vk, nblk, rgba, ns, queue, queues, workgroups, st);
}

template <int P, int NCOMP, typename CT, int MODE, int COLOR>
void launch_trace(const SceneK& s, const lr_view& v, const int32_t* pix, int64_t n, int32_t m, float* t, int32_t* e,
                  float* ds, int32_t* cnt, hipStream_t st) {
  const dim3 grid((unsigned)((n + 63) / 64));
  if (s.shading != LR_SHADE_NONE)
    hipLaunchKernelGGL((trace_kernel<P, NCOMP, CT, MODE, COLOR, LR_LOOKUP_FOREST, 1>), grid, dim3(64), 0, st, s, v, pix,
                       n, m, t, e, ds, cnt);
  else if (s.lookup == LR_LOOKUP_OCTREE)
    hipLaunchKernelGGL((trace_kernel<P, NCOMP, CT, MODE, COLOR, LR_LOOKUP_OCTREE, 0>), grid, dim3(64), 0, st, s, v, pix,
                       n, m, t, e, ds, cnt);
  else
    hipLaunchKernelGGL((trace_kernel<P, NCOMP, CT, MODE, COLOR, LR_LOOKUP_FOREST, 0>), grid, dim3(64), 0, st, s, v, pix,
                       n, m, t, e, ds, cnt);
}

template <int P>
void dispatch_trace(const lr_scene* sc, const SceneK& s, const lr_view& v, const int32_t* pix, int64_t n, int32_t m,
                    float* t, int32_t* e, float* ds, int32_t* cnt, hipStream_t st) {
  const bool f16 = sc->bezier_dtype == LR_F16, fixed = sc->step_mode == LR_STEP_FIXED;
#define LR_TRACE(NC, COL)                                                                                  \
  if (fixed) {                                                                                             \
    if (f16) launch_trace<P, NC, _Float16, LR_STEP_FIXED, COL>(s, v, pix, n, m, t, e, ds, cnt, st);        \
    else launch_trace<P, NC, float, LR_STEP_FIXED, COL>(s, v, pix, n, m, t, e, ds, cnt, st);               \
  } else {                                                                                                 \
    if (f16) launch_trace<P, NC, _Float16, LR_STEP_ADAPTIVE, COL>(s, v, pix, n, m, t, e, ds, cnt, st);     \
    else launch_trace<P, NC, float, LR_STEP_ADAPTIVE, COL>(s, v, pix, n, m, t, e, ds, cnt, st);            \
  }
  if (sc->ncomp == 1) {
    LR_TRACE(1, LR_COLOR_LUT)
  } else {
    LR_TRACE(3, LR_COLOR_HUE)
  }
#undef LR_TRACE
}

}  // namespace

using lrvr::fail;

// Bytes of the dispatch-order workspace for one launch: the blocks' estimates
// (4 bytes each), the groups' XCDs (1 byte per 4 slots) and the order (4
// bytes per slot), each 256-byte aligned.
static int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }
static int64_t cost_bytes(const ViewsK& vk) { return round256(vk.quad_base[vk.n] * 4); }
static int64_t xmap_bytes(const ViewsK& vk) { return round256(vk.slot_base[vk.n] / (kGS * kGS)); }
static int64_t order_bytes(const ViewsK& vk) {
  return cost_bytes(vk) + xmap_bytes(vk) + round256(vk.slot_base[vk.n] * 4);
}

// Largest workspace any launch of these views needs (views in launches of
// kMaxViews); -1 if a launch would be too large.
static int64_t order_workspace(const lr_view* views, int32_t n_views) {
  int64_t need = 0;
  for (int base = 0; base < n_views; base += kMaxViews) {
    const int cnt = n_views - base < kMaxViews ? n_views - base : kMaxViews;
    ViewsK vk;
    const int64_t nblk = pack_views(views + base, cnt, vk);
    if (nblk <= 0 || nblk > 0x7fffffff || ordered_workgroups(vk) > 0x7fffffff) return -1;
    const int64_t b = order_bytes(vk);
    need = b > need ? b : need;
  }
  return need;
}

// Estimates the blocks' costs and deals them into ws (order_bytes of the
// launch), and points vk at the order.
static void schedule(const lr_scene* sc, const SceneK& s, ViewsK& vk, void* ws, hipStream_t st) {
  const int64_t nq = vk.quad_base[vk.n];
  float* cost = static_cast<float*>(ws);
  int8_t* xmap = reinterpret_cast<int8_t*>(static_cast<char*>(ws) + cost_bytes(vk));
  int32_t* order = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + cost_bytes(vk) + xmap_bytes(vk));
  const int fixed = sc->step_mode == LR_STEP_FIXED;
  if (s.lookup == LR_LOOKUP_OCTREE)
    hipLaunchKernelGGL(quad_cost_kernel<LR_LOOKUP_OCTREE>, dim3((unsigned)((nq + 1) / 2)), dim3(64), 0, st, s, vk,
                       fixed, cost);
  else
    hipLaunchKernelGGL(quad_cost_kernel<LR_LOOKUP_FOREST>, dim3((unsigned)((nq + 1) / 2)), dim3(64), 0, st, s, vk,
                       fixed, cost);
  hipLaunchKernelGGL(quad_order_kernel, dim3((unsigned)vk.n), dim3(kOrderThreads), 0, st, vk, cost, xmap, order);
  vk.order = order;
}

// How a launch's blocks reach the GPU: in ring order or longest first
// (cost_order, the order in the workspace), through the hardware's dispatch
// (queues 0) or persistent workgroups taking them from 1 or 8 counters (the
// first 256 bytes of the workspace, free once the order is made).
struct Dispatch {
  bool cost_order = false;
  int queues = 0;
  int workgroups = 0;
};

// lr_render, lr_render_scheduled and lr_render_persistent; ws is needed
// when d orders the blocks or queues them.
static lr_status render_views(const char* who, const lr_scene* sc, const lr_view* views, int32_t n_views,
                              float* rgba, uint32_t* nsamples, void* ws, int64_t ws_bytes, Dispatch d, void* stream) {
  SceneK s;
  lr_status st = make_scene(sc, s);
  if (st != LR_OK) return st;
  if (!views || n_views < 1 || !rgba) return fail(LR_EINVAL, "%s: need views, n_views >= 1 and rgba", who);
  for (int i = 0; i < n_views; ++i)
    if ((st = check_view(views[i])) != LR_OK) return st;
  if (d.queues && (s.lookup != LR_LOOKUP_FOREST || s.shading != LR_SHADE_NONE))
    return fail(LR_EINVAL, "%s: the persistent form covers the forest look-up without shading", who);
  if ((d.cost_order || d.queues) && !ws) return fail(LR_EINVAL, "%s: null workspace", who);
  if (ws) {
    const int64_t need = order_workspace(views, n_views);
    if (need < 0) return fail(LR_EINVAL, "%s: image too large for one launch", who);
    if (ws_bytes < need)
      return fail(LR_ECAPACITY, "%s: workspace of %lld bytes, the views need %lld", who, (long long)ws_bytes,
                  (long long)need);
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(LR_EINVAL, "%s: workspace not 256-byte aligned", who);
  }
  hipStream_t hs = static_cast<hipStream_t>(stream);
  for (int base = 0; base < n_views; base += kMaxViews) {
    const int cnt = n_views - base < kMaxViews ? n_views - base : kMaxViews;
    ViewsK vk;
    int64_t nblk = pack_views(views + base, cnt, vk);
    if (d.cost_order) nblk = ordered_workgroups(vk);
    if (nblk <= 0 || nblk > 0x7fffffff) return fail(LR_EINVAL, "%s: image too large for one launch", who);
    if (d.cost_order) schedule(sc, s, vk, ws, hs);
    hipError_t err = hipSuccess;
    if (d.queues) {
      uint32_t* queue = static_cast<uint32_t*>(ws);
      switch (sc->p[0]) {
        case 1: err = dispatch_queue<1>(sc, s, vk, nblk, rgba, nsamples, queue, d.queues, d.workgroups, hs); break;
        case 2: err = dispatch_queue<2>(sc, s, vk, nblk, rgba, nsamples, queue, d.queues, d.workgroups, hs); break;
        default: err = dispatch_queue<3>(sc, s, vk, nblk, rgba, nsamples, queue, d.queues, d.workgroups, hs); break;
      }
    } else {
      switch (sc->p[0]) {
        case 1: dispatch_render<1>(sc, s, vk, nblk, rgba, nsamples, hs); break;
        case 2: dispatch_render<2>(sc, s, vk, nblk, rgba, nsamples, hs); break;
        default: dispatch_render<3>(sc, s, vk, nblk, rgba, nsamples, hs); break;
      }
    }
    if (err == hipSuccess) err = hipGetLastError();
    if (err != hipSuccess) return fail(LR_EHIP, "%s: %s", who, hipGetErrorString(err));
  }
  return LR_OK;
}

LR_API lr_status lr_render(const lr_scene* sc, const lr_view* views, int32_t n_views, float* rgba, uint32_t* nsamples,
                           void* stream) {
  return render_views("lr_render", sc, views, n_views, rgba, nsamples, nullptr, 0, Dispatch{}, stream);
}

// Dispatch-order scratch of lr_render_scheduled_noalloc: one array per GPU,
// held until the process ends, for callers that cannot allocate.  Host code
// uses only the device address hipGetSymbolAddress gives for it (per device,
// on that device's first call); the array's name is no device address on the
// host.  Calls that overlap on one GPU share the array and race.
constexpr int64_t kScheduleScratchBytes = ((int64_t)2 << 20) + (64 << 10);   // 16 views of 2048^2 per launch
static __device__ __align__(256) unsigned char scratch[kScheduleScratchBytes];
static std::mutex g_scratch_mutex;
static void* g_scratch[256];   // per device id

static lr_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(LR_EHIP, "lr_render_scheduled_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= 256) return fail(LR_EINVAL, "lr_render_scheduled_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LR_EHIP, "lr_render_scheduled_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return LR_OK;
}

LR_API lr_status lr_render_scheduled_noalloc(const lr_scene* sc, const lr_view* views, int32_t n_views, float* rgba,
                                             uint32_t* nsamples, void* stream) {
  if (!views || n_views < 1) return fail(LR_EINVAL, "lr_render_scheduled_noalloc: need views and n_views >= 1");
  for (int i = 0; i < n_views; ++i) {
    const lr_status st = check_view(views[i]);
    if (st != LR_OK) return st;
  }
  const int64_t need = order_workspace(views, n_views);
  if (need < 0) return fail(LR_EINVAL, "lr_render_scheduled_noalloc: image too large for one launch");
  if (need > kScheduleScratchBytes)
    return fail(LR_ECAPACITY,
                "lr_render_scheduled_noalloc: a launch of these views needs %lld bytes of dispatch-order scratch; "
                "the library holds %lld (16 views of 2048^2 per launch)",
                (long long)need, (long long)kScheduleScratchBytes);
  void* ws = nullptr;
  const lr_status st = scratch_address(&ws);
  if (st != LR_OK) return st;
  return render_views("lr_render_scheduled_noalloc", sc, views, n_views, rgba, nsamples, ws, kScheduleScratchBytes,
                      Dispatch{true, 0, 0}, stream);
}

LR_API lr_status lr_render_workspace_size(const lr_view* views, int32_t n_views, int64_t* bytes) {
  if (!views || n_views < 1 || !bytes) return fail(LR_EINVAL, "lr_render_workspace_size: need views and bytes");
  for (int i = 0; i < n_views; ++i) {
    const lr_status st = check_view(views[i]);
    if (st != LR_OK) return st;
  }
  const int64_t need = order_workspace(views, n_views);
  if (need < 0) return fail(LR_EINVAL, "lr_render_workspace_size: image too large for one launch");
  *bytes = need;
  return LR_OK;
}

LR_API lr_status lr_render_scheduled(const lr_scene* sc, const lr_view* views, int32_t n_views, float* rgba,
                                     uint32_t* nsamples, void* workspace, int64_t workspace_bytes, void* stream) {
  if (!workspace) return fail(LR_EINVAL, "lr_render_scheduled: null workspace");
  return render_views("lr_render_scheduled", sc, views, n_views, rgba, nsamples, workspace, workspace_bytes,
                      Dispatch{true, 0, 0}, stream);
}

LR_API lr_status lr_render_persistent(const lr_scene* sc, const lr_view* views, int32_t n_views, float* rgba,
                                      uint32_t* nsamples, int32_t queues, int32_t cost_order, int32_t workgroups,
                                      void* workspace, int64_t workspace_bytes, void* stream) {
  if (queues != 1 && queues != 8) return fail(LR_EINVAL, "lr_render_persistent: queues must be 1 or 8, not %d", queues);
  if (cost_order != 0 && cost_order != 1)
    return fail(LR_EINVAL, "lr_render_persistent: cost_order must be 0 or 1, not %d", cost_order);
  if (workgroups < 0 || workgroups > (1 << 20))
    return fail(LR_EINVAL, "lr_render_persistent: workgroups %d outside [0, 2^20]", workgroups);
  return render_views("lr_render_persistent", sc, views, n_views, rgba, nsamples, workspace, workspace_bytes,
                      Dispatch{cost_order == 1, queues, workgroups}, stream);
}

LR_API lr_status lr_trace_rays(const lr_scene* sc, const lr_view* view, const int32_t* pix, int64_t n, int32_t max_out,
                               float* t_out, int32_t* elem_out, float* ds_out, int32_t* count, void* stream) {
  SceneK s;
  lr_status st = make_scene(sc, s);
  if (st != LR_OK) return st;
  if (!view || !pix || n < 1 || max_out < 1 || !t_out || !elem_out || !ds_out || !count)
    return fail(LR_EINVAL, "lr_trace_rays: null pointer or empty request");
  if (n > ((int64_t)1 << 30)) return fail(LR_EINVAL, "lr_trace_rays: too many rays");
  if ((st = check_view(*view)) != LR_OK) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  switch (sc->p[0]) {
    case 1: dispatch_trace<1>(sc, s, *view, pix, n, max_out, t_out, elem_out, ds_out, count, hs); break;
    case 2: dispatch_trace<2>(sc, s, *view, pix, n, max_out, t_out, elem_out, ds_out, count, hs); break;
    default: dispatch_trace<3>(sc, s, *view, pix, n, max_out, t_out, elem_out, ds_out, count, hs); break;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LR_EHIP, "lr_trace_rays: %s", hipGetErrorString(err));
  return LR_OK;
}

LR_API lr_status lr_lookup(const uint32_t* heads, const lr_kdnode* nodes, int64_t n_nodes, const int32_t blocks[3],
                           int64_t n_elem, const float* points, int64_t n, int32_t* elem_out, void* stream) {
  if (!heads || !blocks || !points || !elem_out || n < 0 || n_nodes < 0 || (n_nodes > 0 && !nodes))
    return fail(LR_EINVAL, "lr_lookup: null pointer or negative size");
  if (n_elem <= 0 || n_elem >= (int64_t)LR_LEAF) return fail(LR_EINVAL, "lr_lookup: bad n_elem");
  for (int d = 0; d < 3; ++d)
    if (!lrvr::is_pow2(blocks[d]) || blocks[d] > 512) return fail(LR_ENOTPOW2, "lr_lookup: blocks must be powers of two <= 512");
  if (n == 0) return LR_OK;
  if (n > (int64_t)0x7fffffff * 256) return fail(LR_EINVAL, "lr_lookup: too many points (at most 2^31-1 workgroups of 256)");
  const int64_t nblk = (n + 255) / 256;
  hipLaunchKernelGGL(lookup_kernel, dim3((unsigned)nblk), dim3(256), 0, static_cast<hipStream_t>(stream), heads, nodes,
                     n_nodes, n_elem, blocks[0], blocks[1], blocks[2], points, n, elem_out);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LR_EHIP, "lr_lookup: %s", hipGetErrorString(err));
  return LR_OK;
}

LR_API lr_status lr_render_backward(const lr_scene* sc, const lr_view* views, int32_t n_views, const float* rgba_fwd,
                                    const float* grad_rgba, float* grad_bezier, float* grad_lut, void* stream) {
  SceneK s;
  lr_status st = make_scene(sc, s);
  if (st != LR_OK) return st;
  if (sc->ncomp != 1 || sc->color_mode != LR_COLOR_LUT || sc->bezier_dtype != LR_F32)
    return fail(LR_EINVAL, "lr_render_backward: scalar fields with FP32 blocks only");
  if (sc->shading != LR_SHADE_NONE) return fail(LR_EINVAL, "lr_render_backward: no shading");
  if (!views || n_views < 1 || !rgba_fwd || !grad_rgba || !grad_bezier || !grad_lut)
    return fail(LR_EINVAL, "lr_render_backward: null pointer or no views");
  for (int i = 0; i < n_views; ++i)
    if ((st = check_view(views[i])) != LR_OK) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  for (int base = 0; base < n_views; base += kMaxViews) {
    const int cnt = n_views - base < kMaxViews ? n_views - base : kMaxViews;
    ViewsK vk;
    const int64_t nblk = pack_views(views + base, cnt, vk);
    if (nblk <= 0 || nblk > 0x7fffffff) return fail(LR_EINVAL, "lr_render_backward: image too large");
    const dim3 grid((unsigned)nblk), blk(kThreads);
    const float4* f = reinterpret_cast<const float4*>(rgba_fwd);
    const float4* g = reinterpret_cast<const float4*>(grad_rgba);
    const bool fixed = sc->step_mode == LR_STEP_FIXED, oct = sc->lookup == LR_LOOKUP_OCTREE;
#define LR_BWD(PP)                                                                                              \
  if (oct && fixed) hipLaunchKernelGGL((backward_kernel<PP, LR_STEP_FIXED, LR_LOOKUP_OCTREE>), grid, blk, 0, hs, s, vk, f, g, \
                                       grad_bezier, grad_lut);                                                     \
  else if (oct) hipLaunchKernelGGL((backward_kernel<PP, LR_STEP_ADAPTIVE, LR_LOOKUP_OCTREE>), grid, blk, 0, hs, s, vk, f, g, \
                                   grad_bezier, grad_lut);                                                         \
  else if (fixed) hipLaunchKernelGGL((backward_kernel<PP, LR_STEP_FIXED, LR_LOOKUP_FOREST>), grid, blk, 0, hs, s, vk, f, g, \
                                     grad_bezier, grad_lut);                                                       \
  else hipLaunchKernelGGL((backward_kernel<PP, LR_STEP_ADAPTIVE, LR_LOOKUP_FOREST>), grid, blk, 0, hs, s, vk, f, g,         \
                          grad_bezier, grad_lut);
    switch (sc->p[0]) {
      case 1: LR_BWD(1) break;
      case 2: LR_BWD(2) break;
      default: LR_BWD(3) break;
    }
#undef LR_BWD
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(LR_EHIP, "lr_render_backward: %s", hipGetErrorString(err));
  }
  return LR_OK;
}

LR_API lr_status lr_lookup_octree(const uint32_t* root, const uint32_t* nodes, int64_t n_nodes, int64_t n_elem,
                                  const float* points, int64_t n, int32_t* elem_out, void* stream) {
  if (!root || !points || !elem_out || n < 0 || n_nodes < 0 || (n_nodes > 0 && !nodes))
    return fail(LR_EINVAL, "lr_lookup_octree: null pointer or negative size");
  if (n_elem <= 0 || n_elem >= (int64_t)LR_LEAF || n_nodes >= (int64_t)LR_LEAF)
    return fail(LR_EINVAL, "lr_lookup_octree: bad n_elem / n_nodes");
  if (n == 0) return LR_OK;
  if (n > (int64_t)0x7fffffff * 256) return fail(LR_EINVAL, "lr_lookup_octree: too many points (at most 2^31-1 workgroups of 256)");
  const int64_t nblk = (n + 255) / 256;
  hipLaunchKernelGGL(lookup_octree_kernel, dim3((unsigned)nblk), dim3(256), 0, static_cast<hipStream_t>(stream), root,
                     nodes, n_nodes, n_elem, points, n, elem_out);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LR_EHIP, "lr_lookup_octree: %s", hipGetErrorString(err));
  return LR_OK;
}
