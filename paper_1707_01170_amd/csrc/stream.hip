// Streamlines of an LR-spline vector field on gfx950 (Sec. 5): explicit
// Runge-Kutta integration of dx/dt = f(x) (Eq. 5, Eq. 6) with the Eq. 4
// sampling distance as the local step (Sec. 5.2), a constant step, or
// embedded error control; the compute stage of Sec. 5.3 that fills a
// seeds x samples buffer of (x, y, z, active).
//
// Three lanes integrate one seed (21 seeds per wavefront): all three carry the
// same position, stages and step, and lane q evaluates only component q of the
// field, from that component's part of the Bezier block, with the same
// arithmetic as a whole-block contraction; the three values are exchanged by
// lane shuffles.  This shortens each stage's dependent chain (the contraction
// is most of it) and each lane loads a third of the block.  A group keeps its
// current element like the ray caster and descends the look-up structure only
// when a stage position leaves it.  Mixed precision (Sec. 5.6):
// the position, time, step and stage sums are FP64 and only the field is
// evaluated in FP32 from the FP32 Bezier block; single precision does the
// outer loop in FP32 too.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "common.h"
#include "eval.h"

namespace {

using namespace lrvr;

struct StreamK {
  const float* box;
  const float* bez;
  const uint32_t* heads;
  const void* nodes;
  int64_t n_elem, n_nodes, stride;
  int32_t bx, by, bz, lookup;
  float fbx, fby, fbz;
  int32_t step_mode, max_samples;
  double base, t_end, tol;
  const double* seeds;
  int64_t n;
  float4* out;
  double* t_out;
  int32_t* count;
};

// Butcher tableaus (published coefficients); entries are read with constant
// indices after unrolling.
template <int M>
struct Tab;

template <>
struct Tab<LR_RK1> {
  static constexpr int S = 1, Q = 1;
  static constexpr bool EMB = false;
  static constexpr double A[1][1] = {{0}};
  static constexpr double B[1] = {1};
  static constexpr double BL[1] = {0};
};
template <>
struct Tab<LR_RK2> {
  static constexpr int S = 2, Q = 2;
  static constexpr bool EMB = false;
  static constexpr double A[2][2] = {{0, 0}, {0.5, 0}};
  static constexpr double B[2] = {0, 1};
  static constexpr double BL[2] = {0, 0};
};
template <>
struct Tab<LR_RK3> {
  static constexpr int S = 3, Q = 3;
  static constexpr bool EMB = false;
  static constexpr double A[3][3] = {{0, 0, 0}, {0.5, 0, 0}, {-1, 2, 0}};
  static constexpr double B[3] = {1.0 / 6, 2.0 / 3, 1.0 / 6};
  static constexpr double BL[3] = {0, 0, 0};
};
template <>
struct Tab<LR_RK4> {
  static constexpr int S = 4, Q = 4;
  static constexpr bool EMB = false;
  static constexpr double A[4][4] = {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {0, 0.5, 0, 0}, {0, 0, 1, 0}};
  static constexpr double B[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
  static constexpr double BL[4] = {0, 0, 0, 0};
};
template <>
struct Tab<LR_RK4_38> {
  static constexpr int S = 4, Q = 4;
  static constexpr bool EMB = false;
  static constexpr double A[4][4] = {{0, 0, 0, 0}, {1.0 / 3, 0, 0, 0}, {-1.0 / 3, 1, 0, 0}, {1, -1, 1, 0}};
  static constexpr double B[4] = {1.0 / 8, 3.0 / 8, 3.0 / 8, 1.0 / 8};
  static constexpr double BL[4] = {0, 0, 0, 0};
};
// Fehlberg's 4(5) pair: RKF5 steps with the fifth-order weights; RKF45 also
// estimates the error with the fourth-order ones.
struct Fehlberg {
  static constexpr int S = 6, Q = 5;
  static constexpr double A[6][6] = {
      {0, 0, 0, 0, 0, 0},
      {1.0 / 4, 0, 0, 0, 0, 0},
      {3.0 / 32, 9.0 / 32, 0, 0, 0, 0},
      {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0, 0},
      {439.0 / 216, -8, 3680.0 / 513, -845.0 / 4104, 0, 0},
      {-8.0 / 27, 2, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40, 0}};
  static constexpr double B[6] = {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55};
  static constexpr double BL[6] = {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0};
};
template <>
struct Tab<LR_RKF5> : Fehlberg {
  static constexpr bool EMB = false;
};
template <>
struct Tab<LR_RKF45> : Fehlberg {
  static constexpr bool EMB = true;
};
template <>
struct Tab<LR_HE> {
  static constexpr int S = 2, Q = 2;
  static constexpr bool EMB = true;
  static constexpr double A[2][2] = {{0, 0}, {1, 0}};
  static constexpr double B[2] = {0.5, 0.5};
  static constexpr double BL[2] = {1, 0};
};
template <>
struct Tab<LR_BS> {
  static constexpr int S = 4, Q = 3;
  static constexpr bool EMB = true;
  static constexpr double A[4][4] = {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {0, 0.75, 0, 0}, {2.0 / 9, 1.0 / 3, 4.0 / 9, 0}};
  static constexpr double B[4] = {2.0 / 9, 1.0 / 3, 4.0 / 9, 0};
  static constexpr double BL[4] = {7.0 / 24, 1.0 / 4, 1.0 / 3, 1.0 / 8};
};

constexpr int kLanesPerSeed = 3;
constexpr int kSeedsPerWave = 64 / kLanesPerSeed;   // lane 63 idles

// Component q of the field at stage positions, with the group's current
// element cached; f receives all three components.
template <int P>
struct Field {
  static constexpr int NB = (P + 1) * (P + 1) * (P + 1);
  static constexpr int NW = (NB + 3) / 4 * 4 + 4;   // 16-byte aligned window holding one component
  float lo[3] = {2.0f, 2.0f, 2.0f}, hi[3] = {-1.0f, -1.0f, -1.0f}, inv[3] = {0.0f, 0.0f, 0.0f};
  float ds = 0.0f;    // Eq. 4 distance of the cached element
  float c[NB];        // component q of the cached element's block
  int q = 0;          // component of this lane
  int lane0 = 0;      // first lane of the group
  bool bad = false;   // a look-up met a corrupt reference

  __device__ inline void load_component(const StreamK& k, int32_t e) {
    // Component q starts at float q * NB of the row, not always 16-byte
    // aligned: load the aligned window around it (inside the row, whose
    // length is a multiple of 4 floats) and select with constant indices.
    const float* row = k.bez + (int64_t)e * k.stride;
    const int start = q * NB, a0 = start & ~3, off = start - a0;
    const float4* r4 = reinterpret_cast<const float4*>(row + a0);
    float w[NW];
#pragma unroll
    for (int i = 0; i < NW / 4; ++i) {
      if (a0 + 4 * i < k.stride) {
        const float4 v = r4[i];
        w[4 * i] = v.x;
        w[4 * i + 1] = v.y;
        w[4 * i + 2] = v.z;
        w[4 * i + 3] = v.w;
      } else {
        w[4 * i] = w[4 * i + 1] = w[4 * i + 2] = w[4 * i + 3] = 0.0f;
      }
    }
#pragma unroll
    for (int o = 0; o < 4; ++o)
      if (off == o) {
#pragma unroll
        for (int j = 0; j < NB; ++j) c[j] = w[j + o];
      }
  }

  template <typename R>
  __device__ inline void at(const StreamK& k, const R y[3], R f[3]) {
    float p[3];
    for (int a = 0; a < 3; ++a) p[a] = fminf(fmaxf((float)y[a], 0.0f), 1.0f);
    if (!inside(p, lo, hi)) {
      const int32_t e = k.lookup == LR_LOOKUP_OCTREE
                            ? octree_lookup(k.heads, static_cast<const uint32_t*>(k.nodes), k.n_nodes, k.n_elem, p)
                            : forest_lookup(k.heads, static_cast<const lr_kdnode*>(k.nodes), k.n_nodes, k.n_elem,
                                            k.bx, k.by, k.bz, k.fbx, k.fby, k.fbz, p);
      if (e < 0) {           // corrupt look-up structure: the value is NaN and the line ends
        bad = true;
        for (int a = 0; a < 3; ++a) f[a] = (R)NAN;
        return;
      }
      const float* b = k.box + 6 * (int64_t)e;
      for (int a = 0; a < 3; ++a) {
        lo[a] = b[a];
        hi[a] = b[3 + a];
        inv[a] = __builtin_amdgcn_rcpf(hi[a] - lo[a]);
      }
      ds = fminf(fminf(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]) * (1.0f / (float)(1 << P));
      load_component(k, e);
    }
    float bx[P + 1], by[P + 1], bz[P + 1];
    bernstein<P>(fminf(fmaxf((p[0] - lo[0]) * inv[0], 0.0f), 1.0f), bx);
    bernstein<P>(fminf(fmaxf((p[1] - lo[1]) * inv[1], 0.0f), 1.0f), by);
    bernstein<P>(fminf(fmaxf((p[2] - lo[2]) * inv[2], 0.0f), 1.0f), bz);
    const float fq = contract<P, Coef<NB, float>>(c, 0, bx, by, bz);
    // The three lanes of a group follow the same control flow (same state),
    // so the lanes read here are active.
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = (R)__shfl(fq, lane0 + a);
  }
};

template <typename R>
__device__ inline R rpow(R x, R y);
template <>
__device__ inline double rpow<double>(double x, double y) { return pow(x, y); }
template <>
__device__ inline float rpow<float>(float x, float y) { return powf(x, y); }

template <int P, int M, typename R>
__global__ __launch_bounds__(64) void stream_kernel(const StreamK k) {
  using T = Tab<M>;
  constexpr int S = T::S;
  const int grp = threadIdx.x / kLanesPerSeed;
  if (grp >= kSeedsPerWave) return;
  const int64_t j = (int64_t)blockIdx.x * kSeedsPerWave + grp;
  if (j >= k.n) return;
  const bool writer = threadIdx.x == kLanesPerSeed * grp;   // lane 0 of the group stores the line
  float4* out = k.out + j * k.max_samples;
  double* tout = k.t_out ? k.t_out + j * k.max_samples : nullptr;
  R x[3];
  for (int a = 0; a < 3; ++a) x[a] = (R)k.seeds[3 * j + a];
  R t = 0;
  const R t_end = (R)k.t_end, base = (R)k.base, tol = (R)k.tol;
  if (writer) out[0] = make_float4((float)x[0], (float)x[1], (float)x[2], 1.0f);
  if (writer && tout) tout[0] = 0.0;
  int32_t n = 1;
  Field<P> fld;
  fld.lane0 = kLanesPerSeed * grp;
  fld.q = threadIdx.x - fld.lane0;
  R h_next = 0;
  bool first = true;
  while (n < k.max_samples && t < t_end) {
    R kk[S][3];
    fld.template at<R>(k, x, kk[0]);                       // k_1 = f(x_n); caches the element of x_n
    if (first && k.step_mode == LR_STREAM_EMBEDDED) h_next = base * (R)fld.ds;
    first = false;
    const R rem = t_end - t;
    R h;
    if (k.step_mode == LR_STREAM_HEURISTIC) h = base * (R)fld.ds;
    else if (k.step_mode == LR_STREAM_CONSTANT) h = base;
    else h = h_next;
    h = h < rem ? h : rem;
    R xn[3];
    for (int rej = 0;; ++rej) {
#pragma unroll
      for (int i = 1; i < S; ++i) {
        R y[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          R acc = 0;
#pragma unroll
          for (int m = 0; m < i; ++m)
            if (T::A[i][m] != 0.0) acc += (R)T::A[i][m] * kk[m][a];
          y[a] = x[a] + h * acc;
        }
        fld.template at<R>(k, y, kk[i]);
      }
      if (fld.bad) break;
      R err2 = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        R hi = 0, lo = 0;
#pragma unroll
        for (int i = 0; i < S; ++i) {
          if (T::B[i] != 0.0) hi += (R)T::B[i] * kk[i][a];
          if (T::EMB && T::BL[i] != 0.0) lo += (R)T::BL[i] * kk[i][a];
        }
        xn[a] = x[a] + h * hi;
        if (T::EMB) {
          const R d = (x[a] + h * lo) - xn[a];
          err2 += d * d;
        }
      }
      if (!T::EMB || k.step_mode != LR_STREAM_EMBEDDED) break;
      const R err = sqrt(err2);
      const R fac = err > 0 ? (R)0.9 * rpow<R>(tol / err, (R)1 / (R)T::Q) : (R)5;
      if (err <= tol || h <= (R)1e-14 || rej >= 64) {
        h_next = h * (fac < (R)5 ? (fac > (R)0.2 ? fac : (R)0.2) : (R)5);
        break;
      }
      h = h * (fac > (R)0.2 ? fac : (R)0.2);
      h = h > (R)1e-14 ? h : (R)1e-14;
    }
    if (fld.bad) break;
    bool in = true;
    for (int a = 0; a < 3; ++a) in = in && xn[a] >= 0 && xn[a] <= 1;
    if (!in) break;
    for (int a = 0; a < 3; ++a) x[a] = xn[a];
    t += h;
    if (writer) out[n] = make_float4((float)x[0], (float)x[1], (float)x[2], 1.0f);
    if (writer && tout) tout[n] = (double)t;
    ++n;
  }
  if (!writer) return;
  if (k.count) k.count[j] = n;
  for (int32_t i = n; i < k.max_samples; ++i) {
    // after a line ended at a corrupt look-up structure, its next entry is NaN
    const float z = (fld.bad && i == n) ? NAN : 0.0f;
    out[i] = make_float4(z, z, z, 0.0f);
    if (tout) tout[i] = 0.0;
  }
}

template <int P, typename R>
void launch_method(int32_t method, const StreamK& k, hipStream_t st) {
  const dim3 grid((unsigned)((k.n + kSeedsPerWave - 1) / kSeedsPerWave)), blk(64);
  switch (method) {
    case LR_RK1: hipLaunchKernelGGL((stream_kernel<P, LR_RK1, R>), grid, blk, 0, st, k); break;
    case LR_RK2: hipLaunchKernelGGL((stream_kernel<P, LR_RK2, R>), grid, blk, 0, st, k); break;
    case LR_RK3: hipLaunchKernelGGL((stream_kernel<P, LR_RK3, R>), grid, blk, 0, st, k); break;
    case LR_RK4: hipLaunchKernelGGL((stream_kernel<P, LR_RK4, R>), grid, blk, 0, st, k); break;
    case LR_RK4_38: hipLaunchKernelGGL((stream_kernel<P, LR_RK4_38, R>), grid, blk, 0, st, k); break;
    case LR_RKF5: hipLaunchKernelGGL((stream_kernel<P, LR_RKF5, R>), grid, blk, 0, st, k); break;
    case LR_HE: hipLaunchKernelGGL((stream_kernel<P, LR_HE, R>), grid, blk, 0, st, k); break;
    case LR_BS: hipLaunchKernelGGL((stream_kernel<P, LR_BS, R>), grid, blk, 0, st, k); break;
    default: hipLaunchKernelGGL((stream_kernel<P, LR_RKF45, R>), grid, blk, 0, st, k); break;
  }
}

template <int P>
void launch_precision(const lr_stream_params* prm, const StreamK& k, hipStream_t st) {
  if (prm->precision == LR_PREC_SINGLE) launch_method<P, float>(prm->method, k, st);
  else launch_method<P, double>(prm->method, k, st);
}

}  // namespace

using lrvr::fail;

LR_API lr_status lr_streamlines(const lr_scene* sc, const lr_stream_params* prm, const double* seeds, int64_t n,
                                float* points, double* times, int32_t* count, void* stream) {
  if (!sc || !prm || !seeds || !points) return fail(LR_EINVAL, "lr_streamlines: null pointer");
  if (n < 0 || n > ((int64_t)1 << 30)) return fail(LR_EINVAL, "lr_streamlines: seed count out of range");
  const int P = sc->p[0];
  if (sc->p[1] != P || sc->p[2] != P || P < 1 || P > 3)
    return fail(LR_EINVAL, "lr_streamlines: equal degrees p1 = p2 = p3 in [1,3]");
  if (sc->ncomp != 3) return fail(LR_EINVAL, "lr_streamlines: a 3-component field is needed");
  if (sc->bezier_dtype != LR_F32) return fail(LR_EINVAL, "lr_streamlines: FP32 Bezier blocks");
  if (!sc->elem_box || !sc->bezier || !sc->heads || (!sc->nodes && sc->n_nodes > 0))
    return fail(LR_EINVAL, "lr_streamlines: null device array in the scene");
  if (sc->n_elem <= 0 || sc->n_elem >= (int64_t)LR_LEAF || sc->n_nodes < 0 || sc->n_nodes >= (int64_t)LR_LEAF)
    return fail(LR_EINVAL, "lr_streamlines: bad n_elem / n_nodes");
  if (sc->lookup != LR_LOOKUP_FOREST && sc->lookup != LR_LOOKUP_OCTREE)
    return fail(LR_EINVAL, "lr_streamlines: bad lookup");
  if (sc->lookup == LR_LOOKUP_FOREST)
    for (int d = 0; d < 3; ++d)
      if (!lrvr::is_pow2(sc->blocks[d]) || sc->blocks[d] > 512)
        return fail(LR_ENOTPOW2, "lr_streamlines: blocks must be powers of two <= 512");
  if (prm->method < LR_RK1 || prm->method > LR_RKF45) return fail(LR_EINVAL, "lr_streamlines: unknown method");
  if (prm->step_mode != LR_STREAM_HEURISTIC && prm->step_mode != LR_STREAM_CONSTANT &&
      prm->step_mode != LR_STREAM_EMBEDDED)
    return fail(LR_EINVAL, "lr_streamlines: unknown step mode");
  if (prm->step_mode == LR_STREAM_EMBEDDED && prm->method != LR_HE && prm->method != LR_BS && prm->method != LR_RKF45)
    return fail(LR_EINVAL, "lr_streamlines: embedded steps need LR_HE, LR_BS or LR_RKF45");
  if (prm->precision != LR_PREC_MIXED && prm->precision != LR_PREC_SINGLE)
    return fail(LR_EINVAL, "lr_streamlines: precision must be LR_PREC_MIXED or LR_PREC_SINGLE");
  if (prm->max_samples < 1) return fail(LR_EINVAL, "lr_streamlines: max_samples < 1");
  if (!(prm->base > 0.0) || !(prm->t_end > 0.0) || !std::isfinite(prm->base) || !std::isfinite(prm->t_end) ||
      (prm->step_mode == LR_STREAM_EMBEDDED && !(prm->tol > 0.0)))
    return fail(LR_EINVAL, "lr_streamlines: need base > 0, t_end > 0 (and tol > 0 for embedded steps)");
  if (n == 0) return LR_OK;
  StreamK k;
  std::memset(&k, 0, sizeof k);
  k.box = sc->elem_box;
  k.bez = static_cast<const float*>(sc->bezier);
  k.heads = sc->heads;
  k.nodes = sc->nodes;
  k.n_elem = sc->n_elem;
  k.n_nodes = sc->n_nodes;
  k.stride = lr_bezier_stride(sc->p, 3, LR_F32);
  k.lookup = sc->lookup;
  const bool oct = sc->lookup == LR_LOOKUP_OCTREE;
  k.bx = oct ? 1 : sc->blocks[0];
  k.by = oct ? 1 : sc->blocks[1];
  k.bz = oct ? 1 : sc->blocks[2];
  k.fbx = (float)k.bx;
  k.fby = (float)k.by;
  k.fbz = (float)k.bz;
  k.step_mode = prm->step_mode;
  k.max_samples = prm->max_samples;
  k.base = prm->base;
  k.t_end = prm->t_end;
  k.tol = prm->tol;
  k.seeds = seeds;
  k.n = n;
  k.out = reinterpret_cast<float4*>(points);
  k.t_out = times;
  k.count = count;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (P) {
    case 1: launch_precision<1>(prm, k, st); break;
    case 2: launch_precision<2>(prm, k, st); break;
    default: launch_precision<3>(prm, k, st); break;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LR_EHIP, "lr_streamlines: %s", hipGetErrorString(err));
  return LR_OK;
}
