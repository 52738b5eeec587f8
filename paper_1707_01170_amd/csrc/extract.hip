// FP64 change of basis to Bezier blocks on the GPU (Sec. 3.2.3).
//
// One 64-lane wavefront per element.  Each lane takes one B-spline acting on
// the element and computes its three 1-D Bernstein coefficient vectors on the
// element by blossoming: the polynomial piece of a B-spline on a knot span has
// Bernstein coefficients beta_j = blossom(lo^(p-j), hi^j), evaluated with de
// Boor's recurrence (one knot argument per level) on the B-spline's local knot
// vector padded by repeating its end knots.  Lanes then own output
// coefficients and sum gamma_i c_i bx_i[jx] by_i[jy] bz_i[jz] over the
// B-splines in csr order, so the FP64 sum is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "common.h"

namespace {

constexpr int kLanes = 64;
constexpr int64_t kExtractGrid = 8192;   // wavefronts of the forward (grid-stride over elements)

struct ExtractArgs {
  int32_t p[3];
  int32_t ncomp;
  int32_t kstride;
  int32_t nb;         // (p1+1)(p2+1)(p3+1)
  int32_t dtype;
  int32_t pad;
  int64_t stride;     // output row length in elements of dtype
  int64_t n_bspl;
  int64_t n_elem;
  const double* knots;
  const double* coef;
  const double* gamma;
  const double* elem_box;
  const int64_t* csr_ptr;
  const int32_t* csr_idx;
  void* out;
  unsigned long long* range;   // order-preserving keys while the kernels run
  const void* grad;            // backward: dL/dC in the bezier layout of dtype
  double* grad_coef;           // backward: dL/dc [n_bspl][ncomp], accumulated
};

// Order-preserving map of doubles to unsigned 64-bit keys (no NaNs).
__host__ __device__ inline unsigned long long dkey(double x) {
  unsigned long long b;
  memcpy(&b, &x, 8);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double dunkey(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  double x;
  memcpy(&x, &b, 8);
  return x;
}

// Bernstein coefficients beta[0..P] of the B-spline with local knots
// u[0..P+1] on [a, b], which must lie inside one non-empty knot span [u_S,
// u_S+1] (the first such span is taken; false if there is none).  With the
// knot vector padded by repeating its end knots, T[R] = u[clamp(R - P, 0,
// P + 1)], the B-spline is basis function P of T and the span is span S + P
// of T; beta_j = blossom(a^(P-j), b^j) by de Boor's recurrence, one knot
// argument per level.  The knots the recurrence reads, T[S + q] for
// q = 1..2P, are gathered once into a window by selects, so the lanes of a
// wavefront run the same code whatever their span: the B-splines acting on
// one element sit in all P+1 spans along each axis, and code unrolled per
// span ran the P+1 variants one after another (vortex200k 0.72 -> 0.57 ms,
// blobs50k 0.54 -> 0.34, the same values bit for bit).  Each knot difference
// of the recurrence is inverted once and the quotients for both interval ends
// become products (vortex200k 0.51 -> 0.48 ms, blobs50k 0.31 -> 0.27; the
// FP64 blocks move by at most a few units in the last place).
template <int P>
__device__ inline bool bezier_span(const double (&u)[P + 2], double a, double b, double (&beta)[P + 1]) {
  int S = -1;
#pragma unroll
  for (int s = P; s >= 0; --s)
    if (u[s] < u[s + 1] && u[s] <= a && b <= u[s + 1]) S = s;
  if (S < 0) return false;
  double W[2 * P + 1];   // W[q] = T[S + q]
#pragma unroll
  for (int q = 1; q <= 2 * P; ++q) {
    double w = u[0];
#pragma unroll
    for (int i = 1; i <= P + 1; ++i) w = S + q - P >= i ? u[i] : w;
    W[q] = w;
  }
  double inv[P + 1][P + 1];   // inv[l][r] = 1 / (T[S + r + P + 1 - l] - T[S + r])
#pragma unroll
  for (int l = 1; l <= P; ++l)
#pragma unroll
    for (int r = l; r <= P; ++r) inv[l][r] = 1.0 / (W[r + P + 1 - l] - W[r]);
#pragma unroll
  for (int j = 0; j <= P; ++j) {
    double d[P + 1];
#pragma unroll
    for (int r = 0; r <= P; ++r) d[r] = r == P - S ? 1.0 : 0.0;
#pragma unroll
    for (int l = 1; l <= P; ++l) {
      const double x = (l <= P - j) ? a : b;
#pragma unroll
      for (int r = P; r >= l; --r) {
        const double al = (x - W[r]) * inv[l][r];
        d[r] = (1.0 - al) * d[r - 1] + al * d[r];
      }
    }
    beta[j] = d[P];
  }
  return true;
}

// The B-spline's Bernstein vector on [a, b] written to out[0..3] (zeros
// beyond P and on failure).  Each degree writes its own vector to the
// caller's (LDS) row: returning it through one local array for all degrees
// made the compiler index that array at run time, in scratch memory.
template <int P>
__device__ inline bool bezier_1d_p(const double* ug, double a, double b, double* out) {
  double u[P + 2];
#pragma unroll
  for (int i = 0; i < P + 2; ++i) u[i] = ug[i];
  double beta[P + 1];
  const bool ok = bezier_span<P>(u, a, b, beta);
#pragma unroll
  for (int j = 0; j < 4; ++j) out[j] = (ok && j <= P) ? beta[j] : 0.0;
  return ok;
}

// Bernstein coefficients of the B-spline with local knots u[0..p+1] (global
// memory) on [a, b], into out[0..3]; false if [a, b] is not inside one
// non-empty knot span.
__device__ inline bool bezier_1d(const double* u, int p, double a, double b, double* out) {
  switch (p) {
    case 1: return bezier_1d_p<1>(u, a, b, out);
    case 2: return bezier_1d_p<2>(u, a, b, out);
    case 3: return bezier_1d_p<3>(u, a, b, out);
    default:
      for (int j = 0; j < 4; ++j) out[j] = 0.0;
      return false;
  }
}

// FP64 -> FP16 with a single round-to-nearest-even: round to odd in FP32
// first (keeps enough bits that the second rounding is exact), then RNE.
__device__ inline unsigned short f64_to_f16_bits(double x) {
  float f = (float)x;
  const double back = (double)f;
  if (back != x) {
    unsigned int u = __float_as_uint(f);
    if (fabs(back) > fabs(x)) u -= 1u;   // truncate toward zero
    u |= 1u;                             // sticky bit
    f = __uint_as_float(u);
  }
  _Float16 h = (_Float16)f;
  unsigned short bits;
  memcpy(&bits, &h, 2);
  return bits;
}

__global__ void range_init(unsigned long long* r) {
  r[0] = dkey(INFINITY);
  r[1] = dkey(-INFINITY);
}

__global__ void range_final(unsigned long long* r) {
  double* d = reinterpret_cast<double*>(r);
  const double lo = dunkey(r[0]), hi = dunkey(r[1]);
  d[0] = lo;
  d[1] = hi;
}

// One wavefront per element, looping over elements with the grid's stride.
// The value range is folded into registers over all of a wavefront's
// elements and merged into the global pair once per wavefront, and only if it
// extends the pair as last seen: one global atomic per element on the same
// two words serialised the whole launch.
//
// Compiled for four waves per SIMD (127 registers; left alone the compiler
// takes 129 and three waves fit): vortex200k 0.63 -> 0.51 ms, blobs50k 0.34
// -> 0.31.
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(4))) void extract_kernel(ExtractArgs a) {
  __shared__ double sb[kLanes][3][4];
  __shared__ double sw[kLanes][4];
  __shared__ double so[256];
  const int lane = threadIdx.x;
  const int NC = a.nb * a.ncomp;
  const int px = a.p[0] + 1, py = a.p[1] + 1;
  double lo = INFINITY, hi = a.ncomp == 1 ? -INFINITY : 0.0;
  for (int64_t e = blockIdx.x; e < a.n_elem; e += gridDim.x) {
    const int64_t b0 = a.csr_ptr[e], b1 = a.csr_ptr[e + 1];
    const double* eb = a.elem_box + 6 * e;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t base = b0; base < b1; base += kLanes) {
      const int64_t q = base + lane;
      if (q < b1) {
        const int32_t bi = a.csr_idx[q];
        bool ok = bi >= 0 && bi < a.n_bspl;
        for (int d = 0; d < 3; ++d) {
          if (ok) ok = bezier_1d(a.knots + ((int64_t)bi * 3 + d) * a.kstride, a.p[d], eb[d], eb[3 + d], sb[lane][d]);
          else for (int j = 0; j < 4; ++j) sb[lane][d][j] = 0.0;
        }
        for (int c = 0; c < 4; ++c)
          sw[lane][c] = (ok && c < a.ncomp) ? a.gamma[bi] * a.coef[(int64_t)bi * a.ncomp + c] : 0.0;
      }
      __syncthreads();
      const int cnt = (int)((b1 - base) < kLanes ? (b1 - base) : kLanes);
      for (int o = 0; o < 4; ++o) {
        const int jj = lane + kLanes * o;
        if (jj >= NC) break;
        const int c = jj / a.nb, j = jj % a.nb;
        const int jx = j % px, jy = (j / px) % py, jz = j / (px * py);
        double s = acc[o];
        for (int m = 0; m < cnt; ++m) s += sw[m][c] * sb[m][0][jx] * sb[m][1][jy] * sb[m][2][jz];
        acc[o] = s;
      }
      __syncthreads();
    }
    for (int o = 0; o < 4; ++o) {
      const int jj = lane + kLanes * o;
      if (jj < NC) so[jj] = acc[o];
    }
    __syncthreads();
    for (int64_t jj = lane; jj < a.stride; jj += kLanes) {
      const double v = jj < NC ? so[jj] : 0.0;
      const int64_t off = e * a.stride + jj;
      if (a.dtype == LR_F64)
        static_cast<double*>(a.out)[off] = v;
      else if (a.dtype == LR_F32)
        static_cast<float*>(a.out)[off] = (float)v;
      else
        static_cast<unsigned short*>(a.out)[off] = f64_to_f16_bits(v);
    }
    if (a.range) {
      if (a.ncomp == 1) {
        for (int jj = lane; jj < NC; jj += kLanes) {
          lo = fmin(lo, so[jj]);
          hi = fmax(hi, so[jj]);
        }
      } else {
        lo = 0.0;
        for (int j = lane; j < a.nb; j += kLanes) {
          double n2 = 0.0;
          for (int c = 0; c < a.ncomp; ++c) n2 += so[c * a.nb + j] * so[c * a.nb + j];
          hi = fmax(hi, sqrt(n2));
        }
      }
    }
    __syncthreads();   // so is rewritten by the next element
  }
  if (a.range) {
    for (int off = kLanes / 2; off > 0; off >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, off));
      hi = fmax(hi, __shfl_xor(hi, off));
    }
    if (lane == 0) {
      const unsigned long long klo = dkey(lo), khi = dkey(hi);
      if (klo < __hip_atomic_load(&a.range[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(&a.range[0], klo);
      if (khi > __hip_atomic_load(&a.range[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&a.range[1], khi);
    }
  }
}

// Adjoint of extract_kernel with respect to c: the same wavefront-per-element
// split and the same 1-D Bernstein vectors; each lane contracts the element's
// gradient block with its B-spline's tensor Bernstein coefficients and adds
// gamma_i times the result to dL/dc_i.  Elements whose gradient block is zero
// (no ray reached them) add nothing.  Each lane's Bernstein vectors live in an
// LDS row: the contraction reads them at run-time indices, which a register
// array would serve from scratch memory (vortex200k 1.27 -> 0.82 ms, blobs50k
// 0.63 -> 0.37).
__global__ __launch_bounds__(kLanes) void extract_backward_kernel(ExtractArgs a) {
  __shared__ double sg[256];
  __shared__ double sbeta[kLanes][3][4];   // each lane's Bernstein vectors (read at run-time indices)
  const int64_t e = blockIdx.x;
  const int lane = threadIdx.x;
  const int NC = a.nb * a.ncomp;
  bool any = false;
  for (int jj = lane; jj < NC; jj += kLanes) {
    const int64_t off = e * a.stride + jj;
    const double g = a.dtype == LR_F64 ? static_cast<const double*>(a.grad)[off]
                                       : (double)static_cast<const float*>(a.grad)[off];
    sg[jj] = g;
    any |= g != 0.0;
  }
  if (!__syncthreads_or(any)) return;
  const int64_t b0 = a.csr_ptr[e], b1 = a.csr_ptr[e + 1];
  const double* eb = a.elem_box + 6 * e;
  const int px = a.p[0] + 1, py = a.p[1] + 1, pz = a.p[2] + 1;
  for (int64_t q = b0 + lane; q < b1; q += kLanes) {
    const int32_t bi = a.csr_idx[q];
    if (bi < 0 || bi >= a.n_bspl) continue;
    double (&beta)[3][4] = sbeta[lane];
    bool ok = true;
    for (int d = 0; d < 3 && ok; ++d)
      ok = bezier_1d(a.knots + ((int64_t)bi * 3 + d) * a.kstride, a.p[d], eb[d], eb[3 + d], beta[d]);
    if (!ok) continue;
    const double gw = a.gamma[bi];
    for (int c = 0; c < a.ncomp; ++c) {
      const double* g = sg + c * a.nb;
      double s = 0.0;
      for (int jz = 0; jz < pz; ++jz) {
        double sy = 0.0;
        for (int jy = 0; jy < py; ++jy) {
          double sx = 0.0;
          for (int jx = 0; jx < px; ++jx) sx += g[jx + px * (jy + py * jz)] * beta[0][jx];
          sy += sx * beta[1][jy];
        }
        s += sy * beta[2][jz];
      }
      atomicAdd(a.grad_coef + (int64_t)bi * a.ncomp + c, gw * s);
    }
  }
}

// Checks shared by the forward and the adjoint; fills the kernel arguments.
lr_status prepare(const char* who, const lr_lrspline* spl, bool need_coef, int32_t dtype, ExtractArgs* a) {
  using lrvr::fail;
  if (!spl->knots || (need_coef && !spl->coef) || !spl->gamma || !spl->elem_box || !spl->csr_ptr ||
      !spl->csr_idx)
    return fail(LR_EINVAL, "%s: null array in the spline", who);
  if (spl->n_elem <= 0 || spl->n_bspl <= 0 || spl->n_elem >= (int64_t)1 << 31)
    return fail(LR_EINVAL, "%s: n_elem / n_bspl out of range", who);
  if (spl->ncomp < 1 || spl->ncomp > 4) return fail(LR_EINVAL, "%s: ncomp must be 1..4", who);
  int pmax = 0;
  int nb = 1;
  for (int d = 0; d < 3; ++d) {
    if (spl->p[d] < 1 || spl->p[d] > 3) return fail(LR_EINVAL, "%s: degree out of [1,3]", who);
    pmax = spl->p[d] > pmax ? spl->p[d] : pmax;
    nb *= spl->p[d] + 1;
  }
  if (spl->kstride < pmax + 2) return fail(LR_EINVAL, "%s: kstride < max(p)+2", who);
  if (nb * spl->ncomp > 256) return fail(LR_EINVAL, "%s: more than 256 coefficients per element", who);
  std::memset(a, 0, sizeof *a);
  for (int d = 0; d < 3; ++d) a->p[d] = spl->p[d];
  a->ncomp = spl->ncomp;
  a->kstride = spl->kstride;
  a->nb = nb;
  a->dtype = dtype;
  a->stride = lr_bezier_stride(spl->p, spl->ncomp, dtype);
  a->n_bspl = spl->n_bspl;
  a->n_elem = spl->n_elem;
  a->knots = spl->knots;
  a->coef = spl->coef;
  a->gamma = spl->gamma;
  a->elem_box = spl->elem_box;
  a->csr_ptr = spl->csr_ptr;
  a->csr_idx = spl->csr_idx;
  return LR_OK;
}

}  // namespace

using lrvr::fail;

LR_API lr_status lr_extract_bezier(const lr_lrspline* spl, int32_t out_dtype, void* bezier, double* range,
                                   void* stream) {
  if (!spl || !bezier) return fail(LR_EINVAL, "lr_extract_bezier: null pointer");
  if (out_dtype != LR_F32 && out_dtype != LR_F16 && out_dtype != LR_F64)
    return fail(LR_EINVAL, "lr_extract_bezier: out_dtype must be LR_F32, LR_F16 or LR_F64");
  ExtractArgs a;
  const lr_status st0 = prepare("lr_extract_bezier", spl, true, out_dtype, &a);
  if (st0 != LR_OK) return st0;
  a.out = bezier;
  a.range = reinterpret_cast<unsigned long long*>(range);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (range) hipLaunchKernelGGL(range_init, dim3(1), dim3(1), 0, st, a.range);
  const int64_t grid = spl->n_elem < kExtractGrid ? spl->n_elem : kExtractGrid;
  hipLaunchKernelGGL(extract_kernel, dim3((unsigned)grid), dim3(kLanes), 0, st, a);
  if (range) hipLaunchKernelGGL(range_final, dim3(1), dim3(1), 0, st, a.range);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LR_EHIP, "lr_extract_bezier: %s", hipGetErrorString(err));
  return LR_OK;
}

LR_API lr_status lr_extract_bezier_backward(const lr_lrspline* spl, int32_t grad_dtype, const void* grad_bezier,
                                            double* grad_coef, void* stream) {
  if (!spl || !grad_bezier || !grad_coef) return fail(LR_EINVAL, "lr_extract_bezier_backward: null pointer");
  if (grad_dtype != LR_F32 && grad_dtype != LR_F64)
    return fail(LR_EINVAL, "lr_extract_bezier_backward: grad_dtype must be LR_F32 or LR_F64");
  ExtractArgs a;
  const lr_status st0 = prepare("lr_extract_bezier_backward", spl, false, grad_dtype, &a);
  if (st0 != LR_OK) return st0;
  a.grad = grad_bezier;
  a.grad_coef = grad_coef;
  hipLaunchKernelGGL(extract_backward_kernel, dim3((unsigned)spl->n_elem), dim3(kLanes), 0,
                     static_cast<hipStream_t>(stream), a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LR_EHIP, "lr_extract_bezier_backward: %s", hipGetErrorString(err));
  return LR_OK;
}
