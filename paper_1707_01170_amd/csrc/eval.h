// Device-side evaluation shared by the ray caster and the streamline
// integrator: loading of an element's Bezier block and its tensor Bernstein
// evaluation with optional gradient (Sec. 3.2.3).  The look-up descents
// (Alg. 1 and the octree) are in lookup.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>

#include "common.h"
#include "lookup.h"

namespace lrvr {

__device__ inline bool inside(const float p[3], const float lo[3], const float hi[3]) {
  bool in = true;
  for (int a = 0; a < 3; ++a) in = in && lo[a] <= p[a] && (p[a] < hi[a] || (p[a] == 1.0f && hi[a] == 1.0f));
  return in;
}

// ---------------------------------------------------------------- Bezier blocks
// A lane's copy of one element's block: Reg is the register type, get(c, j)
// the coefficient j as an FP32 value.  FP16 blocks stay packed two to a
// register and are widened inside the multiply-add (the conversion is exact).
template <int NCF, typename CT>
struct Coef;

template <int NCF>
struct Coef<NCF, float> {
  using Reg = float;
  static constexpr int N4 = (NCF + 3) / 4;
  static constexpr int kRegs = 4 * N4;
  __device__ static inline void load(const void* bez, int64_t stride, int32_t e, float* c) {
    const float4* r4 = reinterpret_cast<const float4*>(static_cast<const float*>(bez) + (int64_t)e * stride);
#pragma unroll
    for (int i = 0; i < N4; ++i) {
      const float4 v = r4[i];
      c[4 * i + 0] = v.x;
      c[4 * i + 1] = v.y;
      c[4 * i + 2] = v.z;
      c[4 * i + 3] = v.w;
    }
  }
  __device__ static inline float get(const float* c, int j) { return c[j]; }
};

template <int NCF>
struct Coef<NCF, _Float16> {
  using Reg = uint32_t;
  static constexpr int N8 = (NCF + 7) / 8;
  static constexpr int kRegs = 4 * N8;     // two coefficients per register
  __device__ static inline void load(const void* bez, int64_t stride, int32_t e, uint32_t* c) {
    const uint4* r8 = reinterpret_cast<const uint4*>(static_cast<const _Float16*>(bez) + (int64_t)e * stride);
#pragma unroll
    for (int i = 0; i < N8; ++i) {
      const uint4 v = r8[i];
      c[4 * i + 0] = v.x;
      c[4 * i + 1] = v.y;
      c[4 * i + 2] = v.z;
      c[4 * i + 3] = v.w;
    }
  }
  __device__ static inline float get(const uint32_t* c, int j) {
    const uint32_t w = c[j >> 1];
    const unsigned short bits = (j & 1) ? (unsigned short)(w >> 16) : (unsigned short)(w & 0xffffu);
    _Float16 h;
    memcpy(&h, &bits, 2);
    return (float)h;
  }
};

// FP16 storage widened to FP32 registers when the block is loaded: twice the
// registers of the packed form, plain FP32 multiply-adds in the contraction.
// Used where the register count is capped anyway (the illuminated vector
// kernel), and there faster than widening inside every multiply-add.
struct F16Widened {};

template <int NCF>
struct Coef<NCF, F16Widened> {
  using Reg = float;
  static constexpr int N8 = (NCF + 7) / 8;
  static constexpr int kRegs = 8 * N8;
  __device__ static inline void load(const void* bez, int64_t stride, int32_t e, float* c) {
    const uint4* r8 = reinterpret_cast<const uint4*>(static_cast<const _Float16*>(bez) + (int64_t)e * stride);
#pragma unroll
    for (int i = 0; i < N8; ++i) {
      const uint4 v = r8[i];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const unsigned short lo = (unsigned short)(w[k] & 0xffffu), hi = (unsigned short)(w[k] >> 16);
        _Float16 a, b;
        memcpy(&a, &lo, 2);
        memcpy(&b, &hi, 2);
        c[8 * i + 2 * k] = (float)a;
        c[8 * i + 2 * k + 1] = (float)b;
      }
    }
  }
  __device__ static inline float get(const float* c, int j) { return c[j]; }
};

template <int P>
__device__ inline void bernstein(float u, float b[P + 1]) {
  const float v = 1.0f - u;
  if constexpr (P == 1) {
    b[0] = v;
    b[1] = u;
  } else if constexpr (P == 2) {
    b[0] = v * v;
    b[1] = 2.0f * u * v;
    b[2] = u * u;
  } else {
    const float v2 = v * v, u2 = u * u;
    b[0] = v2 * v;
    b[1] = 3.0f * u * v2;
    b[2] = 3.0f * u2 * v;
    b[3] = u2 * u;
  }
}

// sum_j c[base + j] Bx[jx] By[jy] Bz[jz] for one component (x fastest).
template <int P, class CF>
__device__ inline float contract(const typename CF::Reg* c, int base, const float* bx, const float* by,
                                 const float* bz) {
  constexpr int Q = P + 1;
  float acc = 0.0f;
#pragma unroll
  for (int kz = 0; kz < Q; ++kz) {
    float ay = 0.0f;
#pragma unroll
    for (int jy = 0; jy < Q; ++jy) {
      float ax = 0.0f;
#pragma unroll
      for (int ix = 0; ix < Q; ++ix) ax = fmaf(CF::get(c, base + (kz * Q + jy) * Q + ix), bx[ix], ax);
      ay = fmaf(ax, by[jy], ay);
    }
    acc = fmaf(ay, bz[kz], acc);
  }
  return acc;
}

// Bernstein basis and its derivative: d/du B^P_j = P (B^{P-1}_{j-1} - B^{P-1}_j).
template <int P>
__device__ inline void bernstein_d(float u, float b[P + 1], float db[P + 1]) {
  const float v = 1.0f - u;
  if constexpr (P == 1) {
    b[0] = v;
    b[1] = u;
    db[0] = -1.0f;
    db[1] = 1.0f;
  } else if constexpr (P == 2) {
    b[0] = v * v;
    b[1] = 2.0f * u * v;
    b[2] = u * u;
    db[0] = -2.0f * v;
    db[1] = 2.0f * (v - u);
    db[2] = 2.0f * u;
  } else {
    const float v2 = v * v, u2 = u * u, uv = u * v;
    b[0] = v2 * v;
    b[1] = 3.0f * u * v2;
    b[2] = 3.0f * u2 * v;
    b[3] = u2 * u;
    db[0] = -3.0f * v2;
    db[1] = 3.0f * (v2 - 2.0f * uv);
    db[2] = 3.0f * (2.0f * uv - u2);
    db[3] = 3.0f * u2;
  }
}

// Value and local-coordinate gradient (d/du, d/dv, d/dw) of one component,
// sharing the partial sums: out = {f, f_u, f_v, f_w}.
template <int P, class CF>
__device__ inline void contract_grad(const typename CF::Reg* c, int base, const float* bx, const float* by,
                                     const float* bz, const float* dx, const float* dy, const float* dz,
                                     float out[4]) {
  constexpr int Q = P + 1;
  float f = 0.0f, fu = 0.0f, fv = 0.0f, fw = 0.0f;
#pragma unroll
  for (int kz = 0; kz < Q; ++kz) {
    float ay = 0.0f, ayu = 0.0f, ayv = 0.0f;
#pragma unroll
    for (int jy = 0; jy < Q; ++jy) {
      float ax = 0.0f, axu = 0.0f;
#pragma unroll
      for (int ix = 0; ix < Q; ++ix) {
        const float cv = CF::get(c, base + (kz * Q + jy) * Q + ix);
        ax = fmaf(cv, bx[ix], ax);
        axu = fmaf(cv, dx[ix], axu);
      }
      ay = fmaf(ax, by[jy], ay);
      ayu = fmaf(axu, by[jy], ayu);
      ayv = fmaf(ax, dy[jy], ayv);
    }
    f = fmaf(ay, bz[kz], f);
    fu = fmaf(ayu, bz[kz], fu);
    fv = fmaf(ayv, bz[kz], fv);
    fw = fmaf(ay, dz[kz], fw);
  }
  out[0] = f;
  out[1] = fu;
  out[2] = fv;
  out[3] = fw;
}

// Diffuse intensity max(0.4, |l . n|) with n = g / |g| (0.4 where g = 0).
__device__ inline float diffuse(const float l[3], const float g[3]) {
  const float nn = fmaf(g[0], g[0], fmaf(g[1], g[1], g[2] * g[2]));
  if (!(nn > 0.0f)) return 0.4f;
  const float dot = fabsf(fmaf(l[0], g[0], fmaf(l[1], g[1], l[2] * g[2])));
  return fmaxf(0.4f, dot * __builtin_amdgcn_rsqf(nn));
}

}  // namespace lrvr
