// Device-side helpers shared by the HIP kernels of libtgv: storage types,
// correctly rounded narrowing conversions, periodic index arithmetic and the
// kernel-side parameter block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tgv {

// bfloat16 storage: the upper 16 bits of an IEEE binary32.
struct bf16 {
  uint16_t bits;
};

using f16 = _Float16;
// Two FP16 values in one 32-bit register: arithmetic on it is element-wise
// and compiles to the packed FP16 VALU instructions (two results per lane).
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t f32_bits(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ float bits_f32(uint32_t u) { return __builtin_bit_cast(float, u); }

// binary32 -> bfloat16, round to nearest even; NaN stays NaN (quietened).
__device__ __forceinline__ bf16 f32_to_bf16(float x) {
  uint32_t u = f32_bits(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{(uint16_t)((u >> 16) | 0x40u)};
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16{(uint16_t)(u >> 16)};
}

// binary64 -> binary32 rounded to odd (Boldo & Melquiond, "Emulation of FMA and
// correctly rounded sums: proved algorithms using rounding to odd", IEEE TC 2008):
// truncate toward zero, then set the last bit if the conversion was inexact.
// A second rounding of the result to any format with at least two fewer
// significand bits (binary16, bfloat16) is then the correctly rounded value.
__device__ __forceinline__ float f64_to_f32_odd(double x) {
  float f = (float)x;  // round to nearest even
  double back = (double)f;
  if (back == x || !(x == x)) return f;
  uint32_t u = f32_bits(f);
  // step toward zero if RNE rounded away from zero
  if ((back > x && x > 0.0) || (back < x && x < 0.0)) u -= 1u;
  return bits_f32(u | 1u);
}

// Storage conversions, templated on the storage type.
template <class T>
struct Conv;

template <>
struct Conv<double> {
  __device__ __forceinline__ static double load_f64(double v) { return v; }
  __device__ __forceinline__ static float load_f32(double v) { return (float)v; }
  __device__ __forceinline__ static double from(double x) { return x; }
  __device__ __forceinline__ static double from(float x) { return (double)x; }
  __device__ __forceinline__ static double from(_Float16 x) { return (double)(float)x; }
};

template <>
struct Conv<float> {
  __device__ __forceinline__ static double load_f64(float v) { return (double)v; }
  __device__ __forceinline__ static float load_f32(float v) { return v; }
  __device__ __forceinline__ static float from(double x) { return (float)x; }
  __device__ __forceinline__ static float from(float x) { return x; }
  __device__ __forceinline__ static float from(_Float16 x) { return (float)x; }
};

// An FP32 value is first rounded in FP32 and then to FP16 (the arithmetic
// type, then the storage type).  The empty asm pins the FP32 value so the
// compiler cannot merge a producing fma with the conversion into a mixed
// fma that rounds only once.  It is not volatile: a volatile asm would also
// be a scheduling boundary for everything around it.
__device__ __forceinline__ f16 f32_to_f16(float x) {
  asm("" : "+v"(x));
  return (f16)x;
}

template <>
struct Conv<f16> {
  __device__ __forceinline__ static double load_f64(f16 v) { return (double)(float)v; }
  __device__ __forceinline__ static float load_f32(f16 v) { return (float)v; }
  __device__ __forceinline__ static f16 from(double x) { return f32_to_f16(f64_to_f32_odd(x)); }
  __device__ __forceinline__ static f16 from(float x) { return f32_to_f16(x); }
  __device__ __forceinline__ static f16 from(f16 x) { return x; }
};

template <>
struct Conv<bf16> {
  __device__ __forceinline__ static double load_f64(bf16 v) {
    return (double)bits_f32((uint32_t)v.bits << 16);
  }
  __device__ __forceinline__ static float load_f32(bf16 v) { return bits_f32((uint32_t)v.bits << 16); }
  __device__ __forceinline__ static bf16 from(double x) { return f32_to_bf16(f64_to_f32_odd(x)); }
  __device__ __forceinline__ static bf16 from(float x) { return f32_to_bf16(x); }
};

// Load a stored value into arithmetic type Tc.
template <class Tc, class T>
__device__ __forceinline__ Tc load_as(T v);
template <>
__device__ __forceinline__ double load_as<double, double>(double v) { return v; }
template <>
__device__ __forceinline__ double load_as<double, float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double load_as<double, f16>(f16 v) { return (double)(float)v; }
template <>
__device__ __forceinline__ double load_as<double, bf16>(bf16 v) { return Conv<bf16>::load_f64(v); }
template <>
__device__ __forceinline__ float load_as<float, double>(double v) { return (float)v; }
template <>
__device__ __forceinline__ float load_as<float, float>(float v) { return v; }
template <>
__device__ __forceinline__ float load_as<float, f16>(f16 v) { return (float)v; }
template <>
__device__ __forceinline__ float load_as<float, bf16>(bf16 v) { return Conv<bf16>::load_f32(v); }
// (a value read from memory has no producing fma to merge with: plain RNE)
template <>
__device__ __forceinline__ f16 load_as<f16, float>(float v) { return (f16)v; }
template <>
__device__ __forceinline__ f16 load_as<f16, f16>(f16 v) { return v; }

// Points per lane of an arithmetic type: 2 for the packed FP16 pair, else 1;
// lane_get reads point e of a lane value.
template <class Tc>
struct LaneT {
  static constexpr int P = 1;
  using E = Tc;
};
template <>
struct LaneT<h2> {
  static constexpr int P = 2;
  using E = f16;
};
template <class Tc>
constexpr int kLanes = LaneT<Tc>::P;
template <class Tc>
__device__ __forceinline__ typename LaneT<Tc>::E lane_get(Tc v, int e) {
  if constexpr (kLanes<Tc> == 1)
    return v;
  else
    return e == 0 ? v.x : v.y;
}
// A lane value from P consecutive stored points.
template <class Tc, class T>
__device__ __forceinline__ Tc lane_load(const T* pts) {
  if constexpr (kLanes<Tc> == 1)
    return load_as<Tc>(pts[0]);
  else
    return h2{load_as<f16>(pts[0]), load_as<f16>(pts[1])};
}

// Store an arithmetic value into storage type T (RNE, correctly rounded).
// Store that streams past the caches (the nontemporal hint on a vector
// store): for outputs written once and not read again by the same kernel.
template <class T>
__device__ __forceinline__ void stream_store(T* p, T v) {
  if constexpr (std::is_arithmetic<T>::value || std::is_same<T, _Float16>::value)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Load with the nontemporal hint: for inputs each point reads once (the RK
// register Q~), unlike Q, whose halo rows neighbouring tiles re-read from L2.
template <class T>
__device__ __forceinline__ T stream_load(const T* p) {
  if constexpr (std::is_arithmetic<T>::value || std::is_same<T, _Float16>::value)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <class T, class Tc>
__device__ __forceinline__ T store_as(Tc x) {
  return Conv<T>::from(x);
}

// Two-register RK update of one element (Sec. 3.1 update equations), shared
// by the stand-alone stage kernel and the fused residual + stage kernel so
// both round identically:  t = A qt + dt r (t = dt r at stage 0), stored as
// Tqt;  q_new = q + B t_stored.  Explicit fma fixes the contraction.
__device__ __forceinline__ double fused_ma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fused_ma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <class Ta>
__device__ __forceinline__ Ta rk_register(bool first, Ta A, Ta dt, Ta qt, Ta r) {
  return first ? dt * r : fused_ma(A, qt, dt * r);
}
template <class Ta>
__device__ __forceinline__ Ta rk_state(Ta B, Ta q, Ta t) {
  return fused_ma(B, t, q);
}

// 1/x from the hardware reciprocal estimate refined by Newton-Raphson steps
// r <- r + r (1 - x r), each of which squares the relative error: two steps
// in FP64, one in FP32, leave it at the rounding level of the type (within
// an ulp or two; x is a density, far from the overflow/underflow range).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);
}
// FP16 arithmetic: the FP32 reciprocal rounded once to FP16.
__device__ __forceinline__ f16 recip(f16 x) { return f32_to_f16(recip((float)x)); }
__device__ __forceinline__ h2 recip(h2 x) { return h2{recip(x.x), recip(x.y)}; }

// One-dimensional launches: a dispatch holds fewer than 2^32 work-items, so
// element-wise kernels loop grid-stride over their index range and their block
// count is capped here (a single pass for every grid up to 1024^3 x 5 values
// at 256 threads per block).
inline unsigned blocks_1d(long long work, int threads) {
  long long b = (work + threads - 1) / threads;
  const long long cap = (long long)(0xffffffffu / (unsigned)threads);
  return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

// Grid description passed to kernels by value.
struct Grid {
  int nx, ny, nz;
  long long N;       // nx * ny * nz
  long long plane;   // nx * ny
};

// Physical coefficients in arithmetic type Tc (computed on the host in FP64,
// rounded once).
template <class Tc>
struct Coef {
  Tc c1[3];   // 1 / (12 h_d): first-derivative scale
  Tc c2[3];   // 1 / (12 h_d^2): second-derivative scale
  Tc gm1;     // gamma - 1
  Tc igm1;    // 1 / (gamma - 1)
  Tc gm2;     // gamma M^2
  Tc ire;     // 1 / Re
  Tc kap;     // 1 / ((gamma - 1) M^2 Pr Re)
  Tc vis2[3];   // (1/Re) / (12 h_d^2): transverse viscous second derivative
  Tc vis2l[3];  // (4/3)(1/Re) / (12 h_d^2): longitudinal (D2_a u_a counted in X_a too)
  Tc kap2[3];   // kappa / (12 h_d^2): heat flux
  int viscous;
};

}  // namespace tgv
