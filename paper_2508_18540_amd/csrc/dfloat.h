// Double-float (unevaluated float32 pair) arithmetic for the few per-primitive quantities
// that need more than float32 precision (projected means).  Requires -ffp-contract=off so
// the error-free transformations are evaluated exactly as written.
#pragma once

#include <hip/hip_runtime.h>

namespace lf {

struct df {
  float hi, lo;
};

__device__ __forceinline__ df quick_two_sum(float a, float b) {
  const float s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ df two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ df two_prod(float a, float b) {
  const float p = a * b;
  return {p, fmaf(a, b, -p)};
}

__device__ __forceinline__ df df_add(df a, df b) {
  const df s = two_sum(a.hi, b.hi);
  return quick_two_sum(s.hi, s.lo + (a.lo + b.lo));
}

__device__ __forceinline__ df df_add_f(df a, float b) {
  const df s = two_sum(a.hi, b);
  return quick_two_sum(s.hi, s.lo + a.lo);
}

__device__ __forceinline__ df df_mul(df a, df b) {
  df p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ df df_mul_f(df a, float b) {
  df p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return quick_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ df df_div(df a, df b) {
  const float q1 = a.hi / b.hi;
  const df r = df_add(a, df_mul_f(b, -q1));
  const float q2 = r.hi / b.hi;
  return quick_two_sum(q1, q2);
}

}  // namespace lf
