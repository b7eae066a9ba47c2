// Float-float arithmetic (Dekker 1971; Knuth TAOCP vol. 2, 4.2.2): a value
// is the unevaluated sum hi + lo of two float32 numbers with |lo| <= ulp(hi)/2,
// which carries about 48 significant bits while every operation stays in
// float32.  The float32 result of an accumulation is hi.
#pragma once

#include <hip/hip_runtime.h>

namespace fr {
namespace ffa {

struct ff {
  float hi, lo;
};

__device__ __forceinline__ ff two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ ff fast_two_sum(float a, float b) {
  const float s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ ff add(ff x, ff y) {
  const ff s = two_sum(x.hi, y.hi);
  return fast_two_sum(s.hi, s.lo + (x.lo + y.lo));
}

// x * f for a float32 factor f.
__device__ __forceinline__ ff mul_f(ff x, float f) {
  const float p = x.hi * f;
  return fast_two_sum(p, fmaf(x.hi, f, -p) + x.lo * f);
}

// What a donor holding x passes along an edge of fraction f, with the
// donor's conservation correction d (its fractions, rounded to float32, sum
// to 1 - d to first order): x * f * (1 + d).
__device__ __forceinline__ ff mul_fd(ff x, float f, float d) {
  const ff p = mul_f(x, f);
  return fast_two_sum(p.hi, fmaf(p.hi, d, p.lo));
}

}  // namespace ffa
}  // namespace fr
