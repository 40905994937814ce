// Double-float ("double-word" of binary32) arithmetic for the compensated products.
//
// A value is the unevaluated sum hi + lo of two floats with |lo| <= ulp(hi) / 2, which
// carries about 48 significant bits.  The building blocks are the error-free
// transformations
//   TwoSum (Knuth):      s = fl(a + b), e = (a + b) - s exactly, any a, b;
//   Fast2Sum (Dekker):   the same when |a| >= |b| (or a = 0), three operations;
//   2Prod (with FMA):    p = fl(a b), e = fma(a, b, -p) = a b - p exactly;
// and, on top of them, the double-word algorithms analysed by Joldes, Muller and Popescu
// ("Tight and rigorous error bounds for basic building blocks of double-word
// arithmetic", ACM TOMS 44(2), 2017):
//   addition  AccurateDWPlusDW   relative error <= 3 u^2 / (1 - 4u),
//   product   DWTimesDW (FMA)    relative error <= 5 u^2,
//   quotient  one correction step on the float quotient,
// with u = 2^-24.  FMA contraction is switched off inside these functions: contracting
// fl(a * b) + e into one fma would break the exactness the transformations rely on.

#pragma once

#include <hip/hip_runtime.h>

namespace birk {

struct df32 {
  float hi, lo;
  df32() = default;
  __host__ __device__ constexpr df32(float h, float l) : hi(h), lo(l) {}
  // Nearest double-float to a double: hi = rn(d), lo = rn(d - hi) (d - hi is exact).
  __host__ __device__ constexpr df32(double d) : hi((float)d), lo((float)(d - (double)(float)d)) {}
  __host__ __device__ constexpr df32(float f) : hi(f), lo(0.0f) {}
  __host__ __device__ constexpr df32(int i) : df32((double)i) {}
  __host__ __device__ constexpr df32(long i) : df32((double)i) {}
  __host__ __device__ constexpr df32(long long i) : df32((double)i) {}
  __host__ __device__ explicit operator double() const { return (double)hi + (double)lo; }
};

struct __align__(16) df32c {
  df32 x, y;
};

namespace dfw {

__host__ __device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__host__ __device__ __forceinline__ void fast_two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  e = b - (s - a);
}

}  // namespace dfw

__host__ __device__ __forceinline__ df32 operator+(df32 x, df32 y) {
#pragma clang fp contract(off)
  float sh, sl, th, tl, vh, vl, zh, zl;
  dfw::two_sum(x.hi, y.hi, sh, sl);
  dfw::two_sum(x.lo, y.lo, th, tl);
  const float c = sl + th;
  dfw::fast_two_sum(sh, c, vh, vl);
  const float w = tl + vl;
  dfw::fast_two_sum(vh, w, zh, zl);
  return df32(zh, zl);
}

__host__ __device__ __forceinline__ df32 operator-(df32 x) { return df32(-x.hi, -x.lo); }
__host__ __device__ __forceinline__ df32 operator-(df32 x, df32 y) { return x + (-y); }

__host__ __device__ __forceinline__ df32 operator*(df32 x, df32 y) {
#pragma clang fp contract(off)
  const float ch = x.hi * y.hi;
  const float cl1 = __builtin_fmaf(x.hi, y.hi, -ch);
  const float tl0 = x.lo * y.lo;
  const float tl1 = __builtin_fmaf(x.hi, y.lo, tl0);
  const float cl2 = __builtin_fmaf(x.lo, y.hi, tl1);
  const float cl3 = cl1 + cl2;
  float zh, zl;
  dfw::fast_two_sum(ch, cl3, zh, zl);
  return df32(zh, zl);
}

__host__ __device__ __forceinline__ df32 operator/(df32 x, df32 y) {
#pragma clang fp contract(off)
  const float q1 = x.hi / y.hi;
  const df32 r = x - y * df32(q1, 0.0f);
  const float q2 = r.hi / y.hi;
  float zh, zl;
  dfw::fast_two_sum(q1, q2, zh, zl);
  return df32(zh, zl);
}

__host__ __device__ __forceinline__ df32& operator+=(df32& a, df32 b) { return a = a + b; }
__host__ __device__ __forceinline__ df32& operator-=(df32& a, df32 b) { return a = a - b; }
__host__ __device__ __forceinline__ df32& operator*=(df32& a, df32 b) { return a = a * b; }

}  // namespace birk
