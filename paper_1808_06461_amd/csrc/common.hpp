// Shared device helpers for the channel RK3 kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "host.hpp"  // FftPlan: radices of the Stockham passes and twiddle offsets

namespace chn {

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };
template <typename T> using c2 = typename V2<T>::type;

template <typename T> __device__ __forceinline__ c2<T> mk(T x, T y) { c2<T> r; r.x = x; r.y = y; return r; }
// v where c holds, else zero: selected per component (a select of the whole
// pair can be lowered through a stack copy of both candidates)
template <typename T> __device__ __forceinline__ c2<T> keep_if(bool c, c2<T> v) {
  return mk<T>(c ? v.x : T(0), c ? v.y : T(0));
}
template <typename T> __device__ __forceinline__ c2<T> cadd(c2<T> a, c2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ c2<T> csub(c2<T> a, c2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ c2<T> cscale(c2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by +i (sgn > 0) or -i (sgn < 0)
template <typename T> __device__ __forceinline__ c2<T> cmuli(c2<T> a, int sgn) {
  return sgn > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
template <typename T> __device__ __forceinline__ c2<T> cconj(c2<T> a) { return mk<T>(a.x, -a.y); }

// Maximum that propagates NaN from either argument (fmax drops a NaN
// operand), for the CFL reductions that guard against blown-up states.
template <typename T> __device__ __forceinline__ T nanmax(T a, T b) { return (b > a || b != b) ? b : a; }

// Instability guard of a context, four words in device memory:
//   [0] CFL maximum of the current sub-step as the bits of a non-negative
//       float (reset by the z inverse, raised by atomicMax in the x pass; as
//       unsigned integers the bits order like the values, +inf and NaN
//       above every finite one),
//   [1] fail code: 0, or 1 + 3 step + sub-step of the first sub-step whose
//       CFL was not finite or above the limit (set by the pencil kernel),
//   [2] steps completed since the host cleared the guard,
//   [3] unused.
constexpr unsigned kGuardNonFinite = 0x7f800000u;  // bits of +inf

// Plans with a composite radix (6, 9, 12, 16): their kernels take the
// runtime passes that include those radices.
__host__ __device__ inline bool plan_is_composite(const FftPlan& pl) {
  for (int p = 0; p < pl.npass; ++p)
    if (pl.radix[p] != 2 && pl.radix[p] != 3 && pl.radix[p] != 4 && pl.radix[p] != 8) return true;
  return false;
}

// Plans with a compile-time radix schedule (FN template argument of the plane kernels).
__host__ __device__ inline bool plan_is_576(const FftPlan& pl) {
  return pl.n == 576 && pl.npass == 4 && pl.radix[0] == 8 && pl.radix[1] == 8 && pl.radix[2] == 3 &&
         pl.radix[3] == 3;
}
// 576 points in the composite radix set: 9, 8, 8.
__host__ __device__ inline bool plan_is_576c(const FftPlan& pl) {
  return pl.n == 576 && pl.npass == 3 && pl.radix[0] == 9 && pl.radix[1] == 8 && pl.radix[2] == 8;
}
// The long lines of the 8192 x 6144 planes: 9216 points (radices 8, 8, 8, 2,
// 3, 3) and 12288 points (8, 8, 8, 8, 3), compile-time schedules like 576.
__host__ __device__ inline bool plan_has(const FftPlan& pl, int n, int np, const int* r) {
  if (pl.n != n || pl.npass != np) return false;
  for (int p = 0; p < np; ++p)
    if (pl.radix[p] != r[p]) return false;
  return true;
}
__host__ __device__ inline bool plan_is_9216(const FftPlan& pl) {
  const int r[6] = {8, 8, 8, 2, 3, 3};
  return plan_has(pl, 9216, 6, r);
}
__host__ __device__ inline bool plan_is_12288(const FftPlan& pl) {
  const int r[5] = {8, 8, 8, 8, 3};
  return plan_has(pl, 12288, 5, r);
}
// The product grid of the 1536 x 385 x 1152 low-storage stage: 1728-point x
// lines in the composite set (12, 12, 12).
__host__ __device__ inline bool plan_is_1728c(const FftPlan& pl) {
  const int r[3] = {12, 12, 12};
  return plan_has(pl, 1728, 3, r);
}

// XCD-aware order of a launch's n workgroups.  The dispatcher deals
// workgroup w to XCD w % 8, and each XCD has its own L2; this gives XCD x the
// contiguous range of logical tiles [x q + min(x, r), ...) (q = n / 8,
// r = n % 8), so neighbouring tiles, which share cache lines at their edges,
// run on one XCD close together in time.  A bijection of [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int w, int n) {
  const int q = n / kXcds, r = n % kXcds;
  const int x = w % kXcds, j = w / kXcds;
  return x * q + (x < r ? x : r) + j;
}

}  // namespace chn
