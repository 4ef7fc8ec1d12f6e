// wave.h -- wave64 helpers shared by the HIP kernels of libgmhc: bit casts of FP64
// values and wave-wide reductions through DPP row shifts (no LDS round trips).
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

namespace gmhc {

__device__ __forceinline__ uint64_t as_u64(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double as_f64(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | (uint64_t)lo));
}

// ---- wave-wide reductions through DPP row shifts (no LDS): an inclusive scan within each
// row of 16 lanes (shifts by 1, 2, 4 and 8; lanes without a source take the identity),
// then the four row results are read from lanes 15, 31, 47 and 63 and combined in order.
// All 64 lanes must be active; the result is wave-uniform.
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int id, int v) {
  return __builtin_amdgcn_update_dpp(id, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ int wave_min_i32(int v) {
  v = min(v, dpp_i32<kDppShr1>(INT_MAX, v));
  v = min(v, dpp_i32<kDppShr2>(INT_MAX, v));
  v = min(v, dpp_i32<kDppShr4>(INT_MAX, v));
  v = min(v, dpp_i32<kDppShr8>(INT_MAX, v));
  return min(min(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             min(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}
__device__ __forceinline__ int wave_max_i32(int v) {
  v = max(v, dpp_i32<kDppShr1>(INT_MIN, v));
  v = max(v, dpp_i32<kDppShr2>(INT_MIN, v));
  v = max(v, dpp_i32<kDppShr4>(INT_MIN, v));
  v = max(v, dpp_i32<kDppShr8>(INT_MIN, v));
  return max(max(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             max(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}
// the source lane's x, or id where there is none
template <int CTRL>
__device__ __forceinline__ double dpp_f64_id(double id, double x) {
  const uint64_t u = as_u64(x), e = as_u64(id);
  const uint32_t lo = (uint32_t)dpp_i32<CTRL>((int)(uint32_t)e, (int)(uint32_t)u);
  const uint32_t hi = (uint32_t)dpp_i32<CTRL>((int)(uint32_t)(e >> 32), (int)(uint32_t)(u >> 32));
  return as_f64(lo, hi);
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const uint64_t u = as_u64(x);
  return as_f64((uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l),
                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l));
}
// wave sum (MAX = false) or maximum (MAX = true) of x
template <bool MAX>
__device__ __forceinline__ double wave_reduce_f64(double x) {
  const double id = MAX ? -INFINITY : 0.0;
  auto op = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
  x = op(x, dpp_f64_id<kDppShr1>(id, x));
  x = op(x, dpp_f64_id<kDppShr2>(id, x));
  x = op(x, dpp_f64_id<kDppShr4>(id, x));
  x = op(x, dpp_f64_id<kDppShr8>(id, x));
  return op(op(readlane_f64(x, 15), readlane_f64(x, 31)), op(readlane_f64(x, 47), readlane_f64(x, 63)));
}

}  // namespace gmhc
