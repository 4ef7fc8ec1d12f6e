// fixsum.h -- order-independent accumulation of FP64 values in device memory.
//
// A sum built from floating-point atomic adds of many workgroups rounds after every
// addition, so its last bits depend on the order in which the workgroups arrive: the
// same step gives different currents from run to run, and nodes that should hold equal
// values (by a symmetry of the particle loading) can differ in the last bit.
//
// Here every value v is taken as the integer V = round(v 2^s), held in two int64 limbs
//   H = floor(v 2^(s-K)),   L = round((v 2^(s-K) - H) 2^K)  in [0, 2^K],
// so that V = H 2^K + L, and both limbs are summed with integer atomics.  Integer
// addition is exact and associative: the accumulated pair, and the FP64 value read from
// it, are the same for every order of arrival.
//
// The exponent s is fixed per run from a bound B >= the sum of |v| reaching one entry
// (for the current, kappa sum_i |q_i| / dV; see fix_scale): then |sum H| < 2^62 when
// B 2^(s-K) <= 2^61, and sum L < 2^63 for fewer than 2^(63-K) additions to one entry.
// The resolution 2^-s = B 2^(K-61) lies about 2^-91 below B, far under the FP64 rounding
// of any sum that occurs.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace gmhc {

constexpr int kFixK = 30;  // bits of the low limb

// Scale factors of one run: up = 2^(s-K) (value -> high limb), hi = 2^(K-s) and
// lo = 2^-s (limbs -> value).
struct FixScale {
  double up, hi, lo;
};

// Scale for sums whose absolute values stay below `bound` (host side).
inline FixScale fix_scale(double bound) {
  if (!(bound > 0.0) || !isfinite(bound)) bound = 1.0;
  const int eb = (int)ceil(log2(bound));
  const int s = kFixK + 61 - eb;  // B 2^(s-K) <= 2^61
  return FixScale{ldexp(1.0, s - kFixK), ldexp(1.0, kFixK - s), ldexp(1.0, -s)};
}

__device__ __forceinline__ void fix_split(double v, double up, long long& H, long long& L) {
  const double t = v * up;        // exact: a power-of-two scaling
  const double h = floor(t);
  H = (long long)h;
  L = (long long)rint((t - h) * (double)(1ll << kFixK));  // t - h is exact, in [0, 1)
}

// acc holds one (H, L) pair per entry: entry i at acc[2 i], acc[2 i + 1].
__device__ __forceinline__ void fix_add(unsigned long long* acc, int64_t i, double v, double up) {
  long long H, L;
  fix_split(v, up, H, L);
  if (H) atomicAdd(acc + 2 * i, (unsigned long long)H);
  if (L) atomicAdd(acc + 2 * i + 1, (unsigned long long)L);
}

__device__ __forceinline__ double fix_value(const unsigned long long* acc, int64_t i, double hi, double lo) {
  return (double)(long long)acc[2 * i] * hi + (double)(long long)acc[2 * i + 1] * lo;
}

}  // namespace gmhc
