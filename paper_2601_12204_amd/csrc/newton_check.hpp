// Checks of the Newton-Raphson step (fully implicit central convection, Sec. 2.4, eqs. 10-14), shared by
// its whole-system and array-path kernels.  The Jacobian systems are solved without pivoting, which is
// sound while every row is strictly diagonally dominant; and the step takes a fixed number of
// iterations, which is meant to reach rounding level.  Both are checked on the device, and a failure is
// recorded in two flags of the context (plain stores of 1, read and cleared by burgers_sync):
//   flags[0]  some Jacobian row was not strictly diagonally dominant (or not finite);
//   flags[1]  the last iteration's increment was not small against the iterate (or not finite).
#pragma once

#include <hip/hip_runtime.h>

namespace burgers {

// Largest relative size of the last Newton increment that counts as converged: against the largest
// magnitude of the iterate and old state over the wave's 64 nodes.  A binary32 iterate is rounded to
// binary32 after every iteration, so its last increment is of the order of that rounding.
template <typename S>
constexpr double newton_increment_tol() {
  return sizeof(S) == 8 ? 1e-10 : 1e-5;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = __builtin_fmax(v, __shfl_xor(v, m, 64));
  return v;
}

// Row (sub, diag, sup) of the Jacobian that is not strictly diagonally dominant (or not finite).
__device__ __forceinline__ bool newton_row_not_dominant(double sub, double diag, double sup) {
  return !(__builtin_fabs(diag) > __builtin_fabs(sub) + __builtin_fabs(sup));
}

// Flag such a row.
__device__ __forceinline__ void newton_check_row(double sub, double diag, double sup, int* flags) {
  if (newton_row_not_dominant(sub, diag, sup)) flags[0] = 1;
}

// Last iteration of a node: increment delta, new iterate xn, old state u.  `active` is false for lanes
// without a node; every lane of the wave must call this (it reduces over the wave).
__device__ __forceinline__ void newton_check_increment(bool active, double delta, double xn, double u, double tol,
                                                       int* flags) {
  const bool finite = __builtin_isfinite(delta) && __builtin_isfinite(xn);
  const double inc = active ? (finite ? __builtin_fabs(delta) : __builtin_inf()) : 0.0;
  const double scale = active && finite ? __builtin_fmax(__builtin_fabs(xn), __builtin_fabs(u)) : 0.0;
  const double inc_max = wave_max(inc);
  const double scale_max = wave_max(scale);
  if ((threadIdx.x & 63) == 0 && !(inc_max <= tol * scale_max)) flags[1] = 1;
}

}  // namespace burgers
