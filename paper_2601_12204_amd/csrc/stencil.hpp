// Pointwise arithmetic of the two steppers, shared by every kernel of this library so that all kernel
// variants of one scheme round identically.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace burgers {

// a * b + c rounded once.  Used only where a * b is exact (a = +-2), so it rounds exactly like the
// unfused a * b + c while taking one instruction instead of two (for |b| below half the largest
// finite value, where 2b cannot overflow).
template <typename T>
__device__ __forceinline__ T fma_exact(T a, T b, T c) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_fma(a, b, c);
  } else {
    return __builtin_fmaf(a, b, c);
  }
}

// Explicit forward-Euler update of one node (Sec. 2.3, eq. 21): first-order upwind convection whose
// side follows the sign of c = r u_i (eq. 3 and the text after it), central diffusion (eq. 4):
//   u' = ((u - max(c,0) (u - u_m)) - min(c,0) (u_p - u)) + D ((u_p + u_m) - 2u).
// At most one of max(c,0), min(c,0) is nonzero; the other one's product is a zero, and subtracting a
// zero leaves a value unchanged, so selecting the upwind difference by the sign of c and subtracting
// c times it rounds exactly like the formula above (up to the sign of a zero result).
template <typename T>
__device__ __forceinline__ T upwind_central(T ui, T um, T up, T r, T D) {
  const T c = r * ui;
  const T diff = c > T(0) ? ui - um : up - ui;
  const T lap = fma_exact(T(-2), ui, up + um);  // (u_p + u_m) - 2u
  return (ui - c * diff) + D * lap;
}

// Increment dt L(v) of one node for the classical RK4 step (Sec. 2.7.1, eq. 22) over eq. 21's spatial
// operator:  K = D ((v_p + v_m) - 2v) - (max(c,0) (v - v_m) + min(c,0) (v_p - v)),  c = r v.  As in
// upwind_central, one of the two products is a zero, so selecting the upwind difference rounds the same.
template <typename T>
__device__ __forceinline__ T rk4_increment(T vi, T vm, T vp, T r, T D) {
  const T c = r * vi;
  const T diff = c > T(0) ? vi - vm : vp - vi;
  const T lap = fma_exact(T(-2), vi, vp + vm);  // (v_p + v_m) - 2v
  return D * lap - c * diff;
}

// Row of the BTCS matrix (Sec. 2.4, eq. 23) at a node with old value ui, convective coefficient
// c = r u_i lagged at u^n:  sub = -(D + max(c,0)), diag = 1 + 2D + |c|, super = min(c,0) - D.
// Every row sums to one, and the matrix is a strictly diagonally dominant M-matrix.
template <typename T>
__device__ __forceinline__ void btcs_row(T ui, T r, T D, T& sub, T& diag, T& sup) {
  const T c = r * ui;
  const T cpos = c > T(0) ? c : T(0);
  const T cneg = c < T(0) ? c : T(0);
  const T cabs = __builtin_fabs(c);
  sub = -(D + cpos);
  diag = (T(1) + T(2) * D) + cabs;
  sup = cneg - D;
}

}  // namespace burgers
