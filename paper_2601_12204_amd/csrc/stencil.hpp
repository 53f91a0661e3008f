// Pointwise arithmetic of the two steppers, shared by every kernel of this library so that all kernel
// variants of one scheme round identically.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace burgers {

// Explicit forward-Euler update of one node (Sec. 2.3, eq. 21): first-order upwind convection whose
// side follows the sign of c = r u_i (eq. 3 and the text after it), central diffusion (eq. 4).
template <typename T>
__device__ __forceinline__ T upwind_central(T ui, T um, T up, T r, T D) {
  const T c = r * ui;
  const T cpos = c > T(0) ? c : T(0);
  const T cneg = c < T(0) ? c : T(0);
  const T lap = (up + um) - T(2) * ui;
  return ((ui - cpos * (ui - um)) - cneg * (up - ui)) + D * lap;
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
