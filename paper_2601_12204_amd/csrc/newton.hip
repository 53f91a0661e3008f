// Fully implicit step with central convection, solved by Newton-Raphson (Sec. 2.4, eqs. 10-14).
// With r = dt/dx and D = nu dt/dx^2, one step solves F(x) = 0 for
//   F_i(x) = (x_i - u_i) + ((r/2) x_i (x_{i+1} - x_{i-1}) - D ((x_{i+1} + x_{i-1}) - 2 x_i)),
// starting from x = u and iterating J(x) delta = -F(x), x = x + delta a fixed number of times.  J is
// tridiagonal (cyclic for periodic instances), with the derivatives of eq. 11 as its entries:
//   J_{i,i-1} = -(r/2) x_i - D,   J_{i,i} = (1 + 2D) + (r/2)(x_{i+1} - x_{i-1}),   J_{i,i+1} = (r/2) x_i - D.
// Each iteration assembles J's rows divided by their diagonal and -F / J_ii into binary64 arrays (one
// system per instance at its offset) for the partition solver's array path, then adds delta to x.
// Dirichlet nodes are fixed (delta = 0) and enter F as known neighbours.  The iterate x lives in the
// output state buffer, in the state's type.
#include "internal.hpp"
#include "newton_check.hpp"

#pragma clang fp contract(off)

namespace burgers {
namespace {

constexpr int kNewtonThreads = 256;

// x = u on the instance's nodes, Dirichlet nodes set to their values.
template <typename S>
__global__ __launch_bounds__(kNewtonThreads) void newton_init_kernel(const InstDesc* __restrict__ inst,
                                                                     const AdjTile* __restrict__ tiles,
                                                                     const S* __restrict__ u, S* __restrict__ x) {
  const AdjTile t = tiles[blockIdx.x];
  const int j = t.start + static_cast<int>(threadIdx.x);
  if (j >= t.n) return;
  S v = u[t.off + j];
  if (t.bc == kDirichlet && (j == 0 || j == t.n - 1)) {
    const InstDesc d = inst[t.inst];
    v = static_cast<S>(j == 0 ? d.a : d.b);
  }
  x[t.off + j] = v;
}

template <typename S>
__global__ __launch_bounds__(kNewtonThreads) void newton_assemble_kernel(
    const InstDesc* __restrict__ inst, const AdjTile* __restrict__ tiles, const S* __restrict__ u,
    const S* __restrict__ x, double* __restrict__ NA, double* __restrict__ NC, double* __restrict__ ND,
    int* __restrict__ flags) {
  const AdjTile t = tiles[blockIdx.x];
  const int n = t.n;
  const int i = t.start + static_cast<int>(threadIdx.x);
  const bool periodic = t.bc == kPeriodic;
  const int first = periodic ? 0 : 1;
  const int m = periodic ? n : n - 2;
  const int k = i - first;
  if (i >= n || k < 0 || k >= m) return;
  const InstDesc d = inst[t.inst];
  const S* __restrict__ xs = x + t.off;
  double xm, xp;
  if (periodic) {
    xm = static_cast<double>(xs[i == 0 ? n - 1 : i - 1]);
    xp = static_cast<double>(xs[i == n - 1 ? 0 : i + 1]);
  } else {
    xm = i == 1 ? d.a : static_cast<double>(xs[i - 1]);
    xp = i == n - 2 ? d.b : static_cast<double>(xs[i + 1]);
  }
  const double xi = static_cast<double>(xs[i]);
  const double half_r = d.r / 2.0, D = d.D;
  const double F = (xi - static_cast<double>(u[t.off + i])) + (half_r * xi * (xp - xm) - D * ((xp + xm) - 2.0 * xi));
  double sub = -(half_r * xi) - D;
  const double diag = (1.0 + 2.0 * D) + half_r * (xp - xm);
  double sup = half_r * xi - D;
  if (!periodic) {              // known Dirichlet neighbours do not move
    if (k == 0) sub = 0.0;
    if (k == m - 1) sup = 0.0;
  }
  newton_check_row(sub, diag, sup, flags);
  const int64_t o = t.sys_off + k;
  NA[o] = sub / diag;
  NC[o] = sup / diag;
  ND[o] = -F / diag;
}

// x += delta on the unknowns; on the last iteration the increments are checked against the iterate
// (every lane takes part in the wave's reduction).
template <typename S>
__global__ __launch_bounds__(kNewtonThreads) void newton_update_kernel(const AdjTile* __restrict__ tiles,
                                                                       const S* __restrict__ u, S* __restrict__ x,
                                                                       const double* __restrict__ NX, int last,
                                                                       int* __restrict__ flags) {
  const AdjTile t = tiles[blockIdx.x];
  const int n = t.n;
  const int i = t.start + static_cast<int>(threadIdx.x);
  const bool periodic = t.bc == kPeriodic;
  const int first = periodic ? 0 : 1;
  const int m = periodic ? n : n - 2;
  const int k = i - first;
  const bool active = i < n && k >= 0 && k < m;
  double delta = 0.0, xn = 0.0, uo = 0.0;
  if (active) {
    delta = NX[t.sys_off + k];
    const S v = static_cast<S>(static_cast<double>(x[t.off + i]) + delta);
    x[t.off + i] = v;
    xn = static_cast<double>(v);
    if (last) uo = static_cast<double>(u[t.off + i]);
  }
  if (last) newton_check_increment(active, delta, xn, uo, newton_increment_tol<S>(), flags);
}

}  // namespace

hipError_t launch_newton_init(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles, const void* u, void* x) {
  if (n_tiles <= 0) return hipSuccess;
  const unsigned g = static_cast<unsigned>(n_tiles);
  if (ctx->dtype == BURGERS_F64)
    newton_init_kernel<double><<<g, kNewtonThreads, 0, ctx->stream>>>(
        ctx->inst.as<InstDesc>(), tiles, static_cast<const double*>(u), static_cast<double*>(x));
  else
    newton_init_kernel<float><<<g, kNewtonThreads, 0, ctx->stream>>>(
        ctx->inst.as<InstDesc>(), tiles, static_cast<const float*>(u), static_cast<float*>(x));
  return hipGetLastError();
}

hipError_t launch_newton_assemble(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles, const void* u,
                                  const void* x, double* NA, double* NC, double* ND, int* flags) {
  if (n_tiles <= 0) return hipSuccess;
  const unsigned g = static_cast<unsigned>(n_tiles);
  if (ctx->dtype == BURGERS_F64)
    newton_assemble_kernel<double><<<g, kNewtonThreads, 0, ctx->stream>>>(
        ctx->inst.as<InstDesc>(), tiles, static_cast<const double*>(u), static_cast<const double*>(x), NA, NC, ND, flags);
  else
    newton_assemble_kernel<float><<<g, kNewtonThreads, 0, ctx->stream>>>(
        ctx->inst.as<InstDesc>(), tiles, static_cast<const float*>(u), static_cast<const float*>(x), NA, NC, ND, flags);
  return hipGetLastError();
}

hipError_t launch_newton_update(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles, const void* u,
                                void* x, const double* NX, bool last, int* flags) {
  if (n_tiles <= 0) return hipSuccess;
  const unsigned g = static_cast<unsigned>(n_tiles);
  if (ctx->dtype == BURGERS_F64)
    newton_update_kernel<double><<<g, kNewtonThreads, 0, ctx->stream>>>(
        tiles, static_cast<const double*>(u), static_cast<double*>(x), NX, last ? 1 : 0, flags);
  else
    newton_update_kernel<float><<<g, kNewtonThreads, 0, ctx->stream>>>(
        tiles, static_cast<const float*>(u), static_cast<float*>(x), NX, last ? 1 : 0, flags);
  return hipGetLastError();
}

}  // namespace burgers
