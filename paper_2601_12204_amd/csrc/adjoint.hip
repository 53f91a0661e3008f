// Discrete adjoint of the two steppers (binary64), for gradients of a loss of the final state with
// respect to the initial state and the viscosity.  The paper obtains such gradients by reverse-mode AD
// through its solvers (Sec. 2.7.1 and 2.7.3); here the derivatives of the discrete steps are written
// out by hand.  The upwind switch is differentiated on its u_i >= 0 branch at u_i = 0, dt is a
// constant, and nu enters through D = nu dt/dx^2 only.  Dirichlet boundary nodes are constants.
//
// Explicit step (Sec. 2.3, eq. 21): the adjoint of u' = E(u) is the transpose of the 3-point Jacobian,
// a gather stencil.  BTCS step (Sec. 2.4, eq. 23): x = A(y)^{-1} y gives
//   mu = A(y)^{-T} lam',   lam = (1 - G) mu,   G_i = r [H (x_i - x_{i-1}) + (1 - H)(x_{i+1} - x_i)],
//   dJ/dD += -sum_i mu_i (2 x_i - x_{i-1} - x_{i+1}),
// with the Dirichlet values standing in as x_0 = a, x_{n-1} = b.  A^T is tridiagonal with the neighbours'
// coefficients (sub p_{i-1}, super l_{i+1}, the cyclic corners swapped); it is assembled with unit
// diagonal into binary64 arrays and solved by the partition solver's array path.
//
// dJ/dD is accumulated per tile, one workgroup per tile per launch, so the sums are deterministic.
#include "internal.hpp"
#include "stencil.hpp"

#pragma clang fp contract(off)

namespace burgers {
namespace {

constexpr int kAdjThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kAdjThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = red[t] + red[t + s];
    __syncthreads();
  }
  return red[0];
}

// lam = (dE/du)^T lamp at state u; partial dJ/dD of the tile added to gslot[tile.slot].
__global__ __launch_bounds__(kAdjThreads) void adj_explicit_kernel(
    const InstDesc* __restrict__ inst, const AdjTile* __restrict__ tiles, const double* __restrict__ u,
    const double* __restrict__ lamp, double* __restrict__ lam, double* __restrict__ gslot) {
  __shared__ double red[kAdjThreads];
  const AdjTile t = tiles[blockIdx.x];
  const InstDesc d = inst[t.inst];
  const int n = t.n;
  const int j = t.start + static_cast<int>(threadIdx.x);
  const bool periodic = t.bc == kPeriodic;
  const double* __restrict__ y = u + t.off;
  const double* __restrict__ lp = lamp + t.off;
  const double r = d.r, D = d.D;
  double g = 0.0;
  if (j < n) {
    double acc = 0.0;
    if (periodic || (j > 0 && j < n - 1)) {
      const int jm = j == 0 ? n - 1 : j - 1;
      const int jp = j == n - 1 ? 0 : j + 1;
      const double uj = y[j];
      const double um = (!periodic && j == 1) ? d.a : y[jm];
      const double up = (!periodic && j == n - 2) ? d.b : y[jp];
      // own update
      const double self = uj >= 0.0 ? ((1.0 - r * (uj - um)) - r * uj) - 2.0 * D
                                    : ((1.0 - r * (up - uj)) + r * uj) - 2.0 * D;
      acc = self * lp[j];
      g = lp[j] * ((up + um) - 2.0 * uj);
      // node j+1 reads u_j as its left neighbour
      if (periodic || j + 1 <= n - 2) {
        const double uk = y[jp];
        acc = acc + (uk >= 0.0 ? r * uk + D : D) * lp[jp];
      }
      // node j-1 reads u_j as its right neighbour
      if (periodic || j - 1 >= 1) {
        const double uk = y[jm];
        acc = acc + (uk >= 0.0 ? D : D - r * uk) * lp[jm];
      }
    }
    lam[t.off + j] = acc;
  }
  const double tot = block_sum(g, red);
  if (threadIdx.x == 0) gslot[t.slot] = gslot[t.slot] + tot;
}

// Row k of A(y)^T, normalised by its diagonal, and the right-hand side lamp / d, for every unknown of
// the tile's instance; written at t.sys_off of the adjoint arrays.
__global__ __launch_bounds__(kAdjThreads) void adj_btcs_assemble_kernel(
    const InstDesc* __restrict__ inst, const AdjTile* __restrict__ tiles, const double* __restrict__ u,
    const double* __restrict__ lamp, double* __restrict__ LA, double* __restrict__ LC,
    double* __restrict__ LD) {
  const AdjTile t = tiles[blockIdx.x];
  const InstDesc d = inst[t.inst];
  const int n = t.n;
  const bool periodic = t.bc == kPeriodic;
  const int first = periodic ? 0 : 1;
  const int m = periodic ? n : n - 2;
  const int k = t.start + static_cast<int>(threadIdx.x) - first;   // unknown index of this node
  if (t.start + static_cast<int>(threadIdx.x) >= n || k < 0 || k >= m) return;
  const double* __restrict__ y = u + t.off;
  double sub, diag, sup, tmp1, tmp2;
  btcs_row(y[first + k], d.r, d.D, sub, diag, sup);
  double sub_t = 0.0, sup_t = 0.0;   // p_{k-1} and l_{k+1}
  if (periodic || k > 0) {
    const int km = k == 0 ? m - 1 : k - 1;
    btcs_row(y[first + km], d.r, d.D, tmp1, tmp2, sub_t);
  }
  if (periodic || k < m - 1) {
    const int kp = k == m - 1 ? 0 : k + 1;
    btcs_row(y[first + kp], d.r, d.D, sup_t, tmp1, tmp2);
  }
  const int64_t o = t.sys_off + k;
  LA[o] = sub_t / diag;
  LC[o] = sup_t / diag;
  LD[o] = lamp[t.off + first + k] / diag;
}

// lam = (1 - G) mu and the tile's partial -mu . (L x); boundary nodes get zero.
__global__ __launch_bounds__(kAdjThreads) void adj_btcs_finish_kernel(
    const InstDesc* __restrict__ inst, const AdjTile* __restrict__ tiles, const double* __restrict__ u,
    const double* __restrict__ x, const double* __restrict__ X, double* __restrict__ lam,
    double* __restrict__ gslot) {
  __shared__ double red[kAdjThreads];
  const AdjTile t = tiles[blockIdx.x];
  const InstDesc d = inst[t.inst];
  const int n = t.n;
  const int j = t.start + static_cast<int>(threadIdx.x);
  const bool periodic = t.bc == kPeriodic;
  double g = 0.0;
  if (j < n) {
    double out = 0.0;
    if (periodic || (j > 0 && j < n - 1)) {
      const double* __restrict__ xs = x + t.off;
      const int first = periodic ? 0 : 1;
      const double mu = X[t.sys_off + (j - first)];
      const double xm = periodic ? xs[j == 0 ? n - 1 : j - 1] : (j == 1 ? d.a : xs[j - 1]);
      const double xp = periodic ? xs[j == n - 1 ? 0 : j + 1] : (j == n - 2 ? d.b : xs[j + 1]);
      const double xj = xs[j];
      const double G = u[t.off + j] >= 0.0 ? d.r * (xj - xm) : d.r * (xp - xj);
      out = (1.0 - G) * mu;
      g = -(mu * ((2.0 * xj - xm) - xp));
    }
    lam[t.off + j] = out;
  }
  const double tot = block_sum(g, red);
  if (threadIdx.x == 0) gslot[t.slot] = gslot[t.slot] + tot;
}

// grad_nu[i] = (sum of instance i's tile partials, in tile order) * dt/dx^2.
__global__ void adj_nu_kernel(const InstDesc* __restrict__ inst, const int32_t* __restrict__ slot_begin,
                              const double* __restrict__ gslot, double* __restrict__ grad_nu, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int k = slot_begin[i]; k < slot_begin[i + 1]; ++k) s = s + gslot[k];
  grad_nu[i] = s * inst[i].dtdx2;
}

// Dirichlet boundary nodes carry no gradient.
__global__ void zero_ends_kernel(const InstDesc* __restrict__ inst, double* __restrict__ g, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const InstDesc d = inst[i];
  if (d.bc == kDirichlet) {
    g[d.off] = 0.0;
    g[d.off + d.n - 1] = 0.0;
  }
}

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

int adjoint_tile_nodes() { return kAdjThreads; }

hipError_t launch_adj_explicit(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles, const double* u,
                               const double* lamp, double* lam, double* gslot) {
  if (n_tiles <= 0) return hipSuccess;
  adj_explicit_kernel<<<static_cast<unsigned>(n_tiles), kAdjThreads, 0, ctx->stream>>>(
      ctx->inst.as<InstDesc>(), tiles, u, lamp, lam, gslot);
  return hipGetLastError();
}

hipError_t launch_adj_btcs_assemble(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles,
                                    const double* u, const double* lamp, double* LA, double* LC, double* LD) {
  if (n_tiles <= 0) return hipSuccess;
  adj_btcs_assemble_kernel<<<static_cast<unsigned>(n_tiles), kAdjThreads, 0, ctx->stream>>>(
      ctx->inst.as<InstDesc>(), tiles, u, lamp, LA, LC, LD);
  return hipGetLastError();
}

hipError_t launch_adj_btcs_finish(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles,
                                  const double* u, const double* x, const double* X, double* lam,
                                  double* gslot) {
  if (n_tiles <= 0) return hipSuccess;
  adj_btcs_finish_kernel<<<static_cast<unsigned>(n_tiles), kAdjThreads, 0, ctx->stream>>>(
      ctx->inst.as<InstDesc>(), tiles, u, x, X, lam, gslot);
  return hipGetLastError();
}

hipError_t launch_adj_nu(const burgers_ctx* ctx, const int32_t* slot_begin, const double* gslot,
                         double* grad_nu) {
  const int count = static_cast<int>(ctx->count);
  adj_nu_kernel<<<(count + 255) / 256, 256, 0, ctx->stream>>>(ctx->inst.as<InstDesc>(), slot_begin, gslot,
                                                              grad_nu, count);
  return hipGetLastError();
}

hipError_t launch_zero_dirichlet_ends(const burgers_ctx* ctx, double* g) {
  const int count = static_cast<int>(ctx->count);
  zero_ends_kernel<<<(count + 255) / 256, 256, 0, ctx->stream>>>(ctx->inst.as<InstDesc>(), g, count);
  return hipGetLastError();
}

hipError_t launch_fill(const burgers_ctx* ctx, double* p, int64_t n, double v) {
  if (n <= 0) return hipSuccess;
  fill_kernel<<<static_cast<unsigned>((n + 255) / 256), 256, 0, ctx->stream>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace burgers
