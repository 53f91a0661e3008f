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
constexpr int kAdjLaneNodes = 4;                          // BTCS tiles: consecutive nodes per lane
constexpr int kAdjTile = kAdjThreads * kAdjLaneNodes;     // nodes of one BTCS adjoint tile (one dJ/dD slot)
// Explicit tiles: one 16-byte vector per lane (C5, 256 x 16384: 74.4 ms per gradient with two vectors
// per lane, 69.2 ms with one, 80.6 ms with four)
constexpr int kAdjExpNodes = 2;
constexpr int kAdjExpTile = kAdjThreads * kAdjExpNodes;

// Sum over the workgroup in a fixed order (a butterfly within each wave, lane 0's result, then the waves
// in order), so that the per-tile partials of dJ/dD are deterministic.  Valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = v + __shfl_xor(v, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double tot = red[0];
#pragma unroll
  for (int w = 1; w < kAdjThreads / 64; ++w) tot = tot + red[w];
  return tot;
}

// lam = (dE/du)^T lamp at state u; partial dJ/dD of the tile added to gslot[tile.slot].  Each lane takes
// kAdjExpNodes consecutive nodes, loaded as 16-byte vectors with one neighbour on each side.
__global__ __launch_bounds__(kAdjThreads) void adj_explicit_kernel(
    const InstDesc* __restrict__ inst, const AdjTile* __restrict__ tiles, const double* __restrict__ u,
    const double* __restrict__ lamp, double* __restrict__ lam, double* __restrict__ gslot) {
  constexpr int V = kAdjExpNodes;
  __shared__ double red[kAdjThreads / 64];
  const AdjTile t = tiles[blockIdx.x];
  const InstDesc d = inst[t.inst];
  const int n = t.n;
  const int j0 = t.start + V * static_cast<int>(threadIdx.x);
  const bool periodic = t.bc == kPeriodic;
  const double* __restrict__ y = u + t.off;
  const double* __restrict__ lp = lamp + t.off;
  const double r = d.r, D = d.D;
  double g = 0.0;
  if (j0 < n) {
    // Y[q], L[q]: state and lamp at node j0 - 1 + q (periodic neighbours wrap; positions outside a
    // Dirichlet grid are never used)
    double Y[V + 2], L[V + 2];
    if (j0 + V <= n) {
#pragma unroll
      for (int q = 0; q < V; q += 2) {
        const double2 yv = *reinterpret_cast<const double2*>(y + j0 + q);
        const double2 lv = *reinterpret_cast<const double2*>(lp + j0 + q);
        Y[q + 1] = yv.x; Y[q + 2] = yv.y;
        L[q + 1] = lv.x; L[q + 2] = lv.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const int j = j0 + q < n ? j0 + q : (periodic ? j0 + q - n : n - 1);
        Y[q + 1] = y[j];
        L[q + 1] = lp[j];
      }
    }
    const int jl = j0 > 0 ? j0 - 1 : (periodic ? n - 1 : 0);
    int jr = j0 + V;
    if (jr >= n) jr = periodic ? jr - n : n - 1;
    Y[0] = y[jl];
    L[0] = lp[jl];
    Y[V + 1] = y[jr];
    L[V + 1] = lp[jr];
    double out[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int j = j0 + q;
      double acc = 0.0;
      if (j < n && (periodic || (j > 0 && j < n - 1))) {
        const double uj = Y[q + 1];
        const double um = (!periodic && j == 1) ? d.a : Y[q];
        const double up = (!periodic && j == n - 2) ? d.b : Y[q + 2];
        // own update
        const double self = uj >= 0.0 ? ((1.0 - r * (uj - um)) - r * uj) - 2.0 * D
                                      : ((1.0 - r * (up - uj)) + r * uj) - 2.0 * D;
        acc = self * L[q + 1];
        g = g + L[q + 1] * ((up + um) - 2.0 * uj);
        // node j+1 reads u_j as its left neighbour
        if (periodic || j + 1 <= n - 2) {
          const double uk = Y[q + 2];
          acc = acc + (uk >= 0.0 ? r * uk + D : D) * L[q + 2];
        }
        // node j-1 reads u_j as its right neighbour
        if (periodic || j - 1 >= 1) {
          const double uk = Y[q];
          acc = acc + (uk >= 0.0 ? D : D - r * uk) * L[q];
        }
      }
      out[q] = acc;
    }
    double* __restrict__ dst = lam + t.off;
    if (j0 + V <= n) {
#pragma unroll
      for (int q = 0; q < V; q += 2) *reinterpret_cast<double2*>(dst + j0 + q) = double2{out[q], out[q + 1]};
    } else {
#pragma unroll
      for (int q = 0; q < V; ++q)
        if (j0 + q < n) dst[j0 + q] = out[q];
    }
  }
  const double tot = block_sum(g, red);
  if (threadIdx.x == 0) gslot[t.slot] = gslot[t.slot] + tot;
}

// Row k of A(y)^T, normalised by its diagonal, and the right-hand side lamp / d, for every unknown of
// the tile's instance; written at t.sys_off of the adjoint arrays.
__global__ __launch_bounds__(kAdjThreads) void adj_btcs_assemble_kernel(
    const InstDesc* __restrict__ inst, const AdjTile* __restrict__ tiles, const double* __restrict__ u,
    const double* __restrict__ lamp, double* __restrict__ LA, double* __restrict__ LC,
    double* __restrict__ LD, const int* __restrict__ only) {
  if (only && only[-1] == 0) return;          // no window of this step failed
  const AdjTile t = tiles[blockIdx.x];
  if (only && only[t.inst] == 0) return;      // this instance's windows held
  const InstDesc d = inst[t.inst];
  const int n = t.n;
  const bool periodic = t.bc == kPeriodic;
  const int first = periodic ? 0 : 1;
  const int m = periodic ? n : n - 2;
  for (int q = 0; q < kAdjLaneNodes; ++q) {
  const int node = t.start + static_cast<int>(threadIdx.x) + q * kAdjThreads;
  const int k = node - first;   // unknown index of this node
  if (node >= n || k < 0 || k >= m) continue;
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
}

// lam = (1 - G) mu and the tile's partial -mu . (L x); boundary nodes get zero.  With windows (n_win > 0),
// workgroup b first adds window b's partial (wpart) to the window's slot unless its instance was flagged,
// and only the flagged instances' tiles are finished here.
__global__ __launch_bounds__(kAdjThreads) void adj_btcs_finish_kernel(
    const InstDesc* __restrict__ inst, const AdjTile* __restrict__ tiles, const double* __restrict__ u,
    const double* __restrict__ x, const double* __restrict__ X, double* __restrict__ lam,
    double* __restrict__ gslot, const int* __restrict__ only, const WinDesc* __restrict__ wins, int64_t n_win,
    const int32_t* __restrict__ win_slot, const double* __restrict__ wpart) {
  __shared__ double red[kAdjThreads / 64];
  if (static_cast<int64_t>(blockIdx.x) < n_win && threadIdx.x == 0) {
    const int wi = wins[blockIdx.x].inst;
    if (only[wi] == 0) gslot[win_slot[blockIdx.x]] = gslot[win_slot[blockIdx.x]] + wpart[blockIdx.x];
  }
  if (only && only[-1] == 0) return;          // no window of this step failed
  const AdjTile t = tiles[blockIdx.x];
  if (only && only[t.inst] == 0) return;
  const InstDesc d = inst[t.inst];
  const int n = t.n;
  const bool periodic = t.bc == kPeriodic;
  double g = 0.0;
  for (int q = 0; q < kAdjLaneNodes; ++q) {
  const int j = t.start + static_cast<int>(threadIdx.x) + q * kAdjThreads;
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
      g = g - mu * ((2.0 * xj - xm) - xp);
    }
    lam[t.off + j] = out;
  }
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

int adjoint_tile_nodes(bool btcs) { return btcs ? kAdjTile : kAdjExpTile; }

hipError_t launch_adj_explicit(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles, const double* u,
                               const double* lamp, double* lam, double* gslot) {
  if (n_tiles <= 0) return hipSuccess;
  adj_explicit_kernel<<<static_cast<unsigned>(n_tiles), kAdjThreads, 0, ctx->stream>>>(
      ctx->inst.as<InstDesc>(), tiles, u, lamp, lam, gslot);
  return hipGetLastError();
}

hipError_t launch_adj_btcs_assemble(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles,
                                    const double* u, const double* lamp, double* LA, double* LC, double* LD,
                                    const int* only) {
  if (n_tiles <= 0) return hipSuccess;
  adj_btcs_assemble_kernel<<<static_cast<unsigned>(n_tiles), kAdjThreads, 0, ctx->stream>>>(
      ctx->inst.as<InstDesc>(), tiles, u, lamp, LA, LC, LD, only);
  return hipGetLastError();
}

hipError_t launch_adj_btcs_finish(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles,
                                  const double* u, const double* x, const double* X, double* lam,
                                  double* gslot, const int* only, const WinDesc* wins, int64_t n_win,
                                  const int32_t* win_slot, const double* wpart) {
  if (n_tiles <= 0) return hipSuccess;
  if (n_win > n_tiles) return hipErrorInvalidValue;   // every window's partial needs a workgroup
  adj_btcs_finish_kernel<<<static_cast<unsigned>(n_tiles), kAdjThreads, 0, ctx->stream>>>(
      ctx->inst.as<InstDesc>(), tiles, u, x, X, lam, gslot, only, wins, n_win, win_slot, wpart);
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
