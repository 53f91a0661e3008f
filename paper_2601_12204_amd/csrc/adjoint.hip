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
// dJ/dD is accumulated per tile of nodes in a fixed order (for the explicit instances per tile and step,
// whatever the grouping of steps into launches), so the sums are deterministic.
#include "internal.hpp"
#include "stencil.hpp"

#pragma clang fp contract(off)

namespace burgers {
namespace {

constexpr int kAdjThreads = 256;
constexpr int kAdjLaneNodes = 4;                          // BTCS tiles: consecutive nodes per lane
constexpr int kAdjTile = kAdjThreads * kAdjLaneNodes;     // nodes of one BTCS adjoint tile (one dJ/dD slot)

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

// ---- Explicit reverse steps, blocked ----------------------------------------------------------------
// lam^k = (dE/du at u^k)^T lam^(k+1) is a 3-point gather stencil whose coefficients come from u^k alone.
// A workgroup of 256 lanes holds lam over a window of up to 4096 nodes (16 consecutive nodes per lane) in
// registers for a run of reverse steps: each step reads u^k of the window from HBM (coalesced, passed to
// the lanes' chunks through a region of LDS private to each wave), exchanges the chunks' end values of u
// and lam through LDS, and updates lam in place.  lam is read once and written once per launch.  Windows
// of longer instances keep their middle nodes and carry kAdjHalo nodes on either side, recomputed
// redundantly: an error at a window edge travels one node per step, so a launch takes at most kAdjHalo
// steps.
//
// dJ/dD, the sum over nodes and steps of lam^(k+1)_j (u_{j+1} + u_{j-1} - 2 u_j), is accumulated per
// tile of kAdjSumTile nodes of an instance: per step, each lane sums its kept nodes in node order, the 16
// lanes of a tile combine by a butterfly, and the tile's first lane adds the result to the tile's running
// sum (loaded from its slot at launch start, stored at the end).  Tiles are aligned to 16-lane groups in
// every window, so each (tile, step) partial is formed alike whichever window and launch computes it:
// the gradient does not depend on how the steps are grouped into launches (the checkpoint interval).
constexpr int kAdjWinLanes = 256;
constexpr int kAdjWinChunk = 16;
constexpr int kAdjWinRegion = 32 * (kAdjWinChunk + 1);   // a half-wave's chunks, padded by one per chunk
static_assert(kAdjWinLanes * kAdjWinChunk == kAdjWinNodes, "window capacity");
static_assert(kAdjSumTile == 16 * kAdjWinChunk, "a tile is 16 lanes' chunks");

__device__ __forceinline__ int apad(int i) { return i + (i >> 4); }

// A lane index that the compiler cannot treat as known, so that the addresses built on it are formed
// where they are used rather than kept live across the step loop.
__device__ __forceinline__ int fresh_lane() {
  int v = static_cast<int>(threadIdx.x);
  asm volatile("" : "+v"(v));
  return v;
}

// Wave-private LDS exchanges are ordered by the wave's own in-order LDS accesses; the fences keep the
// compiler from moving them.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Window nodes of src (the instance's first node) for the lane's chunk [16 t, 16 t + 16), in two steps so
// that the loads can be issued long before their values are needed: window_fetch loads, for each of the
// two halves of the wave, the 512 consecutive window nodes of that half's chunks (64 per instruction,
// coalesced) into v; window_spread passes them to the lanes' chunks through the wave's region of LDS.
__device__ __forceinline__ void window_fetch(const double* __restrict__ src, const AdjWindow& w, int n,
                                             double (&v)[2 * 8]) {
  const int lt = fresh_lane();
  const int lane = lt & 63, wave = lt >> 6;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int w0 = kAdjWinChunk * (64 * wave + 32 * h);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = w0 + lane + 64 * i;
      int g = w.first + k;
      if (g >= n) g -= n;
      v[8 * h + i] = k < w.width ? src[g] : 0.0;
    }
  }
}

__device__ __forceinline__ void window_spread(const double (&v)[2 * 8], double* lds, double (&out)[kAdjWinChunk]) {
  const int lt = fresh_lane();
  const int lane = lt & 63, wave = lt >> 6;
  double* region = lds + wave * kAdjWinRegion;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int i = 0; i < 8; ++i) region[apad(lane + 64 * i)] = v[8 * h + i];
    wave_sync();
    if ((lane >> 5) == h) {
#pragma unroll
      for (int j = 0; j < kAdjWinChunk; ++j) out[j] = region[apad(kAdjWinChunk * (lane & 31) + j)];
    }
    wave_sync();
  }
}

// The lane's chunk to the window's kept nodes of dst (the instance's first node), the way back.
__device__ __forceinline__ void window_store(const double (&x)[kAdjWinChunk], const AdjWindow& w, int n,
                                             double* lds, double* __restrict__ dst) {
  const int lt = fresh_lane();
  const int lane = lt & 63, wave = lt >> 6;
  double* region = lds + wave * kAdjWinRegion;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if ((lane >> 5) == h) {
#pragma unroll
      for (int j = 0; j < kAdjWinChunk; ++j) region[apad(kAdjWinChunk * (lane & 31) + j)] = x[j];
    }
    wave_sync();
    const int w0 = kAdjWinChunk * (64 * wave + 32 * h);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int q = lane + 64 * i, k = w0 + q;
      const double v = region[apad(q)];
      if (k >= w.lo && k < w.lo + w.count) {
        int g = w.first + k;
        if (g >= n) g -= n;
        dst[g] = v;
      }
    }
    wave_sync();
  }
}

// (Four workgroups of 256 lanes per CU, 128 registers, the next step's loads in flight: C5, 256 x 16384,
// 36.6 ms per gradient, against 41.5 ms with windows of 8192 nodes on 512 lanes, two per CU, whose halos
// are a smaller share; 54.4 ms with 131 registers and one 512-lane workgroup per CU.)
// Reverse steps k = k_hi - 1 down to k_lo of a segment: u^k at u0 for k = 0, else at useg + (k - 1) ustride
// (binary64 states); lam^(k_hi) from lamp, lam^(k_lo) to lam (the window's kept nodes).
// PERIODIC: every window of the launch belongs to a periodic instance (no boundary cases are compiled);
// otherwise every window belongs to a Dirichlet one.
template <bool PERIODIC>
__global__ __launch_bounds__(kAdjWinLanes, 4) void adj_explicit_block_kernel(
    const InstDesc* __restrict__ inst, const AdjWindow* __restrict__ wins, const double* __restrict__ u0,
    const double* __restrict__ useg, int64_t ustride, int k_lo, int k_hi, const double* __restrict__ lamp,
    double* __restrict__ lam, double* __restrict__ gslot) {
  constexpr int M = kAdjWinChunk, NT = kAdjWinLanes;
  __shared__ double ends[2][4][NT];            // per step parity: u first, u last, lam first, lam last
  __shared__ double region[(NT / 64) * kAdjWinRegion];
  const AdjWindow w = wins[blockIdx.x];
  const InstDesc d = inst[w.inst];
  const int n = d.n;
  constexpr bool periodic = PERIODIC;
  const double r = d.r, D = d.D;
  const int t = threadIdx.x;
  const int P = (w.width + M - 1) / M;         // lanes holding nodes; the last holds mlast
  const int mlast = w.width - M * (P - 1);
  const int m = t < P ? (t == P - 1 ? mlast : M) : 0;
  // the lane's kept nodes are a prefix of its chunk (w.lo is a multiple of M): the first kc
  const int kc = M * t >= w.lo ? min(M, max(0, w.lo + w.count - M * t)) : 0;
  // the lane's tile (16-lane groups start on tile boundaries) and its running dJ/dD sum
  const bool tile_lane = (t & 15) == 0 && M * t >= w.lo && M * t < w.lo + w.count;
  const int slot = w.slot0 + (M * t - w.lo) / kAdjSumTile;
  double tile_sum = tile_lane ? gslot[slot] : 0.0;
  auto state = [&](int k) { return (k == 0 ? u0 : useg + static_cast<int64_t>(k - 1) * ustride) + d.off; };
  double L[M], U[M], V[2 * 8];
  window_fetch(lamp + d.off, w, n, V);
  window_spread(V, region, L);
  window_fetch(state(k_hi - 1), w, n, V);
  for (int k = k_hi - 1; k >= k_lo; --k) {
    window_spread(V, region, U);
    const int b = k & 1;
    if (t < P) {
      double ul = U[M - 1], ll = L[M - 1];
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (j == m - 1) {
          ul = U[j];
          ll = L[j];
        }
      ends[b][0][t] = U[0];
      ends[b][1][t] = ul;
      ends[b][2][t] = L[0];
      ends[b][3][t] = ll;
    }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    double g = 0.0;
    // neighbours beyond the window's ends wrap around it: exact for a whole periodic instance, and only
    // the halo is affected otherwise (the indices are formed here, not kept live across the step)
    const int tf = fresh_lane();
    const int tl = tf > 0 ? tf - 1 : P - 1, tr = tf < P - 1 ? tf + 1 : 0;
    const double uL = ends[b][1][tl], uR = ends[b][0][tr];
    const double lL = ends[b][3][tl], lR = ends[b][2][tr];
    // the next step's state is in flight during this step's update: issued after every read that the
    // update waits for, since a wait on the in-order memory counter would also wait for these loads
    if (k > k_lo) window_fetch(state(k - 1), w, n, V);
    if (t < P) {
      double lprev = lL;                        // lam^(k+1) of the node before, kept before it is overwritten
#pragma unroll
      for (int j = 0; j < M; ++j) {
        if (j < m) {
          int jn = w.first + M * t + j;         // instance node (only a Dirichlet window needs it)
          if (jn >= n) jn -= n;
          const double uj = U[j];
          const double uprev = j == 0 ? uL : U[j > 0 ? j - 1 : 0];
          const double unext = j + 1 < m ? U[j + 1 < M ? j + 1 : j] : uR;
          const double lj = L[j];
          const double lnext = j + 1 < m ? L[j + 1 < M ? j + 1 : j] : lR;
          double acc = 0.0;
          if (periodic || (jn > 0 && jn < n - 1)) {
            const double um = (!periodic && jn == 1) ? d.a : uprev;
            const double up = (!periodic && jn == n - 2) ? d.b : unext;
            // own update
            const double self = uj >= 0.0 ? ((1.0 - r * (uj - um)) - r * uj) - 2.0 * D
                                          : ((1.0 - r * (up - uj)) + r * uj) - 2.0 * D;
            acc = self * lj;
            if (j < kc) g = g + lj * ((up + um) - 2.0 * uj);
            // node j+1 reads u_j as its left neighbour
            if (periodic || jn + 1 <= n - 2) acc = acc + (unext >= 0.0 ? r * unext + D : D) * lnext;
            // node j-1 reads u_j as its right neighbour
            if (periodic || jn - 1 >= 1) acc = acc + (uprev >= 0.0 ? D : D - r * uprev) * lprev;
          }
          lprev = lj;
          L[j] = acc;
        }
      }
    }
    // the tile's partial for this step: a butterfly over its 16 lanes, taken from its first lane
#pragma unroll
    for (int s = 8; s >= 1; s >>= 1) g = g + __shfl_xor(g, s, 64);
    if (tile_lane) tile_sum = tile_sum + g;
  }
  window_store(L, w, n, region, lam + d.off);
  if (tile_lane) gslot[slot] = tile_sum;
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

int adjoint_tile_nodes() { return kAdjTile; }

hipError_t launch_adj_explicit_block(const burgers_ctx* ctx, const AdjWindow* wins, int64_t n_wins, int64_t n_periodic,
                                     const double* u0, const double* useg, int64_t ustride, int k_lo, int k_hi,
                                     const double* lamp, double* lam, double* gslot) {
  if (n_wins <= 0 || k_hi <= k_lo) return hipSuccess;
  if (n_periodic > 0)
    adj_explicit_block_kernel<true><<<static_cast<unsigned>(n_periodic), kAdjWinLanes, 0, ctx->stream>>>(
        ctx->inst.as<InstDesc>(), wins, u0, useg, ustride, k_lo, k_hi, lamp, lam, gslot);
  if (n_wins > n_periodic)
    adj_explicit_block_kernel<false><<<static_cast<unsigned>(n_wins - n_periodic), kAdjWinLanes, 0, ctx->stream>>>(
        ctx->inst.as<InstDesc>(), wins + n_periodic, u0, useg, ustride, k_lo, k_hi, lamp, lam, gslot);
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
