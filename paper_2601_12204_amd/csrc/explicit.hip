// Explicit forward-Euler upwind/central step (Sec. 2.3, eq. 21) for gfx950.
//
// One step is a 3-point stencil per node; it moves 2 words per node-step (read u^n, write u^{n+1}) and
// does about a dozen flops, far below the machine balance, so the streaming kernel is bound by HBM:
// every workgroup streams one tile of 256 x (16 bytes / word) nodes with 16-byte vector loads and
// stores, and the two neighbours a lane needs beyond its own vector come from the same cache lines.
//
// The update is evaluated in exactly this association, with contraction disabled, so that it rounds
// like a plain scalar evaluation of the formula:
//   c = r u_i;  lap = (u_{i+1} + u_{i-1}) - 2 u_i
//   u_i' = ((u_i - max(c,0) (u_i - u_{i-1})) - min(c,0) (u_{i+1} - u_i)) + D lap
// The upwind side follows the sign of u_i (backward difference for u_i >= 0, eq. 3; forward for
// u_i < 0, as the text after eq. 3 prescribes).  Diffusion uses the central difference of eq. 4.
#include "internal.hpp"
#include "stencil.hpp"

#pragma clang fp contract(off)

namespace burgers {
namespace {

constexpr int kStreamThreads = 256;

template <typename T> struct Vec;
template <> struct Vec<double> { using type = double2; static constexpr int n = 2; };
template <> struct Vec<float> { using type = float4; static constexpr int n = 4; };

template <typename T>
__global__ __launch_bounds__(kStreamThreads) void explicit_stream_kernel(
    const InstDesc* __restrict__ inst, const Tile* __restrict__ tiles, const T* __restrict__ u,
    T* __restrict__ out) {
  constexpr int V = Vec<T>::n;
  using VT = typename Vec<T>::type;
  const Tile t = tiles[blockIdx.x];
  const InstDesc d = inst[t.inst];
  const int n = d.n;
  const int i0 = t.start + static_cast<int>(threadIdx.x) * V;
  if (i0 >= n) return;
  const T* __restrict__ src = u + d.off;
  T* __restrict__ dst = out + d.off;
  const T r = static_cast<T>(d.r), D = static_cast<T>(d.D);
  const T a = static_cast<T>(d.a), b = static_cast<T>(d.b);
  const bool periodic = d.bc == kPeriodic;

  // Instance starts are aligned to 64 elements and i0 is a multiple of V, so this vector lies inside
  // the instance's padded extent even when it runs past node n-1.
  const VT vv = *reinterpret_cast<const VT*>(src + i0);
  T v[V];
  __builtin_memcpy(v, &vv, sizeof(VT));
  const T left = i0 > 0 ? src[i0 - 1] : (periodic ? src[n - 1] : a);
  const T right = i0 + V < n ? src[i0 + V] : (periodic ? src[0] : b);
  const T wrap_right = periodic ? src[0] : b;   // neighbour of node n-1

  T o[V];
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const int j = i0 + k;
    T um = k == 0 ? left : v[k - 1];
    T up = k == V - 1 ? right : v[k + 1];
    if (j == n - 1) up = wrap_right;
    if (!periodic) {
      if (j == 1) um = a;
      if (j == n - 2) up = b;
    }
    T res = upwind_central(v[k], um, up, r, D);
    if (!periodic) {
      if (j == 0) res = a;
      if (j == n - 1) res = b;
    }
    o[k] = res;
  }
  if (i0 + V <= n) {
    VT ov;
    __builtin_memcpy(&ov, o, sizeof(VT));
    *reinterpret_cast<VT*>(dst + i0) = ov;
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k)
      if (i0 + k < n) dst[i0 + k] = o[k];
  }
}

}  // namespace

int explicit_tile_nodes(burgers_dtype dt) {
  return kStreamThreads * (dt == BURGERS_F64 ? Vec<double>::n : Vec<float>::n);
}

hipError_t launch_explicit_stream(const burgers_ctx* ctx, const Tile* tiles, int64_t n_tiles,
                                  const void* u, void* out) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(n_tiles)), block(kStreamThreads);
  if (ctx->dtype == BURGERS_F64) {
    explicit_stream_kernel<double><<<grid, block, 0, ctx->stream>>>(
        ctx->inst.as<InstDesc>(), tiles, static_cast<const double*>(u), static_cast<double*>(out));
  } else {
    explicit_stream_kernel<float><<<grid, block, 0, ctx->stream>>>(
        ctx->inst.as<InstDesc>(), tiles, static_cast<const float*>(u), static_cast<float*>(out));
  }
  return hipGetLastError();
}

}  // namespace burgers
