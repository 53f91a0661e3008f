// Explicit forward-Euler upwind/central step (Sec. 2.3, eq. 21) for gfx950.
//
// The update of one node is the 3-point stencil
//   c = r u_i;  u_i' = ((u_i - max(c,0) (u_i - u_{i-1})) - min(c,0) (u_{i+1} - u_i)) + D ((u_{i+1} + u_{i-1}) - 2 u_i)
// The upwind side follows the sign of u_i (backward difference for u_i >= 0, eq. 3; forward for
// u_i < 0, as the text after eq. 3 prescribes).  Diffusion uses the central difference of eq. 4.
// Every kernel evaluates it through upwind_central (stencil.hpp): binary64 as the equivalent fused
// combination u + alpha (u_{i+1} - u_i) - beta (u_i - u_{i-1}), binary32 in exactly the association
// above with contraction disabled.
//
// Two kernels:
//  * explicit_stream_kernel: one step per pass over HBM.  It moves 2 words per node-step and does 12
//    flops, far below the machine balance, so it is bound by HBM: each workgroup streams one tile of
//    256 lanes x 2 x 16 bytes with vector loads and stores; a tile's descriptor carries everything
//    needed to address it, so the vector loads issue after a single scalar load.
//  * explicit_block_kernel: temporal blocking.  A workgroup of up to 512 lanes holds a window of up to
//    8192 nodes in registers (16 consecutive nodes per lane, in two arrays that alternate as old and new
//    state, so no value is copied between registers), exchanges only the chunk end values through LDS
//    each step (double buffered, one barrier per step) and advances many steps per pass over HBM.  The
//    window is loaded and stored through LDS so that HBM sees coalesced accesses.  A whole instance
//    that fits is advanced for all its steps in one launch with exact boundaries, in the narrowest of
//    64, 128, 256 or 512 lanes that holds it; longer grids are cut into windows with a halo of T nodes
//    per side that are recomputed redundantly, so that after T steps the window's interior is exact.
//    Every node goes through the same arithmetic as in the streaming kernel, so both kernels give
//    bitwise identical results.
#include "internal.hpp"
#include "stencil.hpp"

#pragma clang fp contract(off)

namespace burgers {
namespace {

constexpr int kStreamThreads = 256;
constexpr int kBlockThreads = 512;
constexpr int kBlockChunk = 16;

template <typename T> struct Vec;
template <> struct Vec<double> {
  using type = double2;
  typedef double ext __attribute__((ext_vector_type(2)));
  static constexpr int n = 2;
};
template <> struct Vec<float> {
  using type = float4;
  typedef float ext __attribute__((ext_vector_type(4)));
  static constexpr int n = 4;
};

// 16-byte vectors per lane of the streaming kernels: two (tiles of 8 KB), which halves the launch's
// workgroups and doubles the loads each lane has in flight (C2 batch: binary64 88.8 -> 86.4 us per step,
// binary32 48.4 -> 45.0 us; four per lane are slower again).
template <typename T>
constexpr int kStreamVecs = 2;

template <typename T>
__global__ __launch_bounds__(kStreamThreads) void explicit_stream_kernel(
    const InstDesc* __restrict__ inst, const Tile* __restrict__ tiles, const T* __restrict__ u,
    T* __restrict__ out) {
  constexpr int V = Vec<T>::n, K = kStreamVecs<T>;
  using VT = typename Vec<T>::type;
  const Tile t = tiles[blockIdx.x];
  const int n = t.n;
  const T* __restrict__ src = u + t.off;
  T* __restrict__ dst = out + t.off;
  const bool periodic = t.bc == kPeriodic;

  // Lane vectors q = 0..K-1 start at t.start + (q kStreamThreads + lane) V (each wave instruction
  // covers consecutive vectors).  A vector past the instance's end repeats the last vector's work and
  // stores the same values to the same nodes as the lane that owns it, so no lane branches before its
  // loads.  Instance starts are aligned to 64 elements and i0 is a multiple of V, so every vector lies
  // inside the instance's padded extent even when it runs past node n-1.  The neighbour loads take
  // selected addresses (wrapping periodically) rather than branches, so every lane issues all its loads
  // right after the tile's scalar loads; a Dirichlet end then replaces the wrapped value by its boundary
  // value.
  int i0[K];
  VT vv[K];
  T lraw[K], rraw[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    i0[q] = min(t.start + (q * kStreamThreads + static_cast<int>(threadIdx.x)) * V, (n - 1) / V * V);
    vv[q] = *reinterpret_cast<const VT*>(src + i0[q]);
    lraw[q] = src[i0[q] > 0 ? i0[q] - 1 : n - 1];
    rraw[q] = src[i0[q] + V < n ? i0[q] + V : 0];
  }
  // (keeps the instance's scalar load, and its wait, behind every vector load)
  __builtin_amdgcn_sched_barrier(0);
  const InstDesc d = inst[t.inst];
  const T r = static_cast<T>(d.r), D = static_cast<T>(d.D);
  const T a = static_cast<T>(d.a), b = static_cast<T>(d.b);
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int j0 = i0[q];
    T v[V];
    __builtin_memcpy(v, &vv[q], sizeof(VT));
    const T left = periodic || j0 > 0 ? lraw[q] : a;
    // the value beyond node n-1 (node 0, or b); only the lane whose vector reaches node n-1 uses it
    const T right = periodic || j0 + V < n ? rraw[q] : b;
    T o[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const int j = j0 + k;
      T um = k == 0 ? left : v[k - 1];
      T up = k == V - 1 ? right : v[k + 1];
      if (j == n - 1) up = right;
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
    if (j0 + V <= n) {
      // The new state is not read again by this launch: stream it past the caches.
      typename Vec<T>::ext ov;
      __builtin_memcpy(&ov, o, sizeof(ov));
      __builtin_nontemporal_store(ov, reinterpret_cast<typename Vec<T>::ext*>(dst + j0));
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k)
        if (j0 + k < n) dst[j0 + k] = o[k];
    }
  }
}

// LDS staging of window I/O: half the lanes' chunks at a time (at most 4096 nodes), padded by one element
// every 16 nodes so that lanes reading their 16-node chunks (a stride of 17 elements) hit distinct banks.
template <int NT>
constexpr int stage_nodes() { return NT * kBlockChunk / 2; }
__device__ __forceinline__ int spad(int i) { return i + (i >> 4); }

// One step of a lane's chunk: out[j] from in[j-1], in[j], in[j+1], with the neighbours' end values
// `left` and `right`; fixed nodes (a Dirichlet end, a window edge) keep their value: they run the same
// update with zero coefficients, which returns the node's value unchanged, so nothing branches.
//
// EXACT (every chunk full): the chunk's two end nodes take their own coefficients (r0, D0) and
// (r1, D1), zero at a fixed node, and the interior nodes, which need no neighbour value, come first,
// so that they run while `left` and `right` are still in flight from LDS.
//
// Otherwise every lane holds a full chunk of M nodes except the last, which holds ML (the same for the
// whole workgroup, and a compile-time constant here), and every lane runs the same code.  Node ML - 1
// is the last lane's last real node: its right neighbour is `right` there and in[ML] in the other
// lanes (one select), and it takes (r1, D1), zero only where it is a fixed node; the last lane's slots
// past ML - 1 are computed from finite values and never used.  With ML = 1, node 0 is both a first and
// a last node and takes (rE, DE), zero where either end is fixed.
template <typename T, bool EXACT, int ML>
__device__ __forceinline__ void chunk_step(const T (&in)[kBlockChunk], T (&out)[kBlockChunk], T left, T right,
                                           T r, T D, T r0, T D0, T r1, T D1, bool is_last, T rE, T DE) {
  constexpr int M = kBlockChunk;
  if constexpr (EXACT) {
#pragma unroll
    for (int j = 1; j < M - 1; ++j) out[j] = upwind_central(in[j], in[j - 1], in[j + 1], r, D);
    out[0] = upwind_central(in[0], left, in[1], r0, D0);
    out[M - 1] = upwind_central(in[M - 1], in[M - 2], right, r1, D1);
  } else {
    static_assert(ML >= 1 && ML <= M, "ragged chunks need the last lane's count at compile time");
#pragma unroll
    for (int j = 1; j < M; ++j)
      if (j != ML - 1) out[j] = upwind_central(in[j], in[j - 1], j + 1 < M ? in[j + 1 < M ? j + 1 : j] : right, r, D);
    constexpr int kNext = ML < M ? ML : M - 1;   // in[ML] exists only for ML < M
    const T up = ML < M ? (is_last ? right : in[kNext]) : right;
    if constexpr (ML == 1) {
      out[0] = upwind_central(in[0], left, up, rE, DE);
    } else {
      out[0] = upwind_central(in[0], left, in[1], r0, D0);
      out[ML - 1] = upwind_central(in[ML - 1], in[ML - 2], up, r1, D1);
    }
  }
}


// One RK4 stage of a lane's chunk (Sec. 2.7.1, eq. 22): K = increment of the stage input `in` (with
// the neighbours' end values `left`, `right`; fixed nodes have K = 0), then by stage
//   1: acc = K,             out = v + K/2
//   2: acc = acc + 2K,      out = v + K/2
//   3: acc = acc + 2K,      out = v + K
//   4: v = v + (acc + K)/6  (out unused)
// `in` and `out` may be the same array: node j reads in[j-1] from a register kept before it is
// overwritten.
template <typename T, int STAGE>
__device__ __forceinline__ void rk4_apply(T (&v)[kBlockChunk], T (&out)[kBlockChunk], T (&acc)[kBlockChunk], int j,
                                          T K) {
  if constexpr (STAGE == 1) {
    acc[j] = K;
    out[j] = v[j] + T(0.5) * K;
  } else if constexpr (STAGE == 2) {
    acc[j] = fma_exact(T(2), K, acc[j]);
    out[j] = v[j] + T(0.5) * K;
  } else if constexpr (STAGE == 3) {
    acc[j] = fma_exact(T(2), K, acc[j]);
    out[j] = v[j] + K;
  } else {
    v[j] = v[j] + (acc[j] + K) / T(6);
  }
}

// EXACT (every chunk full): as in chunk_step, the two end nodes take their own coefficients (zero at a
// fixed node, where K is then a zero) and come after the interior nodes; the four inputs the end nodes
// read are kept first, since `out` may overwrite `in`.
//
// Otherwise (ML, the last lane's count, a compile-time constant) the coefficients and the right
// neighbour of each node are chosen as in chunk_step, in one ascending pass that keeps in[j-1] in a
// register before out[j] may overwrite it.
template <typename T, bool EXACT, int STAGE, int ML>
__device__ __forceinline__ void rk4_stage(T (&v)[kBlockChunk], const T (&in)[kBlockChunk], T (&out)[kBlockChunk],
                                          T (&acc)[kBlockChunk], T left, T right, T r, T D, T r0, T D0, T r1,
                                          T D1, bool is_last, T rE, T DE) {
  constexpr int M = kBlockChunk;
  if constexpr (EXACT) {
    const T i0 = in[0], i1 = in[1], i2 = in[M - 2], i3 = in[M - 1];
    T prev = i0;
#pragma unroll
    for (int j = 1; j < M - 1; ++j) {
      const T cur = in[j];
      const T K = rk4_increment(cur, prev, in[j + 1], r, D);
      prev = cur;
      rk4_apply<T, STAGE>(v, out, acc, j, K);
    }
    rk4_apply<T, STAGE>(v, out, acc, 0, rk4_increment(i0, left, i1, r0, D0));
    rk4_apply<T, STAGE>(v, out, acc, M - 1, rk4_increment(i3, i2, right, r1, D1));
  } else {
    static_assert(ML >= 1 && ML <= M, "ragged chunks need the last lane's count at compile time");
    T prev = left;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const T next = j + 1 < M ? in[j + 1 < M ? j + 1 : j] : right;
      const T up = (j == ML - 1 && ML < M) ? (is_last ? right : next) : next;
      const T rr = j == 0 ? (ML == 1 ? rE : r0) : (j == ML - 1 ? r1 : r);
      const T dd = j == 0 ? (ML == 1 ? DE : D0) : (j == ML - 1 ? D1 : D);
      const T cur = in[j];
      const T K = rk4_increment(cur, prev, up, rr, dd);
      prev = cur;
      rk4_apply<T, STAGE>(v, out, acc, j, K);
    }
  }
}

// Publish a lane's chunk end values in exchange buffer `buf`, wait, and read the neighbours' ends.
// LdsOnly: the barrier waits for this wave's LDS accesses only, not for its stores to HBM, which then
// stay in flight across the step (the recording kernel's states).
template <typename T, bool EXACT, int NT, int ML = 0, bool LdsOnly = false>
__device__ __forceinline__ void exchange_ends(const T (&x)[kBlockChunk], int buf, int t, int P, int mlast,
                                              bool active, T (*s_first)[NT], T (*s_last)[NT],
                                              T& left, T& right) {
  constexpr int M = kBlockChunk;
  if (active) {
    s_first[buf][t] = x[0];
    T last = x[M - 1];
    if constexpr (!EXACT && ML > 0) {
      if (t == P - 1) last = x[ML - 1];
    } else if (!EXACT) {   // the window's last lane holds mlast nodes (uniform index, one select)
      T tail = x[M - 1];
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (j == mlast - 1) tail = x[j];
      if (t == P - 1) last = tail;
    }
    s_last[buf][t] = last;
  }
  if constexpr (LdsOnly) asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else __syncthreads();
  if (active) {
    left = t > 0 ? s_last[buf][t - 1] : s_last[buf][P - 1];
    right = t < P - 1 ? s_first[buf][t + 1] : s_first[buf][0];
  }
}

// Stores one step's state of the window's output nodes [bt.lo, bt.lo + bt.count) at `rec` (the
// instance's first node).  Each wave passes its lanes' chunks through a region of the staging buffer of
// its own, half the wave at a time (32 chunks of 16 nodes, padded like the staging), and stores them as
// 64 consecutive nodes per instruction.  The region is private to the wave, so no workgroup barrier is
// needed; a wave's LDS accesses are performed in order, which the wavefront-scope fences keep the
// compiler from reordering.
// (The lane index passes through an empty asm statement at every step, so that no address of these
// stores is formed once and kept live across the step loop.)
template <typename T, int NT>
__device__ __forceinline__ void record_window(const T (&x)[kBlockChunk], T* stage, const BlockTile& bt, int n,
                                              T* __restrict__ rec) {
  constexpr int M = kBlockChunk, kHalf = 32, kRegion = kHalf * (M + 1);
  static_assert((NT / 64) * kRegion <= stage_nodes<NT>() + stage_nodes<NT>() / 16 + 1,
                "every wave's region must fit in the staging buffer");
  int lt = static_cast<int>(threadIdx.x);
  asm volatile("" : "+v"(lt));
  const int lane = lt & 63, wave = lt >> 6;
  T* region = stage + wave * kRegion;
  const int lo = bt.lo, hi = bt.lo + bt.count;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if ((lane >> 5) == h) {
#pragma unroll
      for (int j = 0; j < M; ++j) region[spad(M * (lane & 31) + j)] = x[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int w0 = M * (64 * wave + kHalf * h);   // window node of the half-wave's first slot
#pragma unroll
    for (int i = 0; i < kHalf * M / 64; ++i) {
      const int q = lane + 64 * i;
      const T v = region[spad(q)];
      const int w = w0 + q;
      if (w >= lo && w < hi) {
        int g = bt.first + w;
        if (g >= n) g -= n;
        rec[g] = v;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Temporal-blocking body over NT lanes.  EXACT: the window has exactly NT * kBlockChunk nodes, so every lane
// holds a full chunk and the guards below fold away.
// t: the lane's index among the NT lanes that take the window (the workgroup's lane, or its lane within
// its sub-group when several windows share a workgroup).  Every call executes the same sequence of
// workgroup barriers for a given `steps`, whatever the window (an empty one included).
// REC (forward Euler, t the workgroup's lane): instead of the final state, the state after each step k
// (1 <= k <= steps) is stored at rec + (k - 1) rstride (the instance's first node), so that a segment of
// states is computed in one pass over HBM that writes each of them once.
template <typename T, bool EXACT, bool RK4, int NT, int ML = 0, bool REC = false>
__device__ __forceinline__ void block_body(const BlockTile& bt, const InstDesc& d, const T* __restrict__ src,
                                           T* __restrict__ dst, int steps, T* stage,
                                           T (*s_first)[NT], T (*s_last)[NT], int t, T* __restrict__ rec = nullptr,
                                           int64_t rstride = 0) {
  static_assert(!(REC && RK4), "recording is for forward Euler");
  constexpr int M = kBlockChunk;
  const T r = static_cast<T>(d.r), D = static_cast<T>(d.D);
  const int n = d.n;
  const bool periodic = d.bc == kPeriodic;
  const int W = bt.width;                       // window nodes
  // lane t holds nodes [M t, M t + m): full chunks, except that the last of the P lanes holds mlast
  const int P = EXACT ? NT : (W + M - 1) / M;
  const int mlast = EXACT ? M : W - M * (P - 1);
  const bool active = t < P;
  const int s = M * t;
  const int m = !active ? 0 : (t == P - 1 ? mlast : M);
  const int half = P / 2;                       // lanes [0, half) and [half, P) are staged in turn
  T v[M];
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = T(0);
  // window node w is instance node (bt.first + w) mod n; the window wraps only for periodic instances
  for (int h = 0; h < 2; ++h) {
    const int r0 = h == 0 ? 0 : M * half;
    const int r1 = h == 0 ? M * half : W;
    for (int w = r0 + t; w < r1; w += NT) {
      int g = bt.first + w;
      if (g >= n) g -= n;
      stage[spad(w - r0)] = src[g];
    }
    __syncthreads();
    if (active && (h == 0) == (t < half)) {
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (EXACT || j < m) v[j] = stage[spad(s + j - r0)];
    }
    __syncthreads();
  }
  // Window ends that are not periodic neighbours are held fixed: at a Dirichlet boundary they carry
  // a or b (and node 1 then reads a exactly as the streaming kernel does); at an interior window edge
  // their stale value only corrupts nodes within `steps` of the edge, which lie in the halo.
  const bool wraps = bt.wrap != 0;
  const bool fix_first = active && t == 0 && !wraps;
  const bool fix_last = active && t == P - 1 && !wraps;
  if (!periodic && active) {
    if (bt.first + s == 0) v[0] = static_cast<T>(d.a);
#pragma unroll
    for (int j = 0; j < M; ++j)
      if (j == m - 1 && bt.first + s + j == n - 1) v[j] = static_cast<T>(d.b);
  }

  T w[M];
  T left = T(0), right = T(0);
  // a full chunk's end nodes: zero coefficients where the node is held fixed (see chunk_step)
  const T r0 = fix_first ? T(0) : r, D0 = fix_first ? T(0) : D;
  const T r1 = fix_last ? T(0) : r, D1 = fix_last ? T(0) : D;
  const bool fix_either = fix_first || fix_last;
  const T rE = fix_either ? T(0) : r, DE = fix_either ? T(0) : D;
  const bool is_last = t == P - 1;
  if constexpr (RK4) {
    // four stages per step, each after an exchange of the stage's end values (buffers alternate)
    T acc[M];
    for (int step = 0; step < steps; ++step) {
      exchange_ends<T, EXACT, NT, ML>(v, 0, t, P, mlast, active, s_first, s_last, left, right);
      if (active) rk4_stage<T, EXACT, 1, ML>(v, v, w, acc, left, right, r, D, r0, D0, r1, D1, is_last, rE, DE);
      exchange_ends<T, EXACT, NT, ML>(w, 1, t, P, mlast, active, s_first, s_last, left, right);
      if (active) rk4_stage<T, EXACT, 2, ML>(v, w, w, acc, left, right, r, D, r0, D0, r1, D1, is_last, rE, DE);
      exchange_ends<T, EXACT, NT, ML>(w, 0, t, P, mlast, active, s_first, s_last, left, right);
      if (active) rk4_stage<T, EXACT, 3, ML>(v, w, w, acc, left, right, r, D, r0, D0, r1, D1, is_last, rE, DE);
      exchange_ends<T, EXACT, NT, ML>(w, 1, t, P, mlast, active, s_first, s_last, left, right);
      if (active) rk4_stage<T, EXACT, 4, ML>(v, w, w, acc, left, right, r, D, r0, D0, r1, D1, is_last, rE, DE);
    }
  } else {
  // two steps per iteration: v -> w, then w -> v (exchange buffers 0 and 1 alternate)
  int step = 0;
  // (a wave with no active lane skips the arithmetic; inside a step nothing branches on the lane)
  for (; step + 2 <= steps; step += 2) {
    exchange_ends<T, EXACT, NT, ML, REC>(v, 0, t, P, mlast, active, s_first, s_last, left, right);
    if (active) {
      chunk_step<T, EXACT, ML>(v, w, left, right, r, D, r0, D0, r1, D1, is_last, rE, DE);
    }
    if constexpr (REC) record_window<T, NT>(w, stage, bt, n, rec + step * rstride);
    exchange_ends<T, EXACT, NT, ML, REC>(w, 1, t, P, mlast, active, s_first, s_last, left, right);
    if (active) {
      chunk_step<T, EXACT, ML>(w, v, left, right, r, D, r0, D0, r1, D1, is_last, rE, DE);
    }
    if constexpr (REC) record_window<T, NT>(v, stage, bt, n, rec + (step + 1) * rstride);
  }
  if (step < steps) {
    exchange_ends<T, EXACT, NT, ML, REC>(v, 0, t, P, mlast, active, s_first, s_last, left, right);
    if (active) {
      chunk_step<T, EXACT, ML>(v, w, left, right, r, D, r0, D0, r1, D1, is_last, rE, DE);
#pragma unroll
      for (int j = 0; j < M; ++j) v[j] = w[j];
    }
    if constexpr (REC) record_window<T, NT>(v, stage, bt, n, rec + step * rstride);
  }
  }
  if constexpr (REC) return;   // the last state is recorded

  // store the window's output nodes [bt.lo, bt.lo + bt.count), staged like the load
  for (int h = 0; h < 2; ++h) {
    const int r0 = h == 0 ? 0 : M * half;
    const int r1 = h == 0 ? M * half : W;
    if (active && (h == 0) == (t < half)) {
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (EXACT || j < m) stage[spad(s + j - r0)] = v[j];
    }
    __syncthreads();
    const int o0 = r0 > bt.lo ? r0 : bt.lo;
    const int o1 = r1 < bt.lo + bt.count ? r1 : bt.lo + bt.count;
    for (int w = o0 + t; w < o1; w += NT) {
      int g = bt.first + w;
      if (g >= n) g -= n;
      dst[g] = stage[spad(w - r0)];
    }
    __syncthreads();
  }
}

// One window on NT lanes: full-size windows of the widest class take the exact body, others the body
// compiled for their last lane's node count.
template <typename T, bool RK4, int NT, bool REC = false>
__device__ __forceinline__ void window_body(const BlockTile& bt, const InstDesc& d, const T* __restrict__ src,
                                            T* __restrict__ dst, int steps, T* stage, T (*s_first)[NT],
                                            T (*s_last)[NT], int t, T* __restrict__ rec = nullptr,
                                            int64_t rstride = 0) {
  if constexpr (NT == kBlockThreads) {
    if (bt.width == NT * kBlockChunk) {
      block_body<T, true, RK4, NT, 0, REC>(bt, d, src, dst, steps, stage, s_first, s_last, t, rec, rstride);
      return;
    }
  }
  // the last lane's node count, uniform over the lanes of the window: one specialised body per count
  const int mlast = bt.width - kBlockChunk * ((bt.width + kBlockChunk - 1) / kBlockChunk - 1);
  switch (mlast) {
#define BURGERS_RAGGED_CASE(K) \
  case K: block_body<T, false, RK4, NT, K, REC>(bt, d, src, dst, steps, stage, s_first, s_last, t, rec, rstride); break;
    BURGERS_RAGGED_CASE(1) BURGERS_RAGGED_CASE(2) BURGERS_RAGGED_CASE(3) BURGERS_RAGGED_CASE(4)
    BURGERS_RAGGED_CASE(5) BURGERS_RAGGED_CASE(6) BURGERS_RAGGED_CASE(7) BURGERS_RAGGED_CASE(8)
    BURGERS_RAGGED_CASE(9) BURGERS_RAGGED_CASE(10) BURGERS_RAGGED_CASE(11) BURGERS_RAGGED_CASE(12)
    BURGERS_RAGGED_CASE(13) BURGERS_RAGGED_CASE(14) BURGERS_RAGGED_CASE(15) BURGERS_RAGGED_CASE(16)
#undef BURGERS_RAGGED_CASE
    default: break;
  }
}

// One workgroup of NT lanes per window or whole instance; full-size windows of the widest class take the
// specialised body.  RK4 windows run in a kernel of their own, so that the forward-Euler kernel keeps its
// smaller register footprint.  Narrower classes serve smaller whole instances: fewer idle waves at each
// step's barrier, and more workgroups per CU.
template <typename T, bool RK4, int NT = kBlockThreads>
__global__ __launch_bounds__(NT) void explicit_block_kernel(
    const InstDesc* __restrict__ inst, const BlockTile* __restrict__ tiles, const T* __restrict__ u,
    T* __restrict__ out, int steps, int first_step) {
  constexpr int kStage = stage_nodes<NT>();
  __shared__ T s_first[2][NT];
  __shared__ T s_last[2][NT];
  __shared__ T stage[kStage + kStage / 16 + 1];
  const BlockTile bt = tiles[blockIdx.x];
  if (bt.width <= 0) return;                   // an empty slot of a resident pool
  // a slot with `limit` steps left in the call takes those of this launch's steps (steps [first_step,
  // first_step + steps) of the call) that remain; with none left it still carries its window over
  if (bt.limit > 0) steps = max(0, min(steps, bt.limit - first_step));
  const InstDesc d = inst[bt.inst];
  const T* src = u + d.off;
  T* dst = out + d.off;
  window_body<T, RK4, NT>(bt, d, src, dst, steps, stage, s_first, s_last, static_cast<int>(threadIdx.x));
}

// Forward-Euler windows and whole instances that record every step's state (the adjoint's recompute of
// a checkpoint segment): states 1..steps of the launch at rec + (k - 1) rstride; the source is only read.
template <typename T>
__global__ __launch_bounds__(kBlockThreads) void explicit_record_kernel(
    const InstDesc* __restrict__ inst, const BlockTile* __restrict__ tiles, const T* __restrict__ u,
    T* __restrict__ rec, int64_t rstride, int steps) {
  constexpr int NT = kBlockThreads;
  constexpr int kStage = stage_nodes<NT>();
  __shared__ T s_first[2][NT];
  __shared__ T s_last[2][NT];
  __shared__ T stage[kStage + kStage / 16 + 1];
  const BlockTile bt = tiles[blockIdx.x];
  if (bt.width <= 0) return;
  const InstDesc d = inst[bt.inst];
  window_body<T, false, NT, true>(bt, d, u + d.off, nullptr, steps, stage, s_first, s_last,
                                  static_cast<int>(threadIdx.x), rec + d.off, rstride);
}

// LDS of a sub-group of NT lanes in the pack kernel: its exchange buffers and staging area.
template <int NT>
constexpr int sub_stage_size() {
  return stage_nodes<NT>() + stage_nodes<NT>() / 16 + 1;
}
constexpr int pack_stage_size() {
  constexpr int a = (kBlockThreads / 64) * sub_stage_size<64>(), b = (kBlockThreads / 128) * sub_stage_size<128>();
  constexpr int c = (kBlockThreads / 256) * sub_stage_size<256>(), e = sub_stage_size<kBlockThreads>();
  constexpr int ab = a > b ? a : b, ce = c > e ? c : e;
  return ab > ce ? ab : ce;
}

template <typename T, bool RK4, int NT>
__device__ __forceinline__ void pack_member(const InstDesc* __restrict__ inst, const BlockTile* __restrict__ tiles,
                                            const BlockPack& pk, const T* __restrict__ u, T* __restrict__ out,
                                            int steps, T* s_first_all, T* s_last_all, T* stage_all) {
  const int g = static_cast<int>(threadIdx.x) / NT, t = static_cast<int>(threadIdx.x) % NT;
  // a sub-group without an instance runs an empty window: no loads or stores, the same barriers
  BlockTile bt{0, 0, 0, 0, 0, 0, RK4 ? 1 : 0, 0};
  if (g < pk.count) bt = tiles[pk.first + g];
  const InstDesc d = inst[bt.inst];
  auto s_first = reinterpret_cast<T(*)[NT]>(s_first_all + g * 2 * NT);
  auto s_last = reinterpret_cast<T(*)[NT]>(s_last_all + g * 2 * NT);
  window_body<T, RK4, NT>(bt, d, u + d.off, out + d.off, steps, stage_all + g * sub_stage_size<NT>(), s_first, s_last,
                          t);
}

// The whole instances of a call's narrower width classes (64, 128 and 256 lanes) in one launch over a
// list of packs, widest class first: a workgroup of 512 lanes runs 512 / lanes instances side by side
// (instances of 512 lanes would run one per workgroup too, but their own kernel compiles the step loop
// to fewer registers).  The instances of a pack take the same number of steps, so their barriers
// coincide.
template <typename T, bool RK4>
__global__ __launch_bounds__(kBlockThreads) void explicit_pack_kernel(const InstDesc* __restrict__ inst,
                                                                      const BlockTile* __restrict__ tiles,
                                                                      const BlockPack* __restrict__ packs,
                                                                      T* __restrict__ u, int steps) {
  __shared__ T s_first[2 * kBlockThreads];
  __shared__ T s_last[2 * kBlockThreads];
  __shared__ T stage[pack_stage_size()];
  const BlockPack pk = packs[blockIdx.x];
  switch (pk.lanes) {
    case 64: pack_member<T, RK4, 64>(inst, tiles, pk, u, u, steps, s_first, s_last, stage); break;
    case 128: pack_member<T, RK4, 128>(inst, tiles, pk, u, u, steps, s_first, s_last, stage); break;
    case 256: pack_member<T, RK4, 256>(inst, tiles, pk, u, u, steps, s_first, s_last, stage); break;
    default: pack_member<T, RK4, kBlockThreads>(inst, tiles, pk, u, u, steps, s_first, s_last, stage); break;
  }
}

// Copy the nodes of a set of tiles (the instances of one subset) from src to dst.
template <typename T>
__global__ __launch_bounds__(kStreamThreads) void copy_tiles_kernel(const Tile* __restrict__ tiles,
                                                                    const T* __restrict__ src,
                                                                    T* __restrict__ dst) {
  constexpr int V = Vec<T>::n, K = kStreamVecs<T>;
  using VT = typename Vec<T>::type;
  const Tile t = tiles[blockIdx.x];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int i0 = t.start + (q * kStreamThreads + static_cast<int>(threadIdx.x)) * V;
    if (i0 >= t.n) return;
    const VT v = *reinterpret_cast<const VT*>(src + t.off + i0);
    if (i0 + V <= t.n) {
      *reinterpret_cast<VT*>(dst + t.off + i0) = v;
    } else {
      T e[V];
      __builtin_memcpy(e, &v, sizeof(VT));
#pragma unroll
      for (int k = 0; k < V; ++k)
        if (i0 + k < t.n) dst[t.off + i0 + k] = e[k];
    }
  }
}

}  // namespace

hipError_t launch_copy_tiles(const burgers_ctx* ctx, const Tile* tiles, int64_t n_tiles, const void* src,
                             void* dst) {
  if (n_tiles <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(n_tiles)), block(kStreamThreads);
  if (ctx->dtype == BURGERS_F64) {
    copy_tiles_kernel<double><<<grid, block, 0, ctx->stream>>>(tiles, static_cast<const double*>(src),
                                                               static_cast<double*>(dst));
  } else {
    copy_tiles_kernel<float><<<grid, block, 0, ctx->stream>>>(tiles, static_cast<const float*>(src),
                                                              static_cast<float*>(dst));
  }
  return hipGetLastError();
}

int explicit_tile_nodes(burgers_dtype dt) {
  return dt == BURGERS_F64 ? kStreamThreads * Vec<double>::n * kStreamVecs<double>
                           : kStreamThreads * Vec<float>::n * kStreamVecs<float>;
}

int explicit_block_capacity() { return kBlockThreads * kBlockChunk; }

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

template <typename T, int NT>
void block_launch(const burgers_ctx* ctx, const BlockTile* tiles, int64_t n_fe, int64_t n_rk4, const void* u,
                  void* out, int steps, int first_step) {
  const InstDesc* inst = ctx->inst.as<InstDesc>();
  const T* src = static_cast<const T*>(u);
  T* dst = static_cast<T*>(out);
  if (n_fe > 0)
    explicit_block_kernel<T, false, NT><<<static_cast<unsigned>(n_fe), NT, 0, ctx->stream>>>(inst, tiles, src, dst,
                                                                                            steps, first_step);
  if (n_rk4 > 0)
    explicit_block_kernel<T, true, NT><<<static_cast<unsigned>(n_rk4), NT, 0, ctx->stream>>>(inst, tiles + n_fe, src,
                                                                                            dst, steps, first_step);
}

template <typename T>
void block_launch_lanes(const burgers_ctx* ctx, const BlockTile* tiles, int64_t n_fe, int64_t n_rk4, const void* u,
                        void* out, int steps, int lanes, int first_step) {
  switch (lanes) {
    case 64: block_launch<T, 64>(ctx, tiles, n_fe, n_rk4, u, out, steps, first_step); break;
    case 128: block_launch<T, 128>(ctx, tiles, n_fe, n_rk4, u, out, steps, first_step); break;
    case 256: block_launch<T, 256>(ctx, tiles, n_fe, n_rk4, u, out, steps, first_step); break;
    default: block_launch<T, kBlockThreads>(ctx, tiles, n_fe, n_rk4, u, out, steps, first_step); break;
  }
}

hipError_t launch_explicit_block(const burgers_ctx* ctx, const BlockTile* tiles, int64_t n_fe, int64_t n_rk4,
                                 const void* u, void* out, int steps, int lanes, int first_step) {
  if (n_fe + n_rk4 <= 0 || steps <= 0) return hipSuccess;
  if (ctx->dtype == BURGERS_F64) block_launch_lanes<double>(ctx, tiles, n_fe, n_rk4, u, out, steps, lanes, first_step);
  else block_launch_lanes<float>(ctx, tiles, n_fe, n_rk4, u, out, steps, lanes, first_step);
  return hipGetLastError();
}

hipError_t launch_explicit_packs(const burgers_ctx* ctx, const BlockTile* tiles, const BlockPack* packs,
                                 int64_t n_fe, int64_t n_rk4, void* u, int steps) {
  if (n_fe + n_rk4 <= 0 || steps <= 0) return hipSuccess;
  const InstDesc* inst = ctx->inst.as<InstDesc>();
  if (ctx->dtype == BURGERS_F64) {
    if (n_fe > 0)
      explicit_pack_kernel<double, false><<<static_cast<unsigned>(n_fe), kBlockThreads, 0, ctx->stream>>>(
          inst, tiles, packs, static_cast<double*>(u), steps);
    if (n_rk4 > 0)
      explicit_pack_kernel<double, true><<<static_cast<unsigned>(n_rk4), kBlockThreads, 0, ctx->stream>>>(
          inst, tiles, packs + n_fe, static_cast<double*>(u), steps);
  } else {
    if (n_fe > 0)
      explicit_pack_kernel<float, false><<<static_cast<unsigned>(n_fe), kBlockThreads, 0, ctx->stream>>>(
          inst, tiles, packs, static_cast<float*>(u), steps);
    if (n_rk4 > 0)
      explicit_pack_kernel<float, true><<<static_cast<unsigned>(n_rk4), kBlockThreads, 0, ctx->stream>>>(
          inst, tiles, packs + n_fe, static_cast<float*>(u), steps);
  }
  return hipGetLastError();
}

hipError_t launch_explicit_record(const burgers_ctx* ctx, const BlockTile* tiles, int64_t n_tiles, const void* u,
                                  void* rec, int64_t rstride, int steps) {
  if (n_tiles <= 0 || steps <= 0) return hipSuccess;
  if (ctx->dtype != BURGERS_F64) return hipErrorInvalidValue;
  explicit_record_kernel<double><<<static_cast<unsigned>(n_tiles), kBlockThreads, 0, ctx->stream>>>(
      ctx->inst.as<InstDesc>(), tiles, static_cast<const double*>(u), static_cast<double*>(rec), rstride, steps);
  return hipGetLastError();
}

int explicit_pack_lanes() { return kBlockThreads; }

int explicit_block_lanes(int n) {
  int lanes = 64;
  while (lanes < kBlockThreads && lanes * kBlockChunk < n) lanes *= 2;
  return lanes;
}

}  // namespace burgers
