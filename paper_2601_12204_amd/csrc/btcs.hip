// BTCS step (Sec. 2.4, eq. 23) for gfx950: one tridiagonal solve A(u^n) u^{n+1} = u^n per step, cyclic
// for periodic instances, with the Dirichlet boundary values moved to the right-hand side.
//
// Thomas' recurrence is serial, so the solve is split by the partition method:
//   1. Each thread owns a contiguous chunk of rows.  Eliminating the chunk's interior expresses every
//      row through the chunk's first unknown F and last unknown E, and leaves two rows per chunk that
//      couple only F_k, E_k and the neighbouring chunks' E_{k-1}, F_{k+1}: a tridiagonal system of
//      2P rows over (F_0, E_0, F_1, E_1, ...), cyclic whenever the original one is.
//   2. That reduced system is solved by cyclic parallel cyclic reduction (PCR) in LDS when it is small,
//      or reduced again by the same chunk elimination in a further level (long systems).
//   3. Each chunk recovers its interior rows from F and E.
// Rows are assembled on the fly from u^n (no coefficient arrays in HBM).  The reduced systems have
// unit diagonals and |sub| + |super| < 1, since A is strictly diagonally dominant (row sums 1), so no
// pivoting is needed at any level.
//
// Arithmetic is binary64 for both state types; a binary32 state is widened on load and rounded once per
// step on store.  A binary32 partition solve drifts by a systematic bias of a few ulp per step, which
// over 10^3 steps exceeds the serial binary32 solve's own error; the binary64 solve keeps the binary32
// path within its one rounding per step of the exact discrete solution.  On CDNA the binary64 vector
// rate equals the non-packed binary32 rate, and this step is bound by HBM, so the wider arithmetic costs
// nothing measurable.
#include "internal.hpp"
#include "stencil.hpp"

#pragma clang fp contract(off)

namespace burgers {
namespace {

constexpr int kWgThreads = 256;   // threads of the whole-system solver
constexpr int kWgChunk = 32;      // longest chunk a thread of the whole-system solver eliminates
constexpr int kRedChunk = 16;     // chunk length in the partition levels

// Rows of a level-0 system, assembled from the old state (type S) of one instance.
template <typename S>
struct StateRows {
  const S* __restrict__ u;   // node 0 of the instance
  double r, D, a, b;
  int first;                 // node of row 0: 0 periodic, 1 Dirichlet
  bool dirichlet;
  __device__ __forceinline__ void row(int k, int R, double& al, double& be, double& ga,
                                      double& de) const {
    const double ui = static_cast<double>(u[first + k]);
    btcs_row(ui, r, D, al, be, ga);
    de = ui;
    if (dirichlet) {
      if (k == 0) { de = de - al * a; al = 0.0; }
      if (k == R - 1) { de = de - ga * b; ga = 0.0; }
    }
  }
};

template <typename S>
__device__ __forceinline__ StateRows<S> state_rows(const InstDesc& d, const S* u) {
  const bool dir = d.bc == kDirichlet;
  return StateRows<S>{u + d.off, d.r, d.D, d.a, d.b, dir ? 1 : 0, dir};
}

// Rows of a reduced system stored with unit diagonal.
template <typename T>
struct ArrayRows {
  const T* __restrict__ A;
  const T* __restrict__ C;
  const T* __restrict__ Dv;
  __device__ __forceinline__ void row(int k, int, T& al, T& be, T& ga, T& de) const {
    al = A[k];
    be = T(1);
    ga = C[k];
    de = Dv[k];
  }
};

// Chunk elimination.  Rows s..s+m-1 (2 <= m <= M) of a system with R rows.  On return, for
// 1 <= j <= m-2, row j reads  x_j + al[j] F + ga[j] E = de[j]  with F = x_0, E = x_{m-1}, and the two
// reduced rows are
//   F row:  AF * E_prev + F + CF * E      = DF
//   E row:  AE * F      + E + CE * F_next = DE.
template <typename T, int M, typename Src>
__device__ __forceinline__ void chunk_eliminate(const Src& src, int s, int m, int R, T (&al)[M],
                                                T (&ga)[M], T (&de)[M], T& AF, T& CF, T& DF, T& AE,
                                                T& CE, T& DE) {
  T a0, b0, c0, d0;
  src.row(s, R, a0, b0, c0, d0);
  // forward: x_j + al[j] x_0 + ga[j] x_{j+1} = de[j]
#pragma unroll
  for (int j = 1; j < M; ++j) {
    if (j < m) {
      T aj, bj, cj, dj;
      src.row(s + j, R, aj, bj, cj, dj);
      // Each coefficient is divided separately: scaling all three by one rounded reciprocal biases
      // the row, and in FP32 that bias accumulates over many steps.
      if (j == 1) {
        al[1] = aj / bj;
        ga[1] = cj / bj;
        de[1] = dj / bj;
      } else {
        const T den = bj - aj * ga[j - 1];
        al[j] = -(aj * al[j - 1]) / den;
        ga[j] = cj / den;
        de[j] = (dj - aj * de[j - 1]) / den;
      }
      if (j == m - 1) {
        AE = al[j];
        CE = ga[j];
        DE = de[j];
      }
    }
  }
  // backward: x_j + al[j] x_0 + ga[j] x_{m-1} = de[j]  (row m-2 already has this form)
#pragma unroll
  for (int j = M - 3; j >= 1; --j) {
    if (j <= m - 3) {
      const T g = ga[j];
      de[j] = de[j] - g * de[j + 1];
      al[j] = al[j] - g * al[j + 1];
      ga[j] = -(g * ga[j + 1]);
    }
  }
  // row 0 with x_1 eliminated (for m == 2, x_1 is E itself)
  T a1 = T(0), g1 = T(-1), d1 = T(0);
  if (m > 2) {
    a1 = al[1];
    g1 = ga[1];
    d1 = de[1];
  }
  const T den0 = b0 - c0 * a1;
  AF = a0 / den0;
  CF = -(c0 * g1) / den0;
  DF = (d0 - c0 * d1) / den0;
}

// Interior rows from the chunk's end values.
template <typename T, int M, typename Dst>
__device__ __forceinline__ void chunk_recover(const Dst& dst, int s, int m, const T (&al)[M],
                                              const T (&ga)[M], const T (&de)[M], T F, T E) {
  dst.write(s, F);
#pragma unroll
  for (int j = 1; j < M; ++j) {
    if (j < m - 1) dst.write(s + j, de[j] - al[j] * F - ga[j] * E);
  }
  dst.write(s + m - 1, E);
}

template <typename S>
struct PtrDst {
  S* __restrict__ x;
  __device__ __forceinline__ void write(int k, double v) const { x[k] = static_cast<S>(v); }
};

// Chunk layout of a system of R rows split into P chunks: sizes q or q+1, the longer ones first.
__device__ __forceinline__ void chunk_span(int k, int R, int P, int& s, int& m) {
  const int q = R / P, rho = R - q * P;
  s = k * q + (k < rho ? k : rho);
  m = q + (k < rho ? 1 : 0);
}

// Cyclic PCR on R2 (a power of two, <= 2 NT) rows with coefficients in LDS.  Indices wrap modulo R2;
// a non-cyclic system simply carries zero corner couplings.  After log2(R2) steps every row couples
// only to itself and the solution is D / (A + B + C); it is left in sD.
template <typename T, int NT>
__device__ __forceinline__ void pcr_cyclic(T* sA, T* sB, T* sC, T* sD, int R2) {
  const int tid = threadIdx.x;
  for (int s = 1; s < R2; s <<= 1) {
    T nA[2], nB[2], nC[2], nD[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = tid + h * NT;
      if (i < R2) {
        const int im = (i - s) & (R2 - 1);
        const int ip = (i + s) & (R2 - 1);
        const T k1 = sA[i] / sB[im];
        const T k2 = sC[i] / sB[ip];
        nB[h] = (sB[i] - k1 * sC[im]) - k2 * sA[ip];
        nD[h] = (sD[i] - k1 * sD[im]) - k2 * sD[ip];
        nA[h] = -(k1 * sA[im]);
        nC[h] = -(k2 * sC[ip]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = tid + h * NT;
      if (i < R2) {
        sA[i] = nA[h];
        sB[i] = nB[h];
        sC[i] = nC[h];
        sD[i] = nD[h];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = tid + h * NT;
    if (i < R2) sD[i] = sD[i] / ((sB[i] + sA[i]) + sC[i]);
  }
  __syncthreads();
}

// Whole-system solver: one workgroup per system.  Level-0 systems read the old state and write the
// new state (and the Dirichlet boundary nodes); reduced systems read (A, C, D) and write X.
template <typename S, bool FromState>
__global__ __launch_bounds__(kWgThreads) void btcs_wg_kernel(
    const InstDesc* __restrict__ inst, const SysDesc* __restrict__ systems, const S* __restrict__ u,
    S* __restrict__ out, const double* __restrict__ LA, const double* __restrict__ LC,
    const double* __restrict__ LD, double* __restrict__ LX) {
  using T = double;
  __shared__ T sA[2 * kWgThreads], sB[2 * kWgThreads], sC[2 * kWgThreads], sD[2 * kWgThreads];
  const SysDesc sys = systems[blockIdx.x];
  const int R = sys.rows, P = sys.chunks;
  const int tid = threadIdx.x;

  StateRows<S> ssrc{};
  ArrayRows<T> asrc{};
  PtrDst<S> sdst{};
  PtrDst<T> adst{};
  if constexpr (FromState) {
    const InstDesc d = inst[sys.inst];
    ssrc = state_rows(d, u);
    sdst.x = out + d.off + ssrc.first;
    if (ssrc.dirichlet && tid == 0) {
      out[d.off] = static_cast<S>(d.a);
      out[d.off + d.n - 1] = static_cast<S>(d.b);
    }
  } else {
    asrc = ArrayRows<T>{LA + sys.in_off, LC + sys.in_off, LD + sys.in_off};
    adst.x = LX + sys.in_off;
  }

  if (R == 1) {   // a single Dirichlet unknown
    if (tid == 0) {
      T al, be, ga, de;
      if constexpr (FromState) {
        ssrc.row(0, 1, al, be, ga, de);
        sdst.write(0, de / be);
      } else {
        asrc.row(0, 1, al, be, ga, de);
        adst.write(0, de / be);
      }
    }
    return;
  }

  T al[kWgChunk], ga[kWgChunk], de[kWgChunk];
  T AF, CF, DF, AE, CE, DE;
  int s = 0, m = 0;
  if (tid < P) {
    chunk_span(tid, R, P, s, m);
    if constexpr (FromState) {
      chunk_eliminate<T, kWgChunk>(ssrc, s, m, R, al, ga, de, AF, CF, DF, AE, CE, DE);
    } else {
      chunk_eliminate<T, kWgChunk>(asrc, s, m, R, al, ga, de, AF, CF, DF, AE, CE, DE);
    }
    sA[2 * tid] = AF; sB[2 * tid] = T(1); sC[2 * tid] = CF; sD[2 * tid] = DF;
    sA[2 * tid + 1] = AE; sB[2 * tid + 1] = T(1); sC[2 * tid + 1] = CE; sD[2 * tid + 1] = DE;
  }
  __syncthreads();
  pcr_cyclic<T, kWgThreads>(sA, sB, sC, sD, 2 * P);
  if (tid < P) {
    if constexpr (FromState) {
      chunk_recover<T, kWgChunk>(sdst, s, m, al, ga, de, sD[2 * tid], sD[2 * tid + 1]);
    } else {
      chunk_recover<T, kWgChunk>(adst, s, m, al, ga, de, sD[2 * tid], sD[2 * tid + 1]);
    }
  }
}

// Partition level, forward half: every thread eliminates one chunk and stores its two reduced rows.
template <typename S, bool FromState>
__global__ __launch_bounds__(kReduceBlock) void btcs_reduce_kernel(
    const InstDesc* __restrict__ inst, const SysDesc* __restrict__ systems,
    const ChunkBlock* __restrict__ blocks, const S* __restrict__ u, double* __restrict__ LA,
    double* __restrict__ LC, double* __restrict__ LD) {
  using T = double;
  const ChunkBlock cb = blocks[blockIdx.x];
  const SysDesc sys = systems[cb.sys];
  const int k = cb.chunk0 + static_cast<int>(threadIdx.x);
  if (k >= sys.chunks) return;
  int s, m;
  chunk_span(k, sys.rows, sys.chunks, s, m);
  T al[kRedChunk], ga[kRedChunk], de[kRedChunk];
  T AF, CF, DF, AE, CE, DE;
  if constexpr (FromState) {
    const StateRows<S> src = state_rows(inst[sys.inst], u);
    chunk_eliminate<T, kRedChunk>(src, s, m, sys.rows, al, ga, de, AF, CF, DF, AE, CE, DE);
  } else {
    const ArrayRows<T> src{LA + sys.in_off, LC + sys.in_off, LD + sys.in_off};
    chunk_eliminate<T, kRedChunk>(src, s, m, sys.rows, al, ga, de, AF, CF, DF, AE, CE, DE);
  }
  const int64_t o = sys.red_off + 2 * static_cast<int64_t>(k);
  LA[o] = AF; LC[o] = CF; LD[o] = DF;
  LA[o + 1] = AE; LC[o + 1] = CE; LD[o + 1] = DE;
}

// Partition level, backward half: re-eliminate the chunk and recover its rows from the solved
// reduced unknowns.
template <typename S, bool FromState>
__global__ __launch_bounds__(kReduceBlock) void btcs_backsub_kernel(
    const InstDesc* __restrict__ inst, const SysDesc* __restrict__ systems,
    const ChunkBlock* __restrict__ blocks, const S* __restrict__ u, S* __restrict__ out,
    const double* __restrict__ LA, const double* __restrict__ LC, const double* __restrict__ LD,
    double* __restrict__ LX) {
  using T = double;
  const ChunkBlock cb = blocks[blockIdx.x];
  const SysDesc sys = systems[cb.sys];
  const int k = cb.chunk0 + static_cast<int>(threadIdx.x);
  if (k >= sys.chunks) return;
  int s, m;
  chunk_span(k, sys.rows, sys.chunks, s, m);
  T al[kRedChunk], ga[kRedChunk], de[kRedChunk];
  T AF, CF, DF, AE, CE, DE;
  const int64_t o = sys.red_off + 2 * static_cast<int64_t>(k);
  const T F = LX[o], E = LX[o + 1];
  if constexpr (FromState) {
    const InstDesc d = inst[sys.inst];
    const StateRows<S> src = state_rows(d, u);
    chunk_eliminate<T, kRedChunk>(src, s, m, sys.rows, al, ga, de, AF, CF, DF, AE, CE, DE);
    chunk_recover<T, kRedChunk>(PtrDst<S>{out + d.off + src.first}, s, m, al, ga, de, F, E);
    if (src.dirichlet) {
      if (k == 0) out[d.off] = static_cast<S>(d.a);
      if (k == sys.chunks - 1) out[d.off + d.n - 1] = static_cast<S>(d.b);
    }
  } else {
    const ArrayRows<T> src{LA + sys.in_off, LC + sys.in_off, LD + sys.in_off};
    chunk_eliminate<T, kRedChunk>(src, s, m, sys.rows, al, ga, de, AF, CF, DF, AE, CE, DE);
    chunk_recover<T, kRedChunk>(PtrDst<T>{LX + sys.in_off}, s, m, al, ga, de, F, E);
  }
}

template <typename S>
hipError_t launch_step(const burgers_ctx* ctx, const BtcsPlan& plan, const void* uv, void* outv) {
  const S* u = static_cast<const S*>(uv);
  S* out = static_cast<S*>(outv);
  double* LA = ctx->level_a.as<double>();
  double* LC = ctx->level_c.as<double>();
  double* LD = ctx->level_d.as<double>();
  double* LX = ctx->level_x.as<double>();
  const InstDesc* inst = ctx->inst.as<InstDesc>();
  hipStream_t st = ctx->stream;
  const int L = static_cast<int>(plan.levels.size());
  // forward: reduce level by level
  for (int l = 0; l < L; ++l) {
    const auto& lv = plan.levels[l];
    if (lv.n_blocks == 0) continue;
    if (l == 0) {
      btcs_reduce_kernel<S, true><<<lv.n_blocks, kReduceBlock, 0, st>>>(
          inst, lv.sys->as<SysDesc>(), lv.blocks->as<ChunkBlock>(), u, LA, LC, LD);
    } else {
      btcs_reduce_kernel<S, false><<<lv.n_blocks, kReduceBlock, 0, st>>>(
          inst, lv.sys->as<SysDesc>(), lv.blocks->as<ChunkBlock>(), u, LA, LC, LD);
    }
  }
  // backward: whole-system solves of each level, then back-substitution of the reduced systems
  for (int l = L - 1; l >= 1; --l) {
    const auto& lv = plan.levels[l];
    if (lv.n_wg) {
      btcs_wg_kernel<S, false><<<lv.n_wg, kWgThreads, 0, st>>>(inst, lv.wg->as<SysDesc>(), u, out, LA,
                                                               LC, LD, LX);
    }
    if (lv.n_blocks) {
      btcs_backsub_kernel<S, false><<<lv.n_blocks, kReduceBlock, 0, st>>>(
          inst, lv.sys->as<SysDesc>(), lv.blocks->as<ChunkBlock>(), u, out, LA, LC, LD, LX);
    }
  }
  if (plan.n_wg_state) {
    btcs_wg_kernel<S, true><<<plan.n_wg_state, kWgThreads, 0, st>>>(
        inst, plan.wg_state->as<SysDesc>(), u, out, LA, LC, LD, LX);
  }
  if (L > 0 && plan.levels[0].n_blocks) {
    const auto& lv = plan.levels[0];
    btcs_backsub_kernel<S, true><<<lv.n_blocks, kReduceBlock, 0, st>>>(
        inst, lv.sys->as<SysDesc>(), lv.blocks->as<ChunkBlock>(), u, out, LA, LC, LD, LX);
  }
  return hipGetLastError();
}

}  // namespace

int btcs_wg_capacity() { return kWgThreads * kWgChunk; }

int btcs_wg_chunks(int rows) {
  // largest power of two P <= min(threads, rows / 2); rows <= capacity keeps every chunk <= kWgChunk
  int P = 1;
  while (2 * P <= kWgThreads && 2 * (2 * P) <= rows) P *= 2;
  return P;
}

int btcs_reduce_chunk() { return kRedChunk; }

hipError_t launch_btcs_step(const burgers_ctx* ctx, const BtcsPlan& plan, const void* u, void* out) {
  if (ctx->dtype == BURGERS_F64) return launch_step<double>(ctx, plan, u, out);
  return launch_step<float>(ctx, plan, u, out);
}

}  // namespace burgers
