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

constexpr int kWgThreads = 512;   // threads of the whole-system solver
constexpr int kWgChunk = 16;      // longest chunk a thread of the whole-system solver eliminates
constexpr int kRedChunk = 16;     // chunk length in the partition levels
constexpr int kWgRows = kWgThreads * kWgChunk;            // longest system solved whole
constexpr int kRedRows = kReduceBlock * kRedChunk;        // rows one partition workgroup stages

// Rows staged in LDS are padded by one element every 32 rows: a thread reads its chunk with a lane
// stride of q rows, and without the pad q = 16 or 32 would put every lane of a wave on one bank.
__device__ __forceinline__ int padded(int i) { return i + (i >> 5); }
constexpr int padded_size(int rows) { return rows + rows / 32 + 1; }

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

// Rows of a level-0 system whose old values sit in LDS (staged coalesced from HBM); row k is held at
// padded(k - base).
template <typename S>
struct LdsRows {
  const S* st;
  int base;
  double r, D, a, b;
  bool dirichlet;
  __device__ __forceinline__ void row(int k, int R, double& al, double& be, double& ga,
                                      double& de) const {
    const double ui = static_cast<double>(st[padded(k - base)]);
    btcs_row(ui, r, D, al, be, ga);
    de = ui;
    if (dirichlet) {
      if (k == 0) { de = de - al * a; al = 0.0; }
      if (k == R - 1) { de = de - ga * b; ga = 0.0; }
    }
  }
};

template <typename S>
struct LdsDst {
  S* st;
  int base;
  __device__ __forceinline__ void write(int k, double v) const { st[padded(k - base)] = static_cast<S>(v); }
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

// Whole-system solver: one workgroup per system.  Level-0 systems stage the old state through LDS
// (coalesced loads), eliminate chunks from LDS, solve the reduced system by PCR in the same LDS, write
// the new values back into the staging buffer and store them coalesced, with the Dirichlet boundary
// nodes.  Reduced systems of the partition levels read (A, C, D) and write X in HBM directly.
template <typename S, bool FromState>
__global__ __launch_bounds__(kWgThreads, 4) void btcs_wg_kernel(
    const InstDesc* __restrict__ inst, const SysDesc* __restrict__ systems, const S* __restrict__ u,
    S* __restrict__ out, const double* __restrict__ LA, const double* __restrict__ LC,
    const double* __restrict__ LD, double* __restrict__ LX) {
  using T = double;
  constexpr int kPcrBytes = 4 * 2 * kWgThreads * static_cast<int>(sizeof(T));
  constexpr int kStageBytes = FromState ? padded_size(kWgRows) * static_cast<int>(sizeof(S)) : 0;
  constexpr int kBytes = kStageBytes > kPcrBytes ? kStageBytes : kPcrBytes;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kBytes];
  T* sA = reinterpret_cast<T*>(smem);
  T* sB = sA + 2 * kWgThreads;
  T* sC = sB + 2 * kWgThreads;
  T* sD = sC + 2 * kWgThreads;
  S* stage = reinterpret_cast<S*>(smem);

  const SysDesc sys = systems[blockIdx.x];
  const int R = sys.rows, P = sys.chunks;
  const int tid = threadIdx.x;

  LdsRows<S> ssrc{};
  ArrayRows<T> asrc{};
  LdsDst<S> sdst{};
  PtrDst<T> adst{};
  InstDesc d{};
  if constexpr (FromState) {
    d = inst[sys.inst];
    const bool dir = d.bc == kDirichlet;
    const S* src = u + d.off + (dir ? 1 : 0);
    for (int i = tid; i < R; i += kWgThreads) stage[padded(i)] = src[i];
    ssrc = LdsRows<S>{stage, 0, d.r, d.D, d.a, d.b, dir};
    sdst = LdsDst<S>{stage, 0};
    if (dir && tid == 0) {
      out[d.off] = static_cast<S>(d.a);
      out[d.off + d.n - 1] = static_cast<S>(d.b);
    }
    __syncthreads();
  } else {
    asrc = ArrayRows<T>{LA + sys.in_off, LC + sys.in_off, LD + sys.in_off};
    adst.x = LX + sys.in_off;
  }

  if (R == 1) {   // a single Dirichlet unknown
    if (tid == 0) {
      T al, be, ga, de;
      if constexpr (FromState) {
        ssrc.row(0, 1, al, be, ga, de);
        out[d.off + 1] = static_cast<S>(de / be);
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
  }
  if constexpr (FromState) __syncthreads();   // the PCR arrays overlay the staged rows
  if (tid < P) {
    sA[2 * tid] = AF; sB[2 * tid] = T(1); sC[2 * tid] = CF; sD[2 * tid] = DF;
    sA[2 * tid + 1] = AE; sB[2 * tid + 1] = T(1); sC[2 * tid + 1] = CE; sD[2 * tid + 1] = DE;
  }
  __syncthreads();
  pcr_cyclic<T, kWgThreads>(sA, sB, sC, sD, 2 * P);
  T F = T(0), E = T(0);
  if (tid < P) {
    F = sD[2 * tid];
    E = sD[2 * tid + 1];
  }
  if constexpr (FromState) {
    __syncthreads();                           // all ends read before the staging buffer is reused
    if (tid < P) chunk_recover<T, kWgChunk>(sdst, s, m, al, ga, de, F, E);
    __syncthreads();
    S* dst = out + d.off + (d.bc == kDirichlet ? 1 : 0);
    for (int i = tid; i < R; i += kWgThreads) dst[i] = stage[padded(i)];
  } else {
    if (tid < P) chunk_recover<T, kWgChunk>(adst, s, m, al, ga, de, F, E);
  }
}

// Rows [rs, re) of the chunks a partition workgroup owns: chunk k spans chunk_span(k).
__device__ __forceinline__ void block_rows(const SysDesc& sys, int c0, int& rs, int& re) {
  int m;
  chunk_span(c0, sys.rows, sys.chunks, rs, m);
  const int c1 = c0 + kReduceBlock;
  if (c1 >= sys.chunks) {
    re = sys.rows;
  } else {
    chunk_span(c1, sys.rows, sys.chunks, re, m);
  }
}

// Partition level, forward half: every thread eliminates one chunk and stores its two reduced rows.
// At level 0 the workgroup's rows are staged through LDS first (coalesced loads).
template <typename S, bool FromState>
__global__ __launch_bounds__(kReduceBlock) void btcs_reduce_kernel(
    const InstDesc* __restrict__ inst, const SysDesc* __restrict__ systems,
    const ChunkBlock* __restrict__ blocks, const S* __restrict__ u, double* __restrict__ LA,
    double* __restrict__ LC, double* __restrict__ LD) {
  using T = double;
  __shared__ S stage[FromState ? padded_size(kRedRows) : 1];
  const ChunkBlock cb = blocks[blockIdx.x];
  const SysDesc sys = systems[cb.sys];
  const int k = cb.chunk0 + static_cast<int>(threadIdx.x);
  T al[kRedChunk], ga[kRedChunk], de[kRedChunk];
  T AF, CF, DF, AE, CE, DE;
  int s = 0, m = 0;
  if constexpr (FromState) {
    const InstDesc d = inst[sys.inst];
    const bool dir = d.bc == kDirichlet;
    int rs, re;
    block_rows(sys, cb.chunk0, rs, re);
    const S* src = u + d.off + (dir ? 1 : 0);
    for (int i = rs + static_cast<int>(threadIdx.x); i < re; i += kReduceBlock) stage[padded(i - rs)] = src[i];
    __syncthreads();
    if (k >= sys.chunks) return;
    chunk_span(k, sys.rows, sys.chunks, s, m);
    const LdsRows<S> rows{stage, rs, d.r, d.D, d.a, d.b, dir};
    chunk_eliminate<T, kRedChunk>(rows, s, m, sys.rows, al, ga, de, AF, CF, DF, AE, CE, DE);
  } else {
    if (k >= sys.chunks) return;
    chunk_span(k, sys.rows, sys.chunks, s, m);
    const ArrayRows<T> rows{LA + sys.in_off, LC + sys.in_off, LD + sys.in_off};
    chunk_eliminate<T, kRedChunk>(rows, s, m, sys.rows, al, ga, de, AF, CF, DF, AE, CE, DE);
  }
  const int64_t o = sys.red_off + 2 * static_cast<int64_t>(k);
  LA[o] = AF; LC[o] = CF; LD[o] = DF;
  LA[o + 1] = AE; LC[o + 1] = CE; LD[o + 1] = DE;
}

// Partition level, backward half: re-eliminate the chunk and recover its rows from the solved
// reduced unknowns.  At level 0 the rows are staged through LDS both ways.
template <typename S, bool FromState>
__global__ __launch_bounds__(kReduceBlock) void btcs_backsub_kernel(
    const InstDesc* __restrict__ inst, const SysDesc* __restrict__ systems,
    const ChunkBlock* __restrict__ blocks, const S* __restrict__ u, S* __restrict__ out,
    const double* __restrict__ LA, const double* __restrict__ LC, const double* __restrict__ LD,
    double* __restrict__ LX) {
  using T = double;
  __shared__ S stage[FromState ? padded_size(kRedRows) : 1];
  const ChunkBlock cb = blocks[blockIdx.x];
  const SysDesc sys = systems[cb.sys];
  const int k = cb.chunk0 + static_cast<int>(threadIdx.x);
  const bool active = k < sys.chunks;
  T al[kRedChunk], ga[kRedChunk], de[kRedChunk];
  T AF, CF, DF, AE, CE, DE;
  int s = 0, m = 0;
  T F = T(0), E = T(0);
  if (active) {
    chunk_span(k, sys.rows, sys.chunks, s, m);
    const int64_t o = sys.red_off + 2 * static_cast<int64_t>(k);
    F = LX[o];
    E = LX[o + 1];
  }
  if constexpr (FromState) {
    const InstDesc d = inst[sys.inst];
    const bool dir = d.bc == kDirichlet;
    int rs, re;
    block_rows(sys, cb.chunk0, rs, re);
    const S* src = u + d.off + (dir ? 1 : 0);
    for (int i = rs + static_cast<int>(threadIdx.x); i < re; i += kReduceBlock) stage[padded(i - rs)] = src[i];
    __syncthreads();
    if (active) {
      const LdsRows<S> rows{stage, rs, d.r, d.D, d.a, d.b, dir};
      chunk_eliminate<T, kRedChunk>(rows, s, m, sys.rows, al, ga, de, AF, CF, DF, AE, CE, DE);
    }
    __syncthreads();                           // every chunk read before the buffer is overwritten
    if (active) chunk_recover<T, kRedChunk>(LdsDst<S>{stage, rs}, s, m, al, ga, de, F, E);
    __syncthreads();
    S* dst = out + d.off + (dir ? 1 : 0);
    for (int i = rs + static_cast<int>(threadIdx.x); i < re; i += kReduceBlock) dst[i] = stage[padded(i - rs)];
    if (dir && threadIdx.x == 0) {
      if (cb.chunk0 == 0) out[d.off] = static_cast<S>(d.a);
      if (cb.chunk0 + kReduceBlock >= sys.chunks) out[d.off + d.n - 1] = static_cast<S>(d.b);
    }
  } else {
    if (!active) return;
    const ArrayRows<T> rows{LA + sys.in_off, LC + sys.in_off, LD + sys.in_off};
    chunk_eliminate<T, kRedChunk>(rows, s, m, sys.rows, al, ga, de, AF, CF, DF, AE, CE, DE);
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

int btcs_wg_capacity() { return kWgRows; }

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
