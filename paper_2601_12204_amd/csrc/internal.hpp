// Internal declarations of the gfx950 Burgers library: device-side descriptors, the context and the
// launchers each kernel translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "burgers.h"

namespace burgers {

constexpr int kPeriodic = BURGERS_BC_PERIODIC;
constexpr int kDirichlet = BURGERS_BC_DIRICHLET;

// Per-instance scalars as the kernels read them (binary64; FP32 kernels round them once).
struct InstDesc {
  int64_t off;  // first element of the instance in a packed state buffer
  int32_t n;    // stored nodes
  int32_t bc;   // burgers_bc
  double r;     // dt / dx
  double D;     // nu dt / dx^2
  double a;     // Dirichlet left value
  double b;     // Dirichlet right value
  double dtdx2; // dt / dx^2 = dD / dnu
};

// A run of consecutive nodes of one instance handled by one workgroup of a streaming kernel.  It
// carries the instance's offset, size and boundary type so that a kernel can address its data after a
// single scalar load.
struct Tile {
  int64_t off;
  int32_t n;
  int32_t start;   // off, n and start share the first 16 bytes: one scalar load addresses the tile
  int32_t bc;
  int32_t inst;
};

// A window of one instance advanced several steps per launch by the temporal-blocking kernel.  Window
// node w is instance node (first + w) mod n; nodes [lo, lo + count) of the window are written back.
struct BlockTile {
  int32_t inst;
  int32_t first;
  int32_t width;
  int32_t lo;
  int32_t count;
  int32_t wrap;   // 1: the window is a whole periodic instance and its ends are neighbours
  int32_t rk4;    // 1: classical RK4 steps (4 stages) instead of forward Euler
  int32_t limit;  // > 0: advance at most this many of the launch's steps (a slot finishing mid-tick)
};

// Whole instances of one width class (`lanes` lanes each) that share a 512-lane workgroup of the explicit
// pack kernel: tiles first .. first + count - 1 of the whole-instance list.
struct BlockPack {
  int32_t first;
  int32_t count;
  int32_t lanes;
  int32_t unused;
};

// A run of 256 nodes of one instance in the adjoint sweep; `slot` indexes the tile's accumulator of
// dJ/dD and `sys_off` the instance's transposed system in the adjoint arrays (BTCS instances).
struct AdjTile {
  int64_t off;
  int64_t sys_off;
  int32_t n;
  int32_t bc;
  int32_t inst;
  int32_t start;
  int32_t slot;
  int32_t pad;
};

// A window of the explicit adjoint's blocked reverse steps: window node w (0 <= w < width) is instance
// node (first + w) mod n; nodes [lo, lo + count) are kept, and their tiles of kAdjSumTile nodes take the
// dJ/dD slots slot0, slot0 + 1, ...  (lo and the instance node of window node lo are multiples of
// kAdjSumTile.)
struct AdjWindow {
  int32_t inst, first, width, lo, count, slot0;
};
constexpr int kAdjWinNodes = 4096;   // window capacity (256 lanes x 16 nodes)
constexpr int kAdjHalo = 256;        // halo nodes per side of a window of a longer instance; steps per launch
constexpr int kAdjSumTile = 256;     // nodes per dJ/dD slot of an explicit instance

// One tridiagonal system of the BTCS solve at some level of the partition hierarchy.
//   level 0: rows assembled from the state of instance `inst`; level > 0: rows (A, 1, C, D) stored in
//   the level arrays starting at row `in_off`.  A system that is reduced writes its 2*chunks reduced
//   rows at `red_off` of the level arrays; the solution of those rows comes back in X at `red_off`.
struct SysDesc {
  int64_t in_off;
  int64_t red_off;
  int32_t rows;
  int32_t chunks;
  int32_t inst;
  int32_t level;
  int32_t cn = 0;   // level-0 Crank-Nicolson system: the solve is the half-dt BTCS one, stored as 2y - u
  int32_t limit = 0;  // > 0: the on-chip solver advances at most this many of the launch's steps
};

// A window of a long BTCS system (truncated partition): rows [start, start + 8192) of the system (mod its
// row count for periodic systems) are solved as a plain system whose neighbours beyond both ends take
// their old values; rows [start + lo, start + lo + count) of that solve are written to the new state.
struct WinDesc {
  int32_t inst;
  int32_t start;
  int32_t lo;
  int32_t count;
  int32_t cn;    // Crank-Nicolson system: the half-dt solve y is stored as 2y - u
  int32_t limit; // > 0: only the first `limit` steps of a call solve; later ones copy the kept rows
};

// Flags of truncated windows over `count` instances, one slot per step parity: slot p starts with a word
// that is nonzero when any window of that step failed its bound, followed by one word per instance (the
// instance must be redone); after both slots, a sticky word per instance (resident pools report it).
// Fallback kernels read the slot's first word before anything else and exit when it is zero.
inline int64_t win_flags_words(int64_t count) { return 3 * count + 2; }
inline int* win_flag_slot(int* base, int64_t count, int64_t step) { return base + (step & 1) * (count + 1) + 1; }
inline int* win_sticky(int* base, int64_t count) { return base + 2 * (count + 1); }

// A block of consecutive chunks of one system (reduce and back-substitution kernels).
struct ChunkBlock {
  int32_t sys;
  int32_t chunk0;
};

// A fixed device region that buffers are carved from instead of allocated (the entry point that
// allocates nothing): while a thread has one installed, DevBuf::alloc takes 256-byte-aligned pieces of
// it in order and fails with hipErrorOutOfMemory once it is used up; carved pieces are never freed.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};
inline thread_local Arena* tl_arena = nullptr;

// Device buffer owned by a context, allocated and released in stream order on the context's stream:
// hipFree would synchronise the whole device and stall every other context's work in flight.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  bool carved = false;   // a piece of an Arena: nothing to free
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr && !carved) (void)hipFreeAsync(ptr, stream);
    ptr = nullptr;
    bytes = 0;
    carved = false;
  }
  hipError_t alloc(size_t n, hipStream_t s) {
    release();
    stream = s;
    if (!n) return hipSuccess;
    if (Arena* a = tl_arena) {
      const size_t at = (a->used + 255) & ~static_cast<size_t>(255);
      if (at > a->cap || n > a->cap - at) return hipErrorOutOfMemory;
      ptr = a->base + at;
      a->used = at + n;
      bytes = n;
      carved = true;
      return hipSuccess;
    }
    hipError_t e = hipMallocAsync(&ptr, n, s);
    if (e != hipSuccess) {
      ptr = nullptr;
      return e;
    }
    bytes = n;
    return hipSuccess;
  }
  template <typename T> T* as() const { return static_cast<T*>(ptr); }
};

// Shape of the workgroup that solves a system of up to 8192 rows whole: `lanes` threads with chunks of
// at most `chunk` rows; `exact` when the system has exactly lanes x chunk rows (no ragged chunks).
struct WidthClass {
  int lanes = 0;
  int chunk = 0;
  bool exact = false;
  bool stream = false;   // exact systems with 16-byte aligned rows: the persistent pipelined per-step kernel
};

// Systems of one width class, one workgroup each.
struct WgGroup {
  WidthClass shape;
  std::unique_ptr<DevBuf> sys;               // SysDesc[]
  int32_t n = 0;
};

// Launch list of the BTCS solve for a set of instances, built once per context and set.
struct BtcsPlan {
  int path = 0;                              // 0 automatic, 1 per-step, 2 resident, 3 partition levels
  int threads = 0;                           // lanes for systems of exactly 8192 rows (512 or 1024)
  std::vector<WgGroup> resident;             // kept on chip for all steps of a launch (in place)
  std::unique_ptr<DevBuf> copy;              // Tile[] of the instances stepped through HBM (copy-back)
  int64_t n_copy = 0;
  std::vector<WgGroup> wg_state;             // solved whole per step, straight from and to the state
  // Crank-Nicolson instances: solved per step with the coefficients of dt/2 (a copy of the instance
  // table with r and D halved); their systems carry the `cn` flag and store u' = 2 y - u
  std::unique_ptr<DevBuf> inst_half;         // InstDesc[count], or empty: the context's table
  bool newton = false;                       // the context's Newton instances step with this plan
  // partition hierarchy for the long systems
  struct Level {
    std::unique_ptr<DevBuf> sys;             // SysDesc[] of the systems reduced at this level
    std::unique_ptr<DevBuf> blocks;          // ChunkBlock[]
    int32_t n_blocks = 0;
    std::unique_ptr<DevBuf> wg;              // SysDesc[] of the reduced systems solved whole
    int32_t n_wg = 0;
    int32_t wg_lanes = 512;                  // workgroup width for them (64..512: their widest chunk count)
    bool wg_exact = false;                   // every one of them has exactly 512 chunks of 16 rows
  };
  std::vector<Level> levels;                 // levels[0] reduces from the state
  int64_t level_rows = 0;                    // rows of A, C, D, X used by this plan
  // truncated windows of the long systems (every system of the partition levels at level 0 when
  // present); the partition levels then solve only the systems whose windows flag a failed bound
  int longmode = 0;                          // burgers_plan.btcs_long the plan was built for
  std::unique_ptr<DevBuf> win;               // WinDesc[]
  int64_t n_win = 0;
  int win_rows = 8192;                       // rows per window: 8192 (512 lanes) or 4096 (256 lanes)
  bool stream_exact = false;                 // per-step exact 8192-row systems: the persistent pipelined kernel
  DevBuf win_flags;                          // win_flags_words(count) int32 (see win_flag_slot)
};

// Launch lists of the explicit scheme for a set of instances.
struct ExplicitPlan {
  std::unique_ptr<DevBuf> stream;            // Tile[] covering every node of the set
  int64_t n_stream = 0;
  // temporal blocking: whole instances (all steps in place) and windows of long instances
  std::unique_ptr<DevBuf> whole, win;        // BlockTile[]
  int64_t n_whole = 0, n_win = 0;            // of which the last n_*_rk4 take RK4 steps
  int64_t n_whole_rk4 = 0, n_win_rk4 = 0;
  // whole instances by workgroup width: `whole` holds each class's tiles contiguously (forward Euler
  // first, then RK4)
  struct WholeClass {
    int lanes;
    int64_t offset, n_fe, n_rk4;
  };
  std::vector<WholeClass> whole_classes;
  // the narrower classes' instances packed for one launch per scheme (forward Euler packs, then RK4)
  std::unique_ptr<DevBuf> packs;             // BlockPack[]
  int64_t n_packs_fe = 0, n_packs_rk4 = 0;
  std::unique_ptr<DevBuf> win_copy;          // Tile[] of the windowed instances (copy-back)
  int64_t n_win_copy = 0;
  int path = 1;                              // 1 stream, 2 resident, 3 tiled
  int depth = 0;                             // steps per launch of the windows (and whole tiles, path 3)
};

// Launch lists and buffers of the adjoint sweep (built on the first burgers_adjoint call).
struct AdjointPlan {
  std::unique_ptr<DevBuf> exp_wins, btcs_tiles;     // AdjWindow[] of the explicit instances, AdjTile[]
  int64_t n_exp_wins = 0, n_btcs_tiles = 0;
  int64_t n_exp_wins_periodic = 0;                 // the first windows of exp_wins, of periodic instances
  std::unique_ptr<DevBuf> slot_begin;               // int32[count + 1]
  int64_t n_slots = 0;
  BtcsPlan solve;                                   // partition hierarchy over the transposed systems
  DevBuf LA, LC, LD, LX, gslot;
  DevBuf ckpt, seg, seg2, lam0, lam1;               // grown on demand (seg2: the segment recomputed alongside)
  // truncated windows of the transposed systems (when every BTCS instance has more than 8192 rows); the
  // array path above is then the fallback of the instances whose windows flag a failed bound
  std::unique_ptr<DevBuf> win, win_slot;           // WinDesc[], int32[] (dJ/dD slot of each window)
  int64_t n_win = 0;
  DevBuf wpart, flags;                              // double[n_win]; win_flags_words(count) int32
  // every BTCS instance of exactly 16384 rows: each transposed system solved whole, exactly, by one
  // workgroup per step (WinDesc covering it, and its dJ/dD slot); the array path is then not used
  std::unique_ptr<DevBuf> whole, whole_slot;
  int64_t n_whole = 0;
};

// Fully implicit central-convection instances (Newton-Raphson, a fixed number of iterations per step):
// per iteration the Jacobian rows and the residual are assembled, normalised to unit diagonal, into
// binary64 arrays and solved by the partition solver's array path.
constexpr int kNewtonIters = 4;
struct NewtonPlan {
  std::unique_ptr<DevBuf> tiles;                    // AdjTile[] (256 nodes each) of all Newton instances
  int64_t n_tiles = 0;
  std::vector<WgGroup> whole;                       // systems of up to 8192 rows: one fused kernel per iteration
  std::unique_ptr<DevBuf> long_tiles;               // AdjTile[] of the longer ones (array path)
  int64_t n_long_tiles = 0;
  BtcsPlan solve;                                   // partition hierarchy over the longer systems
  DevBuf NA, NC, ND, NX;
  DevBuf flags;                                     // int32[2]: dominance lost, not converged (read by burgers_sync)
};

}  // namespace burgers

struct burgers_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  burgers_dtype dtype = BURGERS_F64;
  size_t word = 8;
  int64_t count = 0;
  std::vector<burgers_problem> probs;
  std::vector<int64_t> offsets;
  int64_t total = 0;
  std::vector<burgers::InstDesc> inst_host;
  burgers::DevBuf inst;                      // InstDesc[count]
  burgers::DevBuf work;                      // second state buffer (ping-pong)
  burgers::DevBuf level_a, level_c, level_d, level_x;  // reduced systems of the BTCS partition
  int64_t level_capacity = 0;                // rows
  burgers_plan plan{};
  // instance subsets: all, explicit-scheme, btcs-scheme
  std::vector<int32_t> set_all, set_explicit, set_btcs;
  // launch plans per instance subset
  std::map<int, std::unique_ptr<burgers::ExplicitPlan>> explicit_plans;
  std::map<int, std::unique_ptr<burgers::BtcsPlan>> btcs;
  std::map<int, std::pair<std::unique_ptr<burgers::DevBuf>, int64_t>> copy_tiles;   // per subset
  // launch sequences captured as graphs, keyed by (subset, scheme, steps, BTCS steps, state buffer)
  std::map<std::tuple<int, int, int64_t, int64_t, void*>, hipGraphExec_t> graph_cache;
  hipStream_t capture_stream = nullptr;      // private non-blocking stream used only for capture
  // side streams (default priority) and events of the concurrent launch groups of a call
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t joined[3] = {nullptr, nullptr, nullptr};
  hipEvent_t forked = nullptr;
  std::unique_ptr<burgers::AdjointPlan> adjoint;
  std::unique_ptr<burgers::NewtonPlan> newton;
  hipError_t sticky = hipSuccess;
};

namespace burgers {

// explicit.hip
hipError_t launch_explicit_stream(const burgers_ctx* ctx, const Tile* tiles, int64_t n_tiles,
                                  const void* u, void* out);
// Windows tiles[0, n_fe) advance by forward Euler and tiles[n_fe, n_fe + n_rk4) by RK4.
// Temporal-blocking launch over `lanes`-wide workgroups (64, 128, 256 or 512; windows always take 512).
// `first_step`: the launch's first step counted from the start of the call (tiles with a step limit
// take only the steps of the call they have left).
hipError_t launch_explicit_block(const burgers_ctx* ctx, const BlockTile* tiles, int64_t n_fe, int64_t n_rk4,
                                 const void* u, void* out, int steps, int lanes = 512, int first_step = 0);
// Whole instances in place, the narrower width classes in one launch per scheme over packs (n_fe
// forward-Euler packs, then n_rk4 RK4 packs).
int explicit_pack_lanes();                  // lanes of a pack kernel workgroup
hipError_t launch_explicit_packs(const burgers_ctx* ctx, const BlockTile* tiles, const BlockPack* packs,
                                 int64_t n_fe, int64_t n_rk4, void* u, int steps);
// Forward-Euler block tiles (whole instances or windows with a halo of at least `steps`) recording the
// state after each step k (1 <= k <= steps) at rec + (k - 1) rstride (binary64; u is only read).
hipError_t launch_explicit_record(const burgers_ctx* ctx, const BlockTile* tiles, int64_t n_tiles, const void* u,
                                  void* rec, int64_t rstride, int steps);
// Windows of a long explicit instance `i` of n nodes advanced `depth` steps per launch (halo = depth x
// stages per side); appends them to `out`.  Returns false when the halo leaves no kept node.
bool explicit_windows(int32_t i, int32_t n, bool periodic, int depth, bool rk4, std::vector<BlockTile>& out);
// Truncated BTCS windows of `W` rows over a system of R rows of instance i; appends them to `out`.
void btcs_windows(int32_t i, int32_t R, bool periodic, int W, bool cn, std::vector<WinDesc>& out);
hipError_t launch_clear_ints(const burgers_ctx* ctx, int* p, int64_t n);
// capi.hip: argument checks and the kernels' per-instance scalars of a problem at state offset `off`
bool problem_valid(const burgers_problem& p);
InstDesc inst_desc(const burgers_problem& p, int64_t off);
int explicit_block_lanes(int n);   // narrowest workgroup that holds a whole instance of n nodes
hipError_t launch_copy_tiles(const burgers_ctx* ctx, const Tile* tiles, int64_t n_tiles, const void* src,
                             void* dst);
int explicit_tile_nodes(burgers_dtype dt);
int explicit_block_capacity();

// adjoint.hip
int adjoint_tile_nodes();   // nodes per dJ/dD slot of a BTCS instance
// Explicit reverse steps k = k_hi - 1 .. k_lo over the windows (those of periodic instances first, n_periodic
// of them): u^k at u0 (k = 0) or useg + (k - 1) ustride, lam^(k_hi) in lamp, lam^(k_lo) to lam (out of
// place), dJ/dD added to the windows' tile slots of gslot.  Windows of longer instances take at most
// kAdjHalo steps per launch.
hipError_t launch_adj_explicit_block(const burgers_ctx* ctx, const AdjWindow* wins, int64_t n_wins, int64_t n_periodic,
                                     const double* u0, const double* useg, int64_t ustride, int k_lo, int k_hi,
                                     const double* lamp, double* lam, double* gslot);
// `only` (optional): only the instances whose entry is nonzero (those whose windows flagged a failed
// bound); the finish launch also adds the windows' partials (wins/win_slot/wpart, n_win may be 0).
hipError_t launch_adj_btcs_assemble(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles,
                                    const double* u, const double* lamp, double* LA, double* LC, double* LD,
                                    const int* only);
hipError_t launch_adj_btcs_finish(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles,
                                  const double* u, const double* x, const double* X, double* lam,
                                  double* gslot, const int* only, const WinDesc* wins, int64_t n_win,
                                  const int32_t* win_slot, const double* wpart);
hipError_t launch_adj_nu(const burgers_ctx* ctx, const int32_t* slot_begin, const double* gslot,
                         double* grad_nu);
hipError_t launch_fill(const burgers_ctx* ctx, double* p, int64_t n, double v);
hipError_t launch_zero_dirichlet_ends(const burgers_ctx* ctx, double* g);

// newton.hip
hipError_t launch_newton_init(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles, const void* u, void* x);
// Jacobian rows and -F (checked for strict diagonal dominance into flags[0]); the update x += delta,
// whose increments are checked against the iterate into flags[1] when `last`.
hipError_t launch_newton_assemble(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles, const void* u,
                                  const void* x, double* NA, double* NC, double* ND, int* flags);
hipError_t launch_newton_update(const burgers_ctx* ctx, const AdjTile* tiles, int64_t n_tiles, const void* u,
                                void* x, const double* NX, bool last, int* flags);

// btcs.hip
int btcs_wg_capacity();                 // longest system of the exact 512-lane kernels and of the
                                        // partition levels' reduced systems (8192 rows)
int btcs_whole_capacity();              // longest system one workgroup solves whole (16384 rows)
bool btcs_solved_whole(int64_t rows);   // up to 8192 rows, or exactly 16384: one workgroup per system
int btcs_wg_chunks(int rows);
int btcs_wg_lanes(const std::vector<SysDesc>& systems);
bool btcs_wg_exact(const std::vector<SysDesc>& systems);   // all of 512 chunks x 16 rows (a constant layout)   // workgroup width that serves all of them           // chunk count the workgroup solver uses for `rows` rows
int btcs_reduce_chunk();                // target rows per chunk in the partition levels
constexpr int kReduceBlock = 256;       // chunks per workgroup in the partition kernels
// One BTCS step of the plan from u to out; `step` counts the steps of the current call from 0 (it selects
// the parity slot of the window flags, which launch_btcs_window_reset clears at the start of a call).
hipError_t launch_btcs_step(const burgers_ctx* ctx, const BtcsPlan& plan, const void* u, void* out, int64_t step);
hipError_t launch_btcs_window_reset(const burgers_ctx* ctx, const BtcsPlan& plan);
int btcs_window_halo();                 // halo rows on each side of a window's output rows
hipError_t launch_btcs_resident(const burgers_ctx* ctx, const WgGroup& group, void* u, int steps);
// The resident solver recording the state after each step k (1 <= k <= steps) at rec + (k - 1) rstride
// (binary64; src is only read).
hipError_t launch_btcs_record(const burgers_ctx* ctx, const WgGroup& group, const void* src, void* rec,
                              int64_t rstride, int steps);
hipError_t launch_newton_whole(const burgers_ctx* ctx, const WgGroup& group, const void* u, void* x, bool last,
                               int* flags);
WidthClass btcs_width_class(int rows, int threads);
int btcs_chunks(int rows, int threads);
// `only` (optional): solve only the systems of instances whose entry is nonzero.
hipError_t launch_array_solve(const burgers_ctx* ctx, const BtcsPlan& plan, double* LA, double* LC,
                              double* LD, double* LX, const int* only = nullptr);
// Adjoint BTCS steps k = k_hi - 1 .. k_lo of systems of exactly 16384 rows, each transposed system solved
// whole (u^k at u0 for k = 0, else useg + (k - 1) ustride; lam^(k_hi) in lamp, lam^(k_lo) to lam, out of
// place); each system's dJ/dD partial added to gslot[slots[b]] after every step.
hipError_t launch_adj_btcs_whole(const burgers_ctx* ctx, const WinDesc* wins, int64_t n, const double* u0,
                                 const double* useg, int64_t ustride, int k_lo, int k_hi, const double* lamp,
                                 double* lam, double* gslot, const int32_t* slots);
// Adjoint BTCS step of the long instances on truncated windows of the transposed system (lam from lamp
// at the forward pair u -> x); per-window partials of dJ/dD into wpart; failed bounds flag instances.
hipError_t launch_adj_btcs_windows(const burgers_ctx* ctx, const WinDesc* wins, int64_t n_win, const double* u,
                                   const double* x, const double* lamp, double* lam, double* wpart, int* flag_now,
                                   int* flag_next);
constexpr int kResidentThreadsDefault = 512;

}  // namespace burgers
