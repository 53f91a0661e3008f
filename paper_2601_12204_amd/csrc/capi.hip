// C ABI and host runtime of the gfx950 Burgers library: contexts, packed layout, launch plans and the
// stepping loops (ping-pong between the caller's state buffer and the context's second buffer).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <tuple>

#include "internal.hpp"

using burgers::ChunkBlock;
using burgers::DevBuf;
using burgers::InstDesc;
using burgers::SysDesc;
using burgers::Tile;
using burgers::BlockTile;

namespace burgers {

bool explicit_windows(int32_t i, int32_t n, bool periodic, int depth, bool rk4, std::vector<BlockTile>& out) {
  const int cap = explicit_block_capacity();
  // each step consumes one halo node per side per stage
  const int32_t halo = depth * (rk4 ? 4 : 1);
  const int32_t wout = cap - 2 * halo;
  if (wout < 1) return false;
  const int64_t nn = n;
  for (int64_t lo = 0; lo < nn; lo += wout) {
    const int64_t hi = std::min<int64_t>(nn, lo + wout);
    BlockTile bt{i, 0, 0, 0, static_cast<int32_t>(hi - lo), 0, rk4 ? 1 : 0, 0};
    if (periodic) {
      bt.first = static_cast<int32_t>(((lo - halo) % nn + nn) % nn);
      bt.width = static_cast<int32_t>((hi - lo) + 2 * halo);
      bt.lo = halo;
    } else {
      const int64_t first = std::max<int64_t>(0, lo - halo);
      bt.first = static_cast<int32_t>(first);
      bt.width = static_cast<int32_t>(std::min<int64_t>(nn, hi + halo) - first);
      bt.lo = static_cast<int32_t>(lo - first);
    }
    out.push_back(bt);
  }
  return true;
}

void btcs_windows(int32_t i, int32_t R, bool periodic, int W, bool cn, std::vector<WinDesc>& out) {
  const int64_t halo = btcs_window_halo(), kept = W - 2 * halo;
  for (int64_t lo = 0; lo < R; lo += kept) {
    const int64_t hi = std::min<int64_t>(R, lo + kept);
    const int64_t start =
        periodic ? ((lo - halo) % R + R) % R : std::min<int64_t>(std::max<int64_t>(lo - halo, 0), R - W);
    const int64_t rel = periodic ? halo : lo - start;
    out.push_back(WinDesc{i, static_cast<int32_t>(start), static_cast<int32_t>(rel), static_cast<int32_t>(hi - lo),
                          cn ? 1 : 0, 0});
  }
}

}  // namespace burgers

namespace {

// Instance subsets a plan is built for; kSetBtcsHbm holds the BTCS-scheme instances like kSetBtcs but
// steps every one through HBM (the adjoint's out-of-place recompute of a checkpoint segment).
enum SetId { kSetAll = 0, kSetExplicit = 1, kSetBtcs = 2, kSetBtcsHbm = 3 };

bool valid_problem(const burgers_problem& p);
double grid_dx(const burgers_problem& p);

}  // namespace

namespace burgers {

bool problem_valid(const burgers_problem& p) { return valid_problem(p); }

InstDesc inst_desc(const burgers_problem& p, int64_t off) {
  InstDesc d{};
  d.off = off;
  d.n = static_cast<int32_t>(p.n);
  d.bc = p.bc;
  burgers_ratios(&p, &d.r, &d.D);
  const double dxv = grid_dx(p);
  d.dtdx2 = p.dt / (dxv * dxv);
  d.a = p.bc == BURGERS_BC_DIRICHLET ? p.left : 0.0;
  d.b = p.bc == BURGERS_BC_DIRICHLET ? p.right : 0.0;
  return d;
}

}  // namespace burgers

namespace {

bool is_finite(double x) { return std::isfinite(x); }

double grid_dx(const burgers_problem& p) {
  return p.bc == BURGERS_BC_PERIODIC ? p.length / static_cast<double>(p.n)
                                     : p.length / static_cast<double>(p.n - 1);
}

// Largest instance: node indices of a window (first node + up to 8192) and of staged blocks stay within
// 32-bit integers.
constexpr int64_t kMaxNodes = (int64_t{1} << 31) - 65536;

bool valid_problem(const burgers_problem& p) {
  if (p.n < 3 || p.n > kMaxNodes) return false;
  if (!is_finite(p.length) || p.length <= 0) return false;
  if (!is_finite(p.nu) || p.nu < 0) return false;
  if (!is_finite(p.dt) || p.dt <= 0) return false;
  if (p.bc != BURGERS_BC_PERIODIC && p.bc != BURGERS_BC_DIRICHLET) return false;
  if (p.scheme < BURGERS_EXPLICIT || p.scheme > BURGERS_NEWTON) return false;
  if (!is_finite(p.left) || !is_finite(p.right)) return false;
  return true;
}

burgers_status from_hip(hipError_t e) {
  if (e == hipSuccess) return BURGERS_OK;
  if (e == hipErrorOutOfMemory) return BURGERS_E_NOMEM;
  return BURGERS_E_DEVICE;
}

// Record a device error as sticky and translate it.
burgers_status note(burgers_ctx* ctx, hipError_t e) {
  if (e != hipSuccess && ctx->sticky == hipSuccess) ctx->sticky = e;
  return from_hip(e);
}

const std::vector<int32_t>& set_members(const burgers_ctx* ctx, int set) {
  return set == kSetAll ? ctx->set_all : (set == kSetExplicit ? ctx->set_explicit : ctx->set_btcs);
}

bool own_scheme_set(int set) { return set == kSetBtcs || set == kSetBtcsHbm; }

// Copy a host table to a new device buffer, in stream order (a pageable source may be released as soon
// as the call returns).
template <typename T>
hipError_t upload_on(hipStream_t stream, DevBuf& buf, const std::vector<T>& v) {
  hipError_t e = buf.alloc(v.size() * sizeof(T), stream);
  if (e != hipSuccess) return e;
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(buf.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream);
}

// Streaming tiles covering every node of the members of one subset.
std::vector<Tile> stream_tiles(const burgers_ctx* ctx, const std::vector<int32_t>& members) {
  const int tile = burgers::explicit_tile_nodes(ctx->dtype);
  std::vector<Tile> tiles;
  for (int32_t i : members) {
    const int32_t n = static_cast<int32_t>(ctx->probs[i].n);
    for (int64_t s = 0; s < n; s += tile)   // 64-bit counter: n may be close to INT32_MAX
      tiles.push_back(Tile{ctx->offsets[i], n, static_cast<int32_t>(s), ctx->probs[i].bc, i});
  }
  return tiles;
}

// Tiles of a subset used to copy its instances back from the second buffer.
hipError_t ensure_copy(burgers_ctx* ctx, int set) {
  if (ctx->copy_tiles.count(set)) return hipSuccess;
  auto tiles = stream_tiles(ctx, set_members(ctx, set));
  auto buf = std::make_unique<DevBuf>();
  hipError_t e = upload_on(ctx->stream, *buf, tiles);
  if (e != hipSuccess) return e;
  ctx->copy_tiles[set] = {std::move(buf), static_cast<int64_t>(tiles.size())};
  return hipSuccess;
}

// Steps per launch of the explicit windows.  Each launch moves a window through HBM once (load and
// store) and recomputes 2 T halo nodes of its 8192 per step; T = 128 balances the two (3% halo work).
constexpr int kDefaultDepth = 128;
constexpr int kMaxDepth = 512;

// Explicit launch plan of one subset under the context's forced path (0 = automatic).
//   path 1: streaming kernel, one step per launch.
//   path 2: whole instances on chip, all steps in one launch (every instance must fit).
//   path 3: temporal blocking with `depth` steps per launch for every instance.
//   automatic: whole instances for those that fit, windows of `depth` steps for longer ones.
burgers_status ensure_explicit(burgers_ctx* ctx, int set) {
  auto it = ctx->explicit_plans.find(set);
  const int want_path = ctx->plan.explicit_path;
  const int want_depth = ctx->plan.tblock_depth > 0 ? ctx->plan.tblock_depth : kDefaultDepth;
  if (it != ctx->explicit_plans.end() && it->second->path == (want_path ? want_path : 0) &&
      it->second->depth == want_depth)
    return BURGERS_OK;
  auto plan = std::make_unique<burgers::ExplicitPlan>();
  plan->path = want_path ? want_path : 0;
  plan->depth = want_depth;
  const auto& members = set_members(ctx, set);
  // instances advanced by their own scheme (burgers_run) take RK4 where they ask for it; a forward-Euler
  // call (burgers_step_explicit) steps every instance with forward Euler
  auto is_rk4 = [&](int32_t i) { return set == kSetExplicit && ctx->probs[i].scheme == BURGERS_RK4; };
  bool any_rk4 = false;
  for (int32_t i : members) any_rk4 = any_rk4 || is_rk4(i);
  if (plan->path == 1 && any_rk4) return BURGERS_E_UNSUPPORTED;   // the streaming kernel is forward Euler only
  hipError_t e;
  auto st = stream_tiles(ctx, members);
  plan->stream = std::make_unique<DevBuf>();
  if ((e = upload_on(ctx->stream, *plan->stream, st)) != hipSuccess) return from_hip(e);
  plan->n_stream = static_cast<int64_t>(st.size());
  if (plan->path != 1) {
    const int cap = burgers::explicit_block_capacity();
    const int T = plan->depth;
    std::vector<BlockTile> whole, win;
    std::vector<int32_t> windowed;
    for (int32_t i : members) {
      const burgers_problem& p = ctx->probs[i];
      const int32_t n = static_cast<int32_t>(p.n);
      const bool periodic = p.bc == BURGERS_BC_PERIODIC;
      const int32_t rk4 = is_rk4(i) ? 1 : 0;
      if (n <= cap) {
        whole.push_back(BlockTile{i, 0, n, 0, n, periodic ? 1 : 0, rk4});
        continue;
      }
      if (plan->path == 2) return BURGERS_E_UNSUPPORTED;
      windowed.push_back(i);
      if (!burgers::explicit_windows(i, n, periodic, T, rk4 != 0, win)) return BURGERS_E_UNSUPPORTED;
    }
    auto fe_first = [](const BlockTile& x, const BlockTile& y) { return x.rk4 < y.rk4; };
    // whole instances: by workgroup width (widest first), then forward Euler before RK4
    auto lanes_of = [](const BlockTile& x) { return burgers::explicit_block_lanes(x.width); };
    std::stable_sort(whole.begin(), whole.end(), [&](const BlockTile& x, const BlockTile& y) {
      const int lx = lanes_of(x), ly = lanes_of(y);
      return lx != ly ? lx > ly : x.rk4 < y.rk4;
    });
    plan->whole_classes.clear();
    for (size_t k = 0; k < whole.size();) {
      const int lanes = lanes_of(whole[k]);
      size_t e = k;
      int64_t rk4 = 0;
      while (e < whole.size() && lanes_of(whole[e]) == lanes) rk4 += whole[e++].rk4 ? 1 : 0;
      plan->whole_classes.push_back({lanes, static_cast<int64_t>(k), static_cast<int64_t>(e - k) - rk4, rk4});
      k = e;
    }
    // the narrower classes packed for one launch per scheme, 512 / lanes instances of a class per
    // workgroup (widest first); the widest class keeps its own kernel, whose step loop compiles to fewer
    // registers than the pack kernel's (C2, instances of 8192 nodes: 61.9 against 63.9 ms)
    std::vector<burgers::BlockPack> fe_packs, rk4_packs;
    for (const auto& c : plan->whole_classes) {
      if (c.lanes >= burgers::explicit_pack_lanes()) continue;
      const int per = burgers::explicit_pack_lanes() / c.lanes;
      auto pack = [&](int64_t first, int64_t count, std::vector<burgers::BlockPack>& out) {
        for (int64_t q = 0; q < count; q += per)
          out.push_back(burgers::BlockPack{static_cast<int32_t>(first + q),
                                           static_cast<int32_t>(std::min<int64_t>(per, count - q)), c.lanes, 0});
      };
      pack(c.offset, c.n_fe, fe_packs);
      pack(c.offset + c.n_fe, c.n_rk4, rk4_packs);
    }
    plan->n_packs_fe = static_cast<int64_t>(fe_packs.size());
    plan->n_packs_rk4 = static_cast<int64_t>(rk4_packs.size());
    fe_packs.insert(fe_packs.end(), rk4_packs.begin(), rk4_packs.end());
    plan->packs = std::make_unique<DevBuf>();
    if ((e = upload_on(ctx->stream, *plan->packs, fe_packs)) != hipSuccess) return from_hip(e);
    std::stable_sort(win.begin(), win.end(), fe_first);
    plan->whole = std::make_unique<DevBuf>();
    plan->win = std::make_unique<DevBuf>();
    plan->win_copy = std::make_unique<DevBuf>();
    auto wc = stream_tiles(ctx, windowed);
    if ((e = upload_on(ctx->stream, *plan->whole, whole)) != hipSuccess || (e = upload_on(ctx->stream, *plan->win, win)) != hipSuccess ||
        (e = upload_on(ctx->stream, *plan->win_copy, wc)) != hipSuccess)
      return from_hip(e);
    plan->n_whole = static_cast<int64_t>(whole.size());
    plan->n_win = static_cast<int64_t>(win.size());
    plan->n_whole_rk4 = std::count_if(whole.begin(), whole.end(), [](const BlockTile& b) { return b.rk4 != 0; });
    plan->n_win_rk4 = std::count_if(win.begin(), win.end(), [](const BlockTile& b) { return b.rk4 != 0; });
    plan->n_win_copy = static_cast<int64_t>(wc.size());
  }
  ctx->explicit_plans[set] = std::move(plan);
  return BURGERS_OK;
}

// BTCS launch plan of one instance subset under the context's forced path (0 = automatic).
//   path 1: every step through HBM; whole-system solves for systems of up to 8192 rows, partition
//           levels for longer ones.
//   path 2: systems of up to 8192 rows stay on chip for all steps of a launch (every system must fit).
//   path 3: partition levels for every system of at least 32 rows (shorter ones solved whole).
//   automatic: on chip for systems that fit, partition levels for longer ones.
// Reduced-system rows are carved from the context's level arrays.
burgers_status ensure_newton(burgers_ctx* ctx, const std::vector<int32_t>& members);

// Rows a partition level leaves for the next one.  Level 0 (from the state) runs the block partition,
// which reduces each workgroup's 256 chunks to two rows; deeper levels leave two rows per chunk.
int32_t reduced_rows(int level, int32_t chunks) {
  if (level == 0) return 2 * ((chunks + burgers::kReduceBlock - 1) / burgers::kReduceBlock);
  return 2 * chunks;
}

burgers_status ensure_btcs(burgers_ctx* ctx, int set) {
  const int want = set == kSetBtcsHbm ? 1 : ctx->plan.btcs_path;
  const int threads = ctx->plan.btcs_block ? ctx->plan.btcs_block : burgers::kResidentThreadsDefault;
  const int longmode = ctx->plan.btcs_long;
  auto found = ctx->btcs.find(set);
  const bool pipelined = ctx->plan.btcs_pipeline == 1;
  if (found != ctx->btcs.end() && found->second->path == want && found->second->threads == threads &&
      found->second->longmode == longmode && found->second->stream_exact == pipelined)
    return BURGERS_OK;
  auto plan = std::make_unique<burgers::BtcsPlan>();
  plan->path = want;
  plan->threads = threads;
  plan->longmode = longmode;
  plan->stream_exact = pipelined;
  const int cap = burgers::btcs_wg_capacity();
  const int chunk = burgers::btcs_reduce_chunk();
  // truncated windows of the long systems (automatic and per-step paths): 4096 rows each (8192 when
  // asked), keeping all but `halo` rows at either end; the partition levels stay as the fallback for
  // failed bounds.  Narrower windows read 14% more rows than 8192-row ones but take 256-lane workgroups,
  // four per CU instead of two, whose loads, solves and stores overlap better (C3: 52.6 against 60.8 us
  // per step).
  plan->win_rows = longmode == 2 ? cap : 4096;
  std::vector<burgers::WinDesc> windows;
  auto add_windows = [&](int32_t i, int32_t R, bool is_cn) {
    burgers::btcs_windows(i, R, ctx->probs[i].bc == BURGERS_BC_PERIODIC, plan->win_rows, is_cn, windows);
  };
  // whole-system systems grouped by width class (lanes, chunk, exact)
  std::map<std::tuple<int, int, bool>, std::vector<SysDesc>> wg_state, resident, streamed;
  const int64_t elem = ctx->dtype == BURGERS_F64 ? 8 : 4;
  auto whole = [&](std::map<std::tuple<int, int, bool>, std::vector<SysDesc>>& groups, int32_t rows, int32_t i,
                   bool is_cn) {
    const burgers::WidthClass w = burgers::btcs_width_class(rows, threads);
    groups[std::make_tuple(w.lanes, w.chunk, w.exact)].push_back(
        SysDesc{0, -1, rows, burgers::btcs_chunks(rows, w.lanes), i, 0, is_cn ? 1 : 0});
  };
  std::vector<int32_t> stepped, cn, newton;
  std::vector<std::vector<SysDesc>> red_sys, wg_sys;
  int64_t rows_used = 0;
  for (int32_t i : set_members(ctx, set)) {
    const burgers_problem& p = ctx->probs[i];
    const int32_t R0 = static_cast<int32_t>(p.bc == BURGERS_BC_PERIODIC ? p.n : p.n - 2);
    const bool fits = burgers::btcs_solved_whole(R0);
    // Crank-Nicolson instances (advanced by their own scheme) need the old state after each solve, so
    // they always step through HBM
    const bool is_cn = own_scheme_set(set) && p.scheme == BURGERS_CN;
    if (is_cn) cn.push_back(i);
    const bool is_newton = own_scheme_set(set) && p.scheme == BURGERS_NEWTON;
    if (want == 2 && (!fits || is_cn || is_newton)) return BURGERS_E_UNSUPPORTED;
    if (is_newton) {            // Newton iterations of their own, through HBM every step
      stepped.push_back(i);
      newton.push_back(i);
      continue;
    }
    if ((want == 0 || want == 2) && fits && !is_cn) {
      whole(resident, R0, i, false);
      continue;
    }
    stepped.push_back(i);
    const bool partition = want == 3 ? R0 >= 32 : !fits;
    if (!partition) {
      // exact 8192-row systems whose first row is 16-byte aligned may take the pipelined kernel
      const int64_t first = ctx->inst_host[i].off + (p.bc == BURGERS_BC_PERIODIC ? 0 : 1);
      const bool streams = pipelined && !is_cn && R0 == burgers::btcs_wg_capacity() && (first * elem) % 16 == 0;
      whole(streams ? streamed : wg_state, R0, i, is_cn);
      continue;
    }
    if (want != 3 && longmode != 1) add_windows(i, R0, is_cn);
    int32_t R = R0;
    int64_t in_off = 0;
    for (int level = 0;; ++level) {
      if (static_cast<int>(red_sys.size()) <= level) {
        red_sys.resize(level + 1);
        wg_sys.resize(level + 1);
      }
      if (level > 0 && R <= cap) {
        wg_sys[level].push_back(SysDesc{in_off, -1, R, burgers::btcs_wg_chunks(R), i, level});
        break;
      }
      const int32_t P = (R + chunk - 1) / chunk;
      const int32_t out_rows = reduced_rows(level, P);
      const int64_t red = rows_used;
      rows_used += out_rows;
      red_sys[level].push_back(SysDesc{in_off, red, R, P, i, level, (level == 0 && is_cn) ? 1 : 0});
      in_off = red;
      R = out_rows;
    }
  }
  if (rows_used > ctx->level_capacity) return BURGERS_E_NOMEM;   // sized at create for every path
  plan->level_rows = rows_used;
  hipError_t e;
  auto upload_groups = [&](std::map<std::tuple<int, int, bool>, std::vector<SysDesc>>& groups,
                           std::vector<burgers::WgGroup>& out, bool stream) -> hipError_t {
    for (auto& kv : groups) {
      burgers::WgGroup g;
      g.shape = burgers::WidthClass{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), stream};
      g.sys = std::make_unique<DevBuf>();
      g.n = static_cast<int32_t>(kv.second.size());
      hipError_t err = upload_on(ctx->stream, *g.sys, kv.second);
      if (err != hipSuccess) return err;
      out.push_back(std::move(g));
    }
    return hipSuccess;
  };
  plan->copy = std::make_unique<DevBuf>();
  auto ct = stream_tiles(ctx, stepped);
  plan->n_copy = static_cast<int64_t>(ct.size());
  if (!newton.empty()) {
    burgers_status nst = ensure_newton(ctx, newton);
    if (nst != BURGERS_OK) return nst;
    plan->newton = true;
  }
  plan->inst_half = std::make_unique<DevBuf>();
  if (!cn.empty()) {
    std::vector<burgers::InstDesc> half = ctx->inst_host;
    for (int32_t i : cn) {
      half[i].r = 0.5 * half[i].r;               // the BTCS rows of dt/2 (exact: a power of two)
      half[i].D = 0.5 * half[i].D;
    }
    if ((e = upload_on(ctx->stream, *plan->inst_half, half)) != hipSuccess) return from_hip(e);
  }
  if ((e = upload_groups(wg_state, plan->wg_state, false)) != hipSuccess ||
      (e = upload_groups(streamed, plan->wg_state, true)) != hipSuccess ||
      (e = upload_groups(resident, plan->resident, false)) != hipSuccess ||
      (e = upload_on(ctx->stream, *plan->copy, ct)) != hipSuccess)
    return from_hip(e);
  plan->win = std::make_unique<DevBuf>();
  if ((e = upload_on(ctx->stream, *plan->win, windows)) != hipSuccess) return from_hip(e);
  plan->n_win = static_cast<int64_t>(windows.size());
  if (plan->n_win > 0 &&
      (e = plan->win_flags.alloc(static_cast<size_t>(burgers::win_flags_words(ctx->count)) * sizeof(int), ctx->stream)) !=
          hipSuccess)
    return from_hip(e);
  plan->levels.resize(red_sys.size());
  for (size_t l = 0; l < red_sys.size(); ++l) {
    auto& lv = plan->levels[l];
    std::vector<ChunkBlock> blocks;
    for (size_t si = 0; si < red_sys[l].size(); ++si)
      for (int64_t c = 0; c < red_sys[l][si].chunks; c += burgers::kReduceBlock)
        blocks.push_back(ChunkBlock{static_cast<int32_t>(si), static_cast<int32_t>(c)});
    lv.sys = std::make_unique<DevBuf>();
    lv.blocks = std::make_unique<DevBuf>();
    lv.wg = std::make_unique<DevBuf>();
    if ((e = upload_on(ctx->stream, *lv.sys, red_sys[l])) != hipSuccess || (e = upload_on(ctx->stream, *lv.blocks, blocks)) != hipSuccess ||
        (e = upload_on(ctx->stream, *lv.wg, wg_sys[l])) != hipSuccess)
      return from_hip(e);
    lv.n_blocks = static_cast<int32_t>(blocks.size());
    lv.n_wg = static_cast<int32_t>(wg_sys[l].size());
    lv.wg_lanes = burgers::btcs_wg_lanes(wg_sys[l]);
    lv.wg_exact = burgers::btcs_wg_exact(wg_sys[l]);
  }
  ctx->btcs[set] = std::move(plan);
  return BURGERS_OK;
}

// Rows of the partition levels the instances can need on any path (sizes the level arrays).
int64_t level_rows_needed(const burgers_ctx* ctx) {
  const int cap = burgers::btcs_wg_capacity();
  const int chunk = burgers::btcs_reduce_chunk();
  int64_t rows = 0;
  for (const auto& p : ctx->probs) {
    int64_t R = p.bc == BURGERS_BC_PERIODIC ? p.n : p.n - 2;
    if (R < 32) continue;                      // partition levels serve systems of >= 32 rows
    for (int level = 0;; ++level) {
      if (level > 0 && R <= cap) break;
      const int64_t P = (R + chunk - 1) / chunk;
      const int64_t out_rows = reduced_rows(level, static_cast<int32_t>(P));
      rows += out_rows;
      R = out_rows;
    }
  }
  return rows;
}

// Independent launch groups of a call (they advance disjoint instances): the whole instances held on chip,
// and the instances stepped through HBM (windows, per-step solves), of each scheme.
enum Part { kPartAll = 0, kPartOnChip = 1, kPartThroughHbm = 2 };

// Enqueue nsteps explicit steps of one subset (or of one part of it); the final state lands in u.
hipError_t enqueue_explicit(burgers_ctx* ctx, int set, void* u, int64_t nsteps, int part = kPartAll) {
  const burgers::ExplicitPlan& pl = *ctx->explicit_plans[set];
  void* work = ctx->work.ptr;
  hipError_t e = hipSuccess;
  if (pl.path == 1) {
    if (part == kPartOnChip) return e;
    void* bufs[2] = {u, work};
    int cur = 0;
    for (int64_t s = 0; s < nsteps; ++s) {
      if ((e = burgers::launch_explicit_stream(ctx, pl.stream->as<Tile>(), pl.n_stream, bufs[cur], bufs[cur ^ 1])) != hipSuccess)
        return e;
      cur ^= 1;
    }
    if (cur) e = burgers::launch_copy_tiles(ctx, pl.stream->as<Tile>(), pl.n_stream, work, u);
    return e;
  }
  // whole instances, in place: all steps at once, or `depth` per launch on path 3
  const int64_t whole_chunk = pl.path == 3 ? pl.depth : (int64_t{1} << 30);
  for (int64_t done = 0; part != kPartThroughHbm && done < nsteps;) {
    const int k = static_cast<int>(std::min(whole_chunk, nsteps - done));
    for (const auto& c : pl.whole_classes)
      if (c.lanes >= burgers::explicit_pack_lanes() &&
          (e = burgers::launch_explicit_block(ctx, pl.whole->as<BlockTile>() + c.offset, c.n_fe, c.n_rk4, u, u, k,
                                              c.lanes)) != hipSuccess)
        return e;
    if ((e = burgers::launch_explicit_packs(ctx, pl.whole->as<BlockTile>(), pl.packs->as<burgers::BlockPack>(),
                                            pl.n_packs_fe, pl.n_packs_rk4, u, k)) != hipSuccess)
      return e;
    done += k;
  }
  // windows of long instances: `depth` steps per launch, ping-pong
  if (pl.n_win > 0 && part != kPartOnChip) {
    void* bufs[2] = {u, work};
    int cur = 0;
    for (int64_t done = 0; done < nsteps;) {
      const int k = static_cast<int>(std::min<int64_t>(pl.depth, nsteps - done));
      if ((e = burgers::launch_explicit_block(ctx, pl.win->as<BlockTile>(), pl.n_win - pl.n_win_rk4, pl.n_win_rk4,
                                              bufs[cur], bufs[cur ^ 1], k)) != hipSuccess)
        return e;
      cur ^= 1;
      done += k;
    }
    if (cur) e = burgers::launch_copy_tiles(ctx, pl.win_copy->as<Tile>(), pl.n_win_copy, work, u);
  }
  return e;
}

// Enqueue nsteps BTCS steps of one subset (or of one part of it); the final state lands in u.
hipError_t enqueue_btcs(burgers_ctx* ctx, int set, void* u, int64_t nsteps, int part = kPartAll) {
  const burgers::BtcsPlan& pl = *ctx->btcs[set];
  hipError_t e = hipSuccess;
  for (int64_t done = 0; part != kPartThroughHbm && done < nsteps;) {   // on-chip systems, in place
    const int k = static_cast<int>(std::min<int64_t>(nsteps - done, int64_t{1} << 30));
    for (const burgers::WgGroup& g : pl.resident)
      if ((e = burgers::launch_btcs_resident(ctx, g, u, k)) != hipSuccess) return e;
    done += k;
  }
  if (pl.n_copy == 0 || part == kPartOnChip) return e;
  void* bufs[2] = {u, ctx->work.ptr};
  int cur = 0;
  if (nsteps > 0 && (e = burgers::launch_btcs_window_reset(ctx, pl)) != hipSuccess) return e;
  for (int64_t s = 0; s < nsteps; ++s) {
    if ((e = burgers::launch_btcs_step(ctx, pl, bufs[cur], bufs[cur ^ 1], s)) != hipSuccess) return e;
    if (pl.newton) {
      burgers::NewtonPlan& np = *ctx->newton;
      const burgers::AdjTile* nt = np.tiles->as<burgers::AdjTile>();
      if ((e = burgers::launch_newton_init(ctx, nt, np.n_tiles, bufs[cur], bufs[cur ^ 1])) != hipSuccess) return e;
      const burgers::AdjTile* lt = np.long_tiles->as<burgers::AdjTile>();
      int* flags = np.flags.as<int>();
      for (int it = 0; it < burgers::kNewtonIters; ++it) {
        const bool last = it == burgers::kNewtonIters - 1;
        for (const burgers::WgGroup& g : np.whole)
          if ((e = burgers::launch_newton_whole(ctx, g, bufs[cur], bufs[cur ^ 1], last, flags)) != hipSuccess) return e;
        if (np.n_long_tiles == 0) continue;
        if ((e = burgers::launch_newton_assemble(ctx, lt, np.n_long_tiles, bufs[cur], bufs[cur ^ 1], np.NA.as<double>(),
                                                 np.NC.as<double>(), np.ND.as<double>(), flags)) != hipSuccess ||
            (e = burgers::launch_array_solve(ctx, np.solve, np.NA.as<double>(), np.NC.as<double>(), np.ND.as<double>(),
                                             np.NX.as<double>())) != hipSuccess ||
            (e = burgers::launch_newton_update(ctx, lt, np.n_long_tiles, bufs[cur], bufs[cur ^ 1], np.NX.as<double>(),
                                               last, flags)) != hipSuccess)
          return e;
      }
    }
    cur ^= 1;
  }
  if (cur) e = burgers::launch_copy_tiles(ctx, pl.copy->as<Tile>(), pl.n_copy, ctx->work.ptr, u);
  return e;
}

// Whether a part of a plan launches anything.
bool explicit_part_busy(const burgers::ExplicitPlan& pl, int part) {
  if (pl.path == 1) return part != kPartOnChip && pl.n_stream > 0;
  return part == kPartOnChip ? !pl.whole_classes.empty() : pl.n_win > 0;
}
bool btcs_part_busy(const burgers::BtcsPlan& pl, int part) {
  return part == kPartOnChip ? !pl.resident.empty() : pl.n_copy > 0;
}

// scheme -1: each instance's own scheme, explicit instances nsteps steps and BTCS ones nsteps_btcs.
// The independent parts (on-chip and through-HBM instances of each scheme) run concurrently: the first on
// the context's stream, the others on side streams forked from it and joined back with events (under
// graph capture they become parallel branches of the graph), unless the plan asks for one stream.
hipError_t enqueue_all(burgers_ctx* ctx, int set, int scheme, void* u, int64_t nsteps, int64_t nsteps_btcs = -1) {
  if (nsteps_btcs < 0) nsteps_btcs = nsteps;
  struct Group {
    bool btcs;
    int set, part;
    int64_t steps;
  };
  std::vector<Group> groups;
  const bool mixed = scheme < 0;
  const int es = mixed ? kSetExplicit : set, bs = mixed ? kSetBtcs : set;
  const bool want_exp = scheme == BURGERS_EXPLICIT || (mixed && !ctx->set_explicit.empty() && nsteps > 0);
  const bool want_btcs = scheme == BURGERS_BTCS || (mixed && !ctx->set_btcs.empty() && nsteps_btcs > 0);
  const int64_t bsteps = mixed ? nsteps_btcs : nsteps;
  for (int part : {kPartOnChip, kPartThroughHbm}) {
    if (want_exp && explicit_part_busy(*ctx->explicit_plans[es], part)) groups.push_back({false, es, part, nsteps});
    if (want_btcs && btcs_part_busy(*ctx->btcs[bs], part)) groups.push_back({true, bs, part, bsteps});
  }
  auto run = [&](const Group& g) {
    return g.btcs ? enqueue_btcs(ctx, g.set, u, g.steps, g.part) : enqueue_explicit(ctx, g.set, u, g.steps, g.part);
  };
  if (groups.size() <= 1 || ctx->plan.serial == 1) {
    for (const Group& g : groups) {
      hipError_t e = run(g);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t e;
  const size_t nside = groups.size() - 1;
  for (size_t k = 0; k < nside; ++k) {
    if (!ctx->side[k] && (e = hipStreamCreateWithFlags(&ctx->side[k], hipStreamNonBlocking)) != hipSuccess) return e;
    if (!ctx->joined[k] && (e = hipEventCreateWithFlags(&ctx->joined[k], hipEventDisableTiming)) != hipSuccess)
      return e;
  }
  if (!ctx->forked && (e = hipEventCreateWithFlags(&ctx->forked, hipEventDisableTiming)) != hipSuccess) return e;
  hipStream_t main = ctx->stream;
  if ((e = hipEventRecord(ctx->forked, main)) != hipSuccess) return e;
  hipError_t err = hipSuccess;
  for (size_t k = 0; k < nside && err == hipSuccess; ++k) {
    if ((err = hipStreamWaitEvent(ctx->side[k], ctx->forked, 0)) != hipSuccess) break;
    ctx->stream = ctx->side[k];
    err = run(groups[k + 1]);
    ctx->stream = main;
    if (err == hipSuccess) err = hipEventRecord(ctx->joined[k], ctx->side[k]);
    if (err == hipSuccess) err = hipStreamWaitEvent(main, ctx->joined[k], 0);
  }
  ctx->stream = main;
  if (err != hipSuccess) return err;
  return run(groups[0]);
}

burgers_status prepare(burgers_ctx* ctx, int set, int scheme) {
  burgers_status st;
  hipError_t e;
  const bool need_explicit = scheme == BURGERS_EXPLICIT || (scheme < 0 && !ctx->set_explicit.empty());
  const bool need_btcs = scheme == BURGERS_BTCS || (scheme < 0 && !ctx->set_btcs.empty());
  const int es = scheme < 0 ? kSetExplicit : set;
  const int bs = scheme < 0 ? kSetBtcs : set;
  if (need_explicit && (st = ensure_explicit(ctx, es)) != BURGERS_OK) return st;
  if (need_btcs && (st = ensure_btcs(ctx, bs)) != BURGERS_OK) return st;
  (void)e;
  return BURGERS_OK;
}

// Replay the launch sequence of (set, scheme, steps, u) from a captured graph, capturing it on first use.
hipError_t enqueue_graph(burgers_ctx* ctx, int set, int scheme, void* u, int64_t nsteps, int64_t nsteps_btcs) {
  const auto key = std::make_tuple(set, scheme, nsteps, nsteps_btcs, u);
  auto it = ctx->graph_cache.find(key);
  if (it == ctx->graph_cache.end()) {
    hipError_t e;
    if (!ctx->capture_stream &&
        (e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking)) != hipSuccess)
      return e;
    hipStream_t user = ctx->stream;
    ctx->stream = ctx->capture_stream;
    if ((e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
      ctx->stream = user;
      return e;
    }
    hipError_t le = enqueue_all(ctx, set, scheme, u, nsteps, nsteps_btcs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->capture_stream, &graph);
    ctx->stream = user;
    if (le != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return le; }
    if (e != hipSuccess) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    it = ctx->graph_cache.emplace(key, exec).first;
  }
  return hipGraphLaunch(it->second, ctx->stream);
}

// nsteps steps of `set` with `scheme` (-1: each instance's own; BTCS instances then take nsteps_btcs
// steps); the final state lands in u.
burgers_status advance(burgers_ctx* ctx, void* u, int64_t nsteps, int set, int scheme, int64_t nsteps_btcs = -1) {
  if (nsteps_btcs < 0) nsteps_btcs = nsteps;
  if (!ctx || !u || nsteps < 0) return BURGERS_E_INVALID;
  if (ctx->sticky != hipSuccess) return from_hip(ctx->sticky);
  if (nsteps == 0 && (scheme >= 0 || nsteps_btcs == 0)) return BURGERS_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return note(ctx, e);
  burgers_status st = prepare(ctx, set, scheme);
  if (st != BURGERS_OK) return st == BURGERS_E_UNSUPPORTED || st == BURGERS_E_INVALID ? st : note(ctx, hipErrorOutOfMemory);
  if (ctx->plan.use_graph == 1) e = enqueue_graph(ctx, set, scheme, u, nsteps, nsteps_btcs);
  else e = enqueue_all(ctx, set, scheme, u, nsteps, nsteps_btcs);
  if (e != hipSuccess) return note(ctx, e);
  return BURGERS_OK;
}


// Adjoint launch lists: 256-node tiles of every instance (explicit and BTCS lists), one dJ/dD slot per
// tile, and the partition hierarchy over the transposed BTCS systems, which sit at the start of the
// adjoint arrays followed by their reduced rows.
// Partition hierarchy for systems stored as unit-diagonal rows in binary64 arrays: root (instance, row
// offset, rows) triples; systems of up to 8192 rows are solved whole, longer ones reduced by chunk-
// partition levels whose reduced rows are appended after `rows_used` (updated).
hipError_t build_array_solve(burgers_ctx* ctx, const std::vector<std::tuple<int32_t, int64_t, int32_t>>& roots,
                             burgers::BtcsPlan& plan, int64_t& rows_used) {
  const int cap = burgers::btcs_wg_capacity();
  const int chunk = burgers::btcs_reduce_chunk();
  std::vector<std::vector<SysDesc>> red_sys(1), wg_sys(1);
  for (const auto& root : roots) {
    const int32_t i = std::get<0>(root);
    int64_t in_off = std::get<1>(root);
    int32_t R = std::get<2>(root);
    for (int level = 0;; ++level) {
      if (static_cast<int>(red_sys.size()) <= level) {
        red_sys.resize(level + 1);
        wg_sys.resize(level + 1);
      }
      if (R <= cap) {
        wg_sys[level].push_back(SysDesc{in_off, -1, R, burgers::btcs_chunks(R, 512), i, level});
        break;
      }
      const int32_t P = (R + chunk - 1) / chunk;
      const int64_t red = rows_used;
      rows_used += 2 * static_cast<int64_t>(P);
      red_sys[level].push_back(SysDesc{in_off, red, R, P, i, level});
      in_off = red;
      R = 2 * P;
    }
  }
  hipError_t e;
  plan.levels.resize(red_sys.size());
  for (size_t l = 0; l < red_sys.size(); ++l) {
    auto& lv = plan.levels[l];
    std::vector<ChunkBlock> blocks;
    for (size_t si = 0; si < red_sys[l].size(); ++si)
      for (int64_t c = 0; c < red_sys[l][si].chunks; c += burgers::kReduceBlock)
        blocks.push_back(ChunkBlock{static_cast<int32_t>(si), static_cast<int32_t>(c)});
    lv.sys = std::make_unique<DevBuf>();
    lv.blocks = std::make_unique<DevBuf>();
    lv.wg = std::make_unique<DevBuf>();
    if ((e = upload_on(ctx->stream, *lv.sys, red_sys[l])) != hipSuccess ||
        (e = upload_on(ctx->stream, *lv.blocks, blocks)) != hipSuccess ||
        (e = upload_on(ctx->stream, *lv.wg, wg_sys[l])) != hipSuccess)
      return e;
    lv.n_blocks = static_cast<int32_t>(blocks.size());
    lv.n_wg = static_cast<int32_t>(wg_sys[l].size());
    lv.wg_lanes = burgers::btcs_wg_lanes(wg_sys[l]);
    lv.wg_exact = burgers::btcs_wg_exact(wg_sys[l]);
  }
  return hipSuccess;
}

// Newton plan over the given instances (built once per context): systems of up to 8192 rows iterate in
// one fused kernel per iteration (grouped by width class), longer ones through the array path.
burgers_status ensure_newton(burgers_ctx* ctx, const std::vector<int32_t>& members) {
  if (ctx->newton) return BURGERS_OK;
  auto np = std::make_unique<burgers::NewtonPlan>();
  const int cap = burgers::btcs_wg_capacity();
  std::vector<burgers::AdjTile> tiles, long_tiles;
  std::vector<std::tuple<int32_t, int64_t, int32_t>> roots;
  std::map<std::tuple<int, int, bool>, std::vector<SysDesc>> groups;
  int64_t rows = 0;
  for (int32_t i : members) {
    const burgers_problem& p = ctx->probs[i];
    const int32_t n = static_cast<int32_t>(p.n);
    const int32_t R = p.bc == BURGERS_BC_PERIODIC ? n : n - 2;
    for (int64_t s0 = 0; s0 < n; s0 += 256)
      tiles.push_back(burgers::AdjTile{ctx->offsets[i], 0, n, p.bc, i, static_cast<int32_t>(s0), 0, 0});
    if (R <= cap) {
      // 8192-row systems take 1024 lanes of 8 rows (the Newton rows need more registers than BTCS ones)
      const burgers::WidthClass w = burgers::btcs_width_class(R, 1024);
      groups[std::make_tuple(w.lanes, w.chunk, w.exact)].push_back(
          SysDesc{0, -1, R, burgers::btcs_chunks(R, w.lanes), i, 0});
      continue;
    }
    for (int64_t s0 = 0; s0 < n; s0 += 256)
      long_tiles.push_back(burgers::AdjTile{ctx->offsets[i], rows, n, p.bc, i, static_cast<int32_t>(s0), 0, 0});
    roots.emplace_back(i, rows, R);
    rows += R;
  }
  int64_t rows_used = rows;
  hipError_t e;
  np->tiles = std::make_unique<DevBuf>();
  np->long_tiles = std::make_unique<DevBuf>();
  if ((e = upload_on(ctx->stream, *np->tiles, tiles)) != hipSuccess ||
      (e = upload_on(ctx->stream, *np->long_tiles, long_tiles)) != hipSuccess)
    return from_hip(e);
  np->n_tiles = static_cast<int64_t>(tiles.size());
  np->n_long_tiles = static_cast<int64_t>(long_tiles.size());
  for (auto& kv : groups) {
    burgers::WgGroup g;
    g.shape = burgers::WidthClass{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first)};
    g.sys = std::make_unique<DevBuf>();
    g.n = static_cast<int32_t>(kv.second.size());
    if ((e = upload_on(ctx->stream, *g.sys, kv.second)) != hipSuccess) return from_hip(e);
    np->whole.push_back(std::move(g));
  }
  if ((e = build_array_solve(ctx, roots, np->solve, rows_used)) != hipSuccess) return from_hip(e);
  const size_t lb = static_cast<size_t>(rows_used) * sizeof(double);
  if ((e = np->NA.alloc(lb, ctx->stream)) != hipSuccess || (e = np->NC.alloc(lb, ctx->stream)) != hipSuccess ||
      (e = np->ND.alloc(lb, ctx->stream)) != hipSuccess || (e = np->NX.alloc(lb, ctx->stream)) != hipSuccess ||
      (e = np->flags.alloc(2 * sizeof(int), ctx->stream)) != hipSuccess ||
      (e = hipMemsetAsync(np->flags.ptr, 0, 2 * sizeof(int), ctx->stream)) != hipSuccess)
    return from_hip(e);
  ctx->newton = std::move(np);
  return BURGERS_OK;
}

burgers_status ensure_adjoint(burgers_ctx* ctx) {
  if (ctx->adjoint) return BURGERS_OK;
  auto ap = std::make_unique<burgers::AdjointPlan>();
  const int btcs_tile = burgers::adjoint_tile_nodes();
  std::vector<burgers::AdjTile> bt;
  std::vector<burgers::AdjWindow> ew;
  std::vector<int32_t> slot_begin(ctx->count + 1, 0);
  int32_t slot = 0;
  int64_t sys_rows = 0;
  std::vector<int64_t> sys_off(ctx->count, -1);
  for (int32_t i = 0; i < ctx->count; ++i) {
    const burgers_problem& p = ctx->probs[i];
    if (p.scheme == BURGERS_BTCS) {
      sys_off[i] = sys_rows;
      sys_rows += p.bc == BURGERS_BC_PERIODIC ? p.n : p.n - 2;
    }
  }
  std::vector<std::tuple<int32_t, int64_t, int32_t>> roots;
  int64_t rows_used = sys_rows;
  // every BTCS instance of exactly 16384 rows: each transposed system solved whole; otherwise windows of
  // the transposed systems when every BTCS instance is longer than 8192 rows
  bool whole = !ctx->set_btcs.empty();
  for (int32_t i : ctx->set_btcs) {
    const burgers_problem& p = ctx->probs[i];
    whole = whole && (p.bc == BURGERS_BC_PERIODIC ? p.n : p.n - 2) == burgers::btcs_whole_capacity();
  }
  bool windows = false;
  for (int32_t i : ctx->set_btcs) {
    const burgers_problem& p = ctx->probs[i];
    windows = !whole && (p.bc == BURGERS_BC_PERIODIC ? p.n : p.n - 2) > burgers::btcs_wg_capacity();
    if (!windows) break;
  }
  std::vector<burgers::WinDesc> wins, wholes;
  std::vector<int32_t> win_slot, whole_slot;
  for (int32_t i = 0; i < ctx->count; ++i) {
    const burgers_problem& p = ctx->probs[i];
    const int32_t n = static_cast<int32_t>(p.n);
    const int32_t R = static_cast<int32_t>(p.bc == BURGERS_BC_PERIODIC ? p.n : p.n - 2);
    slot_begin[i] = slot;
    if (p.scheme != BURGERS_BTCS) {
      // explicit: one slot per tile of kAdjSumTile nodes; the whole instance in one window, or windows
      // keeping kAdjWinNodes - 2 kAdjHalo nodes (whole tiles) with kAdjHalo more on either side
      constexpr int32_t H = burgers::kAdjHalo, kept = burgers::kAdjWinNodes - 2 * burgers::kAdjHalo;
      static_assert(kept % burgers::kAdjSumTile == 0, "windows keep whole tiles");
      if (n <= burgers::kAdjWinNodes) {
        ew.push_back(burgers::AdjWindow{i, 0, n, 0, n, slot});
      } else {
        for (int32_t lo = 0; lo < n; lo += kept) {
          const int32_t hi = std::min(n, lo + kept);
          if (p.bc == BURGERS_BC_PERIODIC) {
            ew.push_back(burgers::AdjWindow{i, ((lo - H) % n + n) % n, (hi - lo) + 2 * H, H, hi - lo,
                                            slot + lo / burgers::kAdjSumTile});
          } else {
            const int32_t first = std::max(0, lo - H), end = std::min(n, hi + H);
            ew.push_back(burgers::AdjWindow{i, first, end - first, lo - first, hi - lo,
                                            slot + lo / burgers::kAdjSumTile});
          }
        }
      }
      slot += (n + burgers::kAdjSumTile - 1) / burgers::kAdjSumTile;
      continue;
    }
    for (int64_t s = 0; s < n; s += btcs_tile)
      bt.push_back(burgers::AdjTile{ctx->offsets[i], sys_off[i], n, p.bc, i, static_cast<int32_t>(s), slot++, 0});
    {
      roots.emplace_back(i, sys_off[i], R);
      if (windows) {
        const size_t w0 = wins.size();
        burgers::btcs_windows(i, R, p.bc == BURGERS_BC_PERIODIC, 4096, false, wins);
        for (size_t w = w0; w < wins.size(); ++w) win_slot.push_back(slot++);
      }
      if (whole) {
        wholes.push_back(burgers::WinDesc{i, 0, 0, R, 0, 0});
        whole_slot.push_back(slot++);
      }
    }
  }
  slot_begin[ctx->count] = slot;
  hipError_t e;
  // windows of periodic instances first (their launch compiles no boundary cases)
  std::stable_partition(ew.begin(), ew.end(), [&](const burgers::AdjWindow& w) {
    return ctx->probs[w.inst].bc == BURGERS_BC_PERIODIC;
  });
  ap->n_exp_wins_periodic = std::count_if(ew.begin(), ew.end(), [&](const burgers::AdjWindow& w) {
    return ctx->probs[w.inst].bc == BURGERS_BC_PERIODIC;
  });
  ap->exp_wins = std::make_unique<DevBuf>();
  ap->btcs_tiles = std::make_unique<DevBuf>();
  ap->slot_begin = std::make_unique<DevBuf>();
  if ((e = upload_on(ctx->stream, *ap->exp_wins, ew)) != hipSuccess || (e = upload_on(ctx->stream, *ap->btcs_tiles, bt)) != hipSuccess ||
      (e = upload_on(ctx->stream, *ap->slot_begin, slot_begin)) != hipSuccess)
    return from_hip(e);
  ap->n_exp_wins = static_cast<int64_t>(ew.size());
  ap->n_btcs_tiles = static_cast<int64_t>(bt.size());
  ap->n_slots = slot;
  ap->whole = std::make_unique<DevBuf>();
  ap->whole_slot = std::make_unique<DevBuf>();
  if ((e = upload_on(ctx->stream, *ap->whole, wholes)) != hipSuccess ||
      (e = upload_on(ctx->stream, *ap->whole_slot, whole_slot)) != hipSuccess)
    return from_hip(e);
  ap->n_whole = static_cast<int64_t>(wholes.size());
  ap->win = std::make_unique<DevBuf>();
  ap->win_slot = std::make_unique<DevBuf>();
  if ((e = upload_on(ctx->stream, *ap->win, wins)) != hipSuccess ||
      (e = upload_on(ctx->stream, *ap->win_slot, win_slot)) != hipSuccess)
    return from_hip(e);
  ap->n_win = static_cast<int64_t>(wins.size());
  if (ap->n_win > ap->n_btcs_tiles) return BURGERS_E_UNSUPPORTED;   // (tiles of 1024 nodes outnumber windows)
  if (ap->n_win > 0 && ((e = ap->wpart.alloc(static_cast<size_t>(ap->n_win) * sizeof(double), ctx->stream)) != hipSuccess ||
                        (e = ap->flags.alloc(static_cast<size_t>(burgers::win_flags_words(ctx->count)) * sizeof(int),
                                                          ctx->stream)) != hipSuccess))
    return from_hip(e);
  if ((e = build_array_solve(ctx, roots, ap->solve, rows_used)) != hipSuccess) return from_hip(e);
  const size_t lb = static_cast<size_t>(rows_used) * sizeof(double);
  if ((e = ap->LA.alloc(lb, ctx->stream)) != hipSuccess || (e = ap->LC.alloc(lb, ctx->stream)) != hipSuccess ||
      (e = ap->LD.alloc(lb, ctx->stream)) != hipSuccess || (e = ap->LX.alloc(lb, ctx->stream)) != hipSuccess ||
      (e = ap->gslot.alloc(static_cast<size_t>(std::max<int64_t>(slot, 1)) * sizeof(double), ctx->stream)) != hipSuccess)
    return from_hip(e);
  ctx->adjoint = std::move(ap);
  return BURGERS_OK;
}

hipError_t grow(DevBuf& b, size_t bytes, hipStream_t stream) {
  if (b.bytes >= bytes && b.ptr) return hipSuccess;
  return b.alloc(bytes, stream);
}

// One adjoint step of the BTCS instances: lam_out from lam_in at the forward pair (y = u^k, x = u^{k+1});
// `step` counts the BTCS steps of the reverse sweep (it selects the parity slot of the window flags).
hipError_t enqueue_adjoint_step(burgers_ctx* ctx, const double* y, const double* x, const double* lam_in,
                                double* lam_out, int64_t step) {
  burgers::AdjointPlan& ap = *ctx->adjoint;
  double* g = ap.gslot.as<double>();
  hipError_t e = hipSuccess;
  if (ap.n_btcs_tiles == 0) return e;
  if (ap.n_whole > 0)   // every BTCS system solved whole and exactly: nothing is left for the array path
    return burgers::launch_adj_btcs_whole(ctx, ap.whole->as<burgers::WinDesc>(), ap.n_whole, y, x, 0, 0, 1, lam_in,
                                          lam_out,
                                          g, ap.whole_slot->as<int32_t>());
  const int* only = nullptr;
  if (ap.n_win > 0) {
    int* now = burgers::win_flag_slot(ap.flags.as<int>(), ctx->count, step);
    int* next = burgers::win_flag_slot(ap.flags.as<int>(), ctx->count, step + 1);
    if ((e = burgers::launch_adj_btcs_windows(ctx, ap.win->as<burgers::WinDesc>(), ap.n_win, y, x, lam_in, lam_out,
                                              ap.wpart.as<double>(), now, next)) != hipSuccess)
      return e;
    only = now;
  }
  if ((e = burgers::launch_adj_btcs_assemble(ctx, ap.btcs_tiles->as<burgers::AdjTile>(), ap.n_btcs_tiles, y,
                                             lam_in, ap.LA.as<double>(), ap.LC.as<double>(),
                                             ap.LD.as<double>(), only)) != hipSuccess)
    return e;
  if ((e = burgers::launch_array_solve(ctx, ap.solve, ap.LA.as<double>(), ap.LC.as<double>(), ap.LD.as<double>(),
                                       ap.LX.as<double>(), only)) != hipSuccess)
    return e;
  return burgers::launch_adj_btcs_finish(ctx, ap.btcs_tiles->as<burgers::AdjTile>(), ap.n_btcs_tiles, y, x,
                                         ap.LX.as<double>(), lam_out, g, only, ap.win->as<burgers::WinDesc>(),
                                         ap.n_win, ap.win_slot->as<int32_t>(), ap.wpart.as<double>());
}

// A context for `count` problems on the current device: validated, laid out, its workspace allocated
// (or carved from the installed arena).  *out is set only on success.
burgers_status new_context(const burgers_problem* problems, int64_t count, burgers_dtype dtype, void* hip_stream,
                           burgers_ctx** out) {
  if (!problems || count < 1 || (dtype != BURGERS_F32 && dtype != BURGERS_F64))
    return BURGERS_E_INVALID;
  for (int64_t i = 0; i < count; ++i)
    if (!valid_problem(problems[i])) return BURGERS_E_INVALID;
  if (count > INT32_MAX) return BURGERS_E_INVALID;
  burgers_ctx* ctx = new (std::nothrow) burgers_ctx();
  if (!ctx) return BURGERS_E_NOMEM;
  hipError_t e = hipGetDevice(&ctx->device);
  if (e != hipSuccess) { delete ctx; return BURGERS_E_DEVICE; }
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->dtype = dtype;
  ctx->word = dtype == BURGERS_F64 ? 8 : 4;
  ctx->count = count;
  ctx->probs.assign(problems, problems + count);
  ctx->offsets.resize(count + 1);
  ctx->offsets[0] = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t padded = (problems[i].n + BURGERS_ALIGN - 1) / BURGERS_ALIGN * BURGERS_ALIGN;
    ctx->offsets[i + 1] = ctx->offsets[i] + padded;
  }
  ctx->total = ctx->offsets[count];
  ctx->inst_host.resize(count);
  for (int64_t i = 0; i < count; ++i) {
    const burgers_problem& p = problems[i];
    ctx->inst_host[i] = burgers::inst_desc(p, ctx->offsets[i]);
    ctx->set_all.push_back(static_cast<int32_t>(i));
    (p.scheme == BURGERS_EXPLICIT || p.scheme == BURGERS_RK4 ? ctx->set_explicit : ctx->set_btcs)
        .push_back(static_cast<int32_t>(i));
  }
  burgers_status st = BURGERS_OK;
  if ((e = upload_on(ctx->stream, ctx->inst, ctx->inst_host)) != hipSuccess) st = from_hip(e);
  if (st == BURGERS_OK && (e = ctx->work.alloc(static_cast<size_t>(ctx->total) * ctx->word, ctx->stream)) != hipSuccess)
    st = from_hip(e);
  if (st == BURGERS_OK) {
    ctx->level_capacity = level_rows_needed(ctx);
    const size_t lb = static_cast<size_t>(ctx->level_capacity) * sizeof(double);   // binary64 solve
    if ((e = ctx->level_a.alloc(lb, ctx->stream)) != hipSuccess || (e = ctx->level_c.alloc(lb, ctx->stream)) != hipSuccess ||
        (e = ctx->level_d.alloc(lb, ctx->stream)) != hipSuccess || (e = ctx->level_x.alloc(lb, ctx->stream)) != hipSuccess)
      st = from_hip(e);
  }
  if (st != BURGERS_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return BURGERS_OK;
}

// ---- Static scratch: the workspace of burgers_run_static -------------------------------------------
// A file-scope device array, one copy per GPU the library runs on, held until the process ends.  Host
// code never passes the array's name to a kernel or a copy (on the host it is only a stand-in for the
// symbol): its device address is looked up once per device with that device current, and every use
// goes through that address.
__device__ __align__(256) unsigned char scratch[BURGERS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
void* scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_ptr[device] = p;
  }
  *out = scratch_ptr[device];
  return hipSuccess;
}

// Installs an arena on the calling thread for the lifetime of the guard.
struct ArenaGuard {
  explicit ArenaGuard(burgers::Arena* a) { burgers::tl_arena = a; }
  ~ArenaGuard() { burgers::tl_arena = nullptr; }
};

}  // namespace

extern "C" {

int32_t burgers_abi_version(void) { return BURGERS_ABI_VERSION; }

const char* burgers_status_string(burgers_status s) {
  switch (s) {
    case BURGERS_OK: return "ok";
    case BURGERS_E_INVALID: return "invalid argument";
    case BURGERS_E_UNSUPPORTED: return "unsupported request";
    case BURGERS_E_NOMEM: return "out of device memory";
    case BURGERS_E_DEVICE: return "device error";
    case BURGERS_E_NONFINITE: return "non-finite value";
    case BURGERS_E_BUDGET: return "memory budget exceeded";
    case BURGERS_E_NOT_CONVERGED: return "Newton step not converged or Jacobian not diagonally dominant";
    case BURGERS_E_BOUND: return "truncated-window step outside its accuracy bound";
  }
  return "unknown status";
}

double burgers_cfl_dt(const burgers_problem* p, double umax, double sigma) {
  if (!p || p->n < 3 || !(p->length > 0) || !is_finite(p->length) || !(p->nu >= 0) ||
      !(sigma > 0) || !(umax >= 0) || (p->bc != BURGERS_BC_PERIODIC && p->bc != BURGERS_BC_DIRICHLET))
    return NAN;
  const double dx = grid_dx(*p);
  double lim = INFINITY;
  if (umax > 0) lim = std::min(lim, dx / umax);
  if (p->nu > 0) lim = std::min(lim, dx * dx / (2.0 * p->nu));
  return sigma * lim;
}

burgers_status burgers_ratios(const burgers_problem* p, double* r, double* D) {
  if (!p || !r || !D || !valid_problem(*p)) return BURGERS_E_INVALID;
  const double dx = grid_dx(*p);
  *r = p->dt / dx;
  *D = p->nu * p->dt / (dx * dx);
  return BURGERS_OK;
}

burgers_status burgers_create(const burgers_problem* problems, int64_t count, burgers_dtype dtype,
                              void* hip_stream, burgers_ctx** out) {
  if (!out) return BURGERS_E_INVALID;
  *out = nullptr;
  burgers_ctx* ctx = nullptr;
  burgers_status st = new_context(problems, count, dtype, hip_stream, &ctx);
  if (st == BURGERS_OK) *out = ctx;
  return st;
}

void burgers_destroy(burgers_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->graph_cache) (void)hipGraphExecDestroy(kv.second);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  for (int k = 0; k < 3; ++k) {
    if (ctx->side[k]) (void)hipStreamDestroy(ctx->side[k]);
    if (ctx->joined[k]) (void)hipEventDestroy(ctx->joined[k]);
  }
  if (ctx->forked) (void)hipEventDestroy(ctx->forked);
  delete ctx;
}

burgers_status burgers_offsets(const burgers_ctx* ctx, int64_t* out) {
  if (!ctx || !out) return BURGERS_E_INVALID;
  std::memcpy(out, ctx->offsets.data(), sizeof(int64_t) * ctx->offsets.size());
  return BURGERS_OK;
}

int64_t burgers_state_elems(const burgers_ctx* ctx) { return ctx ? ctx->total : -1; }

burgers_status burgers_step_explicit(burgers_ctx* ctx, void* u, int64_t nsteps) {
  return advance(ctx, u, nsteps, kSetAll, BURGERS_EXPLICIT);
}

burgers_status burgers_step_btcs(burgers_ctx* ctx, void* u, int64_t nsteps) {
  return advance(ctx, u, nsteps, kSetAll, BURGERS_BTCS);
}

burgers_status burgers_run(burgers_ctx* ctx, void* u, int64_t nsteps) {
  return advance(ctx, u, nsteps, kSetAll, -1);
}

burgers_status burgers_run_mixed(burgers_ctx* ctx, void* u, int64_t explicit_steps, int64_t btcs_steps) {
  if (btcs_steps < 0) return BURGERS_E_INVALID;
  return advance(ctx, u, explicit_steps, kSetAll, -1, btcs_steps);
}

burgers_status burgers_run_static(const burgers_problem* problems, int64_t count, burgers_dtype dtype,
                                  void* hip_stream, void* u, int64_t nsteps) {
  if (!problems || !u || nsteps < 0 || count < 1 || count > INT32_MAX ||
      (dtype != BURGERS_F32 && dtype != BURGERS_F64))
    return BURGERS_E_INVALID;
  for (int64_t i = 0; i < count; ++i)
    if (!valid_problem(problems[i])) return BURGERS_E_INVALID;
  for (int64_t i = 0; i < count; ++i)
    if (problems[i].scheme == BURGERS_NEWTON) return BURGERS_E_UNSUPPORTED;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return BURGERS_E_DEVICE;
  void* base = nullptr;
  if ((e = scratch_address(device, &base)) != hipSuccess) return BURGERS_E_DEVICE;
  burgers::Arena arena{static_cast<char*>(base), static_cast<size_t>(BURGERS_STATIC_SCRATCH_BYTES), 0};
  burgers_status st;
  {
    ArenaGuard guard(&arena);
    burgers_ctx* ctx = nullptr;
    st = new_context(problems, count, dtype, hip_stream, &ctx);
    if (st == BURGERS_OK) {
      st = advance(ctx, u, nsteps, kSetAll, -1);   // plan tables carved too; eager launches
      if (st == BURGERS_OK && ctx->sticky != hipSuccess) st = from_hip(ctx->sticky);
      delete ctx;                                  // host side only: carved buffers free nothing
    }
  }
  return st == BURGERS_E_NOMEM ? BURGERS_E_BUDGET : st;
}

burgers_status burgers_autotune(burgers_ctx* ctx, const void* u, int64_t explicit_steps, int64_t btcs_steps,
                                burgers_plan* best, double* best_ms) {
  if (!ctx || !u || explicit_steps < 0 || btcs_steps < 0 || explicit_steps + btcs_steps == 0)
    return BURGERS_E_INVALID;
  if (ctx->sticky != hipSuccess) return from_hip(ctx->sticky);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return note(ctx, e);
  const bool has_exp = !ctx->set_explicit.empty() && explicit_steps > 0;
  const bool has_btcs = !ctx->set_btcs.empty() && btcs_steps > 0;
  bool long_exp = false, long_btcs = false;
  for (int32_t i : ctx->set_explicit)
    if (ctx->probs[i].n > burgers::explicit_block_capacity()) long_exp = true;
  for (int32_t i : ctx->set_btcs) {
    const burgers_problem& p = ctx->probs[i];
    if (!burgers::btcs_solved_whole(p.bc == BURGERS_BC_PERIODIC ? p.n : p.n - 2)) long_btcs = true;
  }
  // One knob at a time (coordinate descent from the current plan): the explicit path and window depth,
  // the lanes per 8192-row BTCS system, the long-system BTCS solver, concurrent launch groups, graph
  // replay.  Each candidate runs twice on a scratch copy of u (the first run builds its plans and
  // graphs) and the second run is timed.
  using Setter = void (*)(burgers_plan&, int);
  struct Knob {
    std::vector<int> values;
    Setter set;
  };
  std::vector<Knob> knobs;
  if (has_exp) {
    std::vector<int> v = {0};                                     // automatic (whole instances, windows)
    if (long_exp) v = {4, 8, 16, 32, 64, 128, 256};               // window depth (steps per HBM pass)
    v.push_back(-1);                                              // one step per HBM pass
    knobs.push_back({v, [](burgers_plan& p, int x) {
                       p.explicit_path = x < 0 ? 1 : 0;
                       p.tblock_depth = x > 0 ? x : 0;
                     }});
  }
  if (has_btcs) {
    knobs.push_back({{512, 1024}, [](burgers_plan& p, int x) { p.btcs_block = x; }});
    if (long_btcs) knobs.push_back({{0, 2, 1}, [](burgers_plan& p, int x) { p.btcs_long = x; }});
  }
  knobs.push_back({{0, 1}, [](burgers_plan& p, int x) { p.serial = x; }});
  knobs.push_back({{0, 1}, [](burgers_plan& p, int x) { p.use_graph = x; }});
  const burgers_plan base = ctx->plan;
  DevBuf scratch;
  if ((e = scratch.alloc(static_cast<size_t>(ctx->total) * ctx->word, ctx->stream)) != hipSuccess) return from_hip(e);
  hipEvent_t t0, t1;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return from_hip(e);
  if ((e = hipEventCreate(&t1)) != hipSuccess) { (void)hipEventDestroy(t0); return from_hip(e); }
  const size_t bytes = static_cast<size_t>(ctx->total) * ctx->word;
  burgers_status st = BURGERS_OK;
  // time one plan; +inf when it cannot serve the batch
  auto time_plan = [&](const burgers_plan& p, double& ms_out) -> bool {
    ms_out = INFINITY;
    if ((st = burgers_set_plan(ctx, &p)) != BURGERS_OK) return false;
    float ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {
      if ((e = hipMemcpyAsync(scratch.ptr, u, bytes, hipMemcpyDeviceToDevice, ctx->stream)) != hipSuccess) return false;
      if ((e = hipEventRecord(t0, ctx->stream)) != hipSuccess) return false;
      st = advance(ctx, scratch.ptr, explicit_steps, kSetAll, -1, btcs_steps);
      if (st == BURGERS_E_UNSUPPORTED) {
        st = BURGERS_OK;
        return true;
      }
      if (st != BURGERS_OK) return false;
      if ((e = hipEventRecord(t1, ctx->stream)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess) return false;
      if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) return false;
    }
    ms_out = ms;
    return true;
  };
  burgers_plan best_p = base;
  best_p.explicit_path = 0;
  best_p.btcs_path = 0;
  double best_t = INFINITY;
  bool ok = time_plan(best_p, best_t);
  for (size_t k = 0; ok && k < knobs.size(); ++k) {
    burgers_plan knob_best = best_p;
    for (int v : knobs[k].values) {
      burgers_plan p = best_p;
      knobs[k].set(p, v);
      double t;
      if (!(ok = time_plan(p, t))) break;
      if (t < best_t) {
        best_t = t;
        knob_best = p;
      }
    }
    best_p = knob_best;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (e != hipSuccess) {
    (void)burgers_set_plan(ctx, &base);
    return note(ctx, e);
  }
  if (st != BURGERS_OK || !std::isfinite(best_t)) {
    (void)burgers_set_plan(ctx, &base);
    return st != BURGERS_OK ? st : BURGERS_E_UNSUPPORTED;
  }
  (void)burgers_set_plan(ctx, &best_p);
  if (best) *best = best_p;
  if (best_ms) *best_ms = best_t;
  return BURGERS_OK;
}

burgers_status burgers_adjoint(burgers_ctx* ctx, const void* u0, const void* lambda_T, int64_t nsteps,
                               int64_t ckpt_every, void* grad_u0, void* grad_nu) {
  if (!ctx || !u0 || !lambda_T || !grad_u0 || !grad_nu || nsteps < 0 || ckpt_every < 1)
    return BURGERS_E_INVALID;
  if (ctx->dtype != BURGERS_F64) return BURGERS_E_UNSUPPORTED;
  for (const auto& p : ctx->probs)   // adjoint of forward Euler and BTCS only
    if (p.scheme != BURGERS_EXPLICIT && p.scheme != BURGERS_BTCS) return BURGERS_E_UNSUPPORTED;
  if (ctx->sticky != hipSuccess) return from_hip(ctx->sticky);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return note(ctx, e);
  burgers_status st = prepare(ctx, kSetAll, -1);
  if (st != BURGERS_OK) return st;
  if (!ctx->set_btcs.empty() && (st = ensure_btcs(ctx, kSetBtcsHbm)) != BURGERS_OK) return st;
  if ((st = ensure_adjoint(ctx)) != BURGERS_OK) return st;
  burgers::AdjointPlan& ap = *ctx->adjoint;
  const size_t state_bytes = static_cast<size_t>(ctx->total) * sizeof(double);
  const int64_t K = std::min<int64_t>(ckpt_every, std::max<int64_t>(nsteps, 1));
  const int64_t ncp = (nsteps + K - 1) / K;   // checkpoints at steps 0, K, 2K, ...
  if ((e = grow(ap.ckpt, state_bytes * static_cast<size_t>(std::max<int64_t>(ncp, 1)), ctx->stream)) != hipSuccess ||
      (e = grow(ap.seg, state_bytes * static_cast<size_t>(K), ctx->stream)) != hipSuccess ||
      (ncp > 1 && (e = grow(ap.seg2, state_bytes * static_cast<size_t>(K), ctx->stream)) != hipSuccess) ||
      (e = grow(ap.lam0, state_bytes, ctx->stream)) != hipSuccess || (e = grow(ap.lam1, state_bytes, ctx->stream)) != hipSuccess)
    return from_hip(e);
  auto state = [&](DevBuf& b, int64_t k) { return static_cast<char*>(b.ptr) + static_cast<size_t>(k) * state_bytes; };
  const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
  // forward sweep, keeping checkpoints
  if (ncp > 0 && (e = hipMemcpyAsync(state(ap.ckpt, 0), u0, state_bytes, d2d, ctx->stream)) != hipSuccess)
    return note(ctx, e);
  for (int64_t c = 1; c < ncp; ++c) {
    if ((e = hipMemcpyAsync(state(ap.ckpt, c), state(ap.ckpt, c - 1), state_bytes, d2d, ctx->stream)) != hipSuccess ||
        (e = enqueue_all(ctx, kSetAll, -1, state(ap.ckpt, c), K)) != hipSuccess)
      return note(ctx, e);
  }
  // reverse sweep: recompute each segment's states one step at a time, then step the adjoint back
  // lam of the BTCS instances (per step) and of the explicit ones (per run of steps) ping-pong between the
  // same two buffers, each set in its own nodes
  double* lam = ap.lam0.as<double>();
  double* lam_next = ap.lam1.as<double>();
  double* lam_e = lam;
  double* lam_e_next = lam_next;
  if ((e = hipMemcpyAsync(lam, lambda_T, state_bytes, d2d, ctx->stream)) != hipSuccess ||
      (e = burgers::launch_fill(ctx, ap.gslot.as<double>(), ap.n_slots, 0.0)) != hipSuccess ||
      (ap.n_win > 0 && (e = burgers::launch_clear_ints(ctx, ap.flags.as<int>(), 2 * (ctx->count + 1))) != hipSuccess))
    return note(ctx, e);
  int64_t rstep = 0;
  // State k of segment c: the checkpoint for k = 0, else slot k - 1 of the segment's buffer.
  auto at = [&](int64_t c, DevBuf& seg, int64_t k) { return k == 0 ? state(ap.ckpt, c) : state(seg, k - 1); };
  // A segment's states are recomputed out of place.  Instances that the forward sweep keeps on chip are
  // kept on chip here too, by kernels that store the state after every step (one launch per segment, or
  // per `depth` steps for the explicit windows, whose halos cover that many steps): each state is written
  // once and nothing is read back.  The others step one launch at a time from state k - 1 straight into
  // state k: the streaming kernel for explicit instances, the per-step solves for BTCS ones.
  const burgers::ExplicitPlan* ep = ctx->set_explicit.empty() ? nullptr : ctx->explicit_plans[kSetExplicit].get();
  const bool exp_rec = ep && ep->path != 1;
  const burgers::BtcsPlan* bres = ctx->set_btcs.empty() ? nullptr : ctx->btcs[kSetBtcs].get();
  const bool btcs_rec = bres && bres->n_copy == 0 && !bres->resident.empty();
  const burgers::BtcsPlan* bp = ctx->set_btcs.empty() || btcs_rec ? nullptr : ctx->btcs[kSetBtcsHbm].get();
  const int64_t stride = ctx->total;
  auto recompute = [&](int64_t c, DevBuf& seg) -> hipError_t {
    const int64_t len = std::min(K, nsteps - c * K);
    hipError_t err = hipSuccess;
    for (int64_t k0 = 0; exp_rec && k0 < len && err == hipSuccess; k0 += ep->depth) {
      const int k = static_cast<int>(std::min<int64_t>(ep->depth, len - k0));
      err = burgers::launch_explicit_record(ctx, ep->whole->as<BlockTile>(), ep->n_whole, at(c, seg, k0),
                                            at(c, seg, k0 + 1), stride, k);
      if (err == hipSuccess)
        err = burgers::launch_explicit_record(ctx, ep->win->as<BlockTile>(), ep->n_win, at(c, seg, k0),
                                              at(c, seg, k0 + 1), stride, k);
    }
    if (btcs_rec)
      for (const burgers::WgGroup& g : bres->resident)
        if (err == hipSuccess)
          err = burgers::launch_btcs_record(ctx, g, at(c, seg, 0), at(c, seg, 1), stride, static_cast<int>(len));
    const bool exp_step = ep && !exp_rec;
    if (err == hipSuccess && bp) err = burgers::launch_btcs_window_reset(ctx, *bp);
    for (int64_t k = 1; (exp_step || bp) && k <= len && err == hipSuccess; ++k) {
      if (exp_step)
        err = burgers::launch_explicit_stream(ctx, ep->stream->as<Tile>(), ep->n_stream, at(c, seg, k - 1),
                                              at(c, seg, k));
      if (err == hipSuccess && bp) err = burgers::launch_btcs_step(ctx, *bp, at(c, seg, k - 1), at(c, seg, k), k - 1);
    }
    return err;
  };
  // Segment c's reverse steps run on the context's stream while segment c - 1 is recomputed into the
  // other segment buffer on a side stream (the recompute uses none of the reverse steps' buffers): both
  // are HBM-bound chains of short launches, which fill each other's gaps.  The side stream starts after
  // the previous segment's reverse steps (which read the buffer it overwrites) and the context's stream
  // waits for it before the next segment's reverse steps.
  if (ncp > 1) {
    if (!ctx->side[0] && (e = hipStreamCreateWithFlags(&ctx->side[0], hipStreamNonBlocking)) != hipSuccess)
      return note(ctx, e);
    if (!ctx->joined[0] && (e = hipEventCreateWithFlags(&ctx->joined[0], hipEventDisableTiming)) != hipSuccess)
      return note(ctx, e);
    if (!ctx->forked && (e = hipEventCreateWithFlags(&ctx->forked, hipEventDisableTiming)) != hipSuccess)
      return note(ctx, e);
  }
  DevBuf* segs[2] = {&ap.seg, &ap.seg2};
  if (ncp > 0 && (e = recompute(ncp - 1, ap.seg)) != hipSuccess) return note(ctx, e);
  for (int64_t c = ncp - 1; c >= 0; --c) {
    const int64_t len = std::min(K, nsteps - c * K);
    DevBuf& cur = *segs[(ncp - 1 - c) & 1];
    if (c > 0) {   // fork: recompute the next segment beside this one's reverse steps
      hipStream_t main = ctx->stream;
      e = hipEventRecord(ctx->forked, main);
      if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side[0], ctx->forked, 0);
      if (e == hipSuccess) {
        ctx->stream = ctx->side[0];
        e = recompute(c - 1, *segs[(ncp - c) & 1]);
        ctx->stream = main;
      }
      if (e == hipSuccess) e = hipEventRecord(ctx->joined[0], ctx->side[0]);
      if (e != hipSuccess) return note(ctx, e);
    }
    // explicit instances: runs of up to kAdjHalo reverse steps per launch, lam on chip (out of place)
    for (int64_t hi = len; ap.n_exp_wins > 0 && hi > 0; hi -= burgers::kAdjHalo) {
      const int64_t lo = std::max<int64_t>(0, hi - burgers::kAdjHalo);
      if ((e = burgers::launch_adj_explicit_block(ctx, ap.exp_wins->as<burgers::AdjWindow>(), ap.n_exp_wins,
                                                  ap.n_exp_wins_periodic, reinterpret_cast<const double*>(at(c, cur, 0)),
                                                  reinterpret_cast<const double*>(at(c, cur, 1)), ctx->total,
                                                  static_cast<int>(lo), static_cast<int>(hi), lam_e, lam_e_next,
                                                  ap.gslot.as<double>())) != hipSuccess)
        return note(ctx, e);
      std::swap(lam_e, lam_e_next);
    }
    // BTCS instances: the segment's reverse steps in one launch when every system is solved whole (lam
    // on chip between them), else one reverse step per launch
    if (ap.n_whole > 0) {
      if ((e = burgers::launch_adj_btcs_whole(ctx, ap.whole->as<burgers::WinDesc>(), ap.n_whole,
                                              reinterpret_cast<const double*>(at(c, cur, 0)),
                                              reinterpret_cast<const double*>(at(c, cur, 1)), ctx->total, 0,
                                              static_cast<int>(len), lam, lam_next, ap.gslot.as<double>(),
                                              ap.whole_slot->as<int32_t>())) != hipSuccess)
        return note(ctx, e);
      std::swap(lam, lam_next);
    }
    for (int64_t k = len - 1; ap.n_btcs_tiles > 0 && ap.n_whole == 0 && k >= 0; --k) {
      if ((e = enqueue_adjoint_step(ctx, reinterpret_cast<const double*>(at(c, cur, k)),
                                    reinterpret_cast<const double*>(at(c, cur, k + 1)), lam, lam_next,
                                    rstep++)) != hipSuccess)
        return note(ctx, e);
      std::swap(lam, lam_next);
    }
    if (c > 0 && (e = hipStreamWaitEvent(ctx->stream, ctx->joined[0], 0)) != hipSuccess) return note(ctx, e);   // join
  }
  const bool split = lam_e != lam && !ctx->set_explicit.empty() && !ctx->set_btcs.empty();
  if ((e = ensure_copy(ctx, split ? kSetExplicit : kSetAll)) != hipSuccess ||
      (split && (e = ensure_copy(ctx, kSetBtcs)) != hipSuccess))
    return from_hip(e);
  auto& first_tiles = ctx->copy_tiles[split ? kSetExplicit : kSetAll];
  if ((e = burgers::launch_copy_tiles(ctx, first_tiles.first->as<Tile>(), first_tiles.second,
                                      ctx->set_btcs.empty() || split ? lam_e : lam, grad_u0)) != hipSuccess ||
      (split && (e = burgers::launch_copy_tiles(ctx, ctx->copy_tiles[kSetBtcs].first->as<Tile>(),
                                                ctx->copy_tiles[kSetBtcs].second, lam, grad_u0)) != hipSuccess) ||
      (e = burgers::launch_zero_dirichlet_ends(ctx, static_cast<double*>(grad_u0))) != hipSuccess ||
      (e = burgers::launch_adj_nu(ctx, ap.slot_begin->as<int32_t>(), ap.gslot.as<double>(),
                                  static_cast<double*>(grad_nu))) != hipSuccess)
    return note(ctx, e);
  return BURGERS_OK;
}

burgers_status burgers_sync(burgers_ctx* ctx) {
  if (!ctx) return BURGERS_E_INVALID;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipGetLastError();
  note(ctx, e);
  if (ctx->sticky != hipSuccess) return from_hip(ctx->sticky);
  if (ctx->newton && ctx->newton->flags.ptr) {
    // checks of the Newton steps since the last report; cleared once reported
    int flags[2] = {0, 0};
    e = hipMemcpy(flags, ctx->newton->flags.ptr, sizeof(flags), hipMemcpyDeviceToHost);
    if (e == hipSuccess && (flags[0] || flags[1])) {
      e = hipMemsetAsync(ctx->newton->flags.ptr, 0, sizeof(flags), ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (e == hipSuccess) return BURGERS_E_NOT_CONVERGED;
    }
    if (e != hipSuccess) return note(ctx, e);
  }
  return BURGERS_OK;
}

burgers_status burgers_get_plan(const burgers_ctx* ctx, burgers_plan* out) {
  if (!ctx || !out) return BURGERS_E_INVALID;
  *out = ctx->plan;
  return BURGERS_OK;
}

burgers_status burgers_set_plan(burgers_ctx* ctx, const burgers_plan* plan) {
  if (!ctx || !plan) return BURGERS_E_INVALID;
  if (plan->explicit_path < 0 || plan->explicit_path > 3 || plan->btcs_path < 0 || plan->btcs_path > 3 ||
      plan->tblock_depth < 0 || plan->tblock_depth > kMaxDepth || plan->use_graph < -1 || plan->use_graph > 1 ||
      (plan->btcs_block != 0 && plan->btcs_block != 512 && plan->btcs_block != 1024) ||
      plan->btcs_long < 0 || plan->btcs_long > 2 || plan->serial < 0 || plan->serial > 1 ||
      plan->btcs_pipeline < 0 || plan->btcs_pipeline > 2)
    return BURGERS_E_INVALID;
  const bool explicit_changed = plan->explicit_path != ctx->plan.explicit_path ||
                                plan->tblock_depth != ctx->plan.tblock_depth;
  const bool btcs_changed = plan->btcs_path != ctx->plan.btcs_path || plan->btcs_block != ctx->plan.btcs_block ||
                            plan->btcs_long != ctx->plan.btcs_long || plan->btcs_pipeline != ctx->plan.btcs_pipeline;
  ctx->plan = *plan;
  if (explicit_changed) ctx->explicit_plans.clear();
  if (btcs_changed) ctx->btcs.clear();
  for (auto& kv : ctx->graph_cache) (void)hipGraphExecDestroy(kv.second);
  ctx->graph_cache.clear();
  return BURGERS_OK;
}

}  // extern "C"
