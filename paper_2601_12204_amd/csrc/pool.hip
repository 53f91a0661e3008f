// Resident slot pools for continuous-batching serving.
//
// A pool is a fixed set of device slots of one precision and one scheme (forward Euler or BTCS), each
// able to hold a problem of up to `cap` nodes.  A request is admitted into a free slot between ticks (its
// scalars go into the pool's slot table, its initial state into the slot's part of the pool's state
// buffer), and every tick advances all occupied slots by up to `tick` steps in one launch sequence.
// That sequence depends only on whether long problems (windows) are in flight, so it is captured into one
// of two HIP graphs and replayed; the per-slot work lives in device tables refreshed before each tick.  Every slot runs the same
// kernels, in the same arithmetic, as a context holding its problem alone: the on-chip whole-instance
// kernels for up to 8192 nodes, and for longer problems the explicit windows (temporal blocking) or the
// truncated BTCS windows.  Pools hold no partition levels, so a BTCS window step whose accuracy bound
// fails (far beyond the CFL step) is not redone but reported when its slot is retired.
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "internal.hpp"

namespace {

using burgers::BlockTile;
using burgers::DevBuf;
using burgers::InstDesc;
using burgers::SysDesc;
using burgers::Tile;
using burgers::WinDesc;

constexpr int kWholeLanes[4] = {64, 128, 256, 512};
// BTCS classes of the on-chip solver: (lanes, rows per lane, exact 8192-row layout)
constexpr int kResLanes[5] = {128, 256, 512, 1024, 512};
constexpr int kWinGroup = 5;        // launch groups (bits of a mask): whole classes 0-4, windows 5
constexpr int kWindowDepth = 128;   // explicit window steps per launch (as a context's default)

size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// a DevBuf view of part of another buffer (never freed through the view)
void view(DevBuf& b, void* base, size_t off, size_t bytes, hipStream_t st) {
  b.ptr = static_cast<char*>(base) + off;
  b.bytes = bytes;
  b.stream = st;
  b.carved = true;
}

}  // namespace

struct burgers_pool {
  burgers_ctx ctx;                 // stream, precision, count = slots, inst = the slot table
  int32_t scheme = BURGERS_EXPLICIT;
  int64_t slots = 0, cap = 0, tick = 0;
  int depth = kWindowDepth;
  int64_t wx = 0;                  // window entries per slot
  int64_t tx = 0;                  // copy tiles per slot
  std::vector<burgers_problem> probs;
  std::vector<int64_t> remaining;  // -1: free
  std::vector<int32_t> group;      // launch group of each occupied slot
  std::vector<InstDesc> inst_host;
  // device tables (one buffer) and their host image
  DevBuf tables;
  std::vector<unsigned char> image;
  size_t off_whole[5] = {}, off_win = 0, off_copy = 0;
  std::vector<burgers::WgGroup> res;                 // BTCS on-chip classes (views into `tables`)
  burgers::BtcsPlan bplan;                           // BTCS windows (views into `tables`), no levels
  DevBuf win_view, copy_view;
  DevBuf u, work;
  int* sticky_host = nullptr;      // pinned copy of the windows' failed-bound flags after each tick
  hipEvent_t done = nullptr;
  hipStream_t capture = nullptr;
  std::map<uint32_t, hipGraphExec_t> graphs;
  hipError_t sticky_err = hipSuccess;
};

namespace {

burgers_status status_of(hipError_t e) {
  if (e == hipSuccess) return BURGERS_OK;
  if (e == hipErrorOutOfMemory) return BURGERS_E_NOMEM;
  return BURGERS_E_DEVICE;
}

int rows_of(const burgers_problem& p) { return static_cast<int>(p.bc == BURGERS_BC_PERIODIC ? p.n : p.n - 2); }

// launch group of a problem in the pool
int group_of(const burgers_pool* pl, const burgers_problem& p) {
  const int cap_chip = burgers::btcs_wg_capacity();
  if (pl->scheme == BURGERS_EXPLICIT) {
    if (p.n > burgers::explicit_block_capacity()) return kWinGroup;
    const int lanes = burgers::explicit_block_lanes(static_cast<int>(p.n));
    for (int c = 0; c < 4; ++c)
      if (kWholeLanes[c] == lanes) return c;
    return 3;
  }
  const int R = rows_of(p);
  if (R > cap_chip) return kWinGroup;
  const burgers::WidthClass w = burgers::btcs_width_class(R, 512);
  if (w.exact) return 4;
  for (int c = 0; c < 4; ++c)
    if (kResLanes[c] == w.lanes) return c;
  return 3;
}

// Host image of the device tables for the coming tick: every slot's entries, empty (no-op) for free
// slots, for slots with no steps left and for slots of other groups.
void build_image(burgers_pool* pl) {
  std::fill(pl->image.begin(), pl->image.end(), 0);
  const int64_t K = pl->tick;
  const int tile_nodes = burgers::explicit_tile_nodes(pl->ctx.dtype);
  for (int64_t s = 0; s < pl->slots; ++s) {
    if (pl->remaining[s] <= 0) continue;
    const burgers_problem& p = pl->probs[s];
    const int32_t limit = static_cast<int32_t>(std::min<int64_t>(pl->remaining[s], K));
    const int g = pl->group[s];
    const int32_t i = static_cast<int32_t>(s);
    const bool periodic = p.bc == BURGERS_BC_PERIODIC;
    if (g != kWinGroup) {
      if (pl->scheme == BURGERS_EXPLICIT) {
        BlockTile bt{i, 0, static_cast<int32_t>(p.n), 0, static_cast<int32_t>(p.n), periodic ? 1 : 0, 0, limit};
        std::memcpy(pl->image.data() + pl->off_whole[g] + s * sizeof(BlockTile), &bt, sizeof(bt));
      } else {
        const int R = rows_of(p);
        const burgers::WidthClass w = burgers::btcs_width_class(R, 512);
        SysDesc sd{0, -1, R, burgers::btcs_chunks(R, w.lanes), i, 0, 0, limit};
        std::memcpy(pl->image.data() + pl->off_whole[g] + s * sizeof(SysDesc), &sd, sizeof(sd));
      }
      continue;
    }
    // windows of a long problem, and its copy-back tiles
    if (pl->scheme == BURGERS_EXPLICIT) {
      std::vector<BlockTile> w;
      burgers::explicit_windows(i, static_cast<int32_t>(p.n), periodic, pl->depth, false, w);
      for (auto& bt : w) bt.limit = limit;
      w.resize(std::min<size_t>(w.size(), static_cast<size_t>(pl->wx)));   // (never cut: wx covers cap)
      std::memcpy(pl->image.data() + pl->off_win + s * pl->wx * sizeof(BlockTile), w.data(), w.size() * sizeof(BlockTile));
    } else {
      std::vector<WinDesc> w;
      burgers::btcs_windows(i, rows_of(p), periodic, 4096, false, w);
      for (auto& wd : w) wd.limit = limit;
      w.resize(std::min<size_t>(w.size(), static_cast<size_t>(pl->wx)));
      std::memcpy(pl->image.data() + pl->off_win + s * pl->wx * sizeof(WinDesc), w.data(), w.size() * sizeof(WinDesc));
    }
    std::vector<Tile> ct;
    for (int64_t k = 0; k < p.n && static_cast<int64_t>(ct.size()) < pl->tx; k += tile_nodes)
      ct.push_back(Tile{s * pl->cap, static_cast<int32_t>(p.n), static_cast<int32_t>(k), p.bc, i});
    std::memcpy(pl->image.data() + pl->off_copy + s * pl->tx * sizeof(Tile), ct.data(), ct.size() * sizeof(Tile));
  }
}

// The launch sequence of one tick for the groups in `mask` (all on pl->ctx.stream).
hipError_t enqueue_tick(burgers_pool* pl, uint32_t mask) {
  burgers_ctx* ctx = &pl->ctx;
  const int K = static_cast<int>(pl->tick);
  hipError_t e = hipSuccess;
  void* u = pl->u.ptr;
  void* work = pl->work.ptr;
  const Tile* copy = pl->copy_view.as<Tile>();
  const int64_t n_copy = pl->slots * pl->tx;
  if (pl->scheme == BURGERS_EXPLICIT) {
    for (int c = 0; c < 4; ++c) {
      if (!(mask & (1u << c))) continue;
      const BlockTile* t = reinterpret_cast<const BlockTile*>(static_cast<char*>(pl->tables.ptr) + pl->off_whole[c]);
      if ((e = burgers::launch_explicit_block(ctx, t, pl->slots, 0, u, u, K, kWholeLanes[c], 0)) != hipSuccess) return e;
    }
    if (mask & (1u << kWinGroup)) {
      void* bufs[2] = {u, work};
      int cur = 0;
      for (int done = 0; done < K; done += pl->depth) {
        const int k = std::min(pl->depth, K - done);
        if ((e = burgers::launch_explicit_block(ctx, pl->win_view.as<BlockTile>(), pl->slots * pl->wx, 0, bufs[cur],
                                                bufs[cur ^ 1], k, 512, done)) != hipSuccess)
          return e;
        cur ^= 1;
      }
      if (cur && (e = burgers::launch_copy_tiles(ctx, copy, n_copy, work, u)) != hipSuccess) return e;
    }
    return e;
  }
  for (int c = 0; c < 5; ++c)
    if ((mask & (1u << c)) && (e = burgers::launch_btcs_resident(ctx, pl->res[c], u, K)) != hipSuccess) return e;
  if (mask & (1u << kWinGroup)) {
    if ((e = burgers::launch_btcs_window_reset(ctx, pl->bplan)) != hipSuccess) return e;
    void* bufs[2] = {u, work};
    int cur = 0;
    for (int s = 0; s < K; ++s) {
      if ((e = burgers::launch_btcs_step(ctx, pl->bplan, bufs[cur], bufs[cur ^ 1], s)) != hipSuccess) return e;
      cur ^= 1;
    }
    if (cur && (e = burgers::launch_copy_tiles(ctx, copy, n_copy, work, u)) != hipSuccess) return e;
  }
  return e;
}

hipError_t tick_graph(burgers_pool* pl, uint32_t mask, hipGraphExec_t* out) {
  auto it = pl->graphs.find(mask);
  if (it != pl->graphs.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipError_t e;
  if (!pl->capture && (e = hipStreamCreateWithFlags(&pl->capture, hipStreamNonBlocking)) != hipSuccess) return e;
  hipStream_t user = pl->ctx.stream;
  pl->ctx.stream = pl->capture;
  if ((e = hipStreamBeginCapture(pl->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    pl->ctx.stream = user;
    return e;
  }
  hipError_t le = enqueue_tick(pl, mask);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(pl->capture, &graph);
  pl->ctx.stream = user;
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return le;
  }
  if (e != hipSuccess) return e;
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return e;
  pl->graphs.emplace(mask, exec);
  *out = exec;
  return hipSuccess;
}

void pool_free(burgers_pool* pl) {
  if (!pl) return;
  (void)hipSetDevice(pl->ctx.device);
  (void)hipStreamSynchronize(pl->ctx.stream);
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
  if (pl->capture) (void)hipStreamDestroy(pl->capture);
  if (pl->done) (void)hipEventDestroy(pl->done);
  if (pl->sticky_host) (void)hipHostFree(pl->sticky_host);
  // views into `tables` must not free anything
  for (auto& g : pl->res) g.sys.reset();
  pl->bplan.win.reset();
  delete pl;
}

}  // namespace

extern "C" {

burgers_status burgers_pool_create(burgers_dtype dtype, int32_t scheme, int64_t slots, int64_t max_nodes,
                                   int64_t tick_steps, void* hip_stream, burgers_pool** out) {
  if (!out) return BURGERS_E_INVALID;
  *out = nullptr;
  if ((dtype != BURGERS_F32 && dtype != BURGERS_F64) || (scheme != BURGERS_EXPLICIT && scheme != BURGERS_BTCS) ||
      slots < 1 || slots > (1 << 20) || max_nodes < 3 || max_nodes > (int64_t{1} << 24) || tick_steps < 1 ||
      tick_steps > (1 << 20))
    return BURGERS_E_INVALID;
  burgers_pool* pl = new (std::nothrow) burgers_pool();
  if (!pl) return BURGERS_E_NOMEM;
  hipError_t e = hipGetDevice(&pl->ctx.device);
  if (e != hipSuccess) {
    delete pl;
    return BURGERS_E_DEVICE;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  pl->ctx.stream = st;
  pl->ctx.dtype = dtype;
  pl->ctx.word = dtype == BURGERS_F64 ? 8 : 4;
  pl->ctx.count = slots;
  pl->scheme = scheme;
  pl->slots = slots;
  pl->cap = (max_nodes + BURGERS_ALIGN - 1) / BURGERS_ALIGN * BURGERS_ALIGN;
  pl->tick = tick_steps;
  pl->depth = static_cast<int>(std::min<int64_t>(kWindowDepth, tick_steps));
  pl->probs.resize(slots);
  pl->remaining.assign(slots, -1);
  pl->group.assign(slots, 0);
  pl->inst_host.assign(slots, InstDesc{});
  for (int64_t s = 0; s < slots; ++s) {   // empty slots: a harmless descriptor at the slot's offset
    pl->inst_host[s].off = s * pl->cap;
    pl->inst_host[s].n = 3;
  }
  // windows per slot for the longest problem it may hold
  const int64_t longest = pl->cap;
  const int tile_nodes = burgers::explicit_tile_nodes(dtype);
  size_t entry = 0;
  if (scheme == BURGERS_EXPLICIT) {
    const int64_t kept = burgers::explicit_block_capacity() - 2 * pl->depth;
    pl->wx = longest > burgers::explicit_block_capacity() ? (longest + kept - 1) / kept : 0;
    entry = sizeof(BlockTile);
  } else {
    const int64_t kept = 4096 - 2 * burgers::btcs_window_halo();
    pl->wx = longest - 2 > burgers::btcs_wg_capacity() ? (longest + kept - 1) / kept : 0;
    entry = sizeof(WinDesc);
  }
  pl->tx = pl->wx ? (pl->cap + tile_nodes - 1) / tile_nodes : 0;
  const size_t whole_entry = scheme == BURGERS_EXPLICIT ? sizeof(BlockTile) : sizeof(SysDesc);
  size_t off = 0;
  for (int c = 0; c < 5; ++c) {
    pl->off_whole[c] = off;
    off = align_up(off + static_cast<size_t>(slots) * whole_entry);
  }
  pl->off_win = off;
  off = align_up(off + static_cast<size_t>(slots * pl->wx) * entry);
  pl->off_copy = off;
  off = align_up(off + static_cast<size_t>(slots * pl->tx) * sizeof(Tile));
  pl->image.assign(off, 0);
  const size_t state = static_cast<size_t>(slots) * pl->cap * pl->ctx.word;
  if ((e = pl->tables.alloc(off, st)) != hipSuccess || (e = pl->u.alloc(state, st)) != hipSuccess ||
      (e = pl->work.alloc(pl->wx ? state : 0, st)) != hipSuccess ||
      (e = pl->ctx.inst.alloc(static_cast<size_t>(slots) * sizeof(InstDesc), st)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->ctx.inst.ptr, pl->inst_host.data(), static_cast<size_t>(slots) * sizeof(InstDesc),
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->tables.ptr, pl->image.data(), off, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&pl->done, hipEventDisableTiming)) != hipSuccess ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&pl->sticky_host), static_cast<size_t>(slots) * sizeof(int))) !=
          hipSuccess) {
    pool_free(pl);
    return status_of(e);
  }
  std::memset(pl->sticky_host, 0, static_cast<size_t>(slots) * sizeof(int));
  pl->ctx.work.ptr = nullptr;
  view(pl->win_view, pl->tables.ptr, pl->off_win, static_cast<size_t>(slots * pl->wx) * entry, st);
  view(pl->copy_view, pl->tables.ptr, pl->off_copy, static_cast<size_t>(slots * pl->tx) * sizeof(Tile), st);
  if (scheme == BURGERS_BTCS) {
    for (int c = 0; c < 5; ++c) {
      burgers::WgGroup g;
      g.shape = c == 4 ? burgers::WidthClass{512, 16, true} : burgers::WidthClass{kResLanes[c], 8, false};
      g.sys = std::make_unique<DevBuf>();
      view(*g.sys, pl->tables.ptr, pl->off_whole[c], static_cast<size_t>(slots) * sizeof(SysDesc), st);
      g.n = static_cast<int32_t>(slots);
      pl->res.push_back(std::move(g));
    }
    pl->bplan.win = std::make_unique<DevBuf>();
    view(*pl->bplan.win, pl->tables.ptr, pl->off_win, static_cast<size_t>(slots * pl->wx) * entry, st);
    pl->bplan.n_win = slots * pl->wx;
    pl->bplan.win_rows = 4096;
    if (pl->bplan.n_win > 0) {
      if ((e = pl->bplan.win_flags.alloc(static_cast<size_t>(burgers::win_flags_words(slots)) * sizeof(int), st)) !=
              hipSuccess ||
          (e = burgers::launch_clear_ints(&pl->ctx, pl->bplan.win_flags.as<int>(), burgers::win_flags_words(slots))) !=
              hipSuccess) {
        pool_free(pl);
        return status_of(e);
      }
    }
  }
  *out = pl;
  return BURGERS_OK;
}

void burgers_pool_destroy(burgers_pool* pool) { pool_free(pool); }

burgers_status burgers_pool_admit(burgers_pool* pool, const burgers_problem* p, const void* u0, int64_t nsteps,
                                  int64_t* slot) {
  if (!pool || !p || !u0 || !slot || nsteps < 1 || *slot < -1 || *slot >= pool->slots) return BURGERS_E_INVALID;
  const int64_t want = *slot;
  *slot = -1;
  if (!burgers::problem_valid(*p) || p->scheme != pool->scheme) return BURGERS_E_INVALID;
  if (p->n > pool->cap || (pool->wx == 0 && group_of(pool, *p) == kWinGroup)) return BURGERS_E_UNSUPPORTED;
  if (pool->sticky_err != hipSuccess) return status_of(pool->sticky_err);
  int64_t s = want;
  if (s < 0) {
    s = 0;
    while (s < pool->slots && pool->remaining[s] >= 0) ++s;
    if (s == pool->slots) return BURGERS_E_BUDGET;   // every slot occupied
  } else if (pool->remaining[s] >= 0) {
    return BURGERS_E_BUDGET;                          // the slot asked for is occupied
  }
  hipError_t e = hipSetDevice(pool->ctx.device);
  hipStream_t st = pool->ctx.stream;
  pool->inst_host[s] = burgers::inst_desc(*p, s * pool->cap);
  char* dst = static_cast<char*>(pool->u.ptr) + static_cast<size_t>(s * pool->cap) * pool->ctx.word;
  if (e == hipSuccess)
    e = hipMemcpyAsync(pool->ctx.inst.as<InstDesc>() + s, &pool->inst_host[s], sizeof(InstDesc),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dst, u0, static_cast<size_t>(p->n) * pool->ctx.word, hipMemcpyDefault, st);
  if (e == hipSuccess && pool->bplan.n_win > 0)
    e = burgers::launch_clear_ints(&pool->ctx, burgers::win_sticky(pool->bplan.win_flags.as<int>(), pool->slots) + s, 1);
  if (e != hipSuccess) {
    pool->sticky_err = e;
    return status_of(e);
  }
  pool->sticky_host[s] = 0;
  pool->probs[s] = *p;
  pool->remaining[s] = nsteps;
  pool->group[s] = group_of(pool, *p);
  *slot = s;
  return BURGERS_OK;
}

burgers_status burgers_pool_tick(burgers_pool* pool) {
  if (!pool) return BURGERS_E_INVALID;
  if (pool->sticky_err != hipSuccess) return status_of(pool->sticky_err);
  // The whole-instance classes always launch (a class without a slot costs one empty launch); the
  // windows, many launches per tick, only when a long problem is in flight.  So a pool captures at most
  // two graphs, and a tick never waits for a capture once both exist.
  bool any = false, windows = false;
  for (int64_t s = 0; s < pool->slots; ++s) {
    if (pool->remaining[s] <= 0) continue;
    any = true;
    windows = windows || pool->group[s] == kWinGroup;
  }
  if (!any) return BURGERS_OK;
  const uint32_t mask = ((1u << kWinGroup) - 1) | (windows ? 1u << kWinGroup : 0u);
  hipError_t e = hipSetDevice(pool->ctx.device);
  build_image(pool);
  hipGraphExec_t g = nullptr;
  if (e == hipSuccess)
    e = hipMemcpyAsync(pool->tables.ptr, pool->image.data(), pool->image.size(), hipMemcpyHostToDevice,
                       pool->ctx.stream);
  if (e == hipSuccess) e = tick_graph(pool, mask, &g);
  if (e == hipSuccess) e = hipGraphLaunch(g, pool->ctx.stream);
  if (e == hipSuccess && pool->bplan.n_win > 0)
    e = hipMemcpyAsync(pool->sticky_host, burgers::win_sticky(pool->bplan.win_flags.as<int>(), pool->slots),
                       static_cast<size_t>(pool->slots) * sizeof(int), hipMemcpyDeviceToHost, pool->ctx.stream);
  if (e == hipSuccess) e = hipEventRecord(pool->done, pool->ctx.stream);
  if (e != hipSuccess) {
    pool->sticky_err = e;
    return status_of(e);
  }
  for (int64_t s = 0; s < pool->slots; ++s)
    if (pool->remaining[s] > 0) pool->remaining[s] -= std::min(pool->remaining[s], pool->tick);
  return BURGERS_OK;
}

int32_t burgers_pool_busy(burgers_pool* pool) {
  if (!pool) return 0;
  return hipEventQuery(pool->done) == hipErrorNotReady ? 1 : 0;
}

int64_t burgers_pool_remaining(const burgers_pool* pool, int64_t slot) {
  if (!pool || slot < 0 || slot >= pool->slots) return -2;
  return pool->remaining[slot];
}

burgers_status burgers_pool_retire(burgers_pool* pool, int64_t slot, void* dst) {
  if (!pool || !dst || slot < 0 || slot >= pool->slots || pool->remaining[slot] != 0) return BURGERS_E_INVALID;
  if (pool->sticky_err != hipSuccess) return status_of(pool->sticky_err);
  hipError_t e = hipSetDevice(pool->ctx.device);
  const char* src = static_cast<const char*>(pool->u.ptr) + static_cast<size_t>(slot * pool->cap) * pool->ctx.word;
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst, src, static_cast<size_t>(pool->probs[slot].n) * pool->ctx.word, hipMemcpyDefault,
                       pool->ctx.stream);
  if (e == hipSuccess && pool->bplan.n_win > 0 && hipEventQuery(pool->done) == hipErrorNotReady)
    e = hipEventSynchronize(pool->done);   // the flags of the slot's last tick
  if (e != hipSuccess) {
    pool->sticky_err = e;
    return status_of(e);
  }
  pool->remaining[slot] = -1;
  return pool->bplan.n_win > 0 && pool->sticky_host[slot] ? BURGERS_E_BOUND : BURGERS_OK;
}

}  // extern "C"
