// Internal declarations of the gfx950 Burgers library: device-side descriptors, the context and the
// launchers each kernel translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
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
};

// A run of consecutive nodes of one instance handled by one workgroup of a streaming kernel.
struct Tile {
  int32_t inst;
  int32_t start;
};

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
};

// A block of consecutive chunks of one system (reduce and back-substitution kernels).
struct ChunkBlock {
  int32_t sys;
  int32_t chunk0;
};

// Device buffer owned by a context.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  ~DevBuf() { if (ptr) (void)hipFree(ptr); }
  hipError_t alloc(size_t n) {
    bytes = n;
    return n ? hipMalloc(&ptr, n) : hipSuccess;
  }
  template <typename T> T* as() const { return static_cast<T*>(ptr); }
};

// Launch list of the BTCS solve for a set of instances, built once per context and set.
struct BtcsPlan {
  // small systems solved whole by one workgroup each, straight from and to the state
  std::unique_ptr<DevBuf> wg_state;          // SysDesc[]
  int32_t n_wg_state = 0;
  // partition hierarchy for the long systems
  struct Level {
    std::unique_ptr<DevBuf> sys;             // SysDesc[] of the systems reduced at this level
    std::unique_ptr<DevBuf> blocks;          // ChunkBlock[]
    int32_t n_blocks = 0;
    std::unique_ptr<DevBuf> wg;              // SysDesc[] of the reduced systems solved whole
    int32_t n_wg = 0;
  };
  std::vector<Level> levels;                 // levels[0] reduces from the state
  int64_t level_rows = 0;                    // rows of A, C, D, X used by this plan
};

struct Plan {
  burgers_plan user{};
  int resident_explicit_limit = 0;
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
  // explicit streaming tiles per subset (device)
  std::map<int, std::unique_ptr<burgers::DevBuf>> tiles;
  std::map<int, int64_t> n_tiles;
  std::map<int, std::unique_ptr<burgers::BtcsPlan>> btcs;
  // captured graphs keyed by (kind, steps)
  std::map<std::pair<int, int64_t>, hipGraphExec_t> graphs;
  hipError_t sticky = hipSuccess;
};

namespace burgers {

// explicit.hip
hipError_t launch_explicit_stream(const burgers_ctx* ctx, const Tile* tiles, int64_t n_tiles,
                                  const void* u, void* out);
int explicit_tile_nodes(burgers_dtype dt);

// btcs.hip
int btcs_wg_capacity();                 // longest system one workgroup solves whole
int btcs_wg_chunks(int rows);           // chunk count the workgroup solver uses for `rows` rows
int btcs_reduce_chunk();                // target rows per chunk in the partition levels
constexpr int kReduceBlock = 256;       // chunks per workgroup in the partition kernels
hipError_t launch_btcs_step(const burgers_ctx* ctx, const BtcsPlan& plan, const void* u, void* out);

}  // namespace burgers
