// sc_runtime.h -- host runtime internals shared by the single-run, batch and
// serving parts of the library (not part of the public ABI, see lbm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "sc_launch.h"

namespace sclbm {

void set_error(const std::string& msg);
lbm_status fail(lbm_status code, const std::string& msg);
lbm_status hip_fail(hipError_t e, const char* what);
// Records `where: what` as the thread's error message without throwing.
lbm_status fail_nothrow(lbm_status code, const char* where, const char* what) noexcept;

// Runs the body of a C-ABI entry point with every C++ exception turned into a
// status and a message (std::bad_alloc: LBM_ENOMEM; anything else, e.g.
// std::system_error from a thread, or an exception out of the runtime:
// LBM_EDEVICE), so that no exception crosses the boundary.
template <class F>
lbm_status guarded(const char* where, F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail_nothrow(LBM_ENOMEM, where, "host memory exhausted");
  } catch (const std::exception& e) {
    return fail_nothrow(LBM_EDEVICE, where, e.what());
  } catch (...) {
    return fail_nothrow(LBM_EDEVICE, where, "unknown C++ exception");
  }
}

#define SCLBM_HIP(call)                                     \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return ::sclbm::hip_fail(e_, #call); \
  } while (0)

lbm_status validate_params(const lbm_params* p);
size_t pop_bytes_for(const lbm_params& p);
size_t align_up(size_t v, size_t a);

// Tile shape k -> (variant, rows).
inline int tile_variant(int k) { return k / kNumRows; }
inline int tile_rows(int k) { return kRowChoices[k % kNumRows]; }  // 0: balanced
inline int tile_width(int k) {
  const StepVariant& v = step_variant(tile_variant(k));
  if (v.steps >= 2) return v.width;
  return v.paired ? (v.threads / 64) * kPairColumns : v.threads * v.cells;
}
// Columns one work item of tile shape k covers on a grid nx columns wide: a
// two- or three-step shape marches a grid no wider than its workgroup as one
// periodic strip.
inline int strip_width(int k, int nx) {
  const StepVariant& v = step_variant(tile_variant(k));
  return v.steps >= 2 && nx <= v.threads ? nx : tile_width(k);
}
// Time steps one launch of tile shape k takes.
inline int tile_steps(int k) { return step_variant(tile_variant(k)).steps; }
// Index of the step variant with these parameters (-1 if there is none).
// width: a two-step variant's output columns (0: the widest).
inline int find_variant(int threads, int cells, int prefetch, int paired, int steps = 1,
                        int width = 0) {
  for (int v = 0; v < kNumVariants; ++v) {
    const StepVariant& s = step_variant(v);
    if (s.threads == threads && s.cells == cells && s.prefetch == prefetch && s.paired == paired &&
        s.steps == steps && (width == 0 || s.width == width))
      return v;
  }
  return -1;
}
// Whether tile shape k can run a grid nx columns wide in this storage form
// (moment storage: strip shapes, and two-step shapes whose strips leave four
// halo columns on each side; three-step shapes: FP32 only).
inline bool tile_valid(int k, int nx, int storage) {
  const StepVariant& v = step_variant(tile_variant(k));
  if (v.steps >= 3 && storage != LBM_F32) return false;
  if (storage == LBM_F16_MOMENT && (v.paired || (v.steps == 2 && v.width > v.threads - 8)))
    return false;
  return !v.paired || (nx % 2 == 0 && nx >= kPairMinNx);
}
// Whether a batch can use tile shape k (every shape a run of this storage
// type can use: batches take one, two or three steps per launch).
inline bool tile_batchable(int k, int nx, int storage) { return tile_valid(k, nx, storage); }

// Band height tile shape k uses on an nx x ny grid of this storage type
// (balanced shapes: from the step kernel's occupancy on the current device).
int band_rows(int k, int nx, int ny, int storage);
// Work items of one grid for tile shape k, appended for simulation `inst`.
void make_items(int nx, int ny, int storage, int tile, int inst, std::vector<TileItem>& out);
// Reorders items so that the workgroups a hardware XCD receives (workgroup
// ids congruent mod 8) cover a contiguous run of the original order.
std::vector<TileItem> xcd_order(const std::vector<TileItem>& items);

// Workspace layout of a single run.
struct WorkLayout {
  size_t desc, nitems, items, partials, result;
  // metric series: its tile tables (single-step and two-step recording
  // steps), one partial record per item, records
  size_t s_nitems, s_items, s2_nitems, s2_items, s_partials, s_records;
  size_t total;
  int max_items, series_items, series2_items;
};
WorkLayout work_layout(int nx, int ny);

// Default tile shape of a run; default_strip_tile never picks a paired-column
// variant, so it is valid for every grid width.
int default_tile(const lbm_params& p);
int default_strip_tile(const lbm_params& p);
// Index of a band height in kRowChoices (0 if it is not one).
int row_choice(int rows);
int tuned_tile(const lbm_params& p, const std::string& arch);  // -1 if none
void record_tuned_tile(const lbm_params& p, const std::string& arch, int tile, double ms);
std::string device_arch();
int device_cu_count();

// Multi-simulation stepping: a device descriptor table and one tile table per
// storage type, advanced by a HIP graph of persistent step launches between a
// tick-begin and a tick-end kernel: K single-step launches per storage type;
// for a two-step variant, ceil(K / 2) two-step launches and one single-step
// tail launch (its own tile table, tail_variant) that takes the last step of
// members with an odd step count this tick; for a three-step variant,
// floor(K / 3) three-step launches, a two-step tail launch over the same
// items (pair_variant, the two-step variant of the same strips) for members
// with two steps left over, and the single-step tail for those with one.  The
// graph reads the tables from device memory, so members can change between
// replays without rebuilding it.
struct BatchEngine {
  hipStream_t stream = nullptr;
  int K = 1, cap_inst = 0;
  int cap_items[kNumStorages] = {}, variant[kNumStorages] = {-1, -1, -1, -1},
      grid[kNumStorages] = {}, nitems[kNumStorages] = {};
  // single-step tail launches of multi-step storage types (capacity 0 otherwise)
  int cap_titems[kNumStorages] = {}, tail_variant[kNumStorages] = {-1, -1, -1, -1},
      tgrid[kNumStorages] = {};
  // two-step tail launches of three-step storage types (over the main items)
  int pair_variant[kNumStorages] = {-1, -1, -1, -1}, p2grid[kNumStorages] = {};
  InstDesc* d_desc = nullptr;
  // Grid sized to the resident capacity, looping over the items (needed when
  // the item count changes between replays), instead of one workgroup per item.
  bool persistent = false;
  int* d_nitems[kNumStorages] = {};
  TileItem* d_items[kNumStorages] = {};
  int* d_tnitems[kNumStorages] = {};
  TileItem* d_titems[kNumStorages] = {};
  // pinned staging of the tables, two sets used in turn (stage = next set)
  InstDesc* h_desc[2] = {};
  TileItem* h_items[kNumStorages][2] = {};
  TileItem* h_titems[kNumStorages][2] = {};
  hipEvent_t staged[2] = {};
  bool staged_pending[2] = {};
  int stage = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<lbm_ctx*> members;
  // Storage types whose step launches start disabled in the graph and are
  // enabled by the first load that has members of that type (a server that
  // sees only one storage type then launches no empty kernels).
  bool lazy_storages = false;
  bool enabled[kNumStorages] = {};
  std::vector<hipGraphNode_t> step_nodes[kNumStorages];

  // cap_titems: tail tile-table capacities (0 for single-step storage types).
  static size_t work_bytes(int cap_inst, const int cap_items[kNumStorages],
                           const int cap_titems[kNumStorages], int K);
  lbm_status init(hipStream_t st, int steps_per_tick, int cap_inst,
                  const int cap_items[kNumStorages], const int cap_titems[kNumStorages],
                  const int variants[kNumStorages], void* work, size_t wbytes);
  // Steps per launch of a storage type's step kernel.
  int per_launch(int storage) const {
    return variant[storage] >= 0 ? step_variant(variant[storage]).steps : 1;
  }
  // Tile used for every member instead of the members' own (-1: none).
  int tile_override = -1;
  int row_override = -1;  // band height index for every member (-1: the member's own)
  // Uploads the members' descriptors (with `remaining` steps each, and nsub
  // sub-steps enabled before any tick) and tiles.
  lbm_status load(const std::vector<lbm_ctx*>& m, const std::vector<int64_t>& remaining,
                  int nsub_init = 0);
  // Sets every member's remaining steps on the device.
  lbm_status arm(int64_t steps);
  // One replay: each member takes min(K, remaining) steps.
  lbm_status replay();
  void destroy();
};

int member_tile(const lbm_ctx* c, int variant, int tile_override, int row_override = -1);
int pick_variant(const std::vector<lbm_ctx*>& m, int storage);

// lbm_create / lbm_init_droplets with the stream waits made optional (see
// their definitions); the C-ABI functions call them with waits.
// flag: device-visible address of the run's status word (InstDesc::flag;
// nullptr for none).
lbm_status create_ctx(const lbm_params* p, void* popA, void* popB, size_t pop_bytes, void* work,
                      size_t work_bytes, void* hip_stream, bool standalone, lbm_ctx** out,
                      int* flag = nullptr);
lbm_status init_droplets(lbm_ctx* c, const double* drops, int32_t n, const lbm_init* ip,
                         bool sync);
// tail: the items of the single-step tail launch of a multi-step variant.
int count_items(const std::vector<lbm_ctx*>& m, int storage, int variant, int tile_override,
                bool tail = false);
// Single-step shape that takes the last step of a tick of a multi-step
// variant: strips of kSeriesThreads x 1 cell, 2 rows in flight.
int tail_variant_for(int variant);

}  // namespace sclbm

struct lbm_ctx {
  lbm_params p{};
  void* pop[2] = {nullptr, nullptr};
  size_t pop_bytes = 0;
  void* work = nullptr;
  size_t work_bytes = 0;
  hipStream_t stream = nullptr;
  int parity = 0;  // buffer holding the current state
  int64_t steps = 0;
  int tile = 0;
  int nitems = 0;
  sclbm::WorkLayout lay{};
  sclbm::InstDesc* d_desc = nullptr;
  int* d_nitems = nullptr;
  sclbm::TileItem* d_items = nullptr;
  double* d_partials = nullptr;
  double* d_result = nullptr;
  double* h_result = nullptr;  // pinned
  int* d_snitems = nullptr;     // metric-series tile tables (built on first use)
  sclbm::TileItem* d_sitems = nullptr;
  int* d_s2nitems = nullptr;
  sclbm::TileItem* d_s2items = nullptr;
  int series2_nitems = 0;
  double* d_spartials = nullptr;
  double* d_srecords = nullptr;
  double* h_series = nullptr;  // pinned, kSeriesChunk records
  int series_nitems = 0;
  lbm_batch* batch = nullptr;  // non-null while driven by a batch
  int* flag = nullptr;         // status word set by the step kernels (InstDesc::flag)
  std::string arch;

  sclbm::InstDesc host_desc() const;
  lbm_status upload_tile(int k);
  lbm_status series_tiles();
  // n steps with the run's tile (multi-step tiles: launches of K steps; two
  // steps left over from a three-step tile in the two-step variant of the
  // same strips, one left over in a single step with the series strip tile).
  lbm_status advance(int64_t n);
  lbm_status diagnostics(lbm_metrics* out);
  lbm_status step_series(int64_t n, int32_t every, lbm_metrics* out, int32_t* count);
  lbm_metrics metrics_from_raw(const double* r, int64_t step) const;
};
