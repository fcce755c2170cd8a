// sc_launch.h -- host-side launchers of the gfx950 kernels (internal to the
// library; the public boundary is include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc_device.h"

namespace sclbm {

// Step-kernel variants: NT threads per workgroup, CPT cells per thread, PF
// rows of loads in flight.  Marching-strip variants (paired = 0) cover
// NT * CPT columns per workgroup; paired-column variants (paired = 1, CPT = 2)
// cover kPairColumns per wavefront and need an even nx >= 128.  Two-step
// variants (steps = 2, CPT = 1) advance `width` <= NT - kFusedHalo columns by
// two time steps per launch, three-step variants (steps = 3, FP32 only)
// `width` <= NT - 10 columns by three (0 for the other kinds).
struct StepVariant {
  int threads, cells, prefetch, paired, steps, width;
};
constexpr int kNumVariants = 33;
constexpr int kFusedHalo = 6;
constexpr int kPairColumns = 124;
constexpr int kPairMinNx = 128;
// Band heights a tile shape may use; tile shape k = variant * kNumRows + row
// index.  The short bands (2, 4 rows) give grids too small to fill the GPU
// with long bands enough workgroups in flight.  0 = balanced: the height that
// makes the grid about two rounds of the workgroups the GPU holds at once
// (kBalancedRounds), computed per grid, storage and device.
constexpr int kRowChoices[] = {8, 16, 32, 64, 128, 2, 4, 0};
constexpr int kNumRows = 8;
constexpr int kBalancedRounds = 2;
constexpr int kMaxBalancedRows = 256;
constexpr int kNumTiles = kNumVariants * kNumRows;
constexpr int kMinStripWidth = 64;
constexpr int kMinRows = 2;

// Storage forms (LBM_F32, LBM_F16_SHIFTED, LBM_F16_CELL, LBM_F16_MOMENT).
constexpr int kNumStorages = 4;

// Longest graph of batched steps (time steps per replay).
constexpr int kMaxGraphSteps = 4096;

// Reductions: at most kMaxPartials blocks, kPartialStride doubles each.
constexpr int kMaxPartials = 2048;
constexpr int kPartialStride = 16;

struct InitArgs {
  int nx, ny;
  double rho_l, rho_g, width, noise_amp;
  uint64_t seed;
  int64_t period_x, period_y, origin_x, origin_y;
};

const StepVariant& step_variant(int v);

// One step launch: workgroup b takes items b, b + grid, ...
hipError_t launch_step(int storage, int variant, const InstDesc* descs, const TileItem* items,
                       const int* nitems, int grid, int sub, hipStream_t st);
hipError_t step_occupancy(int storage, int variant, int* blocks_per_cu);
hipError_t launch_tick_end(InstDesc* descs, int n, hipStream_t st);
hipError_t launch_moments(int storage, const void* src, int nx, int ny, float rho0, float G,
                          float* rho, float* ux, float* uy, hipStream_t st);
hipError_t launch_get_state(int storage, const void* src, int nx, int ny, float rho0, float* f,
                            hipStream_t st);
hipError_t launch_set_state(int storage, const float* f, int nx, int ny, float rho0, void* dst,
                            hipStream_t st);
hipError_t launch_init(int storage, const double* drops, int nd, const InitArgs& a, double* rho64,
                       float rho0, void* dst, hipStream_t st);
// Blocks of the diagnostics pass on an nx x ny grid (partial records it
// writes; at most kMaxPartials).
int diagnostics_blocks(int nx, int ny);
// Writes {mass, mom_x, mom_y, bad, n_above, Gmax, sum_grad, sum_grad2, rho_max, rho_min} to out.
hipError_t launch_diagnostics(int storage, const void* src, int nx, int ny, float rho0,
                              double* rho64, double* partials, double* out, hipStream_t st);
// One step that also records the diagnostics of the state it advances (the
// ten values of launch_diagnostics, to out).  Strip tile of kSeriesThreads
// threads x 1 cell, 2 rows in flight; `grid` = number of items (one partial
// record of kPartialStride doubles each).
constexpr int kSeriesThreads = 256;
constexpr int kSeriesChunk = 256;  // records kept on the device between copies
hipError_t launch_step_diag(int storage, const InstDesc* descs, const TileItem* items,
                            const int* nitems, int grid, int sub, double* partials,
                            double* out, hipStream_t st);
// Two steps with the diagnostics of the state they advance: two-step tile of
// kSeriesThreads threads, 1 row in flight (kSeries2Rows-row bands); `grid` =
// number of items (one partial record each).
constexpr int kSeries2Rows = 16;
// Columns of the recording tile's strips: 240 for FP32 storage (strips that
// start and end on 64-byte boundaries), kSeriesThreads - kFusedHalo for the
// FP16 forms (storage index 0 is FP32).
constexpr int kSeries2WidthF32 = 240;
constexpr int series2_width(int storage) {
  return storage == 0 ? kSeries2WidthF32 : kSeriesThreads - kFusedHalo;
}
hipError_t launch_step2_diag(int storage, const InstDesc* descs, const TileItem* items,
                             const int* nitems, int grid, int sub, double* partials, double* out,
                             hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);

}  // namespace sclbm
