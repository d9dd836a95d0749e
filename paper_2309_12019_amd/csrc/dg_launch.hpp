// Interface between the C-ABI layer and the per-(dim, p) kernel objects.
#pragma once

#include "dg_adjoint.hpp"

namespace dgk {

enum LaunchKind { LAUNCH_STAGE = 0, LAUNCH_PROJECT = 1, LAUNCH_LAMBDA = 2, LAUNCH_BATCH = 3,
                  LAUNCH_ADJ_SENSOR = 4, LAUNCH_ADJ_GRAD = 5, LAUNCH_STEP = 6, LAUNCH_ADJ_GRAD_SENSOR = 7,
                  LAUNCH_SIGNATURE = 8 };

// the fused step kernel's tiles: 256 cells in 1D; in 2D 16 columns of
// kStepTile2D or kStepTile2DHalf rows (LAUNCH_STEP: args.ty)
constexpr int kStepTile1D = 256;
constexpr int kStepTile2D = 16;
constexpr int kStepTile2DHalf = 8;
// the adjoint kernels' 2D tile (rows of 32 cells: longer contiguous runs of
// the cell-major state than 16x16 for the same 256 threads); 1D adjoint
// launches use the stage kernel's tile
constexpr int kAdjTileX = 32;
constexpr int kAdjTileY = 8;

struct LaunchReq {
  int kind;
  int flux, mode;
  StageArgs args;       // LAUNCH_STAGE, LAUNCH_STEP, LAUNCH_LAMBDA
  int waves;            // LAUNCH_STAGE, 2D on 8x8 tiles: waves per tile (KPP: 4, 8 or 16, 0: 4;
                        // linear and Burgers: 4 for roles_kernel, else one)
  const double* src;    // LAUNCH_PROJECT: nodal values; LAUNCH_LAMBDA: state
  double* dst;          // LAUNCH_PROJECT: coefficients; LAUNCH_LAMBDA: block maxima
  long long ncells;
  hipStream_t stream;
  BatchStageArgs batch;  // LAUNCH_BATCH (tile shape in args.tx/args.ty, grid in ncells)
  int batch_one;         // LAUNCH_BATCH: one workgroup per tile (grid = batch.ntiles)
  AdjArgs adj;           // LAUNCH_ADJ_* (tile shape in adj.s.tx/adj.s.ty)
  uint32_t* sig;         // LAUNCH_SIGNATURE: branch records [3][cells] (stage input in args.uin)
};

typedef hipError_t (*LaunchFn)(const LaunchReq*);

}  // namespace dgk

extern "C" {
hipError_t dgk_launch_1_1(const dgk::LaunchReq*);
hipError_t dgk_launch_1_2(const dgk::LaunchReq*);
hipError_t dgk_launch_1_3(const dgk::LaunchReq*);
hipError_t dgk_launch_1_4(const dgk::LaunchReq*);
hipError_t dgk_launch_2_1(const dgk::LaunchReq*);
hipError_t dgk_launch_2_2(const dgk::LaunchReq*);
hipError_t dgk_launch_2_3(const dgk::LaunchReq*);
hipError_t dgk_launch_2_4(const dgk::LaunchReq*);
// dg_util.hip: partial[b] = non-finite entries of U[0..n) in block b's share
hipError_t dgk_count_nonfinite(const double* U, long long n, double* partial, int nblocks, hipStream_t st);
// dg_util.hip: clock[0] = t (one thread, on the stream: stage kernels read
// the BC_RIEMANN clock from device memory, so captured graphs replay at any time)
hipError_t dgk_set_clock(double* clock, double t, hipStream_t st);
// dg_util.hip: dst[0..n) = src[0..n)
hipError_t dgk_stream_copy(const double* src, double* dst, long long n, hipStream_t st);
}
