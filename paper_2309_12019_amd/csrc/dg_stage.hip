// Kernel instantiations for one (dimension, degree) pair.  The build compiles
// this file once per pair with -DDGK_DIM=<d> -DDGK_P=<p>, so the 8 pairs build
// in parallel; each object exports dgk_launch_<d>_<p>.
#include "dg_euler.hpp"
#include "dg_launch.hpp"

#ifndef DGK_DIM
#error "DGK_DIM must be defined"
#endif
#ifndef DGK_P
#error "DGK_P must be defined"
#endif

namespace dgk {
namespace {

template <int FLUX, int MODE, int TX, int TY, bool XBC = false>
hipError_t launch_tile(const StageArgs& A, hipStream_t st) {
  constexpr int NL = DGK_DIM == 1 ? DGK_P + 1 : (DGK_P + 1) * (DGK_P + 1);
  auto k = stage_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY, XBC>;
  const size_t lds = sizeof(double) * (size_t)stage_lds_doubles(DGK_DIM, NL, FLUX, TX, TY);
  if (lds > 65536) {
    // tiles above 64 KB of LDS: raise the per-kernel limit to what this launch needs
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((A.nx + TX - 1) / TX, DGK_DIM == 2 ? (A.ny + TY - 1) / TY : 1);
  dim3 block(DGK_DIM == 2 ? TX * TY : TX);
  hipLaunchKernelGGL(k, grid, block, lds, st, A);
  return hipGetLastError();
}

// the KPP flux on 8x8 tiles: NTH / 64 waves per tile (kpp_split_kernel)
template <int MODE, int NTH>
hipError_t launch_kpp_split_n(const StageArgs& A, hipStream_t st) {
  constexpr int NL = (DGK_P + 1) * (DGK_P + 1);
  auto k = kpp_split_kernel<DGK_P, MODE, NTH>;
  const size_t lds = sizeof(double) * (size_t)split_lds_doubles(NL, quad_points(2, DGK_P, FLUX_KPP));
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((A.nx + 7) / 8, (A.ny + 7) / 8);
  hipLaunchKernelGGL(k, grid, dim3(NTH), lds, st, A);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_kpp_split(const StageArgs& A, hipStream_t st, int waves) {
  // only the thread counts this degree runs without spilling are built
  if constexpr (split_max_waves(DGK_P) >= 16) {
    if (waves == 16) return launch_kpp_split_n<MODE, 1024>(A, st);
  }
  if constexpr (split_max_waves(DGK_P) >= 8) {
    if (waves >= 8) return launch_kpp_split_n<MODE, 512>(A, st);
  }
  return launch_kpp_split_n<MODE, 256>(A, st);
}

// linear and Burgers fluxes on 8x8 tiles, four waves per tile (roles_kernel)
template <int FLUX, int MODE, bool XBC>
hipError_t launch_roles(const StageArgs& A, hipStream_t st) {
  constexpr int NL = (DGK_P + 1) * (DGK_P + 1);
  auto k = roles_kernel<DGK_P, FLUX, MODE, XBC>;
  const size_t lds = sizeof(double) * (size_t)roles_lds_doubles(NL, DGK_P + 1);
  dim3 grid((A.nx + 7) / 8, (A.ny + 7) / 8);
  hipLaunchKernelGGL(k, grid, dim3(kRoleThreads), lds, st, A);
  return hipGetLastError();
}

template <int FLUX, int MODE>
hipError_t launch_stage_fm(const StageArgs& A, hipStream_t st, int waves = 0) {
  if constexpr (DGK_DIM == 1) {
    if (A.tx == 64) return launch_tile<FLUX, MODE, 64, 1>(A, st);
    return launch_tile<FLUX, MODE, 256, 1>(A, st);
  } else {
    // 2D Burgers: the kernel with the exact-solution exterior state only
    // where it is needed; 8x8 tiles of four waves on small meshes (waves = 4)
    if constexpr (FLUX == FLUX_BURGERS) {
      if (A.bc_kind == BC_RIEMANN) {
        if (A.tx == 8) {
          if (waves == 4) return launch_roles<FLUX, MODE, true>(A, st);
          return launch_tile<FLUX, MODE, 8, 8, true>(A, st);
        }
        return launch_tile<FLUX, MODE, 16, 16, true>(A, st);
      }
    }
    if constexpr (FLUX == FLUX_KPP) {
      if (A.tx == 8) return launch_kpp_split<MODE>(A, st, waves);
    } else {
      if (A.tx == 8) {
        if (waves == 4) return launch_roles<FLUX, MODE, false>(A, st);
        return launch_tile<FLUX, MODE, 8, 8>(A, st);
      }
    }
    return launch_tile<FLUX, MODE, 16, 16>(A, st);
  }
}

template <int FLUX, int MODE, int TY>
hipError_t launch_step_fmt(const StageArgs& A, hipStream_t st) {
  if constexpr (DGK_DIM == 2 && DGK_P == 4) {
    // the three tiles (242 KB) exceed the LDS of a workgroup: not built (the
    // library never selects the fused step here)
    return hipErrorInvalidValue;
  } else {
    constexpr int NL = DGK_DIM == 1 ? DGK_P + 1 : (DGK_P + 1) * (DGK_P + 1);
    constexpr int TX = DGK_DIM == 1 ? kStepTile1D : kStepTile2D;
    using G = StepGeom<DGK_DIM, TX, TY>;
    auto k = step_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY>;
    const size_t lds = sizeof(double) * (size_t)step_lds_doubles(DGK_DIM, NL, TX, TY);
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    dim3 grid((A.nx + TX - 1) / TX, DGK_DIM == 2 ? (A.ny + TY - 1) / TY : 1);
    hipLaunchKernelGGL(k, grid, dim3(G::NT), lds, st, A);
    return hipGetLastError();
  }
}

// 2D: A.ty = kStepTile2D or kStepTile2DHalf rows per tile
template <int FLUX, int MODE>
hipError_t launch_step_fm(const StageArgs& A, hipStream_t st) {
  if constexpr (DGK_DIM == 1) {
    return launch_step_fmt<FLUX, MODE, 1>(A, st);
  } else {
    if (A.ty == kStepTile2DHalf) return launch_step_fmt<FLUX, MODE, kStepTile2DHalf>(A, st);
    return launch_step_fmt<FLUX, MODE, kStepTile2D>(A, st);
  }
}

template <int FLUX>
hipError_t launch_step_f(int mode, const StageArgs& A, hipStream_t s) {
  switch (mode) {
    case MODE_DG: return launch_step_fm<FLUX, MODE_DG>(A, s);
    case MODE_LO: return launch_step_fm<FLUX, MODE_LO>(A, s);
    case MODE_ZHAO: return launch_step_fm<FLUX, MODE_ZHAO>(A, s);
    default: return launch_step_fm<FLUX, MODE_WENO>(A, s);
  }
}

template <int FLUX, int MODE, int TX, int TY, bool ONE>
hipError_t launch_batch_tile_k(const BatchStageArgs& B, int grid, hipStream_t st) {
  constexpr int NL = DGK_DIM == 1 ? DGK_P + 1 : (DGK_P + 1) * (DGK_P + 1);
  auto k = batch_stage_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY, ONE>;
  const size_t lds = sizeof(double) * (size_t)stage_lds_doubles(DGK_DIM, NL, FLUX, TX, TY);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(DGK_DIM == 2 ? TX * TY : TX), lds, st, B);
  return hipGetLastError();
}

template <int FLUX, int MODE, int TX, int TY>
hipError_t launch_batch_tile(const BatchStageArgs& B, int grid, bool one, hipStream_t st) {
  if (one) return launch_batch_tile_k<FLUX, MODE, TX, TY, true>(B, grid, st);
  return launch_batch_tile_k<FLUX, MODE, TX, TY, false>(B, grid, st);
}

template <int FLUX, int MODE>
hipError_t launch_batch_fm(const LaunchReq* r) {
  const int grid = (int)r->ncells;
  if constexpr (DGK_DIM == 1) {
    if (r->args.tx == 64) return launch_batch_tile<FLUX, MODE, 64, 1>(r->batch, grid, r->batch_one != 0, r->stream);
    return launch_batch_tile<FLUX, MODE, 256, 1>(r->batch, grid, r->batch_one != 0, r->stream);
  } else {
    if (r->args.tx == 8) return launch_batch_tile<FLUX, MODE, 8, 8>(r->batch, grid, r->batch_one != 0, r->stream);
    return launch_batch_tile<FLUX, MODE, 16, 16>(r->batch, grid, r->batch_one != 0, r->stream);
  }
}

template <int FLUX>
hipError_t launch_batch_f(const LaunchReq* r) {
  switch (r->mode) {
    case MODE_DG: return launch_batch_fm<FLUX, MODE_DG>(r);
    case MODE_LO: return launch_batch_fm<FLUX, MODE_LO>(r);
    case MODE_ZHAO: return launch_batch_fm<FLUX, MODE_ZHAO>(r);
    default: return launch_batch_fm<FLUX, MODE_WENO>(r);
  }
}

template <int FLUX, int MODE, int TX, int TY>
hipError_t launch_adj_tile(const LaunchReq* r) {
  constexpr int NL = DGK_DIM == 1 ? DGK_P + 1 : (DGK_P + 1) * (DGK_P + 1);
  constexpr int S = TileGeom<DGK_DIM, TX, TY>::S;
  const AdjArgs& Ad = r->adj;
  dim3 grid((Ad.s.nx + TX - 1) / TX, DGK_DIM == 2 ? (Ad.s.ny + TY - 1) / TY : 1);
  dim3 block(DGK_DIM == 2 ? TX * TY : TX);
  const bool sens = r->kind == LAUNCH_ADJ_SENSOR;
  const size_t lds = sizeof(double) * (size_t)NL * S * (sens ? 1 : 2);
  const void* k;
  if (r->kind == LAUNCH_ADJ_GRAD_SENSOR) {
    // only the stabilised operator has a sensor to reverse
    if constexpr (MODE != MODE_WENO)
      return hipErrorInvalidValue;
    else
      k = reinterpret_cast<const void*>(adj_grad_sensor_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY>);
  } else {
    k = sens ? reinterpret_cast<const void*>(adj_sensor_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY>)
             : reinterpret_cast<const void*>(adj_grad_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY>);
  }
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (r->kind == LAUNCH_ADJ_GRAD_SENSOR) {
    if constexpr (MODE == MODE_WENO)
      hipLaunchKernelGGL((adj_grad_sensor_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY>), grid, block, lds, r->stream,
                         Ad);
  } else if (sens) {
    hipLaunchKernelGGL((adj_sensor_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY>), grid, block, lds, r->stream, Ad);
  } else {
    hipLaunchKernelGGL((adj_grad_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY>), grid, block, lds, r->stream, Ad);
  }
  return hipGetLastError();
}

template <int FLUX, int MODE>
hipError_t launch_adj_fm(const LaunchReq* r) {
  if constexpr (DGK_DIM == 1) {
    if (r->adj.s.tx == 64) return launch_adj_tile<FLUX, MODE, 64, 1>(r);
    return launch_adj_tile<FLUX, MODE, 256, 1>(r);
  } else {
    return launch_adj_tile<FLUX, MODE, kAdjTileX, kAdjTileY>(r);
  }
}

template <int FLUX>
hipError_t launch_adj_f(const LaunchReq* r) {
  switch (r->mode) {
    case MODE_DG: return launch_adj_fm<FLUX, MODE_DG>(r);
    case MODE_LO: return launch_adj_fm<FLUX, MODE_LO>(r);
    case MODE_ZHAO: return hipErrorInvalidValue;  // no adjoint for this sensor
    default: return launch_adj_fm<FLUX, MODE_WENO>(r);
  }
}

template <int MODE, int TX>
hipError_t launch_euler_tile(const StageArgs& A, hipStream_t st) {
  constexpr int NLE = 3 * (DGK_P + 1);
  const size_t lds = sizeof(double) * (size_t)tile_lds_doubles(1, NLE, TX, 1);
  dim3 grid((A.nx + TX - 1) / TX), block(TX);
  hipLaunchKernelGGL((euler_stage_kernel<DGK_P, MODE, TX>), grid, block, lds, st, A);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_euler_m(const StageArgs& A, hipStream_t st) {
  if (A.tx == 64) return launch_euler_tile<MODE, 64>(A, st);
  return launch_euler_tile<MODE, 256>(A, st);
}

// the fused SSP-RK3 step of the Euler system (euler_step_kernel)
template <int MODE>
hipError_t launch_euler_step_m(const StageArgs& A, hipStream_t st) {
  auto k = euler_step_kernel<DGK_P, MODE>;
  const size_t lds = sizeof(double) * (size_t)euler_step_lds_doubles(DGK_P);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3((A.nx + kEulerStepTile - 1) / kEulerStepTile), dim3(kEulerStepThreads), lds, st, A);
  return hipGetLastError();
}

hipError_t launch_euler_step(int mode, const StageArgs& A, hipStream_t s) {
  switch (mode) {
    case MODE_DG: return launch_euler_step_m<MODE_DG>(A, s);
    case MODE_LO: return launch_euler_step_m<MODE_LO>(A, s);
    case MODE_ZHAO: return launch_euler_step_m<MODE_ZHAO>(A, s);
    default: return launch_euler_step_m<MODE_WENO>(A, s);
  }
}

hipError_t launch_euler(int mode, const StageArgs& A, hipStream_t s) {
  switch (mode) {
    case MODE_DG: return launch_euler_m<MODE_DG>(A, s);
    case MODE_LO: return launch_euler_m<MODE_LO>(A, s);
    case MODE_ZHAO: return launch_euler_m<MODE_ZHAO>(A, s);
    default: return launch_euler_m<MODE_WENO>(A, s);
  }
}

// branch records of a stage input (linear and Burgers fluxes, modes DG, LO,
// WENO: the adjoint's coverage), on the context's tile
template <int FLUX, int MODE, int TX, int TY>
hipError_t launch_sig_tile(const LaunchReq* r) {
  constexpr int NL = DGK_DIM == 1 ? DGK_P + 1 : (DGK_P + 1) * (DGK_P + 1);
  const StageArgs& A = r->args;
  auto k = signature_kernel<DGK_DIM, DGK_P, FLUX, MODE, TX, TY>;
  const size_t lds = sizeof(double) * (size_t)tile_lds_doubles(DGK_DIM, NL, TX, TY);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((A.nx + TX - 1) / TX, DGK_DIM == 2 ? (A.ny + TY - 1) / TY : 1);
  hipLaunchKernelGGL(k, grid, dim3(DGK_DIM == 2 ? TX * TY : TX), lds, r->stream, A, r->sig);
  return hipGetLastError();
}

template <int FLUX, int MODE>
hipError_t launch_sig_fm(const LaunchReq* r) {
  if constexpr (DGK_DIM == 1) {
    if (r->args.tx == 64) return launch_sig_tile<FLUX, MODE, 64, 1>(r);
    return launch_sig_tile<FLUX, MODE, 256, 1>(r);
  } else {
    if (r->args.tx == 8) return launch_sig_tile<FLUX, MODE, 8, 8>(r);
    return launch_sig_tile<FLUX, MODE, 16, 16>(r);
  }
}

template <int FLUX>
hipError_t launch_sig_f(const LaunchReq* r) {
  switch (r->mode) {
    case MODE_DG: return launch_sig_fm<FLUX, MODE_DG>(r);
    case MODE_LO: return launch_sig_fm<FLUX, MODE_LO>(r);
    case MODE_WENO: return launch_sig_fm<FLUX, MODE_WENO>(r);
    default: return hipErrorInvalidValue;
  }
}

template <int FLUX>
hipError_t launch_stage_f(int mode, const StageArgs& A, hipStream_t s, int waves = 0) {
  switch (mode) {
    case MODE_DG: return launch_stage_fm<FLUX, MODE_DG>(A, s, waves);
    case MODE_LO: return launch_stage_fm<FLUX, MODE_LO>(A, s, waves);
    case MODE_ZHAO: return launch_stage_fm<FLUX, MODE_ZHAO>(A, s, waves);
    default: return launch_stage_fm<FLUX, MODE_WENO>(A, s, waves);
  }
}

}  // namespace
}  // namespace dgk

#define DGK_CAT2(a, b, c) a##_##b##_##c
#define DGK_CAT(a, b, c) DGK_CAT2(a, b, c)

using namespace dgk;

extern "C" hipError_t DGK_CAT(dgk_launch, DGK_DIM, DGK_P)(const LaunchReq* r) {
  const StageArgs& A = r->args;
  switch (r->kind) {
    case LAUNCH_STAGE: {
      if (r->flux == FLUX_EULER) {
        if constexpr (DGK_DIM == 1) return launch_euler(r->mode, A, r->stream);
        return hipErrorInvalidValue;
      }
      if (r->flux == FLUX_LINADV) return launch_stage_f<FLUX_LINADV>(r->mode, A, r->stream, r->waves);
      if (r->flux == FLUX_BURGERS) return launch_stage_f<FLUX_BURGERS>(r->mode, A, r->stream, r->waves);
      if constexpr (DGK_DIM == 2) return launch_stage_f<FLUX_KPP>(r->mode, A, r->stream, r->waves);
      return hipErrorInvalidValue;
    }
    case LAUNCH_STEP: {
      if constexpr (DGK_DIM == 1) {
        if (r->flux == FLUX_EULER) return launch_euler_step(r->mode, A, r->stream);
      }
      if (r->flux == FLUX_LINADV) return launch_step_f<FLUX_LINADV>(r->mode, A, r->stream);
      if (r->flux == FLUX_BURGERS) return launch_step_f<FLUX_BURGERS>(r->mode, A, r->stream);
      if constexpr (DGK_DIM == 2) return launch_step_f<FLUX_KPP>(r->mode, A, r->stream);
      return hipErrorInvalidValue;
    }
    case LAUNCH_BATCH: {
      if (r->flux == FLUX_LINADV) return launch_batch_f<FLUX_LINADV>(r);
      if (r->flux == FLUX_BURGERS) return launch_batch_f<FLUX_BURGERS>(r);
      if constexpr (DGK_DIM == 2) return launch_batch_f<FLUX_KPP>(r);
      return hipErrorInvalidValue;
    }
    case LAUNCH_ADJ_SENSOR:
    case LAUNCH_ADJ_GRAD:
    case LAUNCH_ADJ_GRAD_SENSOR: {
      // the adjoint covers the linear and Burgers fluxes
      if (r->flux == FLUX_LINADV) return launch_adj_f<FLUX_LINADV>(r);
      if (r->flux == FLUX_BURGERS) return launch_adj_f<FLUX_BURGERS>(r);
      return hipErrorInvalidValue;
    }
    case LAUNCH_SIGNATURE: {
      if (r->flux == FLUX_LINADV) return launch_sig_f<FLUX_LINADV>(r);
      if (r->flux == FLUX_BURGERS) return launch_sig_f<FLUX_BURGERS>(r);
      return hipErrorInvalidValue;
    }
    case LAUNCH_PROJECT: {
      const long long n = r->ncells;
      dim3 grid((unsigned)((n + 255) / 256)), block(256);
      hipLaunchKernelGGL((project_kernel<DGK_DIM, DGK_P>), grid, block, 0, r->stream, r->src, r->dst, n);
      return hipGetLastError();
    }
    case LAUNCH_LAMBDA: {
      const long long n = r->ncells;
      dim3 grid((unsigned)((n + 255) / 256)), block(256);
      if (r->flux == FLUX_EULER) {
        if constexpr (DGK_DIM == 1) {
          hipLaunchKernelGGL((euler_lambda_kernel<DGK_P>), grid, block, 0, r->stream, A, r->src, r->dst);
          return hipGetLastError();
        }
        return hipErrorInvalidValue;
      }
      if (r->flux == FLUX_LINADV)
        hipLaunchKernelGGL((lambda_kernel<DGK_DIM, DGK_P, FLUX_LINADV>), grid, block, 0, r->stream, A, r->src,
                           r->dst);
      else if (r->flux == FLUX_BURGERS)
        hipLaunchKernelGGL((lambda_kernel<DGK_DIM, DGK_P, FLUX_BURGERS>), grid, block, 0, r->stream, A, r->src,
                           r->dst);
      else if constexpr (DGK_DIM == 2)
        hipLaunchKernelGGL((lambda_kernel<DGK_DIM, DGK_P, FLUX_KPP>), grid, block, 0, r->stream, A, r->src,
                           r->dst);
      else
        return hipErrorInvalidValue;
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}
