// Kernel instantiations for one (dimension, degree) pair.  The build compiles
// this file once per pair with -DDGK_DIM=<d> -DDGK_P=<p>, so the 8 pairs build
// in parallel; each object exports dgk_launch_<d>_<p>.
#include "dg_launch.hpp"

#ifndef DGK_DIM
#error "DGK_DIM must be defined"
#endif
#ifndef DGK_P
#error "DGK_P must be defined"
#endif

namespace dgk {
namespace {

template <int FLUX, int MODE>
hipError_t launch_stage_fm(const StageArgs& A, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
  auto k = stage_kernel<DGK_DIM, DGK_P, FLUX, MODE>;
  if (lds > 65536) {
    // tiles above 64 KB of LDS: raise the per-kernel limit to what this launch needs
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, grid, block, lds, st, A);
  return hipGetLastError();
}

template <int FLUX>
hipError_t launch_stage_f(int mode, const StageArgs& A, dim3 g, dim3 b, size_t l, hipStream_t s) {
  switch (mode) {
    case MODE_DG: return launch_stage_fm<FLUX, MODE_DG>(A, g, b, l, s);
    case MODE_LO: return launch_stage_fm<FLUX, MODE_LO>(A, g, b, l, s);
    default: return launch_stage_fm<FLUX, MODE_WENO>(A, g, b, l, s);
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
      const int tx = A.tx, ty = DGK_DIM == 2 ? A.ty : 1;
      dim3 grid((A.nx + tx - 1) / tx, DGK_DIM == 2 ? (A.ny + ty - 1) / ty : 1);
      dim3 block(tx * ty);
      constexpr int NL = DGK_DIM == 1 ? DGK_P + 1 : (DGK_P + 1) * (DGK_P + 1);
      size_t lds = sizeof(double) * NL * (size_t)A.lds_stride;
      if (r->flux == FLUX_LINADV) return launch_stage_f<FLUX_LINADV>(r->mode, A, grid, block, lds, r->stream);
      return launch_stage_f<FLUX_BURGERS>(r->mode, A, grid, block, lds, r->stream);
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
      if (r->flux == FLUX_LINADV)
        hipLaunchKernelGGL((lambda_kernel<DGK_DIM, DGK_P, FLUX_LINADV>), grid, block, 0, r->stream, A, r->src,
                           r->dst);
      else
        hipLaunchKernelGGL((lambda_kernel<DGK_DIM, DGK_P, FLUX_BURGERS>), grid, block, 0, r->stream, A, r->src,
                           r->dst);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}
