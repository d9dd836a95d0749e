// Device utilities outside the method: the count of non-finite state
// entries (dg_check_finite) and a plain streaming copy (dg_stream_copy), the
// measured bandwidth ceiling the stage kernels' traffic is read against.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg_launch.hpp"

namespace dgk {
namespace {

// Non-finite entries of U[0..n): grid-stride; block b writes its count (a
// double, exact below 2^53) to partial[b].
__global__ void __launch_bounds__(256) count_nonfinite_kernel(const double* __restrict__ U, long long n,
                                                               double* __restrict__ partial) {
  __shared__ double red[256];
  double bad = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    bad += isfinite(U[i]) ? 0.0 : 1.0;
  red[threadIdx.x] = bad;
  tile_barrier();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    tile_barrier();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dst = src, 16 bytes per lane (both 16-byte aligned), one pair per thread
__global__ void __launch_bounds__(256) copy2_kernel(const double2* __restrict__ src, double2* __restrict__ dst,
                                                     long long n2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n2) dst[i] = src[i];
}

// dst = src, 8 bytes per lane
__global__ void __launch_bounds__(256) copy1_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                     long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace
}  // namespace dgk

namespace dgk {
__global__ void __launch_bounds__(64) set_clock_kernel(double* clock, double t) {
  if (threadIdx.x == 0) clock[0] = t;
}
}  // namespace dgk

extern "C" hipError_t dgk_set_clock(double* clock, double t, hipStream_t st) {
  hipLaunchKernelGGL(dgk::set_clock_kernel, dim3(1), dim3(64), 0, st, clock, t);
  return hipGetLastError();
}

extern "C" hipError_t dgk_count_nonfinite(const double* U, long long n, double* partial, int nblocks,
                                          hipStream_t st) {
  hipLaunchKernelGGL(dgk::count_nonfinite_kernel, dim3(nblocks), dim3(256), 0, st, U, n, partial);
  return hipGetLastError();
}

extern "C" hipError_t dgk_stream_copy(const double* src, double* dst, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const bool a16 = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0;
  if (a16) {
    const long long n2 = n / 2;
    if (n2 > 0)
      hipLaunchKernelGGL(dgk::copy2_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st,
                         reinterpret_cast<const double2*>(src), reinterpret_cast<double2*>(dst), n2);
    if (n & 1) hipLaunchKernelGGL(dgk::copy1_kernel, dim3(1), dim3(256), 0, st, src + 2 * n2, dst + 2 * n2, 1LL);
  } else {
    hipLaunchKernelGGL(dgk::copy1_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  }
  return hipGetLastError();
}
