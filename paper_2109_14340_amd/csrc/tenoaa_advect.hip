// Scalar linear advection u_t + u_x = 0 on a periodic 1D grid, the accuracy
// test of the paper's Sec. 5.1 (Gaussian pulse): the flux f = u moves with
// speed +1, so each face takes the upwind-biased TENO-AA reconstruction
// fhat_{i+1/2} of f from cells i-G+1 .. i+G (Sec. 3-4), the semi-discrete
// form is du_i/dt = -(fhat_{i+1/2} - fhat_{i-1/2}) / dx (Sec. 2) and SSP-RK3
// (Sec. 5) advances it.
//
// The grids of this test are small (tens to a few thousand cells) and are
// run for very many steps with a tiny dt, so one workgroup keeps the whole
// grid in LDS and runs every step of a call in a single launch, with
// workgroup barriers between the reconstruction and update phases; no state
// leaves LDS until the last step.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa.h"
#include "tenoaa_device.h"
#include "tenoaa_internal.h"

namespace tenoaa {
namespace {

constexpr int ADV_THREADS = 1024;
constexpr int64_t ADV_MAX_CELLS = 2048;  // three LDS arrays of doubles: 48 KiB

template <int ORDER>
__global__ __launch_bounds__(ADV_THREADS) void advect_kernel(double* u, int n, double dx, double dt, int64_t nsteps) {
  constexpr int G = ORDER / 2;
  extern __shared__ double lds[];
  double* un = lds;         // u^n
  double* us = lds + n;     // the stage state u1, then u2 (in place)
  double* fh = lds + 2 * n; // fhat_{i+1/2}
  for (int i = threadIdx.x; i < n; i += ADV_THREADS) un[i] = u[i];
  __syncthreads();
  // fhat of every face from the state s, then the stage combination
  auto faces = [&](const double* s) {
    for (int i = threadIdx.x; i < n; i += ADV_THREADS) {
      double v[ORDER];
      unroll<ORDER>([&](auto k) {
        int j = i - G + 1 + (int)k;
        j = j < 0 ? j + n : (j >= n ? j - n : j);
        v[k] = s[j];
      });
      uint8_t flag;
      fh[i] = teno_aa<ORDER>(v, flag);
    }
    __syncthreads();
  };
  auto dudt = [&](int i) {
    const int im = i == 0 ? n - 1 : i - 1;
    return -div_rn(fh[i] - fh[im], dx);
  };
  for (int64_t step = 0; step < nsteps; ++step) {
    faces(un);
    for (int i = threadIdx.x; i < n; i += ADV_THREADS) us[i] = un[i] + dt * dudt(i);
    __syncthreads();
    faces(us);
    for (int i = threadIdx.x; i < n; i += ADV_THREADS) us[i] = 0.75 * un[i] + 0.25 * us[i] + (0.25 * dt) * dudt(i);
    __syncthreads();
    faces(us);
    for (int i = threadIdx.x; i < n; i += ADV_THREADS)
      un[i] = (1.0 / 3.0) * un[i] + (2.0 / 3.0) * us[i] + ((2.0 / 3.0) * dt) * dudt(i);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += ADV_THREADS) u[i] = un[i];
}

}  // namespace
}  // namespace tenoaa

extern "C" int tenoaa_advect(int32_t order, int64_t n, double dx, double dt, int64_t nsteps, double* u,
                             void* stream) {
  if (order != 8 && order != 10 && order != 12) return TENOAA_EINVAL;
  if (n < order || n > tenoaa::ADV_MAX_CELLS || !u || nsteps < 0) return TENOAA_EINVAL;
  if (!(dx > 0.0) || !(dt > 0.0) || dx > 1e300 || dt > 1e300) return TENOAA_EINVAL;
  if (nsteps == 0) return TENOAA_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t lds = 3 * (size_t)n * sizeof(double);
  if (order == 12)
    hipLaunchKernelGGL(tenoaa::advect_kernel<12>, dim3(1), dim3(tenoaa::ADV_THREADS), lds, st, u, (int)n, dx, dt,
                       nsteps);
  else if (order == 10)
    hipLaunchKernelGGL(tenoaa::advect_kernel<10>, dim3(1), dim3(tenoaa::ADV_THREADS), lds, st, u, (int)n, dx, dt,
                       nsteps);
  else
    hipLaunchKernelGGL(tenoaa::advect_kernel<8>, dim3(1), dim3(tenoaa::ADV_THREADS), lds, st, u, (int)n, dx, dt,
                       nsteps);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    tenoaa::record_hip_error(e);
    return TENOAA_EHIP;
  }
  return TENOAA_OK;
}
