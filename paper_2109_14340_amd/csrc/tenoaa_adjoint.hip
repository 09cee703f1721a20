// Reverse-sweep launchers of the common case (LLF or Rusanov, no prescribed
// sides) in whole tiles, and the element-wise kernels of the step adjoint's
// SSP-RK3 chain.  The reverse sweep itself is in tenoaa_vjp.h.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa_internal.h"
#include "tenoaa_vjp.h"

namespace tenoaa {
namespace {

__global__ void zero_kernel(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// out = a*x + b*y + c*z (element-wise; null operands skipped) for the RK3 chain.
__global__ void axpbypcz_kernel(double* out, double a, const double* x, double b, const double* y, double c,
                                const double* z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * x[i];
    if (y) v = v + b * y[i];
    if (z) v = v + c * z[i];
    out[i] = v;
  }
}

// out = a*x + (c * dt) * z with dt read on the device.
__global__ void axpdtz_kernel(double* out, double a, const double* x, double c, const double* dt, const double* z,
                              int64_t n) {
  const double cd = c * (*dt);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a * x[i] + cd * z[i];
}

}  // namespace

hipError_t launch_sweep_vjp(int order, int ndim, int dir, const AdjointArgs& a, hipStream_t st) {
  // the Roe flux's one-sided fields and the ghost rules of prescribed sides
  // in a variant of their own (whole tiles only), which the common case does
  // not carry.  The common case sends a remainder of at most SWEEP_TAIL_TN
  // faces beyond the last whole 64-face tile of a direction (non-periodic
  // directions have n + 1) to one-wave tail tiles
  if (a.splitting == TENOAA_ROE || a.bcv[0] || a.bcv[1]) return launch_vjp_general(order, ndim, dir, a, st);
  const int64_t rem = a.nf % (dir == 0 ? TENOAA_ADJ_TN_X : TENOAA_ADJ_TN_YZ);
  const bool tail = ndim > 1 && rem > 0 && rem <= SWEEP_TAIL_TN;
  const int64_t whole = tail ? a.nf - rem : a.nf;
  if (whole > 0) {
    const hipError_t e = launch_vjp_kind<false>(order, ndim, dir, a, whole, st);
    if (e != hipSuccess || whole == a.nf) return e;
  }
  AdjointArgs t = a;
  t.f_begin = whole;
  return launch_vjp_tail(order, ndim, dir, t, st);
}

static unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_axpbypcz(double* out, double a, const double* x, double b, const double* y, double c,
                           const double* z, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpbypcz_kernel, dim3(grid_for(n)), dim3(256), 0, st, out, a, x, b, y, c, z, n);
  return hipGetLastError();
}

hipError_t launch_axpdtz(double* out, double a, const double* x, double c, const double* dt, const double* z,
                         int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpdtz_kernel, dim3(grid_for(n)), dim3(256), 0, st, out, a, x, c, dt, z, n);
  return hipGetLastError();
}

}  // namespace tenoaa
