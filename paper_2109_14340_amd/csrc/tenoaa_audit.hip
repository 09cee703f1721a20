// The audit sweep: the forward sweep with every decision taken live except
// those a near-threshold mask marks, which replay recorded decisions, and
// with each live decision's distance to its thresholds reported (1 where a
// test lies within a relative tolerance of its threshold).  It serves the
// finite-difference check of the adjoint, whose perturbed runs must take the
// decisions that are far from a threshold live and freeze only the near
// ones.  Built in a translation unit of its own so that it compiles beside
// the other sweeps; LLF and Rusanov splitting (chosen at run time), whole
// tiles over every face of a direction.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa_device.h"
#include "tenoaa_internal.h"
#include "tenoaa_stencil.h"

namespace tenoaa {
namespace {

template <int ORDER, int NDIM, int DIR, int TT, int TN, bool LIMIT>
__global__ __launch_bounds__(TT* TN) __attribute__((amdgpu_waves_per_eu(3)))
void sweep_audit_kernel(SweepArgs A) {
  __shared__ __align__(16) char arena[SweepShape<ORDER, NDIM, TT, TN>::LDS_BYTES];
  const double mu = LIMIT ? A.mu[DIR] : 0.0;
  sweep_tile<ORDER, NDIM, DIR, TT, TN, LIMIT, SPLIT_RUNTIME, true>(A, arena, blockIdx.x, blockIdx.y, blockIdx.z, mu);
}

template <int ORDER, int NDIM, int DIR, bool LIMIT>
hipError_t launch_t(const SweepArgs& a, hipStream_t st) {
  constexpr int TT = (NDIM == 1) ? 1 : (DIR == 0 ? 4 : 8);
  constexpr int TN = (DIR == 0) ? 64 : 32;
  constexpr int AX_A = (DIR == 0) ? 1 : 0;
  constexpr int AX_B = (DIR == 2) ? 1 : 2;
  dim3 grid((unsigned)((a.nf + TN - 1) / TN), (unsigned)((a.n[AX_A] + TT - 1) / TT), (unsigned)a.n[AX_B]);
  hipLaunchKernelGGL((sweep_audit_kernel<ORDER, NDIM, DIR, TT, TN, LIMIT>), grid, dim3(TT * TN), 0, st, a);
  return hipGetLastError();
}

template <int ORDER, int NDIM, int DIR>
hipError_t launch_o(const SweepArgs& a, bool limit, hipStream_t st) {
  return limit ? launch_t<ORDER, NDIM, DIR, true>(a, st) : launch_t<ORDER, NDIM, DIR, false>(a, st);
}

template <int ORDER>
hipError_t launch_ord(int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st) {
  if (ndim == 1) return launch_o<ORDER, 1, 0>(a, limit, st);
  if (ndim == 2) return dir == 0 ? launch_o<ORDER, 2, 0>(a, limit, st) : launch_o<ORDER, 2, 1>(a, limit, st);
  if (dir == 0) return launch_o<ORDER, 3, 0>(a, limit, st);
  if (dir == 1) return launch_o<ORDER, 3, 1>(a, limit, st);
  return launch_o<ORDER, 3, 2>(a, limit, st);
}

}  // namespace

hipError_t launch_sweep_audit(int order, int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st) {
  if (a.splitting == TENOAA_ROE || a.f_begin != 0) return hipErrorInvalidValue;
  if (order == 12) return launch_ord<12>(ndim, dir, a, limit, st);
  return order == 10 ? launch_ord<10>(ndim, dir, a, limit, st) : launch_ord<8>(ndim, dir, a, limit, st);
}

}  // namespace tenoaa
