// Tail tiles of the forward sweeps: the few faces of a direction beyond its
// last whole 32- or 64-face tile (one face per pencil when a non-periodic
// direction has n + 1 faces) in tiles of 16 pencils x 4 faces, one wave each,
// with the same per-face code as the whole tiles.  Built in a translation
// unit of its own so that it compiles beside the whole-tile kernels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa_device.h"
#include "tenoaa_internal.h"
#include "tenoaa_stencil.h"

namespace tenoaa {
namespace {

constexpr int TAIL_TT = SWEEP_TAIL_TT, TAIL_TN = SWEEP_TAIL_TN;
static_assert(TAIL_TT * TAIL_TN == 64, "a tail tile is one wave");

template <int ORDER, int NDIM, int DIR, bool LIMIT, bool ROE>
__global__ __launch_bounds__(TAIL_TT* TAIL_TN) __attribute__((amdgpu_waves_per_eu(3)))
void sweep_tail_kernel(SweepArgs A) {
  __shared__ __align__(16) char arena[SweepShape<ORDER, NDIM, TAIL_TT, TAIL_TN>::LDS_BYTES];
  const double mu = LIMIT ? A.mu[DIR] : 0.0;
  sweep_tile<ORDER, NDIM, DIR, TAIL_TT, TAIL_TN, LIMIT, ROE ? TENOAA_ROE : SPLIT_RUNTIME>(A, arena, blockIdx.x, blockIdx.y,
                                                                                  blockIdx.z, mu);
}

template <int ORDER, int NDIM, int DIR, bool LIMIT, bool ROE>
hipError_t launch_t(const SweepArgs& a, hipStream_t st) {
  constexpr int AX_A = (DIR == 0) ? 1 : 0;
  constexpr int AX_B = (DIR == 2) ? 1 : 2;
  const int64_t rest = a.nf - a.f_begin;
  dim3 grid((unsigned)((rest + TAIL_TN - 1) / TAIL_TN), (unsigned)((a.n[AX_A] + TAIL_TT - 1) / TAIL_TT),
            (unsigned)a.n[AX_B]);
  hipLaunchKernelGGL((sweep_tail_kernel<ORDER, NDIM, DIR, LIMIT, ROE>), grid, dim3(TAIL_TT * TAIL_TN), 0, st, a);
  return hipGetLastError();
}

template <int ORDER, int NDIM, int DIR>
hipError_t launch_o(const SweepArgs& a, bool limit, hipStream_t st) {
  if (a.splitting == TENOAA_ROE) return limit ? launch_t<ORDER, NDIM, DIR, true, true>(a, st)
                                              : launch_t<ORDER, NDIM, DIR, false, true>(a, st);
  return limit ? launch_t<ORDER, NDIM, DIR, true, false>(a, st) : launch_t<ORDER, NDIM, DIR, false, false>(a, st);
}

template <int ORDER>
hipError_t launch_ord(int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st) {
  if (ndim == 2) return dir == 0 ? launch_o<ORDER, 2, 0>(a, limit, st) : launch_o<ORDER, 2, 1>(a, limit, st);
  if (dir == 0) return launch_o<ORDER, 3, 0>(a, limit, st);
  if (dir == 1) return launch_o<ORDER, 3, 1>(a, limit, st);
  return launch_o<ORDER, 3, 2>(a, limit, st);
}

}  // namespace

hipError_t launch_sweep_tail(int order, int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st) {
  if (ndim < 2 || a.f_begin >= a.nf) return hipErrorInvalidValue;
  if (order == 12) return launch_ord<12>(ndim, dir, a, limit, st);
  return order == 10 ? launch_ord<10>(ndim, dir, a, limit, st) : launch_ord<8>(ndim, dir, a, limit, st);
}

}  // namespace tenoaa
