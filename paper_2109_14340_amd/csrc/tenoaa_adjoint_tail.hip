// Reverse-sweep tail tiles of the common variant: the few faces of a 2D or 3D
// sweep beyond its last whole 64-face tile (one face per pencil when the
// direction is non-periodic, n + 1 faces) in one-wave tiles of SWEEP_TAIL_TT
// pencils x SWEEP_TAIL_TN faces.  A translation unit of its own so that it
// compiles beside the whole-tile kernels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa_internal.h"
#include "tenoaa_vjp.h"

namespace tenoaa {

namespace {
template <int ORDER>
hipError_t tail(int ndim, int dir, const AdjointArgs& a, hipStream_t st) {
  constexpr int TT = SWEEP_TAIL_TT, TN = SWEEP_TAIL_TN;
  if (ndim == 2) {
    return dir == 0 ? launch_vjp_tiles<ORDER, 2, 0, TT, TN, false>(a, a.nf, st)
                    : launch_vjp_tiles<ORDER, 2, 1, TT, TN, false>(a, a.nf, st);
  }
  if (dir == 0) return launch_vjp_tiles<ORDER, 3, 0, TT, TN, false>(a, a.nf, st);
  if (dir == 1) return launch_vjp_tiles<ORDER, 3, 1, TT, TN, false>(a, a.nf, st);
  return launch_vjp_tiles<ORDER, 3, 2, TT, TN, false>(a, a.nf, st);
}
}  // namespace

hipError_t launch_vjp_tail(int order, int ndim, int dir, const AdjointArgs& a, hipStream_t st) {
  if (ndim < 2 || a.f_begin >= a.nf) return hipErrorInvalidValue;
  if (order == 12) return tail<12>(ndim, dir, a, st);
  return order == 10 ? tail<10>(ndim, dir, a, st) : tail<8>(ndim, dir, a, st);
}

}  // namespace tenoaa
