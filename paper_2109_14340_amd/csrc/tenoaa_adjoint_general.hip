// Reverse-sweep launches of the general variant: the Roe flux (fields
// reconstructed from one side) and grids with Dirichlet or inflow sides (the
// ghost rules and their Jacobians), in whole tiles.  A translation unit of
// its own so that it compiles beside the common variant.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa_internal.h"
#include "tenoaa_vjp.h"

namespace tenoaa {

hipError_t launch_vjp_general(int order, int ndim, int dir, const AdjointArgs& a, hipStream_t st) {
  return launch_vjp_kind<true>(order, ndim, dir, a, a.nf, st);
}

}  // namespace tenoaa
