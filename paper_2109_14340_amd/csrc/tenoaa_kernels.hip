// TENO-AA8/10 Euler right-hand side: HIP kernels for gfx950 (FP64 VALU).
//
// One sweep kernel per direction evaluates every face flux of that direction:
// a block stages a tile of cells (plus the reconstruction halo, with the
// boundary conditions applied by index mapping) in LDS as per-cell records
// (conserved state and physical flux in the face's local frame, normal and
// tangential velocity, sound speed, sqrt(rho), enthalpy), then each thread
// takes one face: Roe average and eigenvectors (Sec. 5 of the paper),
// projection of the window onto one characteristic field at a time, LLF or
// Rusanov splitting, the scalar TENO-AA reconstruction of both split sides
// (Sec. 3, 4), back-projection and the optional positivity limiter.  Face
// fluxes go to a face array; a separate element-wise kernel forms the flux
// difference and the SSP-RK3 stage.
//
// Bit-for-bit agreement with the reference evaluation.  Every value that
// feeds a threshold decision (the split characteristic fluxes) is computed
// with one fixed order of IEEE operations: no contraction (this file is built
// with -ffp-contract=off), fma only where written, correctly rounded division
// and square root.  The smoothness indicators, the scale-separation test and
// the C_T bucket may differ from a reference evaluation by a few ulps, which
// can only move a decision that lies within ~1e-14 of its threshold.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "tenoaa_device.h"
#include "tenoaa_internal.h"
#include "tenoaa_stencil.h"

// Launch-shape tunables (overridable at build time).
#ifndef TENOAA_WAVES_PER_EU
#define TENOAA_WAVES_PER_EU 3
#endif
#ifndef TENOAA_TN_X
#define TENOAA_TN_X 64
#endif
#ifndef TENOAA_TT_X
#define TENOAA_TT_X 4
#endif
#ifndef TENOAA_TN_YZ
#define TENOAA_TN_YZ 32
#endif
#ifndef TENOAA_TT_YZ
#define TENOAA_TT_YZ 8
#endif

namespace tenoaa {
namespace {

// ------------------------------------------------------------ sweep kernel
template <int ORDER, int NDIM, int DIR, int TT, int TN, bool LIMIT, int SPLIT>
__global__ __launch_bounds__(TT* TN)
#if TENOAA_WAVES_PER_EU > 0
__attribute__((amdgpu_waves_per_eu(TENOAA_WAVES_PER_EU)))
#endif
void sweep_kernel(SweepArgs A) {
  __shared__ __align__(16) char arena[SweepShape<ORDER, NDIM, TT, TN>::LDS_BYTES];
  const double mu = LIMIT ? A.mu[DIR] : 0.0;
  sweep_tile<ORDER, NDIM, DIR, TT, TN, LIMIT, SPLIT>(A, arena, blockIdx.x, blockIdx.y, blockIdx.z, mu);
}

// --------------------------------------------------- flux difference / RK
template <int NDIM, int MODE>
__global__ __launch_bounds__(256) void update_kernel(UpdateArgs A) {
  const int64_t ncell = A.n[0] * A.n[1] * A.n[2];
  const double dt = (MODE == 0) ? 0.0 : *A.dt;
  const bool small = ncell < ((int64_t)1 << 32);
  const FastDiv d0{A.div_m[0], A.div_l[0]}, d1{A.div_m[1], A.div_l[1]};
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ncell;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t co[3];
    if (small) {
      const uint32_t q0 = fastdiv((uint32_t)idx, d0);
      const uint32_t q1 = fastdiv(q0, d1);
      co[0] = (int64_t)((uint32_t)idx - q0 * (uint32_t)A.n[0]);
      co[1] = (int64_t)(q0 - q1 * (uint32_t)A.n[1]);
      co[2] = (int64_t)q1;
    } else {
      co[0] = idx % A.n[0];
      co[1] = (idx / A.n[0]) % A.n[1];
      co[2] = idx / (A.n[0] * A.n[1]);
    }
    double Wn[NDIM + 2];
    update_cell<NDIM, MODE>(A, idx, co, dt, Wn);
  }
}

// ---------------------------------------------------------- wave speeds / dt
__global__ void init_scalars_kernel(Scalars* S) {
  if (threadIdx.x == 0) {
    S->amax_bits[0] = S->amax_bits[1] = S->amax_bits[2] = 0ull;
  }
}

template <int NDIM>
__global__ __launch_bounds__(256) void wave_speed_kernel(const double* U, int64_t ncell, double gam, Scalars* S,
                                                         int* status) {
  constexpr int NV = NDIM + 2;
  double amax[NDIM];
  unroll<NDIM>([&](auto d) { amax[d] = 0.0; });
  bool bad = false;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ncell;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double Wc[NV];
    unroll<NV>([&](auto c) { Wc[c] = U[c * ncell + idx]; });
    cell_speeds<NDIM>(Wc, gam, amax, bad);
  }
  if (bad) atomicOr(status, 1);
  __shared__ double red[NDIM][256];
  unroll<NDIM>([&](auto d) { red[d][threadIdx.x] = amax[d]; });
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      unroll<NDIM>([&](auto d) { red[d][threadIdx.x] = dmax(red[d][threadIdx.x], red[d][threadIdx.x + s]); });
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    unroll<NDIM>([&](auto d) {
      // non-negative doubles order like their bit patterns
      atomicMax(&S->amax_bits[d], (unsigned long long)__double_as_longlong(red[d][0]));
    });
  }
}

// The ghost cells next to the faces of one side with prescribed values
// (Dirichlet: the boundary cell reflected through the face values; inflow:
// the first prescribed layer) folded into the wave speeds, as the boundary
// faces see them.  One thread per cell of the face plane.
template <int NDIM>
__global__ __launch_bounds__(256) void ghost_speed_kernel(GhostSpeedArgs A, Scalars* S, int* status) {
  constexpr int NV = NDIM + 2;
  double amax[NDIM];
  unroll<NDIM>([&](auto d) { amax[d] = 0.0; });
  bool bad = false;
  const int64_t ncell = A.n[0] * A.n[1] * A.n[2];
  const int64_t stride[3] = {1, A.n[0], A.n[0] * A.n[1]};
  const int a0 = (A.dir == 0) ? 1 : 0, a1 = (A.dir == 2) ? 1 : 2;
  const int64_t plane = A.n[a0] * A.n[a1];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o0 = p % A.n[a0], o1 = p / A.n[a0];
    const int64_t cell = (A.hi ? A.n[A.dir] - 1 : 0) * stride[A.dir] + o0 * stride[a0] + o1 * stride[a1];
    double Wc[NV];
    if (A.bc == TENOAA_BC_DIRICHLET) {
      unroll<NV>([&](auto c) { Wc[c] = A.U[c * ncell + cell]; });
      dirichlet_ghost<NDIM>(Wc, A.fv + p, plane, A.gamma - 1.0);
    } else if (A.bc == TENOAA_BC_INFLOW) {
      inflow_ghost<NDIM>(Wc, A.fv + p, plane, A.gamma - 1.0);
    } else {  // halo, first layer: the neighbour's cell next to the face
      unroll<NV>([&](auto c) { Wc[c] = A.fv[c * plane + p]; });
    }
    cell_speeds<NDIM>(Wc, A.gamma, amax, bad);
  }
  if (bad) atomicOr(status, 1);
  __shared__ double red[NDIM][256];
  unroll<NDIM>([&](auto d) { red[d][threadIdx.x] = amax[d]; });
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      unroll<NDIM>([&](auto d) { red[d][threadIdx.x] = dmax(red[d][threadIdx.x], red[d][threadIdx.x + s]); });
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    unroll<NDIM>([&](auto d) { atomicMax(&S->amax_bits[d], (unsigned long long)__double_as_longlong(red[d][0])); });
  }
}

// dt and the limiter factors from the wave speeds; dt is taken from dt_fixed
// or *dt_dev when positive, else from the CFL condition, and stored back.
__global__ void finalize_dt_kernel(Scalars* S, int ndim, double dx0, double dx1, double dx2, double cfl,
                                   double* dt_dev, double dt_fixed) {
  if (threadIdx.x != 0) return;
  const double dx[3] = {dx0, dx1, dx2};
  double given = dt_fixed;
  if (!(given > 0.0) && dt_dev) given = *dt_dev;
  double dt;
  dt_and_mu(S->amax_bits, ndim, dx, cfl, given, dt, S->mu);
  if (dt_dev) *dt_dev = dt;
  S->dt = dt;
}

// The wave speeds of the scalars as doubles, and back (their bit patterns
// order like the values: the speeds are non-negative).
__global__ void speeds_out_kernel(const Scalars* S, int ndim, double* amax) {
  if (threadIdx.x < (unsigned)ndim) amax[threadIdx.x] = __longlong_as_double((long long)S->amax_bits[threadIdx.x]);
}

// A speed that is negative or not a number marks the status word.
__global__ void speeds_in_kernel(Scalars* S, int ndim, const double* amax) {
  if (threadIdx.x >= 3) return;
  const double a = threadIdx.x < (unsigned)ndim ? amax[threadIdx.x] : 0.0;
  if (!(a >= 0.0)) atomicOr(&S->status, 1);
  S->amax_bits[threadIdx.x] = (unsigned long long)__double_as_longlong(a >= 0.0 ? a : 0.0);
}

}  // namespace

// ------------------------------------------------------------ host launchers
template <int ORDER, int NDIM, int DIR, bool LIMIT, int SPLIT>
static hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t st) {
  constexpr int TT = (NDIM == 1) ? 1 : (DIR == 0 ? TENOAA_TT_X : TENOAA_TT_YZ);
  constexpr int TN = (DIR == 0) ? TENOAA_TN_X : TENOAA_TN_YZ;
  constexpr int AX_A = (DIR == 0) ? 1 : 0;
  constexpr int AX_B = (DIR == 2) ? 1 : 2;
  // Whole tiles here; a small remainder of faces (a non-periodic direction
  // has n + 1) goes to one-wave tail tiles, since a block of full-tile LDS
  // with one busy wave would hold a CU slot as long as a full tile.  Larger
  // remainders take one more full-size tile, which stages fewer cells per face.
  const int64_t rem = a.nf % TN;
  const int64_t whole = (NDIM == 1 || rem == 0 || rem > SWEEP_TAIL_TN) ? a.nf : a.nf - rem;
  if (whole > 0) {
    dim3 grid((unsigned)((whole + TN - 1) / TN), (unsigned)((a.n[AX_A] + TT - 1) / TT), (unsigned)a.n[AX_B]);
    hipLaunchKernelGGL((sweep_kernel<ORDER, NDIM, DIR, TT, TN, LIMIT, SPLIT>), grid, dim3(TT * TN), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || whole == a.nf) return e;
  }
  SweepArgs t = a;
  t.f_begin = whole;
  return launch_sweep_tail(ORDER, NDIM, DIR, t, LIMIT, st);
}

template <int ORDER, int NDIM, int DIR, int SPLIT>
static hipError_t launch_sweep_s(const SweepArgs& a, bool limit, hipStream_t st) {
  return limit ? launch_sweep_t<ORDER, NDIM, DIR, true, SPLIT>(a, st) : launch_sweep_t<ORDER, NDIM, DIR, false, SPLIT>(a, st);
}

template <int ORDER, int NDIM, int DIR>
static hipError_t launch_sweep_o(const SweepArgs& a, bool limit, hipStream_t st) {
  if (a.splitting == TENOAA_ROE) return launch_sweep_s<ORDER, NDIM, DIR, TENOAA_ROE>(a, limit, st);
  if (a.splitting == TENOAA_RUSANOV) return launch_sweep_s<ORDER, NDIM, DIR, TENOAA_RUSANOV>(a, limit, st);
  return launch_sweep_s<ORDER, NDIM, DIR, TENOAA_LLF>(a, limit, st);
}

template <int ORDER>
static hipError_t launch_sweep_ord(int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st) {
  if (ndim == 1) return launch_sweep_o<ORDER, 1, 0>(a, limit, st);
  if (ndim == 2) {
    return dir == 0 ? launch_sweep_o<ORDER, 2, 0>(a, limit, st) : launch_sweep_o<ORDER, 2, 1>(a, limit, st);
  }
  if (dir == 0) return launch_sweep_o<ORDER, 3, 0>(a, limit, st);
  if (dir == 1) return launch_sweep_o<ORDER, 3, 1>(a, limit, st);
  return launch_sweep_o<ORDER, 3, 2>(a, limit, st);
}

hipError_t launch_sweep(int order, int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st) {
  if (order == 12) return launch_sweep_ord<12>(ndim, dir, a, limit, st);
  return order == 10 ? launch_sweep_ord<10>(ndim, dir, a, limit, st) : launch_sweep_ord<8>(ndim, dir, a, limit, st);
}

// Multiplier and shift of fastdiv for the divisor d (1 <= d < 2^32).
static void fastdiv_make(uint64_t d, uint32_t& m, uint32_t& l) {
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  l = s;
  m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
}

template <int NDIM>
static hipError_t launch_update_n(int mode, const UpdateArgs& a0, hipStream_t st) {
  UpdateArgs a = a0;
  const int64_t ncell = a.n[0] * a.n[1] * a.n[2];
  for (int k = 0; k < 2; ++k) {
    const uint64_t d = (uint64_t)a.n[k];
    if (d >= 1 && d < (1ull << 32)) fastdiv_make(d, a.div_m[k], a.div_l[k]);
  }
  int64_t blocks = (ncell + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  dim3 g((unsigned)blocks);
  switch (mode) {
    case 0: hipLaunchKernelGGL((update_kernel<NDIM, 0>), g, dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL((update_kernel<NDIM, 1>), g, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((update_kernel<NDIM, 2>), g, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((update_kernel<NDIM, 3>), g, dim3(256), 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_update(int ndim, int mode, const UpdateArgs& a, hipStream_t st) {
  if (ndim == 1) return launch_update_n<1>(mode, a, st);
  if (ndim == 2) return launch_update_n<2>(mode, a, st);
  return launch_update_n<3>(mode, a, st);
}

hipError_t launch_wave_speeds(int ndim, const double* U, int64_t ncell, double gam, Scalars* S, int* status,
                              hipStream_t st) {
  hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, st, S);
  int64_t blocks = (ncell + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (ndim == 1) hipLaunchKernelGGL(wave_speed_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, U, ncell, gam, S, status);
  if (ndim == 2) hipLaunchKernelGGL(wave_speed_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, st, U, ncell, gam, S, status);
  if (ndim == 3) hipLaunchKernelGGL(wave_speed_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, st, U, ncell, gam, S, status);
  return hipGetLastError();
}

hipError_t launch_ghost_speeds(int ndim, const GhostSpeedArgs& a, Scalars* S, int* status, hipStream_t st) {
  const int a0 = (a.dir == 0) ? 1 : 0, a1 = (a.dir == 2) ? 1 : 2;
  const int64_t plane = a.n[a0] * a.n[a1];
  int64_t blocks = (plane + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (ndim == 1) hipLaunchKernelGGL(ghost_speed_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, a, S, status);
  if (ndim == 2) hipLaunchKernelGGL(ghost_speed_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, st, a, S, status);
  if (ndim == 3) hipLaunchKernelGGL(ghost_speed_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, st, a, S, status);
  return hipGetLastError();
}

hipError_t launch_speeds_out(const Scalars* S, int ndim, double* amax, hipStream_t st) {
  hipLaunchKernelGGL(speeds_out_kernel, dim3(1), dim3(64), 0, st, S, ndim, amax);
  return hipGetLastError();
}

hipError_t launch_speeds_in(Scalars* S, int ndim, const double* amax, hipStream_t st) {
  hipLaunchKernelGGL(speeds_in_kernel, dim3(1), dim3(64), 0, st, S, ndim, amax);
  return hipGetLastError();
}

hipError_t launch_finalize_dt(Scalars* S, int ndim, const double* dx, double cfl, double* dt_dev, double dt_fixed,
                              hipStream_t st) {
  hipLaunchKernelGGL(finalize_dt_kernel, dim3(1), dim3(64), 0, st, S, ndim, dx[0], dx[1], dx[2], cfl, dt_dev,
                     dt_fixed);
  return hipGetLastError();
}

}  // namespace tenoaa
