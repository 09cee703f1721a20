// Batched persistent form: many independent 2D Euler problems of uneven size
// advanced together by SSP-RK3 steps, each with its own dt, in one launch.
//
// The launch is a resident grid (compute units x blocks per unit) that walks
// the phases of the whole batch in order:
//
//   phase 0                 wave speeds of every problem's initial state
//   per step n, stage s:    SWEEP (x and y face tiles of every problem)
//                           UPDATE (flux difference and stage s of every cell;
//                                   at s = 3 also the next step's wave speeds)
//
// Within a phase the items (tiles or 2048-cell blocks of any problem) are
// handed out by an atomic counter, largest problems first; phases are
// separated by a grid barrier (release fence, arrival count, acquire fence).
// Every item is evaluated by the same device bodies as the per-grid kernels
// (sweep_tile, update_cell, cell_speeds, dt_and_mu), so the batched results
// equal per-problem tenoaa_step calls bit for bit, whatever tiles are chosen.
//
// A barrier wait gives up after a wall-clock limit (the grid is sized to be
// resident, so this only guards against a launch that is not): the launch then
// raises an abort word that every block checks, and every block exits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tenoaa.h"
#include "tenoaa_device.h"
#include "tenoaa_internal.h"
#include "tenoaa_stencil.h"

namespace tenoaa {
namespace {

#ifndef TENOAA_BATCH_WAVES_PER_EU
#define TENOAA_BATCH_WAVES_PER_EU 3
#endif

constexpr int BT = 256;         // threads per block
#ifndef TENOAA_BATCH_CELLS_ITEM
#define TENOAA_BATCH_CELLS_ITEM 2048
#endif
constexpr int CELLS_ITEM = TENOAA_BATCH_CELLS_ITEM;  // cells per update / wave-speed item
constexpr int NBUCKET = 3;        // size buckets of the tile choice (by n_x)

// Tile candidates (TT pencils x TN faces, 256 threads).
// x sweep: 0 -> 4 x 64, 1 -> 8 x 32.   y sweep: 0 -> 16 x 16, 1 -> 32 x 8.
template <int DIR, int C>
struct Cand;
template <> struct Cand<0, 0> { static constexpr int TT = 4, TN = 64; };
template <> struct Cand<0, 1> { static constexpr int TT = 8, TN = 32; };
template <> struct Cand<1, 0> { static constexpr int TT = 16, TN = 16; };
template <> struct Cand<1, 1> { static constexpr int TT = 32, TN = 8; };

template <int ORDER, int DIR, int C>
constexpr int cand_lds() {
  return SweepShape<ORDER, 2, Cand<DIR, C>::TT, Cand<DIR, C>::TN>::LDS_BYTES;
}
template <int ORDER>
constexpr int arena_bytes() {
  int m = 2 * BT * 8;  // block reduction of two maxima
  m = std::max(m, cand_lds<ORDER, 0, 0>());
  m = std::max(m, cand_lds<ORDER, 0, 1>());
  m = std::max(m, cand_lds<ORDER, 1, 0>());
  m = std::max(m, cand_lds<ORDER, 1, 1>());
  return m;
}

struct BatchProblem {
  int64_t n[2];       // cells along x, y
  int64_t nf[2];      // faces along x, y
  int64_t nft[2];     // faces of each direction in total
  double dx[3];
  double rdx[3];      // 1 / dx, correctly rounded (host)
  int32_t bc_lo[2], bc_hi[2];
  const double* bcv[2][2];  // Dirichlet/inflow values of side [d][low/high] (one set), else null
  int64_t u_off;      // state offset in the packed buffer (doubles)
  int64_t s_off;      // stage state offset
  int64_t f_off[2];   // face flux arrays
  int64_t along[2];   // tiles along each sweep direction
  int64_t across[2];  // tiles across it
  int32_t tile[2];    // candidate per direction
  int32_t orig;       // index of the problem in the caller's order
  int32_t pad;
};

struct BatchArgs {
  const BatchProblem* probs;  // processing order
  const int64_t* pre_sweep;   // prefix sums of sweep items, nprob + 1
  const int64_t* pre_cell;    // prefix sums of cell items, nprob + 1
  double* U;                  // packed states (caller)
  double* S;                  // stage states
  double* F;                  // face fluxes
  unsigned long long* amax;   // [nprob][nsteps][2] wave-speed bit patterns
  double* dt_out;             // [orig][nsteps] or null
  int* status;                // [nprob] non-physical-state words
  unsigned long long* ctl;    // [0] barrier arrivals, [1] abort, [2 + phase] item counters
  unsigned long long* bstat;  // per block b, ticks: [4 b] waited at phase barriers, [4 b + 1] resident,
                              // [4 b + 2] in sweep items, [4 b + 3] in update and wave-speed items
  double gamma, cfl;
  int64_t timeout_ticks;
  int32_t nprob, nsteps, splitting, chunk;
};

struct InitArgs {
  unsigned long long* ctl;
  int64_t nctl;
  unsigned long long* amax;
  int64_t namax;
  int* status;
  int64_t nstatus;
};

__global__ __launch_bounds__(256) void batch_init_kernel(InitArgs I) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < I.nctl; i += step) I.ctl[i] = 0ull;
  for (int64_t i = i0; i < I.namax; i += step) I.amax[i] = 0ull;
  for (int64_t i = i0; i < I.nstatus; i += step) I.status[i] = 0;
}

__device__ __forceinline__ int find_problem(const int64_t* pre, int nprob, int64_t it) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= it) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Block-wide maximum of two per-thread values, folded into dst[0..1] with
// bit-pattern atomics (non-negative doubles order like their bits).
__device__ __forceinline__ void block_max2(char* arena, double a0, double a1, unsigned long long* dst) {
  double* red = reinterpret_cast<double*>(arena);
  red[threadIdx.x] = a0;
  red[BT + threadIdx.x] = a1;
  __syncthreads();
  for (int s = BT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] = dmax(red[threadIdx.x], red[threadIdx.x + s]);
      red[BT + threadIdx.x] = dmax(red[BT + threadIdx.x], red[BT + threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(&dst[0], (unsigned long long)__double_as_longlong(red[0]));
    atomicMax(&dst[1], (unsigned long long)__double_as_longlong(red[BT]));
  }
}

template <int ORDER, int DIR, bool LIMIT, bool ROE>
__device__ __forceinline__ void run_sweep_tile(const SweepArgs& A, char* arena, int cand, int64_t k,
                                               int64_t along, double mu) {
  const int64_t bx = k % along, by = k / along;
  if (cand == 0) {
    sweep_tile<ORDER, 2, DIR, Cand<DIR, 0>::TT, Cand<DIR, 0>::TN, LIMIT, ROE ? TENOAA_ROE : SPLIT_RUNTIME>(
        A, arena, bx, by, 0, mu);
  } else {
    sweep_tile<ORDER, 2, DIR, Cand<DIR, 1>::TT, Cand<DIR, 1>::TN, LIMIT, ROE ? TENOAA_ROE : SPLIT_RUNTIME>(
        A, arena, bx, by, 0, mu);
  }
}

template <int ORDER, bool LIMIT, bool ROE, bool BV>
__device__ __forceinline__ void sweep_item(const BatchArgs& B, char* arena, int p, int64_t k, int n, int stage) {
  const BatchProblem& P = B.probs[p];
  const double* in = (stage == 1 ? B.U + P.u_off : B.S + P.s_off);
  double mu[3] = {0.0, 0.0, 0.0};
  if (LIMIT) {
    double dt;
    dt_and_mu(B.amax + ((int64_t)p * B.nsteps + n) * 2, 2, P.dx, B.cfl, 0.0, dt, mu);
  }
  SweepArgs A{};  // every pointer the batch does not use stays null
  A.U = in;
  A.flags = nullptr;
  A.frozen = nullptr;
  A.fh_out = nullptr;
  A.n[0] = P.n[0];
  A.n[1] = P.n[1];
  A.n[2] = 1;
  A.splitting = B.splitting;
  A.gamma = B.gamma;
  A.mu = nullptr;
  A.status = B.status + p;
  const int64_t ntx = P.along[0] * P.across[0];
  const int dir = k < ntx ? 0 : 1;
  if (dir == 1) k -= ntx;
  A.F = B.F + P.f_off[dir];
  A.nf = P.nf[dir];
  A.nft = P.nft[dir];
  A.bc_lo = P.bc_lo[dir];
  A.bc_hi = P.bc_hi[dir];
  // (without prescribed sides the pointers stay null constants, and their
  // ghost rules drop out of the staging)
  if constexpr (BV) {
    A.bcv[0] = P.bcv[dir][0];
    A.bcv[1] = P.bcv[dir][1];
  }
  if (dir == 0) run_sweep_tile<ORDER, 0, LIMIT, ROE>(A, arena, P.tile[0], k, P.along[0], mu[0]);
  else run_sweep_tile<ORDER, 1, LIMIT, ROE>(A, arena, P.tile[1], k, P.along[1], mu[1]);
}

// The ghost cells next to the faces of a problem's sides with prescribed
// values count in its CFL speeds (as in the single-grid step): for a cell W
// at coordinates co on such a side, the ghost it makes (Dirichlet: W
// reflected through the face values; inflow: the first prescribed layer).
__device__ __forceinline__ void boundary_speeds(const BatchProblem& P, const int64_t (&co)[3], const double (&W)[4],
                                                double gam, double (&amax)[2], bool& bad) {
  unroll<2>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    unroll<2>([&](auto hh) {
      constexpr int h = decltype(hh)::value;
      const double* fv = P.bcv[d][h];
      if (fv && co[d] == (h ? P.n[d] - 1 : 0)) {
        const int64_t plane = P.n[1 - d];
        double Wg[4] = {W[0], W[1], W[2], W[3]};
        if ((h ? P.bc_hi[d] : P.bc_lo[d]) == TENOAA_BC_DIRICHLET) dirichlet_ghost<2>(Wg, fv + co[1 - d], plane, gam - 1.0);
        else inflow_ghost<2>(Wg, fv + co[1 - d], plane, gam - 1.0);
        cell_speeds<2>(Wg, gam, amax, bad);
      }
    });
  });
}

template <int MODE, bool BV>
__device__ __forceinline__ void update_item(const BatchArgs& B, char* arena, int p, int64_t k, int n) {
  const BatchProblem& P = B.probs[p];
  double dt, mu[3];
  dt_and_mu(B.amax + ((int64_t)p * B.nsteps + n) * 2, 2, P.dx, B.cfl, 0.0, dt, mu);
  if (MODE == 1 && k == 0 && threadIdx.x == 0 && B.dt_out) B.dt_out[(int64_t)P.orig * B.nsteps + n] = dt;
  UpdateArgs A{};
  A.F[0] = B.F + P.f_off[0];
  A.F[1] = B.F + P.f_off[1];
  A.F[2] = nullptr;
  for (int d = 0; d < 2; ++d) {
    A.nft[d] = P.nft[d];
    A.nf[d] = P.nf[d];
    A.n[d] = P.n[d];
  }
  A.nft[2] = 0;
  A.nf[2] = 1;
  A.n[2] = 1;
  for (int d = 0; d < 3; ++d) {
    A.dx[d] = P.dx[d];
    A.rdx[d] = P.rdx[d];
  }
  A.Un = B.U + P.u_off;
  A.Us = B.S + P.s_off;
  A.out = (MODE == 3) ? B.U + P.u_off : B.S + P.s_off;
  A.dt = nullptr;
  const int64_t ncell = P.n[0] * P.n[1];
  const bool speeds = (MODE == 3) && (n + 1 < B.nsteps);
  const bool bvals = P.bcv[0][0] || P.bcv[0][1] || P.bcv[1][0] || P.bcv[1][1];
  double amax[2] = {0.0, 0.0};
  bool bad = false;
  for (int r = 0; r < CELLS_ITEM / BT; ++r) {
    const int64_t idx = k * CELLS_ITEM + r * BT + threadIdx.x;
    if (idx < ncell) {
      // a problem has fewer than 2^31 cells (checked when the plan is made)
      const uint32_t q = (uint32_t)idx / (uint32_t)P.n[0];
      const int64_t co[3] = {(int64_t)((uint32_t)idx - q * (uint32_t)P.n[0]), (int64_t)q, 0};
      double Wn[4];
      update_cell<2, MODE>(A, idx, co, dt, Wn);
      if (speeds) {
        cell_speeds<2>(Wn, B.gamma, amax, bad);
        if constexpr (BV) boundary_speeds(P, co, Wn, B.gamma, amax, bad);
      }
    }
  }
  if (speeds) {
    if (bad) atomicOr(B.status + p, 1);
    block_max2(arena, amax[0], amax[1], B.amax + ((int64_t)p * B.nsteps + n + 1) * 2);
  }
}

template <bool BV>
__device__ __forceinline__ void speeds_item(const BatchArgs& B, char* arena, int p, int64_t k) {
  const BatchProblem& P = B.probs[p];
  const int64_t ncell = P.n[0] * P.n[1];
  const double* U = B.U + P.u_off;
  double amax[2] = {0.0, 0.0};
  bool bad = false;
  for (int r = 0; r < CELLS_ITEM / BT; ++r) {
    const int64_t idx = k * CELLS_ITEM + r * BT + threadIdx.x;
    if (idx < ncell) {
      double Wc[4];
      unroll<4>([&](auto c) { Wc[c] = U[c * ncell + idx]; });
      cell_speeds<2>(Wc, B.gamma, amax, bad);
      if constexpr (BV) {
        const uint32_t q = (uint32_t)idx / (uint32_t)P.n[0];
        const int64_t co[3] = {(int64_t)((uint32_t)idx - q * (uint32_t)P.n[0]), (int64_t)q, 0};
        boundary_speeds(P, co, Wc, B.gamma, amax, bad);
      }
    }
  }
  if (bad) atomicOr(B.status + p, 1);
  block_max2(arena, amax[0], amax[1], B.amax + (int64_t)p * B.nsteps * 2);
}

// All blocks arrive; returns false if the launch is being abandoned.  The
// ticks thread 0 spends between its arrival and the release are added to the
// block's wait counter.
__device__ __forceinline__ bool grid_barrier(const BatchArgs& B, unsigned long long target, int* s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(&B.ctl[0], 1ull);
    const uint64_t t0 = wall_clock64();
    int ok = 1;
    while (true) {
      if (__hip_atomic_load(&B.ctl[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(&B.ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull) {
        ok = 0;
        break;
      }
      if ((int64_t)(wall_clock64() - t0) > B.timeout_ticks) {
        atomicMax(&B.ctl[1], 1ull);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    B.bstat[4 * blockIdx.x] += wall_clock64() - t0;
    __threadfence();
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

template <int ORDER, bool LIMIT, bool ROE, bool BV>
__global__ __launch_bounds__(BT)
#if TENOAA_BATCH_WAVES_PER_EU > 0
__attribute__((amdgpu_waves_per_eu(TENOAA_BATCH_WAVES_PER_EU)))
#endif
void batch_kernel(BatchArgs B) {
  __shared__ __align__(16) char arena[arena_bytes<ORDER>()];
  __shared__ int64_t s_first;
  __shared__ int s_flag;
  const uint64_t t_start = wall_clock64();
  uint64_t t_sweep = 0, t_cell = 0;  // thread 0's ticks in the items of each kind
  const int nphase = 1 + 6 * B.nsteps;
  for (int ph = 0; ph < nphase; ++ph) {
    int kind = 0, n = 0, stage = 0;
    if (ph > 0) {
      const int q = ph - 1;
      n = q / 6;
      stage = (q % 6) / 2 + 1;
      kind = (q % 2 == 0) ? 1 : 2;
    }
    const int64_t* pre = (kind == 1) ? B.pre_sweep : B.pre_cell;
    const int64_t total = pre[B.nprob];
    while (true) {
      __syncthreads();  // the previous item is done with the arena and s_first
      if (threadIdx.x == 0) {
        s_first = (int64_t)atomicAdd(&B.ctl[2 + ph], (unsigned long long)B.chunk);
        s_flag = __hip_atomic_load(&B.ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull;
      }
      __syncthreads();
      if (s_flag) return;
      const int64_t first = s_first;
      if (first >= total) break;
      const int64_t last = (first + B.chunk < total) ? first + B.chunk : total;
      const uint64_t t_items = wall_clock64();
      int p = -1;
      for (int64_t it = first; it < last; ++it) {
        if (it > first) __syncthreads();
        // the items of a chunk mostly belong to one problem: search only on leaving it
        if (p < 0 || it >= pre[p + 1]) p = find_problem(pre, B.nprob, it);
        const int64_t k = it - pre[p];
        if (kind == 0) {
          speeds_item<BV>(B, arena, p, k);
        } else if (kind == 1) {
          sweep_item<ORDER, LIMIT, ROE, BV>(B, arena, p, k, n, stage);
        } else if (stage == 1) {
          update_item<1, BV>(B, arena, p, k, n);
        } else if (stage == 2) {
          update_item<2, BV>(B, arena, p, k, n);
        } else {
          update_item<3, BV>(B, arena, p, k, n);
        }
      }
      if (threadIdx.x == 0) (kind == 1 ? t_sweep : t_cell) += wall_clock64() - t_items;
    }
    if (ph + 1 < nphase && !grid_barrier(B, (unsigned long long)(ph + 1) * gridDim.x, &s_flag)) return;
  }
  if (threadIdx.x == 0) {
    B.bstat[4 * blockIdx.x + 1] = wall_clock64() - t_start;
    B.bstat[4 * blockIdx.x + 2] = t_sweep;
    B.bstat[4 * blockIdx.x + 3] = t_cell;
  }
}

// Uniform state for tuning runs: rho = 1, u = 0.3, v = 0.2, p = 1.
__global__ __launch_bounds__(256) void batch_fill_kernel(double* U, const int64_t* offs, const int64_t* cells,
                                                         int nprob, double gamma) {
  const double E = 1.0 / (gamma - 1.0) + 0.5 * (0.3 * 0.3 + 0.2 * 0.2);
  for (int p = blockIdx.y; p < nprob; p += gridDim.y) {
    const int64_t nc = cells[p];
    double* u = U + offs[p];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (int64_t)gridDim.x * blockDim.x) {
      u[i] = 1.0;
      u[nc + i] = 0.3;
      u[2 * nc + i] = 0.2;
      u[3 * nc + i] = E;
    }
  }
}

using KernelFn = void (*)(BatchArgs);

// The variant with prescribed sides (BV) only without the Roe flux.
KernelFn pick_kernel(int order, bool limit, bool roe, bool bv) {
  if (bv) {
    if (order == 8) return limit ? batch_kernel<8, true, false, true> : batch_kernel<8, false, false, true>;
    if (order == 12) return limit ? batch_kernel<12, true, false, true> : batch_kernel<12, false, false, true>;
    return limit ? batch_kernel<10, true, false, true> : batch_kernel<10, false, false, true>;
  }
  if (roe) {
    if (order == 8) return limit ? batch_kernel<8, true, true, false> : batch_kernel<8, false, true, false>;
    if (order == 12) return limit ? batch_kernel<12, true, true, false> : batch_kernel<12, false, true, false>;
    return limit ? batch_kernel<10, true, true, false> : batch_kernel<10, false, true, false>;
  }
  if (order == 8) return limit ? batch_kernel<8, true, false, false> : batch_kernel<8, false, false, false>;
  if (order == 12) return limit ? batch_kernel<12, true, false, false> : batch_kernel<12, false, false, false>;
  return limit ? batch_kernel<10, true, false, false> : batch_kernel<10, false, false, false>;
}

int64_t faces_along2(const tenoaa_grid& g, int d) {
  return g.bc_lo[d] == TENOAA_BC_PERIODIC ? g.n[d] : g.n[d] + 1;
}

int bucket_of(int64_t nx) { return nx <= 160 ? 0 : (nx <= 320 ? 1 : 2); }

int cand_tt(int dir, int c) { return dir == 0 ? (c == 0 ? 4 : 8) : (c == 0 ? 16 : 32); }
int cand_tn(int dir, int c) { return dir == 0 ? (c == 0 ? 64 : 32) : (c == 0 ? 16 : 8); }

}  // namespace
}  // namespace tenoaa

using namespace tenoaa;

struct tenoaa_batch_plan {
  int nprob = 0, nsteps = 0;
  tenoaa_scheme scheme{};
  double gamma = 1.4, cfl = 0.4;
  std::vector<tenoaa_grid> grids;
  std::vector<int64_t> offsets;  // caller order, nprob + 1
  std::vector<int> order;        // processing order -> caller index
  int tile_x[NBUCKET] = {0, 0, 0}, tile_y[NBUCKET] = {0, 0, 0};
  int chunk = 1, bpc = 1, max_bpc = 1, ncu = 0, tuned = 0;
  KernelFn kernel = nullptr;
  // device memory owned by the plan
  BatchProblem* d_table = nullptr;
  int64_t* d_pre = nullptr;  // pre_sweep (nprob + 1) then pre_cell (nprob + 1)
  double* d_S = nullptr;
  double* d_F = nullptr;
  unsigned long long* d_amax = nullptr;
  int* d_status = nullptr;
  unsigned long long* d_ctl = nullptr;
  int64_t nctl = 0;        // queue words (nctl_queue) then two per block slot (ncu * max_bpc)
  int64_t nctl_queue = 0;
  int rate_khz = 0;        // wall_clock64 ticks per millisecond
  BatchArgs args{};
  InitArgs iargs{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t n_init = nullptr, n_main = nullptr;
  bool bound = false;
  std::string cache_key;
};

namespace {

int fail_hip(hipError_t e) {
  tenoaa::record_hip_error(e);
  return TENOAA_EHIP;
}

// Rebuilds the problem table (tile choices) and uploads it with the prefix sums.
hipError_t upload_table(tenoaa_batch_plan* P) {
  std::vector<BatchProblem> tab(P->nprob);
  std::vector<int64_t> pre(2 * (P->nprob + 1), 0);
  int64_t s_off = 0, f_off = 0;
  for (int i = 0; i < P->nprob; ++i) {
    const int q = P->order[i];
    const tenoaa_grid& g = P->grids[q];
    BatchProblem& b = tab[i];
    std::memset(&b, 0, sizeof(b));
    const int bk = bucket_of(g.n[0]);
    b.tile[0] = P->tile_x[bk];
    b.tile[1] = P->tile_y[bk];
    for (int d = 0; d < 2; ++d) {
      b.n[d] = g.n[d];
      b.nf[d] = faces_along2(g, d);
      b.nft[d] = b.nf[d] * g.n[1 - d];
      b.bc_lo[d] = g.bc_lo[d];
      b.bc_hi[d] = g.bc_hi[d];
      for (int h = 0; h < 2; ++h) {
        const int bc = h ? g.bc_hi[d] : g.bc_lo[d];
        b.bcv[d][h] = (bc == TENOAA_BC_DIRICHLET || bc == TENOAA_BC_INFLOW) ? g.bc_values[d][h] : nullptr;
      }
      const int tt = cand_tt(d, b.tile[d]), tn = cand_tn(d, b.tile[d]);
      b.along[d] = (b.nf[d] + tn - 1) / tn;
      b.across[d] = (g.n[1 - d] + tt - 1) / tt;
    }
    for (int d = 0; d < 3; ++d) {
      b.dx[d] = g.dx[d];
      b.rdx[d] = 1.0 / g.dx[d];
    }
    b.u_off = P->offsets[q];
    b.s_off = s_off;
    s_off += 4 * g.n[0] * g.n[1];
    b.f_off[0] = f_off;
    f_off += 4 * b.nft[0];
    b.f_off[1] = f_off;
    f_off += 4 * b.nft[1];
    b.orig = q;
    const int64_t cells = g.n[0] * g.n[1];
    pre[i + 1] = pre[i] + b.along[0] * b.across[0] + b.along[1] * b.across[1];
    pre[P->nprob + 1 + i + 1] = pre[P->nprob + 1 + i] + (cells + CELLS_ITEM - 1) / CELLS_ITEM;
  }
  hipError_t e = hipMemcpy(P->d_table, tab.data(), sizeof(BatchProblem) * tab.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(P->d_pre, pre.data(), sizeof(int64_t) * pre.size(), hipMemcpyHostToDevice);
  return e;
}

void fill_args(tenoaa_batch_plan* P, double* U, double* dt_out, int nsteps) {
  BatchArgs& a = P->args;
  a.probs = P->d_table;
  a.pre_sweep = P->d_pre;
  a.pre_cell = P->d_pre + P->nprob + 1;
  a.U = U;
  a.S = P->d_S;
  a.F = P->d_F;
  a.amax = P->d_amax;
  a.dt_out = dt_out;
  a.status = P->d_status;
  a.ctl = P->d_ctl;
  a.bstat = P->d_ctl + P->nctl_queue;
  a.gamma = P->gamma;
  a.cfl = P->cfl;
  a.nprob = P->nprob;
  a.nsteps = nsteps;
  a.splitting = P->scheme.splitting;
  a.chunk = P->chunk;
}

// One direct launch (tuning); the state is the caller's or the tuning buffer.
hipError_t launch_direct(tenoaa_batch_plan* P, double* U, int nsteps, hipStream_t st) {
  fill_args(P, U, nullptr, nsteps);
  InitArgs ia = P->iargs;
  hipLaunchKernelGGL(batch_init_kernel, dim3(256), dim3(256), 0, st, ia);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(P->kernel, dim3(P->ncu * P->bpc), dim3(BT), 0, st, P->args);
  return hipGetLastError();
}

hipError_t time_config(tenoaa_batch_plan* P, double* U, hipStream_t st, float* best_ms) {
  hipError_t e = upload_table(P);
  if (e != hipSuccess) return e;
  hipEvent_t a, b;
  if ((e = hipEventCreate(&a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) return e;
  float best = 1e30f;
  for (int r = 0; r < 4 && e == hipSuccess; ++r) {
    e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch_direct(P, U, 1, st);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (r > 0 && ms < best) best = ms;  // the first run warms up
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *best_ms = best;
  return e;
}

std::string make_key(const tenoaa_batch_plan* P) {
  int cnt[NBUCKET] = {0, 0, 0};
  for (const tenoaa_grid& g : P->grids) cnt[bucket_of(g.n[0])]++;
  char buf[160];
  std::snprintf(buf, sizeof(buf), "gfx950 order=%d split=%d limit=%d buckets=%d,%d,%d", P->scheme.order,
                P->scheme.splitting, P->scheme.positivity, cnt[0], cnt[1], cnt[2]);
  return buf;
}

bool parse_ints(const std::string& line, const char* field, int* out, int n) {
  const std::string pat = std::string("\"") + field + "\":";
  size_t pos = line.find(pat);
  if (pos == std::string::npos) return false;
  pos += pat.size();
  for (int i = 0; i < n; ++i) {
    while (pos < line.size() && !(line[pos] == '-' || (line[pos] >= '0' && line[pos] <= '9'))) ++pos;
    if (pos >= line.size()) return false;
    out[i] = std::atoi(line.c_str() + pos);
    while (pos < line.size() && (line[pos] == '-' || (line[pos] >= '0' && line[pos] <= '9'))) ++pos;
  }
  return true;
}

// Looks the key up in a JSON-lines cache; the last matching line wins.
bool read_cache(tenoaa_batch_plan* P, const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char buf[1024];
  const std::string want = "\"key\": \"" + P->cache_key + "\"";
  while (std::fgets(buf, sizeof(buf), f)) {
    const std::string line(buf);
    if (line.find(want) == std::string::npos) continue;
    int tx[NBUCKET], ty[NBUCKET], ch[1], bp[1];
    if (!parse_ints(line, "tile_x", tx, NBUCKET) || !parse_ints(line, "tile_y", ty, NBUCKET) ||
        !parse_ints(line, "chunk", ch, 1) || !parse_ints(line, "blocks_per_cu", bp, 1))
      continue;
    bool ok = ch[0] >= 1 && ch[0] <= 64 && bp[0] >= 1 && bp[0] <= P->max_bpc;
    for (int b = 0; b < NBUCKET; ++b) ok = ok && (tx[b] == 0 || tx[b] == 1) && (ty[b] == 0 || ty[b] == 1);
    if (!ok) continue;
    for (int b = 0; b < NBUCKET; ++b) {
      P->tile_x[b] = tx[b];
      P->tile_y[b] = ty[b];
    }
    P->chunk = ch[0];
    P->bpc = bp[0];
    found = true;
  }
  std::fclose(f);
  return found;
}

void append_cache(const tenoaa_batch_plan* P, const char* path, float ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"key\": \"%s\", \"tile_x\": [%d, %d, %d], \"tile_y\": [%d, %d, %d], \"chunk\": %d, "
               "\"blocks_per_cu\": %d, \"step_ms\": %.4f}\n",
               P->cache_key.c_str(), P->tile_x[0], P->tile_x[1], P->tile_x[2], P->tile_y[0], P->tile_y[1],
               P->tile_y[2], P->chunk, P->bpc, (double)ms);
  std::fclose(f);
}

// Coordinate search over the tile candidates per size bucket, then the item
// chunk and the blocks per compute unit, each timed on one step of the whole
// batch from a uniform state.
hipError_t tune(tenoaa_batch_plan* P, float* out_ms) {
  hipStream_t st;
  hipError_t e = hipStreamCreate(&st);
  if (e != hipSuccess) return e;
  double* U = nullptr;
  int64_t* aux = nullptr;
  e = hipMalloc(&U, sizeof(double) * P->offsets[P->nprob]);
  if (e == hipSuccess) e = hipMalloc(&aux, sizeof(int64_t) * 2 * P->nprob);
  if (e == hipSuccess) {
    std::vector<int64_t> h(2 * P->nprob);
    for (int q = 0; q < P->nprob; ++q) {
      h[q] = P->offsets[q];
      h[P->nprob + q] = P->grids[q].n[0] * P->grids[q].n[1];
    }
    e = hipMemcpy(aux, h.data(), sizeof(int64_t) * h.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    const unsigned gy = (unsigned)std::min(P->nprob, 65535);
    hipLaunchKernelGGL(batch_fill_kernel, dim3(64, gy), dim3(256), 0, st, U, aux, aux + P->nprob, P->nprob,
                       P->gamma);
    e = hipGetLastError();
  }
  float best = 0.0f;
  if (e == hipSuccess) e = time_config(P, U, st, &best);
  for (int b = 0; b < NBUCKET && e == hipSuccess; ++b) {
    for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
      int* slot = dir == 0 ? &P->tile_x[b] : &P->tile_y[b];
      const int keep = *slot;
      *slot = 1 - keep;
      float ms;
      e = time_config(P, U, st, &ms);
      if (e == hipSuccess && ms < best) best = ms;
      else *slot = keep;
    }
  }
  for (int ch : {2, 4}) {
    if (e != hipSuccess) break;
    const int keep = P->chunk;
    P->chunk = ch;
    float ms;
    e = time_config(P, U, st, &ms);
    if (e == hipSuccess && ms < best) best = ms;
    else P->chunk = keep;
  }
  for (int bp = 1; bp < P->max_bpc && e == hipSuccess; ++bp) {
    const int keep = P->bpc;
    P->bpc = bp;
    float ms;
    e = time_config(P, U, st, &ms);
    if (e == hipSuccess && ms < best) best = ms;
    else P->bpc = keep;
  }
  if (U) (void)hipFree(U);
  if (aux) (void)hipFree(aux);
  (void)hipStreamDestroy(st);
  *out_ms = best;
  return e;
}

hipError_t build_graph(tenoaa_batch_plan* P) {
  hipError_t e = hipGraphCreate(&P->graph, 0);
  if (e != hipSuccess) return e;
  void* ip[1] = {&P->iargs};
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.func = reinterpret_cast<void*>(batch_init_kernel);
  kp.gridDim = dim3(256);
  kp.blockDim = dim3(256);
  kp.sharedMemBytes = 0;
  kp.kernelParams = ip;
  kp.extra = nullptr;
  e = hipGraphAddKernelNode(&P->n_init, P->graph, nullptr, 0, &kp);
  if (e != hipSuccess) return e;
  fill_args(P, nullptr, nullptr, P->nsteps);
  void* mp[1] = {&P->args};
  std::memset(&kp, 0, sizeof(kp));
  kp.func = reinterpret_cast<void*>(P->kernel);
  kp.gridDim = dim3(P->ncu * P->bpc);
  kp.blockDim = dim3(BT);
  kp.sharedMemBytes = 0;
  kp.kernelParams = mp;
  kp.extra = nullptr;
  e = hipGraphAddKernelNode(&P->n_main, P->graph, &P->n_init, 1, &kp);
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
}

void release(tenoaa_batch_plan* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  for (void* p : {(void*)P->d_table, (void*)P->d_pre, (void*)P->d_S, (void*)P->d_F, (void*)P->d_amax,
                  (void*)P->d_status, (void*)P->d_ctl})
    if (p) (void)hipFree(p);
  delete P;
}

}  // namespace

extern "C" {

int tenoaa_batch_plan_create(const tenoaa_grid* grids, int32_t nprob, const tenoaa_scheme* scheme, double gamma,
                             double cfl, int32_t nsteps, const char* tune_cache_path, tenoaa_batch_plan** out) {
  if (!out) return TENOAA_EINVAL;
  *out = nullptr;
  if (!grids || !scheme || nprob < 1 || nprob > (1 << 20) || nsteps < 1 || nsteps > 100000) return TENOAA_EINVAL;
  if (!(gamma > 1.0) || !(cfl > 0.0) || cfl > 1.0) return TENOAA_EINVAL;
  if (scheme->positivity && cfl > 0.5) return TENOAA_EINVAL;
  int64_t total = 0;
  for (int q = 0; q < nprob; ++q) {
    if (!tenoaa::grid_ok(&grids[q], scheme)) return TENOAA_EINVAL;
    if (grids[q].ndim != 2 || tenoaa::has_halo(&grids[q])) return TENOAA_EUNSUPPORTED;
    if (tenoaa::has_boundary_values(&grids[q]) && (grids[q].bc_sets != 1 || scheme->splitting == TENOAA_ROE))
      return TENOAA_EUNSUPPORTED;
    if (grids[q].n[0] * grids[q].n[1] >= ((int64_t)1 << 31)) return TENOAA_EINVAL;
    total += 4 * grids[q].n[0] * grids[q].n[1];
    if (total > ((int64_t)1 << 40)) return TENOAA_EINVAL;
  }
  tenoaa_batch_plan* P = new tenoaa_batch_plan();
  P->nprob = nprob;
  P->nsteps = nsteps;
  P->scheme = *scheme;
  P->gamma = gamma;
  P->cfl = cfl;
  P->grids.assign(grids, grids + nprob);
  P->offsets.resize(nprob + 1);
  P->offsets[0] = 0;
  for (int q = 0; q < nprob; ++q) P->offsets[q + 1] = P->offsets[q] + 4 * grids[q].n[0] * grids[q].n[1];
  P->order.resize(nprob);
  for (int q = 0; q < nprob; ++q) P->order[q] = q;
  std::stable_sort(P->order.begin(), P->order.end(), [&](int a, int b) {
    return grids[a].n[0] * grids[a].n[1] > grids[b].n[0] * grids[b].n[1];
  });
  bool bv = false;
  for (const tenoaa_grid& g : P->grids) bv = bv || tenoaa::has_boundary_values(&g);
  P->kernel = pick_kernel(scheme->order, scheme->positivity != 0, scheme->splitting == TENOAA_ROE, bv);
  P->cache_key = make_key(P);

  int dev = 0, rate_khz = 0, nblk = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&P->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, P->kernel, BT, 0);
  if (e != hipSuccess) {
    release(P);
    return fail_hip(e);
  }
  if (nblk < 1 || P->ncu < 1) {
    release(P);
    return TENOAA_EUNSUPPORTED;
  }
  P->max_bpc = nblk;
  P->bpc = nblk;
  // a barrier wait longer than 20 s means the grid is not resident; the
  // environment can shorten the limit to exercise the abandon path
  double limit_us = 20.0e6;
  if (const char* env = std::getenv("TENOAA_BATCH_BARRIER_TIMEOUT_US")) limit_us = std::atof(env);
  if (!(limit_us >= 0.0) || limit_us > 600.0e6) limit_us = 20.0e6;
  P->args.timeout_ticks = (int64_t)((double)(rate_khz > 0 ? rate_khz : 100000) * 1e-3 * limit_us);

  int64_t s_total = 0, f_total = 0;
  for (const tenoaa_grid& g : P->grids) {
    s_total += 4 * g.n[0] * g.n[1];
    f_total += 4 * (faces_along2(g, 0) * g.n[1] + faces_along2(g, 1) * g.n[0]);
  }
  P->nctl_queue = 2 + 1 + 6 * (int64_t)nsteps;
  P->nctl = P->nctl_queue + 4 * (int64_t)P->ncu * P->max_bpc;
  P->rate_khz = rate_khz > 0 ? rate_khz : 100000;
  e = hipMalloc(&P->d_table, sizeof(BatchProblem) * nprob);
  if (e == hipSuccess) e = hipMalloc(&P->d_pre, sizeof(int64_t) * 2 * (nprob + 1));
  if (e == hipSuccess) e = hipMalloc(&P->d_S, sizeof(double) * s_total);
  if (e == hipSuccess) e = hipMalloc(&P->d_F, sizeof(double) * f_total);
  if (e == hipSuccess) e = hipMalloc(&P->d_amax, sizeof(unsigned long long) * 2 * nprob * (int64_t)nsteps);
  if (e == hipSuccess) e = hipMalloc(&P->d_status, sizeof(int) * nprob);
  if (e == hipSuccess) e = hipMalloc(&P->d_ctl, sizeof(unsigned long long) * P->nctl);
  if (e != hipSuccess) {
    release(P);
    return fail_hip(e);
  }
  P->iargs.ctl = P->d_ctl;
  P->iargs.nctl = P->nctl;
  P->iargs.amax = P->d_amax;
  P->iargs.namax = 2 * (int64_t)nprob * nsteps;
  P->iargs.status = P->d_status;
  P->iargs.nstatus = nprob;

  if (tune_cache_path && tune_cache_path[0]) {
    if (read_cache(P, tune_cache_path)) {
      P->tuned = 2;
    } else {
      float ms = 0.0f;
      e = tune(P, &ms);
      if (e != hipSuccess) {
        release(P);
        return fail_hip(e);
      }
      append_cache(P, tune_cache_path, ms);
      P->tuned = 1;
    }
  }
  e = upload_table(P);
  if (e == hipSuccess) e = build_graph(P);
  if (e != hipSuccess) {
    release(P);
    return fail_hip(e);
  }
  *out = P;
  return TENOAA_OK;
}

int tenoaa_batch_offsets(const tenoaa_batch_plan* plan, int64_t* out) {
  if (!plan || !out) return TENOAA_EINVAL;
  for (int q = 0; q <= plan->nprob; ++q) out[q] = plan->offsets[q];
  return TENOAA_OK;
}

int tenoaa_batch_run(tenoaa_batch_plan* plan, double* U_packed, double* dt_out, void* stream) {
  if (!plan || !U_packed) return TENOAA_EINVAL;
  if (!plan->bound || plan->args.U != U_packed || plan->args.dt_out != dt_out) {
    fill_args(plan, U_packed, dt_out, plan->nsteps);
    void* mp[1] = {&plan->args};
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = reinterpret_cast<void*>(plan->kernel);
    kp.gridDim = dim3(plan->ncu * plan->bpc);
    kp.blockDim = dim3(BT);
    kp.sharedMemBytes = 0;
    kp.kernelParams = mp;
    kp.extra = nullptr;
    hipError_t e = hipGraphExecKernelNodeSetParams(plan->exec, plan->n_main, &kp);
    if (e != hipSuccess) return fail_hip(e);
    plan->bound = true;
  }
  hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TENOAA_OK : fail_hip(e);
}

int tenoaa_batch_get_status(tenoaa_batch_plan* plan, void* stream, int32_t* status_out) {
  if (!plan) return TENOAA_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int> s(plan->nprob);
  unsigned long long abort_word = 0;
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpy(s.data(), plan->d_status, sizeof(int) * plan->nprob, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&abort_word, plan->d_ctl + 1, sizeof(abort_word), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e);
  bool any = false;
  for (int i = 0; i < plan->nprob; ++i) {
    const int q = plan->order[i];
    if (status_out) status_out[q] = s[i] ? 1 : 0;
    any = any || s[i];
  }
  if (abort_word) return TENOAA_ETIMEOUT;
  return any ? TENOAA_ENONPHYSICAL : TENOAA_OK;
}

int tenoaa_batch_run_stats(tenoaa_batch_plan* plan, void* stream, double* out, int32_t n) {
  if (!plan || !out || n < 5) return TENOAA_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nblk = plan->ncu * plan->bpc;
  std::vector<unsigned long long> b(4 * (size_t)nblk);
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess)
    e = hipMemcpy(b.data(), plan->d_ctl + plan->nctl_queue, sizeof(unsigned long long) * b.size(),
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e);
  double wait = 0.0, resident = 0.0, sweep = 0.0, cell = 0.0;
  for (int i = 0; i < nblk; ++i) {
    wait += (double)b[4 * i];
    resident += (double)b[4 * i + 1];
    sweep += (double)b[4 * i + 2];
    cell += (double)b[4 * i + 3];
  }
  const double nbar = 6.0 * plan->nsteps;
  const double r = resident > 0.0 ? 1.0 / resident : 0.0;
  out[0] = wait * r;
  out[1] = resident / nblk / plan->rate_khz * 1e-3;
  out[2] = wait / nblk / nbar / plan->rate_khz * 1e3;
  out[3] = sweep * r;
  out[4] = cell * r;
  return TENOAA_OK;
}

int tenoaa_batch_plan_info(const tenoaa_batch_plan* plan, int32_t* info, int32_t n) {
  if (!plan || !info || n < 10) return TENOAA_EINVAL;
  info[0] = plan->ncu * plan->bpc;
  info[1] = plan->bpc;
  info[2] = plan->chunk;
  info[3] = plan->tuned;
  for (int b = 0; b < NBUCKET; ++b) {
    info[4 + b] = plan->tile_x[b];
    info[7 + b] = plan->tile_y[b];
  }
  return TENOAA_OK;
}

int tenoaa_batch_plan_destroy(tenoaa_batch_plan* plan) {
  if (!plan) return TENOAA_EINVAL;
  release(plan);
  return TENOAA_OK;
}

}  // extern "C"
