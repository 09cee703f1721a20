// Internal interface between the C ABI layer and the kernels of libtenoaa.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tenoaa.h"

namespace tenoaa {

// Device-resident scalars at the head of every workspace.
struct Scalars {
  unsigned long long amax_bits[3];  // max_cells |u_d| + c, as bit patterns
  double dt;
  double mu[3];  // limiter factors kappa_d * dt / dx_d
  int status;    // 0 = ok, 1 = a non-physical state was read
  int pad;
};

// Every member has a default (null pointers, zero sizes), so an argument
// block that a caller fills only in part never carries an indeterminate
// pointer into a kernel.
struct SweepArgs {
  const double* U = nullptr;
  double* F = nullptr;               // face fluxes of this direction, [nvar][nft]
  uint8_t* flags = nullptr;          // flags of this direction, [nvar][2][nft], or null
  const uint8_t* frozen = nullptr;   // decisions to replay instead of taking them, or null
  double* fh_out = nullptr;          // per-field reconstructed fluxes fh_s = f+_s + f-_s, [nvar][nft], or null
  double* theta_out = nullptr;       // per face: the limiter's theta_rho * theta_p (1 where it leaves the flux), or null
  int64_t n[3] = {0, 0, 0};
  int64_t nf = 0;       // faces along the direction
  int64_t nft = 0;      // faces of the direction in total
  int64_t f_begin = 0;  // first face along the direction of this launch's tiles
  int bc_lo = 0, bc_hi = 0;
  int splitting = 0;
  // 1: flags, fh_out and theta_out are indexed pencil by pencil (face f of
  // pencil (t, b) at f + nf (t + n_A b)), the layout the reverse sweep reads
  // along its waves; 0: in grid order, the layout of the C ABI's flag arrays
  int rec_pencil_major = 0;
  double gamma = 0.0;
  const double* bcv[2] = {nullptr, nullptr};  // boundary (Dirichlet, inflow, halo) values of the low/high side, this evaluation's set, or null
  const double* mu = nullptr;  // device: limiter factors
  int* status = nullptr;       // device: status word
  // near-threshold audit (the audit sweep only): decisions whose byte in
  // near_in is non-zero replay `frozen`, the others are taken live; near_out
  // receives 1 where a live decision came within near_tol (relative) of one
  // of its thresholds, and 1 for a replayed one
  const uint8_t* near_in = nullptr;
  uint8_t* near_out = nullptr;
  double near_tol = 0.0;
};

struct UpdateArgs {
  uint32_t div_m[2] = {0, 0}, div_l[2] = {0, 0};  // fast division by n0 and n1 (grids below 2^32 cells)
  const double* F[3] = {nullptr, nullptr, nullptr};
  int64_t nft[3] = {0, 0, 0};
  int64_t nf[3] = {0, 0, 0};
  int64_t n[3] = {0, 0, 0};
  double dx[3] = {0.0, 0.0, 0.0};
  double rdx[3] = {0.0, 0.0, 0.0};  // 1 / dx, correctly rounded (host)
  const double* Un = nullptr;
  const double* Us = nullptr;
  double* out = nullptr;
  const double* dt = nullptr;  // device
};

// One side with prescribed values, for the ghost-cell wave speeds.
struct GhostSpeedArgs {
  const double* U = nullptr;
  const double* fv = nullptr;  // the side's values, set 0 (face values or the first inflow layer)
  int64_t n[3] = {0, 0, 0};
  int dir = 0, hi = 0, bc = 0, pad = 0;
  double gamma = 0.0;
};

struct AdjointArgs {
  const double* U = nullptr;       // state at which the right-hand side is differentiated
  const double* R = nullptr;       // seed: adjoint of dU/dt, layout of U
  double* Ubar = nullptr;          // accumulated in a fixed order (caller zeroes it)
  const uint8_t* flags = nullptr;  // decisions of this direction's forward sweep at U, [nvar][2][nft], pencil by pencil
  const double* fh = nullptr;      // per-field fluxes of that sweep, [nvar][nft], pencil by pencil
  const double* theta = nullptr;   // the sweep's limiter factors per face (pencil by pencil), or null (no limiter)
  const double* bcv[2] = {nullptr, nullptr};  // boundary values of the low/high side (Dirichlet, inflow, halo), else null
  double* hbar[2] = {nullptr, nullptr};       // adjoints of the low/high halo cells (accumulated), or null
  int64_t nft = 0;
  int64_t f_begin = 0;     // first face along the direction of this launch's tiles
  int64_t tile_first = 0;  // block x of a launch runs tile tile_first + x * tile_step (tiles of TN faces from f_begin)
  int64_t n[3] = {0, 0, 0};
  int64_t nf = 0;
  int bc_lo = 0, bc_hi = 0;
  int splitting = 0;
  int tile_step = 1;
  double gamma = 0.0;
  double dx = 0.0;
};

// Argument check of a grid and scheme (shared by every entry point).
bool grid_ok(const tenoaa_grid* g, const tenoaa_scheme* s);
// True if a side of the grid takes prescribed or halo values.
bool has_boundary_values(const tenoaa_grid* g);
// True if a side of the grid takes halo values.
bool has_halo(const tenoaa_grid* g);
// Keeps e for tenoaa_last_hip_error().
void record_hip_error(hipError_t e);

hipError_t launch_sweep_vjp(int order, int ndim, int dir, const AdjointArgs& a, hipStream_t st);
// The reverse sweep's general variant (Roe flux, Dirichlet or inflow sides)
// over all faces, and the common variant's one-wave tail tiles over the faces
// [a.f_begin, a.nf) of a 2D or 3D sweep.
hipError_t launch_vjp_general(int order, int ndim, int dir, const AdjointArgs& a, hipStream_t st);
hipError_t launch_vjp_tail(int order, int ndim, int dir, const AdjointArgs& a, hipStream_t st);
hipError_t launch_zero(double* p, int64_t n, hipStream_t st);
hipError_t launch_axpbypcz(double* out, double a, const double* x, double b, const double* y, double c,
                           const double* z, int64_t n, hipStream_t st);
hipError_t launch_axpdtz(double* out, double a, const double* x, double c, const double* dt, const double* z,
                         int64_t n, hipStream_t st);
hipError_t launch_sweep(int order, int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st);
// The audit sweep (LLF or Rusanov): decisions replayed where a.near_in says,
// taken live elsewhere, with their distance to the thresholds reported in
// a.near_out; whole tiles over every face of the direction.
hipError_t launch_sweep_audit(int order, int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st);
hipError_t launch_update(int ndim, int mode, const UpdateArgs& a, hipStream_t st);
hipError_t launch_wave_speeds(int ndim, const double* U, int64_t ncell, double gam, Scalars* S, int* status,
                              hipStream_t st);
hipError_t launch_ghost_speeds(int ndim, const GhostSpeedArgs& a, Scalars* S, int* status, hipStream_t st);
// One-wave tail tiles of the sweeps (pencils x faces) and their launch over
// the faces [a.f_begin, a.nf) of a direction: a remainder of at most
// SWEEP_TAIL_TN faces beyond the direction's last whole tile.
constexpr int SWEEP_TAIL_TT = 16, SWEEP_TAIL_TN = 4;
hipError_t launch_sweep_tail(int order, int ndim, int dir, const SweepArgs& a, bool limit, hipStream_t st);
hipError_t launch_finalize_dt(Scalars* S, int ndim, const double* dx, double cfl, double* dt_dev, double dt_fixed,
                              hipStream_t st);
// The scalars' wave speeds to amax (ndim doubles), and from it.
hipError_t launch_speeds_out(const Scalars* S, int ndim, double* amax, hipStream_t st);
hipError_t launch_speeds_in(Scalars* S, int ndim, const double* amax, hipStream_t st);

}  // namespace tenoaa
