/*
 * tenoaa.h - C ABI of the MI355X TENO-AA8/10 compressible-Euler library.
 *
 * The library evaluates the finite-difference right-hand side of the Euler
 * equations (arXiv 2109.14340, Sec. 1 for the equations and ideal-gas EOS,
 * Sec. 2 for the conservative flux-difference form) with the eight- or
 * ten-point TENO-AA reconstruction (Sec. 3 and 4; also a twelve-point
 * member of the same framework) applied to Roe-averaged characteristic
 * fields with LLF or Rusanov flux splitting or the Roe flux with entropy fix
 * (Sec. 5), optionally the positivity-preserving flux limiter the paper
 * applies in its extreme cases (Sec. 5.3), and advances it with the SSP-RK3
 * scheme of Sec. 5.  Added forms: vector-Jacobian products (the adjoint), a
 * batched solver for many 2D grids, and the per-piece entry points of a grid
 * split into one piece per GPU.
 *
 * Conventions shared by every entry point
 *  - Memory: every double/uint8 array argument is DEVICE memory on the
 *    current HIP device unless stated otherwise.  Grid and scheme structs are
 *    HOST memory and are read before the call returns.  The caller owns all
 *    buffers; the library never allocates or frees, except that a batch plan
 *    owns the device memory it allocates at creation and frees at destruction.
 *  - Layout of a state array U: float64, structure of arrays
 *    U[v][k][j][i] with i (x) fastest, v = 0..nvar-1, nvar = ndim + 2 and
 *    components (rho, rho*u, [rho*v], [rho*w], E).  Sizes of unused
 *    dimensions are 1.  No ghost cells: boundaries are applied internally.
 *  - Faces: along direction d, face f is the left face of cell f; there are
 *    nf_d = n_d faces for a periodic direction and n_d + 1 otherwise.  A face
 *    array of direction d has the cell array's shape with axis d of length
 *    nf_d.
 *  - Flags (optional output): uint8 per (direction, characteristic field,
 *    split side, face), laid out [d][field][side][face array of d] with the
 *    directions concatenated in order x, y, z.  Fields are ordered
 *    (u-c, u, shear..., u+c); side 0 is the upwind-biased (+) side.  Bits
 *    0-1: large stencil chosen (0 none, 1 S3, 2 S4, 3 S5, or S6 of TENO12-AA
 *    when bit 2 is also set); bits 2-4: the cut-off deltas of the three
 *    small stencils when none was chosen; bits 5-7: [beta] - 7 of the
 *    adaptive C_T = 10^-[beta] (Sec. 3.4).  With the Roe flux the byte of a
 *    side that is not reconstructed is 0, which no decision produces.
 *  - Streams: `stream` is a hipStream_t passed as void*; NULL is the null
 *    stream.  Calls enqueue work and return without synchronising, except
 *    where stated.  Calls on distinct (stream, workspace) pairs are
 *    independent; calls sharing a workspace must be ordered by the caller.
 *  - Errors: 0 on success; TENOAA_EINVAL for a bad argument (nothing is
 *    enqueued); TENOAA_EUNSUPPORTED for a valid but unimplemented option;
 *    TENOAA_EHIP when a HIP call fails (tenoaa_last_hip_error() returns
 *    the hipError_t); TENOAA_EWORKSPACE when ws_bytes is too small.
 *    Physical failures (rho <= 0, p <= 0 or NaN in a state the kernels read)
 *    are asynchronous: they set a status word inside the workspace that
 *    tenoaa_get_status() reports.
 */
#ifndef TENOAA_H
#define TENOAA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TENOAA_OK = 0,
  TENOAA_EINVAL = -1,
  TENOAA_EUNSUPPORTED = -2,
  TENOAA_EHIP = -3,
  TENOAA_ENONPHYSICAL = -4,
  TENOAA_EWORKSPACE = -5,
  TENOAA_ETIMEOUT = -6
};

/* Boundary conditions (Appendix A of the paper; OUTFLOW copies the nearest
 * interior cell into every ghost layer).  A direction is either periodic on
 * both sides or on neither.  DIRICHLET is the Appendix's second-order form:
 * with prescribed face primitives (rho', u', p'), ghost cell r (r = 1, 2, ...)
 * takes, in primitive variables, 2 (rho', u', p') minus the primitives of
 * interior cell r - 1 counted from that face; the face values come from
 * tenoaa_grid.bc_values.  INFLOW is a supersonic inflow (every
 * characteristic enters the domain, as at the outer boundaries of the Noh
 * problem in Sec. 5): the ghost cells take prescribed states, also from
 * tenoaa_grid.bc_values.  HALO (not a boundary of the paper): the ghost
 * cells take given CONSERVED states as they are, so that a grid split into
 * pieces (one per GPU) computes on each piece exactly what the whole grid
 * computes there when each side facing a neighbour piece holds the
 * neighbour's order/2 cells next to that face (a halo exchange before every
 * SSP-RK3 stage; see tenoaa_rk3_stage). */
enum {
  TENOAA_BC_PERIODIC = 0,
  TENOAA_BC_OUTFLOW = 1,
  TENOAA_BC_SYMMETRY = 2,
  TENOAA_BC_NOSLIP = 3,
  TENOAA_BC_DIRICHLET = 4,
  TENOAA_BC_INFLOW = 5,
  TENOAA_BC_HALO = 6
};

/* Flux splitting (Sec. 5): LLF uses, per characteristic field, the largest
 * |eigenvalue| over the reconstruction window; RUSANOV one max(|u_n| + c)
 * over the window for every field.  ROE is the Roe flux with entropy fix
 * that Sec. 5.2 uses for its blast waves and Rayleigh-Taylor runs: per field,
 * where the eigenvalue has one strict sign at both cells of the face, the
 * unsplit characteristic flux is reconstructed from the upwind side alone
 * (the flag byte of the other side is 0, which no decision produces);
 * elsewhere the field is split as with LLF.  Decision replay
 * (TENOAA_FLAGS_REPLAY, recorded flags given to the adjoint entry points)
 * replays the side each field reconstructs with the other decisions: the side
 * whose recorded byte is 0 is not reconstructed. */
enum { TENOAA_LLF = 0, TENOAA_RUSANOV = 1, TENOAA_ROE = 2 };

/* Workspace purposes for tenoaa_workspace_bytes: tenoaa_rhs (and the split-
 * grid pieces), tenoaa_step, tenoaa_rhs_vjp, tenoaa_step_vjp, and the taped
 * step (tenoaa_step_tape and tenoaa_step_vjp_tape). */
enum { TENOAA_WS_RHS = 0, TENOAA_WS_STEP = 1, TENOAA_WS_RHS_VJP = 2, TENOAA_WS_STEP_VJP = 3, TENOAA_WS_STEP_TAPE = 4 };

/* Uniform cell-centred grid: cell i of direction d has centre (i + 1/2) dx[d].
 * n[d] >= order/2 for d < ndim and n[d] == 1 otherwise; dx[d] > 0; in 2D
 * and 3D n[1], n[2] <= 65535 and n[0] <= 524280 (the launch grids' y and z
 * extents); nvar x the cell count below 9e15.
 *
 * Boundary values (read only where bc_lo[d] / bc_hi[d] is
 * TENOAA_BC_DIRICHLET, TENOAA_BC_INFLOW or TENOAA_BC_HALO, else ignored and
 * may be NULL):
 * bc_values[d][0] (low side) and bc_values[d][1] (high side) are DEVICE
 * arrays owned by the caller.  With P = the product of n[k] over k != d (the
 * face plane, the lower of the two remaining axes fastest), a "layer" is
 * nvar x P doubles: the planes rho, u_x, [u_y], [u_z], p (primitives,
 * velocities in axis order).  A Dirichlet side holds bc_sets layers (the face
 * values); an inflow side bc_sets x (order / 2) layers, per set the ghost
 * cells r = 1 .. order/2 counted outward from the face.  A halo side has the
 * inflow layout with conserved planes (rho, rho u_x, [rho u_y], [rho u_z], E)
 * instead of primitives.  bc_sets is 1 or 3:
 * with 3, stage s of an SSP-RK3 step reads set s (the caller supplies the
 * values at t, t + dt and t + dt/2, the times the three stages approximate)
 * and tenoaa_rhs reads set 0; with 1 every evaluation reads set 0.  A smaller
 * array than this is undefined behaviour (the library cannot check device
 * allocations).  The batch plan takes Dirichlet and inflow sides with one
 * value set (used by every step of a run) and without the Roe flux, and
 * rejects other cases with TENOAA_EUNSUPPORTED; tenoaa_rhs_vjp,
 * tenoaa_step_vjp and the taped step reject halo sides (tenoaa_rhs_vjp_halo
 * takes them).  The adjoint entry points differentiate a Dirichlet
 * ghost through its reflection rule (the face values are constants), take
 * inflow ghosts as constants, and read set s in stage s as the step does. */
typedef struct {
  int32_t ndim;
  int32_t bc_sets;
  int64_t n[3];
  double dx[3];
  int32_t bc_lo[3];
  int32_t bc_hi[3];
  const double* bc_values[3][2];
} tenoaa_grid;

/* order: 8 (TENO8-AA) or 10 (TENO10-AA), Sec. 4, or 12 (TENO12-AA: the
 * Sec. 3.1 framework with one more symmetric large stencil S6 = cells
 * i-5 .. i+6 tried before S5; the paper prints no optimised scheme for it, so
 * S6 uses the maximum-order (12th) reconstruction); splitting: TENOAA_LLF,
 * TENOAA_RUSANOV or TENOAA_ROE; positivity: 1 enables the flux limiter. */
typedef struct {
  int32_t order;
  int32_t splitting;
  int32_t positivity;
  int32_t pad;
} tenoaa_scheme;

/* Bytes of device workspace a call of the given purpose needs for this grid.
 * Returns 0 for invalid arguments.  The workspace must be 256-byte aligned
 * and stays owned by the caller. */
size_t tenoaa_workspace_bytes(const tenoaa_grid* grid, const tenoaa_scheme* scheme, int32_t which);

/* Semi-discrete right-hand side dUdt = -sum_d (F_{f+1} - F_f)/dx_d
 * (Sec. 2) of the state U, directions in order x, y, z.  dUdt (same layout as
 * U, must not alias it) is overwritten.  gamma > 1 is the ratio of specific
 * heats.  The limiter acts only if scheme->positivity and dt_limiter > 0;
 * its CFL weights use the wave speeds of U.  flags may be NULL. */
int tenoaa_rhs(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U, double* dUdt,
               double dt_limiter, uint8_t* flags, void* ws, size_t ws_bytes, void* stream);

/* Size of the buffer tenoaa_rhs_noalloc uses instead of a workspace: 80 MiB
 * (a right-hand side of up to 2D 1024^2 or 3D 80^3 cells). */
#define TENOAA_SCRATCH_BYTES ((size_t)80 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * tenoaa_rhs without a caller's workspace.  Its workspace is a buffer of
 * TENOAA_SCRATCH_BYTES the library holds in device memory, one per GPU, from
 * the first call on that GPU (made with that GPU current) until the process
 * ends; the call allocates nothing (nor does it take part in
 * tenoaa_timing_enable's measurement, whose events would).  Arguments as
 * tenoaa_rhs, plus
 * status_dev (device int32, or NULL): receives 0, or 1 if a non-physical
 * state was read during this call.  Every call on one GPU shares that GPU's
 * buffer and leaves it holding its face fluxes: calls that overlap on one
 * GPU (other streams or host threads) race and must be serialised by the
 * caller.  Returns TENOAA_EWORKSPACE if the grid's right-hand-side workspace
 * (tenoaa_workspace_bytes(grid, scheme, TENOAA_WS_RHS)) exceeds
 * TENOAA_SCRATCH_BYTES, and the errors of tenoaa_rhs otherwise. */
int tenoaa_rhs_noalloc(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U,
                       double* dUdt, double dt_limiter, uint8_t* flags, int32_t* status_dev, void* stream);

/* One SSP-RK3 step (Sec. 5, Shu-Osher form) of U in place.  dt_dev is a
 * device double: if it holds a value > 0 on entry that dt is used, otherwise
 * dt = cfl / sum_d (a_d / dx_d) with a_d = max over cells of |u_d| + c is
 * computed from U^n on the device and stored there.  No host
 * synchronisation.  0 < cfl <= 1; with the limiter on, cfl <= 0.5. */
int tenoaa_step(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl, double* U,
                double* dt_dev, void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of the right-hand side (the adjoint form; not a
 * formula of the paper).  U_bar (overwritten) = (d dUdt / dU)^T dUdt_bar at
 * U, with every threshold decision frozen: the stencil chosen by the cascade
 * and the small-stencil deltas (Sec. 3.3), i.e. the linear weights of each
 * reconstruction, and the cell and sign that attain each splitting speed
 * (with TENOAA_ROE also the side each field reconstructs).
 * flags: NULL to freeze the decisions taken at U, or a flag array (layout
 * above, e.g. recorded by tenoaa_rhs at another state) whose decisions are
 * used instead.  The limiter is not part of the differentiated map (it acts
 * only with a dt).  Every sum is taken in a fixed order, so U_bar is the
 * same bit for bit from run to run.  U_bar must not alias U or dUdt_bar. */
int tenoaa_rhs_vjp(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U,
                   const double* dUdt_bar, double* U_bar, const uint8_t* flags, void* ws, size_t ws_bytes,
                   void* stream);

/* tenoaa_rhs_vjp for a piece of a split grid: the grid may have halo sides,
 * whose cells belong to neighbour pieces, so their share of the adjoint goes
 * back to those pieces.  halo_bar (host array of 6 device pointers, entry
 * 2 d + side) holds, for every halo side, order/2 x nvar x P doubles in the
 * halo layout of one set (layer r = 1 .. order/2 outward, conserved planes);
 * they are overwritten with (d dUdt / d halo)^T dUdt_bar, the adjoint of
 * that side's halo cells, which the caller adds to the neighbour's U_bar at
 * the same cells.  Entries of other sides are ignored.  U_bar covers the
 * piece's own cells as in tenoaa_rhs_vjp; with the halos of a piece's
 * neighbours summed in, the pieces give the whole grid's adjoint (up to the
 * order of the sums).  Same errors as tenoaa_rhs_vjp, and
 * TENOAA_EINVAL for a null halo_bar or a halo side without its pointer. */
int tenoaa_rhs_vjp_halo(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U,
                        const double* dUdt_bar, double* U_bar, const uint8_t* flags, double* const* halo_bar,
                        void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of one SSP-RK3 step with the time step frozen:
 * Un_bar (overwritten) = (d U^{n+1} / d U^n)^T Unp1_bar.  dt_dev is the device
 * double holding the dt the forward step used (> 0).  The three stage states
 * are recomputed from Un inside the call; each stage's decisions are frozen at
 * its own state, or, with flags3 non-NULL, taken from flags3 (the three
 * stages' decisions as recorded by tenoaa_step_flags).  With the limiter on,
 * the limiter acts as in tenoaa_step (its speeds from Un, the given dt) and
 * its factors theta per face, F = F_LF + theta (F_H - F_LF), are frozen like
 * the other decisions, as is the cell giving the Lax-Friedrichs speed of
 * F_LF.  Un_bar must not alias Un or Unp1_bar. */
int tenoaa_step_vjp(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* Un,
                    const double* dt_dev, const double* Unp1_bar, double* Un_bar, const uint8_t* flags3, void* ws,
                    size_t ws_bytes, void* stream);

/* One SSP-RK3 step (Sec. 5) that keeps what its adjoint needs: Unp1 =
 * U^{n+1} from Un, bit for bit what tenoaa_step gives on a copy of Un (same
 * dt rule: *dt_dev <= 0 on entry takes dt from the CFL condition and stores
 * it there, a positive value is used as given; the same limits on cfl), and
 * ws (TENOAA_WS_STEP_TAPE bytes) left holding the step's tape: the two
 * intermediate stage states and every stage's decisions, per-field fluxes
 * and limiter factors.  tenoaa_step_vjp_tape then runs only the reverse
 * sweeps, where tenoaa_step_vjp recomputes the stages first.  The tape is
 * two states plus about 5 (1D) to 7 (3D) doubles per face, direction and
 * stage (the whole workspace is 14 GB for a 256^3 TENO10-AA step with the
 * limiter), kept as long as the caller keeps ws.  Unp1 must not alias Un.  EINVAL for null
 * pointers or a bad cfl, EWORKSPACE, EUNSUPPORTED for halo sides. */
int tenoaa_step_tape(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl,
                     const double* Un, double* dt_dev, double* Unp1, void* ws, size_t ws_bytes, void* stream);

/* The vector-Jacobian product of the step whose tape tenoaa_step_tape left
 * in ws: Un_bar (overwritten) = (d U^{n+1} / d Un)^T Unp1_bar with every
 * decision, limiter factor and dt frozen as in tenoaa_step_vjp (equal to it
 * bit for bit).  Un and dt_dev must be the step's own (unchanged since the
 * tape was taken; the tape is not checked against them); the tape stays
 * whole, so several seeds may use it.  Un_bar must not alias Un or
 * Unp1_bar.  Same errors as tenoaa_step_vjp. */
int tenoaa_step_vjp_tape(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* Un,
                         const double* dt_dev, const double* Unp1_bar, double* Un_bar, void* ws, size_t ws_bytes,
                         void* stream);

/* Wave speeds a_d = max (|u_d| + c) over the cells of U and the first ghost
 * layer of every side with prescribed or halo values (value set 0), d <
 * ndim, written to amax_dev (device, ndim doubles; the CFL condition of
 * Sec. 5 and the limiter's weights use them).  For a grid split into pieces
 * the step's speeds are the maxima over the pieces.  Workspace: RHS. */
int tenoaa_wave_speeds(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U,
                       double* amax_dev, void* ws, size_t ws_bytes, void* stream);

/* Stage `stage` (1, 2, 3) of the SSP-RK3 step (Sec. 5, Shu-Osher form):
 *   1: out = Un + dt L(Un)
 *   2: out = 3/4 Un + 1/4 Us + 1/4 dt L(Us)
 *   3: out = 1/3 Un + 2/3 Us + 2/3 dt L(Us)
 * with the arithmetic of tenoaa_step, so the three stages with the same dt
 * and speeds give tenoaa_step's result bit for bit.  amax_dev (device, ndim
 * doubles): the wave speeds of Un (tenoaa_wave_speeds; for a split grid the
 * maxima over the pieces), which the limiter's weights use; dt_dev (device
 * double): if it holds a value <= 0 on entry, dt = cfl / sum_d (a_d / dx_d)
 * from amax_dev is computed and stored there (pass the same dt_dev to the
 * later stages).  Sides with boundary or halo values read set stage - 1 when
 * bc_sets is 3, else set 0: a split grid refreshes its halo sides from the
 * neighbours' stage state before each stage.  Us is ignored in stage 1 and
 * required in stages 2 and 3; out may alias Un or Us (each cell's update
 * reads only its own Un, Us values after the sweeps).  0 < cfl <= 1, with
 * the limiter cfl <= 0.5.  Workspace: RHS. */
int tenoaa_rk3_stage(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl, int32_t stage,
                     const double* amax_dev, double* dt_dev, const double* Un, const double* Us, double* out,
                     void* ws, size_t ws_bytes, void* stream);

/* Decision modes of tenoaa_step_flags. */
enum { TENOAA_FLAGS_NONE = 0, TENOAA_FLAGS_RECORD = 1, TENOAA_FLAGS_REPLAY = 2 };

/* tenoaa_step with the threshold decisions of its three stages recorded or
 * replayed.  flags3 (device, 3 x the flag-array size, stage-major, each
 * stage in the flag layout above): with TENOAA_FLAGS_RECORD it receives the
 * decisions every stage takes; with TENOAA_FLAGS_REPLAY each reconstruction
 * uses the recorded stencil and deltas instead of deciding (the map whose
 * derivative tenoaa_step_vjp computes), and flags3 is only read;
 * TENOAA_FLAGS_NONE is tenoaa_step (flags3 may be NULL). */
int tenoaa_step_flags(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl, double* U,
                      double* dt_dev, uint8_t* flags3, int32_t mode, void* ws, size_t ws_bytes, void* stream);

/* tenoaa_step with every threshold decision (Sec. 3.3 selection cascade and
 * its fallback deltas, Sec. 3.4 cut-off bucket) audited for its distance to
 * the threshold: the finite-difference check of the adjoint freezes only the
 * decisions near a threshold and takes the others live.  All arrays are
 * device arrays of 3 x the flag-array size (stage-major, the flag layout
 * above), one byte per reconstruction:
 *   near_in3 (or NULL): where non-zero the reconstruction replays the byte of
 *     base3 (required with near_in3) instead of deciding; elsewhere, and
 *     everywhere with NULL, it decides live;
 *   flags_out3 (or NULL): the decision bytes used (live or replayed);
 *   near_out3 (or NULL): 1 where a live decision made a test within the
 *     relative distance near_tol of its threshold (chi_p / C_T or chi_k / C_T
 *     within 1 +- near_tol, or the cut-off exponent within near_tol of an
 *     integer), 1 for a replayed one, else 0.
 * dt_dev as in tenoaa_step (> 0: used as given).  0 < near_tol < 1; LLF or
 * Rusanov splitting (TENOAA_EUNSUPPORTED for the Roe flux); other errors as
 * tenoaa_step.  Workspace: STEP. */
int tenoaa_step_near(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl, double* U,
                     double* dt_dev, const uint8_t* base3, const uint8_t* near_in3, uint8_t* flags_out3,
                     uint8_t* near_out3, double near_tol, void* ws, size_t ws_bytes, void* stream);

/* Scalar linear advection u_t + u_x = 0 on a periodic grid of n cells of
 * width dx (Sec. 5.1, the paper's accuracy test): `nsteps` SSP-RK3 steps of
 * size dt of du_i/dt = -(fhat_{i+1/2} - fhat_{i-1/2}) / dx, where fhat_{i+1/2}
 * is the TENO-AA reconstruction (order 8, 10 or 12) of the flux f = u from cells
 * i - order/2 + 1 .. i + order/2 (the speed is +1, so no splitting).  u (device,
 * n doubles) is advanced in place.  n in [order, 2048] (one workgroup holds
 * the grid in LDS); dx > 0, dt > 0, nsteps >= 0; TENOAA_EINVAL otherwise.  Enqueued on `stream` as one launch. */
int tenoaa_advect(int32_t order, int64_t n, double dx, double dt, int64_t nsteps, double* u, void* stream);

/* Synchronises `stream`, reads and clears the workspace status word.
 * *out = 0 if every state read since the last call was physical, else 1.
 * Returns TENOAA_ENONPHYSICAL if *out != 0, otherwise 0 (or an error). */
int tenoaa_get_status(void* ws, void* stream, int32_t* out);

/* ---- Batched form (not a formula of the paper): many independent 2D
 * problems of uneven size, each advanced by SSP-RK3 steps with its own dt, in
 * one persistent launch replayed from a HIP graph.  Every problem evolves
 * exactly (bit for bit) as nsteps calls of tenoaa_step on it would. */
typedef struct tenoaa_batch_plan tenoaa_batch_plan;

/* Plans nprob >= 1 problems (grids[p]: host array, each with ndim == 2 and
 * valid as for tenoaa_step) sharing one scheme, gamma and cfl (dt of every
 * step of every problem from the CFL condition on its own state), nsteps >= 1
 * steps per run.  The plan owns its device workspace (a stage state and the
 * face fluxes of every problem, about 3 states' worth) and a HIP graph of
 * one clearing kernel and the persistent kernel, all created here on the
 * current device.  Tile shapes (two candidates per sweep direction for each
 * of three n_x buckets: <= 160, <= 320, larger), the items taken per queue
 * access and the blocks per compute unit are chosen as follows: with
 * tune_cache_path NULL or "", defaults; otherwise the JSON-lines file is
 * searched for this plan's key ("gfx950 order=O split=S limit=L
 * buckets=a,b,c", the counts of problems per n_x bucket) and, when absent,
 * the choices are tuned now on the device by timing one step of the batch
 * from a uniform state, and appended to the file as
 * {"key": ..., "tile_x": [3], "tile_y": [3], "chunk": c, "blocks_per_cu": b,
 * "step_ms": t}.  Results do not depend on these choices.  A phase barrier
 * of the persistent kernel gives up after 20 s (the environment variable
 * TENOAA_BATCH_BARRIER_TIMEOUT_US, read here, sets another limit; tests use it
 * to exercise tenoaa_batch_get_status's TENOAA_ETIMEOUT).  Returns EINVAL
 * for bad arguments, EUNSUPPORTED for ndim != 2, a halo side, three value
 * sets, or prescribed sides with the Roe flux, EHIP on a HIP failure;
 * *out is NULL unless 0 is returned. */
int tenoaa_batch_plan_create(const tenoaa_grid* grids, int32_t nprob, const tenoaa_scheme* scheme, double gamma,
                             double cfl, int32_t nsteps, const char* tune_cache_path, tenoaa_batch_plan** out);

/* Packed layout of the batch state: out (host, nprob + 1 entries) receives
 * the offset in doubles of problem p's state (the single-grid layout) for
 * p < nprob, then the total length.  Problems are packed densely in the
 * caller's order. */
int tenoaa_batch_offsets(const tenoaa_batch_plan* plan, int64_t* out);

/* Advances every problem of the packed device state U_packed by the plan's
 * nsteps steps in place: one graph launch on `stream`, no allocation and no
 * host synchronisation.  dt_out (device, nprob * nsteps doubles, problem-major)
 * receives every dt used, or is NULL.  Runs of one plan share its workspace:
 * the caller orders them (one stream, or events). */
int tenoaa_batch_run(tenoaa_batch_plan* plan, double* U_packed, double* dt_out, void* stream);

/* Synchronises `stream` and reports the last run: status_out (host, nprob
 * entries, or NULL) receives 1 for each problem in which a non-physical
 * state was read.  Returns TENOAA_ETIMEOUT if the launch abandoned the run
 * at a phase barrier (its grid was not resident; results invalid),
 * TENOAA_ENONPHYSICAL if any problem was non-physical, else 0. */
int tenoaa_batch_get_status(tenoaa_batch_plan* plan, void* stream, int32_t* status_out);

/* Synchronises `stream` and reports how the blocks of the last
 * tenoaa_batch_run spent their time (read from per-block wall-clock counters
 * the persistent kernel keeps): out (host, n >= 5 entries) receives the share
 * of the blocks' resident time spent waiting at phase barriers (imbalance
 * between blocks plus the barrier's own latency), the mean time a block was
 * resident in seconds, the mean wait per block and barrier in microseconds,
 * and the shares of the resident time spent in sweep items and in update and
 * wave-speed items (the rest: taking items from the queue).  Meaningful only
 * after a run that completed; EINVAL for a null plan or out, or n < 5; EHIP
 * on a HIP failure. */
int tenoaa_batch_run_stats(tenoaa_batch_plan* plan, void* stream, double* out, int32_t n);

/* Launch choices of a plan: info (host, n >= 10 entries) receives blocks
 * launched, blocks per compute unit, items per queue access, how the choices
 * were made (0 defaults, 1 tuned now, 2 from the cache file), then the x-tile
 * and y-tile candidates of the three n_x buckets. */
int tenoaa_batch_plan_info(const tenoaa_batch_plan* plan, int32_t* info, int32_t n);

/* Releases the plan's device memory and graph (after its runs completed). */
int tenoaa_batch_plan_destroy(tenoaa_batch_plan* plan);

/* hipError_t of the last failed HIP call in this thread (0 if none). */
int tenoaa_last_hip_error(void);

/* Kernel classes for per-kernel timing. */
enum {
  TENOAA_KCLASS_SWEEP_X = 0,
  TENOAA_KCLASS_SWEEP_Y = 1,
  TENOAA_KCLASS_SWEEP_Z = 2,
  TENOAA_KCLASS_UPDATE = 3,
  TENOAA_KCLASS_WAVESPEED = 4,
  TENOAA_KCLASS_VJP_X = 5,
  TENOAA_KCLASS_VJP_Y = 6,
  TENOAA_KCLASS_VJP_Z = 7,
  TENOAA_KCLASS_COUNT = 8
};

/* Measurement aid (host state shared by all threads, guarded by a mutex).
 * While enabled (on != 0), every kernel launch of the library is bracketed by
 * HIP events recorded on the launch's own stream; this adds two event records
 * per launch and should stay off outside measurements. */
int tenoaa_timing_enable(int32_t on);

/* Waits for every bracketed launch so far, then returns for one kernel class
 * the number of launches and their summed duration in milliseconds since the
 * previous read of that class, and resets that class.  TENOAA_EINVAL for a
 * bad class or null pointers. */
int tenoaa_timing_read(int32_t kclass, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* TENOAA_H */
