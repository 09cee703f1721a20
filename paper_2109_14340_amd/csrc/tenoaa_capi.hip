// C ABI of libtenoaa (declared in include/tenoaa.h): argument validation,
// workspace layout and the launch sequence of one right-hand side or one
// SSP-RK3 step.  Nothing here allocates device memory.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "tenoaa.h"
#include "tenoaa_internal.h"

// The library's own workspace for tenoaa_rhs_noalloc: one buffer of
// TENOAA_SCRATCH_BYTES on each GPU the library runs on, held until the
// process ends.  In host code this name is only a stand-in for the symbol:
// the buffer's device address on a GPU comes from hipGetSymbolAddress with
// that GPU current, and that address is what kernels and copies are given.
static __device__ __align__(256) char scratch[TENOAA_SCRATCH_BYTES];

namespace {

// The stage kernels read dt from the workspace scalars; the step adjoint takes
// it from the caller's device double.
__global__ void copy_dt_kernel(tenoaa::Scalars* S, const double* dt) {
  if (threadIdx.x == 0) S->dt = *dt;
}

thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e) {
  g_last_hip_error = (int)e;
  return TENOAA_EHIP;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// ---- optional per-kernel timing (measurement aid)
struct TimedLaunch {
  int cls;
  hipEvent_t a, b;
};
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<TimedLaunch> g_timed;
int64_t g_launches[TENOAA_KCLASS_COUNT];
double g_total_ms[TENOAA_KCLASS_COUNT];

// Set for the duration of a call that must not allocate (event creation
// allocates): its launches are not timed.
thread_local bool g_untimed = false;

// Brackets one launch with events on `st` when timing is enabled.
template <class F>
hipError_t timed(int cls, hipStream_t st, F&& launch) {
  if (g_untimed) return launch();
  bool on;
  {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    on = g_timing_on;
  }
  if (!on) return launch();
  TimedLaunch t{cls, nullptr, nullptr};
  hipError_t e = hipEventCreate(&t.a);
  if (e == hipSuccess) e = hipEventCreate(&t.b);
  if (e == hipSuccess) e = hipEventRecord(t.a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(t.b, st);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timed.push_back(t);
  return hipSuccess;
}

// Folds completed timed launches into the per-class totals (waits for them).
hipError_t collect_timing() {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  for (const TimedLaunch& t : g_timed) {
    hipError_t e = hipEventSynchronize(t.b);
    if (e != hipSuccess) return e;
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) return e;
    g_launches[t.cls] += 1;
    g_total_ms[t.cls] += ms;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  g_timed.clear();
  return hipSuccess;
}

bool valid_grid(const tenoaa_grid* g, const tenoaa_scheme* s) {
  if (!g || !s) return false;
  if (g->ndim < 1 || g->ndim > 3) return false;
  if (s->order != 8 && s->order != 10 && s->order != 12) return false;
  if (s->splitting != TENOAA_LLF && s->splitting != TENOAA_RUSANOV && s->splitting != TENOAA_ROE) return false;
  if (s->positivity != 0 && s->positivity != 1) return false;
  for (int d = 0; d < 3; ++d) {
    if (d < g->ndim) {
      if (g->n[d] < s->order / 2 || !(g->dx[d] > 0.0)) return false;
      if (g->bc_lo[d] < 0 || g->bc_lo[d] > TENOAA_BC_HALO || g->bc_hi[d] < 0 || g->bc_hi[d] > TENOAA_BC_HALO)
        return false;
      if ((g->bc_lo[d] == TENOAA_BC_PERIODIC) != (g->bc_hi[d] == TENOAA_BC_PERIODIC)) return false;
      for (int h = 0; h < 2; ++h)
        if ((h ? g->bc_hi[d] : g->bc_lo[d]) >= TENOAA_BC_DIRICHLET) {
          if (!g->bc_values[d][h] || (g->bc_sets != 1 && g->bc_sets != 3)) return false;
        }
    } else if (g->n[d] != 1) {
      return false;
    }
  }
  // flat indices stay within int64, and the y and z extents of every sweep's
  // launch grid (tiles across the direction, the remaining axis) within 65535
  // blocks: n_y, n_z <= 65535, and n_x <= 8 x 65535 (y and z sweeps tile x by
  // at least 8 pencils)
  const double cells = (double)g->n[0] * (double)g->n[1] * (double)g->n[2];
  if (cells * (g->ndim + 2) > 9.0e15) return false;
  if (g->ndim >= 2 && (g->n[1] > 65535 || g->n[2] > 65535 || g->n[0] > 8 * 65535)) return false;
  return true;
}

int64_t faces_along(const tenoaa_grid* g, int d) {
  return g->bc_lo[d] == TENOAA_BC_PERIODIC ? g->n[d] : g->n[d] + 1;
}

int64_t faces_total(const tenoaa_grid* g, int d) {
  int64_t t = faces_along(g, d);
  for (int k = 0; k < 3; ++k)
    if (k != d) t *= g->n[k];
  return t;
}

struct Layout {
  size_t scalars;       // offset of tenoaa::Scalars
  size_t fbuf[3];       // face flux arrays per direction
  size_t vjp[3][3];     // adjoint calls: [stage][direction] decisions, then per-field fluxes
  size_t vjp_fh_rel[3]; // offset of a direction's per-field fluxes after its decisions
  size_t vjp_th_rel[3]; // offset of a direction's limiter factors after its decisions (limiter only)
  size_t stage;         // RK stage state(s)
  size_t state_bytes;   // aligned size of one state
  size_t total;
};

Layout layout(const tenoaa_grid* g, int which, bool limiter = false) {
  Layout L;
  const int nv = g->ndim + 2;
  const int64_t ncell = g->n[0] * g->n[1] * g->n[2];
  size_t off = 0;
  L.scalars = off;
  off += align256(sizeof(tenoaa::Scalars));
  for (int d = 0; d < 3; ++d) {
    L.fbuf[d] = off;
    if (d < g->ndim) off += align256((size_t)nv * (size_t)faces_total(g, d) * sizeof(double));
  }
  // decisions and per-field fluxes of every direction, for one stage (RHS_VJP)
  // or the three stages of a step (STEP_VJP)
  const bool step_adj = which == TENOAA_WS_STEP_VJP || which == TENOAA_WS_STEP_TAPE;
  const int nstage = step_adj ? 3 : (which == TENOAA_WS_RHS_VJP ? 1 : 0);
  for (int st = 0; st < 3; ++st) {
    for (int d = 0; d < 3; ++d) {
      L.vjp[st][d] = off;
      if (st < nstage && d < g->ndim) {
        const size_t nft = (size_t)faces_total(g, d);
        L.vjp_fh_rel[d] = align256((size_t)nv * 2 * nft);
        L.vjp_th_rel[d] = L.vjp_fh_rel[d] + align256((size_t)nv * nft * sizeof(double));
        off += L.vjp_th_rel[d] + (limiter ? align256(nft * sizeof(double)) : 0);
      }
    }
  }
  L.stage = off;
  const size_t state = align256((size_t)nv * (size_t)ncell * sizeof(double));
  if (which == TENOAA_WS_STEP) off += state;
  if (which == TENOAA_WS_STEP_VJP) off += 4 * state;  // U1, U2 (later B1), V, B2
  if (which == TENOAA_WS_STEP_TAPE) off += 5 * state;  // U1, U2, V, B2, B1: the tape stays whole
  L.state_bytes = state;
  L.total = off;
  return L;
}

struct Ctx {
  const tenoaa_grid* g;
  const tenoaa_scheme* s;
  double gamma;
  char* ws;
  Layout L;
  tenoaa::Scalars* S;
  hipStream_t st;
};

// True if a side takes prescribed or halo values.
bool boundary_values_any(const tenoaa_grid* g) {
  for (int d = 0; d < g->ndim; ++d)
    if (g->bc_lo[d] >= TENOAA_BC_DIRICHLET || g->bc_hi[d] >= TENOAA_BC_DIRICHLET) return true;
  return false;
}

// Boundary values of side (d, h) for SSP-RK3 stage `stage` (0 outside a
// step), or null: a set holds one layer of nvar face-plane arrays
// (Dirichlet) or order/2 layers (inflow, halo).
const double* face_values(const tenoaa_grid* g, int order, int d, int h, int stage) {
  const int bc = h ? g->bc_hi[d] : g->bc_lo[d];
  if (bc != TENOAA_BC_DIRICHLET && bc != TENOAA_BC_INFLOW && bc != TENOAA_BC_HALO) return nullptr;
  int64_t plane = 1;
  for (int k = 0; k < 3; ++k)
    if (k != d) plane *= g->n[k];
  const int64_t layers = bc == TENOAA_BC_DIRICHLET ? 1 : order / 2;
  const int set = g->bc_sets == 3 ? stage : 0;
  return g->bc_values[d][h] + (int64_t)set * layers * (g->ndim + 2) * plane;
}

// a_d over the cells of U and over the ghost cells next to the faces of every
// side with prescribed values (value set 0), which the boundary faces see.
hipError_t wave_speeds(const Ctx& c, const double* U) {
  const tenoaa_grid* g = c.g;
  const int64_t ncell = g->n[0] * g->n[1] * g->n[2];
  hipError_t e = tenoaa::launch_wave_speeds(g->ndim, U, ncell, c.gamma, c.S, &c.S->status, c.st);
  for (int d = 0; d < g->ndim && e == hipSuccess; ++d)
    for (int h = 0; h < 2 && e == hipSuccess; ++h) {
      const double* fv = face_values(g, c.s->order, d, h, 0);
      if (!fv) continue;
      tenoaa::GhostSpeedArgs a{};
      a.U = U;
      a.fv = fv;
      for (int k = 0; k < 3; ++k) a.n[k] = g->n[k];
      a.dir = d;
      a.hi = h;
      a.bc = h ? g->bc_hi[d] : g->bc_lo[d];
      a.gamma = c.gamma;
      e = tenoaa::launch_ghost_speeds(g->ndim, a, c.S, &c.S->status, c.st);
    }
  return e;
}

// Near-threshold audit of a step's sweeps (tenoaa_step_near): arrays in the
// flag layout of one right-hand side.
struct Audit {
  const uint8_t* base = nullptr;     // recorded decisions, replayed where near_in is set
  const uint8_t* near_in = nullptr;  // or null: every decision live
  uint8_t* flags_out = nullptr;      // decisions used, or null
  uint8_t* near_out = nullptr;       // 1 = within tol of a threshold (or replayed), or null
  double tol = 0.0;
};

// Face fluxes of every direction for state U; flags optional.  `stage`
// selects the Dirichlet value set.  With `audit` the audit sweep runs instead
// (flags and frozen are then taken from it).
int sweeps(const Ctx& c, const double* U, bool limit, uint8_t* flags, const uint8_t* frozen = nullptr,
           int only_dir = -1, double* fh_out = nullptr, int stage = 0, double* theta_out = nullptr,
           const Audit* audit = nullptr, bool pencil_major = false) {
  const tenoaa_grid* g = c.g;
  const int nv = g->ndim + 2;
  int64_t flag_off = 0;
  for (int d = 0; d < g->ndim; ++d) {
    if (only_dir >= 0 && d != only_dir) {
      flag_off += (int64_t)nv * 2 * faces_total(g, d);
      continue;
    }
    tenoaa::SweepArgs a{};
    a.U = U;
    a.F = reinterpret_cast<double*>(c.ws + c.L.fbuf[d]);
    // with only_dir set, flags/frozen point at that direction's own array
    const int64_t fo = only_dir >= 0 ? 0 : flag_off;
    a.flags = flags ? flags + fo : nullptr;
    a.frozen = frozen ? frozen + fo : nullptr;
    a.fh_out = fh_out;
    a.theta_out = theta_out;
    a.rec_pencil_major = pencil_major ? 1 : 0;
    for (int k = 0; k < 3; ++k) a.n[k] = g->n[k];
    a.nf = faces_along(g, d);
    a.nft = faces_total(g, d);
    a.bc_lo = g->bc_lo[d];
    a.bc_hi = g->bc_hi[d];
    a.bcv[0] = face_values(g, c.s->order, d, 0, stage);
    a.bcv[1] = face_values(g, c.s->order, d, 1, stage);
    a.splitting = c.s->splitting;
    a.gamma = c.gamma;
    a.mu = c.S->mu;
    a.status = &c.S->status;
    if (audit) {
      a.frozen = audit->base ? audit->base + fo : nullptr;
      a.flags = audit->flags_out ? audit->flags_out + fo : nullptr;
      a.near_in = audit->near_in ? audit->near_in + fo : nullptr;
      a.near_out = audit->near_out ? audit->near_out + fo : nullptr;
      a.near_tol = audit->tol;
    }
    hipError_t e = timed(TENOAA_KCLASS_SWEEP_X + d, c.st, [&] {
      return audit ? tenoaa::launch_sweep_audit(c.s->order, g->ndim, d, a, limit, c.st)
                   : tenoaa::launch_sweep(c.s->order, g->ndim, d, a, limit, c.st);
    });
    if (e != hipSuccess) return hip_fail(e);
    flag_off += (int64_t)nv * 2 * a.nft;
  }
  return TENOAA_OK;
}

int update(const Ctx& c, int mode, const double* Un, const double* Us, double* out) {
  const tenoaa_grid* g = c.g;
  tenoaa::UpdateArgs a{};
  for (int d = 0; d < 3; ++d) {
    a.F[d] = reinterpret_cast<const double*>(c.ws + c.L.fbuf[d]);
    a.nft[d] = d < g->ndim ? faces_total(g, d) : 0;
    a.nf[d] = d < g->ndim ? faces_along(g, d) : 1;
    a.n[d] = g->n[d];
    a.dx[d] = g->dx[d];
    a.rdx[d] = 1.0 / g->dx[d];
  }
  a.Un = Un;
  a.Us = Us;
  a.out = out;
  a.dt = &c.S->dt;
  hipError_t e = timed(TENOAA_KCLASS_UPDATE, c.st, [&] { return tenoaa::launch_update(g->ndim, mode, a, c.st); });
  return e == hipSuccess ? TENOAA_OK : hip_fail(e);
}

// Forward sweeps of U in every direction that also leave the decisions and
// per-field fluxes (and with `limit` the limiter factors) of adjoint stage
// slot `st` in the workspace.  With `frozen` (a flag array in the layout of
// tenoaa_rhs) the sweeps replay those decisions instead of taking them.
int recorded_sweeps(const Ctx& c, const double* U, int st, const uint8_t* frozen, bool limit = false) {
  int64_t off = 0;
  for (int d = 0; d < c.g->ndim; ++d) {
    uint8_t* flags = reinterpret_cast<uint8_t*>(c.ws + c.L.vjp[st][d]);
    double* fh = reinterpret_cast<double*>(c.ws + c.L.vjp[st][d] + c.L.vjp_fh_rel[d]);
    double* th = limit ? reinterpret_cast<double*>(c.ws + c.L.vjp[st][d] + c.L.vjp_th_rel[d]) : nullptr;
    int rc = sweeps(c, U, limit, flags, frozen ? frozen + off : nullptr, d, fh, st, th, nullptr, true);
    if (rc) return rc;
    off += (int64_t)(c.g->ndim + 2) * 2 * faces_total(c.g, d);
  }
  return TENOAA_OK;
}

int64_t flag_count(const tenoaa_grid* g) {
  int64_t n = 0;
  for (int d = 0; d < g->ndim; ++d) n += (int64_t)(g->ndim + 2) * 2 * faces_total(g, d);
  return n;
}

// U_bar = (d(dU/dt)/dU)^T R at U, decisions frozen at U, from the decisions
// and per-field fluxes that recorded_sweeps(U) left in stage slot `st`.
int rhs_vjp(const Ctx& c, const double* U, const double* R, double* Ubar, int st, bool limit = false,
            double* const* halo_bar = nullptr) {
  const tenoaa_grid* g = c.g;
  const int nv = g->ndim + 2;
  const int64_t ncell = g->n[0] * g->n[1] * g->n[2];
  hipError_t e = tenoaa::launch_zero(Ubar, (int64_t)nv * ncell, c.st);
  if (e != hipSuccess) return hip_fail(e);
  for (int d = 0; d < g->ndim; ++d) {
    tenoaa::AdjointArgs a{};
    a.U = U;
    a.R = R;
    a.Ubar = Ubar;
    a.flags = reinterpret_cast<const uint8_t*>(c.ws + c.L.vjp[st][d]);
    a.fh = reinterpret_cast<const double*>(c.ws + c.L.vjp[st][d] + c.L.vjp_fh_rel[d]);
    a.theta = limit ? reinterpret_cast<const double*>(c.ws + c.L.vjp[st][d] + c.L.vjp_th_rel[d]) : nullptr;
    a.nft = faces_total(g, d);
    for (int k = 0; k < 3; ++k) a.n[k] = g->n[k];
    a.nf = faces_along(g, d);
    a.bc_lo = g->bc_lo[d];
    a.bc_hi = g->bc_hi[d];
    a.bcv[0] = face_values(g, c.s->order, d, 0, st);
    a.bcv[1] = face_values(g, c.s->order, d, 1, st);
    for (int h = 0; h < 2; ++h)
      a.hbar[h] = (halo_bar && (h ? g->bc_hi[d] : g->bc_lo[d]) == TENOAA_BC_HALO) ? halo_bar[2 * d + h] : nullptr;
    a.splitting = c.s->splitting;
    a.gamma = c.gamma;
    a.dx = g->dx[d];
    e = timed(TENOAA_KCLASS_VJP_X + d, c.st, [&] { return tenoaa::launch_sweep_vjp(c.s->order, g->ndim, d, a, c.st); });
    if (e != hipSuccess) return hip_fail(e);
  }
  return TENOAA_OK;
}

int prepare(Ctx& c, const tenoaa_grid* g, const tenoaa_scheme* s, double gamma, void* ws, size_t ws_bytes,
            void* stream, int which) {
  if (!valid_grid(g, s) || !(gamma > 1.0) || !ws) return TENOAA_EINVAL;
  if (((uintptr_t)ws & 255) != 0) return TENOAA_EINVAL;
  c.g = g;
  c.s = s;
  c.gamma = gamma;
  c.ws = static_cast<char*>(ws);
  c.L = layout(g, which, s->positivity != 0);
  if (ws_bytes < c.L.total) return TENOAA_EWORKSPACE;
  c.S = reinterpret_cast<tenoaa::Scalars*>(c.ws + c.L.scalars);
  c.st = static_cast<hipStream_t>(stream);
  return TENOAA_OK;
}

// First device work of an entry point, after every argument check passed.
int begin(const Ctx&) { return TENOAA_OK; }

// The three stages of a step from Un with the speeds, dt and limiter weights
// already in c.S: the sweeps of each stage record (or, with flags3, replay)
// their decisions, per-field fluxes and limiter factors into the adjoint
// slots; U1 -> S1, U2 -> S2; with Unp1 non-null also stage 3 -> Unp1 (the
// arithmetic of tenoaa_step, so the result is the same bit for bit).
int recorded_stages(const Ctx& c, const double* Un, double* S1, double* S2, const uint8_t* flags3, double* Unp1,
                    bool limit) {
  const int64_t nfl = flag_count(c.g);
  auto stage_flags = [&](int st) { return flags3 ? flags3 + st * nfl : nullptr; };
  int rc;
  if ((rc = recorded_sweeps(c, Un, 0, stage_flags(0), limit))) return rc;
  if ((rc = update(c, 1, Un, nullptr, S1))) return rc;
  if ((rc = recorded_sweeps(c, S1, 1, stage_flags(1), limit))) return rc;
  if ((rc = update(c, 2, Un, S1, S2))) return rc;
  if ((rc = recorded_sweeps(c, S2, 2, stage_flags(2), limit))) return rc;
  return Unp1 ? update(c, 3, Un, S2, Unp1) : TENOAA_OK;
}

// The reverse of the three stages from what recorded_stages left (S1, S2 and
// the adjoint slots): Un_bar = (d U^{n+1} / d Un)^T Unp1_bar.  Scratch: the
// workspace's V and B2 slots and B1 (which may be the S2 slot: it is written
// after the stage-3 reverse sweep has read S2).
int reverse_stages(const Ctx& c, const double* Un, const double* S1, const double* S2, const double* dt_dev,
                   const double* Unp1_bar, double* Un_bar, double* B1, bool limit) {
  const int64_t N = (int64_t)(c.g->ndim + 2) * c.g->n[0] * c.g->n[1] * c.g->n[2];
  double* V = reinterpret_cast<double*>(c.ws + c.L.stage + 2 * c.L.state_bytes);
  double* B2 = reinterpret_cast<double*>(c.ws + c.L.stage + 3 * c.L.state_bytes);
  int rc;
  hipError_t e;
  // B2 = 2/3 B3 + 2/3 dt J(U2)^T B3
  if ((rc = rhs_vjp(c, S2, Unp1_bar, V, 2, limit))) return rc;
  if ((e = tenoaa::launch_axpdtz(B2, 2.0 / 3.0, Unp1_bar, 2.0 / 3.0, dt_dev, V, N, c.st)) != hipSuccess) return hip_fail(e);
  // B1 = 1/4 B2 + 1/4 dt J(U1)^T B2
  if ((rc = rhs_vjp(c, S1, B2, V, 1, limit))) return rc;
  if ((e = tenoaa::launch_axpdtz(B1, 0.25, B2, 0.25, dt_dev, V, N, c.st)) != hipSuccess) return hip_fail(e);
  // Bn = 1/3 B3 + 3/4 B2 + B1 + dt J(Un)^T B1
  if ((rc = rhs_vjp(c, Un, B1, V, 0, limit))) return rc;
  if ((e = tenoaa::launch_axpbypcz(Un_bar, 1.0 / 3.0, Unp1_bar, 0.75, B2, 1.0, B1, N, c.st)) != hipSuccess)
    return hip_fail(e);
  if ((e = tenoaa::launch_axpdtz(Un_bar, 1.0, Un_bar, 1.0, dt_dev, V, N, c.st)) != hipSuccess) return hip_fail(e);
  return TENOAA_OK;
}

// One right-hand side (tenoaa_rhs after its argument checks).
int rhs_body(const Ctx& c, const double* U, double* dUdt, double dt_limiter, uint8_t* flags) {
  const tenoaa_grid* grid = c.g;
  const bool limit = c.s->positivity && dt_limiter > 0.0;
  if (limit) {
    hipError_t e = timed(TENOAA_KCLASS_WAVESPEED, c.st, [&] {
      hipError_t r = wave_speeds(c, U);
      if (r == hipSuccess) r = tenoaa::launch_finalize_dt(c.S, grid->ndim, grid->dx, 1.0, nullptr, dt_limiter, c.st);
      return r;
    });
    if (e != hipSuccess) return hip_fail(e);
  }
  int rc = sweeps(c, U, limit, flags);
  if (rc) return rc;
  return update(c, 0, nullptr, nullptr, dUdt);
}

// The device address of `scratch` on each GPU, from hipGetSymbolAddress with
// that GPU current (kept after the first call on it).
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch[SCRATCH_DEVICES] = {};

int scratch_of_current_device(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= SCRATCH_DEVICES) return TENOAA_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!p || ((uintptr_t)p & 255) != 0) return TENOAA_EUNSUPPORTED;
    g_scratch[dev] = static_cast<char*>(p);
  }
  *out = g_scratch[dev];
  return TENOAA_OK;
}

__global__ void clear_scalars_kernel(tenoaa::Scalars* S) {
  if (threadIdx.x == 0) {
    S->amax_bits[0] = S->amax_bits[1] = S->amax_bits[2] = 0ull;
    S->status = 0;
  }
}

__global__ void status_out_kernel(const tenoaa::Scalars* S, int32_t* out) {
  if (threadIdx.x == 0) *out = S->status ? 1 : 0;
}

}  // namespace

namespace tenoaa {
bool grid_ok(const tenoaa_grid* g, const tenoaa_scheme* s) { return valid_grid(g, s); }
bool has_boundary_values(const tenoaa_grid* g) { return boundary_values_any(g); }
bool has_halo(const tenoaa_grid* g) {
  for (int d = 0; d < g->ndim; ++d)
    if (g->bc_lo[d] == TENOAA_BC_HALO || g->bc_hi[d] == TENOAA_BC_HALO) return true;
  return false;
}
void record_hip_error(hipError_t e) { g_last_hip_error = (int)e; }
}  // namespace tenoaa

extern "C" {

size_t tenoaa_workspace_bytes(const tenoaa_grid* grid, const tenoaa_scheme* scheme, int32_t which) {
  if (!valid_grid(grid, scheme)) return 0;
  if (which < TENOAA_WS_RHS || which > TENOAA_WS_STEP_TAPE) return 0;
  return layout(grid, which, scheme->positivity != 0).total;
}

int tenoaa_rhs(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U, double* dUdt,
               double dt_limiter, uint8_t* flags, void* ws, size_t ws_bytes, void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_RHS);
  if (rc) return rc;
  if (!U || !dUdt || U == dUdt) return TENOAA_EINVAL;
  if ((rc = begin(c))) return rc;
  return rhs_body(c, U, dUdt, dt_limiter, flags);
}

int tenoaa_rhs_noalloc(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U,
                       double* dUdt, double dt_limiter, uint8_t* flags, int32_t* status_dev, void* stream) {
  if (!valid_grid(grid, scheme) || !(gamma > 1.0)) return TENOAA_EINVAL;
  if (!U || !dUdt || U == dUdt) return TENOAA_EINVAL;
  if (layout(grid, TENOAA_WS_RHS, scheme->positivity != 0).total > (size_t)TENOAA_SCRATCH_BYTES)
    return TENOAA_EWORKSPACE;
  char* ws = nullptr;
  int rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  Ctx c;
  if ((rc = prepare(c, grid, scheme, gamma, ws, (size_t)TENOAA_SCRATCH_BYTES, stream, TENOAA_WS_RHS))) return rc;
  struct Untimed {
    Untimed() { g_untimed = true; }
    ~Untimed() { g_untimed = false; }
  } untimed;
  // this call's status and wave speeds start from zero (a kernel, not a
  // memset, so that the call can be captured in a graph)
  hipLaunchKernelGGL(clear_scalars_kernel, dim3(1), dim3(64), 0, c.st, c.S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  if ((rc = rhs_body(c, U, dUdt, dt_limiter, flags))) return rc;
  if (status_dev) {
    hipLaunchKernelGGL(status_out_kernel, dim3(1), dim3(64), 0, c.st, (const tenoaa::Scalars*)c.S, status_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
  }
  return TENOAA_OK;
}

int tenoaa_step(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl, double* U,
                double* dt_dev, void* ws, size_t ws_bytes, void* stream) {
  return tenoaa_step_flags(grid, scheme, gamma, cfl, U, dt_dev, nullptr, TENOAA_FLAGS_NONE, ws, ws_bytes, stream);
}

int tenoaa_step_flags(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl, double* U,
                      double* dt_dev, uint8_t* flags3, int32_t mode, void* ws, size_t ws_bytes, void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_STEP);
  if (rc) return rc;
  if (!U || !dt_dev) return TENOAA_EINVAL;
  if (!(cfl > 0.0) || cfl > 1.0) return TENOAA_EINVAL;
  if (scheme->positivity && cfl > 0.5) return TENOAA_EINVAL;
  if (mode < TENOAA_FLAGS_NONE || mode > TENOAA_FLAGS_REPLAY) return TENOAA_EINVAL;
  if (mode != TENOAA_FLAGS_NONE && !flags3) return TENOAA_EINVAL;
  if ((rc = begin(c))) return rc;
  const int64_t ncell = grid->n[0] * grid->n[1] * grid->n[2];
  double* Us = reinterpret_cast<double*>(c.ws + c.L.stage);
  int64_t nfl = 0;
  for (int d = 0; d < grid->ndim; ++d) nfl += (int64_t)(grid->ndim + 2) * 2 * faces_total(grid, d);
  auto rec = [&](int st) { return mode == TENOAA_FLAGS_RECORD ? flags3 + st * nfl : nullptr; };
  auto rep = [&](int st) { return mode == TENOAA_FLAGS_REPLAY ? (const uint8_t*)flags3 + st * nfl : nullptr; };
  const bool limit = scheme->positivity != 0;
  hipError_t e = timed(TENOAA_KCLASS_WAVESPEED, c.st, [&] {
    hipError_t r = wave_speeds(c, U);
    if (r == hipSuccess) r = tenoaa::launch_finalize_dt(c.S, grid->ndim, grid->dx, cfl, dt_dev, 0.0, c.st);
    return r;
  });
  if (e != hipSuccess) return hip_fail(e);
  // stage 1: U1 = Un + dt L(Un)            -> Us
  if ((rc = sweeps(c, U, limit, rec(0), rep(0), -1, nullptr, 0))) return rc;
  if ((rc = update(c, 1, U, nullptr, Us))) return rc;
  // stage 2: U2 = 3/4 Un + 1/4 U1 + 1/4 dt L(U1)   -> Us (in place)
  if ((rc = sweeps(c, Us, limit, rec(1), rep(1), -1, nullptr, 1))) return rc;
  if ((rc = update(c, 2, U, Us, Us))) return rc;
  // stage 3: U = 1/3 Un + 2/3 U2 + 2/3 dt L(U2)    -> U (in place)
  if ((rc = sweeps(c, Us, limit, rec(2), rep(2), -1, nullptr, 2))) return rc;
  return update(c, 3, U, Us, U);
}

int tenoaa_step_near(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl, double* U,
                     double* dt_dev, const uint8_t* base3, const uint8_t* near_in3, uint8_t* flags_out3,
                     uint8_t* near_out3, double near_tol, void* ws, size_t ws_bytes, void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_STEP);
  if (rc) return rc;
  if (!U || !dt_dev) return TENOAA_EINVAL;
  if (!(cfl > 0.0) || cfl > 1.0) return TENOAA_EINVAL;
  if (scheme->positivity && cfl > 0.5) return TENOAA_EINVAL;
  if (!(near_tol > 0.0) || !(near_tol < 1.0)) return TENOAA_EINVAL;
  if (near_in3 && !base3) return TENOAA_EINVAL;
  if (scheme->splitting == TENOAA_ROE) return TENOAA_EUNSUPPORTED;
  if ((rc = begin(c))) return rc;
  double* Us = reinterpret_cast<double*>(c.ws + c.L.stage);
  const int64_t nfl = flag_count(grid);
  auto audit = [&](int st) {
    Audit a;
    a.base = base3 ? base3 + st * nfl : nullptr;
    a.near_in = near_in3 ? near_in3 + st * nfl : nullptr;
    a.flags_out = flags_out3 ? flags_out3 + st * nfl : nullptr;
    a.near_out = near_out3 ? near_out3 + st * nfl : nullptr;
    a.tol = near_tol;
    return a;
  };
  const bool limit = scheme->positivity != 0;
  hipError_t e = timed(TENOAA_KCLASS_WAVESPEED, c.st, [&] {
    hipError_t r = wave_speeds(c, U);
    if (r == hipSuccess) r = tenoaa::launch_finalize_dt(c.S, grid->ndim, grid->dx, cfl, dt_dev, 0.0, c.st);
    return r;
  });
  if (e != hipSuccess) return hip_fail(e);
  const Audit a0 = audit(0), a1 = audit(1), a2 = audit(2);
  if ((rc = sweeps(c, U, limit, nullptr, nullptr, -1, nullptr, 0, nullptr, &a0))) return rc;
  if ((rc = update(c, 1, U, nullptr, Us))) return rc;
  if ((rc = sweeps(c, Us, limit, nullptr, nullptr, -1, nullptr, 1, nullptr, &a1))) return rc;
  if ((rc = update(c, 2, U, Us, Us))) return rc;
  if ((rc = sweeps(c, Us, limit, nullptr, nullptr, -1, nullptr, 2, nullptr, &a2))) return rc;
  return update(c, 3, U, Us, U);
}

int tenoaa_rhs_vjp(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U,
                   const double* dUdt_bar, double* U_bar, const uint8_t* flags, void* ws, size_t ws_bytes,
                   void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_RHS_VJP);
  if (rc) return rc;
  if (!U || !dUdt_bar || !U_bar || U_bar == U || U_bar == dUdt_bar) return TENOAA_EINVAL;
  if (tenoaa::has_halo(grid)) return TENOAA_EUNSUPPORTED;
  if ((rc = begin(c))) return rc;
  if ((rc = recorded_sweeps(c, U, 0, flags))) return rc;
  return rhs_vjp(c, U, dUdt_bar, U_bar, 0);
}

int tenoaa_rhs_vjp_halo(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U,
                        const double* dUdt_bar, double* U_bar, const uint8_t* flags, double* const* halo_bar,
                        void* ws, size_t ws_bytes, void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_RHS_VJP);
  if (rc) return rc;
  if (!U || !dUdt_bar || !U_bar || U_bar == U || U_bar == dUdt_bar || !halo_bar) return TENOAA_EINVAL;
  const int64_t G = scheme->order / 2, nv = grid->ndim + 2;
  for (int d = 0; d < grid->ndim; ++d)
    for (int h = 0; h < 2; ++h)
      if ((h ? grid->bc_hi[d] : grid->bc_lo[d]) == TENOAA_BC_HALO && !halo_bar[2 * d + h]) return TENOAA_EINVAL;
  if ((rc = begin(c))) return rc;
  for (int d = 0; d < grid->ndim; ++d)
    for (int h = 0; h < 2; ++h) {
      if ((h ? grid->bc_hi[d] : grid->bc_lo[d]) != TENOAA_BC_HALO) continue;
      int64_t plane = 1;
      for (int k = 0; k < 3; ++k)
        if (k != d) plane *= grid->n[k];
      const hipError_t e = tenoaa::launch_zero(halo_bar[2 * d + h], G * nv * plane, c.st);
      if (e != hipSuccess) return hip_fail(e);
    }
  if ((rc = recorded_sweeps(c, U, 0, flags))) return rc;
  return rhs_vjp(c, U, dUdt_bar, U_bar, 0, false, halo_bar);
}

int tenoaa_step_vjp(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* Un,
                    const double* dt_dev, const double* Unp1_bar, double* Un_bar, const uint8_t* flags3, void* ws,
                    size_t ws_bytes, void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_STEP_VJP);
  if (rc) return rc;
  if (!Un || !dt_dev || !Unp1_bar || !Un_bar || Un_bar == Unp1_bar || Un_bar == Un) return TENOAA_EINVAL;
  if (tenoaa::has_halo(grid)) return TENOAA_EUNSUPPORTED;
  const bool limit = scheme->positivity != 0;
  if ((rc = begin(c))) return rc;
  double* S1 = reinterpret_cast<double*>(c.ws + c.L.stage);
  double* S2 = reinterpret_cast<double*>(c.ws + c.L.stage + c.L.state_bytes);
  hipError_t e;
  // recompute the stages, recording each stage's decisions and per-field
  // fluxes: U1 = Un + dt L(Un), U2 = 3/4 Un + 1/4 U1 + 1/4 dt L(U1), and the
  // sweeps of U2
  if (limit) {
    // the limiter factors of every stage from the wave speeds of Un (and of the
    // ghost cells of prescribed sides) and the given dt, as in the forward step
    e = wave_speeds(c, Un);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(copy_dt_kernel, dim3(1), dim3(64), 0, c.st, c.S, dt_dev);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = tenoaa::launch_finalize_dt(c.S, grid->ndim, grid->dx, 1.0, &c.S->dt, 0.0, c.st);
  } else {
    hipLaunchKernelGGL(copy_dt_kernel, dim3(1), dim3(64), 0, c.st, c.S, dt_dev);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(e);
  if ((rc = recorded_stages(c, Un, S1, S2, flags3, nullptr, limit))) return rc;
  // the second stage state's slot holds B1 once the stage-3 reverse sweep has read it
  return reverse_stages(c, Un, S1, S2, dt_dev, Unp1_bar, Un_bar, S2, limit);
}

int tenoaa_step_tape(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl,
                     const double* Un, double* dt_dev, double* Unp1, void* ws, size_t ws_bytes, void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_STEP_TAPE);
  if (rc) return rc;
  if (!Un || !dt_dev || !Unp1 || Unp1 == Un) return TENOAA_EINVAL;
  if (!(cfl > 0.0) || cfl > 1.0) return TENOAA_EINVAL;
  if (scheme->positivity && cfl > 0.5) return TENOAA_EINVAL;
  if (tenoaa::has_halo(grid)) return TENOAA_EUNSUPPORTED;
  const bool limit = scheme->positivity != 0;
  if ((rc = begin(c))) return rc;
  double* S1 = reinterpret_cast<double*>(c.ws + c.L.stage);
  double* S2 = reinterpret_cast<double*>(c.ws + c.L.stage + c.L.state_bytes);
  // the speeds, dt and limiter weights as tenoaa_step takes them
  hipError_t e = timed(TENOAA_KCLASS_WAVESPEED, c.st, [&] {
    hipError_t r = wave_speeds(c, Un);
    if (r == hipSuccess) r = tenoaa::launch_finalize_dt(c.S, grid->ndim, grid->dx, cfl, dt_dev, 0.0, c.st);
    return r;
  });
  if (e != hipSuccess) return hip_fail(e);
  return recorded_stages(c, Un, S1, S2, nullptr, Unp1, limit);
}

int tenoaa_step_vjp_tape(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* Un,
                         const double* dt_dev, const double* Unp1_bar, double* Un_bar, void* ws, size_t ws_bytes,
                         void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_STEP_TAPE);
  if (rc) return rc;
  if (!Un || !dt_dev || !Unp1_bar || !Un_bar || Un_bar == Unp1_bar || Un_bar == Un) return TENOAA_EINVAL;
  if (tenoaa::has_halo(grid)) return TENOAA_EUNSUPPORTED;
  if ((rc = begin(c))) return rc;
  double* S1 = reinterpret_cast<double*>(c.ws + c.L.stage);
  double* S2 = reinterpret_cast<double*>(c.ws + c.L.stage + c.L.state_bytes);
  double* B1 = reinterpret_cast<double*>(c.ws + c.L.stage + 4 * c.L.state_bytes);
  return reverse_stages(c, Un, S1, S2, dt_dev, Unp1_bar, Un_bar, B1, scheme->positivity != 0);
}

int tenoaa_wave_speeds(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, const double* U,
                       double* amax_dev, void* ws, size_t ws_bytes, void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_RHS);
  if (rc) return rc;
  if (!U || !amax_dev) return TENOAA_EINVAL;
  if ((rc = begin(c))) return rc;
  hipError_t e = timed(TENOAA_KCLASS_WAVESPEED, c.st, [&] { return wave_speeds(c, U); });
  if (e == hipSuccess) e = tenoaa::launch_speeds_out(c.S, grid->ndim, amax_dev, c.st);
  return e == hipSuccess ? TENOAA_OK : hip_fail(e);
}

int tenoaa_rk3_stage(const tenoaa_grid* grid, const tenoaa_scheme* scheme, double gamma, double cfl, int32_t stage,
                     const double* amax_dev, double* dt_dev, const double* Un, const double* Us, double* out,
                     void* ws, size_t ws_bytes, void* stream) {
  Ctx c;
  int rc = prepare(c, grid, scheme, gamma, ws, ws_bytes, stream, TENOAA_WS_RHS);
  if (rc) return rc;
  if (stage < 1 || stage > 3 || !amax_dev || !dt_dev || !Un || !out || (stage > 1 && !Us)) return TENOAA_EINVAL;
  if (!(cfl > 0.0) || cfl > 1.0) return TENOAA_EINVAL;
  if (scheme->positivity && cfl > 0.5) return TENOAA_EINVAL;
  if ((rc = begin(c))) return rc;
  // the step's speeds and dt (computed from the speeds if *dt_dev <= 0), and the limiter factors
  hipError_t e = tenoaa::launch_speeds_in(c.S, grid->ndim, amax_dev, c.st);
  if (e == hipSuccess) e = tenoaa::launch_finalize_dt(c.S, grid->ndim, grid->dx, cfl, dt_dev, 0.0, c.st);
  if (e != hipSuccess) return hip_fail(e);
  const double* Ul = stage == 1 ? Un : Us;
  if ((rc = sweeps(c, Ul, scheme->positivity != 0, nullptr, nullptr, -1, nullptr, stage - 1))) return rc;
  return update(c, stage, Un, stage == 1 ? nullptr : Us, out);
}

int tenoaa_get_status(void* ws, void* stream, int32_t* out) {
  if (!ws || !out) return TENOAA_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  tenoaa::Scalars* S = reinterpret_cast<tenoaa::Scalars*>(ws);
  int v = 0;
  hipError_t e = hipMemcpyAsync(&v, &S->status, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  const int zero = 0;
  e = hipMemcpyAsync(&S->status, &zero, sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  *out = v ? 1 : 0;
  return v ? TENOAA_ENONPHYSICAL : TENOAA_OK;
}

int tenoaa_last_hip_error(void) { return g_last_hip_error; }

int tenoaa_timing_enable(int32_t on) {
  {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timing_on = on != 0;
  }
  return TENOAA_OK;
}

int tenoaa_timing_read(int32_t kclass, int64_t* launches, double* total_ms) {
  if (kclass < 0 || kclass >= TENOAA_KCLASS_COUNT || !launches || !total_ms) return TENOAA_EINVAL;
  hipError_t e = collect_timing();
  if (e != hipSuccess) return hip_fail(e);
  std::lock_guard<std::mutex> lk(g_timing_mu);
  *launches = g_launches[kclass];
  *total_ms = g_total_ms[kclass];
  g_launches[kclass] = 0;
  g_total_ms[kclass] = 0.0;
  return TENOAA_OK;
}

}  // extern "C"
