"""Python binding of libtenoaa (include/tenoaa.h): argument marshalling only.

Tensors are torch float64 tensors on the current HIP device in the library
layout (nvar, nz, ny, nx); the work is enqueued on torch's current stream.
Every step of the computation runs in the HIP library; if the library is not
built this module raises instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtenoaa.so")

BC_PERIODIC, BC_OUTFLOW, BC_SYMMETRY, BC_NOSLIP, BC_DIRICHLET, BC_INFLOW, BC_HALO = 0, 1, 2, 3, 4, 5, 6
LLF, RUSANOV, ROE = 0, 1, 2
WS_RHS, WS_STEP, WS_RHS_VJP, WS_STEP_VJP, WS_STEP_TAPE = 0, 1, 2, 3, 4
ERRORS = {-1: "EINVAL", -2: "EUNSUPPORTED", -3: "EHIP", -4: "ENONPHYSICAL", -5: "EWORKSPACE", -6: "ETIMEOUT"}

FLAGS_NONE, FLAGS_RECORD, FLAGS_REPLAY = 0, 1, 2
EXPORTS = ["tenoaa_workspace_bytes", "tenoaa_rhs", "tenoaa_step", "tenoaa_step_flags", "tenoaa_rhs_vjp", "tenoaa_step_vjp",
           "tenoaa_get_status", "tenoaa_last_hip_error", "tenoaa_timing_enable", "tenoaa_timing_read",
           "tenoaa_batch_plan_create", "tenoaa_batch_offsets", "tenoaa_batch_run", "tenoaa_batch_get_status",
           "tenoaa_batch_plan_info", "tenoaa_batch_run_stats", "tenoaa_batch_plan_destroy", "tenoaa_advect", "tenoaa_wave_speeds",
           "tenoaa_rk3_stage", "tenoaa_rhs_vjp_halo", "tenoaa_step_near", "tenoaa_rhs_noalloc",
           "tenoaa_step_tape", "tenoaa_step_vjp_tape"]
KCLASS_SWEEP = (0, 1, 2)
KCLASS_UPDATE, KCLASS_WAVESPEED = 3, 4
KCLASS_VJP = (5, 6, 7)


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("bc_sets", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("dx", ctypes.c_double * 3), ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
                ("bc_values", (ctypes.c_void_p * 2) * 3)]


class Scheme(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("splitting", ctypes.c_int32), ("positivity", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class TenoaaError(RuntimeError):
    pass


_lib = None


def load():
    """ctypes handle of libtenoaa.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TenoaaError("libtenoaa.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        gp, sp = ctypes.POINTER(Grid), ctypes.POINTER(Scheme)
        vp = ctypes.c_void_p
        L.tenoaa_workspace_bytes.restype = ctypes.c_size_t
        L.tenoaa_workspace_bytes.argtypes = [gp, sp, ctypes.c_int32]
        L.tenoaa_rhs.restype = ctypes.c_int
        L.tenoaa_rhs.argtypes = [gp, sp, ctypes.c_double, vp, vp, ctypes.c_double, vp, vp, ctypes.c_size_t, vp]
        L.tenoaa_step.restype = ctypes.c_int
        L.tenoaa_step.argtypes = [gp, sp, ctypes.c_double, ctypes.c_double, vp, vp, vp, ctypes.c_size_t, vp]
        L.tenoaa_step_flags.restype = ctypes.c_int
        L.tenoaa_step_flags.argtypes = [gp, sp, ctypes.c_double, ctypes.c_double, vp, vp, vp, ctypes.c_int32, vp,
                                        ctypes.c_size_t, vp]
        L.tenoaa_rhs_noalloc.restype = ctypes.c_int
        L.tenoaa_rhs_noalloc.argtypes = [gp, sp, ctypes.c_double, vp, vp, ctypes.c_double, vp, vp, vp]
        L.tenoaa_step_near.restype = ctypes.c_int
        L.tenoaa_step_near.argtypes = [gp, sp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, vp, vp,
                                       ctypes.c_double, vp, ctypes.c_size_t, vp]
        L.tenoaa_rhs_vjp.restype = ctypes.c_int
        L.tenoaa_rhs_vjp.argtypes = [gp, sp, ctypes.c_double, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.tenoaa_step_vjp.restype = ctypes.c_int
        L.tenoaa_step_vjp.argtypes = [gp, sp, ctypes.c_double, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.tenoaa_step_tape.restype = ctypes.c_int
        L.tenoaa_step_tape.argtypes = [gp, sp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.tenoaa_step_vjp_tape.restype = ctypes.c_int
        L.tenoaa_step_vjp_tape.argtypes = [gp, sp, ctypes.c_double, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.tenoaa_get_status.restype = ctypes.c_int
        L.tenoaa_get_status.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32)]
        L.tenoaa_last_hip_error.restype = ctypes.c_int
        L.tenoaa_last_hip_error.argtypes = []
        L.tenoaa_timing_enable.restype = ctypes.c_int
        L.tenoaa_timing_enable.argtypes = [ctypes.c_int32]
        L.tenoaa_timing_read.restype = ctypes.c_int
        L.tenoaa_timing_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double)]
        L.tenoaa_batch_plan_create.restype = ctypes.c_int
        L.tenoaa_batch_plan_create.argtypes = [gp, ctypes.c_int32, sp, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(vp)]
        L.tenoaa_batch_offsets.restype = ctypes.c_int
        L.tenoaa_batch_offsets.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.tenoaa_batch_run.restype = ctypes.c_int
        L.tenoaa_batch_run.argtypes = [vp, vp, vp, vp]
        L.tenoaa_batch_get_status.restype = ctypes.c_int
        L.tenoaa_batch_get_status.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32)]
        L.tenoaa_batch_plan_info.restype = ctypes.c_int
        L.tenoaa_batch_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
        L.tenoaa_batch_run_stats.restype = ctypes.c_int
        L.tenoaa_batch_run_stats.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
        L.tenoaa_batch_plan_destroy.restype = ctypes.c_int
        L.tenoaa_batch_plan_destroy.argtypes = [vp]
        L.tenoaa_advect.restype = ctypes.c_int
        L.tenoaa_advect.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int64, vp, vp]
        L.tenoaa_wave_speeds.restype = ctypes.c_int
        L.tenoaa_wave_speeds.argtypes = [gp, sp, ctypes.c_double, vp, vp, vp, ctypes.c_size_t, vp]
        L.tenoaa_rhs_vjp_halo.restype = ctypes.c_int
        L.tenoaa_rhs_vjp_halo.argtypes = [gp, sp, ctypes.c_double, vp, vp, vp, vp, ctypes.POINTER(vp), vp,
                                          ctypes.c_size_t, vp]
        L.tenoaa_rk3_stage.restype = ctypes.c_int
        L.tenoaa_rk3_stage.argtypes = [gp, sp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp, vp, vp, vp, vp,
                                       vp, ctypes.c_size_t, vp]
        _lib = L
    return _lib


def make_grid(shape, dx=None, bc_lo=None, bc_hi=None, bc_values=None):
    """shape = (nx,), (nx, ny) or (nx, ny, nz) in axis order; bc per axis (default periodic).

    bc_values: {(d, side): tensor} for the Dirichlet and inflow sides (side 0
    low, 1 high) as set_face_values takes them."""
    nd = len(shape)
    g = Grid()
    g.ndim = nd
    g.bc_sets = 1
    dx = dx if dx is not None else [1.0 / n for n in shape]
    bc_lo = bc_lo if bc_lo is not None else [BC_PERIODIC] * nd
    bc_hi = bc_hi if bc_hi is not None else bc_lo
    for d in range(3):
        g.n[d] = shape[d] if d < nd else 1
        g.dx[d] = dx[d] if d < nd else 1.0
        g.bc_lo[d] = bc_lo[d] if d < nd else 0
        g.bc_hi[d] = bc_hi[d] if d < nd else 0
    g._faces = {}
    for (d, side), v in (bc_values or {}).items():
        set_face_values(g, d, side, v)
    return g


def face_plane(grid, d):
    """Cells of the face plane of direction d (the grid without axis d)."""
    return int(np.prod([grid.n[k] for k in range(3) if k != d]))


def set_face_values(grid, d, side, values):
    """Binds the boundary values of side (d, side) (0 low, 1 high): a
    contiguous float64 device tensor of primitives (rho, u_x, [u_y], [u_z], p)
    over the face plane (the grid without axis d, the lower remaining axis
    fastest).  A Dirichlet side takes the face values, shape
    (sets, nvar, plane) or (nvar, plane); an inflow side the ghost cells
    r = 1 .. order/2 outward from the face, shape (sets, order/2, nvar, plane);
    a halo side the same layers as conserved states (rho, rho u_x, [rho u_y],
    [rho u_z], E): a neighbour piece's cells next to the face.
    sets is 1, or 3 for the three SSP-RK3 stages (values at t, t + dt,
    t + dt/2), and the same on every side.  The grid keeps a reference to the
    tensor; its contents may be rewritten between calls."""
    torch = _torch()
    nv = grid.ndim + 2
    plane = face_plane(grid, d)
    bc = grid.bc_hi[d] if side else grid.bc_lo[d]
    if bc not in (BC_DIRICHLET, BC_INFLOW, BC_HALO):
        raise TenoaaError("side (%d, %d) takes no boundary values" % (d, side))
    layered = bc in (BC_INFLOW, BC_HALO)
    if values.dtype != torch.float64 or not values.is_cuda or not values.is_contiguous():
        raise TenoaaError("boundary values must be a contiguous float64 device tensor")
    want_dims = 4 if layered else 3
    shape = tuple(values.shape) if values.dim() == want_dims else (1,) + tuple(values.shape)
    if len(shape) != want_dims or shape[-2:] != (nv, plane) or shape[0] not in (1, 3):
        raise TenoaaError("boundary values of side (%d, %d): shape %s, want (sets,%s %d, %d) with sets 1 or 3"
                          % (d, side, tuple(values.shape), " layers," if layered else "", nv, plane))
    sets = shape[0]
    others = [k for k in grid._faces if k != (d, side)]
    if others and grid.bc_sets != sets:
        raise TenoaaError("every side with boundary values needs the same number of value sets")
    grid._faces[(d, side)] = values
    grid._layers = getattr(grid, "_layers", {})
    grid._layers[(d, side)] = shape[1] if layered else 1
    grid.bc_sets = sets
    grid.bc_values[d][side] = values.data_ptr()


def _check_boundary_values(grid, scheme):
    """Every Dirichlet/inflow side is bound, and inflow sides hold order/2 layers."""
    faces = getattr(grid, "_faces", {})
    for d in range(grid.ndim):
        for side, bc in ((0, grid.bc_lo[d]), (1, grid.bc_hi[d])):
            if bc in (BC_DIRICHLET, BC_INFLOW, BC_HALO):
                if (d, side) not in faces:
                    raise TenoaaError("side (%d, %d) has no boundary values bound" % (d, side))
                if bc != BC_DIRICHLET and grid._layers[(d, side)] != scheme.order // 2:
                    raise TenoaaError("inflow/halo side (%d, %d) holds %d ghost layers, order %d needs %d"
                                      % (d, side, grid._layers[(d, side)], scheme.order, scheme.order // 2))


def _torch():
    import torch
    return torch


def make_scheme(order=10, splitting=LLF, positivity=0):
    s = Scheme()
    s.order, s.splitting, s.positivity = order, splitting, positivity
    return s


def flags_size(grid):
    nd = grid.ndim
    tot = 0
    for d in range(nd):
        nf = grid.n[d] if grid.bc_lo[d] == BC_PERIODIC else grid.n[d] + 1
        t = nf
        for k in range(3):
            if k != d:
                t *= grid.n[k]
        tot += (nd + 2) * 2 * t
    return tot


def _check(rc, what):
    if rc != 0:
        hip = load().tenoaa_last_hip_error()
        raise TenoaaError("%s failed: %s (hip error %d)" % (what, ERRORS.get(rc, rc), hip))


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def workspace_bytes(grid, scheme, which):
    b = load().tenoaa_workspace_bytes(ctypes.byref(grid), ctypes.byref(scheme), which)
    if b == 0:
        raise TenoaaError("invalid grid/scheme")
    return int(b)


def workspace(grid, scheme, which, device="cuda"):
    """A zero-filled device workspace (the status word starts cleared)."""
    import torch
    return torch.zeros(workspace_bytes(grid, scheme, which), dtype=torch.uint8, device=device)


def _check_state(U, grid):
    import torch
    if U.dtype != torch.float64 or not U.is_cuda or not U.is_contiguous():
        raise TenoaaError("state must be a contiguous float64 device tensor")
    want = (grid.ndim + 2, grid.n[2], grid.n[1], grid.n[0])
    if tuple(U.shape) != want:
        raise TenoaaError("state shape %s, grid wants %s" % (tuple(U.shape), want))


def rhs(grid, scheme, U, gamma=1.4, dt_limiter=0.0, flags=None, out=None, ws=None):
    """dU/dt of U (device tensors); flags: optional uint8 device tensor of flags_size(grid)."""
    import torch
    _check_state(U, grid)
    _check_boundary_values(grid, scheme)
    if out is None:
        out = torch.empty_like(U)
    if ws is None:
        ws = workspace(grid, scheme, WS_RHS, U.device)
    if flags is not None and (flags.dtype != torch.uint8 or flags.numel() < flags_size(grid)):
        raise TenoaaError("flags must be uint8 with flags_size(grid) elements")
    rc = load().tenoaa_rhs(ctypes.byref(grid), ctypes.byref(scheme), gamma, _ptr(U), _ptr(out), dt_limiter,
                           _ptr(flags), _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_rhs")
    return out


def step(grid, scheme, U, dt_dev, gamma=1.4, cfl=0.4, ws=None):
    """One SSP-RK3 step of U in place; dt_dev is a 1-element float64 device tensor."""
    _check_state(U, grid)
    _check_boundary_values(grid, scheme)
    if ws is None:
        ws = workspace(grid, scheme, WS_STEP, U.device)
    rc = load().tenoaa_step(ctypes.byref(grid), ctypes.byref(scheme), gamma, cfl, _ptr(U), _ptr(dt_dev),
                            _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_step")
    return U


def rhs_vjp(grid, scheme, U, dUdt_bar, gamma=1.4, out=None, ws=None, flags=None):
    """(d dU/dt / dU)^T dUdt_bar at U with the decisions frozen at U, or taken
    from `flags` (uint8 device tensor of flags_size(grid)) when given."""
    import torch
    _check_state(U, grid)
    _check_state(dUdt_bar, grid)
    _check_boundary_values(grid, scheme)
    if out is None:
        out = torch.empty_like(U)
    if ws is None:
        ws = workspace(grid, scheme, WS_RHS_VJP, U.device)
    if flags is not None and (flags.dtype != torch.uint8 or flags.numel() < flags_size(grid)):
        raise TenoaaError("flags must be uint8 with flags_size(grid) elements")
    rc = load().tenoaa_rhs_vjp(ctypes.byref(grid), ctypes.byref(scheme), gamma, _ptr(U), _ptr(dUdt_bar), _ptr(out),
                               _ptr(flags), _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_rhs_vjp")
    return out


def rhs_vjp_halo(grid, scheme, U, dUdt_bar, gamma=1.4, out=None, ws=None, flags=None):
    """rhs_vjp for a piece of a split grid: returns (U_bar, {(d, side):
    adjoint of that halo side's cells}), the latter shaped (order/2, nvar,
    plane) like one set of its halo values, for the neighbour piece."""
    import torch
    _check_state(U, grid)
    _check_state(dUdt_bar, grid)
    _check_boundary_values(grid, scheme)
    if out is None:
        out = torch.empty_like(U)
    if ws is None:
        ws = workspace(grid, scheme, WS_RHS_VJP, U.device)
    if flags is not None and (flags.dtype != torch.uint8 or flags.numel() < flags_size(grid)):
        raise TenoaaError("flags must be uint8 with flags_size(grid) elements")
    bars, ptrs = {}, (ctypes.c_void_p * 6)()
    for d in range(grid.ndim):
        for side, bc in ((0, grid.bc_lo[d]), (1, grid.bc_hi[d])):
            if bc == BC_HALO:
                t = torch.empty((scheme.order // 2, grid.ndim + 2, face_plane(grid, d)), dtype=torch.float64,
                                device=U.device)
                bars[(d, side)] = t
                ptrs[2 * d + side] = t.data_ptr()
    rc = load().tenoaa_rhs_vjp_halo(ctypes.byref(grid), ctypes.byref(scheme), gamma, _ptr(U), _ptr(dUdt_bar),
                                    _ptr(out), _ptr(flags), ptrs, _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_rhs_vjp_halo")
    return out, bars


def step_vjp(grid, scheme, Un, dt_dev, Unp1_bar, gamma=1.4, out=None, ws=None, flags3=None):
    """(d U^{n+1} / d U^n)^T Unp1_bar for the step of size *dt_dev from Un;
    flags3: optional recorded decisions of the three stages."""
    import torch
    _check_state(Un, grid)
    _check_state(Unp1_bar, grid)
    _check_boundary_values(grid, scheme)
    if out is None:
        out = torch.empty_like(Un)
    if ws is None:
        ws = workspace(grid, scheme, WS_STEP_VJP, Un.device)
    if flags3 is not None and (flags3.dtype != torch.uint8 or flags3.numel() < 3 * flags_size(grid)):
        raise TenoaaError("flags3 must be uint8 with 3 * flags_size(grid) elements")
    rc = load().tenoaa_step_vjp(ctypes.byref(grid), ctypes.byref(scheme), gamma, _ptr(Un), _ptr(dt_dev),
                                _ptr(Unp1_bar), _ptr(out), _ptr(flags3), _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_step_vjp")
    return out


def step_tape(grid, scheme, Un, dt_dev, gamma=1.4, cfl=0.4, out=None, ws=None):
    """One SSP-RK3 step of Un into `out` (Un kept), as tenoaa_step computes it,
    leaving its tape in `ws` (a WS_STEP_TAPE workspace) for step_vjp_tape:
    returns (out, ws)."""
    import torch
    _check_state(Un, grid)
    _check_boundary_values(grid, scheme)
    if out is None:
        out = torch.empty_like(Un)
    if ws is None:
        ws = workspace(grid, scheme, WS_STEP_TAPE, Un.device)
    rc = load().tenoaa_step_tape(ctypes.byref(grid), ctypes.byref(scheme), gamma, cfl, _ptr(Un), _ptr(dt_dev),
                                 _ptr(out), _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_step_tape")
    return out, ws


def step_vjp_tape(grid, scheme, Un, dt_dev, Unp1_bar, ws, gamma=1.4, out=None):
    """step_vjp from the tape step_tape(Un, dt_dev) left in `ws` (no
    recomputation of the stages)."""
    import torch
    _check_state(Un, grid)
    _check_state(Unp1_bar, grid)
    _check_boundary_values(grid, scheme)
    if out is None:
        out = torch.empty_like(Un)
    rc = load().tenoaa_step_vjp_tape(ctypes.byref(grid), ctypes.byref(scheme), gamma, _ptr(Un), _ptr(dt_dev),
                                     _ptr(Unp1_bar), _ptr(out), _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_step_vjp_tape")
    return out


def step_flags(grid, scheme, U, dt_dev, flags3, mode, gamma=1.4, cfl=0.4, ws=None):
    """tenoaa_step recording (mode FLAGS_RECORD) or replaying (FLAGS_REPLAY) the
    decisions of its three stages in flags3 (uint8, 3 * flags_size(grid))."""
    _check_state(U, grid)
    _check_boundary_values(grid, scheme)
    if ws is None:
        ws = workspace(grid, scheme, WS_STEP, U.device)
    rc = load().tenoaa_step_flags(ctypes.byref(grid), ctypes.byref(scheme), gamma, cfl, _ptr(U), _ptr(dt_dev),
                                  _ptr(flags3), mode, _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_step_flags")
    return U


def step_near(grid, scheme, U, dt_dev, base3=None, near_in3=None, flags_out3=None, near_out3=None, tol=1e-3,
              gamma=1.4, cfl=0.4, ws=None):
    """tenoaa_step with its decisions audited: replayed from base3 where
    near_in3 is non-zero, live elsewhere; the decisions used go to flags_out3
    and the live ones within `tol` of a threshold are marked in near_out3
    (all uint8, 3 * flags_size(grid), or None)."""
    _check_state(U, grid)
    _check_boundary_values(grid, scheme)
    nfl = 3 * flags_size(grid)
    for a in (base3, near_in3, flags_out3, near_out3):
        if a is not None and (a.dtype != _torch().uint8 or a.numel() != nfl or not a.is_contiguous()):
            raise TenoaaError("decision arrays must be contiguous uint8 of 3 x flags_size(grid)")
    if ws is None:
        ws = workspace(grid, scheme, WS_STEP, U.device)
    opt = lambda a: _ptr(a) if a is not None else None  # noqa: E731
    rc = load().tenoaa_step_near(ctypes.byref(grid), ctypes.byref(scheme), gamma, cfl, _ptr(U), _ptr(dt_dev),
                                 opt(base3), opt(near_in3), opt(flags_out3), opt(near_out3), tol, _ptr(ws),
                                 ws.numel(), _stream())
    _check(rc, "tenoaa_step_near")
    return U


def advect(order, u, dx, dt, nsteps):
    """nsteps SSP-RK3 steps of the periodic scalar advection u_t + u_x = 0 on
    the 1D float64 device tensor u, in place."""
    import torch
    if u.dtype != torch.float64 or not u.is_cuda or not u.is_contiguous() or u.dim() != 1:
        raise TenoaaError("u must be a contiguous 1D float64 device tensor")
    _check(load().tenoaa_advect(order, u.numel(), dx, dt, nsteps, _ptr(u), _stream()), "tenoaa_advect")
    return u


def wave_speeds(grid, scheme, U, gamma=1.4, out=None, ws=None):
    """a_d = max(|u_d| + c) over the cells of U and the first ghost layer of
    sides with boundary or halo values: a float64 device tensor of ndim."""
    import torch
    _check_state(U, grid)
    _check_boundary_values(grid, scheme)
    if out is None:
        out = torch.empty(grid.ndim, dtype=torch.float64, device=U.device)
    if ws is None:
        ws = workspace(grid, scheme, WS_RHS, U.device)
    rc = load().tenoaa_wave_speeds(ctypes.byref(grid), ctypes.byref(scheme), gamma, _ptr(U), _ptr(out), _ptr(ws),
                                   ws.numel(), _stream())
    _check(rc, "tenoaa_wave_speeds")
    return out


def rk3_stage(grid, scheme, stage, amax, dt_dev, Un, Us, out, gamma=1.4, cfl=0.4, ws=None):
    """Stage 1, 2 or 3 of the SSP-RK3 step into `out` (tenoaa_rk3_stage):
    amax the step's wave speeds (ndim float64 on the device), dt_dev the
    step's dt (computed from amax and cfl if it holds a value <= 0)."""
    _check_state(Un, grid)
    _check_state(out, grid)
    if Us is not None:
        _check_state(Us, grid)
    _check_boundary_values(grid, scheme)
    if ws is None:
        ws = workspace(grid, scheme, WS_RHS, Un.device)
    rc = load().tenoaa_rk3_stage(ctypes.byref(grid), ctypes.byref(scheme), gamma, cfl, stage, _ptr(amax),
                                 _ptr(dt_dev), _ptr(Un), _ptr(Us), _ptr(out), _ptr(ws), ws.numel(), _stream())
    _check(rc, "tenoaa_rk3_stage")
    return out


def get_status(ws):
    """Synchronises the current stream; 0 if every state read was physical."""
    out = ctypes.c_int32(0)
    rc = load().tenoaa_get_status(_ptr(ws), _stream(), ctypes.byref(out))
    if rc not in (0, -4):
        _check(rc, "tenoaa_get_status")
    return int(out.value)


def timing_enable(on=True):
    _check(load().tenoaa_timing_enable(1 if on else 0), "tenoaa_timing_enable")


def timing_read(kclass):
    """(launches, total_ms) of one kernel class since its last read."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(load().tenoaa_timing_read(kclass, ctypes.byref(n), ctypes.byref(ms)), "tenoaa_timing_read")
    return int(n.value), float(ms.value)


class BatchPlan:
    """A tenoaa_batch_plan: nprob independent 2D grids (tenoaa Grid structs,
    ndim 2) advanced together by `nsteps` SSP-RK3 steps per run.  Dirichlet
    and inflow sides take one value set, used by every step."""

    def __init__(self, grids, scheme, nsteps, gamma=1.4, cfl=0.4, tune_cache=None):
        L = load()
        for g in grids:
            _check_boundary_values(g, scheme)
        self._keep = [getattr(g, "_faces", {}) for g in grids]  # the boundary-value tensors stay alive
        self.nprob = len(grids)
        arr = (Grid * self.nprob)(*grids)
        self._grids = arr
        self.nsteps = nsteps
        h = ctypes.c_void_p(None)
        path = tune_cache.encode() if tune_cache else None
        rc = L.tenoaa_batch_plan_create(arr, self.nprob, ctypes.byref(scheme), gamma, cfl, nsteps, path,
                                        ctypes.byref(h))
        _check(rc, "tenoaa_batch_plan_create")
        self._h = h
        offs = (ctypes.c_int64 * (self.nprob + 1))()
        _check(L.tenoaa_batch_offsets(h, offs), "tenoaa_batch_offsets")
        self.offsets = [int(o) for o in offs]

    def info(self):
        """(blocks, blocks per CU, chunk, how chosen, x tiles per bucket, y tiles per bucket)."""
        buf = (ctypes.c_int32 * 10)()
        _check(load().tenoaa_batch_plan_info(self._h, buf, 10), "tenoaa_batch_plan_info")
        v = list(buf)
        return {"blocks": v[0], "blocks_per_cu": v[1], "chunk": v[2], "chosen": ("defaults", "tuned", "cache")[v[3]],
                "tile_x": v[4:7], "tile_y": v[7:10]}

    def run_stats(self):
        """Synchronises; where the blocks of the last run spent their resident
        time: shares waiting at phase barriers, in sweep items and in update
        and wave-speed items (the rest: taking items from the queue), the
        mean time a block was resident (s) and the mean wait per block and
        barrier (us)."""
        buf = (ctypes.c_double * 5)()
        _check(load().tenoaa_batch_run_stats(self._h, _stream(), buf, 5), "tenoaa_batch_run_stats")
        return {"barrier_wait_share": buf[0], "resident_s": buf[1], "wait_per_barrier_us": buf[2],
                "sweep_share": buf[3], "cell_share": buf[4]}

    def pack(self, states, device="cuda"):
        """Packed float64 device tensor of the problems' (4, 1, ny, nx) states."""
        import torch
        out = torch.empty(self.offsets[-1], dtype=torch.float64, device=device)
        for p, U in enumerate(states):
            t = U if isinstance(U, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(U))
            out[self.offsets[p]:self.offsets[p + 1]].copy_(t.reshape(-1))
        return out

    def unpack(self, packed, p):
        g = self._grids[p]
        return packed[self.offsets[p]:self.offsets[p + 1]].view(4, 1, g.n[1], g.n[0])

    def run(self, packed, dt_out=None):
        """Advances every problem in place on torch's current stream; dt_out:
        optional float64 device tensor of nprob * nsteps."""
        import torch
        if packed.dtype != torch.float64 or not packed.is_cuda or packed.numel() != self.offsets[-1]:
            raise TenoaaError("packed state must be float64 on the device with %d elements" % self.offsets[-1])
        if dt_out is not None and (dt_out.dtype != torch.float64 or dt_out.numel() != self.nprob * self.nsteps):
            raise TenoaaError("dt_out must be float64 with nprob * nsteps elements")
        _check(load().tenoaa_batch_run(self._h, _ptr(packed), _ptr(dt_out), _stream()), "tenoaa_batch_run")
        return packed

    def status(self):
        """Synchronises; per-problem non-physical flags (list of 0/1)."""
        out = (ctypes.c_int32 * self.nprob)()
        rc = load().tenoaa_batch_get_status(self._h, _stream(), out)
        if rc not in (0, -4):
            _check(rc, "tenoaa_batch_get_status")
        return list(out)

    def close(self):
        if getattr(self, "_h", None):
            load().tenoaa_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_cache_key(scheme, grids):
    """Key under which tenoaa_batch_plan_create files its tuned choices."""
    cnt = [0, 0, 0]
    for g in grids:
        nx = g.n[0]
        cnt[0 if nx <= 160 else (1 if nx <= 320 else 2)] += 1
    return "gfx950 order=%d split=%d limit=%d buckets=%d,%d,%d" % (scheme.order, scheme.splitting,
                                                                   scheme.positivity, *cnt)


def grid_for(U, bc=None, dx=None):
    """Grid of a layout array/tensor (nvar, nz, ny, nx)."""
    nv, nz, ny, nx = tuple(U.shape)
    nd = nv - 2
    shape = (nx, ny, nz)[:nd]
    bcs = [bc if bc is not None else BC_PERIODIC] * nd if not isinstance(bc, (list, tuple)) else list(bc)
    return make_grid(shape, dx, bcs)


def to_numpy(t):
    return np.ascontiguousarray(t.detach().cpu().numpy())
