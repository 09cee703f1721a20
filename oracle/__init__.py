"""Oracle for the TENO-AA8/10 Euler right-hand side (test infrastructure only).

A plain serial FP64 CPU implementation written from the paper (arXiv
2109.14340) in ``tenoaa_oracle.cpp``; this module is its ctypes wrapper over
numpy arrays.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
GPU library.

Array layout (same as the GPU library's): conserved state U of shape
(nvar, nz, ny, nx) in C order (x fastest), nvar = ndim + 2 with components
(rho, m_x, [m_y], [m_z], E).  For ndim < 3 the unused sizes are 1.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tenoaa_oracle.cpp")
_LIB = os.path.join(_HERE, "libtenoaa_oracle.so")

BC_PERIODIC, BC_OUTFLOW, BC_SYMMETRY, BC_NOSLIP, BC_DIRICHLET, BC_INFLOW = 0, 1, 2, 3, 4, 5
LLF, RUSANOV, ROE = 0, 1, 2


def build():
    """Compile the oracle (plain C++17, no contraction) into oracle/."""
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)


class OrGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("bc_sets", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("dx", ctypes.c_double * 3),
                ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
                ("bc_values", (ctypes.c_void_p * 2) * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        gp = ctypes.POINTER(OrGrid)
        L.or_beta.restype = ctypes.c_double
        L.or_beta.argtypes = [ctypes.c_int, dp]
        L.or_teno.restype = ctypes.c_double
        L.or_teno.argtypes = [ctypes.c_int, dp, u8, dp]
        L.or_candidate_flux.restype = ctypes.c_double
        L.or_candidate_flux.argtypes = [ctypes.c_int, dp]
        L.or_wave_speeds.restype = None
        L.or_wave_speeds.argtypes = [gp, ctypes.c_double, dp, dp]
        L.or_dt.restype = ctypes.c_double
        L.or_dt.argtypes = [gp, ctypes.c_double, ctypes.c_double, dp]
        L.or_flags_size.restype = ctypes.c_int64
        L.or_flags_size.argtypes = [gp]
        L.or_rhs.restype = ctypes.c_int
        L.or_rhs.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                             dp, dp, ctypes.c_double, u8, dp]
        L.or_rhs_cells.restype = ctypes.c_int
        L.or_rhs_cells.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                   ctypes.c_double, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp]
        L.or_rhs_jvp.restype = ctypes.c_int
        L.or_rhs_jvp.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, u8, dp, dp]
        L.or_step_jvp.restype = ctypes.c_int
        L.or_step_jvp.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_double,
                                  u8, dp]
        L.or_step.restype = ctypes.c_int
        L.or_step.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, dp, dp, u8, dp]
        L.or_advect_rhs.restype = ctypes.c_int
        L.or_advect_rhs.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, dp, dp, u8]
        L.or_advect_step.restype = ctypes.c_int
        L.or_advect_step.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double, dp, u8]
        L.or_eigen.restype = None
        L.or_eigen.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, dp,
                               ctypes.POINTER(ctypes.c_int32)]
        L.or_face_fluxes.restype = ctypes.c_int
        L.or_face_fluxes.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                     ctypes.c_double, dp, dp, dp]
        L.or_limit_face.restype = None
        L.or_limit_face.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if a is not None else None


def make_grid(shape, dx, bc_lo, bc_hi=None, bc_values=None):
    """shape = (nx,) / (nx, ny) / (nx, ny, nz) in axis order; bc per axis.

    bc_values: {(d, side): array} for the Dirichlet and inflow sides (side 0
    low, 1 high).  Dirichlet: shape (sets, nvar, plane) or (nvar, plane), the
    face primitives (rho, u_x, [u_y], [u_z], p) over the face plane of
    direction d (the grid without axis d, lower remaining axis fastest).
    Inflow: shape (sets, G, nvar, plane), the primitives of the G ghost cells
    outward from the face (G = order / 2).  sets is 1 or 3 (one per SSP-RK3
    stage) and the same for every side."""
    ndim = len(shape)
    g = OrGrid()
    g.ndim = ndim
    g.bc_sets = 1
    for d in range(3):
        g.n[d] = shape[d] if d < ndim else 1
        g.dx[d] = (dx[d] if d < ndim else 1.0)
        lo = bc_lo[d] if d < ndim else 0
        hi = (bc_hi if bc_hi is not None else bc_lo)[d] if d < ndim else 0
        g.bc_lo[d] = lo
        g.bc_hi[d] = hi
    g._keep = []
    for (d, side), v in (bc_values or {}).items():
        plane = int(np.prod([g.n[k] for k in range(3) if k != d]))
        v = np.ascontiguousarray(v, dtype=np.float64)
        inflow = (g.bc_hi[d] if side else g.bc_lo[d]) == BC_INFLOW
        g.bc_sets = (v.shape[0] if v.ndim == 4 else 1) if inflow else (v.shape[0] if v.ndim == 3 else 1)
        v = v.reshape(g.bc_sets, -1, ndim + 2, plane)
        g._keep.append(v)
        g.bc_values[d][side] = v.ctypes.data
    return g


def flags_size(grid):
    return int(lib().or_flags_size(ctypes.byref(grid)))


def beta(k, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().or_beta(int(k), _dp(f))


def teno(order, fv):
    """Scalar TENO-AA flux from f_{-G+1..G}; returns (fhat, flag, margin)."""
    fv = np.ascontiguousarray(fv, dtype=np.float64)
    fl = np.zeros(1, np.uint8)
    mg = np.zeros(1, np.float64)
    h = lib().or_teno(int(order), _dp(fv), _u8(fl), _dp(mg))
    return h, int(fl[0]), float(mg[0])


def candidate_flux(k, window, i_index):
    """Candidate flux k at i+1/2 with window[i_index] = f_i."""
    w = np.ascontiguousarray(window, dtype=np.float64)
    ptr = ctypes.cast(ctypes.addressof(_dp(w).contents) + 8 * i_index, ctypes.POINTER(ctypes.c_double))
    return lib().or_candidate_flux(int(k), ptr)


def wave_speeds(grid, gamma, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    a = np.zeros(3)
    lib().or_wave_speeds(ctypes.byref(grid), gamma, _dp(U), _dp(a))
    return a


def dt(grid, gamma, cfl, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().or_dt(ctypes.byref(grid), gamma, cfl, _dp(U))


def rhs(grid, U, order=10, splitting=LLF, positivity=0, gamma=1.4, dt_lim=0.0, want_flags=True):
    """Returns (dUdt, flags, margins); flags/margins None if not wanted."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    dU = np.empty_like(U)
    nf = flags_size(grid)
    fl = np.zeros(nf, np.uint8) if want_flags else None
    mg = np.zeros(nf, np.float64) if want_flags else None
    rc = lib().or_rhs(ctypes.byref(grid), order, splitting, positivity, gamma, _dp(U), _dp(dU), dt_lim,
                      _u8(fl), _dp(mg) if mg is not None else None)
    if rc:
        raise ValueError("oracle rhs rejected its arguments (rc=%d)" % rc)
    return dU, fl, mg


def face_fluxes(grid, U, order=10, splitting=LLF, positivity=0, gamma=1.4, dt_lim=0.0):
    """Face fluxes of every direction of the right-hand side `rhs` evaluates:
    a list of (nvar, faces of d) arrays, faces in the flag arrays' order."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    nd = grid.ndim
    out = []
    for d in range(3):
        if d < nd:
            nf = grid.n[d] if grid.bc_lo[d] == BC_PERIODIC else grid.n[d] + 1
            tot = nf * int(np.prod([grid.n[k] for k in range(nd) if k != d]))
            out.append(np.zeros((nd + 2, tot)))
    ptrs = [_dp(a) for a in out] + [None] * (3 - nd)
    rc = lib().or_face_fluxes(ctypes.byref(grid), order, splitting, positivity, gamma, _dp(U), dt_lim, *ptrs)
    if rc:
        raise ValueError("oracle face_fluxes rejected its arguments (rc=%d)" % rc)
    return out


def rhs_cells(grid, U, cells, order=10, splitting=LLF, positivity=0, gamma=1.4, dt_lim=0.0, amax=None):
    """dU/dt at flat cell indices `cells` only; returns (len(cells), nvar)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    nv = grid.ndim + 2
    out = np.empty((cells.size, nv))
    am = np.ascontiguousarray(amax, dtype=np.float64) if amax is not None else None
    rc = lib().or_rhs_cells(ctypes.byref(grid), order, splitting, positivity, gamma, _dp(U), dt_lim,
                            _dp(am) if am is not None else None, cells.size,
                            cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out))
    if rc:
        raise ValueError("oracle rhs_cells rejected its arguments (rc=%d)" % rc)
    return out


def rhs_jvp(grid, U, V, flags, order=10, splitting=LLF, gamma=1.4):
    """RHS(U) and its exact directional derivative J(U) V (forward mode), decisions
    frozen to `flags`."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    out = np.empty_like(U)
    jv = np.empty_like(U)
    rc = lib().or_rhs_jvp(ctypes.byref(grid), order, splitting, gamma, _dp(U), _dp(V), _u8(flags),
                          _dp(out), _dp(jv))
    if rc:
        raise ValueError("oracle rhs_jvp rejected its arguments (rc=%d)" % rc)
    return out, jv


def step_jvp(grid, U, V, dt, flags3, order=10, splitting=LLF, gamma=1.4, positivity=0):
    """Exact derivative of one RK3 step along V (dt fixed, stage decisions frozen;
    with positivity the limiter's factors frozen too)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    flags3 = np.ascontiguousarray(flags3, dtype=np.uint8)
    out = np.empty_like(U)
    rc = lib().or_step_jvp(ctypes.byref(grid), order, splitting, positivity, gamma, _dp(U), _dp(V), dt,
                           _u8(flags3), _dp(out))
    if rc:
        raise ValueError("oracle step_jvp rejected its arguments (rc=%d)" % rc)
    return out


def step(grid, U, order=10, splitting=LLF, positivity=0, gamma=1.4, cfl=0.4, dt=0.0, want_flags=False):
    """One SSP-RK3 step; returns (U_new, dt_used, flags3, margins3)."""
    Un = np.array(U, dtype=np.float64, copy=True, order="C")
    d = np.array([dt], dtype=np.float64)
    nf = flags_size(grid)
    fl = np.zeros(3 * nf, np.uint8) if want_flags else None
    mg = np.zeros(3 * nf, np.float64) if want_flags else None
    rc = lib().or_step(ctypes.byref(grid), order, splitting, positivity, gamma, cfl, _dp(Un), _dp(d),
                       _u8(fl), _dp(mg) if mg is not None else None)
    if rc:
        raise ValueError("oracle step rejected its arguments (rc=%d)" % rc)
    return Un, float(d[0]), fl, mg


def advect_rhs(order, u, dx):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    fl = np.zeros(u.size, np.uint8)
    rc = lib().or_advect_rhs(order, u.size, dx, _dp(u), _dp(out), _u8(fl))
    if rc:
        raise ValueError("oracle advect_rhs rejected its arguments")
    return out, fl


def advect_step(order, u, dx, dt):
    """One SSP-RK3 step of periodic scalar advection; returns (u_new, flags3)."""
    out = np.array(u, dtype=np.float64, copy=True)
    fl = np.zeros(3 * out.size, np.uint8)
    rc = lib().or_advect_step(order, out.size, dx, dt, _dp(out), _u8(fl))
    if rc:
        raise ValueError("oracle advect_step rejected its arguments")
    return out, fl


def eigen(ndim, gamma, d, Wa, Wb):
    nv = ndim + 2
    Wa = np.ascontiguousarray(Wa, dtype=np.float64)
    Wb = np.ascontiguousarray(Wb, dtype=np.float64)
    L = np.zeros((nv, nv))
    R = np.zeros((nv, nv))
    lam = np.zeros(nv)
    perm = np.zeros(nv, np.int32)
    lib().or_eigen(ndim, gamma, d, _dp(Wa), _dp(Wb), _dp(L), _dp(R), _dp(lam),
                   perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return L, R, lam, perm


def limit_face(ndim, gamma, d, mu, Wa, Wb, F):
    """The positivity limiter of one face (direction d, factor mu = kappa_d
    dt/dx_d) between conserved states Wa, Wb for the high-order flux F (all in
    axis order); returns (limited flux, (theta_rho, theta_p))."""
    Wa = np.ascontiguousarray(Wa, dtype=np.float64)
    Wb = np.ascontiguousarray(Wb, dtype=np.float64)
    out = np.array(F, dtype=np.float64)
    th = np.zeros(2)
    lib().or_limit_face(int(ndim), gamma, int(d), mu, _dp(Wa), _dp(Wb), _dp(out), _dp(th))
    return out, (float(th[0]), float(th[1]))


def decode_flag(flag):
    """(large stencil chosen: 0 none / 3 / 4 / 5 / 6, (delta0, delta1, delta2), K).
    S6 (TENO12-AA only) is bits 0-1 = 3 with bit 2 set; the deltas are those of
    the fallback and (0, 0, 0) when a large stencil is chosen."""
    sel = flag & 3
    K = 7 + (flag >> 5)
    if sel == 3 and (flag & 4):
        return 6, (0, 0, 0), K
    return (sel + 2 if sel else 0), ((flag >> 2) & 1, (flag >> 3) & 1, (flag >> 4) & 1), K
