"""Seeded synthetic inputs for the TENO-AA Euler workloads.

This module holds no arithmetic of the numerical method: it only draws the
initial conserved states (with the ideal-gas equation of state of the paper's
Sec. 1, E = p/(gamma-1) + rho|u|^2/2) that both the GPU library and the CPU
oracle consume.  Every array is float64 in the library layout
(nvar, nz, ny, nx), x fastest, nvar = ndim + 2.

Workloads (cell centres at (i + 1/2) dx on the unit interval/square/cube):

* ``shock_tube_1d`` - left/right constant states (rho, u, p) drawn from
  U[0.1, 4] x U[-1, 1] x U[0.1, 4], jump at x0 ~ U[0.3, 0.7], the right state's
  density multiplied by (1 + 0.2 sin(5 pi x)) so it stays positive.
* ``batch_sizes`` / ``riemann_2d`` - the batched workload: side lengths
  n_x, n_y ~ U{64..512} independently per problem, and per problem a planar
  jump in x between two constant states drawn like the shock tube's, with a
  transverse velocity v ~ U[-1, 1] per side (outflow boundaries).
* ``grf_2d`` / ``grf_3d`` - Gaussian random fields (integer wave-vectors with
  1 <= |k| <= 32, shell-summed spectrum ~ k^-2) mapped affinely to [0.5, 2]
  for rho and p; velocity components are independent fields of the same
  type scaled so that max |u|/c = 0.5.  The 2D field carries a 10:1 pressure
  jump inside the circle |x - (1/2, 1/2)| < 0.2; the 3D field carries a blast
  sphere (centre (0.3, 0.5, 0.5), radius 0.1, p = 1e3, u = 0) and a cavity
  (centre (0.7, 0.5, 0.5), radius 0.1, rho = 1e-6, p = 1e-10, u = 0).
"""
import numpy as np

SEED_BASE = 14340


def conserved_from_primitive(rho, vel, p, gamma):
    """(rho, [u, v, w], p) arrays -> conserved array (nvar, ...) in axis order."""
    nd = len(vel)
    U = np.empty((nd + 2,) + rho.shape, dtype=np.float64)
    U[0] = rho
    ke = np.zeros_like(rho)
    for k in range(nd):
        U[1 + k] = rho * vel[k]
        ke += vel[k] * vel[k]
    U[nd + 1] = p / (gamma - 1.0) + 0.5 * rho * ke
    return U


def _as_layout(U, ndim):
    """(nvar, nx[, ny[, nz]]) axis-ordered arrays -> (nvar, nz, ny, nx)."""
    if ndim == 1:
        return np.ascontiguousarray(U[:, None, None, :])
    if ndim == 2:
        return np.ascontiguousarray(np.transpose(U, (0, 2, 1))[:, None, :, :])
    return np.ascontiguousarray(np.transpose(U, (0, 3, 2, 1)))


def cell_centres(n):
    return (np.arange(n) + 0.5) / n


def grf(rng, shape, kmax=32):
    """Real Gaussian random field on a periodic grid, spectrum E(k) ~ k^-2."""
    D = len(shape)
    ks = [np.fft.fftfreq(n, 1.0 / n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1], 1.0 / shape[-1])]
    K = np.meshgrid(*ks, indexing="ij")
    kk = np.sqrt(sum(k * k for k in K))
    amp = np.zeros_like(kk)
    sel = (kk >= 1.0) & (kk <= kmax)
    amp[sel] = kk[sel] ** (-(1.0 + D) / 2.0)
    coef = amp * (rng.standard_normal(kk.shape) + 1j * rng.standard_normal(kk.shape))
    field = np.fft.irfftn(coef, s=shape, axes=list(range(D)))
    return field


def _map(field, lo, hi):
    fmin, fmax = field.min(), field.max()
    return lo + (hi - lo) * (field - fmin) / (fmax - fmin)


def _grf_state(rng, shape, gamma):
    rho = _map(grf(rng, shape), 0.5, 2.0)
    p = _map(grf(rng, shape), 0.5, 2.0)
    vel = [grf(rng, shape) for _ in shape]
    c = np.sqrt(gamma * p / rho)
    speed = np.sqrt(sum(v * v for v in vel))
    scale = 0.5 / np.max(speed / c)
    vel = [v * scale for v in vel]
    return rho, vel, p


def shock_tube_1d(n=256, gamma=1.4, seed=SEED_BASE + 1):
    rng = np.random.default_rng(seed)
    rl, rr = rng.uniform(0.1, 4.0, 2)
    ul, ur = rng.uniform(-1.0, 1.0, 2)
    pl, pr = rng.uniform(0.1, 4.0, 2)
    x0 = rng.uniform(0.3, 0.7)
    x = cell_centres(n)
    left = x < x0
    rho = np.where(left, rl, rr * (1.0 + 0.2 * np.sin(5.0 * np.pi * x)))
    u = np.where(left, ul, ur)
    p = np.where(left, pl, pr)
    return _as_layout(conserved_from_primitive(rho, [u], p, gamma), 1)


def grf_2d(n=1024, gamma=1.4, seed=SEED_BASE + 2, jump=True):
    rng = np.random.default_rng(seed)
    rho, vel, p = _grf_state(rng, (n, n), gamma)
    if jump:
        x = cell_centres(n)
        X, Y = np.meshgrid(x, x, indexing="ij")
        inside = (X - 0.5) ** 2 + (Y - 0.5) ** 2 < 0.2 ** 2
        p = np.where(inside, 10.0 * p, p)
    return _as_layout(conserved_from_primitive(rho, vel, p, gamma), 2)


def batch_sizes(nprob=512, seed=SEED_BASE + 4, lo=64, hi=512):
    """Side lengths (n_x, n_y) of the batched workload's problems."""
    rng = np.random.default_rng(seed)
    return [(int(a), int(b)) for a, b in rng.integers(lo, hi + 1, size=(nprob, 2))]


def riemann_2d(nx, ny, index, gamma=1.4, seed=SEED_BASE + 4):
    """Problem `index` of the batched workload on an nx x ny grid."""
    rng = np.random.default_rng([seed, index])
    rl, rr = rng.uniform(0.1, 4.0, 2)
    ul, ur = rng.uniform(-1.0, 1.0, 2)
    vl, vr = rng.uniform(-1.0, 1.0, 2)
    pl, pr = rng.uniform(0.1, 4.0, 2)
    x0 = rng.uniform(0.3, 0.7)
    x = cell_centres(nx)[:, None] * np.ones((1, ny))
    left = x < x0
    rho = np.where(left, rl, rr * (1.0 + 0.2 * np.sin(5.0 * np.pi * x)))
    u = np.where(left, ul, ur)
    v = np.where(left, vl, vr)
    p = np.where(left, pl, pr)
    return _as_layout(conserved_from_primitive(rho, [u, v], p, gamma), 2)


def grf_3d(n=256, gamma=1.4, seed=SEED_BASE + 3, spheres=True):
    rng = np.random.default_rng(seed)
    rho, vel, p = _grf_state(rng, (n, n, n), gamma)
    if spheres:
        x = cell_centres(n)
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        blast = (X - 0.3) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2 < 0.1 ** 2
        cav = (X - 0.7) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2 < 0.1 ** 2
        p = np.where(blast, 1e3, p)
        p = np.where(cav, 1e-10, p)
        rho = np.where(cav, 1e-6, rho)
        for k in range(3):
            vel[k] = np.where(blast | cav, 0.0, vel[k])
    return _as_layout(conserved_from_primitive(rho, vel, p, gamma), 3)


def random_smooth(shape, gamma=1.4, seed=0, kmax=4):
    """Small smooth periodic test state of any dimension (shape in axis order)."""
    rng = np.random.default_rng(seed)
    rho, vel, p = _grf_state_k(rng, shape, gamma, kmax)
    return _as_layout(conserved_from_primitive(rho, vel, p, gamma), len(shape))


def _grf_state_k(rng, shape, gamma, kmax):
    rho = _map(grf(rng, shape, kmax), 0.5, 2.0)
    p = _map(grf(rng, shape, kmax), 0.5, 2.0)
    vel = [grf(rng, shape, kmax) for _ in shape]
    c = np.sqrt(gamma * p / rho)
    speed = np.sqrt(sum(v * v for v in vel))
    scale = 0.5 / np.max(speed / c)
    return rho, [v * scale for v in vel], p


def blast_cavity_3d(n, gamma=1.4, seed=SEED_BASE + 3):
    """The 3D workload's recipe at a reduced resolution n^3."""
    return grf_3d(n, gamma, seed, spheres=True)


def grid_shape(U):
    """(nx, ny, nz) of a layout array and its dimension count."""
    _, nz, ny, nx = U.shape
    nd = U.shape[0] - 2
    return (nx, ny, nz)[:nd], nd
