"""Exact solution of the Riemann problem of the 1D Euler equations for an
ideal gas: TEST INFRASTRUCTURE ONLY (the reference for the shock-tube
validation cases of the paper's Sec. 5, whose figures compare with the
theoretical Riemann solutions).  Only tests/ may import it.

The solution is self-similar in xi = (x - x0)/t.  When the two rarefactions
cannot meet (2 (c_L + c_R) / (gamma - 1) <= u_R - u_L) a vacuum opens between
their fronts u_L + 2 c_L / (gamma - 1) and u_R - 2 c_R / (gamma - 1).
Otherwise the star pressure p* solves
f_L(p*) + f_R(p*) + (u_R - u_L) = 0, where f_K is the velocity jump across the
K wave: a shock (Rankine-Hugoniot) when p* > p_K, a rarefaction (isentropic,
Riemann invariant) otherwise.  Newton's method on p with a positive starting
value converges because f_L + f_R is monotone and concave in p.
"""
import math

import numpy as np


def _wave_f(p, rho, pk, ck, g):
    """Velocity jump across a wave from state (rho, pk, ck) to pressure p, and
    its derivative with respect to p."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    r = (p / pk) ** ((g - 1.0) / (2.0 * g))
    return 2.0 * ck / (g - 1.0) * (r - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rho * ck)


def star_state(left, right, g=1.4, tol=1e-14, maxit=100):
    """(p*, u*) of the Riemann problem with primitive states left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("the states generate vacuum")
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(maxit):
        fl, dl = _wave_f(p, rl, pl, cl, g)
        fr, dr = _wave_f(p, rr, pr, cr, g)
        step = (fl + fr + ur - ul) / (dl + dr)
        pn = p - step
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _wave_f(p, rl, pl, cl, g)
    fr, _ = _wave_f(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def _sample_vacuum(left, right, xi, g):
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    rho = np.zeros_like(xi)
    u = np.zeros_like(xi)
    p = np.zeros_like(xi)
    sl, sr = ul + 2.0 * cl / (g - 1.0), ur - 2.0 * cr / (g - 1.0)
    # left state, left fan up to the vacuum front
    a = xi < ul - cl
    rho[a], u[a], p[a] = rl, ul, pl
    f = (xi >= ul - cl) & (xi < sl)
    uf = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + xi[f])
    cf = uf - xi[f]
    rho[f] = rl * (cf / cl) ** (2.0 / (g - 1.0))
    p[f] = pl * (cf / cl) ** (2.0 * g / (g - 1.0))
    u[f] = uf
    # right fan from the vacuum front, right state
    f = (xi > sr) & (xi <= ur + cr)
    uf = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + xi[f])
    cf = xi[f] - uf
    rho[f] = rr * (cf / cr) ** (2.0 / (g - 1.0))
    p[f] = pr * (cf / cr) ** (2.0 * g / (g - 1.0))
    u[f] = uf
    b = xi > ur + cr
    rho[b], u[b], p[b] = rr, ur, pr
    return rho, u, p


def generates_vacuum(left, right, g=1.4):
    cl, cr = math.sqrt(g * left[2] / left[0]), math.sqrt(g * right[2] / right[0])
    return 2.0 * (cl + cr) / (g - 1.0) <= right[1] - left[1]


def sample(left, right, xi, g=1.4):
    """Primitive (rho, u, p) arrays of the exact solution at xi = (x - x0)/t
    (zero density and pressure, and u = 0, in a vacuum)."""
    rl, ul, pl = left
    rr, ur, pr = right
    if generates_vacuum(left, right, g):
        return _sample_vacuum(left, right, np.asarray(xi, dtype=np.float64), g)
    ps, us = star_state(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for side, (rk, uk, pk), sgn in (("L", left, -1.0), ("R", right, 1.0)):
        ck = math.sqrt(g * pk / rk)
        sel = (xi < us) if side == "L" else (xi >= us)
        x = xi[sel]
        if ps > pk:  # shock of speed S
            S = uk + sgn * ck * math.sqrt((g + 1.0) / (2.0 * g) * ps / pk + (g - 1.0) / (2.0 * g))
            rs = rk * (ps / pk + gm) / (gm * ps / pk + 1.0)
            outside = (x < S) if side == "L" else (x >= S)
            rho[sel] = np.where(outside, rk, rs)
            u[sel] = np.where(outside, uk, us)
            p[sel] = np.where(outside, pk, ps)
        else:  # rarefaction: head, tail, fan
            rs = rk * (ps / pk) ** (1.0 / g)
            cs = ck * (ps / pk) ** ((g - 1.0) / (2.0 * g))
            head = uk + sgn * ck
            tail = us + sgn * cs
            if side == "L":
                outside, star = x < head, x > tail
            else:
                outside, star = x > head, x < tail
            fan_u = 2.0 / (g + 1.0) * (-sgn * ck + (g - 1.0) / 2.0 * uk + x)
            fan_c = -sgn * (fan_u - x)
            fan_c = np.maximum(fan_c, 0.0)
            fan_rho = rk * (fan_c / ck) ** (2.0 / (g - 1.0))
            fan_p = pk * (fan_c / ck) ** (2.0 * g / (g - 1.0))
            rho[sel] = np.where(outside, rk, np.where(star, rs, fan_rho))
            u[sel] = np.where(outside, uk, np.where(star, us, fan_u))
            p[sel] = np.where(outside, pk, np.where(star, ps, fan_p))
    return rho, u, p


def cell_averages(left, right, x0, t, n, g=1.4, sub=64):
    """Conserved cell averages (rho, m, E) of the exact solution at time t on
    [0, 1] with n cells, each averaged over `sub` equally spaced samples."""
    x = (np.arange(n * sub) + 0.5) / (n * sub)
    rho, u, p = sample(left, right, (x - x0) / t, g)
    E = p / (g - 1.0) + 0.5 * rho * u * u
    U = np.stack([rho, rho * u, E]).reshape(3, n, sub).mean(axis=2)
    return U
