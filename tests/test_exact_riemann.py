"""Pins of the exact Riemann solver that the shock-tube validation uses as its
reference (the paper's Sec. 5 shock tubes compare with theoretical Riemann
solutions): jump conditions across each wave, invariants through the
rarefaction, and conservation of the exact solution."""
import math

import numpy as np
import pytest

from oracle import exact_riemann as er

G = 1.4
SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))


def _flux(rho, u, p):
    E = p / (G - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)]), np.array([rho, rho * u, E])


@pytest.mark.parametrize("case", ["sod", "lax"])
def test_right_shock_rankine_hugoniot(case):
    left, right = SOD if case == "sod" else LAX
    ps, us = er.star_state(left, right, G)
    rr, ur, pr = right
    assert ps > pr  # a right-moving shock
    cr = math.sqrt(G * pr / rr)
    S = ur + cr * math.sqrt((G + 1) / (2 * G) * ps / pr + (G - 1) / (2 * G))
    # states just behind and ahead of the shock from the sampled solution
    rho, u, p = er.sample(left, right, np.array([S - 1e-9, S + 1e-9]), G)
    Fa, Ua = _flux(rho[0], u[0], p[0])
    Fb, Ub = _flux(rho[1], u[1], p[1])
    # F(behind) - F(ahead) = S (U(behind) - U(ahead))
    assert np.allclose(Fa - Fb, S * (Ua - Ub), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("case", ["sod", "lax"])
def test_left_rarefaction_invariants(case):
    left, right = SOD if case == "sod" else LAX
    ps, us = er.star_state(left, right, G)
    rl, ul, pl = left
    assert ps < pl
    cl = math.sqrt(G * pl / rl)
    cs = cl * (ps / pl) ** ((G - 1) / (2 * G))
    xi = np.linspace(ul - cl, us - cs, 41)
    rho, u, p = er.sample(left, right, xi, G)
    c = np.sqrt(G * p / rho)
    # the C+ Riemann invariant and the entropy are constant through the fan
    assert np.allclose(u + 2 * c / (G - 1), ul + 2 * cl / (G - 1), rtol=1e-12)
    assert np.allclose(p / rho ** G, pl / rl ** G, rtol=1e-12)
    # the fan is a C- characteristic fan: xi = u - c
    assert np.allclose(xi, u - c, atol=1e-12)


@pytest.mark.parametrize("case", ["sod", "lax"])
def test_contact_continuity(case):
    left, right = SOD if case == "sod" else LAX
    ps, us = er.star_state(left, right, G)
    rho, u, p = er.sample(left, right, np.array([us - 1e-9, us + 1e-9]), G)
    assert abs(p[0] - ps) <= 1e-13 * ps and abs(p[1] - ps) <= 1e-13 * ps
    assert abs(u[0] - us) <= 1e-13 and abs(u[1] - us) <= 1e-13
    assert abs(rho[0] - rho[1]) > 1e-3  # the density jumps


@pytest.mark.parametrize("case,t", [("sod", 0.2), ("lax", 0.14)])
def test_exact_solution_conserves(case, t):
    """While the waves stay inside [0, 1], the integral of U changes by
    -t (F(U_R) - F(U_L))."""
    left, right = SOD if case == "sod" else LAX
    n = 2000
    U = er.cell_averages(left, right, 0.5, t, n, G, sub=256).sum(axis=1) / n
    FL, UL = _flux(*left)
    FR, UR = _flux(*right)
    U0 = 0.5 * UL + 0.5 * UR
    assert np.allclose(U, U0 - t * (FR - FL), rtol=2e-5, atol=2e-5)


def test_equal_states_give_a_uniform_solution():
    s = (1.3, 0.4, 2.0)
    ps, us = er.star_state(s, s, G)
    assert abs(ps - 2.0) <= 1e-13 and abs(us - 0.4) <= 1e-13


def test_double_rarefaction_vacuum():
    """Sec. 5's double rarefaction opens a vacuum: the fans end at the fronts
    u_L + 2 c_L/(gamma-1) and u_R - 2 c_R/(gamma-1), with the Riemann
    invariants carried through them, and mass is conserved."""
    left, right = (1.0, -2.0, 0.1), (1.0, 2.0, 0.1)
    assert er.generates_vacuum(left, right, G)
    c = math.sqrt(G * 0.1)
    front = -2.0 + 2 * c / (G - 1)
    xi = np.linspace(-2.0 - c, front - 1e-9, 51)
    rho, u, p = er.sample(left, right, xi, G)
    cs = np.sqrt(G * p / rho)
    assert np.allclose(u + 2 * cs / (G - 1), -2.0 + 2 * c / (G - 1), rtol=1e-12)
    assert np.allclose(p / rho ** G, 0.1, rtol=1e-10)
    rho0, _, p0 = er.sample(left, right, np.array([0.0, front + 1e-9]), G)
    assert np.all(rho0 == 0.0) and np.all(p0 == 0.0)
    # mass of the exact solution on [0, 1] at t = 0.1: 1 - t (flux_R - flux_L) = 1 - 0.1 * (2 + 2)
    U = er.cell_averages(left, right, 0.5, 0.1, 2000, G, sub=256).sum(axis=1) / 2000
    assert abs(U[0] - (1.0 - 0.1 * 4.0)) <= 2e-5
