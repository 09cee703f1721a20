"""Pins of the oracle's Roe flux with entropy fix (the face flux of the
paper's Sec. 5.2 blast-wave and Rayleigh-Taylor runs): per characteristic
field, where the eigenvalue has one strict sign at both cells of a face the
unsplit characteristic flux is reconstructed from the upwind side alone;
elsewhere the field falls back to the LLF split.

* Supersonic smooth flow: every eigenvalue has the flow's sign and every
  reconstruction takes the largest stencil, so, since R L = I at each face,
  the flux is the upwind linear scheme applied to the physical flux component
  by component: the right-hand side equals -(lin(F)_{i+1/2} - lin(F)_{i-1/2})/dx
  with the stencil mirrored for flow to the left (a downwind choice, a split
  or a dropped back-projection term each break it).
* The side not reconstructed records flag 0, which no real decision has.
* A constant state is steady, the periodic cell sums of dU/dt vanish, and the
  scheme is mirror-symmetric (x -> -x, u -> -u) across sonic points.
"""
import numpy as np
import pytest

import oracle
from paper_2109_14340_amd import inputs

G_ = 1.4


def _state_1d(n, u0):
    x = (np.arange(n) + 0.5) / n
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * x)
    u = u0 + 0.1 * np.cos(2 * np.pi * x)
    p = 1.0 + 0.1 * np.sin(4 * np.pi * x)
    return rho, u, p


def _flux_1d(rho, u, p):
    E = p / (G_ - 1.0) + 0.5 * rho * u * u
    return np.stack([rho * u, rho * u * u + p, u * (E + p)])


@pytest.mark.parametrize("order", [8, 10])
@pytest.mark.parametrize("u0", [3.0, -3.0])
def test_supersonic_flow_is_upwind_linear_scheme_of_the_flux(order, u0):
    n = 64
    G = order // 2
    big = 5 if order == 10 else 4  # the largest candidate stencil
    rho, u, p = _state_1d(n, u0)
    U = inputs._as_layout(inputs.conserved_from_primitive(rho, [u], p, G_), 1)
    g = oracle.make_grid((n,), [1.0 / n], [oracle.BC_PERIODIC])
    dU, fl, _ = oracle.rhs(g, U, order=order, splitting=oracle.ROE, gamma=G_)
    F = _flux_1d(rho, u, p)
    Fh = np.empty((3, n))  # F at face i+1/2
    for c in range(3):
        ext = np.concatenate([F[c, -G:], F[c], F[c, :G]])  # periodic extension, ext[i + G] = F_i
        for i in range(n):
            if u0 > 0:
                Fh[c, i] = oracle.candidate_flux(big, ext, i + G)
            else:  # mirrored: the "f_i" slot holds F_{i+1}, the stencil reversed
                rev = ext[i + 1: i + 2 * G + 1][::-1].copy()
                Fh[c, i] = oracle.candidate_flux(big, rev, G - 1)
    want = -(Fh - np.roll(Fh, 1, axis=1)) * n
    got = dU[:, 0, 0]
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()
    # flags: [field][side][face]; the upwind side took the largest stencil, the other none
    f = fl.reshape(3, 2, n)
    up, down = (0, 1) if u0 > 0 else (1, 0)
    assert np.all(f[:, up] & 3 == (3 if order == 10 else 2))
    assert np.all(f[:, down] == 0)
    # LLF differs (it adds dissipation)
    dL, _, _ = oracle.rhs(g, U, order=order, splitting=oracle.LLF, gamma=G_)
    assert np.abs(dL - dU).max() > 1e-6 * np.abs(want).max()


def test_constant_state_is_steady_and_periodic_sums_vanish():
    n = (14, 12)
    U = inputs._as_layout(inputs.conserved_from_primitive(np.full(n, 1.3), [np.full(n, 0.2), np.full(n, -0.4)],
                                                          np.full(n, 0.9), G_), 2)
    g = oracle.make_grid(n, [1.0 / 14, 1.0 / 12], [oracle.BC_PERIODIC] * 2)
    dU, _, _ = oracle.rhs(g, U, order=10, splitting=oracle.ROE, gamma=G_)
    assert np.all(dU == 0.0)
    V = inputs.random_smooth((24, 20), seed=3, kmax=3)
    g2 = oracle.make_grid((24, 20), [1.0 / 24, 1.0 / 20], [oracle.BC_PERIODIC] * 2)
    d2, _, _ = oracle.rhs(g2, V, order=10, splitting=oracle.ROE, gamma=G_)
    assert np.abs(d2.sum(axis=(1, 2, 3))).max() <= 1e-12 * np.abs(d2).max() * d2[0].size


@pytest.mark.parametrize("order", [8, 10])
def test_mirror_symmetry_across_sonic_points(order):
    """u changes sign (the entropy field's eigenvalue is sonic at two faces):
    mirroring the data mirrors the right-hand side."""
    n = 80
    x = (np.arange(n) + 0.5) / n
    rho = 1.0 + 0.3 * np.exp(-40 * (x - 0.4) ** 2)
    u = 0.8 * np.sin(2 * np.pi * x) + 0.1
    p = 1.0 + 0.5 * (x > 0.55)
    U = inputs._as_layout(inputs.conserved_from_primitive(rho, [u], p, G_), 1)
    Um = inputs._as_layout(inputs.conserved_from_primitive(rho[::-1].copy(), [-u[::-1]], p[::-1].copy(), G_), 1)
    g = oracle.make_grid((n,), [1.0 / n], [oracle.BC_PERIODIC])
    d, fl, _ = oracle.rhs(g, U, order=order, splitting=oracle.ROE, gamma=G_)
    dm, _, _ = oracle.rhs(g, Um, order=order, splitting=oracle.ROE, gamma=G_)
    mir = dm[:, 0, 0, ::-1].copy()
    mir[1] = -mir[1]
    assert np.abs(d[:, 0, 0] - mir).max() <= 1e-11 * np.abs(d).max()
    f = fl.reshape(3, 2, n)
    # the entropy field (1) is split at the sonic faces and one-sided elsewhere; the acoustic fields one-sided
    split = (f[1, 0] != 0) & (f[1, 1] != 0)
    assert 1 <= split.sum() <= 4
    assert np.all((f[0, 0] == 0) & (f[0, 1] != 0)) and np.all((f[2, 0] != 0) & (f[2, 1] == 0))


@pytest.mark.parametrize("order", [8, 10])
def test_replayed_decisions_replay_the_side(order):
    """Recorded decisions fix the side each field reconstructs as well: the
    decisions of supersonic flow to the right (every field one-sided from the
    left, largest stencil), replayed on a subsonic state whose own decisions
    take the left-going acoustic field from the right, give the upwind linear
    scheme of the subsonic state's physical flux from the left (R L = I at
    each face); the state's own decisions replay to its own right-hand side
    bit for bit."""
    n = 32
    G = order // 2
    big = 5 if order == 10 else 4
    g = oracle.make_grid((n,), [1.0 / n], [oracle.BC_PERIODIC])
    rho, u, p = _state_1d(n, 3.0)
    UA = inputs._as_layout(inputs.conserved_from_primitive(rho, [u], p, G_), 1)
    _, flA, _ = oracle.rhs(g, UA, order=order, splitting=oracle.ROE, gamma=G_)
    assert np.all(flA.reshape(3, 2, n)[:, 1] == 0)
    rho, u, p = _state_1d(n, 0.3)
    UB = inputs._as_layout(inputs.conserved_from_primitive(rho, [u], p, G_), 1)
    dB, flB, _ = oracle.rhs(g, UB, order=order, splitting=oracle.ROE, gamma=G_)
    fB = flB.reshape(3, 2, n)
    assert np.all((fB[0, 0] == 0) & (fB[0, 1] != 0))  # u - c < 0: from the right at this state
    again, _ = oracle.rhs_jvp(g, UB, np.zeros_like(UB), flB, order=order, splitting=oracle.ROE, gamma=G_)
    assert np.array_equal(again, dB)
    got, _ = oracle.rhs_jvp(g, UB, np.zeros_like(UB), flA, order=order, splitting=oracle.ROE, gamma=G_)
    F = _flux_1d(rho, u, p)
    Fh = np.empty((3, n))
    for c in range(3):
        ext = np.concatenate([F[c, -G:], F[c], F[c, :G]])
        for i in range(n):
            Fh[c, i] = oracle.candidate_flux(big, ext, i + G)
    want = -(Fh - np.roll(Fh, 1, axis=1)) * n
    assert np.abs(got[:, 0, 0] - want).max() <= 1e-11 * np.abs(want).max()
    # the state's own choice (field 0 from the right) gives a different result
    assert np.abs(dB[:, 0, 0] - want).max() > 1e-9 * np.abs(want).max()
