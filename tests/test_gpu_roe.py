"""The Roe flux with entropy fix (Sec. 5.2's face flux for the blast waves
and the Rayleigh-Taylor runs) on the GPU: right-hand sides against the oracle
in 1D/2D/3D, with and without the limiter; the Woodward-Colella blast waves
(N = 400, t = 0.038, reflective walls) stepped bit for bit as the oracle does,
conserving mass and energy; and the batched form with this flux."""
import numpy as np
import pytest

import oracle
from paper_2109_14340_amd import inputs
from tests.parity import compare_rhs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import tenoaa  # noqa: E402

ROE = tenoaa.ROE


def _rhs_case(U, shape, bc_lo, bc_hi, order, limit):
    dx = [1.0 / n for n in shape]
    g_or = oracle.make_grid(shape, dx, bc_lo, bc_hi)
    g = tenoaa.make_grid(shape, dx, bc_lo, bc_hi)
    dt = oracle.dt(g_or, 1.4, 0.4, U) if limit else 0.0
    d_or, fl_or, mg_or = oracle.rhs(g_or, U, order=order, splitting=ROE, positivity=limit, dt_lim=dt)
    sch = tenoaa.make_scheme(order, ROE, limit)
    fl = torch.zeros(tenoaa.flags_size(g), dtype=torch.uint8, device="cuda")
    ws = tenoaa.workspace(g, sch, tenoaa.WS_RHS)
    out = tenoaa.rhs(g, sch, torch.from_numpy(np.ascontiguousarray(U)).cuda(), dt_limiter=dt, flags=fl, ws=ws)
    torch.cuda.synchronize()
    assert tenoaa.get_status(ws) == 0
    rep = compare_rhs(g_or, tenoaa.to_numpy(out), d_or, tenoaa.to_numpy(fl), fl_or, mg_or)
    print(shape, order, limit, rep)


@pytest.mark.parametrize("order,limit", [(8, 0), (10, 0), (10, 1)])
def test_roe_rhs_1d_shock_tube(order, limit):
    _rhs_case(inputs.shock_tube_1d(64), (64,), [1], [1], order, limit)


@pytest.mark.parametrize("order", [8, 10])
def test_roe_rhs_2d_ragged_walls(order):
    U = np.ascontiguousarray(inputs.grf_2d(72, seed=12)[:, :, :45, :37])
    _rhs_case(U, (37, 45), [tenoaa.BC_SYMMETRY, tenoaa.BC_NOSLIP], [tenoaa.BC_OUTFLOW, tenoaa.BC_SYMMETRY],
              order, 0)


@pytest.mark.parametrize("order,limit", [(10, 1), (8, 0)])
def test_roe_rhs_3d_blast_cavity(order, limit):
    _rhs_case(inputs.blast_cavity_3d(20), (20, 20, 20), [0] * 3, [0] * 3, order, limit)


def _blast_init(n, gamma=1.4):
    x = (np.arange(n) + 0.5) / n
    p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
    return inputs._as_layout(inputs.conserved_from_primitive(np.ones(n), [np.zeros(n)], p, gamma), 1)


@pytest.mark.parametrize("order", [8, 10])
def test_woodward_colella_blast_waves(order):
    """Sec. 5.2: (rho, u, p) = (1, 0, 1000 | 0.01 | 100) split at 0.1 and 0.9,
    reflective walls, N = 400, t = 0.038, Roe flux with entropy fix; the
    positivity limiter keeps the collision of the two blast waves physical
    (without it the oracle's state turns non-physical near t = 0.0273 with
    every one of the three fluxes)."""
    n, tf = 400, 0.038
    U0 = _blast_init(n)
    g = tenoaa.make_grid((n,), bc_lo=[tenoaa.BC_SYMMETRY])
    g_or = oracle.make_grid((n,), [1.0 / n], [oracle.BC_SYMMETRY])
    sch = tenoaa.make_scheme(order, ROE, 1)
    ws = tenoaa.workspace(g, sch, tenoaa.WS_STEP)
    U = torch.from_numpy(U0).cuda()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    Uo, t, k = U0, 0.0, 0
    while t < tf - 1e-15:
        h = min(oracle.dt(g_or, 1.4, 0.4, Uo), tf - t)
        dt.fill_(h)
        tenoaa.step(g, sch, U, dt, ws=ws)
        Uo, _, _, _ = oracle.step(g_or, Uo, order=order, splitting=ROE, positivity=1, dt=h)
        t += h
        k += 1
    assert tenoaa.get_status(ws) == 0
    Ug = U.cpu().numpy()
    assert np.array_equal(Ug, Uo), "GPU and oracle differ after %d steps" % k
    rho = Ug[0, 0, 0]
    p = 0.4 * (Ug[2, 0, 0] - 0.5 * Ug[1, 0, 0] ** 2 / rho)
    assert rho.min() > 0 and p.min() > 0
    # reflective walls: mass and energy are conserved
    assert abs(rho.sum() / n - 1.0) <= 1e-12
    e0 = U0[2, 0, 0].sum() / n
    assert abs(Ug[2, 0, 0].sum() / n - e0) <= 1e-12 * e0
    x = (np.arange(n) + 0.5) / n
    print("order", order, "steps", k, "density peak %.3f at x = %.4f" % (rho.max(), x[rho.argmax()]))
    # the paper's figure: the density peak near x = 0.78
    assert 5.5 < rho.max() < 7.0 and 0.76 < x[rho.argmax()] < 0.80


def test_roe_batched_equals_per_problem():
    sch = tenoaa.make_scheme(10, ROE, 1)
    sizes = [(64, 72), (150, 64), (96, 130)]
    out = [tenoaa.BC_OUTFLOW] * 2
    grids = [tenoaa.make_grid(s, bc_lo=out, bc_hi=out) for s in sizes]
    states = [inputs.riemann_2d(nx, ny, p) for p, (nx, ny) in enumerate(sizes)]
    plan = tenoaa.BatchPlan(grids, sch, 3)
    packed = plan.pack(states)
    dtb = torch.zeros(len(grids) * 3, dtype=torch.float64, device="cuda")
    plan.run(packed, dtb)
    assert plan.status() == [0] * 3
    for p, (g, U0) in enumerate(zip(grids, states)):
        U = torch.from_numpy(U0).cuda()
        ws = tenoaa.workspace(g, sch, tenoaa.WS_STEP)
        dt = torch.zeros(3, dtype=torch.float64, device="cuda")
        for s in range(3):
            tenoaa.step(g, sch, U, dt[s:s + 1], ws=ws)
        assert torch.equal(dtb.view(3, 3)[p], dt)
        assert torch.equal(plan.unpack(packed, p), U)
