"""The prescribed-value boundaries on the GPU, the Dirichlet boundary of
Appendix A and the supersonic inflow: right-hand sides and SSP-RK3 steps with
such sides, mixed with the other boundaries, against the oracle on the same
values (one value set, and three per-stage sets)."""
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

D = tenoaa.BC_DIRICHLET
I = tenoaa.BC_INFLOW  # noqa: E741


def _prims(U, gamma):
    nd = {1: 1, 2: 2, 3: 3}[U.shape[0] - 2]
    rho = U[0]
    vel = [U[1 + k] / rho for k in range(nd)]
    p = (gamma - 1.0) * (U[-1] - 0.5 * rho * sum(v * v for v in vel))
    return [rho] + vel + [p]


def _face_values(U, shape, bc_lo, bc_hi, gamma, sets, seed, order=10):
    """Boundary values near the boundary cells' own primitives (perturbed per
    set and layer), as {(d, side): (sets, nvar, plane)} for Dirichlet sides and
    (sets, order/2, nvar, plane) for inflow sides, in the face-plane order of
    the ABI.  Asserts that the Dirichlet ghosts they make are physical."""
    rng = np.random.default_rng(seed)
    nd = len(shape)
    G = order // 2
    P = _prims(U, gamma)  # each (nz, ny, nx)
    out = {}
    for d in range(nd):
        for side, bc in ((0, bc_lo[d]), (1, bc_hi[d])):
            if bc not in (D, I):
                continue
            ax = 2 - d  # array axis of direction d in (nz, ny, nx)
            idx = 0 if side == 0 else shape[d] - 1
            # plane over the remaining axes, the lower axis fastest = C order of the remaining array axes
            planes = np.stack([np.take(q, idx, axis=ax).ravel() for q in P])

            def perturbed():
                v = planes.copy()
                v[0] *= 1.0 + 0.05 * rng.uniform(-1, 1, v[0].shape)
                v[-1] *= 1.0 + 0.05 * rng.uniform(-1, 1, v[-1].shape)
                v[1:-1] += 0.05 * rng.uniform(-1, 1, v[1:-1].shape)
                return v
            if bc == D:
                vals = np.stack([perturbed() for _ in range(sets)])
                for r in range(1, G + 1):  # ghost r mirrors cell r - 1 from the face
                    m = r - 1 if side == 0 else shape[d] - r
                    mir = np.stack([np.take(q, m, axis=ax).ravel() for q in P])
                    gh = 2.0 * vals - mir[None]
                    assert gh[:, 0].min() > 0 and gh[:, -1].min() > 0, "test data: non-physical Dirichlet ghost"
            else:
                vals = np.stack([np.stack([perturbed() for _ in range(G)]) for _ in range(sets)])
            out[(d, side)] = np.ascontiguousarray(vals)
    return out


def _grids(shape, bc_lo, bc_hi, faces):
    dx = [1.0 / n for n in shape]
    g_or = oracle.make_grid(shape, dx, bc_lo, bc_hi, bc_values=faces)
    g_gpu = tenoaa.make_grid(shape, dx, bc_lo, bc_hi,
                             bc_values={k: torch.from_numpy(v).cuda() for k, v in faces.items()})
    return g_or, g_gpu


def _smooth(shape, seed, gamma=1.4):
    """A smooth state whose density and pressure vary by about +-20 % (so that
    the Dirichlet reflections 2 face - mirror stay physical)."""
    U = inputs.random_smooth(shape, seed=seed, kmax=2)
    P = _prims(U, gamma)
    rho = 1.0 + 0.3 * (P[0] - P[0].mean())
    p = 1.0 + 0.3 * (P[-1] - P[-1].mean())
    nd = len(shape)
    W = np.empty_like(U)
    W[0] = rho
    ke = np.zeros_like(rho)
    for k in range(nd):
        W[1 + k] = rho * P[1 + k]
        ke += P[1 + k] ** 2
    W[-1] = p / (gamma - 1.0) + 0.5 * rho * ke
    return W


CASES = {
    "1d": ((64,), [D], [I], lambda: inputs.shock_tube_1d(64)),
    "2d_mixed": ((37, 45), [D, tenoaa.BC_SYMMETRY], [I, D], lambda: _smooth((37, 45), 12)),
    "3d_all": ((20, 18, 16), [D, I, D], [I, D, D], lambda: _smooth((20, 18, 16), 13)),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("order,splitting,limit", [(8, 0, 0), (10, 1, 0), (10, 0, 1)])
def test_rhs_dirichlet(case, order, splitting, limit):
    shape, lo, hi, make = CASES[case]
    U = make()
    faces = _face_values(U, shape, lo, hi, 1.4, 1, seed=7, order=order)
    g_or, g_gpu = _grids(shape, lo, hi, faces)
    dt = oracle.dt(g_or, 1.4, 0.4, U) if limit else 0.0
    d_or, fl_or, mg_or = oracle.rhs(g_or, U, order=order, splitting=splitting, positivity=limit, dt_lim=dt)
    sch = tenoaa.make_scheme(order, splitting, limit)
    fl = torch.zeros(tenoaa.flags_size(g_gpu), dtype=torch.uint8, device="cuda")
    ws = tenoaa.workspace(g_gpu, sch, tenoaa.WS_RHS)
    out = tenoaa.rhs(g_gpu, sch, torch.from_numpy(U).cuda(), dt_limiter=dt, flags=fl, ws=ws)
    torch.cuda.synchronize()
    assert tenoaa.get_status(ws) == 0
    rep = compare_rhs(g_or, tenoaa.to_numpy(out), d_or, tenoaa.to_numpy(fl), fl_or, mg_or)
    print(case, order, splitting, limit, rep)


@pytest.mark.parametrize("sets", [1, 3])
def test_step_prescribed_values_per_stage_sets(sets):
    """Three steps with Dirichlet and inflow sides: the GPU state equals the
    oracle's bit for bit (stage s reads value set s when there are three)."""
    shape, lo, hi = (40, 36), [D, tenoaa.BC_NOSLIP], [I, D]
    U0 = _smooth(shape, 5)
    faces = _face_values(U0, shape, lo, hi, 1.4, sets, seed=3, order=10)
    g_or, g_gpu = _grids(shape, lo, hi, faces)
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    ws = tenoaa.workspace(g_gpu, sch, tenoaa.WS_STEP)
    U = torch.from_numpy(U0).cuda()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    Uo = U0
    for _ in range(3):
        dt.zero_()
        tenoaa.step(g_gpu, sch, U, dt, ws=ws)
        Uo, dto, _, _ = oracle.step(g_or, Uo, order=10, splitting=0, positivity=1, cfl=0.4)
        assert float(dt.item()) == dto
    assert tenoaa.get_status(ws) == 0
    assert np.array_equal(U.cpu().numpy(), Uo)


def test_inflow_layers_must_match_the_order():
    shape = (24, 20)
    U = _smooth(shape, 2)
    faces = _face_values(U, shape, [I, 1], [I, 1], 1.4, 1, seed=1, order=8)
    _, g = _grids(shape, [I, 1], [I, 1], faces)
    with pytest.raises(tenoaa.TenoaaError, match="ghost layers"):
        tenoaa.rhs(g, tenoaa.make_scheme(10), torch.from_numpy(U).cuda())


def test_stage_entry_points_equal_the_step():
    """tenoaa_wave_speeds + tenoaa_rk3_stage 1, 2, 3 (stage s reading value set
    s of three) give tenoaa_step's state and dt bit for bit, with the limiter,
    on a grid with Dirichlet, inflow and wall sides."""
    shape, lo, hi = (40, 36), [D, tenoaa.BC_NOSLIP], [I, D]
    U0 = _smooth(shape, 6)
    faces = _face_values(U0, shape, lo, hi, 1.4, 3, seed=8, order=10)
    _, g = _grids(shape, lo, hi, faces)
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    Uw = torch.from_numpy(U0).cuda()
    dtw = torch.zeros(1, dtype=torch.float64, device="cuda")
    tenoaa.step(g, sch, Uw, dtw)
    Un = torch.from_numpy(U0).cuda()
    ws = tenoaa.workspace(g, sch, tenoaa.WS_RHS)
    amax = tenoaa.wave_speeds(g, sch, Un, ws=ws).clone()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    Us = torch.empty_like(Un)
    tenoaa.rk3_stage(g, sch, 1, amax, dt, Un, None, Us, ws=ws)
    tenoaa.rk3_stage(g, sch, 2, amax, dt, Un, Us, Us, ws=ws)
    tenoaa.rk3_stage(g, sch, 3, amax, dt, Un, Us, Un, ws=ws)
    torch.cuda.synchronize()
    assert tenoaa.get_status(ws) == 0
    assert float(dt.item()) == float(dtw.item())
    assert torch.equal(Un, Uw)
