"""The taped step: tenoaa_step_tape steps like tenoaa_step bit for bit and
keeps the stage states and records, and tenoaa_step_vjp_tape, which skips
the stage recomputation, equals tenoaa_step_vjp bit for bit (the tape stays
whole across several seeds); a checkpointed trajectory's gradient with tapes
equals the recomputing one."""
import numpy as np
import pytest

from paper_2109_14340_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import adjoint, tenoaa  # noqa: E402

P, O, S, W = tenoaa.BC_PERIODIC, tenoaa.BC_OUTFLOW, tenoaa.BC_SYMMETRY, tenoaa.BC_NOSLIP


def _seed(U, s):
    return torch.randn(U.shape, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(s))


def _case(name):
    if name == "1d_outflow_llf10":
        U = inputs.shock_tube_1d(96)
        return U, tenoaa.make_grid((96,), bc_lo=[O], bc_hi=[O]), tenoaa.make_scheme(10, tenoaa.LLF, 0)
    if name == "2d_walls_rusanov8_limiter":
        U = np.ascontiguousarray(inputs.grf_2d(72, seed=inputs.SEED_BASE + 21)[:, :, :60, :])
        return U, tenoaa.make_grid((72, 60), bc_lo=[S, W], bc_hi=[O, S]), tenoaa.make_scheme(8, tenoaa.RUSANOV, 1)
    if name == "2d_periodic_roe10":
        U = inputs.grf_2d(64, seed=inputs.SEED_BASE + 22, jump=False)
        return U, tenoaa.make_grid((64, 64)), tenoaa.make_scheme(10, tenoaa.ROE, 0)
    if name == "3d_blast_cavity_llf10_limiter":
        U = inputs.blast_cavity_3d(40)
        return U, tenoaa.make_grid((40, 40, 40)), tenoaa.make_scheme(10, tenoaa.LLF, 1)
    raise KeyError(name)


CASES = ["1d_outflow_llf10", "2d_walls_rusanov8_limiter", "2d_periodic_roe10", "3d_blast_cavity_llf10_limiter"]


@pytest.mark.parametrize("case", CASES)
def test_step_tape_equals_step_and_step_vjp(case):
    Un, grid, sch = _case(case)
    U0 = torch.from_numpy(np.ascontiguousarray(Un)).cuda()
    keep = U0.clone()
    dta = torch.zeros(1, dtype=torch.float64, device="cuda")
    Ua = U0.clone()
    tenoaa.step(grid, sch, Ua, dta, cfl=0.4)
    dtb = torch.zeros(1, dtype=torch.float64, device="cuda")
    Ub, ws = tenoaa.step_tape(grid, sch, U0, dtb, cfl=0.4)
    assert torch.equal(Ub, Ua) and torch.equal(dtb, dta) and torch.equal(U0, keep)
    for s in (3, 4):
        B = _seed(U0, s)
        ga = tenoaa.step_vjp(grid, sch, U0, dta, B)
        gb = tenoaa.step_vjp_tape(grid, sch, U0, dta, B, ws)
        assert torch.isfinite(ga).all()
        assert torch.equal(gb, ga), "%s seed %d: max difference %.3e" % (case, s, float((gb - ga).abs().max()))


def test_step_tape_given_dt():
    """A positive dt on entry is used as given, as tenoaa_step does."""
    Un, grid, sch = _case("3d_blast_cavity_llf10_limiter")
    U0 = torch.from_numpy(np.ascontiguousarray(Un)).cuda()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    tenoaa.step(grid, sch, U0.clone(), dt, cfl=0.4)
    half = dt * 0.5
    Ua = U0.clone()
    da = half.clone()
    tenoaa.step(grid, sch, Ua, da, cfl=0.4)
    db = half.clone()
    Ub, ws = tenoaa.step_tape(grid, sch, U0, db, cfl=0.4)
    assert torch.equal(Ub, Ua) and torch.equal(db, half)
    B = _seed(U0, 5)
    assert torch.equal(tenoaa.step_vjp_tape(grid, sch, U0, half, B, ws), tenoaa.step_vjp(grid, sch, U0, half, B))


def test_trajectory_gradient_with_tapes_equals_recompute():
    n = 96
    U0 = torch.from_numpy(inputs.grf_2d(n, seed=inputs.SEED_BASE + 5, jump=False)).cuda()
    target = torch.from_numpy(inputs.grf_2d(n, seed=inputs.SEED_BASE + 50, jump=False)[0]).cuda()
    grid = tenoaa.make_grid((n, n))
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 0)
    g = []
    for tape in (False, True):
        x = U0.clone().requires_grad_(True)
        UT = adjoint.rk3_trajectory(x, grid, sch, 7, checkpoint_every=3, tape=tape)
        torch.sqrt(((UT[0] - target) ** 2).mean()).backward()
        g.append(x.grad.clone())
    assert torch.equal(g[0], g[1])
