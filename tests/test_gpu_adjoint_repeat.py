"""The adjoint entry points give the same result bit for bit from run to run
(every sum of the reverse sweep in a fixed order), over the boundary kinds,
tile counts and remainders that decide that order; and the 3D 256^3 step
adjoint at full size against the oracle's step derivative at probe cells."""
import numpy as np
import pytest

from paper_2109_14340_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import tenoaa  # noqa: E402

P, O, S, W = tenoaa.BC_PERIODIC, tenoaa.BC_OUTFLOW, tenoaa.BC_SYMMETRY, tenoaa.BC_NOSLIP


def _seed(U, s):
    return torch.randn(U.shape, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(s))


def _state(shape, seed):
    """A random-field state of the given (nx[, ny[, nz]]) shape."""
    n = max(shape)
    if len(shape) == 1:
        U = inputs.shock_tube_1d(n, seed=seed)
    elif len(shape) == 2:
        U = inputs.grf_2d(n, seed=seed, jump=False)[:, :, :shape[1], :shape[0]]
    else:
        U = inputs.grf_3d(n, seed=seed, spheres=False)[:, :shape[2], :shape[1], :shape[0]]
    return torch.from_numpy(np.ascontiguousarray(U)).cuda()


# (shape, low sides, high sides): periodic directions whose last 64-face tile
# is short (conflicts through the wrap), odd and even tile counts, the tails
# of non-periodic directions (n + 1 faces), wall and outflow ghosts, and a
# periodic direction shorter than a tile's window
CASES = {
    "1d_periodic_200": ((200,), [P], [P]),
    "1d_outflow_130": ((130,), [O], [O]),
    "2d_walls_131x70": ((131, 70), [S, W], [O, S]),
    "2d_periodic_200x12": ((200, 12), [P, P], [P, P]),
    "3d_mixed_67x65x40": ((67, 65, 40), [P, O, S], [P, O, W]),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("order", [8, 10])
def test_rhs_vjp_bitwise_repeatable(case, order):
    shape, lo, hi = CASES[case]
    U = _state(shape, 31)
    R = _seed(U, 7)
    grid = tenoaa.make_grid(shape, bc_lo=lo, bc_hi=hi)
    sch = tenoaa.make_scheme(order, tenoaa.LLF, 0)
    first = tenoaa.rhs_vjp(grid, sch, U, R)
    assert torch.isfinite(first).all() and float(first.abs().max()) > 0.0
    for _ in range(3):
        assert torch.equal(tenoaa.rhs_vjp(grid, sch, U, R), first)


@pytest.mark.parametrize("splitting", [tenoaa.RUSANOV, tenoaa.ROE])
def test_rhs_vjp_bitwise_repeatable_other_splittings(splitting):
    shape, lo, hi = CASES["2d_walls_131x70"]
    U = _state(shape, 32)
    R = _seed(U, 8)
    grid = tenoaa.make_grid(shape, bc_lo=lo, bc_hi=hi)
    sch = tenoaa.make_scheme(10, splitting, 0)
    first = tenoaa.rhs_vjp(grid, sch, U, R)
    for _ in range(3):
        assert torch.equal(tenoaa.rhs_vjp(grid, sch, U, R), first)


def test_step_vjp_bitwise_repeatable_limiter():
    """The 3D blast-and-cavity recipe at 64^3 with the limiter acting."""
    U = torch.from_numpy(inputs.blast_cavity_3d(64)).cuda()
    grid = tenoaa.make_grid((64, 64, 64))
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    tenoaa.step(grid, sch, U.clone(), dt, cfl=0.4)
    B = _seed(U, 9)
    first = tenoaa.step_vjp(grid, sch, U, dt, B)
    for _ in range(2):
        assert torch.equal(tenoaa.step_vjp(grid, sch, U, dt, B), first)


def test_rhs_vjp_halo_bitwise_repeatable():
    """A piece of a grid split along y, its halo sides' adjoints included."""
    n, G, lo, hi = 40, 5, 9, 31
    U = _state((n, n), 33)
    R = _seed(U, 10)
    halos = {}
    for side in (0, 1):
        layers = [U[:, :, ((lo - r) % n) if side == 0 else ((hi - 1 + r) % n), :].reshape(4, -1)
                  for r in range(1, G + 1)]
        halos[(1, side)] = torch.stack(layers)[None].contiguous()
    grid = tenoaa.make_grid((n, hi - lo), [1.0 / n] * 2, [P, tenoaa.BC_HALO], [P, tenoaa.BC_HALO], bc_values=halos)
    Up = U[:, :, lo:hi, :].contiguous()
    Rp = R[:, :, lo:hi, :].contiguous()
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 0)
    own, bars = tenoaa.rhs_vjp_halo(grid, sch, Up, Rp)
    own, bars = own.clone(), {k: v.clone() for k, v in bars.items()}
    for _ in range(2):
        o2, b2 = tenoaa.rhs_vjp_halo(grid, sch, Up, Rp)
        assert torch.equal(o2, own)
        assert all(torch.equal(b2[k], bars[k]) for k in bars)


def test_step_vjp_3d_256_headline_repeatable():
    """The full-size 256^3 step adjoint of the headline state (blast and
    cavity spheres, limiter on): twice the same bits."""
    U = torch.from_numpy(inputs.grf_3d(256)).cuda()
    grid = tenoaa.make_grid((256, 256, 256))
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    U1 = U.clone()
    tenoaa.step(grid, sch, U1, dt, cfl=0.4)
    B = _seed(U, 11)
    ws = tenoaa.workspace(grid, sch, tenoaa.WS_STEP_VJP, "cuda")
    first = tenoaa.step_vjp(grid, sch, U, dt, B, ws=ws)
    assert torch.isfinite(first).all()
    again = tenoaa.step_vjp(grid, sch, U, dt, B, ws=ws)
    assert torch.equal(again, first)


def test_step_vjp_3d_256_probes_against_oracle():
    """The full-size 256^3 step adjoint of the headline state (limiter on) at
    probe cells away from the spheres: the row of the step Jacobian that
    tenoaa_step_vjp gives for a one-hot seed, against the oracle's exact step
    derivative (dual numbers, decisions frozen) on a 35^3 box around the probe
    taken out of the same state with the same dt.  One step reaches 3 x 5
    cells, so the box's outflow sides do not reach the probe; away from the
    spheres the limiter leaves every face alone in both runs."""
    import oracle
    n, R = 256, 17
    Un = inputs.grf_3d(n)
    U = torch.from_numpy(Un).cuda()
    grid = tenoaa.make_grid((n, n, n))
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    tenoaa.step(grid, sch, U.clone(), dt, cfl=0.4)
    dtv = float(dt.item())
    ws = tenoaa.workspace(grid, sch, tenoaa.WS_STEP_VJP, "cuda")
    rng = np.random.default_rng(2109)
    og = oracle.make_grid((2 * R + 1,) * 3, [1.0 / n] * 3, [tenoaa.BC_OUTFLOW] * 3)
    for (i, j, k, q) in [(128, 25, 30, 0), (20, 230, 200, 3), (240, 128, 20, 4)]:
        E = torch.zeros_like(U)
        E[q, k, j, i] = 1.0
        g = tenoaa.step_vjp(grid, sch, U, dt, E, ws=ws)
        ii, jj, kk = [(c + np.arange(-R, R + 1)) % n for c in (i, j, k)]
        ix = np.ix_(np.arange(5), kk, jj, ii)
        gbox = g.cpu().numpy()[ix]
        # nothing of the row lies outside the box
        assert int((g != 0).sum()) == int((gbox != 0).sum()) > 0
        box = np.ascontiguousarray(Un[ix])
        _, dto, fl3, _ = oracle.step(og, box, order=10, splitting=0, positivity=1, dt=dtv, want_flags=True)
        assert dto == dtv
        V = rng.standard_normal(box.shape) * np.abs(box).reshape(5, -1).max(axis=1)[:, None, None, None]
        jv = oracle.step_jvp(og, box, V, dtv, fl3, order=10, splitting=0, positivity=1)
        lhs = float(jv[q, R, R, R])
        rhs = float(np.sum(gbox * V))
        ref = float(np.sum(np.abs(gbox * V)))
        print("probe", (i, j, k, q), "oracle (J V)_c %.15e  <S^T e_c, V> %.15e  rel %.2e"
              % (lhs, rhs, abs(lhs - rhs) / ref))
        assert abs(lhs - rhs) <= 1e-11 * ref


def test_rhs_vjp_bitwise_repeatable_prescribed_sides():
    """Dirichlet ghosts fold into their mirror cells through the reflection
    rule's Jacobian (the general kernel variant); inflow ghosts add nothing."""
    from tests.test_gpu_dirichlet import _face_values, _smooth
    D, I = tenoaa.BC_DIRICHLET, tenoaa.BC_INFLOW
    shape, lo, hi = (37, 45), [D, S], [I, D]
    U = _smooth(shape, 12)
    faces = _face_values(U, shape, lo, hi, 1.4, 1, seed=21, order=10)
    grid = tenoaa.make_grid(shape, [1.0 / n for n in shape], lo, hi,
                            bc_values={k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in faces.items()})
    Ud = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    R = _seed(Ud, 14)
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 0)
    first = tenoaa.rhs_vjp(grid, sch, Ud, R)
    for _ in range(3):
        assert torch.equal(tenoaa.rhs_vjp(grid, sch, Ud, R), first)
