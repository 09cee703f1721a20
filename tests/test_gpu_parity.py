"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Small cases compare every face decision and every element; the full-size
workloads compare sampled cells, which the oracle evaluates one by one, and
properties that hold at any size.
"""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pair(shape, bc_lo, bc_hi=None):
    dx = [1.0 / n for n in shape]
    g_or = oracle.make_grid(shape, dx, bc_lo, bc_hi)
    g_gpu = tenoaa.make_grid(shape, dx, bc_lo, bc_hi)
    return g_or, g_gpu


def _run_rhs(U, shape, bc_lo, bc_hi=None, order=10, splitting=0, positivity=0, dt_lim=0.0, gamma=1.4):
    g_or, g_gpu = _pair(shape, bc_lo, bc_hi)
    d_or, fl_or, mg_or = oracle.rhs(g_or, U, order=order, splitting=splitting, positivity=positivity,
                                    gamma=gamma, dt_lim=dt_lim)
    sch = tenoaa.make_scheme(order, splitting, positivity)
    Ud = _dev(U)
    fl = torch.zeros(tenoaa.flags_size(g_gpu), dtype=torch.uint8, device="cuda")
    ws = tenoaa.workspace(g_gpu, sch, tenoaa.WS_RHS)
    out = tenoaa.rhs(g_gpu, sch, Ud, gamma=gamma, dt_limiter=dt_lim, flags=fl, ws=ws)
    torch.cuda.synchronize()
    assert tenoaa.get_status(ws) == 0
    rep = compare_rhs(g_or, tenoaa.to_numpy(out), d_or, tenoaa.to_numpy(fl), fl_or, mg_or)
    print(shape, order, splitting, positivity, rep, flush=True)
    return rep


@pytest.mark.parametrize("order", [8, 10])
@pytest.mark.parametrize("splitting", [0, 1])
@pytest.mark.parametrize("limit", [0, 1])
def test_rhs_1d_shock_tube(order, splitting, limit):
    U = inputs.shock_tube_1d(64)
    dt = 0.0
    if limit:
        g = oracle.make_grid((64,), [1 / 64.0], [1])
        dt = oracle.dt(g, 1.4, 0.4, U)
    _run_rhs(U, (64,), [1], order=order, splitting=splitting, positivity=limit, dt_lim=dt)


@pytest.mark.parametrize("order", [8, 10])
def test_rhs_2d_grf_circle(order):
    U = inputs.grf_2d(48, seed=11)
    _run_rhs(U, (48, 48), [0, 0], order=order)


@pytest.mark.parametrize("bc", [(1, 0), (2, 2), (3, 1)])
def test_rhs_2d_boundaries_ragged(bc):
    U = inputs.grf_2d(72, seed=12)[:, :, :45, :37].copy()  # ragged tiles in both directions
    U = np.ascontiguousarray(U)
    _run_rhs(U, (37, 45), list(bc), order=10, splitting=1)


@pytest.mark.parametrize("order,limit", [(10, 1), (8, 0), (10, 0)])
def test_rhs_3d_blast_cavity(order, limit):
    U = inputs.blast_cavity_3d(20)
    dt = 0.0
    if limit:
        g = oracle.make_grid((20, 20, 20), [0.05] * 3, [0] * 3)
        dt = oracle.dt(g, 1.4, 0.4, U)
    _run_rhs(U, (20, 20, 20), [0, 0, 0], order=order, positivity=limit, dt_lim=dt)


def test_rhs_3d_mixed_boundaries_ragged():
    U = inputs.blast_cavity_3d(24)[:, :13, :17, :22].copy()
    _run_rhs(np.ascontiguousarray(U), (22, 17, 13), [1, 2, 0], order=10)


def test_rhs_minimum_size():
    """n = G along every direction (the smallest grid the boundary mapping allows)."""
    U = inputs.random_smooth((5, 5, 5), seed=4, kmax=1)
    _run_rhs(U, (5, 5, 5), [0, 0, 0], order=10)
    U = inputs.random_smooth((4, 6), seed=5, kmax=1)
    _run_rhs(U, (4, 6), [1, 3], order=8)


def _step_gpu(U, shape, bc, order, positivity, cfl=0.4, dt=0.0, gamma=1.4, splitting=0):
    _, g_gpu = _pair(shape, bc)
    sch = tenoaa.make_scheme(order, splitting, positivity)
    Ud = _dev(U)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    ws = tenoaa.workspace(g_gpu, sch, tenoaa.WS_STEP)
    tenoaa.step(g_gpu, sch, Ud, dtd, gamma=gamma, cfl=cfl, ws=ws)
    torch.cuda.synchronize()
    return tenoaa.to_numpy(Ud), float(dtd.item()), tenoaa.get_status(ws)


def test_step_3d_limiter():
    U = inputs.blast_cavity_3d(16)
    g_or, _ = _pair((16, 16, 16), [0, 0, 0])
    U_or, dt_or, fl, mg = oracle.step(g_or, U, order=10, positivity=1, cfl=0.4, want_flags=True)
    U_g, dt_g, st = _step_gpu(U, (16, 16, 16), [0, 0, 0], 10, 1)
    assert st == 0
    assert dt_g == dt_or
    near = int((mg <= 1e-12).sum())
    assert near == 0
    scale = np.abs(U_or).reshape(5, -1).max(axis=1)
    err = (np.abs(U_g - U_or).reshape(5, -1).max(axis=1) / scale).max()
    print("step 3d: bitwise", int((U_g == U_or).sum()), "of", U.size, "max rel", err)
    assert err <= 1e-11


def test_shock_tube_100_steps_synchronised():
    """1D N=256, TENO8-AA, LLF, CFL 0.4, outflow, 100 SSP-RK3 steps: every GPU step
    starts from the oracle's state and must reproduce the oracle's next state."""
    U = inputs.shock_tube_1d(256)
    g_or, _ = _pair((256,), [1])
    worst = 0.0
    same = 0
    for k in range(100):
        U_next, dt_or, _, mg = oracle.step(g_or, U, order=8, cfl=0.4, want_flags=True)
        U_g, dt_g, st = _step_gpu(U, (256,), [1], 8, 0)
        assert st == 0 and dt_g == dt_or
        scale = np.abs(U_next).reshape(3, -1).max(axis=1)
        # a decision within the near band of a threshold (any stage) may
        # legitimately differ: leave out the cells its face reaches within the
        # step (three stages of the stencil's half-width)
        keep = np.ones(256, bool)
        for f in np.nonzero((mg.reshape(3, -1) <= 1e-12).any(axis=0))[0] % 257:
            keep[max(0, f - 15):min(256, f + 15)] = False
        err = (np.abs(U_g - U_next).reshape(3, -1)[:, keep].max(axis=1) / scale).max()
        assert err <= 1e-11, (k, err)
        worst = max(worst, err)
        same += int((U_g == U_next).all())
        U = U_next
    print("100 steps: bitwise-identical steps", same, "worst rel", worst)


# ------------------------------------------------------------- full sizes


def _sample_cells(ncell, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, ncell, k))


@pytest.mark.parametrize("order", [8, 10])
def test_full_2d_1024_sampled(order):
    """2D 1024^2 periodic GRF with the circular 10:1 pressure jump, one RHS."""
    U = inputs.grf_2d(1024)
    g_or, g_gpu = _pair((1024, 1024), [0, 0])
    sch = tenoaa.make_scheme(order, 0, 0)
    out = tenoaa.rhs(g_gpu, sch, _dev(U))
    d = tenoaa.to_numpy(out).reshape(4, -1)
    # cells on the circle's edge plus random cells
    x = (np.arange(1024) + 0.5) / 1024
    X, Y = np.meshgrid(x, x, indexing="xy")
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2).reshape(-1)
    edge = np.nonzero(np.abs(r - 0.2) < 2e-3)[0][::7]
    cells = np.unique(np.concatenate([edge, _sample_cells(1024 * 1024, 600, 3)]))
    ref = oracle.rhs_cells(g_or, U, cells, order=order)
    scale = np.abs(d).max(axis=1)
    err = (np.abs(d[:, cells].T - ref) / scale).max()
    print("2d 1024 sampled", cells.size, "cells, max rel", err, "bitwise", int((d[:, cells].T == ref).sum()))
    assert err <= 1e-11


def _stage_cells(n):
    """Sampled cells of the 3D workload: random ones plus cells on the blast
    and cavity spheres' surfaces."""
    x = (np.arange(n) + 0.5) / n
    cells = [_sample_cells(n ** 3, 150, 5)]
    for cx in (0.3, 0.7):
        ii = np.nonzero(np.abs(x - cx) < 0.11)[0]
        rng = np.random.default_rng(int(cx * 10))
        k = rng.integers(0, ii.size, (60, 3))
        cells.append((ii[k[:, 2]] * n + (n // 2)) * n + ii[k[:, 0]])
    return np.unique(np.concatenate(cells))


def test_full_3d_256_step_stages_sampled():
    """3D 256^3 blast/cavity workload, TENO10-AA, LLF, limiter on, one SSP-RK3
    step at CFL 0.4 (Sec. 5): tenoaa_step equals its three stages taken by
    tenoaa_rk3_stage bit for bit, and each stage's new state at sampled cells
    equals the Shu-Osher combination of the oracle's right-hand side of that
    stage's input (the GPU's stage state: stage-synchronised), with the
    limiter factors from the step's dt and wave speeds."""
    n = 256
    U = inputs.grf_3d(n)
    g_or, g_gpu = _pair((n, n, n), [0, 0, 0])
    amax_or = oracle.wave_speeds(g_or, 1.4, U)
    dt_or = oracle.dt(g_or, 1.4, 0.4, U)
    sch = tenoaa.make_scheme(10, 0, 1)
    U0 = _dev(U)
    del U
    # the whole step
    Us_ = U0.clone()
    dts = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = tenoaa.workspace(g_gpu, sch, tenoaa.WS_STEP)
    tenoaa.step(g_gpu, sch, Us_, dts, cfl=0.4, ws=ws)
    torch.cuda.synchronize()
    assert float(dts.item()) == dt_or
    assert tenoaa.get_status(ws) == 0
    # the same step stage by stage
    wsr = tenoaa.workspace(g_gpu, sch, tenoaa.WS_RHS)
    amax = tenoaa.wave_speeds(g_gpu, sch, U0, ws=wsr)
    assert np.array_equal(tenoaa.to_numpy(amax), amax_or[:3])
    dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
    S1 = torch.empty_like(U0)
    S2 = torch.empty_like(U0)
    S3 = torch.empty_like(U0)
    tenoaa.rk3_stage(g_gpu, sch, 1, amax, dtg, U0, None, S1, ws=wsr)
    tenoaa.rk3_stage(g_gpu, sch, 2, amax, dtg, U0, S1, S2, ws=wsr)
    tenoaa.rk3_stage(g_gpu, sch, 3, amax, dtg, U0, S2, S3, ws=wsr)
    torch.cuda.synchronize()
    assert float(dtg.item()) == dt_or
    assert torch.equal(S3, Us_), "tenoaa_step differs from its three stages"
    del Us_
    cells = _stage_cells(n)
    Un = tenoaa.to_numpy(U0).reshape(5, -1)
    dt = dt_or
    worst = 0.0
    bitwise = 0
    for stage, (src, dst) in enumerate(((U0, S1), (S1, S2), (S2, S3)), start=1):
        Uin = tenoaa.to_numpy(src)
        ref = oracle.rhs_cells(g_or, Uin, cells, order=10, positivity=1, dt_lim=dt, amax=amax_or).T
        Uin = Uin.reshape(5, -1)[:, cells]
        un = Un[:, cells]
        if stage == 1:
            want = un + dt * ref
        elif stage == 2:
            want = 0.75 * un + 0.25 * Uin + (0.25 * dt) * ref
        else:
            want = (1.0 / 3.0) * un + (2.0 / 3.0) * Uin + ((2.0 / 3.0) * dt) * ref
        got = tenoaa.to_numpy(dst).reshape(5, -1)[:, cells]
        scale = np.abs(tenoaa.to_numpy(dst).reshape(5, -1)).max(axis=1)[:, None]
        err = float((np.abs(got - want) / scale).max())
        worst = max(worst, err)
        bitwise += int((got == want).sum())
        assert err <= 1e-11, (stage, err)
    print("3d 256 step: stage composition bitwise, %d sampled cells x 3 stages, max rel %.3e, bitwise %d of %d"
          % (cells.size, worst, bitwise, 3 * 5 * cells.size))
    # properties of the whole step: conservation (periodic), positivity
    before = U0.reshape(5, -1).sum(dim=1)
    after = S3.reshape(5, -1).sum(dim=1)
    tot = S3.reshape(5, -1).abs().sum(dim=1)
    assert float(((after - before).abs() / tot).max()) < 1e-13
    rho = S3[0]
    p = 0.4 * (S3[4] - 0.5 * (S3[1] ** 2 + S3[2] ** 2 + S3[3] ** 2) / rho)
    assert float(rho.min()) > 0 and float(p.min()) > 0


def test_full_3d_256_rhs_sampled():
    """3D 256^3 blast/cavity workload, TENO10-AA, limiter on: one right-hand
    side at sampled cells against the oracle."""
    n = 256
    U = inputs.grf_3d(n)
    g_or, g_gpu = _pair((n, n, n), [0, 0, 0])
    amax = oracle.wave_speeds(g_or, 1.4, U)
    dt = oracle.dt(g_or, 1.4, 0.4, U)
    sch = tenoaa.make_scheme(10, 0, 1)
    out = tenoaa.rhs(g_gpu, sch, _dev(U), dt_limiter=dt)
    d = tenoaa.to_numpy(out).reshape(5, -1)
    cells = _stage_cells(n)
    ref = oracle.rhs_cells(g_or, U, cells, order=10, positivity=1, dt_lim=dt, amax=amax)
    scale = np.abs(d).max(axis=1)
    err = (np.abs(d[:, cells].T - ref) / scale).max()
    print("3d 256 sampled", cells.size, "cells, max rel", err, "bitwise", int((d[:, cells].T == ref).sum()))
    assert err <= 1e-11
