"""The HIP adjoint (vector-Jacobian products) against the oracle's exact
directional derivatives (forward-mode dual numbers with the same frozen
decisions)."""
import numpy as np
import pytest

import oracle
from paper_2109_14340_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import tenoaa  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _grids(shape, bc_lo):
    dx = [1.0 / n for n in shape]
    return oracle.make_grid(shape, dx, bc_lo), tenoaa.make_grid(shape, dx, bc_lo)


def _dot_check(U, shape, bc, order, splitting, seed, tol=1e-11):
    g_or, g_gpu = _grids(shape, bc)
    rng = np.random.default_rng(seed)
    V = rng.standard_normal(U.shape) * np.abs(U).reshape(U.shape[0], -1).max(axis=1)[:, None, None, None]
    Wt = rng.standard_normal(U.shape)
    _, flags, margins = oracle.rhs(g_or, U, order=order, splitting=splitting)
    assert (margins <= 1e-12).sum() == 0
    _, jv = oracle.rhs_jvp(g_or, U, V, flags, order=order, splitting=splitting)
    sch = tenoaa.make_scheme(order, splitting, 0)
    jtw = tenoaa.to_numpy(tenoaa.rhs_vjp(g_gpu, sch, _dev(U), _dev(Wt)))
    lhs = float(np.sum(Wt * jv))
    rhs = float(np.sum(jtw * V))
    scale = float(np.sum(np.abs(Wt * jv)))
    print(shape, order, splitting, "<w,Jv> %.15e  <J^T w,v> %.15e  rel %.2e" % (lhs, rhs, abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= tol * scale


@pytest.mark.parametrize("order", [8, 10])
@pytest.mark.parametrize("splitting", [0, 1])
def test_rhs_vjp_dot_1d(order, splitting):
    _dot_check(inputs.shock_tube_1d(48), (48,), [1], order, splitting, 1)


@pytest.mark.parametrize("order", [8, 10])
def test_rhs_vjp_dot_2d_periodic(order):
    _dot_check(inputs.grf_2d(24, seed=21)[:, :, :20, :].copy(), (24, 20), [0, 0], order, 0, 2)


@pytest.mark.parametrize("bc", [(1, 2), (3, 1)])
def test_rhs_vjp_dot_2d_walls(bc):
    U = np.ascontiguousarray(inputs.grf_2d(36, seed=22)[:, :, :19, :23])
    _dot_check(U, (23, 19), list(bc), 10, 1, 3)


def test_rhs_vjp_dot_3d():
    U = np.ascontiguousarray(inputs.blast_cavity_3d(16)[:, :11, :13, :14])
    _dot_check(U, (14, 13, 11), [0, 1, 2], 10, 0, 4)


@pytest.mark.parametrize("case", ["1d", "2d"])
def test_rhs_vjp_full_jacobian(case):
    """Every column of the Jacobian from the oracle; J^T w compared element-wise."""
    if case == "1d":
        U, shape, bc, order = inputs.shock_tube_1d(20), (20,), [1], 10
    else:
        U, shape, bc, order = inputs.random_smooth((8, 6), seed=6, kmax=2), (8, 6), [0, 0], 8
    g_or, g_gpu = _grids(shape, bc)
    _, flags, margins = oracle.rhs(g_or, U, order=order)
    assert (margins <= 1e-12).sum() == 0
    N = U.size
    J = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        _, col = oracle.rhs_jvp(g_or, U, e.reshape(U.shape), flags, order=order)
        J[:, k] = col.reshape(-1)
    Wt = np.random.default_rng(7).standard_normal(N)
    ref = J.T @ Wt
    sch = tenoaa.make_scheme(order, 0, 0)
    got = tenoaa.to_numpy(tenoaa.rhs_vjp(g_gpu, sch, _dev(U), _dev(Wt.reshape(U.shape)))).reshape(-1)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(case, "max rel err of J^T w: %.2e" % err)
    assert err <= 1e-11


@pytest.mark.parametrize("case", ["1d", "2d"])
def test_step_vjp_dot(case):
    """One SSP-RK3 step with dt frozen: <w, J v> (oracle forward mode through the
    three stages with their own frozen decisions, dual numbers) = <J^T w, v> (GPU)."""
    if case == "1d":
        U, shape, bc, order = inputs.shock_tube_1d(64), (64,), [1], 8
    else:
        U, shape, bc, order = np.ascontiguousarray(inputs.grf_2d(24, seed=31)[:, :, :18, :]), (24, 18), [0, 0], 10
    g_or, g_gpu = _grids(shape, bc)
    _, dt, flags3, margins3 = oracle.step(g_or, U, order=order, cfl=0.4, want_flags=True)
    assert (margins3 <= 1e-12).sum() == 0
    rng = np.random.default_rng(8)
    V = rng.standard_normal(U.shape)
    Wt = rng.standard_normal(U.shape)
    jv = oracle.step_jvp(g_or, U, V, dt, flags3, order=order)
    sch = tenoaa.make_scheme(order, 0, 0)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    jtw = tenoaa.to_numpy(tenoaa.step_vjp(g_gpu, sch, _dev(U), dtd, _dev(Wt)))
    lhs, rhs = float(np.sum(Wt * jv)), float(np.sum(jtw * V))
    scale = float(np.sum(np.abs(Wt * jv)))
    print(case, "step <w,Jv> %.15e  <J^T w,v> %.15e rel %.2e" % (lhs, rhs, abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= 1e-11 * scale


def _double_rarefaction_state(n=64, steps=15):
    """The Sec. 5.3.1 double rarefaction after a few limited steps: near-vacuum
    at the centre, where the positivity limiter acts."""
    x = (np.arange(n) + 0.5) / n
    U = inputs._as_layout(inputs.conserved_from_primitive(np.ones(n), [np.where(x < 0.5, -2.0, 2.0)],
                                                          np.full(n, 0.1), 1.4), 1)
    g = oracle.make_grid((n,), [1.0 / n], [1])
    for _ in range(steps):
        U, _, _, _ = oracle.step(g, U, order=10, positivity=1, cfl=0.4)
    return U


@pytest.mark.parametrize("case", ["1d_near_vacuum", "3d_blast_cavity"])
def test_step_vjp_dot_with_limiter(case):
    """With the positivity limiter: its factors theta (recorded by the forward
    sweeps) and the Lax-Friedrichs speed's cell frozen, <w, J v> (oracle, dual
    numbers with theta evaluated from the values) = <J^T w, v> (GPU); the
    limiter does act on these states."""
    if case == "1d_near_vacuum":
        U, shape, bc, order = _double_rarefaction_state(), (64,), [1], 10
    else:
        U, shape, bc, order = inputs.blast_cavity_3d(12), (12, 12, 12), [0, 0, 0], 8
    g_or, g_gpu = _grids(shape, bc)
    Ul, dt, flags3, margins3 = oracle.step(g_or, U, order=order, positivity=1, cfl=0.4, want_flags=True)
    Uu, _, _, _ = oracle.step(g_or, U, order=order, positivity=0, dt=dt)
    assert not np.array_equal(Ul, Uu), "the limiter does not act on this state"
    assert (margins3 <= 1e-12).sum() == 0
    rng = np.random.default_rng(9)
    V = rng.standard_normal(U.shape) * np.abs(U).reshape(U.shape[0], -1).max(axis=1)[:, None, None, None]
    Wt = rng.standard_normal(U.shape)
    jv = oracle.step_jvp(g_or, U, V, dt, flags3, order=order, positivity=1)
    sch = tenoaa.make_scheme(order, 0, 1)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    jtw = tenoaa.to_numpy(tenoaa.step_vjp(g_gpu, sch, _dev(U), dtd, _dev(Wt)))
    lhs, rhs = float(np.sum(Wt * jv)), float(np.sum(jtw * V))
    scale = float(np.sum(np.abs(Wt * jv)))
    # without the limiter's terms the products would differ
    jv0 = oracle.step_jvp(g_or, U, V, dt, flags3, order=order, positivity=0)
    print(case, "limited step <w,Jv> %.15e  <J^T w,v> %.15e rel %.2e (unlimited <w,Jv> %.6e)"
          % (lhs, rhs, abs(lhs - rhs) / scale, float(np.sum(Wt * jv0))))
    assert abs(lhs - rhs) <= 1e-11 * scale


def test_rhs_vjp_with_flags_of_another_state():
    """Decisions given by the caller (here those the oracle takes at a
    perturbed state) are the ones differentiated: dot test against the
    oracle's JVP with the same flags."""
    U = np.ascontiguousarray(inputs.grf_2d(24, seed=41)[:, :, :20, :])
    shape, bc = (24, 20), [0, 0]
    g_or, g_gpu = _grids(shape, bc)
    rng = np.random.default_rng(42)
    Up = U * (1.0 + 0.05 * rng.standard_normal(U.shape))
    _, fl_u, _ = oracle.rhs(g_or, U, order=10)
    _, fl_p, _ = oracle.rhs(g_or, Up, order=10)
    assert (fl_p != fl_u).sum() > 0
    V = rng.standard_normal(U.shape) * np.abs(U).reshape(U.shape[0], -1).max(axis=1)[:, None, None, None]
    Wt = rng.standard_normal(U.shape)
    _, jv = oracle.rhs_jvp(g_or, U, V, fl_p, order=10)
    sch = tenoaa.make_scheme(10, 0, 0)
    jtw = tenoaa.to_numpy(tenoaa.rhs_vjp(g_gpu, sch, _dev(U), _dev(Wt), flags=_dev(fl_p)))
    lhs, rhs = float(np.sum(Wt * jv)), float(np.sum(jtw * V))
    scale = float(np.sum(np.abs(Wt * jv)))
    print("flags of another state: %d differ; <w,Jv> %.15e <J^T w,v> %.15e rel %.2e" % (
        int((fl_p != fl_u).sum()), lhs, rhs, abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= 1e-11 * scale


def test_step_vjp_with_recorded_flags_matches_recompute():
    U = np.ascontiguousarray(inputs.grf_2d(32, seed=43)[:, :, :24, :])
    g = tenoaa.make_grid((32, 24))
    sch = tenoaa.make_scheme(10, 0, 0)
    Ud = _dev(U)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    fl3 = torch.zeros(3 * tenoaa.flags_size(g), dtype=torch.uint8, device="cuda")
    tenoaa.step_flags(g, sch, Ud.clone(), dt, fl3, tenoaa.FLAGS_RECORD)
    W = _dev(np.random.default_rng(44).standard_normal(U.shape))
    a = tenoaa.step_vjp(g, sch, Ud, dt, W)
    b = tenoaa.step_vjp(g, sch, Ud, dt, W, flags3=fl3)
    err = float((a - b).abs().max() / a.abs().max())
    print("step VJP with recorded flags vs recomputed: max rel %.2e" % err)
    assert err <= 1e-13
