"""Checkpointed multi-step adjoint (torch.autograd) of the 2D 512^2 TENO10-AA
workload: gradient of an L2 density misfit after 50 SSP-RK3 steps against
fourth-order central differences with the recorded dt schedule and decisions
replayed, plus the replay and checkpoint consistency it relies on."""
import os

import numpy as np
import pytest

from paper_2109_14340_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import adjoint, tenoaa  # noqa: E402

N = 512
STEPS = 50
EVERY = 10
NPROBES = int(os.environ.get("TENOAA_FD_PROBES", "100"))


def _setup(n=N):
    U0 = torch.from_numpy(inputs.grf_2d(n, seed=inputs.SEED_BASE + 5, jump=False)).cuda()
    target = torch.from_numpy(inputs.grf_2d(n, seed=inputs.SEED_BASE + 50, jump=False)[0]).cuda()
    grid = tenoaa.make_grid((n, n))
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 0)
    return U0, target, grid, sch


def _loss(U, target, n):
    return torch.sqrt(((U[0] - target) ** 2).sum() / (n * n))


def test_replay_reproduces_trajectory():
    U0, _, grid, sch = _setup(128)
    Ua, dts, flags = adjoint.record_trajectory(U0, grid, sch, 8)
    Ub = adjoint.replay_trajectory(U0, grid, sch, dts, flags)
    assert torch.equal(Ua, Ub)
    # and the plain step with the recorded dt gives the same states
    U = U0.clone()
    for n in range(8):
        d = dts[n:n + 1].clone()
        tenoaa.step(grid, sch, U, d)
    assert torch.equal(U, Ua)


def test_checkpointed_gradient_equals_unsegmented():
    U0, target, grid, sch = _setup(128)
    g = []
    for every in (3, 100):
        x = U0.clone().requires_grad_(True)
        UT = adjoint.rk3_trajectory(x, grid, sch, 7, checkpoint_every=every)
        _loss(UT, target, 128).backward()
        g.append(x.grad.clone())
    assert torch.allclose(g[0], g[1], rtol=1e-12, atol=1e-15 * float(g[1].abs().max()))


def _dloss(T, T0, d0, L0, target):
    """L(T) - L(T0) through the state difference, so that the cancellation
    happens cell by cell instead of in the two norms."""
    d = T[0] - target
    S = float(((T[0] - T0[0]) * (d + d0)).sum()) / (N * N)
    return S / (float(torch.sqrt((d ** 2).sum() / (N * N))) + L0)


def test_gradient_vs_finite_differences_512():
    """Fourth-order central differences of the replayed map (dt and every
    decision frozen at the base run) against the checkpointed adjoint.  The
    step h = 1e-4 is where the difference quotient is cleanest: with frozen
    decisions the map is smooth, and at smaller h rounding noise (which grows
    as 1/h) dominates.  The perturbed runs are also made once with live
    decisions to count how many faces would have flipped."""
    U0, target, grid, sch = _setup()
    x = U0.clone().requires_grad_(True)
    UT = adjoint.rk3_trajectory(x, grid, sch, STEPS, checkpoint_every=EVERY)
    _loss(UT, target, N).backward()
    g = x.grad
    T0, dts, flags = adjoint.record_trajectory(U0, grid, sch, STEPS)
    d0 = T0[0] - target
    L0 = float(torch.sqrt((d0 ** 2).sum() / (N * N)))
    rng = np.random.default_rng(14345)
    probes = [(int(rng.integers(0, 4)), int(rng.integers(0, N)), int(rng.integers(0, N))) for _ in range(NPROBES)]
    h = 1e-4
    ok, worst, flips = 0, 0.0, 0
    gmax = float(g.abs().max())
    for (c, j, i) in probes:
        dl = {}
        for k in (-2, -1, 1, 2):
            Up = U0.clone()
            Up[c, 0, j, i] += k * h
            dl[k] = _dloss(adjoint.replay_trajectory(Up, grid, sch, dts, flags), T0, d0, L0, target)
        fd = (8.0 * (dl[1] - dl[-1]) - (dl[2] - dl[-2])) / (12.0 * h)
        Ul = U0.clone()
        Ul[c, 0, j, i] += h
        _, _, fl = adjoint.record_trajectory(Ul, grid, sch, STEPS)
        flips += int((fl != flags).sum())
        ga = float(g[c, 0, j, i])
        err = abs(ga - fd)
        worst = max(worst, err / max(abs(fd), 1e-300))
        if err <= 1e-6 * abs(fd) + 1e-9 * gmax:
            ok += 1
    print("FD probes passing: %d / %d, worst relative %.2e, |g|_inf %.3e, live decision flips at +h: %d"
          % (ok, len(probes), worst, gmax, flips))
    assert ok >= 0.99 * len(probes)
