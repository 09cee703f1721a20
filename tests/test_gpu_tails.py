"""Grids whose non-periodic directions end in a remainder of 1-4 faces beyond
the last whole tile (64 faces along x, 32 along y and z in the forward sweep;
64 along x in the reverse sweep): those faces go to one-wave tail tiles.  The
right-hand side, its decisions and a limited step against the oracle, and
the adjoint against the oracle's JVP, on such grids."""
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

# (shape, bc per axis): x n + 1 = 65 (remainder 1), 68 (4); y 33 (1), 35 (3); z 36 (4)
CASES = {
    "3d_r1_r1_r4": ((64, 32, 35), [1, 2, 3]),
    "2d_r4_r3": ((67, 34), [2, 1]),
    "2d_x_only": ((64, 40), [1, 0]),
}


def _state(shape):
    if len(shape) == 3:
        return inputs.blast_cavity_3d(max(shape))[:, :shape[2], :shape[1], :shape[0]].copy()
    return np.ascontiguousarray(inputs.grf_2d(max(shape), seed=33)[:, :, :shape[1], :shape[0]])


def _grids(shape, bc):
    dx = [1.0 / n for n in shape]
    return oracle.make_grid(shape, dx, bc), tenoaa.make_grid(shape, dx, bc)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("order,splitting", [(10, tenoaa.LLF), (8, tenoaa.ROE), (12, tenoaa.RUSANOV)])
def test_rhs_with_tail_tiles(case, order, splitting):
    shape, bc = CASES[case]
    U = _state(shape)
    g_or, g_gpu = _grids(shape, bc)
    d_or, fl_or, mg_or = oracle.rhs(g_or, U, order=order, splitting=splitting)
    sch = tenoaa.make_scheme(order, splitting, 0)
    fl = torch.zeros(tenoaa.flags_size(g_gpu), dtype=torch.uint8, device="cuda")
    ws = tenoaa.workspace(g_gpu, sch, tenoaa.WS_RHS)
    out = tenoaa.rhs(g_gpu, sch, torch.from_numpy(U).cuda(), flags=fl, ws=ws)
    torch.cuda.synchronize()
    assert tenoaa.get_status(ws) == 0
    rep = compare_rhs(g_or, tenoaa.to_numpy(out), d_or, tenoaa.to_numpy(fl), fl_or, mg_or)
    print(case, order, splitting, rep)
    assert rep["bitwise_equal"] == rep["elements"] or rep["near_faces"] > 0


def test_step_with_tail_tiles():
    """A step with the limiter on the 3D case's grid (the random field without
    the spheres: no decision of the step lies within 1e-12 of its threshold)
    equals the oracle's bit for bit."""
    shape, bc = CASES["3d_r1_r1_r4"]
    U0 = np.ascontiguousarray(inputs.grf_3d(64, spheres=False)[:, :shape[2], :shape[1], :shape[0]])
    g_or, g_gpu = _grids(shape, bc)
    Uo, dto, _, margins = oracle.step(g_or, U0, order=10, positivity=1, cfl=0.4, want_flags=True)
    assert (margins <= 1e-12).sum() == 0
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    U = torch.from_numpy(U0).cuda()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    tenoaa.step(g_gpu, sch, U, dt)
    assert float(dt.item()) == dto
    assert np.array_equal(U.cpu().numpy(), Uo)


@pytest.mark.parametrize("case", ["3d_r1_r1_r4", "2d_x_only"])
@pytest.mark.parametrize("order", [10, 12])
def test_rhs_vjp_with_tail_tiles(case, order):
    shape, bc = CASES[case]
    U = _state(shape)
    g_or, g_gpu = _grids(shape, bc)
    rng = np.random.default_rng(34)
    V = rng.standard_normal(U.shape) * np.abs(U).reshape(U.shape[0], -1).max(axis=1)[:, None, None, None]
    Wt = rng.standard_normal(U.shape)
    _, flags, margins = oracle.rhs(g_or, U, order=order)
    assert (margins <= 1e-12).sum() == 0
    _, jv = oracle.rhs_jvp(g_or, U, V, flags, order=order)
    jtw = tenoaa.to_numpy(tenoaa.rhs_vjp(g_gpu, tenoaa.make_scheme(order), torch.from_numpy(U).cuda(),
                                         torch.from_numpy(Wt).cuda()))
    lhs, rhs = float(np.sum(Wt * jv)), float(np.sum(jtw * V))
    scale = float(np.sum(np.abs(Wt * jv)))
    print(case, "<w,Jv> %.15e  <J^T w,v> %.15e  rel %.2e" % (lhs, rhs, abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= 1e-11 * scale
