"""tenoaa_rhs_noalloc (the entry point for callers that cannot allocate)
through the C ABI against tenoaa_rhs with a caller's workspace: the same
right-hand side, decisions and status on two calls in a row, the second on a
smaller grid, and a clear error for a grid beyond the buffer."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2109_14340_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import tenoaa  # noqa: E402


def _noalloc(grid, scheme, U, dt_lim, flags):
    L = tenoaa.load()
    out = torch.empty_like(U)
    status = torch.full((1,), -7, dtype=torch.int32, device=U.device)
    rc = L.tenoaa_rhs_noalloc(ctypes.byref(grid), ctypes.byref(scheme), 1.4, ctypes.c_void_p(U.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), dt_lim, ctypes.c_void_p(flags.data_ptr()),
                              ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, rc
    return out, status


def _reference(grid, scheme, U, dt_lim):
    fl = torch.zeros(tenoaa.flags_size(grid), dtype=torch.uint8, device=U.device)
    ws = tenoaa.workspace(grid, scheme, tenoaa.WS_RHS, U.device)
    out = tenoaa.rhs(grid, scheme, U, dt_limiter=dt_lim, flags=fl, ws=ws)
    return out, fl, tenoaa.get_status(ws)


def test_noalloc_matches_workspace_entry_two_calls():
    cases = []
    # first: 3D blast/cavity with the limiter; second: a smaller 2D grid
    U3 = inputs.blast_cavity_3d(40)[:, :32, :36, :40].copy()
    g3 = tenoaa.make_grid((40, 36, 32))
    go3 = oracle.make_grid((40, 36, 32), [1 / 40, 1 / 36, 1 / 32], [0, 0, 0])
    cases.append((g3, tenoaa.make_scheme(10, tenoaa.LLF, 1), U3, oracle.dt(go3, 1.4, 0.4, U3)))
    U2 = inputs.grf_2d(48, seed=21)[:, :, :40, :48].copy()
    g2 = tenoaa.make_grid((48, 40), bc_lo=[1, 2], bc_hi=[1, 2])
    cases.append((g2, tenoaa.make_scheme(8, tenoaa.RUSANOV, 0), U2, 0.0))
    L = tenoaa.load()
    for grid, scheme, Un, dt_lim in cases:
        assert L.tenoaa_workspace_bytes(ctypes.byref(grid), ctypes.byref(scheme), 0) <= (80 << 20)
        U = torch.from_numpy(np.ascontiguousarray(Un)).cuda()
        fl = torch.zeros(tenoaa.flags_size(grid), dtype=torch.uint8, device="cuda")
        got, status = _noalloc(grid, scheme, U, dt_lim, fl)
        want, fl_want, st_want = _reference(grid, scheme, U, dt_lim)
        torch.cuda.synchronize()
        assert int(status.item()) == 0 and st_want == 0
        assert torch.equal(fl, fl_want)
        assert torch.equal(got, want)


def test_noalloc_rejects_grid_beyond_buffer():
    L = tenoaa.load()
    grid = tenoaa.make_grid((128, 128, 128))
    scheme = tenoaa.make_scheme(10, tenoaa.LLF, 0)
    assert L.tenoaa_workspace_bytes(ctypes.byref(grid), ctypes.byref(scheme), 0) > (80 << 20)
    rc = L.tenoaa_rhs_noalloc(ctypes.byref(grid), ctypes.byref(scheme), 1.4, ctypes.c_void_p(256),
                              ctypes.c_void_p(512), 0.0, None, None, None)
    assert rc == -5  # TENOAA_EWORKSPACE, before any device work
