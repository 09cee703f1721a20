"""A grid split into pieces, one GPU's share each, run on one GPU: every piece
takes halo sides holding its neighbours' order/2 cells next to each cut
(refreshed before every SSP-RK3 stage), and the step's wave speeds are the
maxima over the pieces.  The pieces' right-hand sides, decisions and steps
equal the whole grid's bit for bit (which the oracle matches on the whole
grid in the parity tests)."""
import numpy as np
import pytest

from paper_2109_14340_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import tenoaa  # noqa: E402

H = tenoaa.BC_HALO


def _ax(ndim, d):
    """Array axis of direction d in the (nvar, nz, ny, nx) layout."""
    return 3 - d


def _halos(U, d, lo, hi, G):
    """Halo layers of the piece [lo, hi) along direction d of the whole state U
    (periodic wrap): {(d, 0): (1, G, nvar, plane), (d, 1): ...}, layer r = 1..G
    counted outward from the cut, the plane in the ABI order (lower remaining
    axis fastest = C order of the remaining array axes)."""
    n = U.shape[_ax(U.ndim, d)]
    nv = U.shape[0]
    out = {}
    for side in (0, 1):
        layers = []
        for r in range(1, G + 1):
            c = (lo - r) % n if side == 0 else (hi - 1 + r) % n
            sl = U.index_select(_ax(U.ndim, d), torch.tensor([c], device=U.device))
            layers.append(sl.reshape(nv, -1))
        out[(d, side)] = torch.stack(layers)[None].contiguous()
    return out


def _piece(U, d, lo, hi):
    return U.narrow(_ax(U.ndim, d), lo, hi - lo).contiguous()


def _piece_grid(shape, d, lo, hi, halos):
    ps = list(shape)
    ps[d] = hi - lo
    dx = [1.0 / n for n in shape]
    bc = [tenoaa.BC_PERIODIC] * len(shape)
    bc[d] = H
    return tenoaa.make_grid(tuple(ps), dx, bc, bc, bc_values=halos)


CUTS = {
    "3d_z": ((24, 20, 16), 2, [0, 7, 16]),
    "3d_x_ragged": ((23, 14, 12), 0, [0, 6, 13, 23]),
    "3d_y": ((16, 22, 12), 1, [0, 11, 22]),
    "2d_y": ((40, 36), 1, [0, 12, 25, 36]),
}


def _state(shape):
    if len(shape) == 3:
        return inputs.blast_cavity_3d(max(shape))[:, :shape[2], :shape[1], :shape[0]].copy()
    return np.ascontiguousarray(inputs.grf_2d(max(shape), seed=31)[:, :, :shape[1], :shape[0]])


def _flag_blocks(shape, periodic, fl):
    """Per direction k, the decision bytes as (nvar, 2, m_z, m_y, m_x) with
    m_k the faces along k (n_k if periodic[k], else n_k + 1)."""
    nd = len(shape)
    n = list(shape) + [1] * (3 - nd)
    out, off = [], 0
    for k in range(nd):
        m = list(n)
        m[k] = n[k] if periodic[k] else n[k] + 1
        size = (nd + 2) * 2 * m[0] * m[1] * m[2]
        out.append(fl[off:off + size].reshape(nd + 2, 2, m[2], m[1], m[0]))
        off += size
    return out


@pytest.mark.parametrize("case", list(CUTS))
@pytest.mark.parametrize("order,splitting", [(10, tenoaa.LLF), (8, tenoaa.ROE)])
def test_pieces_rhs_equal_whole(case, order, splitting):
    """Right-hand side and every decision byte of each piece equal the whole
    grid's at the same cells and faces (the cut faces included)."""
    shape, d, cuts = CUTS[case]
    G = order // 2
    nd = len(shape)
    U = torch.from_numpy(_state(shape)).cuda()
    sch = tenoaa.make_scheme(order, splitting, 0)
    g = tenoaa.make_grid(shape)
    fl = torch.zeros(tenoaa.flags_size(g), dtype=torch.uint8, device="cuda")
    whole = tenoaa.rhs(g, sch, U, flags=fl)
    blocks = _flag_blocks(shape, [True] * nd, fl)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        gp = _piece_grid(shape, d, lo, hi, _halos(U, d, lo, hi, G))
        Up = _piece(U, d, lo, hi)
        flp = torch.zeros(tenoaa.flags_size(gp), dtype=torch.uint8, device="cuda")
        ws = tenoaa.workspace(gp, sch, tenoaa.WS_RHS)
        got = tenoaa.rhs(gp, sch, Up, flags=flp, ws=ws)
        torch.cuda.synchronize()
        assert tenoaa.get_status(ws) == 0
        assert torch.equal(got, _piece(whole, d, lo, hi)), (case, lo, hi)
        ps = list(shape)
        ps[d] = hi - lo
        pb = _flag_blocks(ps, [k != d for k in range(nd)], flp)
        for k in range(nd):
            idx = torch.arange(lo, hi + (1 if k == d else 0), device="cuda") % shape[d]
            assert torch.equal(pb[k], blocks[k].index_select(4 - d, idx)), (case, lo, hi, k)


@pytest.mark.parametrize("case", ["3d_z", "3d_x_ragged", "2d_y"])
def test_pieces_step_equal_whole(case):
    """Two SSP-RK3 steps with the limiter (CFL 0.4): per stage the halos are
    refreshed from the pieces' stage states and the speeds are the maxima over
    the pieces; the result and dt equal tenoaa_step on the whole grid."""
    shape, d, cuts = CUTS[case]
    order, G = 10, 5
    sch = tenoaa.make_scheme(order, tenoaa.LLF, 1)
    U0 = torch.from_numpy(_state(shape)).cuda()
    g = tenoaa.make_grid(shape)
    Uw = U0.clone()
    dtw = torch.zeros(1, dtype=torch.float64, device="cuda")
    spans = list(zip(cuts[:-1], cuts[1:]))
    pieces = [_piece(U0, d, lo, hi) for lo, hi in spans]
    grids = [_piece_grid(shape, d, lo, hi, _halos(U0, d, lo, hi, G)) for lo, hi in spans]
    wss = [tenoaa.workspace(gp, sch, tenoaa.WS_RHS) for gp in grids]
    def exchange(states):
        """Every piece's halo sides from its neighbours' cells of `states`."""
        full = torch.cat(states, dim=_ax(4, d))
        for (lo, hi), gp in zip(spans, grids):
            for key, v in _halos(full, d, lo, hi, G).items():
                gp._faces[key].copy_(v)

    for _ in range(2):
        dtw.zero_()
        tenoaa.step(g, sch, Uw, dtw)
        # the step of the pieces: speeds of U^n (halo cells next to the cuts
        # included), their maxima over the pieces, then the three stages
        exchange(pieces)
        amax = torch.stack([tenoaa.wave_speeds(gp, sch, Up, ws=ws) for gp, Up, ws in zip(grids, pieces, wss)])
        amax = amax.max(dim=0).values.contiguous()
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        stage_states = [torch.empty_like(Up) for Up in pieces]
        for stage in (1, 2, 3):
            if stage > 1:
                exchange(stage_states)
            for k, (gp, ws) in enumerate(zip(grids, wss)):
                out = pieces[k] if stage == 3 else stage_states[k]
                tenoaa.rk3_stage(gp, sch, stage, amax, dt, pieces[k], None if stage == 1 else stage_states[k],
                                 out, ws=ws)
        torch.cuda.synchronize()
        for ws in wss:
            assert tenoaa.get_status(ws) == 0
        assert float(dt.item()) == float(dtw.item())
        got = torch.cat(pieces, dim=_ax(4, d))
        diff = int((got != Uw).sum())
        print(case, "dt %.17g, elements differing from the whole grid: %d" % (float(dt.item()), diff))
        assert torch.equal(got, Uw)


def test_halo_layers_must_match_the_order():
    shape, d = (24, 20, 16), 2
    U = torch.from_numpy(_state(shape)).cuda()
    gp = _piece_grid(shape, d, 0, 8, _halos(U, d, 0, 8, 4))
    with pytest.raises(tenoaa.TenoaaError, match="ghost layers"):
        tenoaa.rhs(gp, tenoaa.make_scheme(10), _piece(U, d, 0, 8))


@pytest.mark.parametrize("case", ["3d_z", "3d_x_ragged", "2d_y"])
@pytest.mark.parametrize("splitting", [tenoaa.LLF, tenoaa.ROE])
def test_pieces_rhs_vjp_sum_to_whole(case, splitting):
    """The adjoint of a split right-hand side: each piece's tenoaa_rhs_vjp_halo
    gives the adjoint of its own cells and of its halo cells; adding every
    halo adjoint to the neighbour's cells it came from gives the whole grid's
    tenoaa_rhs_vjp (up to the order of the sums)."""
    shape, d, cuts = CUTS[case]
    order, G = 10, 5
    U = torch.from_numpy(_state(shape)).cuda()
    R = torch.randn(U.shape, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    sch = tenoaa.make_scheme(order, splitting, 0)
    whole = tenoaa.rhs_vjp(tenoaa.make_grid(shape), sch, U, R)
    n = shape[d]
    ax = _ax(4, d)
    assembled = torch.zeros_like(U)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        gp = _piece_grid(shape, d, lo, hi, _halos(U, d, lo, hi, G))
        own, bars = tenoaa.rhs_vjp_halo(gp, sch, _piece(U, d, lo, hi), _piece(R, d, lo, hi))
        assembled.narrow(ax, lo, hi - lo).add_(own)
        for side in (0, 1):
            hb = bars[(d, side)]  # (G, nvar, plane)
            for r in range(1, G + 1):
                c = (lo - r) % n if side == 0 else (hi - 1 + r) % n
                sl = assembled.narrow(ax, c, 1)
                sl.add_(hb[r - 1].reshape(sl.shape))
    err = float((assembled - whole).abs().max() / whole.abs().max())
    print(case, splitting, "max rel difference of the assembled adjoint: %.2e" % err)
    assert err <= 1e-13


@pytest.mark.parametrize("case", ["3d_z", "2d_y"])
def test_pieces_step_adjoint_equals_whole(case):
    """The adjoint of a split SSP-RK3 step, composed from the pieces'
    tenoaa_rhs_vjp_halo with the stages' transposes (the chain
    tenoaa_step_vjp runs in one piece) and a reverse halo exchange per stage,
    equals the whole grid's tenoaa_step_vjp (limiter off; up to the order of
    the sums)."""
    shape, d, cuts = CUTS[case]
    order, G = 10, 5
    ax = _ax(4, d)
    n = shape[d]
    sch = tenoaa.make_scheme(order, tenoaa.LLF, 0)
    if len(shape) == 3:  # without the limiter: the random field without the near-vacuum sphere
        U0 = torch.from_numpy(inputs.grf_3d(max(shape), spheres=False)[:, :shape[2], :shape[1], :shape[0]].copy()).cuda()
    else:
        U0 = torch.from_numpy(_state(shape)).cuda()
    W = torch.randn(U0.shape, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(7))
    g = tenoaa.make_grid(shape)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    tenoaa.step(g, sch, U0.clone(), dt)
    whole = tenoaa.step_vjp(g, sch, U0, dt, W)
    spans = list(zip(cuts[:-1], cuts[1:]))
    grids = [_piece_grid(shape, d, lo, hi, _halos(U0, d, lo, hi, G)) for lo, hi in spans]

    def exchange(full):
        for (lo, hi), gp in zip(spans, grids):
            for key, v in _halos(full, d, lo, hi, G).items():
                gp._faces[key].copy_(v)

    def jt(state, seed):
        """(dL/dU at state)^T seed over the whole grid, assembled from the pieces."""
        exchange(state)
        out = torch.zeros_like(state)
        for (lo, hi), gp in zip(spans, grids):
            own, bars = tenoaa.rhs_vjp_halo(gp, sch, _piece(state, d, lo, hi), _piece(seed, d, lo, hi))
            out.narrow(ax, lo, hi - lo).add_(own)
            for side in (0, 1):
                for r in range(1, G + 1):
                    c = (lo - r) % n if side == 0 else (hi - 1 + r) % n
                    sl = out.narrow(ax, c, 1)
                    sl.add_(bars[(d, side)][r - 1].reshape(sl.shape))
        return out

    # forward stages of the pieces (the halos of each stage's input exchanged first)
    amax = None
    pieces = [_piece(U0, d, lo, hi) for lo, hi in spans]
    exchange(U0)
    amax = torch.stack([tenoaa.wave_speeds(gp, sch, u) for gp, u in zip(grids, pieces)]).max(dim=0).values
    dts = dt.clone()
    U1p = [torch.empty_like(u) for u in pieces]
    for gp, u, o in zip(grids, pieces, U1p):
        tenoaa.rk3_stage(gp, sch, 1, amax.contiguous(), dts, u, None, o)
    U1 = torch.cat(U1p, dim=ax)
    exchange(U1)
    U2p = [torch.empty_like(u) for u in pieces]
    for gp, u, s1, o in zip(grids, pieces, U1p, U2p):
        tenoaa.rk3_stage(gp, sch, 2, amax.contiguous(), dts, u, s1, o)
    U2 = torch.cat(U2p, dim=ax)
    # reverse: the transposes of the Shu-Osher stages
    h = float(dt.item())
    B3 = W
    B2 = (2.0 / 3.0) * B3 + ((2.0 / 3.0) * h) * jt(U2, B3)
    B1 = 0.25 * B2 + (0.25 * h) * jt(U1, B2)
    Bn = (1.0 / 3.0) * B3 + 0.75 * B2 + B1 + h * jt(U0, B1)
    err = float((Bn - whole).abs().max() / whole.abs().max())
    print(case, "split step adjoint against the whole grid's: max rel %.2e" % err)
    assert err <= 1e-13
