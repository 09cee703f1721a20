"""The batched persistent form: every problem of a batch must evolve bit for
bit as per-problem tenoaa_step calls do (which the parity tests tie to the
oracle), with its own dt, for any tile choice; plus a direct oracle check, the
autotune cache and re-binding of the packed state."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2109_14340_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import tenoaa  # noqa: E402

# (nx, ny) covering the three n_x buckets, tile remainders and thin grids
SIZES = [(64, 64), (67, 131), (200, 64), (131, 67), (96, 250), (321, 70), (64, 333), (170, 100), (400, 81)]
OUT = [tenoaa.BC_OUTFLOW, tenoaa.BC_OUTFLOW]


def _problems(sizes, bcs=None):
    grids, states = [], []
    for p, (nx, ny) in enumerate(sizes):
        bc = bcs[p] if bcs else OUT
        grids.append(tenoaa.make_grid((nx, ny), bc_lo=bc, bc_hi=bc))
        states.append(inputs.riemann_2d(nx, ny, p))
    return grids, states


def _per_problem(grids, states, scheme, nsteps, cfl=0.4):
    outs, dts = [], []
    for g, U0 in zip(grids, states):
        U = torch.from_numpy(U0).cuda()
        ws = tenoaa.workspace(g, scheme, tenoaa.WS_STEP)
        dt = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
        for n in range(nsteps):
            tenoaa.step(g, scheme, U, dt[n:n + 1], cfl=cfl, ws=ws)
        assert tenoaa.get_status(ws) == 0
        outs.append(U)
        dts.append(dt)
    return outs, torch.stack(dts)


def _batched(grids, states, scheme, nsteps, cfl=0.4, cache=None):
    plan = tenoaa.BatchPlan(grids, scheme, nsteps, cfl=cfl, tune_cache=cache)
    packed = plan.pack(states)
    dt = torch.zeros(len(grids) * nsteps, dtype=torch.float64, device="cuda")
    plan.run(packed, dt)
    st = plan.status()
    return plan, packed, dt.view(len(grids), nsteps), st


def _write_cache(path, scheme, grids, tx, ty, chunk, bpc):
    with open(path, "w") as f:
        f.write(json.dumps({"key": tenoaa.batch_cache_key(scheme, grids), "tile_x": tx, "tile_y": ty,
                            "chunk": chunk, "blocks_per_cu": bpc, "step_ms": 0.0}) + "\n")


def _assert_same(plan, packed, dtb, ref, dtr):
    assert torch.equal(dtb, dtr)
    for p, U in enumerate(ref):
        got = plan.unpack(packed, p)
        assert torch.equal(got, U), "problem %d differs (max %.3e)" % (p, float((got - U).abs().max()))


@pytest.mark.parametrize("tiles", ["defaults", "alternate"])
def test_batch_bitwise_equals_per_problem(tiles, tmp_path):
    sch = tenoaa.make_scheme(8, tenoaa.LLF, 0)
    grids, states = _problems(SIZES)
    nsteps = 4
    cache = None
    if tiles == "alternate":
        cache = str(tmp_path / "tune.jsonl")
        _write_cache(cache, sch, grids, [1, 1, 1], [1, 1, 1], 3, 1)
    plan, packed, dtb, st = _batched(grids, states, sch, nsteps, cache=cache)
    info = plan.info()
    print(tiles, info)
    if tiles == "alternate":
        assert info["chosen"] == "cache" and info["tile_x"] == [1, 1, 1] and info["chunk"] == 3
    assert st == [0] * len(grids)
    rs = plan.run_stats()
    print(rs)
    # every block waits at each of the 6 * nsteps barriers, and for less than it was resident
    assert 0.0 < rs["barrier_wait_share"] < 1.0 and rs["resident_s"] > 0.0 and rs["wait_per_barrier_us"] > 0.0
    assert 0.0 < rs["sweep_share"] < 1.0 and 0.0 < rs["cell_share"] < 1.0
    assert rs["barrier_wait_share"] + rs["sweep_share"] + rs["cell_share"] <= 1.0
    ref, dtr = _per_problem(grids, states, sch, nsteps)
    _assert_same(plan, packed, dtb, ref, dtr)


def test_batch_aa10_limiter_mixed_boundaries():
    sch = tenoaa.make_scheme(10, tenoaa.LLF, 1)
    sizes = [(64, 80), (150, 64), (96, 96), (330, 64)]
    bcs = [[tenoaa.BC_PERIODIC] * 2, [tenoaa.BC_SYMMETRY, tenoaa.BC_NOSLIP], OUT,
           [tenoaa.BC_NOSLIP, tenoaa.BC_OUTFLOW]]
    grids, states = _problems(sizes, bcs)
    plan, packed, dtb, st = _batched(grids, states, sch, 3, cfl=0.4)
    ref, dtr = _per_problem(grids, states, sch, 3, cfl=0.4)
    _assert_same(plan, packed, dtb, ref, dtr)


@pytest.mark.parametrize("splitting", [tenoaa.LLF, tenoaa.ROE])
def test_batch_teno12_bitwise_equals_per_problem(splitting):
    """TENO12-AA in the batched form (the S6 stencil), with the Roe flux too."""
    sch = tenoaa.make_scheme(12, splitting, 0)
    sizes = [(64, 64), (131, 67), (70, 150)]
    grids, states = _problems(sizes)
    plan, packed, dtb, st = _batched(grids, states, sch, 3)
    assert st == [0] * len(grids)
    ref, dtr = _per_problem(grids, states, sch, 3)
    _assert_same(plan, packed, dtb, ref, dtr)


@pytest.mark.parametrize("order", [8, 10])
def test_batch_prescribed_boundaries_bitwise(order):
    """Problems with Dirichlet and inflow sides (one value set for every step)
    beside walls and outflow: batched states and dt equal per-problem steps,
    whose CFL speeds include the ghost cells of those sides."""
    from tests.test_gpu_dirichlet import _face_values, _smooth
    D, I = tenoaa.BC_DIRICHLET, tenoaa.BC_INFLOW  # noqa: E741
    sch = tenoaa.make_scheme(order, tenoaa.LLF, 1)
    specs = [((64, 70), [D, tenoaa.BC_OUTFLOW], [I, D]), ((131, 67), [I, tenoaa.BC_NOSLIP], [D, I]),
             ((96, 96), [tenoaa.BC_OUTFLOW, D], [tenoaa.BC_SYMMETRY, D])]
    grids, states = [], []
    for p, ((nx, ny), lo, hi) in enumerate(specs):
        U = _smooth((nx, ny), 40 + p)  # Dirichlet reflections of it stay physical
        faces = _face_values(U, (nx, ny), lo, hi, 1.4, 1, seed=40 + p, order=order)
        if p == 1:
            # a fast inflow through the low x side: its ghost cells set the problem's CFL speed
            faces[(0, 0)][:, :, 1] = 2.5
            g_or = oracle.make_grid((nx, ny), [1.0 / nx, 1.0 / ny], lo, hi, bc_values=faces)
            g_walls = oracle.make_grid((nx, ny), [1.0 / nx, 1.0 / ny], [1, 1])
            assert oracle.dt(g_or, 1.4, 0.4, U) < oracle.dt(g_walls, 1.4, 0.4, U)
        grids.append(tenoaa.make_grid((nx, ny), bc_lo=lo, bc_hi=hi,
                                      bc_values={k: torch.from_numpy(v).cuda() for k, v in faces.items()}))
        states.append(U)
    plan, packed, dtb, st = _batched(grids, states, sch, 3)
    assert st == [0] * len(grids)
    ref, dtr = _per_problem(grids, states, sch, 3)
    _assert_same(plan, packed, dtb, ref, dtr)


def test_batch_rusanov_against_oracle():
    """Two small problems, two steps, compared with the oracle directly."""
    sch = tenoaa.make_scheme(8, tenoaa.RUSANOV, 0)
    sizes = [(64, 64), (72, 64)]
    grids, states = _problems(sizes)
    plan, packed, dtb, st = _batched(grids, states, sch, 2)
    for p, (nx, ny) in enumerate(sizes):
        g = oracle.make_grid((nx, ny), [1.0 / nx, 1.0 / ny], [1, 1])
        U = states[p]
        dts = []
        for _ in range(2):
            U, dt, _, _ = oracle.step(g, U, order=8, splitting=1, cfl=0.4, want_flags=True)
            dts.append(dt)
        got = tenoaa.to_numpy(plan.unpack(packed, p))
        err = np.abs(got - U).max() / np.abs(U).max()
        print("problem", p, "max rel vs oracle %.2e" % err, "dt", dts, tenoaa.to_numpy(dtb[p]))
        assert np.array_equal(tenoaa.to_numpy(dtb[p]), np.array(dts))
        assert err <= 1e-11


def test_batch_autotune_then_cache(tmp_path):
    sch = tenoaa.make_scheme(8, tenoaa.LLF, 0)
    grids, states = _problems(SIZES[:6])
    cache = str(tmp_path / "tune.jsonl")
    plan1, packed1, dt1, _ = _batched(grids, states, sch, 2, cache=cache)
    i1 = plan1.info()
    assert i1["chosen"] == "tuned"
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and json.loads(lines[0])["key"] == tenoaa.batch_cache_key(sch, grids)
    plan2, packed2, dt2, _ = _batched(grids, states, sch, 2, cache=cache)
    i2 = plan2.info()
    print(i1, i2, lines[0])
    assert i2["chosen"] == "cache"
    assert {k: i2[k] for k in ("tile_x", "tile_y", "chunk", "blocks_per_cu")} == \
        {k: i1[k] for k in ("tile_x", "tile_y", "chunk", "blocks_per_cu")}
    assert torch.equal(packed1, packed2) and torch.equal(dt1, dt2)
    assert len(open(cache).read().splitlines()) == 1


def test_batch_rebinds_state_between_runs():
    sch = tenoaa.make_scheme(8, tenoaa.LLF, 0)
    grids, states = _problems(SIZES[:3])
    plan = tenoaa.BatchPlan(grids, sch, 2)
    a = plan.pack(states)
    b = plan.pack(states)
    plan.run(a)
    plan.run(b)  # another buffer: the graph's kernel arguments are re-bound
    plan.run(a)  # and back: a has now advanced 4 steps
    assert plan.status() == [0] * 3
    ref, _ = _per_problem(grids, states, sch, 4)
    ref2, _ = _per_problem(grids, states, sch, 2)
    for p in range(3):
        assert torch.equal(plan.unpack(a, p), ref[p])
        assert torch.equal(plan.unpack(b, p), ref2[p])


def test_batch_reports_non_physical_problem():
    sch = tenoaa.make_scheme(8, tenoaa.LLF, 0)
    grids, states = _problems(SIZES[:3])
    bad = states[1].copy()
    bad[3, 0, 10:20, 10:20] = 0.0  # E = 0 with momentum: negative pressure
    plan = tenoaa.BatchPlan(grids, sch, 1)
    packed = plan.pack([states[0], bad, states[2]])
    plan.run(packed)
    assert plan.status() == [0, 1, 0]
    ref, _ = _per_problem([grids[0]], [states[0]], sch, 1)
    assert torch.equal(plan.unpack(packed, 0), ref[0])


def test_batch_barrier_time_limit_abandons_run(monkeypatch):
    """A barrier limit of zero forces the abandon path from the host: every
    block leaves, the status call reports ETIMEOUT, and a normal plan runs
    correctly afterwards."""
    sch = tenoaa.make_scheme(8, tenoaa.LLF, 0)
    grids, states = _problems(SIZES[:4])
    monkeypatch.setenv("TENOAA_BATCH_BARRIER_TIMEOUT_US", "0")
    plan = tenoaa.BatchPlan(grids, sch, 3)
    monkeypatch.delenv("TENOAA_BATCH_BARRIER_TIMEOUT_US")
    packed = plan.pack(states)
    plan.run(packed)
    with pytest.raises(tenoaa.TenoaaError, match="ETIMEOUT"):
        plan.status()
    plan.close()
    plan2, packed2, dtb, st = _batched(grids, states, sch, 3)
    assert st == [0] * 4
    ref, dtr = _per_problem(grids, states, sch, 3)
    _assert_same(plan2, packed2, dtb, ref, dtr)
