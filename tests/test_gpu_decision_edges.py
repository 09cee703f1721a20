"""Decisions just outside the near band.  Scalar windows built so that the
first (S5) or the second (S4) large-stencil test of one face lies about 1e-8
(relative distance of chi to C_T) on either side of its threshold, at the
C_T buckets K = 14 and K = 11 (Sec. 3.3, 3.4), sit in the periodic grid of
the scalar advection test (Sec. 5.1).  The GPU evaluates these decisions in
its own forms (indicators as sums of squares over first differences, the test
as S b^7 <= 1/C_T - 1, contracted multiply-adds), so it must still take the
oracle's decision at 1e-8 from the threshold, far outside the rounding of
either side: one SSP-RK3 step with dt = 1e-11 dx (every stage state within
~1e-11 of the first, moving chi by ~1e-9, so every stage meets the same
decisions) equals the oracle's bit for bit on both sides of the threshold,
and the two sides' steps differ where the decision acts, so a wrong decision
would show."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2109_14340_amd import tenoaa  # noqa: E402

ORDER, N, I = 10, 64, 31  # the face i + 1/2 with i = 31 reads cells 27 .. 36


def _base(kind):
    if kind == "smooth":  # K = 14
        return lambda x: np.sin(0.3 * x)
    return lambda x: np.sin(0.3 * x) + 0.008 * np.cos(2.1 * x)  # K = 11


def _grid(kind, a, b):
    """The base continued over the periodic grid, with a added to cell i + 5
    (in S5 only) and b to cell i + 4 (in S5 and S4): neither is read by the
    small stencils or the cut-off's differences of this face."""
    u = _base(kind)(np.arange(N, dtype=np.float64) - (I - 4))
    u[I + 5] += a
    u[I + 4] += b
    return u


def _window(u, i):
    return u[[(i - ORDER // 2 + 1 + j) % N for j in range(ORDER)]]


def _flip(kind, level):
    """Bisection (oracle only) for the parameter where the face's stencil
    leaves S5 (level 5: a grows) or S4 (level 4: b grows, a = 20 keeps S5
    out); returns (parameter builder, flip value, selector before, after)."""
    if level == 5:
        make, keep, lo, hi = (lambda p: _grid(kind, p, 0.0)), 3, 0.0, 50.0
    else:
        make, keep, lo, hi = (lambda p: _grid(kind, 20.0, p)), 2, 0.0, 5.0
    sel = lambda p: oracle.teno(ORDER, _window(make(p), I))[1] & 3
    assert sel(lo) == keep and sel(hi) != keep
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sel(mid) == keep:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15 * hi:
            break
    return make, lo, keep


@pytest.mark.parametrize("kind,level,kbucket", [("smooth", 5, 14), ("bumpy", 5, 11), ("bumpy", 4, 11)])
def test_decisions_1e8_from_threshold_match_oracle(kind, level, kbucket):
    make, p0, keep = _flip(kind, level)
    dx = 1.0 / N
    dt = 1e-11 * dx
    steps = {}
    for side, rel in (("in", -1e-9), ("out", 1e-9)):
        u0 = make(p0 * (1.0 + rel))
        _, flag, margin = oracle.teno(ORDER, _window(u0, I))
        assert ((flag & 3) == keep) == (side == "in")
        assert (flag >> 5) + 7 == kbucket
        assert 1e-10 < margin < 1e-6, margin
        # every other face far from its thresholds
        assert min(oracle.teno(ORDER, _window(u0, i))[2] for i in range(N) if i != I) > 1e-6
        want, flags3 = oracle.advect_step(ORDER, u0, dx, dt)
        assert len({int(flags3[st * N + I]) & 3 for st in range(3)}) == 1
        d = torch.from_numpy(u0.copy()).cuda()
        tenoaa.advect(ORDER, d, dx, dt, 1)
        got = d.cpu().numpy()
        assert np.array_equal(got, want), "side %s: max diff %.3e" % (side, np.abs(got - want).max())
        steps[side] = want
    # the decision moves the face's flux: cell I (left of the face, whose own
    # inputs are the same on both sides) changes by tens of ulps
    ulp = np.spacing(abs(steps["in"][I]))
    assert abs(steps["in"][I] - steps["out"][I]) > 20 * ulp
