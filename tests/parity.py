"""Shared helpers for the GPU-vs-oracle parity tests."""
import numpy as np

# Tolerances.  Selection flags must agree exactly except at faces whose oracle
# decision margin |chi/C_T - 1| (or the C_T bucket margin) is within NEAR;
# fluxes and states within REL of each variable's largest magnitude, away from
# the two cells next to such a face.
NEAR = 1e-12
REL = 1e-11


def face_cells(grid, d, flat_face_idx):
    """Cells on both sides of faces (flat indices into direction d's face array)."""
    n = [grid.n[0], grid.n[1], grid.n[2]]
    m = list(n)
    periodic = grid.bc_lo[d] == 0
    m[d] = n[d] if periodic else n[d] + 1
    f = np.asarray(flat_face_idx)
    co = [f % m[0], (f // m[0]) % m[1], f // (m[0] * m[1])]
    out = []
    for shift in (-1, 0):
        c = [x.copy() for x in co]
        c[d] = c[d] + shift
        if periodic:
            c[d] %= n[d]
        ok = (c[d] >= 0) & (c[d] < n[d])
        out.append(((c[2] * n[1] + c[1]) * n[0] + c[0])[ok])
    return np.unique(np.concatenate(out))


def split_flags(grid, arr):
    """Per-direction views [nvar][2][faces] of a concatenated flag/margin array."""
    nd = grid.ndim
    nv = nd + 2
    out = []
    off = 0
    for d in range(nd):
        nf = grid.n[d] if grid.bc_lo[d] == 0 else grid.n[d] + 1
        t = nf
        for k in range(3):
            if k != d:
                t *= grid.n[k]
        out.append(arr[off: off + nv * 2 * t].reshape(nv, 2, t))
        off += nv * 2 * t
    return out


def compare_rhs(grid, d_gpu, d_or, fl_gpu=None, fl_or=None, mg_or=None, rel=REL):
    """Returns a report dict; raises AssertionError on a parity failure."""
    nv = grid.ndim + 2
    excl = np.zeros(d_or[0].size, bool)
    rep = {"near_faces": 0, "flag_mismatch": 0}
    if fl_gpu is not None:
        for d, (fg, fo, mo) in enumerate(zip(split_flags(grid, fl_gpu), split_flags(grid, fl_or),
                                             split_flags(grid, mg_or))):
            near = mo <= NEAR
            rep["near_faces"] += int(near.sum())
            bad = (fg != fo) & ~near
            rep["flag_mismatch"] += int(bad.sum())
            assert not bad.any(), "flag mismatch away from thresholds in direction %d at %s" % (
                d, np.argwhere(bad)[:5].tolist())
            faces = np.unique(np.nonzero(near.any(axis=(0, 1)))[0])
            if faces.size:
                excl[face_cells(grid, d, faces)] = True
    rep["bitwise_equal"] = int((d_gpu == d_or).sum())
    rep["elements"] = int(d_or.size)
    worst = 0.0
    for c in range(nv):
        a = d_gpu[c].reshape(-1)[~excl]
        b = d_or[c].reshape(-1)[~excl]
        scale = np.abs(d_or[c]).max()
        if scale == 0:
            scale = 1.0
        err = np.abs(a - b).max() / scale if a.size else 0.0
        worst = max(worst, err)
        assert err <= rel, "variable %d: max relative difference %.3e" % (c, err)
    rep["max_rel"] = worst
    return rep
