"""Algorithmic operation count of one face reconstruction (one face of one
sweep direction, every characteristic field, both split sides).

Counting rule: +, -, *, / and sqrt count 1, fma counts 2; comparisons,
min/max, abs, floor and selects count 0.  The count follows the formulas the
library evaluates (one reciprocal per gamma, one division for the eta
minimum, the sums of squares of the large-stencil indicators) and only the
work on the path a face actually takes: a large stencil's indicator is
counted only when the cascade reaches it.  Per-cell work (primitives and
physical flux) is counted once per cell and direction, not per halo copy.
"""

# non-zero lower-triangular factors of the sums of squares (tenoaa_sos.h)
SOS_NNZ = {10: 41, 8: 25, 6: 13}


def sos_cost(r):
    """Difference table + factor products + weighted squares of one indicator."""
    return r * (r - 1) // 2 + 2 * SOS_NNZ[r] + 3 * (r - 1)


ETA_CT = 40 + 11        # eta_j, their minimum, m, g(m), [beta]
SMALL = 45              # three small-stencil indicators, gammas, their sum
TEST = 6 + 2            # gamma_p and the threshold product
FLUX = {10: 19, 8: 15, 6: 11}
FALLBACK = 21           # three candidate fluxes and the weighted sum


def scalar_cost(order, sel):
    """sel: 5, 4, 3 = large stencil chosen, 0 = fallback."""
    larges = [10, 8, 6] if order == 10 else [8, 6]
    sel_r = {5: 10, 4: 8, 3: 6}.get(sel, 0)
    c = ETA_CT + SMALL
    for r in larges:
        c += sos_cost(r) + TEST
        if r == sel_r:
            return c + FLUX[r]
    return c + FALLBACK


def face_cost(ndim, order, splitting=0, limiter=False):
    """Per-face work outside the scalar reconstructions."""
    nv = ndim + 2
    W = order
    cell = 4 * ndim + 12
    roe = 27 + 8 * ndim
    entropy_row = ndim + 1
    alpha = 2 * W if splitting == 0 else W
    proj = 3 * W * 2 * (2 * nv - 1) + (ndim - 1) * W * 4
    split = 6 * W * nv
    sides = nv
    back = nv + (nv - 1) * 2 * nv
    lim = 0
    if limiter:
        press = 3 * ndim + 3
        lim = 2 + 5 * nv + 10 + 4 * (2 * nv + press)
    return cell + roe + entropy_row + alpha + proj + split + sides + back + lim


def sweep_flops(ndim, order, sel_counts, nfaces, splitting=0, limiter=False):
    """Total for one sweep: sel_counts maps 5/4/3/0 to the number of scalar
    reconstructions (fields x sides x faces) that took that path."""
    tot = face_cost(ndim, order, splitting, limiter) * nfaces
    for sel, cnt in sel_counts.items():
        tot += scalar_cost(order, sel) * cnt
    return tot


def smooth_face_flops(ndim, order, splitting=0, limiter=False):
    """Work of a face on which every reconstruction takes the largest stencil."""
    nv = ndim + 2
    big = 5 if order == 10 else 4
    return face_cost(ndim, order, splitting, limiter) + 2 * nv * scalar_cost(order, big)
