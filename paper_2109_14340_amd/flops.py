"""Algorithmic operation count of one face reconstruction (one face of one
sweep direction, every characteristic field, both split sides).

Counting rule: +, -, *, / and sqrt count 1, fma counts 2; comparisons,
min/max, abs, floor and selects count 0.  The count follows the formulas the
library evaluates (one reciprocal per gamma, one division for the eta
minimum, the sums of squares of the large-stencil indicators) and only the
work on the path a face actually takes: a large stencil's indicator is
counted only when the cascade reaches it.  Products by a coefficient that is
0 or 1 (the unit diagonal of the sum-of-squares factors, the zero and unit
entries of the shear fields' eigenvectors) are not counted, and a first
difference is counted once however many indicators use it.  Per-cell work
(primitives, physical flux, the split's factor 1/2) is counted once per cell
and direction, not per halo copy.
"""

# non-zero entries below the unit diagonal of the sum-of-squares factors
# (tenoaa_sos.h): stencil width -> count
SOS_NNZ = {12: 55, 10: 36, 8: 21, 6: 10}

# first differences f_{j+1} - f_j, j = -2..2, that the cut-off's eta and the
# small-stencil indicators use; the first (largest) large stencil's first
# differences contain them, and every nested stencil's are among its
SHARED_DIFFS = 5


def sos_cost(r, shared=0):
    """First differences + factor products + weighted squares of one indicator
    (`shared` first differences already computed)."""
    return (r - 1) - shared + 2 * SOS_NNZ[r] + 3 * (r - 1)


ETA_CT = 40 + 11        # eta_j, their minimum, m, g(m), [beta]
SMALL = 45              # three small-stencil indicators, gammas, their sum
TEST = 6 + 2            # gamma_p and the threshold product
FLUX = {12: 23, 10: 19, 8: 15, 6: 11}
FALLBACK = 21           # three candidate fluxes and the weighted sum


def large_stencils(order):
    return {12: [12, 10, 8, 6], 10: [10, 8, 6], 8: [8, 6]}[order]


def scalar_cost(order, sel):
    """sel: 6, 5, 4, 3 = large stencil chosen, 0 = fallback."""
    sel_r = {6: 12, 5: 10, 4: 8, 3: 6}.get(sel, 0)
    c = ETA_CT + SMALL
    for k, r in enumerate(large_stencils(order)):
        c += sos_cost(r, SHARED_DIFFS if k == 0 else r - 1) + TEST
        if r == sel_r:
            return c + FLUX[r]
    return c + FALLBACK


def face_cost(ndim, order, splitting=0, limiter=False):
    """Per-face work outside the scalar reconstructions."""
    nv = ndim + 2
    W = order
    cell = 4 * ndim + 12 + 2 * nv   # primitives, flux, halving of state and flux
    roe = 27 + 8 * ndim
    entropy_row = ndim + 1
    alpha = 2 * W if splitting == 0 else W
    # acoustic and entropy rows: 1 product + (nv - 1) fma, state and flux;
    # shear rows: -u_t rho + m_t (a product and a sum), state and flux
    proj = 3 * W * 2 * (2 * nv - 1) + (ndim - 1) * W * 4
    split = 2 * 2 * W * nv          # one fma per side on the halved projections
    sides = nv
    # R column of the first acoustic field (its unit density entry is free),
    # the entropy and second acoustic columns (unit density entry: an add),
    # the shear columns (a unit momentum entry and the energy entry)
    back = (ndim + 1) + 2 * (2 * ndim + 3) + (ndim - 1) * 3
    lim = 0
    if limiter:
        press = 3 * ndim + 3
        lim = 2 + 5 * nv + 10 + 4 * (2 * nv + press)
    return cell + roe + entropy_row + alpha + proj + split + sides + back + lim


def sweep_flops(ndim, order, sel_counts, nfaces, splitting=0, limiter=False):
    """Total for one sweep: sel_counts maps 6/5/4/3/0 to the number of scalar
    reconstructions (fields x sides x faces) that took that path."""
    tot = face_cost(ndim, order, splitting, limiter) * nfaces
    for sel, cnt in sel_counts.items():
        tot += scalar_cost(order, sel) * cnt
    return tot


def smooth_face_flops(ndim, order, splitting=0, limiter=False):
    """Work of a face on which every reconstruction takes the largest stencil."""
    nv = ndim + 2
    big = {12: 6, 10: 5, 8: 4}[order]
    return face_cost(ndim, order, splitting, limiter) + 2 * nv * scalar_cost(order, big)
