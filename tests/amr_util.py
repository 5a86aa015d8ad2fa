"""Hierarchy bookkeeping used by the AMR tests (coverage masks, composite
sums).  Plain numpy over the grid list; no scheme arithmetic."""

import numpy as np


def covered_mask(ndim, grids, gi, R=2):
    l, lo, hi = grids[gi]
    n = [hi[a] - lo[a] for a in range(ndim)]
    shape = (n[2] if ndim == 3 else 1, n[1], n[0])
    m = np.zeros(shape, dtype=bool)
    for (lf, flo, fhi) in grids:
        if lf != l + 1:
            continue
        clo = [flo[a] // R for a in range(ndim)]
        chi = [fhi[a] // R for a in range(ndim)]
        a0 = [max(clo[a], lo[a]) - lo[a] for a in range(ndim)]
        a1 = [min(chi[a], hi[a]) - lo[a] for a in range(ndim)]
        if any(a1[a] <= a0[a] for a in range(ndim)):
            continue
        if ndim == 3:
            m[a0[2]:a1[2], a0[1]:a1[1], a0[0]:a1[0]] = True
        else:
            m[0, a0[1]:a1[1], a0[0]:a1[0]] = True
    return m


def composite_sums(ndim, N0, grids, states, R=2):
    """Sum of U dV over uncovered cells of every level (5 conserved fields)."""
    tot = np.zeros(5)
    for gi, (l, lo, hi) in enumerate(grids):
        dv = 1.0
        for a in range(ndim):
            dv /= N0[a] * R ** l
        unc = ~covered_mask(ndim, grids, gi, R)
        for s in range(5):
            tot[s] += np.sum(states[gi][s][unc]) * dv
    return tot


def composite_divb(ndim, N0, grids, states, R=2):
    """max |div B| dx / max |B| over uncovered cells of every level."""
    worst = 0.0
    bmax = max(np.max(np.abs(states[gi][s])) for gi in range(len(grids)) for s in (5, 6, 7))
    for gi, (l, lo, hi) in enumerate(grids):
        h = [1.0 / (N0[a] * R ** l) for a in range(ndim)]
        bx, by, bz = states[gi][5], states[gi][6], states[gi][7]
        d = (bx[:, :, 1:] - bx[:, :, :-1]) / h[0] + (by[:, 1:, :] - by[:, :-1, :]) / h[1]
        if ndim == 3:
            d = d + (bz[1:] - bz[:-1]) / h[2]
        unc = ~covered_mask(ndim, grids, gi, R)
        if np.any(unc):
            worst = max(worst, float(np.max(np.abs(d[unc]))) * min(h) / bmax)
    return worst
