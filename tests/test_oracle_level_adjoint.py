"""Pins of the oracle's adjoint of one substep of a whole fine level (CPU
only): the batched level map is the same-level band copy (prolonged band
elements held constant) followed by a band-2 step of every grid.  The
vector-Jacobian product from the tape is checked against centred finite
differences of the oracle's plain forward map (the full band fill of the
perturbed level followed by its banded steps), along directions supported
on the selected grid and on a neighbour that feeds it only through the band
copy, so a missing or misplaced fold of band adjoints fails."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import inputs as I

GAMMA = 5.0 / 3.0
N0 = (16, 16, 16)
G = 4


def _case():
    grids = [(0, (0, 0, 0), (8, 16, 16)), (0, (8, 0, 0), (16, 16, 16)),
             (1, (8, 8, 8), (16, 20, 18)), (1, (16, 8, 8), (24, 20, 18)), (1, (8, 20, 8), (24, 26, 14)),
             (1, (24, 24, 24), (30, 30, 30))]
    fields = I.amr_fields(3, N0, 2, grids, seed=21, b_rms=0.3, p_amp=0.1)
    cons, _ = O.amr_run(3, N0, 2, G, grids, fields, 0)
    _, dts = O.amr_run(3, N0, 2, G, grids, fields, 1)
    return grids, cons, dts[0] / 2.0


def _level(grids, lev):
    idx = [i for i, (l, _, _) in enumerate(grids) if l == lev]
    boxes = [(grids[i][1], grids[i][2]) for i in idx]
    return idx, boxes


def _smooth_dir(shapes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for sh in shapes:
        zz, yy, xx = np.meshgrid(*[np.arange(m) for m in sh], indexing="ij")
        k = rng.uniform(0.2, 0.6, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        out.append(np.sin(k[0] * xx + k[1] * yy + k[2] * zz + ph))
    return out


def _forward_J(grids, cons, lev_idx, boxes, dt, sel, lam_out, pert):
    """sum over selected grids of <lam_out, own outputs> of the level map
    applied to the level's interiors plus `pert` (per level grid 8 arrays)."""
    c2 = [list(c) for c in cons]
    for t, gi in enumerate(lev_idx):
        c2[gi] = [np.asarray(a) + p for a, p in zip(cons[gi], pert[t])]
    banded = O.amr_fill(3, N0, 2, G, grids, c2, 1, True)
    J = 0.0
    dx = [1.0 / (2 * n) for n in N0]
    for t, s_idx in enumerate(sel):
        gi = lev_idx[s_idx]
        lo, hi = boxes[s_idx]
        n = tuple(hi[a] - lo[a] for a in range(3))
        out = O.step_banded(3, n, G, 2, GAMMA, dx, dt, banded[gi])
        own = O.interior_from_banded(3, n, G, out)
        J += sum(float(np.sum(a * b)) for a, b in zip(own, lam_out[t]))
    return J


def test_level_vjp_against_finite_differences():
    grids, cons, dt = _case()
    lev_idx, boxes = _level(grids, 1)
    banded = O.amr_fill(3, N0, 2, G, grids, cons, 1, True)
    banded_lev = [banded[i] for i in lev_idx]
    sel = [0]
    rng = np.random.default_rng(5)
    shapes = [O.interior_shapes(3, tuple(hi[a] - lo[a] for a in range(3))) for lo, hi in boxes]
    lam_out = [[rng.standard_normal(sh) for sh in shapes[0]]]
    Nl = tuple(2 * n for n in N0)
    dx = [1.0 / n for n in Nl]
    lam_in = O.level_vjp(3, Nl, G, GAMMA, dx, dt, boxes, banded_lev, sel, lam_out)
    # the neighbours (level grids 1 and 2) feed grid 0 only through grid 0's
    # band; grid 3 lies outside it
    assert max(np.abs(a).max() for a in lam_in[1]) > 0 and max(np.abs(a).max() for a in lam_in[2]) > 0
    assert max(np.abs(a).max() for a in lam_in[3]) == 0
    # one field at a time on its own scale; a minmod kink inside +-eps
    # spoils one difference, so the best of three step sizes is taken
    scale = 1e-2 * sum(abs(float(np.sum(a))) for a in lam_out[0])
    for which in (0, 1, 2, 3):
        for s in range(8):
            d = [[np.zeros(sh) for sh in shapes[t]] for t in range(len(boxes))]
            sc = max(np.abs(np.asarray(cons[lev_idx[which]][s])).max(), 1e-3)
            d[which][s] = _smooth_dir(shapes[which], seed=10 + which)[s] * sc
            adj = sum(float(np.sum(a * b)) for t in range(len(boxes)) for a, b in zip(lam_in[t], d[t]))
            best = np.inf
            for eps in (1e-5, 1e-6, 1e-7):
                jp = _forward_J(grids, cons, lev_idx, boxes, dt, sel, lam_out, [[eps * x for x in y] for y in d])
                jm = _forward_J(grids, cons, lev_idx, boxes, dt, sel, lam_out, [[-eps * x for x in y] for y in d])
                best = min(best, abs((jp - jm) / (2 * eps) - adj))
            if which == 3:
                # outside grid 0's band: no dependence at all
                assert adj == 0.0 and best < 1e-9
                continue
            assert best <= 1e-6 * (abs(adj) + scale), (which, s, adj, best)


def test_level_vjp_single_periodic_grid_is_step_vjp():
    """A level made of one grid covering the periodic domain: every band
    element is a copy of the grid's own interior, so the level map is the
    single-grid periodic step."""
    n = (10, 8, 12)
    ic = I.smooth_mhd(3, n, seed=31, b_rms=0.3, p_amp=0.1)
    U = O.conserved_interior(ic, GAMMA)
    rng = np.random.default_rng(6)
    lam_out = [rng.standard_normal(np.asarray(u).shape) for u in U]
    want = O.step_vjp(3, n, GAMMA, 2e-3, U, lam_out)
    banded = O.fill_banded(3, n, 2, (0, 0, 0), O.banded_from_interior(3, n, 2, U))
    got = O.level_vjp(3, n, 2, GAMMA, ic["dx"], 2e-3, [((0, 0, 0), n)], [banded], [0], [lam_out])[0]
    # the periodic duplicate face n is an own element here and a band copy
    # of face 0 in step_vjp: compare face 0 + face n with step_vjp's face 0
    for s in range(8):
        g = np.array(got[s])
        if s >= 5:
            ax = 2 - (s - 5)
            sl0 = [slice(None)] * 3
            sln = [slice(None)] * 3
            sl0[ax] = 0
            sln[ax] = -1
            g[tuple(sl0)] += g[tuple(sln)]
            g[tuple(sln)] = 0.0
        np.testing.assert_allclose(g, want[s], rtol=0, atol=1e-12 * (np.abs(want[s]).max() + 1e-300))
