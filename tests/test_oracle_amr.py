"""Pins of the oracle's multilevel cycle (CPU only): the paper's level order,
prolongation exactness and divergence-freedom, restriction of prolongation,
and composite conservation / div B of the synchronised hierarchy."""

import os

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import inputs as I
from tests.amr_util import composite_divb, composite_sums, covered_mask

HERE = os.path.dirname(os.path.abspath(__file__))


def test_level_order_matches_paper():
    txt = [l for l in open(os.path.join(HERE, "golden", "level_order_3levels.txt")) if not l.startswith("#")]
    want = [int(x) for x in txt[0].split()]
    assert O.amr_level_order(3) == want
    # one coarse step of L levels advances level l exactly 2^l times
    for L in (1, 2, 4, 5):
        order = O.amr_level_order(L)
        assert [order.count(l) for l in range(L)] == [2 ** l for l in range(L)]


def _two_level(ndim):
    if ndim == 3:
        N0 = (16, 16, 16)
        grids = [(0, (0, 0, 0), (8, 16, 16)), (0, (8, 0, 0), (16, 16, 16)),
                 (1, (8, 8, 8), (16, 20, 18)), (1, (16, 8, 8), (24, 20, 18))]
    else:
        N0 = (16, 16)
        grids = [(0, (0, 0), (8, 16)), (0, (8, 0), (16, 16)), (1, (8, 8), (16, 20)), (1, (16, 8), (24, 20))]
    return N0, grids


def _linear_cons(ndim, N0, grids, coef):
    """Conserved fields linear in position on each level; face B linear and
    divergence-free (B = (a y, b z, c x) + const)."""
    out = []
    for (l, lo, hi) in grids:
        n = [hi[a] - lo[a] for a in range(ndim)]
        h = [1.0 / (N0[a] * 2 ** l) for a in range(ndim)]
        shp = O.interior_shapes(ndim, tuple(n))
        arrs = []
        for s in range(8):
            zz, yy, xx = np.meshgrid(*[np.arange(m) for m in shp[s]], indexing="ij")
            off = [0.5, 0.5, 0.5]
            if s >= 5 and (s - 5) < ndim:
                off[s - 5] = 0.0
            x = (lo[0] + xx + off[0]) * h[0]
            y = (lo[1] + yy + off[1]) * h[1]
            z = (lo[2] + zz + off[2]) * h[2] if ndim == 3 else 0 * xx
            if s < 5:
                v = coef[s][0] + coef[s][1] * x + coef[s][2] * y + coef[s][3] * z
            elif s == 5:
                v = 0.3 + 0.2 * y + 0.1 * z
            elif s == 6:
                v = -0.2 + 0.4 * z + 0.3 * x
            else:
                v = 0.1 + 0.5 * x - 0.2 * y
            arrs.append(np.asarray(v, dtype=np.float64))
        out.append(arrs)
    return out


@pytest.mark.parametrize("ndim", [2, 3])
def test_prolongation_exact_on_linear_data_and_divergence_free(ndim):
    N0, grids = _two_level(ndim)
    rng = np.random.default_rng(1)
    coef = rng.normal(size=(5, 4))
    coef[:, 0] += 3.0
    cons = _linear_cons(ndim, N0, grids, coef)
    g = 4
    banded = O.amr_fill(ndim, N0, 2, g, grids, cons, level=1, full=True)
    for gi, (l, lo, hi) in enumerate(grids):
        if l != 1:
            continue
        n = [hi[a] - lo[a] for a in range(ndim)]
        shp = O.banded_shapes(ndim, tuple(n), g)
        h = [1.0 / (N0[a] * 2) for a in range(ndim)]
        gz = g if ndim == 3 else 0
        for s in range(8):
            zz, yy, xx = np.meshgrid(*[np.arange(m) for m in shp[s]], indexing="ij")
            off = [0.5, 0.5, 0.5]
            if s >= 5 and (s - 5) < ndim:
                off[s - 5] = 0.0
            x = (lo[0] - g + xx + off[0]) * h[0]
            y = (lo[1] - g + yy + off[1]) * h[1]
            z = (lo[2] - gz + zz + off[2]) * h[2] if ndim == 3 else 0 * xx
            if s < 5:
                want = coef[s][0] + coef[s][1] * x + coef[s][2] * y + coef[s][3] * z
            elif s == 5:
                want = 0.3 + 0.2 * y + 0.1 * z
            elif s == 6:
                want = -0.2 + 0.4 * z + 0.3 * x
            else:
                want = 0.1 + 0.5 * x - 0.2 * y
            # periodic positions wrap; compare away from the domain edge only
            got = banded[gi][s]
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
        # every fine cell of the band is divergence free
        bx, by, bz = banded[gi][5], banded[gi][6], banded[gi][7]
        d = (bx[:, :, 1:] - bx[:, :, :-1]) / h[0] + (by[:, 1:, :] - by[:, :-1, :]) / h[1]
        if ndim == 3:
            d = d + (bz[1:] - bz[:-1]) / h[2]
        assert np.max(np.abs(d)) * h[0] < 1e-12


def test_restriction_of_prolongation_is_identity():
    """Fine cells and faces prolonged from a nonlinear coarse field average
    back to the coarse values (minmod slopes cancel in the mean)."""
    ndim = 3
    N0, grids = _two_level(ndim)
    fields = I.amr_fields(ndim, N0, 2, grids, seed=5, b_rms=0.3)
    cons = O.amr_run(ndim, N0, 2, 4, grids, fields, 0)[0]
    g = 4
    banded = O.amr_fill(ndim, N0, 2, g, grids, cons, level=1, full=True)
    # band of fine grid 2 at its low-x side covers coarse cells x = 2..3
    gi = 2
    l, lo, hi = grids[gi]
    fb = banded[gi]
    # coarse cell (3, 5, 5) lies in the band (fine x = 6..7) below the grid
    cx, cy, cz = 3, 5, 5
    fi = [2 * cx - lo[0] + g, 2 * cy - lo[1] + g, 2 * cz - lo[2] + g]
    coarse = cons[0]
    for s in range(5):
        m = fb[s][fi[2]:fi[2] + 2, fi[1]:fi[1] + 2, fi[0]:fi[0] + 2].mean()
        assert abs(m - coarse[s][cz, cy, cx]) <= 1e-14 * max(1.0, abs(m))
    # x-face at coarse index 3: mean of the 4 fine faces at fine index 6
    m = fb[5][fi[2]:fi[2] + 2, fi[1]:fi[1] + 2, fi[0]].mean()
    assert abs(m - coarse[5][cz, cy, cx]) < 1e-14


@pytest.mark.parametrize("ndim,N0,ext,seed", [(3, (24, 24, 24), (8, 16), 11), (2, (32, 32), (8, 16), 4)])
def test_composite_conservation_and_divb(ndim, N0, ext, seed):
    L = 3
    grids = I.amr_hierarchy(ndim, N0, L, seed=seed, ext=ext)
    assert sum(1 for g in grids if g[0] == 2) >= 1
    fields = I.amr_fields(ndim, N0, L, grids, seed=3, b_rms=0.3)
    s0, _ = O.amr_run(ndim, N0, L, 4, grids, fields, 0)
    s2, dts = O.amr_run(ndim, N0, L, 4, grids, fields, 2)
    c0 = composite_sums(ndim, N0, grids, s0)
    c2 = composite_sums(ndim, N0, grids, s2)
    assert np.all(np.abs(c2 - c0) <= 1e-13 * (np.abs(c0) + 1.0)), (c2 - c0)
    assert composite_divb(ndim, N0, grids, s0) < 1e-12
    assert composite_divb(ndim, N0, grids, s2) < 1e-12
    # the hierarchy evolved and fine data differ from the initial state
    assert np.max(np.abs(s2[-1][0] - s0[-1][0])) > 1e-4


def test_sync_restricts_covered_cells():
    ndim, N0, L = 3, (24, 24, 24), 2
    grids = I.amr_hierarchy(ndim, N0, L, seed=11, ext=(8, 16))
    fields = I.amr_fields(ndim, N0, L, grids, seed=3, b_rms=0.3)
    s1, _ = O.amr_run(ndim, N0, L, 4, grids, fields, 1)
    # every covered coarse cell equals the mean of its fine cells
    fine = {gi: g for gi, g in enumerate(grids) if g[0] == 1}
    for gi, (l, lo, hi) in enumerate(grids):
        if l != 0:
            continue
        m = covered_mask(ndim, grids, gi)
        for (k, j, i) in zip(*np.nonzero(m)):
            p = (lo[0] + i, lo[1] + j, lo[2] + k)
            for fgi, (fl, flo, fhi) in fine.items():
                if all(flo[a] <= 2 * p[a] < fhi[a] for a in range(3)):
                    f = s1[fgi][0]
                    q = [2 * p[a] - flo[a] for a in range(3)]
                    mean = f[q[2]:q[2] + 2, q[1]:q[1] + 2, q[0]:q[0] + 2].mean()
                    assert abs(s1[gi][0][k, j, i] - mean) < 1e-14
                    break


@pytest.mark.parametrize("skip,breaks", [(1, "conservation"), (2, "divb"), (4, "divb")])
def test_planted_sync_omissions_are_caught(skip, breaks):
    """Each part of the synchronisation is needed: dropping the reflux breaks
    composite conservation, dropping the EMF correction or the restriction
    breaks composite div B (mistakes planted in the oracle, on the CPU)."""
    ndim, N0, L = 3, (24, 24, 24), 3
    grids = I.amr_hierarchy(ndim, N0, L, seed=11, ext=(8, 16))
    fields = I.amr_fields(ndim, N0, L, grids, seed=3, b_rms=0.3)
    s0, _ = O.amr_run(ndim, N0, L, 4, grids, fields, 0)
    O.lib().orc_amr_set_skip(skip)
    try:
        s2, _ = O.amr_run(ndim, N0, L, 4, grids, fields, 2)
    finally:
        O.lib().orc_amr_set_skip(0)
    if breaks == "conservation":
        c0 = composite_sums(ndim, N0, grids, s0)
        c2 = composite_sums(ndim, N0, grids, s2)
        assert np.any(np.abs(c2 - c0) > 1e-10 * (np.abs(c0) + 1.0))
    else:
        assert composite_divb(ndim, N0, grids, s2) > 1e-8
