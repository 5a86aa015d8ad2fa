"""Pins of the oracle's regridding (flags, nesting, Berger-Rigoutsos) and of
its (O)verlap transfer from a previous iteration of grids (Sec. 2 and 4 of
the paper: successive grid iterations, overlap connections)."""

import numpy as np
import pytest

import oracle as O
from oracle import regrid as RG
from paper_1110_1616_amd import inputs as I
from tests.amr_util import composite_divb, composite_sums

pytestmark = pytest.mark.filterwarnings("ignore")


# ------------------------------------------------------------ clustering
def _check_cover(mask, adm, boxes, eff, maxbox):
    nd = mask.ndim
    cov = np.zeros(mask.shape, dtype=np.int32)
    for lo, hi in boxes:
        sl = tuple(slice(lo[a], hi[a]) for a in range(nd))
        ext = [hi[a] - lo[a] for a in range(nd)]
        vol = int(np.prod(ext))
        cov[sl] += 1
        cnt = int(mask[sl].sum())
        assert vol == 1 or (cnt >= eff * vol and max(ext) <= maxbox and adm[sl].all())
    assert cov.max() <= 1, "boxes overlap"
    assert np.all(cov[mask] == 1), "a flagged cell is not covered"


def test_cluster_one_block_is_one_box():
    m = np.zeros((32, 32), dtype=bool)
    m[5:13, 9:20] = True
    assert RG.cluster(m, np.ones_like(m), 0.7, 16) == [((5, 9), (13, 20))]


def test_cluster_hole_splits_separated_blocks():
    m = np.zeros((32, 16), dtype=bool)
    m[2:6, 3:9] = True
    m[20:26, 4:7] = True
    boxes = RG.cluster(m, np.ones_like(m), 0.7, 32)
    assert boxes == [((2, 3), (6, 9)), ((20, 4), (26, 7))]


def test_cluster_l_shape_cut_at_the_inflection():
    """L made of an 8x2 and a 2x8 bar: signature along x is [8,8,2,2,2,2,2,2],
    second difference -6 at 1 and +6 at 2, so the cut falls at x = 2 (the same
    strength along y; x wins the tie as the lower axis of equal extent)."""
    m = np.zeros((16, 16), dtype=bool)
    m[0:8, 0:2] = True
    m[0:2, 0:8] = True
    boxes = RG.cluster(m, np.ones_like(m), 0.7, 16)
    assert boxes == [((0, 0), (2, 8)), ((2, 0), (8, 2))]


def test_cluster_bisects_when_too_large():
    m = np.ones((40, 8), dtype=bool)
    boxes = RG.cluster(m, np.ones_like(m), 0.7, 16)
    # 40 -> 20 + 20 -> 10 + 10 + 10 + 10 (halving the longest axis)
    assert boxes == [((0, 0), (10, 8)), ((10, 0), (20, 8)), ((20, 0), (30, 8)), ((30, 0), (40, 8))]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cluster_invariants_random_3d(seed):
    rng = np.random.default_rng(seed)
    m = np.zeros((28, 24, 20), dtype=bool)
    for _ in range(6):
        c = rng.integers(0, [28, 24, 20])
        r = rng.integers(1, 5, size=3)
        m[max(c[0] - r[0], 0):c[0] + r[0], max(c[1] - r[1], 0):c[1] + r[1], max(c[2] - r[2], 0):c[2] + r[2]] = True
    m |= rng.random(m.shape) < 0.01
    adm = np.ones_like(m)
    adm[:, :, 17:] = False
    m &= adm
    boxes = RG.cluster(m, adm, 0.7, 12)
    _check_cover(m, adm, boxes, 0.7, 12)


# ---------------------------------------------------------------- nesting
def test_nestable_region_of_one_grid():
    grids = [(0, (0, 0, 0), (16, 16, 16)), (1, (8, 8, 8), (24, 24, 24))]
    adm = RG.nestable(3, (16, 16, 16), 4, grids, 1)
    want = np.zeros((32, 32, 32), dtype=bool)
    want[11:21, 11:21, 11:21] = True
    assert np.array_equal(adm, want)


def test_nestable_level0_periodic_is_everything():
    grids = [(0, (0, 0), (8, 16)), (0, (8, 0), (16, 16))]
    assert RG.nestable(2, (16, 16), 4, grids, 0).all()


def test_forced_cells_of_a_level2_grid():
    grids = [(2, (40, 40), (56, 48))]
    f = RG.forced(2, (32, 32), 4, grids, 0)
    # level-1 cells [20-3, 28+3) x [20-3, 24+3) -> level-0 [8, 16) x [8, 14)
    want = np.zeros((32, 32), dtype=bool)
    want[8:16, 8:14] = True
    assert np.array_equal(f, want)


# ------------------------------------------------------------------ flags
def test_flags_of_a_y_profile_match_the_closed_form():
    """rho = 1 + a sin(2 pi y) on a 2-grid periodic level 0: the relative
    centred jump is |cos(2 pi y) sin(2 pi h)| a / (1 + a sin(2 pi y) cos(2 pi h))
    with h the cell width; x and the grid split play no part."""
    n = (24, 32)
    grids = [(0, (0, 0), (12, 32)), (0, (12, 0), (24, 32))]
    a, h = 0.3, 1.0 / n[1]
    y = (np.arange(n[1]) + 0.5) * h
    rel = a * np.abs(np.cos(2 * np.pi * y) * np.sin(2 * np.pi * h)) / (1 + a * np.sin(2 * np.pi * y) * np.cos(2 * np.pi * h))
    u = np.unique(np.round(rel, 12))
    theta = 0.5 * (u[len(u) // 2] + u[len(u) // 2 + 1])  # between two distinct values: no near tie
    assert np.min(np.abs(rel - theta)) > 1e-6
    cons = []
    for (l, lo, hi) in grids:
        nx = hi[0] - lo[0]
        rho = np.broadcast_to((1 + a * np.sin(2 * np.pi * y))[None, :, None], (1, n[1], nx)).copy()
        z = np.zeros((1, n[1], nx))
        cons.append([rho, z, z, z, np.ones_like(z) * 2.0, np.zeros((1, n[1], nx + 1)), np.zeros((1, n[1] + 1, nx)), z])
    f = RG.flags(2, n, 1, 4, grids, cons, 0, theta)
    want = np.broadcast_to((rel > theta)[None, :], (n[0], n[1]))
    assert np.array_equal(f, want)


# --------------------------------------------------------------- overlap
def _cons(ndim, N0, L, grids, fields):
    return O.amr_run(ndim, N0, L, 4, grids, fields, 0)[0]


@pytest.mark.parametrize("ndim", [2, 3])
def test_overlap_onto_the_same_grids_is_the_identity(ndim):
    N0 = (24, 24, 24)[:ndim]
    grids = I.amr_hierarchy(ndim, N0, 3, seed=11, ext=(8, 16))
    fields = I.amr_fields(ndim, N0, 3, grids, seed=3)
    cons = _cons(ndim, N0, 3, grids, fields)
    new = O.amr_overlap(ndim, N0, 3, 4, grids, cons, grids)
    for a, b in zip(new, cons):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def _linear_state(ndim, N0, grids):
    """Cell means and face means of linear fields with a divergence-free
    linear B (each component independent of its own coordinate)."""
    out = []
    for (l, lo, hi) in grids:
        n = [hi[a] - lo[a] for a in range(ndim)]
        h = [1.0 / (N0[a] * 2 ** l) for a in range(ndim)]
        nz = n[2] if ndim == 3 else 1

        def coords(shift):
            ax = []
            for a in range(3):
                if a < ndim:
                    m = n[a] + (1 if shift == a else 0)
                    off = 0.0 if shift == a else 0.5
                    ax.append((lo[a] + np.arange(m) + off) * h[a])
                else:
                    ax.append(np.array([0.5]))
            zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
            return xx, yy, zz

        x, y, z = coords(-1)
        rho = 1.0 + 0.3 * x - 0.2 * y + 0.1 * z
        mx, my, mz = 0.1 * y, -0.2 * z + 0.05 * x, 0.3 * x
        E = 2.0 + 0.4 * x + 0.1 * y - 0.3 * z
        xb, yb, zb = coords(0)
        bx = 0.5 + 0.7 * yb - 0.4 * zb
        xb, yb, zb = coords(1)
        by = -0.3 + 0.6 * xb + 0.2 * zb
        if ndim == 3:
            xb, yb, zb = coords(2)
            bz = 0.2 - 0.5 * xb + 0.9 * yb
        else:
            bz = 0.25 + 0.1 * x - 0.3 * y
        out.append([rho, mx, my, mz, E, bx, by, bz])
    return out


@pytest.mark.parametrize("ndim", [2, 3])
def test_overlap_reproduces_linear_fields(ndim):
    """Copies are exact; minmod-linear cell prolongation, on-face
    reconstruction and the projected interior faces are exact on linear data
    (all grids kept away from the periodic seam)."""
    N0 = (32, 32, 32)[:ndim]
    lo0 = (0,) * ndim
    old = [(0, lo0, N0),
           (1, (16,) * ndim, (32,) * ndim),
           (1, (32,) + (16,) * (ndim - 1), (40,) + (32,) * (ndim - 1))]
    new = [(0, lo0, N0),
           (1, (20,) * ndim, (36,) * ndim),
           (1, (36,) + (20,) * (ndim - 1), (44,) + (36,) * (ndim - 1)),
           (1, (12,) * ndim, (20,) + (28,) * (ndim - 1))]
    cons = _linear_state(ndim, N0, old)
    got = O.amr_overlap(ndim, N0, 2, 4, old, cons, new)
    want = _linear_state(ndim, N0, new)
    for gi in range(len(new)):
        for s in range(8):
            err = np.max(np.abs(got[gi][s] - want[gi][s]))
            assert err < 1e-14, (gi, s, err)


@pytest.mark.parametrize("ndim", [2, 3])
def test_overlap_conserves_and_keeps_div_b_zero(ndim):
    """After a synchronised coarse step, moving every level-1 and level-2 grid
    keeps the composite sums of the conserved fields to round-off and the
    composite div B at round-off (projected faces inside prolonged coarse
    cells, copied faces at the boundary of the old grids)."""
    N0 = (24, 24, 24)[:ndim]
    grids = I.amr_hierarchy(ndim, N0, 3, seed=11, ext=(8, 16))
    fields = I.amr_fields(ndim, N0, 3, grids, seed=3, b_rms=0.3)
    cons, _ = O.amr_run(ndim, N0, 3, 4, grids, fields, 1)
    # another seeded hierarchy on the same domain: other level-0 tiles, other
    # level-1 and level-2 boxes, partly overlapping the old ones
    new = I.amr_hierarchy(ndim, N0, 3, seed=12, ext=(8, 16))
    got = O.amr_overlap(ndim, N0, 3, 4, grids, cons, new)
    c0 = composite_sums(ndim, N0, grids, cons)
    c1 = composite_sums(ndim, N0, new, got)
    assert np.all(np.abs(c1 - c0) <= 1e-13 * (np.abs(c0) + 1.0)), c1 - c0
    assert composite_divb(ndim, N0, new, got) < 1e-12
    # and the new grids' fine cells each have zero divergence
    for gi, (l, lo, hi) in enumerate(new):
        h = [1.0 / (N0[a] * 2 ** l) for a in range(ndim)]
        bx, by, bz = got[gi][5], got[gi][6], got[gi][7]
        d = (bx[:, :, 1:] - bx[:, :, :-1]) / h[0] + (by[:, 1:, :] - by[:, :-1, :]) / h[1]
        if ndim == 3:
            d = d + (bz[1:] - bz[:-1]) / h[2]
        scale = max(np.max(np.abs(x)) for x in (bx, by, bz)) / min(h)
        assert np.max(np.abs(d)) <= 1e-12 * scale, (gi, np.max(np.abs(d)) / scale)


def test_overlap_rejects_misaligned_boxes():
    N0 = (16, 16)
    old = [(0, (0, 0), N0), (1, (8, 8), (16, 16))]
    new = [(0, (0, 0), N0), (1, (9, 8), (17, 16))]
    cons = _linear_state(2, N0, old)
    with pytest.raises(RuntimeError, match="aligned"):
        O.amr_overlap(2, N0, 2, 4, old, cons, new)


# ------------------------------------------------------------ regrid level
@pytest.mark.parametrize("level", [0, 1])
def test_regrid_level_covers_flags_nests_and_keeps_other_levels(level):
    ndim, N0, L = 3, (24, 24, 24), 3
    grids = I.amr_hierarchy(ndim, N0, L, seed=11, ext=(8, 16))
    fields = I.amr_fields(ndim, N0, L, grids, seed=3, b_rms=0.3)
    cons = _cons(ndim, N0, L, grids, fields)
    theta = 0.02
    new, f = RG.regrid_level(ndim, N0, L, 4, grids, cons, level, theta)
    assert f.sum() > 0
    kept = [g for g in grids if g[0] != level + 1]
    assert [g for g in new if g[0] != level + 1] == kept
    boxes = [(tuple(x // 2 for x in lo), tuple(x // 2 for x in hi)) for (l, lo, hi) in new if l == level + 1]
    adm = RG.nestable(ndim, N0, 4, grids, level)
    _check_cover(f, adm, boxes, 0.7, 16)
    # the level-(l+2) grids nest in the new level l+1, so the overlap runs
    out = O.amr_overlap(ndim, N0, L, 4, grids, cons, new)
    assert len(out) == len(new)
