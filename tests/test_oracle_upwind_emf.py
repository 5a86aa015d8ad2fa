"""Pins of the oracle's upwinded constrained-transport EMF (Gardiner & Stone
2005), the scheme variant beside the arithmetic edge mean: reduction to the
one-dimensional solver for grid-aligned flow, stability of an advected field
loop (and the failure of the planted downwind choice), conservation, div B,
axis permutation, the extended-ghost-zone decoupling invariant and the AMR
composite invariants."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import inputs as I
from tests.amr_util import composite_divb, composite_sums
from tests.test_oracle_scheme import GAMMA, _patch_from_global, div_b


def _brio_wu_sym(N=64, ny=4):
    """Brio-Wu along x with the transverse field split evenly between B_y
    (face-centred, updated by CT) and B_z (cell-centred in 2D, updated by
    its flux): the problem is symmetric under y <-> z."""
    ic = I.brio_wu(N, ny)
    left = (np.arange(N) + 0.5) / N < 0.5
    s = 1.0 / np.sqrt(2.0)
    ic["b"][1] = np.broadcast_to(np.where(left, s, -s), (1, ny + 1, N)).copy()
    ic["b"][2] = np.broadcast_to(np.where(left, s, -s), (1, ny, N)).copy()
    return ic


def test_upwind_emf_reduces_to_the_1d_solver_for_grid_aligned_flow():
    """With the upwinded EMF the CT update of B_y equals the flux update of
    B_z in this y <-> z symmetric problem (the edge EMF is exactly the x-face
    flux), to round-off after 60 steps; the arithmetic mean mixes in cell
    values and does not (its known weakness for grid-aligned problems)."""
    ic = _brio_wu_sym()
    diff = {}
    for mode in (0, 1):
        with O.emf(mode):
            f, _ = O.uniform_run(ic, 2.0, 0.4, 60, bc=(1, 0, 0))
        diff[mode] = np.max(np.abs(f[6][0, 0, :] - f[7][0, 0, :]))
    assert diff[1] < 1e-13, diff
    assert diff[0] > 1e-2, diff


def _field_loop(N=48):
    """Weak field loop (A_z = A0 (R - r) inside r < R, A0 = 1e-3, R = 0.3)
    advected with v = (1, 0.5) on the periodic unit square, rho = p = 1."""
    h = 1.0 / N
    A0, R = 1e-3, 0.3
    xc = np.arange(N + 1) * h
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    Az = np.where(np.hypot(X - 0.5, Y - 0.5) < R, A0 * (R - np.hypot(X - 0.5, Y - 0.5)), 0.0)
    bx = (Az[1:, :] - Az[:-1, :]) / h
    by = -(Az[:, 1:] - Az[:, :-1]) / h
    shp = (1, N, N)
    ic = {"prim": [np.ones(shp), np.full(shp, 1.0), np.full(shp, 0.5), np.zeros(shp), np.ones(shp)],
          "b": [bx[None].copy(), by[None].copy(), np.zeros(shp)], "dx": [h, h, 1.0], "ndim": 2, "n": (N, N)}
    return ic, A0


def _emag(f):
    bx, by = f[5][0], f[6][0]
    return 0.5 * np.sum((0.5 * (bx[:, 1:] + bx[:, :-1])) ** 2 + (0.5 * (by[1:, :] + by[:-1, :])) ** 2)


def test_field_loop_stays_bounded_and_the_downwind_choice_fails():
    """One crossing in x.  Upwinded EMF: no new extremum of |B| (max |B_y|
    <= A0, the initial maximum) and a magnetic energy loss of numerical
    diffusion only; the planted downwind choice of the same formula drives
    the state non-physical."""
    ic, A0 = _field_loop()
    e0 = _emag([None] * 5 + [ic["b"][0], ic["b"][1]])
    with O.emf(1):
        _, d = O.uniform_run(ic, GAMMA, 0.4, 1)
        n = int(np.ceil(1.0 / d[0]))
        f, _ = O.uniform_run(ic, GAMMA, 0.4, n)
    assert np.max(np.abs(f[6])) <= A0 * (1 + 1e-12)
    ratio = _emag(f) / e0
    assert 0.5 < ratio < 1.0, ratio
    with O.emf(2):
        with pytest.raises(RuntimeError, match="non-positive"):
            O.uniform_run(ic, GAMMA, 0.4, n)


@pytest.mark.parametrize("ndim,n,steps", [(2, (48, 48), 60), (3, (16, 16, 16), 20)])
def test_upwind_conservation_and_divb(ndim, n, steps):
    ic = I.smooth_mhd(ndim, n, seed=3, b_rms=0.3, jump=True)
    f0 = O.conserved_interior(ic, GAMMA)
    with O.emf(1):
        f, _ = O.uniform_run(ic, GAMMA, 0.4, steps, g=2)
    for s in range(5):
        scale = np.sum(np.abs(f0[s])) + 1.0
        assert abs(np.sum(f[s]) - np.sum(f0[s])) / scale < 1e-13, O.FIELDS[s]
    bmax = max(np.abs(x).max() for x in f[5:8])
    assert np.abs(div_b(ndim, n, f[5:8])).max() / (bmax * max(n)) < 1e-13
    # and the variant changes the answer (the two EMFs differ off grid alignment)
    g, _ = O.uniform_run(ic, GAMMA, 0.4, steps, g=2)
    assert np.max(np.abs(g[5] - f[5])) > 1e-8


def test_upwind_axis_permutation_3d():
    n = (12, 10, 8)
    ic = I.smooth_mhd(3, n, seed=9, b_rms=0.3, jump=True)

    def perm(a):
        return np.ascontiguousarray(np.transpose(a, (2, 0, 1)))

    rho, vx, vy, vz, p = ic["prim"]
    bx, by, bz = ic["b"]
    ic2 = {"ndim": 3, "n": (n[1], n[2], n[0]), "dx": [ic["dx"][1], ic["dx"][2], ic["dx"][0]],
           "prim": [perm(rho), perm(vy), perm(vz), perm(vx), perm(p)], "b": [perm(by), perm(bz), perm(bx)]}
    with O.emf(1):
        f, _ = O.uniform_run(ic, GAMMA, 0.4, 8, g=2)
        f2, _ = O.uniform_run(ic2, GAMMA, 0.4, 8, g=2)
    pairs = [(0, 0), (1, 2), (2, 3), (3, 1), (4, 4), (5, 6), (6, 7), (7, 5)]
    for new, old in pairs:
        ref = perm(f[old])
        assert np.max(np.abs(f2[new] - ref)) <= 1e-13 * (np.abs(ref).max() + 1e-300), O.FIELDS[new]


@pytest.mark.parametrize("ndim", [2, 3])
def test_upwind_decoupling_invariant_bitwise(ndim):
    """The upwinded EMF reads the same faces and cells as the mean (the cells
    around each edge already carry predicted states), so a band of 4 still
    decouples a patch for two substeps bit for bit."""
    n = (24, 20) if ndim == 2 else (16, 12, 14)
    ic = I.smooth_mhd(ndim, n, seed=21, b_rms=0.3, jump=True)
    f0 = O.conserved_interior(ic, GAMMA)
    with O.emf(1):
        f2, dts = O.uniform_run(ic, GAMMA, 0.4, 2, g=4, fill_every=2)
        lo = (5, 3, 4)[:ndim] + ((0,) if ndim == 2 else ())
        m = (7, 9, 6)[:ndim] + ((1,) if ndim == 2 else ())
        g = 4
        patch = _patch_from_global(ndim, n, g, lo, m, f0)
        mm = m[:ndim]
        a = O.step_banded(ndim, mm, g, 4, GAMMA, ic["dx"], dts[0], patch)
        b = O.step_banded(ndim, mm, g, 2, GAMMA, ic["dx"], dts[1], a)
    got = O.interior_from_banded(ndim, mm, g, b)
    want = _patch_from_global(ndim, n, 0, lo, m, f2)
    for s in range(8):
        assert np.array_equal(got[s], want[s]), O.FIELDS[s]


@pytest.mark.parametrize("ndim", [2, 3])
def test_upwind_amr_composite_invariants(ndim):
    """Refluxing and the EMF correction use the step's own edge EMFs, so the
    composite sums and composite div B stay at round-off with the variant."""
    N0 = (24, 24, 24)[:ndim]
    grids = I.amr_hierarchy(ndim, N0, 3, seed=11, ext=(8, 16))
    fields = I.amr_fields(ndim, N0, 3, grids, seed=3, b_rms=0.3)
    s0, _ = O.amr_run(ndim, N0, 3, 4, grids, fields, 0)
    with O.emf(1):
        s3, _ = O.amr_run(ndim, N0, 3, 4, grids, fields, 2)
    c0, c3 = composite_sums(ndim, N0, grids, s0), composite_sums(ndim, N0, grids, s3)
    assert np.all(np.abs(c3 - c0) <= 1e-13 * (np.abs(c0) + 1.0)), c3 - c0
    assert composite_divb(ndim, N0, grids, s3) < 1e-12
