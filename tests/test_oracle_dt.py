"""Pins of the oracle's time step (CPU only).

The paper defers the solver and fixes no CFL rule; the scheme's time step is
dt = C / max over interior cells of sum_d (|v_d| + c_f,d) / dx_d (C = 0.4),
and with refinement dt0 = min_l R^l dt_l, i.e. the same sum with the
level-0 widths dx0_d over the cells of every level (level l then steps
dt0 / R^l).  The expected values here do not retype the oracle's fast-speed
formula: |v_d| + c_f,d is taken as the largest |eigenvalue| of the
primitive-variable Jacobian of one-dimensional ideal MHD along d, built
from the equations of motion and solved by numpy.  Each test also shows
that a plausible misreading (the largest direction instead of the sum,
the fine spacing dx_l in place of dx0, band cells in the maximum) moves the
result far outside the tolerance.
"""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import inputs as I

GAMMA = 5.0 / 3.0
CFL = 0.4


def max_signal(W, d, gamma):
    """Largest |eigenvalue| of the 1-D ideal-MHD primitive Jacobian along
    axis d (variables rho, u_n, u_t1, u_t2, B_t1, B_t2, p; normal B fixed;
    magnetic pressure |B|^2 / 2)."""
    rho, p = W[0], W[4]
    v = [W[1], W[2], W[3]]
    B = [W[5], W[6], W[7]]
    t1, t2 = (d + 1) % 3, (d + 2) % 3
    u, ut1, ut2 = v[d], v[t1], v[t2]
    bn, b1, b2 = B[d], B[t1], B[t2]
    A = np.array([
        [u, rho, 0, 0, 0, 0, 0],
        [0, u, 0, 0, b1 / rho, b2 / rho, 1 / rho],
        [0, 0, u, 0, -bn / rho, 0, 0],
        [0, 0, 0, u, 0, -bn / rho, 0],
        [0, b1, -bn, 0, u, 0, 0],
        [0, b2, 0, -bn, 0, u, 0],
        [0, gamma * p, 0, 0, 0, 0, u],
    ], dtype=float)
    del ut1, ut2  # advected with the flow: they enter only through u
    return float(np.max(np.abs(np.linalg.eigvals(A).real)))


def expected_dt(W, ndim, dx, gamma=GAMMA, cfl=CFL):
    return cfl / sum(max_signal(W, d, gamma) / dx[d] for d in range(ndim))


STATES = [
    # (rho, vx, vy, vz, p, Bx, By, Bz)
    ("B along x", (1.0, 0.1, -0.05, 0.02, 1.0, 1.5, 0.0, 0.0)),
    ("B across x", (1.2, -0.3, 0.2, 0.1, 0.8, 0.0, 0.9, 0.0)),
    ("B oblique", (0.8, 0.25, -0.4, 0.3, 0.6, 0.7, -0.5, 0.4)),
    ("B along z", (1.0, 0.0, 0.0, 0.6, 1.0, 0.0, 0.0, 2.0)),
    ("no field", (1.0, 0.5, -0.2, 0.1, 2.0, 0.0, 0.0, 0.0)),
]


def _uniform_ic(ndim, n, W):
    return I.uniform_state(ndim, n, rho=W[0], v=W[1:4], p=W[4], B=W[5:8])


@pytest.mark.parametrize("ndim,n", [(2, (24, 10)), (3, (12, 8, 20))])
@pytest.mark.parametrize("name,W", STATES)
def test_uniform_dt_closed_form(ndim, n, name, W):
    ic = _uniform_ic(ndim, n, W)
    _, dts = O.uniform_run(ic, GAMMA, CFL, 1, g=2)
    want = expected_dt(W, ndim, ic["dx"])
    assert dts[0] == pytest.approx(want, rel=1e-12), name
    # the misreading "largest direction" instead of the sum of directions
    wrong = CFL / max(max_signal(W, d, GAMMA) / ic["dx"][d] for d in range(ndim))
    assert abs(wrong - want) > 0.2 * want


@pytest.mark.parametrize("ndim,n", [(2, (16, 12)), (3, (10, 8, 12))])
def test_banded_dt_counts_interior_only(ndim, n):
    """orc_dt_banded: a much faster state in the band must not change dt."""
    g = 3
    Wslow = STATES[2][1]
    ic = _uniform_ic(ndim, n, Wslow)
    cons = O.conserved_interior(ic, GAMMA)
    band = O.banded_from_interior(ndim, n, g, cons)
    # fill the band with a fast state (high pressure and velocity)
    Wfast = (1.0, 3.0, -2.0, 1.0, 40.0, 0.7, -0.5, 0.4)
    icf = _uniform_ic(ndim, tuple(m + 2 * g for m in n), Wfast)
    fast = O.conserved_interior(icf, GAMMA)
    gz = g if ndim == 3 else 0
    for s in range(8):
        sh = np.asarray(cons[s]).shape
        inner = band[s][gz:gz + sh[0], g:g + sh[1], g:g + sh[2]].copy()
        fs = np.asarray(fast[s])
        band[s][...] = fs[:band[s].shape[0], :band[s].shape[1], :band[s].shape[2]]
        band[s][gz:gz + sh[0], g:g + sh[1], g:g + sh[2]] = inner
    dt = O.dt_banded(ndim, n, g, GAMMA, CFL, ic["dx"], band)
    want = expected_dt(Wslow, ndim, ic["dx"])
    assert dt == pytest.approx(want, rel=1e-12)
    assert expected_dt(Wfast, ndim, ic["dx"]) < 0.2 * want  # the band would have set a far smaller dt


def _level_fields(ndim, grids, states):
    out = []
    for (lev, lo, hi), W in zip(grids, states):
        n = tuple(hi[a] - lo[a] for a in range(ndim))
        ic = _uniform_ic(ndim, n, W)
        out.append({"prim": ic["prim"], "b": ic["b"]})
    return out


def _three_levels(ndim):
    if ndim == 3:
        N0 = (16, 12, 20)
        grids = [(0, (0, 0, 0), N0), (1, (8, 6, 10), (24, 18, 30)), (2, (24, 20, 28), (40, 28, 52))]
    else:
        N0 = (16, 12)
        grids = [(0, (0, 0), N0), (1, (8, 6), (24, 18)), (2, (24, 20), (40, 28))]
    return N0, grids


SLOW = (1.0, 0.1, -0.05, 0.02, 1.0, 0.3, 0.2, -0.1)
FAST = (1.0, 0.6, -0.4, 0.3, 1.6, 0.3, 0.2, -0.1)  # same B: no jump in the field across levels


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("fast_level", [0, 1, 2])
def test_multilevel_dt_takes_level0_widths(ndim, fast_level):
    """dt0 = min_l R^l dt_l: the fastest cell on level l sets dt0 through
    dx0, not through its own dx_l."""
    N0, grids = _three_levels(ndim)
    states = [FAST if l == fast_level else SLOW for (l, lo, hi) in grids]
    fields = _level_fields(ndim, grids, states)
    _, dts = O.amr_run(ndim, N0, 3, 4, grids, fields, 1)
    dx0 = [1.0 / N0[a] for a in range(ndim)]
    dts_l = [expected_dt(states[i], ndim, [h / 2 ** l for h in dx0]) for i, (l, _, _) in enumerate(grids)]
    want = min(2 ** l * dt for (l, _, _), dt in zip(grids, dts_l))
    assert dts[0] == pytest.approx(want, rel=1e-12)
    assert want == pytest.approx(expected_dt(FAST, ndim, dx0), rel=1e-13)
    if fast_level > 0:
        # the misreading "dx_l for dx0" (plain min_l dt_l) differs by R^l
        wrong = min(dts_l)
        assert wrong < 0.6 * want


def test_flop_constants_match_oracle_counts():
    """The bench's algorithmic flop constants (the roofline numerator) are
    the oracle's own counts: per cell with predicted states (primitive
    recovery, slopes, Hancock predictor) on large patches, and per HLLD
    evaluation."""
    import ctypes as C

    import bench

    L = O.lib()
    L.orc_count_hlld_flops.restype = C.c_longlong
    assert bench.FLOPS_HLLD == L.orc_count_hlld_flops()
    for ndim, n in ((2, 64), (3, 32)):
        out = np.zeros(8)
        assert L.orc_count_step_flops(ndim, n, out.ctypes.data_as(C.POINTER(C.c_double))) == 0
        per_pred = out[4] / out[2]
        per_face = out[5] / out[3]
        assert per_face == bench.FLOPS_HLLD
        # the count per predicted cell still carries the primitive recovery
        # of the two outer band layers (a few flops per cell at these sizes)
        assert abs(per_pred - bench.FLOPS_PRED[ndim]) <= 0.005 * per_pred, (ndim, per_pred)


def test_update_flop_constants_match_oracle_counts():
    """The update's flop constants (the fused kernel's share of the roofline
    numerator) decompose the oracle's own counts exactly: per updated cell,
    per updated face-centred B component, and per edge EMF over the edges
    the oracle forms (n + 2 along each edge in 3-D)."""
    import ctypes as C

    import bench

    L = O.lib()
    for ndim, sizes in ((3, (16, 24, 32)), (2, (32, 64, 128))):
        for n in sizes:
            out = np.zeros(8)
            assert L.orc_count_step_flops(ndim, n, out.ctypes.data_as(C.POINTER(C.c_double))) == 0
            cells = n ** ndim
            faces = ndim * (n + 1) * n ** (ndim - 1)
            edges = 3 * (n + 1) ** 2 * (n + 2) if ndim == 3 else (n + 1) ** 2
            assert out[7] == bench.FLOPS_UPD_CELL[ndim] * cells + bench.FLOPS_UPD_FACE[ndim] * faces, (ndim, n)
            assert out[6] == bench.FLOPS_EMF_EDGE * edges, (ndim, n)
    # the per-launch count the bench uses: updated box n + 2 gv - 4
    assert bench.update_flops(3, (8, 8, 8), 2) == 55 * 512 + 8 * 3 * 9 * 64 + 4 * 3 * 8 * 81
    assert bench.update_flops(2, (8, 8), 4) == 48 * 144 + 5 * 2 * 13 * 12 + 4 * 169
