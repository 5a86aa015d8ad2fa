"""The paper's predictive balancing (Sec. 5) and the library's launch-cycle
plan built on it: the identity eta_l^p = etabar_l for the continuous
distribution, and the discrete plan's bounds and windows (no GPU)."""

import numpy as np
import pytest

from oracle import schedule as S
from paper_1110_1616_amd import amr as A
from paper_1110_1616_amd import inputs as I


@pytest.mark.parametrize("seed", range(5))
def test_eta_is_equal_across_processors(seed):
    """g_l^p = gbar_l - (eta_{l-1}^p - etabar_{l-1}) / s_l makes every eta_l^p
    equal to its mean for each newly distributed level (nothing of it done
    yet); uneven progress w_0 on the coarse level leaves eta_0 uneven and is
    compensated by the next level."""
    rng = np.random.default_rng(seed)
    L, P = 4, 7
    s = [1, 2, 4, 8]
    gbar = rng.uniform(1.0, 5.0, size=L)
    w = np.zeros((L, P))
    w[0] = rng.uniform(0.0, 0.5, size=P)  # uneven progress on the coarse level
    g = S.successive(s, gbar, w, P)
    e = S.eta(s, g, w)
    assert np.ptp(e[0]) > 0.01
    for l in range(1, L):
        assert np.allclose(e[l], e[l].mean(), rtol=0, atol=1e-12 * abs(e[l].mean())), (l, e[l])
    # the per-level means are the undisturbed sums
    assert np.allclose(g.mean(axis=1), gbar)


def test_a_planted_sign_error_breaks_the_identity():
    rng = np.random.default_rng(9)
    prev = rng.uniform(0, 3, size=5)
    good = S.distribute(2.0, 2.0, prev)
    bad = 2.0 + (prev - prev.mean()) / 2.0
    assert np.ptp(prev + 2.0 * good) < 1e-12
    assert np.ptp(prev + 2.0 * bad) > 1.0


def _hier(ndim, N0, L, seed):
    return I.amr_hierarchy(ndim, N0, L, seed=seed, ext=(8, 16))


@pytest.mark.parametrize("L,seed", [(3, 11), (4, 5)])
def test_plan_windows_and_bounds(L, seed):
    ndim, N0 = 3, (24, 24, 24)
    grids = _hier(ndim, N0, L, seed)
    p = A.make_params(ndim, N0, L, 2, 4)
    R = 2
    ncyc = R ** (L - 1)
    w0, c0 = A.amr_plan_schedule(p, grids, 0)
    w1, c1 = A.amr_plan_schedule(p, grids, 1)
    assert np.isclose(sum(w0), sum(w1))
    for gi, (l, lo, hi) in enumerate(grids):
        span = R ** (L - 1 - l)
        assert len(c0[gi]) == R ** l == len(c1[gi])
        for k in range(R ** l):
            assert c0[gi][k] == k * span  # schedule 0: the window's start
            assert k * span <= c1[gi][k] < (k + 1) * span  # schedule 1: inside the window
    # per window of each level: the discrete loads keep the greedy bound
    # around the continuous balanced value of the oracle's formula
    work = lambda gi, gv: float(np.prod([hi - lo + 2 * gv - 2 for lo, hi in zip(grids[gi][1], grids[gi][2])]))
    load = np.zeros(ncyc)
    for l in range(L - 1, -1, -1):
        span = R ** (L - 1 - l)
        for k in range(R ** l):
            gv = 2 if l == 0 else 4 - 2 * (k % R)
            gl = [gi for gi, g in enumerate(grids) if g[0] == l]
            ws = [work(gi, gv) for gi in gl]
            win = slice(k * span, (k + 1) * span)
            got = np.zeros(span)
            for gi, w in zip(gl, ws):
                got[c1[gi][k] - k * span] += w
            if span > 1 and ws:
                share = S.window_targets(load[win], sum(ws) / span)
                deficit = share - got
                assert np.all(deficit >= -max(ws) - 1e-9)
                assert np.all(deficit <= (span - 1) * max(ws) + 1e-9)
            load[win] += got
    assert np.allclose(load, w1)
    assert max(w1) - min(w1) <= max(w0) - min(w0)
