"""GPU parity of the multilevel advance (fill/prolong, batched advance,
registers, reflux / EMF fix / restriction) against the FP64 oracle's serial
level cycle, through the C ABI."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import amr as A
from paper_1110_1616_amd import inputs as I
from tests.amr_util import composite_divb, composite_sums
from tests.gpu_util import amr_gpu, grid_box, log, normwise_errors

pytestmark = pytest.mark.gpu

CASES = {
    "3d": (3, (24, 24, 24), 3, 11, (8, 16)),
    "2d": (2, (32, 32), 3, 4, (8, 16)),
}


def _setup(key):
    ndim, N0, L, seed, ext = CASES[key]
    grids = I.amr_hierarchy(ndim, N0, L, seed=seed, ext=ext)
    fields = I.amr_fields(ndim, N0, L, grids, seed=3, b_rms=0.3)
    return ndim, N0, L, grids, fields


def _errors(got, want):
    cat_g = [np.concatenate([g[s].ravel() for g in got]) for s in range(8)]
    cat_w = [np.concatenate([w[s].ravel() for w in want]) for s in range(8)]
    return normwise_errors(cat_g, cat_w)


@pytest.mark.parametrize("key", ["3d", "2d"])
def test_fill_prolong_matches_oracle(key):
    ndim, N0, L, grids, fields = _setup(key)
    log(f"case: FULL fill of level 1 and 2, {key}")
    cons = O.amr_run(ndim, N0, L, 4, grids, fields, 0)[0]
    H = A.Hierarchy(ndim, N0, grids, nlevels=L, ghost=4)
    U = H.new_state()
    for gi, f in enumerate(fields):
        H.load_primitive(U, gi, f["prim"], f["b"])
    for lev in range(L):
        H.fill(lev, A.AMR_FILL_SAME_LEVEL if lev == 0 else A.AMR_FILL_FULL, U, U)
        want = O.amr_fill(ndim, N0, L, 4, grids, cons, level=lev, full=lev > 0)
        for gi, (l, lo, hi) in enumerate(grids):
            if l != lev:
                continue
            got = grid_box(H, U, gi)
            for s in range(8):
                scale = np.max(np.abs(want[gi][s])) + 1e-300
                err = np.max(np.abs(got[s] - want[gi][s])) / scale
                assert err <= 1e-13, (lev, gi, s, err)


@pytest.mark.parametrize("key", ["3d", "2d"])
def test_multilevel_parity_f64(key):
    ndim, N0, L, grids, fields = _setup(key)
    log(f"case: {key} 3-level hierarchy, {len(grids)} grids, 2 coarse steps, f64 batched")
    want, dts_o = O.amr_run(ndim, N0, L, 4, grids, fields, 2)
    got, dts_g, flags = amr_gpu(ndim, N0, L, grids, fields, 2)
    assert flags[0] == 0
    err = _errors(got, want)
    log(f"  errors per field: {err}  dt rel diff {np.max(np.abs(dts_g - dts_o) / dts_o):.2e}")
    assert np.all(err <= 1e-10), err


def test_multilevel_parity_f32():
    ndim, N0, L, grids, fields = _setup("3d")
    log("case: 3d 3-level hierarchy f32 vs f64 oracle, 2 coarse steps")
    want, _ = O.amr_run(ndim, N0, L, 4, grids, fields, 2)
    got, _, flags = amr_gpu(ndim, N0, L, grids, fields, 2, dtype="f32")
    err = _errors(got, want)
    log(f"  errors per field: {err}")
    assert np.all(err <= 1e-5), err


@pytest.mark.parametrize("key", ["3d", "2d"])
def test_batched_equals_per_grid_bitwise(key):
    ndim, N0, L, grids, fields = _setup(key)
    log(f"case: batched vs per-grid serial order, {key}")
    a, da, _ = amr_gpu(ndim, N0, L, grids, fields, 2, mode=0)
    b, db, _ = amr_gpu(ndim, N0, L, grids, fields, 2, mode=1)
    assert np.array_equal(da, db)
    for ga, gb in zip(a, b):
        for x, y in zip(ga, gb):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("key", ["3d", "2d"])
def test_composite_conservation_and_divb_gpu(key):
    ndim, N0, L, grids, fields = _setup(key)
    log(f"case: composite invariants on the GPU, {key}")
    s0, _, _ = amr_gpu(ndim, N0, L, grids, fields, 0)
    s3, _, _ = amr_gpu(ndim, N0, L, grids, fields, 3)
    c0 = composite_sums(ndim, N0, grids, s0)
    c3 = composite_sums(ndim, N0, grids, s3)
    log(f"  d(composite) = {c3 - c0}")
    assert np.all(np.abs(c3 - c0) <= 1e-13 * (np.abs(c0) + 1.0))
    assert composite_divb(ndim, N0, grids, s3) < 1e-12


def test_graph_replay_matches_eager_every_replay():
    """Coarse steps captured into HIP graphs replay bit for bit like eager
    steps, replay after replay (eager work and synchronisation between)."""
    import torch
    ndim, N0, L, grids, fields = _setup("3d")
    log("case: hipGraph replay vs eager, 3d, 3 coarse steps")
    ref = []
    for n in (1, 2, 3):
        outs, _, _ = amr_gpu(ndim, N0, L, grids, fields, n)
        ref.append(outs)
    H = A.Hierarchy(ndim, N0, grids, nlevels=L, ghost=4)
    Ua, Ub = H.new_state(), H.new_state()
    for gi, f in enumerate(fields):
        H.load_primitive(Ua, gi, f["prim"], f["b"])
    stream = torch.cuda.Stream()
    # capture from a copy so the captured launches do not run on the state
    with torch.cuda.stream(stream):
        H.graph_capture(Ua, Ub, 0)
    torch.cuda.synchronize()
    # capturing does not execute: reload the initial state to be safe
    for gi, f in enumerate(fields):
        H.load_primitive(Ua, gi, f["prim"], f["b"])
    par = 0
    for n in range(3):
        with torch.cuda.stream(stream):
            par = H.graph_launch(par)
        torch.cuda.synchronize()
        got = [H.store_interior(H.current(Ua, Ub, par, l), gi) for gi, (l, lo, hi) in enumerate(grids)]
        for gg, gw in zip(got, ref[n]):
            for x, y in zip(gg, gw):
                assert np.array_equal(x, y), f"replay {n}"


@pytest.mark.parametrize("key", ["3d", "2d"])
def test_every_launch_configuration_gives_identical_results(key):
    """Tile policy, z-chunk, persistent vs one-block-per-item launches (both
    kernels or the flux kernel only), XCD chunking (fused lists without it
    end in re-cut short items), the update's z-chunk, the claim size and
    the fused flux-update kernel (launch mode bit 3) only
    change how the same per-face and per-cell arithmetic is distributed, and
    the device code contracts multiply-adds inside each source expression
    only: two coarse steps agree bit for bit under all 64 configurations
    (the 48 of the two-kernel path, the 16 fused ones; each with one of the
    update z-chunks 1, 2, 3, 8 and one of the claim sizes 1, 2, 4, 8)."""
    ndim, N0, L, grids, fields = _setup(key)
    ref = {}
    for fused in (False, True):
        for pol in (0, 1):
            for zi, zc in enumerate((8, 12, 16, 64)):
                for per in (0, 1, 2, 3, 4, 6) if not fused else (8, 10, 12, 14):
                    uz = (1, 2, 3, 8)[(zi + per) % 4]
                    # work items per block claim: 1, 2, 4 or 8 (mode bits 4-5)
                    mode = per | (((zi + pol + per) % 4) << 4)
                    log(f"case: launch config {key} policy={pol} zchunk={zc} mode={mode} update zchunk={uz}")
                    H = A.Hierarchy(ndim, N0, grids, nlevels=L, ghost=4)
                    H.set_launch_config(pol, zc, mode, uz)
                    assert A.amr_get_launch_config(H.h) == (pol, zc, mode)
                    assert A.amr_get_update_zchunk(H.h) == uz
                    Ua, Ub = H.new_state(), H.new_state()
                    for gi, f in enumerate(fields):
                        H.load_primitive(Ua, gi, f["prim"], f["b"])
                    par = 0
                    for _ in range(2):
                        par = H.coarse_step(Ua, Ub, par, 0)
                    got = [H.store_interior(H.current(Ua, Ub, par, l), gi) for gi, (l, lo, hi) in enumerate(grids)]
                    assert H.error_flags()[0] == 0
                    if not ref:
                        ref[0] = got
                        continue
                    for gg, gw in zip(got, ref[0]):
                        for x, y in zip(gg, gw):
                            assert np.array_equal(x, y), (fused, pol, zc, mode, uz)


def test_launch_configuration_rejects_bad_values():
    """Out-of-range tile policy, z-chunks and launch modes are refused and
    leave the configuration as it was."""
    ndim, N0, L, grids, fields = _setup("3d")
    H = A.Hierarchy(ndim, N0, grids, nlevels=L, ghost=4)
    H.set_launch_config(1, 12, 6, 2)
    for bad in ((2, 8, 0), (1, 0, 0), (1, 8, 64), (1, 8, -1)):
        with pytest.raises(A.AmrError):
            A.amr_set_launch_config(H.h, *bad)
    with pytest.raises(A.AmrError):
        A.amr_set_update_zchunk(H.h, 0)
    assert A.amr_get_launch_config(H.h) == (1, 12, 6)
    assert A.amr_get_update_zchunk(H.h) == 2


def test_autotune_keeps_the_state_and_the_results():
    """The autotuner times all 100 launch configurations, then the update
    z-chunks under the fastest, then the claim sizes (work items per block
    claim, launch mode bits 4-5), without changing what the next coarse step
    computes."""
    import torch
    ndim, N0, L, grids, fields = _setup("3d")
    ref, _, _ = amr_gpu(ndim, N0, L, grids, fields, 2)
    H = A.Hierarchy(ndim, N0, grids, nlevels=L, ghost=4)
    Ua, Ub = H.new_state(), H.new_state()
    for gi, f in enumerate(fields):
        H.load_primitive(Ua, gi, f["prim"], f["b"])
    par = H.coarse_step(Ua, Ub, 0, 0)
    chosen, table = H.autotune(Ua, Ub, par, reps=2)
    log(f"autotune chose {table[chosen]}")
    assert 0 <= chosen < A.TUNE_CANDIDATES and all(t[3] > 0 for t in table)
    assert A.amr_get_launch_config(H.h) == tuple(table[chosen][:3])
    assert A.amr_get_update_zchunk(H.h) == table[chosen][4]
    assert [t[4] for t in table[100:104]] == [1, 2, 4, 8]
    assert all(tuple(t[:3]) == tuple(table[100][:3]) for t in table[100:104])
    assert [t[2] >> 4 for t in table[104:]] == [1, 2, 3]
    assert all(tuple(t[:2]) == tuple(table[100][:2]) and (t[2] & 15) == table[100][2] for t in table[104:])
    assert len({t[4] for t in table[104:]}) == 1
    assert sorted({t[1] for t in table[:100]}) == [8, 12, 16, 24, 32]
    par = H.coarse_step(Ua, Ub, par, 0)
    torch.cuda.synchronize()
    got = [H.store_interior(H.current(Ua, Ub, par, l), gi) for gi, (l, lo, hi) in enumerate(grids)]
    for gg, gw in zip(got, ref):
        for x, y in zip(gg, gw):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("key", ["3d", "2d"])
def test_eta_schedule_gives_identical_results(key):
    """The predictive (eta) schedule moves coarse-level grid steps to other
    launch cycles of their window; two coarse steps agree bit for bit with
    the window-start schedule, eager and as graph replays."""
    import torch
    ndim, N0, L, grids, fields = _setup(key)
    ref, dref, _ = amr_gpu(ndim, N0, L, grids, fields, 2)
    H = A.Hierarchy(ndim, N0, grids, nlevels=L, ghost=4)
    H.set_schedule(1)
    ncyc = 2 ** (L - 1)
    sched, work = A.amr_get_schedule(H.h, ncyc)
    log(f"case: eta schedule {key}, predicted work per cycle {[round(w) for w in work]}")
    assert sched == 1
    for graph in (False, True):
        Ua, Ub = H.new_state(), H.new_state()
        for gi, f in enumerate(fields):
            H.load_primitive(Ua, gi, f["prim"], f["b"])
        par = 0
        stream = torch.cuda.Stream()
        if graph:
            with torch.cuda.stream(stream):
                H.graph_capture(Ua, Ub, 0)
            torch.cuda.synchronize()
            for gi, f in enumerate(fields):
                H.load_primitive(Ua, gi, f["prim"], f["b"])
        for _ in range(2):
            with torch.cuda.stream(stream):
                par = H.graph_launch(par) if graph else H.coarse_step(Ua, Ub, par, 0)
            torch.cuda.synchronize()
        got = [H.store_interior(H.current(Ua, Ub, par, l), gi) for gi, (l, lo, hi) in enumerate(grids)]
        assert H.error_flags()[0] == 0
        for gg, gw in zip(got, ref):
            for x, y in zip(gg, gw):
                assert np.array_equal(x, y), f"graph={graph}"
