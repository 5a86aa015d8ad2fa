"""The allocation-free advance (amr_advance_patches_noalloc) against
amr_advance_patches with a caller workspace, through the C ABI: two calls
in a row on one device, the second on a smaller hierarchy (the static
scratch array then holds the first call's contents), each bit for bit equal
to the workspace path; a hierarchy whose workspace exceeds the array is
refused."""

import numpy as np
import pytest

from paper_1110_1616_amd import amr as A
from paper_1110_1616_amd import inputs as I
from tests.gpu_util import log

pytestmark = pytest.mark.gpu
GAMMA = 5.0 / 3.0


def _load(H, ic, boxes):
    from tests.test_gpu_invariants import _split_fields
    U = H.new_state()
    for gi, (prim, b) in enumerate(_split_fields(ic, boxes)):
        H.load_primitive(U, gi, prim, b)
    return U


def _run(H, U, steps, noalloc):
    """A band-4 then a band-2 substep of every grid after a same-level fill,
    dt0 fixed; returns each grid's interior."""
    import torch
    V = H.new_state()
    W = H.new_state().copy_(U)
    H.fill(0, A.AMR_FILL_SAME_LEVEL, W)
    for dt, band in steps:
        H.dt0.fill_(dt)
        if noalloc:
            A.amr_advance_patches_noalloc(H.h, 0, None, band, W.c, V.c, 0, H.dt0)
        else:
            A.amr_advance_patches(H.h, 0, None, band, W.c, V.c, 0, H.dt0, H.ws)
        W, V = V, W
    torch.cuda.synchronize()
    return [H.store_interior(W, gi) for gi in range(len(H.grids))]


def _case(ndim, N, cuts, dtype, seed):
    boxes = []
    if ndim == 3:
        xs, ys, zs = cuts
        boxes = [((x0, y0, z0), (x1, y1, z1)) for x0, x1 in zip(xs, xs[1:]) for y0, y1 in zip(ys, ys[1:])
                 for z0, z1 in zip(zs, zs[1:])]
    else:
        xs, ys = cuts
        boxes = [((x0, y0), (x1, y1)) for x0, x1 in zip(xs, xs[1:]) for y0, y1 in zip(ys, ys[1:])]
    ic = I.smooth_mhd(ndim, N, seed=seed, v_rms=0.15, b_rms=0.3, jump=True)
    H = A.Hierarchy(ndim, N, [(0, lo, hi) for lo, hi in boxes], ghost=4, dtype=dtype, dx0=ic["dx"], gamma=GAMMA)
    return H, _load(H, ic, boxes)


def test_noalloc_matches_workspace_path_two_calls():
    steps = [(1.0e-3, 4), (1.0e-3, 2)]
    cases = [(3, (64, 48, 40), ((0, 30, 64), (0, 20, 48), (0, 40)), "f64", 3),
             (3, (24, 20, 16), ((0, 10, 24), (0, 20), (0, 16)), "f64", 4),
             (2, (40, 32), ((0, 18, 40), (0, 32)), "f32", 5)]
    for ndim, N, cuts, dtype, seed in cases:
        H, U = _case(ndim, N, cuts, dtype, seed)
        log(f"case: noalloc vs workspace, {ndim}D {N} {dtype}, {len(H.grids)} grids, workspace "
            f"{H.workspace_bytes / 2**20:.1f} MiB")
        got = _run(H, U, steps, True)
        want = _run(H, U, steps, False)
        assert H.error_flags()[0] == 0
        for gi, (a, b) in enumerate(zip(got, want)):
            for s in range(8):
                assert np.array_equal(a[s], b[s]), (N, gi, s)


def test_noalloc_multilevel_cycle_matches_workspace_path():
    """Launch cycle 0 of a 2-level hierarchy (both levels step; the
    coarse/fine registers go to the scratch array)."""
    import torch
    N0 = (16, 16, 16)
    grids = I.amr_hierarchy(3, N0, 2, seed=11, ext=(8, 16))
    fields = I.amr_fields(3, N0, 2, grids, seed=3, b_rms=0.3)
    log(f"case: noalloc vs workspace, 2-level hierarchy {len(grids)} grids, cycle 0")
    outs = []
    for noalloc in (True, False):
        H = A.Hierarchy(3, N0, grids, nlevels=2, ghost=4, dtype="f64")
        Ua, Ub = H.new_state(), H.new_state()
        for gi, f in enumerate(fields):
            H.load_primitive(Ua, gi, f["prim"], f["b"])
        H.fill(0, A.AMR_FILL_SAME_LEVEL, Ua)
        H.fill(1, A.AMR_FILL_FULL, Ua, Ua)
        H.dt0.fill_(2.0e-3)
        if noalloc:
            A.amr_advance_patches_noalloc(H.h, 0, None, 0, Ua.c, Ub.c, 0, H.dt0)
        else:
            A.amr_advance_patches(H.h, 0, None, 0, Ua.c, Ub.c, 0, H.dt0, H.ws)
        torch.cuda.synchronize()
        outs.append([H.store_interior(Ub, gi) for gi in range(len(grids))])
    for a, b in zip(*outs):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_noalloc_refuses_oversized_workspace():
    N = (136, 136, 136)  # FP64 workspace of 21 flux arrays over 145^3 elements: 489 MiB
    H = A.Hierarchy(3, N, [(0, (0, 0, 0), N)], ghost=4, dtype="f64")
    log(f"case: noalloc refusal, workspace {H.workspace_bytes / 2**20:.0f} MiB")
    U, V = H.new_state(), H.new_state()
    with pytest.raises(A.AmrError) as e:
        A.amr_advance_patches_noalloc(H.h, 0, None, 4, U.c, V.c, 0, H.dt0)
    assert "allocation-free" in str(e.value)
