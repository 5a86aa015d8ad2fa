"""The fused flux-update kernel (launch mode bit 3) against the two-kernel
path: it forms every face flux, edge EMF and update with the same source
expressions, keeping the face fluxes in LDS instead of HBM and storing only
those the coarse/fine registers read.  The device code is compiled with
multiply-add contraction inside each source expression only, so the same
expression gives the same bits in either kernel: the fused results equal
the two-kernel ones bit for bit, in FP64 and FP32, 2-D and 3-D, under every
fused configuration (one block per item, persistent, XCD chunks; batched,
per-grid, graph replay).
Covered: ragged single grids in 3D (FP64, FP32) and 2D, a 3-level hierarchy
over two coarse steps (registers, reflux, EMF fix and restriction read the
stored fluxes), the 6-level subvolume; plus the FP64 oracle at 1e-10."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import amr as A
from paper_1110_1616_amd import inputs as I
from tests.gpu_util import log, normwise_errors

pytestmark = pytest.mark.gpu
GAMMA = 5.0 / 3.0


def _single(ic, steps, mode, dtype, g=4, fill_every=2):
    import torch
    ndim, n = ic["ndim"], tuple(ic["n"])
    H = A.Hierarchy(ndim, n, [(0, (0,) * ndim, n)], ghost=g, dtype=dtype, dx0=ic["dx"], gamma=GAMMA)
    H.set_launch_config(1, 12, mode)
    U, V = H.new_state(), H.new_state()
    H.load_primitive(U, 0, ic["prim"], ic["b"])
    gv = g
    for s in range(steps):
        if s % fill_every == 0:
            H.fill(0, A.AMR_FILL_SAME_LEVEL, U)
            gv = g
        H.compute_dt(U)
        H.advance(U, V, cycle=0, band=gv)
        U, V = V, U
        gv -= 2
    torch.cuda.synchronize()
    assert H.error_flags()[0] == 0
    return H.store_interior(U, 0)


@pytest.mark.parametrize("ndim,n,dtype", [(3, (37, 33, 35), "f64"), (3, (37, 33, 35), "f32"), (3, (9, 70, 12), "f64"),
                                          (2, (70, 53), "f64"), (2, (70, 53), "f32")])
def test_fused_single_grid(ndim, n, dtype):
    log(f"case: fused vs two kernels, single grid {ndim}D {n} {dtype}")
    ic = I.smooth_mhd(ndim, n, seed=2, v_rms=0.1, b_rms=0.3, jump=True)
    ref = _single(ic, 6, 2, dtype)
    fused = [_single(ic, 6, mode, dtype) for mode in (8, 10, 12)]
    for got in fused[1:]:
        for s in range(8):
            assert np.array_equal(got[s], fused[0][s]), A.FIELDS[s]
    err = normwise_errors(fused[0], ref)
    log(f"  fused vs two kernels, normwise: {err}")
    for s in range(8):
        assert np.array_equal(fused[0][s], ref[s]), A.FIELDS[s]


def _amr(grids, fields, N0, L, mode, form, dtype="f64", ncoarse=2):
    import torch
    H = A.Hierarchy(3, N0, grids, nlevels=L, ghost=4, dtype=dtype)
    H.set_launch_config(1, 16, mode)
    Ua, Ub = H.new_state(), H.new_state()
    for gi, f in enumerate(fields):
        H.load_primitive(Ua, gi, f["prim"], f["b"])
    par = 0
    if form == "graph":
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            H.graph_capture(Ua, Ub, 0)
        torch.cuda.synchronize()
        for gi, f in enumerate(fields):
            H.load_primitive(Ua, gi, f["prim"], f["b"])
        for _ in range(ncoarse):
            with torch.cuda.stream(stream):
                par = H.graph_launch(par)
    else:
        for _ in range(ncoarse):
            par = H.coarse_step(Ua, Ub, par, 1 if form == "per_grid" else 0)
    torch.cuda.synchronize()
    assert H.error_flags()[0] == 0
    return [H.store_interior(H.current(Ua, Ub, par, l), gi) for gi, (l, lo, hi) in enumerate(grids)]


def test_fused_multilevel_forms_and_oracle():
    N0, L = (24, 24, 24), 3
    grids = I.amr_hierarchy(3, N0, L, seed=11, ext=(8, 16))
    fields = I.amr_fields(3, N0, L, grids, seed=3, b_rms=0.3)
    log(f"case: fused multilevel, {len(grids)} grids, 2 coarse steps")
    two = _amr(grids, fields, N0, L, 2, "batched")
    ref = _amr(grids, fields, N0, L, 8, "batched")
    for mode, form in ((14, "batched"), (8, "per_grid"), (10, "graph")):
        got = _amr(grids, fields, N0, L, mode, form)
        for gg, gw in zip(got, ref):
            for x, y in zip(gg, gw):
                assert np.array_equal(x, y), (mode, form)
    want, _ = O.amr_run(3, N0, L, 4, grids, fields, 2)
    for name, res in (("fused", ref), ("two-kernel", two)):
        cat_g = [np.concatenate([g[s].ravel() for g in res]) for s in range(8)]
        cat_w = [np.concatenate([w[s].ravel() for w in want]) for s in range(8)]
        err = normwise_errors(cat_g, cat_w)
        log(f"  {name} errors per field vs oracle: {err}")
        assert np.all(err <= 1e-10)
    cat_f = [np.concatenate([g[s].ravel() for g in ref]) for s in range(8)]
    cat_t = [np.concatenate([g[s].ravel() for g in two]) for s in range(8)]
    err = normwise_errors(cat_f, cat_t)
    log(f"  fused vs two-kernel: {err}")
    for x, y in zip(cat_f, cat_t):
        assert np.array_equal(x, y)


def test_fused_deep_subvolume():
    grids, fields = I.deep_hierarchy(100, seed=5)
    N0, L = (100, 100, 100), 6
    log(f"case: fused, 6-level subvolume {len(grids)} grids, FP32, one coarse step")
    ref = _amr(grids, fields, N0, L, 3, "batched", dtype="f32", ncoarse=1)
    got = _amr(grids, fields, N0, L, 11, "batched", dtype="f32", ncoarse=1)
    got2 = _amr(grids, fields, N0, L, 9, "batched", dtype="f32", ncoarse=1)
    for gg, gw in zip(got2, got):
        for x, y in zip(gg, gw):
            assert np.array_equal(x, y)
    cat_g = [np.concatenate([g[s].ravel() for g in got]) for s in range(8)]
    cat_r = [np.concatenate([g[s].ravel() for g in ref]) for s in range(8)]
    err = normwise_errors(cat_g, cat_r)
    log(f"  fused vs two-kernel FP32: {err}")
    for x, y in zip(cat_g, cat_r):
        assert np.array_equal(x, y)
