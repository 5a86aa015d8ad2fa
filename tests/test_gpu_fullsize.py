"""Parity at the benchmark's full sizes, in the launch configuration it
times: the 3-level FP64 hierarchy (base 112^3, 549 grids, 4.3M cells) for
one coarse step replayed from a captured HIP graph in the configuration the
autotuner picks there (fused advance, persistent launches, z-chunk 32,
window-start schedule), checked against the FP64 oracle on every element
and bit for bit against the two-kernel path under the predictive schedule;
and the 128^3 single grid (FP64 and FP32) for a band-4 step pair in its
tuned configuration (fused, XCD chunks), against the oracle."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import amr as A
from paper_1110_1616_amd import inputs as I
from tests.gpu_util import log, normwise_errors

pytestmark = pytest.mark.gpu
GAMMA = 5.0 / 3.0


@pytest.fixture(autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _amr3_graph_step(grids, fields, N0, L, cfg, schedule):
    import torch
    H = A.Hierarchy(3, N0, grids, nlevels=L, ghost=4)
    H.set_launch_config(*cfg)
    H.set_schedule(schedule)
    Ua, Ub = H.new_state(), H.new_state()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        H.graph_capture(Ua, Ub, 0)
    torch.cuda.synchronize()
    for gi, f in enumerate(fields):
        H.load_primitive(Ua, gi, f["prim"], f["b"])
    with torch.cuda.stream(stream):
        par = H.graph_launch(0)
    torch.cuda.synchronize()
    assert H.error_flags()[0] == 0
    got = [H.store_interior(H.current(Ua, Ub, par, l), gi) for gi, (l, lo, hi) in enumerate(grids)]
    return got, float(H.dt0.item())


def test_amr3_full_size_graph_replay_matches_oracle():
    N0, L = (112, 112, 112), 3
    grids = I.amr_hierarchy(3, N0, L, seed=3, ext=(8, 32))
    fields = I.amr_fields(3, N0, L, grids, seed=3, b_rms=0.3)
    log(f"case: 3-level hierarchy base 112^3, {len(grids)} grids, launch config 1,32,12,2, schedule 0, graph replay")
    got, dt0 = _amr3_graph_step(grids, fields, N0, L, (1, 32, 12, 2), 0)
    log("case: the same, two-kernel launch config 1,12,6,2, eta schedule, graph replay")
    two, _ = _amr3_graph_step(grids, fields, N0, L, (1, 12, 6, 2), 1)
    for gg, gt in zip(got, two):
        for x, y in zip(gg, gt):
            assert np.array_equal(x, y)
    log("  oracle coarse step ...")
    want, dts = O.amr_run(3, N0, L, 4, grids, fields, 1)
    cat_g = [np.concatenate([g[s].ravel() for g in got]) for s in range(8)]
    cat_w = [np.concatenate([w[s].ravel() for w in want]) for s in range(8)]
    err = normwise_errors(cat_g, cat_w)
    log(f"  errors per field: {err}; dt0 GPU {dt0:.10e} oracle {dts[0]:.10e}")
    assert abs(dt0 - dts[0]) <= 1e-12 * dts[0]
    assert np.all(err <= 1e-10), err


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_single128_full_size_matches_oracle(dtype, tol):
    n = (128, 128, 128)
    ic = I.smooth_mhd(3, n, seed=2, v_rms=0.1, b_rms=0.3, jump=True)
    log(f"case: single grid 128^3 {dtype}, band 4 step pair, launch config 1,32,10")
    H = A.Hierarchy(3, n, [(0, (0, 0, 0), n)], ghost=4, dtype=dtype, dx0=ic["dx"], gamma=GAMMA, cfl=0.4)
    H.set_launch_config(1, 32, 10)
    U, V = H.new_state(), H.new_state()
    H.load_primitive(U, 0, ic["prim"], ic["b"])
    want, dts = O.uniform_run(ic, GAMMA, 0.4, 2, g=4, fill_every=2)
    H.fill(0, A.AMR_FILL_SAME_LEVEL, U)
    for s, band in enumerate((4, 2)):
        H.dt0.fill_(float(dts[s]))
        H.advance(U, V, cycle=0, band=band)
        U, V = V, U
    got = H.store_interior(U, 0)
    assert H.error_flags()[0] == 0
    err = normwise_errors(got, want)
    log(f"  errors per field: {err}")
    assert np.all(err <= tol), err
