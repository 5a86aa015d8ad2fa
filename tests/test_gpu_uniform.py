"""GPU parity of the single-grid advance against the FP64 oracle, through
the C ABI (HIP kernels for gfx950)."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import inputs as I
from tests.gpu_util import log, normwise_errors, uniform_gpu

pytestmark = pytest.mark.gpu
GAMMA = 5.0 / 3.0


def test_uniform_state_unchanged_bitwise_gpu():
    log("case: uniform state 3D 20x18x22 f64 g=4")
    ic = I.uniform_state(3, (20, 18, 22))
    want = O.conserved_interior(ic, GAMMA)
    got, _, flags = uniform_gpu(ic, 4, g=4, fill_every=2)
    assert flags[0] == 0
    for a, b in zip(got, want):
        assert np.array_equal(a, b)


def test_small_2d_parity_f64():
    """64x64 2D periodic, g = 2 refreshed every step (the plain-method
    configuration), 100 steps."""
    log("case: 2D 64x64 seed 1 f64 100 steps")
    ic = I.smooth_mhd(2, (64, 64), seed=1, v_rms=0.1, b_rms=0.1)
    want, dts_o = O.uniform_run(ic, GAMMA, 0.4, 100, g=2)
    got, dts_g, flags = uniform_gpu(ic, 100, g=2)
    assert flags[0] == 0
    err = normwise_errors(got, want)
    log(f"  errors per field: {err}")
    assert np.all(err <= 1e-10), err
    assert np.max(np.abs(dts_g - dts_o) / dts_o) < 1e-12


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_3d_jump_parity_ragged(dtype, tol):
    """3D ragged extents (several flux tiles and z-chunks plus a partial
    tile), g = 4 filled every 2 steps, density jump 4:1."""
    n = (37, 33, 35)
    log(f"case: 3D {n} seed 2 jump {dtype} 8 steps")
    ic = I.smooth_mhd(3, n, seed=2, v_rms=0.1, b_rms=0.3, jump=True)
    want, dts_o = O.uniform_run(ic, GAMMA, 0.4, 8, g=4, fill_every=2)
    got, dts_g, flags = uniform_gpu(ic, 8, g=4, fill_every=2, dtype=dtype)
    assert flags[0] == 0
    err = normwise_errors(got, want)
    log(f"  errors per field: {err}")
    assert np.all(err <= tol), err


def test_3d_band2_every_step_f64():
    n = (24, 20, 18)
    log(f"case: 3D {n} g=2 f64 6 steps")
    ic = I.smooth_mhd(3, n, seed=5, v_rms=0.2, b_rms=0.3, jump=True)
    want, _ = O.uniform_run(ic, GAMMA, 0.4, 6, g=2)
    got, _, flags = uniform_gpu(ic, 6, g=2)
    assert flags[0] == 0
    err = normwise_errors(got, want)
    log(f"  errors per field: {err}")
    assert np.all(err <= 1e-10), err


def test_outflow_brio_wu_f64():
    log("case: Brio-Wu 2D 200x4 outflow f64")
    ic = I.brio_wu(200)
    nsteps = 120
    dts = np.full(nsteps, 0.1 / 240)
    want, _ = O.uniform_run(ic, 2.0, 0.4, nsteps, g=2, bc=(1, 0, 0), dts=dts)
    got, _, flags = uniform_gpu(ic, nsteps, g=2, gamma=2.0, bc=(1, 0, 0), dts=dts)
    assert flags[0] == 0
    err = normwise_errors(got, want)
    log(f"  errors per field: {err}")
    assert np.all(err <= 1e-10), err


def test_run_twice_bitwise_and_nonphysical_flag():
    log("case: determinism 3D 32^3 f64 4 steps")
    ic = I.smooth_mhd(3, (32, 32, 32), seed=8, b_rms=0.3, jump=True)
    a, _, _ = uniform_gpu(ic, 4, g=4, fill_every=2)
    b, _, _ = uniform_gpu(ic, 4, g=4, fill_every=2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # a negative pressure planted in the input must raise the device flag
    bad = {k: (list(v) if isinstance(v, list) else v) for k, v in ic.items()}
    bad["prim"] = [p.copy() for p in ic["prim"]]
    bad["prim"][4][3, 4, 5] = -1.0
    _, _, flags = uniform_gpu(bad, 1, g=4, fill_every=2)
    assert flags[0] & 1 and flags[1] >= 0
