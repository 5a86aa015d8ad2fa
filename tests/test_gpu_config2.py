"""The single-grid workload at its stated size and length: one 128^3 grid
with a 4-cell halo refilled every 2 steps (a band-4 step, then a band-2
step), seeded smooth Fourier-mode rho / v / A fields (|B| ~ 0.3) plus a 4:1
planar density jump, 50 steps with the CFL time step, run in FP64 and FP32
on the GPU and compared with the FP64 oracle on every interior element."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import inputs as I
from tests.gpu_util import log, normwise_errors, uniform_gpu

pytestmark = pytest.mark.gpu
GAMMA = 5.0 / 3.0
N = (128, 128, 128)
STEPS = 50


@pytest.fixture(scope="module")
def oracle_run():
    ic = I.smooth_mhd(3, N, seed=2, v_rms=0.1, b_rms=0.3, jump=True)
    log(f"oracle: 128^3 jump, {STEPS} steps on {O.max_threads()} threads ...")
    want, dts = O.uniform_run(ic, GAMMA, 0.4, STEPS, g=4, fill_every=2)
    log("oracle: done")
    return ic, want, dts


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_config2_128cubed_50_steps(oracle_run, dtype, tol):
    ic, want, dts_o = oracle_run
    log(f"case: 128^3 jump {dtype}, {STEPS} steps, g=4 refilled every 2 steps, GPU dt")
    got, dts_g, flags = uniform_gpu(ic, STEPS, g=4, fill_every=2, dtype=dtype)
    assert flags[0] == 0
    err = normwise_errors(got, want)
    dterr = np.max(np.abs(dts_g - dts_o) / dts_o)
    log(f"  errors against FP64 per field: {err}; max dt relative difference {dterr:.3e}")
    assert np.all(err <= tol), err
    assert dterr <= (1e-12 if dtype == "f64" else 1e-6)
