"""GPU parity of the upwinded constrained-transport EMF (Gardiner & Stone
2005; the scheme option AMR_EMF_UPWIND) against the FP64 oracle run with the
same option: single grids (2D, 3D with a density jump, FP64 and FP32), the
grid-aligned reduction on the GPU, and the 3-level hierarchy (the coarse/fine
EMF registers use the same edge values), batched == per-grid bitwise."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import amr as A
from paper_1110_1616_amd import inputs as I
from tests.gpu_util import amr_gpu, log, normwise_errors, uniform_gpu
from tests.test_oracle_upwind_emf import _brio_wu_sym

pytestmark = pytest.mark.gpu
GAMMA = 5.0 / 3.0


@pytest.fixture(autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_upwind_3d_jump_ragged(dtype, tol):
    ic = I.smooth_mhd(3, (37, 33, 35), seed=2, v_rms=0.1, b_rms=0.3, jump=True)
    log(f"case: upwind EMF 3D (37, 33, 35) jump {dtype} 8 steps")
    with O.emf(1):
        want, dts = O.uniform_run(ic, GAMMA, 0.4, 8, g=4, fill_every=2)
    got, dts_g, flags = uniform_gpu(ic, 8, g=4, fill_every=2, dtype=dtype, dts=dts, emf=1)
    assert flags[0] == 0
    err = normwise_errors(got, want)
    log(f"  errors per field: {err}")
    assert np.all(err <= tol), err


def test_upwind_2d_smooth_with_cfl():
    ic = I.smooth_mhd(2, (64, 64), seed=1, b_rms=0.1)
    log("case: upwind EMF 2D 64x64 smooth 40 steps, GPU CFL")
    with O.emf(1):
        want, dts = O.uniform_run(ic, GAMMA, 0.4, 40)
    got, dts_g, flags = uniform_gpu(ic, 40, emf=1)
    assert np.max(np.abs(dts_g - dts) / dts) < 1e-12
    err = normwise_errors(got, want)
    log(f"  errors per field: {err}")
    assert np.all(err <= 1e-10), err


def test_upwind_grid_aligned_reduction_on_gpu():
    """B_y (faces, CT with the upwinded EMF) and B_z (cells, flux update) stay
    equal in the y <-> z symmetric Brio-Wu problem (outflow along x)."""
    ic = _brio_wu_sym()
    log("case: upwind EMF Brio-Wu By = Bz, 60 steps")
    got, _, flags = uniform_gpu(ic, 60, gamma=2.0, bc=(1, 0, 0), emf=1)
    d = np.max(np.abs(got[6][0, 0, :] - got[7][0, 0, :]))
    log(f"  max |By_face - Bz_cell| = {d:.2e}")
    assert d < 1e-13
    with O.emf(1):
        want, _ = O.uniform_run(ic, 2.0, 0.4, 60, bc=(1, 0, 0))
    assert np.all(normwise_errors(got, want) <= 1e-10)


@pytest.mark.parametrize("key", ["3d", "2d"])
def test_upwind_multilevel_parity_and_batched_bitwise(key):
    ndim, N0, L, seed, ext = {"3d": (3, (24, 24, 24), 3, 11, (8, 16)), "2d": (2, (32, 32), 3, 4, (8, 16))}[key]
    grids = I.amr_hierarchy(ndim, N0, L, seed=seed, ext=ext)
    fields = I.amr_fields(ndim, N0, L, grids, seed=3, b_rms=0.3)
    log(f"case: upwind EMF {key} 3-level hierarchy, {len(grids)} grids, 2 coarse steps")
    with O.emf(1):
        want, dts_o = O.amr_run(ndim, N0, L, 4, grids, fields, 2)
    got, dts_g, flags = amr_gpu(ndim, N0, L, grids, fields, 2, emf=1)
    assert flags[0] == 0
    cat_g = [np.concatenate([g[s].ravel() for g in got]) for s in range(8)]
    cat_w = [np.concatenate([w[s].ravel() for w in want]) for s in range(8)]
    err = normwise_errors(cat_g, cat_w)
    log(f"  errors per field: {err}")
    assert np.all(err <= 1e-10), err
    ser, _, _ = amr_gpu(ndim, N0, L, grids, fields, 2, mode=1, emf=1)
    for ga, gb in zip(got, ser):
        for x, y in zip(ga, gb):
            assert np.array_equal(x, y)
    # and the option matters off grid alignment
    mean, _, _ = amr_gpu(ndim, N0, L, grids, fields, 2, emf=0)
    assert max(np.max(np.abs(a[5] - b[5])) for a, b in zip(mean, got)) > 1e-10


def test_upwind_rejects_adjoint_and_frozen():
    n = (16, 16, 16)
    H = A.Hierarchy(3, n, [(0, (0, 0, 0), n)], ghost=2, emf=1)
    with pytest.raises(A.AmrError) as e:
        A.amr_adjoint_workspace(H.h, 0, 1)
    assert e.value.status == A.AMR_EUNSUPPORTED
    with pytest.raises(A.AmrError) as e:
        A.amr_frozen_workspace(H.h)
    assert e.value.status == A.AMR_EUNSUPPORTED
