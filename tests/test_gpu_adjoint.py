"""GPU discrete adjoint against the oracle's reverse and forward modes, and
against centred finite differences of the GPU forward run.

The loss is the kinetic energy of the cells of a (periodically wrapped) box
after the last step; the controls are the initial density and velocity.  The
GPU gradient comes from torch.autograd through LoadPrimitive -> Advance ->
StoreInterior (hand-written adjoint kernels), with checkpoints every few
steps."""

import numpy as np
import pytest

import oracle as O
from paper_1110_1616_amd import inputs as I

from gpu_util import log

GAMMA = 5.0 / 3.0
pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def ke_loss_torch(torch, interior, ndim, n, lo, ln):
    """Kinetic energy sum over the box, times the cell volume."""
    rho, mx, my, mz = interior[:4]
    idx = [torch.tensor([(lo[a] + t) % n[a] for t in range(ln[a])], device=rho.device) for a in range(ndim)]
    def sub(x):
        x = x.index_select(2, idx[0]).index_select(1, idx[1])
        return x.index_select(0, idx[2]) if ndim == 3 else x
    dv = 1.0
    for a in range(ndim):
        dv /= n[a]
    r, a, b, c = sub(rho), sub(mx), sub(my), sub(mz)
    return ((a * a + b * b + c * c) / (2.0 * r)).sum() * dv


def gpu_loss_grad(ic, dts, box, every, ghost=2, dtype="f64", tiles=None, need_grad=True):
    """(J, [grad_rho, grad_vx, grad_vy, grad_vz]) on the GPU.  tiles: optional
    list of (lo, hi) sub-boxes that tile the periodic domain as separate
    level-0 grids."""
    torch = _torch()
    from paper_1110_1616_amd import amr as A
    from paper_1110_1616_amd import autodiff as AD
    ndim, n = ic["ndim"], tuple(ic["n"])
    if tiles is None:
        tiles = [((0,) * ndim, n)]
    parts = I.split_grid_fields(ic, tiles)
    H = A.Hierarchy(ndim, n, [(0, lo, hi) for lo, hi in tiles], ghost=ghost, dtype=dtype, dx0=ic["dx"],
                    gamma=GAMMA)
    dev = H.device
    ctrls, pools = [], None
    for gi, f in enumerate(parts):
        c = [torch.tensor(np.asarray(p), dtype=torch.float64, device=dev, requires_grad=(i < 4 and need_grad))
             for i, p in enumerate(f["prim"])]
        bb = [torch.tensor(np.asarray(x), dtype=torch.float64, device=dev) for x in f["b"]]
        ctrls.append(c)
        U = AD.LoadPrimitive.apply(H, gi, *c, *bb)
        pools = list(U) if pools is None else [p + u for p, u in zip(pools, U)]
    out = AD.advance(H, 0, dts, pools, every=every)
    # assemble the global interior cell arrays from the grids
    cz, cy, cx = (n[2] if ndim == 3 else 1), n[1], n[0]
    glob = [torch.zeros((cz, cy, cx), dtype=torch.float64, device=dev) for _ in range(4)]
    for gi, (lo, hi) in enumerate(tiles):
        inter = AD.StoreInterior.apply(H, gi, *out)
        lo3 = tuple(lo) + (0,) * (3 - ndim)
        hi3 = tuple(hi) + (1,) * (3 - ndim)
        sl = (slice(lo3[2], hi3[2]), slice(lo3[1], hi3[1]), slice(lo3[0], hi3[0]))
        for q in range(4):
            glob[q][sl] = inter[q]
    J = ke_loss_torch(torch, glob, ndim, n, box[0], box[1])
    if not need_grad:
        return float(J.item()), None, H
    J.backward()
    torch.cuda.synchronize()
    grads = []
    shp = np.asarray(ic["prim"][0]).shape
    for q in range(4):
        g = np.zeros((cz, cy, cx))
        for gi, (lo, hi) in enumerate(tiles):
            lo3 = tuple(lo) + (0,) * (3 - ndim)
            hi3 = tuple(hi) + (1,) * (3 - ndim)
            g[lo3[2]:hi3[2], lo3[1]:hi3[1], lo3[0]:hi3[0]] = ctrls[gi][q].grad.cpu().numpy()
        grads.append(g.reshape(shp))
    return float(J.item()), grads, H


def _case(ndim):
    if ndim == 3:
        ic = I.smooth_mhd(3, (16, 16, 16), seed=4, v_rms=0.1, b_rms=0.3)
        box = ((11, 2, 9), (6, 6, 6))
        nsteps = 4
    else:
        ic = I.smooth_mhd(2, (24, 24), seed=4, v_rms=0.1, b_rms=0.3)
        box = ((17, 3), (12, 12))
        nsteps = 7
    _, dts = O.uniform_run(ic, GAMMA, 0.4, nsteps, g=2)
    return ic, dts, box


def _relerr(got, want):
    den = max(float(np.max(np.abs(w))) for w in want)
    return max(float(np.max(np.abs(g - w))) for g, w in zip(got, want)) / den


@pytest.mark.parametrize("ndim,ghost,every", [(3, 2, 2), (3, 4, 3), (2, 2, 5), (2, 4, 3)])
def test_gpu_gradient_matches_oracle_adjoint(ndim, ghost, every):
    ic, dts, box = _case(ndim)
    log(f"adjoint parity ndim={ndim} ghost={ghost} every={every} steps={len(dts)}")
    Jo, go = O.ke_grad(ic, GAMMA, dts, box[0], box[1])
    J, g, _ = gpu_loss_grad(ic, dts, box, every, ghost=ghost)
    assert J == pytest.approx(Jo, rel=1e-12)
    err = _relerr(g, go)
    log(f"  J={J:.6e}  max rel grad err vs oracle = {err:.2e}")
    assert err <= 1e-10


def test_gpu_gradient_multigrid_level_matches_oracle():
    """Four level-0 grids tiling the periodic domain: the band copies between
    grids are transposed by the fold, so the gradient is the single-grid one."""
    ic, dts, box = _case(3)
    tiles = [((0, 0, 0), (8, 8, 16)), ((8, 0, 0), (16, 8, 16)), ((0, 8, 0), (8, 16, 16)), ((8, 8, 0), (16, 16, 16))]
    log("adjoint parity, 4 grids on level 0")
    Jo, go = O.ke_grad(ic, GAMMA, dts, box[0], box[1])
    J, g, _ = gpu_loss_grad(ic, dts, box, 2, ghost=4, tiles=tiles)
    assert J == pytest.approx(Jo, rel=1e-12)
    err = _relerr(g, go)
    log(f"  max rel grad err vs oracle = {err:.2e}")
    assert err <= 1e-10


def test_gpu_gradient_fp32_against_fp64_oracle():
    ic, dts, box = _case(3)
    Jo, go = O.ke_grad(ic, GAMMA, dts, box[0], box[1])
    J, g, _ = gpu_loss_grad(ic, dts, box, 2, ghost=2, dtype="f32")
    err = _relerr(g, go)
    log(f"adjoint FP32: J rel err {abs(J - Jo) / abs(Jo):.2e}, grad rel err vs FP64 oracle {err:.2e}")
    assert abs(J - Jo) <= 1e-5 * abs(Jo)
    assert err <= 1e-5


def test_gpu_gradient_dot_tlm_64cubed():
    """The differentiation workload: 64^3 periodic, 20 steps, checkpoints
    every 5; <grad, d> on the GPU equals the oracle's forward-mode dJ[d]."""
    n = (64, 64, 64)
    ic = I.smooth_mhd(3, n, seed=4, v_rms=0.1, b_rms=0.3)
    box = I.loss_box(3, n, 16, seed=44)
    _, dts = O.uniform_run(ic, GAMMA, 0.4, 20, g=2)
    log(f"64^3 x 20 steps adjoint: box {box}")
    J, g, _ = gpu_loss_grad(ic, dts, box, 5, ghost=2)
    dirs = I.control_directions(np.asarray(ic["prim"][0]).shape, 2, seed=444)
    for d in dirs:
        Jt, dJ = O.ke_tlm(ic, GAMMA, dts, box[0], box[1], d)
        adj = sum(float(np.sum(gi * di)) for gi, di in zip(g, d))
        log(f"  J {J:.12e} vs {Jt:.12e}; <g,d> {adj:.12e} vs TLM {dJ:.12e} rel {abs(adj - dJ) / abs(dJ):.2e}")
        assert J == pytest.approx(Jt, rel=1e-12)
        assert abs(adj - dJ) <= 1e-10 * abs(dJ)


def _ke_numpy(interior, ndim, n, lo, ln):
    rho, mx, my, mz = interior[:4]
    sl = [np.array([(lo[a] + t) % n[a] for t in range(ln[a])]) for a in range(ndim)]
    def sub(x):
        x = x[:, :, sl[0]][:, sl[1], :]
        return x[sl[2], :, :] if ndim == 3 else x
    dv = 1.0 / np.prod(n[:ndim])
    return float(np.sum((sub(mx) ** 2 + sub(my) ** 2 + sub(mz) ** 2) / (2.0 * sub(rho))) * dv)


class FrozenRunner:
    """Loss after the frozen-branch run (branches decided by the unperturbed
    run) from controls perturbed along d."""

    def __init__(self, ic, dts, box):
        torch = _torch()
        from paper_1110_1616_amd import amr as A
        self.A, self.torch = A, torch
        self.ic, self.dts, self.box = ic, dts, box
        n = tuple(ic["n"])
        self.H = A.Hierarchy(ic["ndim"], n, [(0, (0,) * ic["ndim"], n)], ghost=2, dtype="f64", dx0=ic["dx"],
                             gamma=GAMMA)
        self.ws = torch.empty(A.amr_frozen_workspace(self.H.h), dtype=torch.uint8, device="cuda")
        self.Ub = self.H.new_state()
        self.H.load_primitive(self.Ub, 0, ic["prim"], ic["b"])
        self.Up = self.H.new_state()

    def loss(self, eps, d):
        ic = self.ic
        prim = [p + eps * dd for p, dd in zip(ic["prim"][:4], d)] + [ic["prim"][4]]
        self.H.load_primitive(self.Up, 0, prim, ic["b"])
        self.A.amr_advance_frozen(self.H.h, 0, self.dts, self.Ub.c, self.Up.c, self.ws)
        out = self.H.store_interior(self.Up, 0)
        return _ke_numpy(out, ic["ndim"], tuple(ic["n"]), self.box[0], self.box[1])


def _config4():
    n = (64, 64, 64)
    ic = I.smooth_mhd(3, n, seed=4, v_rms=0.1, b_rms=0.3)
    box = I.loss_box(3, n, 16, seed=44)
    _, dts = O.uniform_run(ic, GAMMA, 0.4, 20, g=2)
    return n, ic, box, dts


def test_frozen_branch_run_at_zero_perturbation_is_the_forward_run():
    ic, dts, box = _case(3)
    fr = FrozenRunner(ic, dts, box)
    zero = [np.zeros_like(np.asarray(p)) for p in ic["prim"][:4]]
    Jf = fr.loss(0.0, zero)
    Jo = O.ke_loss(ic, GAMMA, dts, box[0], box[1])
    assert Jf == pytest.approx(Jo, rel=1e-13)


def test_gpu_gradient_against_frozen_branch_differences_64cubed():
    """The differentiation workload (64^3, 20 steps, 16^3 loss box) with 32
    seeded white-noise directions (N(0,1) x 0.1 per cell in rho and v) and
    eps = 1e-6.  The differences are taken along the branch of the discrete
    map that the unperturbed run follows (amr_advance_frozen), so kinks of
    the piecewise-smooth map within eps do not enter: every direction must
    agree with <grad J, d> to 1e-6 relative."""
    n, ic, box, dts = _config4()
    J, g, _ = gpu_loss_grad(ic, dts, box, 5, ghost=2)
    fr = FrozenRunner(ic, dts, box)
    dirs = I.control_directions(np.asarray(ic["prim"][0]).shape, 32, seed=444)
    worst = 0.0
    for i, d in enumerate(dirs):
        adj = sum(float(np.sum(gi * di)) for gi, di in zip(g, d))
        fd = (fr.loss(1e-6, d) - fr.loss(-1e-6, d)) / 2e-6
        rel = abs(fd - adj) / abs(adj)
        worst = max(worst, rel)
        log(f"  dir {i:2d}: <g,d>={adj:+.10e} frozen-branch FD rel err {rel:.1e}")
        assert rel <= 1e-6
    log(f"frozen-branch FD: worst of 32 = {worst:.1e}")


def test_gpu_gradient_against_plain_differences_smooth_directions_64cubed():
    """Plain centred differences of the GPU forward run (branches free to
    flip) along 8 seeded smooth directions (low Fourier modes, rms 0.1),
    eps = 1e-6: at most one direction may exceed 1e-6 relative (a branch
    kink within eps), none 1e-5."""
    n, ic, box, dts = _config4()
    J, g, _ = gpu_loss_grad(ic, dts, box, 5, ghost=2)
    dirs = I.smooth_directions(n, 8, seed=4444)
    bad = 0
    for i, d in enumerate(dirs):
        adj = sum(float(np.sum(gi * di)) for gi, di in zip(g, d))
        Jp = gpu_loss_grad({**ic, "prim": [p + 1e-6 * dd for p, dd in zip(ic["prim"][:4], d)] + [ic["prim"][4]]},
                           dts, box, 5, need_grad=False)[0]
        Jm = gpu_loss_grad({**ic, "prim": [p - 1e-6 * dd for p, dd in zip(ic["prim"][:4], d)] + [ic["prim"][4]]},
                           dts, box, 5, need_grad=False)[0]
        rel = abs((Jp - Jm) / 2e-6 - adj) / abs(adj)
        log(f"  smooth dir {i}: <g,d>={adj:+.10e} plain FD rel err {rel:.1e}")
        bad += rel > 1e-6
        assert rel <= 1e-5
    assert bad <= 1


@pytest.mark.parametrize("ndim", [3, 2])
def test_one_step_adjoint_matches_oracle_vjp_every_field(ndim):
    """One reverse step of the single periodic grid with a random adjoint on
    every field (cells and faces) against the oracle's vector-Jacobian
    product, element by element.  The oracle's fill makes the input face n a
    copy of face 0, while the GPU keeps face n as its own element (equal in
    value): the GPU's face-0 and face-n adjoints sum to the oracle's face 0."""
    torch = _torch()
    from paper_1110_1616_amd import amr as A
    n = (16, 12, 14) if ndim == 3 else (20, 18)
    ic = I.smooth_mhd(ndim, n, seed=9, v_rms=0.1, b_rms=0.3, p_amp=0.1)
    H = A.Hierarchy(ndim, n, [(0, (0,) * ndim, n)], ghost=2, dtype="f64", dx0=ic["dx"], gamma=GAMMA)
    U = H.new_state()
    H.load_primitive(U, 0, ic["prim"], ic["b"])
    Uin = H.store_interior(U, 0)
    dt = 1.5e-3
    rng = np.random.default_rng(21)
    lam_out = [rng.normal(size=np.asarray(u).shape) for u in Uin]
    want = O.step_vjp(ndim, n, GAMMA, dt, Uin, lam_out)
    lam = [torch.zeros(H.state_elems, dtype=torch.float64, device="cuda") for _ in range(8)]
    A.amr_store_interior_adjoint(H.h, 0, [torch.tensor(x, device="cuda") for x in lam_out], A.State(lam).c)
    ws = torch.empty(A.amr_adjoint_workspace(H.h, 0, 1), dtype=torch.uint8, device="cuda")
    A.amr_advance_adjoint(H.h, 0, [dt], U.c, A.State(lam).c, ws)
    got = H.store_interior(A.State(lam), 0)
    for a in range(ndim):
        s = 5 + a
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[2 - a] = 0
        hi[2 - a] = -1
        got[s][tuple(lo)] += got[s][tuple(hi)]
        got[s][tuple(hi)] = 0.0
    err = [float(np.max(np.abs(g - w)) / np.max(np.abs(w))) for g, w in zip(got, want)]
    log(f"one-step adjoint vs oracle VJP, {ndim}D, per field: {['%.1e' % e for e in err]}")
    assert max(err) <= 1e-12
