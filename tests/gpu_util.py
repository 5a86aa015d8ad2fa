"""Helpers of the GPU parity tests: drive the HIP path through the C ABI and
compare with the oracle."""

import sys

import numpy as np

from paper_1110_1616_amd import amr as A


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def normwise_errors(got, want):
    """Per field: max|a - b| / max|b| over interior cells / faces."""
    out = []
    for a, b in zip(got, want):
        den = np.max(np.abs(b))
        num = np.max(np.abs(np.asarray(a) - np.asarray(b)))
        out.append(num / den if den > 0 else num)
    return np.array(out)


def uniform_gpu(ic, nsteps, g=2, fill_every=1, dtype="f64", gamma=5.0 / 3.0, cfl=0.4, bc=(0, 0, 0), dts=None,
                return_state=False, emf=0):
    """Single periodic (or outflow) grid advanced on the GPU through the ABI."""
    import torch
    ndim, n = ic["ndim"], tuple(ic["n"])
    lo = (0,) * ndim
    H = A.Hierarchy(ndim, n, [(0, lo, n)], ghost=g, dtype=dtype, bc=bc, dx0=ic["dx"], gamma=gamma, cfl=cfl, emf=emf)
    U, V = H.new_state(), H.new_state()
    H.load_primitive(U, 0, ic["prim"], ic["b"])
    used = []
    gv = g
    for s in range(nsteps):
        if s % fill_every == 0:
            H.fill(0, A.AMR_FILL_SAME_LEVEL, U)
            gv = g
        if dts is None:
            H.compute_dt(U)
        else:
            H.dt0.fill_(float(dts[s]))
        used.append(H.dt0)
        used[-1] = float(H.dt0.item()) if dts is None else float(dts[s])
        H.advance(U, V, cycle=0, band=gv)
        U, V = V, U
        gv -= 2
    torch.cuda.synchronize()
    out = H.store_interior(U, 0)
    flags = H.error_flags()
    if return_state:
        return out, np.array(used), flags, H, U
    return out, np.array(used), flags


def amr_gpu(ndim, N0, L, grids, fields, ncoarse, dtype="f64", mode=0, ghost=4, return_handle=False, emf=0):
    """Hierarchy advanced ncoarse coarse steps on the GPU (mode 0 batched,
    1 per-grid serial).  Returns (per-grid interior arrays, dt0 per step,
    error flags)."""
    import torch
    H = A.Hierarchy(ndim, N0, grids, nlevels=L, ghost=ghost, dtype=dtype, emf=emf)
    Ua, Ub = H.new_state(), H.new_state()
    for gi, f in enumerate(fields):
        H.load_primitive(Ua, gi, f["prim"], f["b"])
    par = 0
    dts = []
    for _ in range(ncoarse):
        par = H.coarse_step(Ua, Ub, par, mode)
        dts.append(float(H.dt0.item()))
    torch.cuda.synchronize()
    outs = [H.store_interior(H.current(Ua, Ub, par, l), gi) for gi, (l, lo, hi) in enumerate(grids)]
    flags = H.error_flags()
    if return_handle:
        return outs, np.array(dts), flags, (H, Ua, Ub, par)
    return outs, np.array(dts), flags


def grid_box(H, U, gi):
    """The padded box of grid gi of pool state U as 8 numpy arrays shaped
    like the oracle's banded layout (layout documented in amr.h)."""
    import torch  # noqa: F401
    l, lo, hi = H.grids[gi]
    ndim, g = H.ndim, H.ghost
    n = [hi[a] - lo[a] for a in range(3)]
    P = [n[a] + 2 * g + 1 if a < ndim else 1 for a in range(3)]
    off = H.offsets[gi]
    size = P[0] * P[1] * P[2]
    out = []
    for s in range(8):
        box = U.fields[s][off:off + size].reshape(P[2], P[1], P[0]).double().cpu().numpy()
        ext = [n[a] + 2 * g if a < ndim else 1 for a in range(3)]
        if s >= 5 and (s - 5) < ndim:
            ext[s - 5] += 1
        out.append(box[:ext[2], :ext[1], :ext[0]].copy())
    return out
