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
                return_state=False):
    """Single periodic (or outflow) grid advanced on the GPU through the ABI."""
    import torch
    ndim, n = ic["ndim"], tuple(ic["n"])
    lo = (0,) * ndim
    H = A.Hierarchy(ndim, n, [(0, lo, n)], ghost=g, dtype=dtype, bc=bc, dx0=ic["dx"], gamma=gamma, cfl=cfl)
    U, V = H.new_state(), H.new_state()
    H.load_primitive(U, 0, ic["prim"], ic["b"])
    used = []
    gv = g
    for s in range(nsteps):
        if s % fill_every == 0:
            H.fill(0, A.AMR_FILL_FULL, U)
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
