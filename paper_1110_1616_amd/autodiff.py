"""Reverse-mode differentiation of the advance under torch.autograd.

Three autograd Functions wrap library calls and their hand-written adjoints
(every step runs in the library's HIP kernels; this module only marshals):

* ``LoadPrimitive``  (rho, vx, vy, vz) of one grid -> state pools, with the
  pressure and face B held fixed (adjoint: amr_load_primitive_adjoint);
* ``Advance``        state pools -> state pools after len(dts) steps of one
  level, each a same-level band copy then a band-2 step (adjoint:
  amr_advance_adjoint).  The forward keeps a copy of the state every
  ``every`` steps; the backward walks the segments last to first, and the
  library recomputes each segment's forward states from its checkpoint
  before sweeping it in reverse;
* ``StoreInterior``  state pools -> interior arrays of one grid (adjoint:
  amr_store_interior_adjoint).

A loss written in torch on the interior arrays then back-propagates to the
initial density and velocity.  The band elements of Advance's output are
not state: a loss must not read them (their adjoint is dropped).
"""

from __future__ import annotations

import torch

from . import amr as A


def _pool_grads(H, grads):
    out = []
    for g in grads:
        if g is None:
            out.append(torch.zeros(H.state_elems, dtype=H.dtype, device=H.device))
        else:
            out.append(g.contiguous().clone())
    return out


class LoadPrimitive(torch.autograd.Function):
    """(rho, vx, vy, vz, p, bx, by, bz) of grid gi -> 8 state pools (zero
    outside the grid's interior).  Differentiable in rho and v."""

    @staticmethod
    def forward(ctx, H, gi, rho, vx, vy, vz, p, bx, by, bz):
        prim = [t.contiguous() for t in (rho, vx, vy, vz, p)]
        out = [torch.zeros(H.state_elems, dtype=H.dtype, device=H.device) for _ in range(8)]
        A.amr_load_primitive(H.h, gi, prim, [bx.contiguous(), by.contiguous(), bz.contiguous()], A.State(out).c)
        ctx.H, ctx.gi = H, gi
        ctx.save_for_backward(*prim[:4])
        return tuple(out)

    @staticmethod
    def backward(ctx, *grads):
        H, gi = ctx.H, ctx.gi
        prim = ctx.saved_tensors
        lam = _pool_grads(H, grads)
        g = [torch.empty_like(prim[0]) for _ in range(4)]
        A.amr_load_primitive_adjoint(H.h, gi, list(prim), A.State(lam).c, g)
        return (None, None, g[0], g[1], g[2], g[3], None, None, None, None)


class Advance(torch.autograd.Function):
    """8 state pools -> 8 state pools after len(dts) steps of `level`
    (level-0 step sizes dts, frozen), checkpointed every `every` steps."""

    @staticmethod
    def forward(ctx, H, level, dts, every, *fields):
        dts = [float(x) for x in dts]
        if not dts:
            raise ValueError("Advance needs at least one step")
        if every < 1:
            raise ValueError("checkpoint interval must be >= 1")
        grids = [gi for gi, (lev, _, _) in enumerate(H.grids) if lev == level]
        if not grids:
            raise ValueError(f"level {level} has no grids")
        U = A.State([f.contiguous().clone() for f in fields])
        V = A.State([f.clone() for f in U.fields])
        ckpts = []
        for k, dt in enumerate(dts):
            if k % every == 0:
                ckpts.append([f.clone() for f in U.fields])
            A.amr_fill_ghosts_prolong(H.h, level, A.AMR_FILL_SAME_LEVEL, U.c, None)
            H.dt0.fill_(dt)
            if H.nlevels == 1:
                A.amr_advance_patches(H.h, 0, None, 2, U.c, V.c, 0, H.dt0, H.ws)
            else:
                A.amr_advance_patches(H.h, -1, grids, 2, U.c, V.c, 0, H.dt0, H.ws)
            U, V = V, U
        ctx.H, ctx.level, ctx.dts, ctx.every, ctx.ckpts = H, level, dts, every, ckpts
        return tuple(U.fields)

    @staticmethod
    def backward(ctx, *grads):
        H, level, dts, every = ctx.H, ctx.level, ctx.dts, ctx.every
        lam = A.State(_pool_grads(H, grads))
        nbytes = A.amr_adjoint_workspace(H.h, -(level + 1), min(every, len(dts)))
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=H.device)
        for si in reversed(range(len(ctx.ckpts))):
            k0 = si * every
            k1 = min(k0 + every, len(dts))
            A.amr_advance_adjoint(H.h, -(level + 1), dts[k0:k1], A.State(ctx.ckpts[si]).c, lam.c, ws)
        ctx.ckpts = None
        return (None, None, None, None, *lam.fields)


class StoreInterior(torch.autograd.Function):
    """8 state pools -> the 8 interior float64 arrays of grid gi."""

    @staticmethod
    def forward(ctx, H, gi, *fields):
        outs = [torch.zeros(s, dtype=torch.float64, device=H.device) for s in H.interior_shapes(gi)]
        A.amr_store_interior(H.h, gi, A.State([f.contiguous() for f in fields]).c, outs)
        ctx.H, ctx.gi = H, gi
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        H, gi = ctx.H, ctx.gi
        shapes = H.interior_shapes(gi)
        g = [torch.zeros(s, dtype=torch.float64, device=H.device) if x is None
             else x.to(torch.float64).contiguous() for x, s in zip(grads, shapes)]
        lam = [torch.zeros(H.state_elems, dtype=H.dtype, device=H.device) for _ in range(8)]
        A.amr_store_interior_adjoint(H.h, gi, g, A.State(lam).c)
        return (None, None, *lam)


def advance(H, level, dts, fields, every=5):
    """Differentiable multi-step advance of one level (see Advance)."""
    return Advance.apply(H, level, list(dts), every, *fields)
