"""ctypes binding of the FP64 oracle (test infrastructure only).

Interior layout of whole fields (x fastest):
  cells (nz, ny, nx); Bx (nz, ny, nx+1); By (nz, ny+1, nx); Bz (nz+1, ny, nx),
  in 2D nz = 1 and Bz is a cell array.
Banded layout (the oracle's own patch storage): the same with every active
axis extended by the band g on both sides.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)

FIELDS = ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_last_error.restype = C.c_char_p
        L.orc_minmod.restype = C.c_double
        L.orc_minmod.argtypes = [C.c_double, C.c_double]
        L.orc_fast_speed.restype = C.c_double
        L.orc_fast_speed.argtypes = [C.c_double] * 5
        L.orc_uniform_time.restype = C.c_double
        L.orc_dt_banded.restype = C.c_double
        L.orc_max_threads.restype = C.c_int
        _LIB = L
    return _LIB


def set_emf(mode):
    """Edge EMF of the oracle's later steps: 0 arithmetic mean (Balsara &
    Spicer 1999), 1 upwinded (Gardiner & Stone 2005); 2 is 1 with the upwind
    side swapped (a planted mistake for sensitivity tests).  Returns the
    previous."""
    old = lib().orc_set_emf(int(mode))
    if old < 0:
        raise ValueError("emf mode must be 0, 1 or 2")
    return old


class emf:
    """Context manager: `with emf(1): ...` runs the oracle with upwinded EMFs."""

    def __init__(self, mode):
        self.mode = mode

    def __enter__(self):
        self.old = set_emf(self.mode)
        return self

    def __exit__(self, *exc):
        set_emf(self.old)
        return False


def _err():
    return lib().orc_last_error().decode()


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _ptrs(arrs):
    keep = [np.ascontiguousarray(a, dtype=np.float64) for a in arrs]
    pp = (_dp * len(keep))(*[k.ctypes.data_as(_dp) for k in keep])
    return keep, pp


def _ivec(v):
    v = list(v) + [1] * (3 - len(v))
    return (C.c_int * 3)(*[int(x) for x in v])


def _dvec(v):
    v = list(v) + [1.0] * (3 - len(v))
    return (C.c_double * 3)(*[float(x) for x in v])


def interior_shapes(ndim, n):
    nx, ny = n[0], n[1]
    nz = n[2] if ndim == 3 else 1
    cell = (nz, ny, nx)
    return [cell] * 5 + [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx) if ndim == 3 else cell]


def banded_shapes(ndim, n, g):
    nx, ny = n[0], n[1]
    nz = n[2] if ndim == 3 else 1
    gz = g if ndim == 3 else 0
    cell = (nz + 2 * gz, ny + 2 * g, nx + 2 * g)
    bz = (nz + 2 * gz + 1, ny + 2 * g, nx + 2 * g) if ndim == 3 else cell
    return [cell] * 5 + [(cell[0], cell[1], cell[2] + 1), (cell[0], cell[1] + 1, cell[2]), bz]


# ------------------------------------------------------------ pointwise pieces
def minmod(a, b):
    return lib().orc_minmod(float(a), float(b))


def prim_to_cons(W, gamma):
    W, pw = _arr(W)
    U = np.zeros(8)
    lib().orc_prim_to_cons(pw, U.ctypes.data_as(_dp), C.c_double(gamma))
    return U


def cons_to_prim(U, gamma):
    U, pu = _arr(U)
    W = np.zeros(8)
    lib().orc_cons_to_prim(pu, W.ctypes.data_as(_dp), C.c_double(gamma))
    return W


def phys_flux(W, d, gamma):
    W, pw = _arr(W)
    F = np.zeros(8)
    lib().orc_phys_flux(pw, C.c_int(d), C.c_double(gamma), F.ctypes.data_as(_dp))
    return F


def fast_speed(rho, p, B2, Bn, gamma):
    return lib().orc_fast_speed(rho, p, B2, Bn, gamma)


def hlld(L, R, gamma):
    """HLLD flux of rotated primitive states (rho, un, ut1, ut2, p, Bn, Bt1, Bt2).
    Returns (F[7], info) with info = (region, degen_L, degen_R, degen_double_star)."""
    L, pl = _arr(L)
    R, pr = _arr(R)
    F = np.zeros(7)
    info = (C.c_int * 4)()
    lib().orc_hlld(pl, pr, C.c_double(gamma), F.ctypes.data_as(_dp), info)
    return F, tuple(info)


class hlld_paths:
    """Context manager counting the oracle's HLLD paths inside it:
    `with hlld_paths() as c: ...` then c.counts = (evaluations, outer star
    degenerate, inner states evaluated, inner states degenerate)."""

    def __enter__(self):
        lib().orc_hlld_stats(C.c_int(1), None)
        self.counts = None
        return self

    def __exit__(self, *exc):
        out = (C.c_longlong * 4)()
        lib().orc_hlld_stats(C.c_int(0), out)
        self.counts = tuple(out)
        return False


# ------------------------------------------------------------------- runs
def uniform_run(ic, gamma, cfl, nsteps, g=2, fill_every=1, bc=(0, 0, 0), dts=None):
    """Run a single uniform grid for nsteps.  Returns (fields[8], dts)."""
    ndim, n = ic["ndim"], ic["n"]
    keep1, pp = _ptrs(ic["prim"])
    keep2, pb = _ptrs(ic["b"])
    outs = [np.zeros(s) for s in interior_shapes(ndim, n)]
    keep3, po = _ptrs(outs)
    dts_out = np.zeros(max(nsteps, 1))
    if dts is not None:
        dts_in = np.ascontiguousarray(dts, dtype=np.float64)
        pin = dts_in.ctypes.data_as(_dp)
    else:
        pin = None
    rc = lib().orc_uniform_run(C.c_int(ndim), _ivec(n), _ivec(bc), C.c_double(gamma), C.c_double(cfl),
                               _dvec(ic["dx"]), C.c_int(g), C.c_int(fill_every), C.c_int(nsteps), pin, pp, pb, po,
                               dts_out.ctypes.data_as(_dp))
    if rc != 0:
        raise RuntimeError("oracle uniform_run: " + _err())
    return keep3, dts_out[:nsteps]


def uniform_time(ic, gamma, cfl, nsteps, g=2, fill_every=1, bc=(0, 0, 0), threads=None):
    """Wall seconds of nsteps of the uniform run (set-up excluded)."""
    if threads:
        lib().orc_set_threads(int(threads))
    ndim, n = ic["ndim"], ic["n"]
    keep1, pp = _ptrs(ic["prim"])
    keep2, pb = _ptrs(ic["b"])
    t = lib().orc_uniform_time(C.c_int(ndim), _ivec(n), _ivec(bc), C.c_double(gamma), C.c_double(cfl),
                               _dvec(ic["dx"]), C.c_int(g), C.c_int(fill_every), C.c_int(nsteps), pp, pb)
    if t < 0:
        raise RuntimeError("oracle uniform_time: " + _err())
    return t


def max_threads():
    return lib().orc_max_threads()


def set_threads(n):
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------- banded patches
def step_banded(ndim, n, g, gv, gamma, dx, dt, fields):
    keep, pin = _ptrs(fields)
    outs = [np.zeros_like(f) for f in keep]
    keep2, pout = _ptrs(outs)
    rc = lib().orc_step_banded(C.c_int(ndim), _ivec(n), C.c_int(g), C.c_int(gv), C.c_double(gamma), _dvec(dx),
                               C.c_double(dt), pin, pout)
    if rc != 0:
        raise RuntimeError("oracle step_banded: " + _err())
    return keep2


def fill_banded(ndim, n, g, bc, fields):
    keep, pf = _ptrs(fields)
    rc = lib().orc_fill_banded(C.c_int(ndim), _ivec(n), C.c_int(g), _ivec(bc), pf)
    if rc != 0:
        raise RuntimeError("oracle fill_banded: " + _err())
    return keep


def dt_banded(ndim, n, g, gamma, cfl, dx, fields):
    keep, pf = _ptrs(fields)
    return lib().orc_dt_banded(C.c_int(ndim), _ivec(n), C.c_int(g), C.c_double(gamma), C.c_double(cfl), _dvec(dx),
                               pf)


def banded_from_interior(ndim, n, g, fields):
    """Place interior-layout conserved fields into banded arrays (band zero)."""
    out = [np.zeros(s) for s in banded_shapes(ndim, n, g)]
    gz = g if ndim == 3 else 0
    for s in range(8):
        f = np.asarray(fields[s])
        out[s][gz:gz + f.shape[0], g:g + f.shape[1], g:g + f.shape[2]] = f
    return out


def interior_from_banded(ndim, n, g, fields):
    shapes = interior_shapes(ndim, n)
    gz = g if ndim == 3 else 0
    return [np.array(fields[s][gz:gz + shapes[s][0], g:g + shapes[s][1], g:g + shapes[s][2]]) for s in range(8)]


def conserved_interior(ic, gamma):
    """The initial conserved state of an input set, as the oracle builds it
    (zero steps of a uniform run)."""
    f, _ = uniform_run(ic, gamma, 0.4, 0, g=2)
    return f


# ------------------------------------------------------------ hierarchies
def _grid_desc(ndim, grids):
    rows = []
    for (l, lo, hi) in grids:
        lo3 = list(lo) + [0] * (3 - len(lo))
        hi3 = list(hi) + [1] * (3 - len(hi))
        rows.append([l] + lo3 + hi3)
    return np.ascontiguousarray(np.array(rows, dtype=np.int32))


def _gshape(ndim, lo, hi):
    n = [hi[a] - lo[a] for a in range(ndim)]
    return tuple(n)


def amr_run(ndim, N0, nlev, g, grids, fields, ncoarse, gamma=5.0 / 3.0, cfl=0.4, dts=None):
    """Run ncoarse coarse steps of a hierarchy in the serial level order
    (level cycle 0, 1, 2, 2, 1, 2, 2 for three levels).  fields: per grid
    dict(prim=[5 arrays], b=[3 arrays]).  Returns (per-grid 8 arrays, dts)."""
    L = lib()
    L.orc_amr_last_error.restype = C.c_char_p
    desc = _grid_desc(ndim, grids)
    prim = [a for f in fields for a in f["prim"]]
    bb = [a for f in fields for a in f["b"]]
    k1, pp = _ptrs(prim)
    k2, pb = _ptrs(bb)
    outs = []
    for (l, lo, hi) in grids:
        outs.append([np.zeros(s) for s in interior_shapes(ndim, _gshape(ndim, lo, hi))])
    k3, po = _ptrs([a for o in outs for a in o])
    dts_out = np.zeros(max(ncoarse, 1))
    pin = None
    if dts is not None:
        dts_in = np.ascontiguousarray(dts, dtype=np.float64)
        pin = dts_in.ctypes.data_as(_dp)
    dx0 = [1.0 / N0[a] for a in range(ndim)]
    rc = L.orc_amr_run(C.c_int(ndim), _ivec(N0), C.c_int(nlev), C.c_int(g), C.c_double(gamma), C.c_double(cfl),
                       _dvec(dx0), C.c_int(len(grids)), desc.ctypes.data_as(_ip), pp, pb, C.c_int(ncoarse), pin, po,
                       dts_out.ctypes.data_as(_dp))
    if rc != 0:
        raise RuntimeError("oracle amr_run: " + L.orc_amr_last_error().decode())
    res = [k3[8 * i:8 * i + 8] for i in range(len(grids))]
    return res, dts_out[:ncoarse]


def amr_time(ndim, N0, nlev, g, grids, fields, ncoarse, gamma=5.0 / 3.0, cfl=0.4, threads=None):
    L = lib()
    L.orc_amr_time.restype = C.c_double
    L.orc_amr_last_error.restype = C.c_char_p
    if threads:
        L.orc_set_threads(int(threads))
    desc = _grid_desc(ndim, grids)
    k1, pp = _ptrs([a for f in fields for a in f["prim"]])
    k2, pb = _ptrs([a for f in fields for a in f["b"]])
    dx0 = [1.0 / N0[a] for a in range(ndim)]
    t = L.orc_amr_time(C.c_int(ndim), _ivec(N0), C.c_int(nlev), C.c_int(g), C.c_double(gamma), C.c_double(cfl),
                       _dvec(dx0), C.c_int(len(grids)), desc.ctypes.data_as(_ip), pp, pb, C.c_int(ncoarse))
    if t < 0:
        raise RuntimeError("oracle amr_time: " + L.orc_amr_last_error().decode())
    return t


def amr_fill(ndim, N0, nlev, g, grids, cons, level, full):
    """Fill the band of every grid of `level` from given conserved interiors
    (per grid 8 interior-layout arrays).  Returns per-grid banded arrays."""
    L = lib()
    L.orc_amr_last_error.restype = C.c_char_p
    desc = _grid_desc(ndim, grids)
    k1, pc = _ptrs([a for c in cons for a in c])
    outs = []
    for (l, lo, hi) in grids:
        outs.append([np.zeros(s) for s in banded_shapes(ndim, _gshape(ndim, lo, hi), g)])
    k2, po = _ptrs([a for o in outs for a in o])
    dx0 = [1.0 / N0[a] for a in range(ndim)]
    rc = L.orc_amr_fill(C.c_int(ndim), _ivec(N0), C.c_int(nlev), C.c_int(g), _dvec(dx0), C.c_int(len(grids)),
                        desc.ctypes.data_as(_ip), pc, C.c_int(level), C.c_int(1 if full else 0), po)
    if rc != 0:
        raise RuntimeError("oracle amr_fill: " + L.orc_amr_last_error().decode())
    return [k2[8 * i:8 * i + 8] for i in range(len(grids))]


def amr_run_cons(ndim, N0, nlev, g, grids, cons, ncoarse, gamma=5.0 / 3.0, cfl=0.4, dts=None):
    """amr_run with conserved interiors given directly (per grid 8
    interior-layout arrays)."""
    L = lib()
    L.orc_amr_last_error.restype = C.c_char_p
    desc = _grid_desc(ndim, grids)
    k1, pc = _ptrs([a for c in cons for a in c])
    outs = []
    for (l, lo, hi) in grids:
        outs.append([np.zeros(s) for s in interior_shapes(ndim, _gshape(ndim, lo, hi))])
    k3, po = _ptrs([a for o in outs for a in o])
    dts_out = np.zeros(max(ncoarse, 1))
    pin = None
    if dts is not None:
        dts_in = np.ascontiguousarray(dts, dtype=np.float64)
        pin = dts_in.ctypes.data_as(_dp)
    dx0 = [1.0 / N0[a] for a in range(ndim)]
    rc = L.orc_amr_run_cons(C.c_int(ndim), _ivec(N0), C.c_int(nlev), C.c_int(g), C.c_double(gamma),
                            C.c_double(cfl), _dvec(dx0), C.c_int(len(grids)), desc.ctypes.data_as(_ip), pc,
                            C.c_int(ncoarse), pin, po, dts_out.ctypes.data_as(_dp))
    if rc != 0:
        raise RuntimeError("oracle amr_run_cons: " + L.orc_amr_last_error().decode())
    return [k3[8 * i:8 * i + 8] for i in range(len(grids))], dts_out[:ncoarse]


def amr_overlap(ndim, N0, nlev, g, old_grids, old_cons, new_grids):
    """(O)verlap: conserved interiors of a new iteration of grids from the
    previous iteration (Sec. 2 and 4 of the paper).  Returns per new grid 8
    interior-layout arrays."""
    L = lib()
    L.orc_amr_last_error.restype = C.c_char_p
    d_old = _grid_desc(ndim, old_grids)
    d_new = _grid_desc(ndim, new_grids)
    k1, pc = _ptrs([a for c in old_cons for a in c])
    outs = []
    for (l, lo, hi) in new_grids:
        outs.append([np.zeros(s) for s in interior_shapes(ndim, _gshape(ndim, lo, hi))])
    k2, po = _ptrs([a for o in outs for a in o])
    dx0 = [1.0 / N0[a] for a in range(ndim)]
    rc = L.orc_amr_overlap(C.c_int(ndim), _ivec(N0), C.c_int(nlev), C.c_int(g), _dvec(dx0),
                           C.c_int(len(old_grids)), d_old.ctypes.data_as(_ip), pc, C.c_int(len(new_grids)),
                           d_new.ctypes.data_as(_ip), po)
    if rc != 0:
        raise RuntimeError("oracle amr_overlap: " + L.orc_amr_last_error().decode())
    return [k2[8 * i:8 * i + 8] for i in range(len(new_grids))]


def amr_level_order(nlev):
    """Levels in the order the serial cycle advances them in one coarse step."""
    buf = (C.c_int * 4096)()
    n = lib().orc_amr_level_order(C.c_int(nlev), buf, 4096)
    return list(buf[:n])


# ------------------------------------------------------------ derivatives
def _ke_args(ic, box_lo, box_len):
    ndim, n = ic["ndim"], ic["n"]
    k1, pp = _ptrs(ic["prim"])
    k2, pb = _ptrs(ic["b"])
    lo = (C.c_int * 3)(*(list(box_lo) + [0] * (3 - len(box_lo))))
    ln = (C.c_int * 3)(*(list(box_len) + [1] * (3 - len(box_len))))
    return ndim, n, (k1, k2), pp, pb, lo, ln


def ke_loss(ic, gamma, dts, box_lo, box_len):
    """Kinetic energy of box S after len(dts) frozen-dt steps (band 2 refilled
    every step, periodic)."""
    ndim, n, keep, pp, pb, lo, ln = _ke_args(ic, box_lo, box_len)
    d = np.ascontiguousarray(dts, dtype=np.float64)
    J = C.c_double()
    rc = lib().orc_ke_loss(C.c_int(ndim), _ivec(n), C.c_double(gamma), C.c_int(len(d)), d.ctypes.data_as(_dp), pp,
                           pb, lo, ln, C.byref(J))
    if rc != 0:
        raise RuntimeError("oracle ke_loss failed")
    return J.value


def ke_tlm(ic, gamma, dts, box_lo, box_len, direction):
    """(J, dJ) along direction = [drho, dvx, dvy, dvz] by forward mode."""
    ndim, n, keep, pp, pb, lo, ln = _ke_args(ic, box_lo, box_len)
    d = np.ascontiguousarray(dts, dtype=np.float64)
    k3, pd = _ptrs(direction)
    J, dJ = C.c_double(), C.c_double()
    rc = lib().orc_ke_tlm(C.c_int(ndim), _ivec(n), C.c_double(gamma), C.c_int(len(d)), d.ctypes.data_as(_dp), pp, pb,
                          lo, ln, pd, C.byref(J), C.byref(dJ))
    if rc != 0:
        raise RuntimeError("oracle ke_tlm failed")
    return J.value, dJ.value


def ke_grad(ic, gamma, dts, box_lo, box_len):
    """(J, [dJ/drho, dJ/dvx, dJ/dvy, dJ/dvz]) by reverse mode (tape)."""
    ndim, n, keep, pp, pb, lo, ln = _ke_args(ic, box_lo, box_len)
    d = np.ascontiguousarray(dts, dtype=np.float64)
    outs = [np.zeros_like(np.asarray(ic["prim"][0], dtype=np.float64)) for _ in range(4)]
    k3, po = _ptrs(outs)
    J = C.c_double()
    L = lib()
    L.orc_adj_last_error.restype = C.c_char_p
    rc = L.orc_ke_grad(C.c_int(ndim), _ivec(n), C.c_double(gamma), C.c_int(len(d)), d.ctypes.data_as(_dp), pp, pb, lo,
                       ln, po, C.byref(J))
    if rc != 0:
        raise RuntimeError("oracle ke_grad: " + L.orc_adj_last_error().decode())
    return J.value, k3


def ke_branch_signature(ic, gamma, dts):
    """Hash of every branch decision of the forward run (equal hashes: the
    same branches were taken everywhere)."""
    ndim, n = ic["ndim"], ic["n"]
    k1, pp = _ptrs(ic["prim"])
    k2, pb = _ptrs(ic["b"])
    d = np.ascontiguousarray(dts, dtype=np.float64)
    sig = C.c_uint64()
    rc = lib().orc_ke_branch_signature(C.c_int(ndim), _ivec(n), C.c_double(gamma), C.c_int(len(d)),
                                       d.ctypes.data_as(_dp), pp, pb, C.byref(sig))
    if rc != 0:
        raise RuntimeError("oracle ke_branch_signature failed")
    return sig.value


def step_vjp(ndim, n, gamma, dt, U, lam_out):
    """(dU'/dU)^T lam_out for one band-2 step of the single periodic grid
    (eight interior arrays in, eight out; see orc_step_vjp)."""
    L = lib()
    shapes = interior_shapes(ndim, n)
    ku, pu = _ptrs([np.asarray(u, dtype=np.float64).reshape(sh) for u, sh in zip(U, shapes)])
    kl, pl = _ptrs([np.asarray(x, dtype=np.float64).reshape(sh) for x, sh in zip(lam_out, shapes)])
    out = [np.zeros(sh) for sh in shapes]
    ko, po = _ptrs(out)
    fn = L.orc_step_vjp
    fn.restype = C.c_int
    rc = fn(C.c_int(ndim), _ivec(n), C.c_double(gamma), C.c_double(dt), pu, pl, po)
    if rc != 0:
        raise RuntimeError(_err())
    return ko


def level_vjp(ndim, Nl, g, gamma, dx, dt, boxes, banded, sel, lam_out):
    """(dM/dU)^T lam_out for M one substep of every grid of a level: the
    same-level band copy (prolonged band elements held constant), then a
    band-2 step of each grid (see orc_level_vjp).  boxes: per grid (lo, hi)
    in level cells; banded: per grid 8 arrays in the banded layout (band g);
    sel: grid indices whose output adjoint lam_out (per entry 8
    interior-layout arrays) is given.  Returns per grid 8 interior-layout
    arrays: the adjoint of the input on its own elements."""
    L = lib()
    L.orc_adj_last_error.restype = C.c_char_p
    ng = len(boxes)
    desc = np.zeros((ng, 6), dtype=np.int32)
    for i, (lo, hi) in enumerate(boxes):
        desc[i, :ndim] = lo[:ndim]
        desc[i, 3:3 + ndim] = hi[:ndim]
        desc[i, ndim:3] = 0
        desc[i, 3 + ndim:] = 1
    kb, pb = _ptrs([a for grid in banded for a in grid])
    shapes = [interior_shapes(ndim, tuple(hi[a] - lo[a] for a in range(ndim))) for lo, hi in boxes]
    kl, pl = _ptrs([np.asarray(a, dtype=np.float64).reshape(shapes[sel[t]][s])
                    for t in range(len(sel)) for s, a in enumerate(lam_out[t])])
    outs = [[np.zeros(sh) for sh in shapes[i]] for i in range(ng)]
    ko, po = _ptrs([a for o in outs for a in o])
    sl = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
    rc = L.orc_level_vjp(C.c_int(ndim), _ivec(Nl), C.c_int(g), C.c_double(gamma), _dvec(dx), C.c_double(dt),
                         C.c_int(ng), desc.ctypes.data_as(_ip), pb, C.c_int(len(sel)), sl.ctypes.data_as(_ip), pl,
                         po)
    if rc != 0:
        raise RuntimeError("oracle level_vjp: " + L.orc_adj_last_error().decode())
    return [ko[8 * i:8 * i + 8] for i in range(ng)]
