"""Thin ctypes binding of libamrmhd.so (include/amr.h).

Argument marshalling only: every step of the advance runs in the library's
HIP kernels.  PyTorch supplies device memory (the state pools and the
workspace are torch tensors) and the stream (the current torch stream).
There is no CPU fallback: if the library is missing this module raises.
"""

from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamrmhd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "amr.h")

AMR_OK, AMR_EINVAL, AMR_EHIP, AMR_ENOMEM, AMR_ESTATE, AMR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
AMR_F32, AMR_F64 = 0, 1
AMR_BC_PERIODIC, AMR_BC_OUTFLOW = 0, 1
AMR_FILL_FULL, AMR_FILL_SAME_LEVEL = 0, 1
AMR_EMF_MEAN, AMR_EMF_UPWIND = 0, 1
FIELDS = ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")


class amr_grid(C.Structure):
    _fields_ = [("level", C.c_int32), ("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3)]


class amr_params(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nlevels", C.c_int32), ("ratio", C.c_int32), ("ghost", C.c_int32),
                ("dtype", C.c_int32), ("bc", C.c_int32 * 3), ("domain", C.c_int32 * 3), ("dx0", C.c_double * 3),
                ("gamma", C.c_double), ("cfl", C.c_double), ("emf", C.c_int32), ("pad", C.c_int32)]


class amr_state(C.Structure):
    _fields_ = [("f", C.c_void_p * 8)]


class amr_tune_entry(C.Structure):
    _fields_ = [("tile_policy", C.c_int32), ("zchunk", C.c_int32), ("launch_mode", C.c_int32), ("update_zchunk", C.c_int32),
                ("ms", C.c_double)]


class amr_regrid_params(C.Structure):
    _fields_ = [("theta", C.c_double), ("efficiency", C.c_double), ("buffer", C.c_int32), ("max_box", C.c_int32)]


class AmrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_LIB = None
_VP = C.c_void_p
_PP = C.POINTER(C.c_void_p)


def lib():
    """Load libamrmhd.so (built in-tree by build()); raise if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        L.amr_last_error.restype = C.c_char_p
        L.amr_strerror.restype = C.c_char_p
        L.amr_create.argtypes = [C.POINTER(amr_params), C.POINTER(amr_grid), C.c_int32, C.POINTER(_VP)]
        L.amr_destroy.argtypes = [_VP]
        L.amr_validate.argtypes = [C.POINTER(amr_params), C.POINTER(amr_grid), C.c_int32, C.POINTER(C.c_int64)]
        L.amr_layout.argtypes = [_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.amr_load_primitive.argtypes = [_VP, C.c_int32, _PP, _PP, C.POINTER(amr_state), _VP]
        L.amr_store_interior.argtypes = [_VP, C.c_int32, C.POINTER(amr_state), _PP, _VP]
        L.amr_compute_dt.argtypes = [_VP, C.POINTER(amr_state), C.POINTER(amr_state), C.c_uint32, _VP, _VP]
        L.amr_fill_ghosts_prolong.argtypes = [_VP, C.c_int32, C.c_int32, C.POINTER(amr_state), C.POINTER(amr_state),
                                              _VP]
        L.amr_advance_patches.argtypes = [_VP, C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                                          C.POINTER(amr_state), C.POINTER(amr_state), C.c_uint32, _VP, _VP, _VP]
        L.amr_advance_patches_noalloc.argtypes = [_VP, C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                                                  C.POINTER(amr_state), C.POINTER(amr_state), C.c_uint32, _VP, _VP]
        L.amr_selfcheck_addressing.argtypes = [C.POINTER(amr_params), C.POINTER(amr_grid), C.c_int32, C.c_int32,
                                               C.POINTER(C.c_int64)]
        L.amr_coarse_step.argtypes = [_VP, C.POINTER(amr_state), C.POINTER(amr_state), C.POINTER(C.c_uint32), _VP,
                                      _VP, C.c_int32, _VP]
        L.amr_restrict_fluxfix.argtypes = [_VP, C.c_int32, C.POINTER(amr_state), C.POINTER(amr_state), _VP, _VP]
        L.amr_advance_adjoint.argtypes = [_VP, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(amr_state),
                                          C.POINTER(amr_state), _VP, _VP]
        L.amr_adjoint_workspace.argtypes = [_VP, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]
        L.amr_store_interior_adjoint.argtypes = [_VP, C.c_int32, _PP, C.POINTER(amr_state), _VP]
        L.amr_load_primitive_adjoint.argtypes = [_VP, C.c_int32, _PP, C.POINTER(amr_state), _PP, _VP]
        L.amr_frozen_workspace.argtypes = [_VP, C.POINTER(C.c_int64)]
        L.amr_advance_frozen.argtypes = [_VP, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(amr_state),
                                         C.POINTER(amr_state), _VP, _VP]
        L.amr_set_launch_config.argtypes = [_VP, C.c_int32, C.c_int32, C.c_int32]
        L.amr_get_launch_config.argtypes = [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.amr_set_update_zchunk.argtypes = [_VP, C.c_int32]
        L.amr_get_update_zchunk.argtypes = [_VP, C.POINTER(C.c_int32)]
        L.amr_autotune.argtypes = [_VP, C.POINTER(amr_state), C.POINTER(amr_state), C.c_uint32, _VP, _VP, C.c_int32,
                                   C.POINTER(amr_tune_entry), C.POINTER(C.c_int32), _VP]
        L.amr_get_error_flags.argtypes = [_VP, C.POINTER(C.c_uint32), C.POINTER(C.c_int64)]
        L.amr_graph_capture.argtypes = [_VP, C.POINTER(amr_state), C.POINTER(amr_state), C.c_uint32, _VP, _VP,
                                        C.c_int32, _VP]
        L.amr_graph_launch.argtypes = [_VP, C.POINTER(C.c_uint32), _VP]
        L.amr_set_kernel_timing.argtypes = [_VP, C.c_int32]
        L.amr_kernel_times.argtypes = [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.amr_cluster_boxes.argtypes = [C.c_int32, C.POINTER(C.c_int32), _VP, _VP, C.c_double, C.c_int32,
                                        C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]
        L.amr_plan_schedule.argtypes = [C.POINTER(amr_params), C.POINTER(amr_grid), C.c_int32, C.c_int32,
                                        C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.amr_set_schedule.argtypes = [_VP, C.c_int32]
        L.amr_get_schedule.argtypes = [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.amr_level_cells.argtypes = [_VP, C.c_int32, C.POINTER(C.c_int64)]
        L.amr_flag_cells.argtypes = [_VP, C.c_int32, C.POINTER(amr_state), C.POINTER(amr_state), C.c_double, _VP,
                                     _VP]
        L.amr_regrid.argtypes = [_VP, C.c_int32, C.POINTER(amr_state), C.POINTER(amr_state),
                                 C.POINTER(amr_regrid_params), C.POINTER(amr_grid), C.c_int32,
                                 C.POINTER(C.c_int32), _VP]
        L.amr_overlap.argtypes = [_VP, C.c_int32, C.POINTER(amr_state), C.POINTER(amr_state), _VP,
                                  C.POINTER(amr_state), _VP]
        _LIB = L
    return _LIB


def header_functions():
    """Names of the functions include/amr.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amr_[a-z_0-9]+)\s*\(", text)))


def _check(rc, what):
    if rc != AMR_OK:
        raise AmrError(rc, f"{what}: {lib().amr_last_error().decode()}")


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


# --------------------------------------------------------------- C names
def amr_create(params, grids):
    arr = (amr_grid * len(grids))(*grids)
    h = C.c_void_p()
    _check(lib().amr_create(C.byref(params), arr, len(grids), C.byref(h)), "amr_create")
    return h


def amr_validate(params, grids):
    """Host-only validation and table build; returns the stats dict."""
    arr = (amr_grid * len(grids))(*grids)
    st = (C.c_int64 * 8)()
    _check(lib().amr_validate(C.byref(params), arr, len(grids), st), "amr_validate")
    keys = ("grids", "state_elems", "workspace_bytes", "copy_entries", "prolong_entries", "sync_entries",
            "flux_items", "update_items")
    return dict(zip(keys, list(st)))


def amr_selfcheck_addressing(params, grids, elem_bytes):
    """Host-only check of the advance kernels' addressing for element size
    elem_bytes (4, 8 or 16); returns (loads, stores, reads) checked."""
    arr = (amr_grid * len(grids))(*grids)
    st = (C.c_int64 * 3)()
    _check(lib().amr_selfcheck_addressing(C.byref(params), arr, len(grids), int(elem_bytes), st),
           "amr_selfcheck_addressing")
    return tuple(st)


def make_params(ndim, domain, nlevels=1, ratio=2, ghost=2, dtype="f64", bc=(0, 0, 0), dx0=None, gamma=5.0 / 3.0,
                cfl=0.4, emf=AMR_EMF_MEAN):
    domain = tuple(domain) + (1,) * (3 - len(domain))
    p = amr_params()
    p.ndim, p.nlevels, p.ratio, p.ghost = ndim, nlevels, ratio, ghost
    p.dtype = AMR_F64 if dtype == "f64" else AMR_F32
    for d in range(3):
        p.bc[d] = bc[d] if d < len(bc) else 0
        p.domain[d] = domain[d]
        p.dx0[d] = (dx0[d] if dx0 is not None else 1.0 / domain[d]) if d < ndim else 1.0
    p.gamma, p.cfl = gamma, cfl
    p.emf = emf
    return p


def make_grids(grids):
    out = []
    for lev, lo, hi in grids:
        lo = tuple(lo) + (0,) * (3 - len(lo))
        hi = tuple(hi) + (1,) * (3 - len(hi))
        out.append(amr_grid(lev, (C.c_int32 * 3)(*lo), (C.c_int32 * 3)(*hi)))
    return out


def amr_destroy(h):
    _check(lib().amr_destroy(h), "amr_destroy")


def amr_layout(h, ngrids):
    se = C.c_int64()
    wb = C.c_int64()
    offs = (C.c_int64 * ngrids)()
    _check(lib().amr_layout(h, C.byref(se), C.byref(wb), offs), "amr_layout")
    return se.value, wb.value, list(offs)


def amr_load_primitive(h, grid, prim, b, U):
    pp = (C.c_void_p * 5)(*[t.data_ptr() for t in prim])
    bb = (C.c_void_p * 3)(*[t.data_ptr() for t in b])
    _check(lib().amr_load_primitive(h, grid, pp, bb, C.byref(U), _stream()), "amr_load_primitive")


def amr_store_interior(h, grid, U, outs):
    oo = (C.c_void_p * 8)(*[t.data_ptr() for t in outs])
    _check(lib().amr_store_interior(h, grid, C.byref(U), oo, _stream()), "amr_store_interior")


def amr_compute_dt(h, Ua, Ub, parity, dt0):
    _check(lib().amr_compute_dt(h, C.byref(Ua), C.byref(Ub), parity, _ptr(dt0), _stream()), "amr_compute_dt")


def amr_fill_ghosts_prolong(h, level, mode, U_level, U_parent=None):
    up = C.byref(U_parent) if U_parent is not None else None
    _check(lib().amr_fill_ghosts_prolong(h, level, mode, C.byref(U_level), up, _stream()), "amr_fill_ghosts_prolong")


def amr_advance_patches(h, cycle, subset, band, Ua, Ub, parity, dt0, ws):
    if subset:
        arr = (C.c_int32 * len(subset))(*subset)
        n = len(subset)
    else:
        arr, n = None, 0
    _check(lib().amr_advance_patches(h, cycle, arr, n, band, C.byref(Ua), C.byref(Ub), parity, _ptr(dt0), _ptr(ws),
                                     _stream()), "amr_advance_patches")


def amr_advance_patches_noalloc(h, cycle, subset, band, Ua, Ub, parity, dt0):
    if subset:
        arr = (C.c_int32 * len(subset))(*subset)
        n = len(subset)
    else:
        arr, n = None, 0
    _check(lib().amr_advance_patches_noalloc(h, cycle, arr, n, band, C.byref(Ua), C.byref(Ub), parity, _ptr(dt0),
                                             _stream()), "amr_advance_patches_noalloc")


def amr_coarse_step(h, Ua, Ub, parity, dt0, ws, mode=0):
    """One coarse step; returns the updated parity word."""
    par = C.c_uint32(parity)
    _check(lib().amr_coarse_step(h, C.byref(Ua), C.byref(Ub), C.byref(par), _ptr(dt0), _ptr(ws), mode, _stream()),
           "amr_coarse_step")
    return par.value


def amr_restrict_fluxfix(h, fine_level, Ufine, Ucoarse, ws):
    _check(lib().amr_restrict_fluxfix(h, fine_level, C.byref(Ufine), C.byref(Ucoarse), _ptr(ws), _stream()),
           "amr_restrict_fluxfix")


def amr_advance_adjoint(h, grid_or_level, dts, Uck, lam, ws):
    d = (C.c_double * len(dts))(*[float(x) for x in dts])
    _check(lib().amr_advance_adjoint(h, grid_or_level, len(dts), d, C.byref(Uck), C.byref(lam), _ptr(ws),
                                     _stream()), "amr_advance_adjoint")


def amr_adjoint_workspace(h, grid_or_level, nsteps):
    b = C.c_int64()
    _check(lib().amr_adjoint_workspace(h, grid_or_level, nsteps, C.byref(b)), "amr_adjoint_workspace")
    return b.value


def amr_store_interior_adjoint(h, grid, g, lam):
    gg = (C.c_void_p * 8)(*[t.data_ptr() for t in g])
    _check(lib().amr_store_interior_adjoint(h, grid, gg, C.byref(lam), _stream()), "amr_store_interior_adjoint")


def amr_load_primitive_adjoint(h, grid, prim, lam, grad):
    pp = (C.c_void_p * 4)(*[t.data_ptr() for t in prim[:4]])
    gg = (C.c_void_p * 4)(*[t.data_ptr() for t in grad])
    _check(lib().amr_load_primitive_adjoint(h, grid, pp, C.byref(lam), gg, _stream()), "amr_load_primitive_adjoint")


def amr_frozen_workspace(h):
    b = C.c_int64()
    _check(lib().amr_frozen_workspace(h, C.byref(b)), "amr_frozen_workspace")
    return b.value


def amr_advance_frozen(h, level, dts, Ubase, Upert, ws):
    d = (C.c_double * len(dts))(*[float(x) for x in dts])
    _check(lib().amr_advance_frozen(h, level, len(dts), d, C.byref(Ubase), C.byref(Upert), _ptr(ws), _stream()),
           "amr_advance_frozen")


def amr_set_launch_config(h, tile_policy, zchunk, launch_mode):
    """launch_mode bit 0: persistent queue; bit 1: one item chunk per XCD;
    bit 2: persistent flux kernel only."""
    _check(lib().amr_set_launch_config(h, tile_policy, zchunk, int(launch_mode)), "amr_set_launch_config")


def amr_get_launch_config(h):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().amr_get_launch_config(h, C.byref(a), C.byref(b), C.byref(c)), "amr_get_launch_config")
    return a.value, b.value, c.value


def amr_set_update_zchunk(h, zchunk):
    _check(lib().amr_set_update_zchunk(h, int(zchunk)), "amr_set_update_zchunk")


def amr_get_update_zchunk(h):
    a = C.c_int32()
    _check(lib().amr_get_update_zchunk(h, C.byref(a)), "amr_get_update_zchunk")
    return a.value


TUNE_CANDIDATES = 107


def amr_autotune(h, Ua, Ub, parity, dt0, ws, reps=3):
    """Returns (chosen index, [(tile_policy, zchunk, launch_mode, ms, update_zchunk), ...])."""
    res = (amr_tune_entry * TUNE_CANDIDATES)()
    ch = C.c_int32()
    _check(lib().amr_autotune(h, C.byref(Ua), C.byref(Ub), parity, _ptr(dt0), _ptr(ws), reps, res, C.byref(ch),
                              _stream()), "amr_autotune")
    return ch.value, [(r.tile_policy, r.zchunk, r.launch_mode, r.ms, r.update_zchunk) for r in res]


def amr_get_error_flags(h):
    fl = C.c_uint32()
    bad = C.c_int64()
    rc = lib().amr_get_error_flags(h, C.byref(fl), C.byref(bad))
    if rc not in (AMR_OK, AMR_ESTATE):
        _check(rc, "amr_get_error_flags")
    return fl.value, bad.value


def amr_graph_capture(h, Ua, Ub, parity, dt0, ws, mode=0):
    _check(lib().amr_graph_capture(h, C.byref(Ua), C.byref(Ub), parity, _ptr(dt0), _ptr(ws), mode, _stream()),
           "amr_graph_capture")


def amr_graph_launch(h, parity):
    par = C.c_uint32(parity)
    _check(lib().amr_graph_launch(h, C.byref(par), _stream()), "amr_graph_launch")
    return par.value


def amr_set_kernel_timing(h, enable):
    _check(lib().amr_set_kernel_timing(h, int(bool(enable))), "amr_set_kernel_timing")


def amr_kernel_times(h):
    a, b, n = C.c_double(), C.c_double(), C.c_int64()
    _check(lib().amr_kernel_times(h, C.byref(a), C.byref(b), C.byref(n)), "amr_kernel_times")
    return a.value, b.value, n.value


def amr_cluster_boxes(mask, admissible=None, efficiency=0.7, max_box=16):
    """Host clustering of a numpy bool mask indexed [x, y(, z)]; returns
    [(lo, hi)] tuples of ndim entries in emission order."""
    nd = mask.ndim
    ext = (C.c_int32 * 3)(*(list(mask.shape) + [1] * (3 - nd)))
    m = np.ascontiguousarray(np.transpose(mask).astype(np.uint8))  # x fastest
    a = None if admissible is None else np.ascontiguousarray(np.transpose(admissible).astype(np.uint8))
    n = C.c_int32(0)
    cap = 4096
    while True:
        out = (C.c_int32 * (6 * cap))()
        rc = lib().amr_cluster_boxes(nd, ext, m.ctypes.data_as(C.c_void_p),
                                     None if a is None else a.ctypes.data_as(C.c_void_p), float(efficiency),
                                     int(max_box), out, cap, C.byref(n))
        if rc == AMR_EINVAL and n.value > cap:
            cap = n.value
            continue
        _check(rc, "amr_cluster_boxes")
        return [(tuple(out[6 * q:6 * q + nd]), tuple(out[6 * q + 3:6 * q + 3 + nd])) for q in range(n.value)]


def amr_plan_schedule(params, grids, schedule):
    """Host-only plan: (predicted work per cycle, per grid the cycle of each
    of its steps)."""
    recs = make_grids(grids)
    arr = (amr_grid * len(recs))(*recs)
    ncyc = params.ratio ** (params.nlevels - 1)
    work = (C.c_double * ncyc)()
    nsteps = [params.ratio ** g.level for g in recs]
    sc = (C.c_int32 * sum(nsteps))()
    _check(lib().amr_plan_schedule(C.byref(params), arr, len(recs), schedule, work, sc), "amr_plan_schedule")
    out, q = [], 0
    for n in nsteps:
        out.append(list(sc[q:q + n]))
        q += n
    return list(work), out


def amr_set_schedule(h, schedule):
    _check(lib().amr_set_schedule(h, schedule), "amr_set_schedule")


def amr_get_schedule(h, ncycles):
    s = C.c_int32()
    work = (C.c_double * ncycles)()
    _check(lib().amr_get_schedule(h, C.byref(s), work), "amr_get_schedule")
    return s.value, list(work)


def amr_level_cells(h, level):
    n = C.c_int64()
    _check(lib().amr_level_cells(h, level, C.byref(n)), "amr_level_cells")
    return n.value


def amr_flag_cells(h, level, U_level, U_parent, theta, flags):
    up = C.byref(U_parent) if U_parent is not None else None
    _check(lib().amr_flag_cells(h, level, C.byref(U_level), up, float(theta), _ptr(flags), _stream()),
           "amr_flag_cells")


def amr_regrid(h, level, U_level, U_parent, theta, efficiency=0.7, buffer=1, max_box=16):
    """New grid list [(level, lo3, hi3)] with level+1 re-clustered."""
    rp = amr_regrid_params(float(theta), float(efficiency), int(buffer), int(max_box))
    up = C.byref(U_parent) if U_parent is not None else None
    n = C.c_int32(0)
    cap = 1024
    while True:
        arr = (amr_grid * cap)()
        rc = lib().amr_regrid(h, level, C.byref(U_level), up, C.byref(rp), arr, cap, C.byref(n), _stream())
        if rc == AMR_EINVAL and n.value > cap:
            cap = n.value
            continue
        _check(rc, "amr_regrid")
        return [(g.level, tuple(g.lo), tuple(g.hi)) for g in arr[:n.value]]


def amr_overlap(h_new, level, U_new, U_new_parent, h_old, U_old):
    up = C.byref(U_new_parent) if U_new_parent is not None else None
    _check(lib().amr_overlap(h_new, level, C.byref(U_new), up, h_old, C.byref(U_old), _stream()), "amr_overlap")


# ----------------------------------------------------------- convenience
class State:
    """Eight device pools (torch tensors) of one hierarchy state."""

    def __init__(self, fields):
        self.fields = fields
        self.c = amr_state()
        for i, t in enumerate(fields):
            self.c.f[i] = t.data_ptr()

    def copy_(self, other):
        for a, b in zip(self.fields, other.fields):
            a.copy_(b)
        return self


class Hierarchy:
    """A grid hierarchy handle plus the torch-owned memory sized for it."""

    def __init__(self, ndim, domain, grids, nlevels=1, ratio=2, ghost=2, dtype="f64", bc=(0, 0, 0), dx0=None,
                 gamma=5.0 / 3.0, cfl=0.4, device="cuda", emf=AMR_EMF_MEAN):
        import torch
        self.torch = torch
        self.ndim = ndim
        self.domain = tuple(domain) + (1,) * (3 - len(domain))
        self.nlevels = nlevels
        self.ratio = ratio
        self.ghost = ghost
        self.gamma = gamma
        self.dtype = torch.float64 if dtype == "f64" else torch.float32
        p = make_params(ndim, domain, nlevels, ratio, ghost, dtype, bc, dx0, gamma, cfl, emf)
        self.params = p
        self.grid_records = make_grids(grids)
        self.grids = [(g.level, tuple(g.lo), tuple(g.hi)) for g in self.grid_records]
        self.h = amr_create(p, self.grid_records)
        self.state_elems, self.workspace_bytes, self.offsets = amr_layout(self.h, len(grids))
        self.device = device
        self.ws = torch.zeros(max(self.workspace_bytes, 256), dtype=torch.uint8, device=device)
        self.dt0 = torch.zeros(1, dtype=torch.float64, device=device)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                amr_destroy(h)
            except Exception:
                pass
            self.h = None

    def new_state(self):
        t = self.torch
        return State([t.zeros(self.state_elems, dtype=self.dtype, device=self.device) for _ in range(8)])

    def grid_shape(self, gi):
        _, lo, hi = self.grids[gi]
        n = [hi[d] - lo[d] for d in range(3)]
        return n

    def interior_shapes(self, gi):
        nx, ny, nz = self.grid_shape(gi)
        cell = (nz, ny, nx)
        bz = (nz + 1, ny, nx) if self.ndim == 3 else cell
        return [cell] * 5 + [(nz, ny, nx + 1), (nz, ny + 1, nx), bz]

    def load_primitive(self, U, gi, prim, b):
        t = self.torch
        pd = [t.as_tensor(np.ascontiguousarray(a), dtype=t.float64, device=self.device) for a in prim]
        bd = [t.as_tensor(np.ascontiguousarray(a), dtype=t.float64, device=self.device) for a in b]
        amr_load_primitive(self.h, gi, pd, bd, U.c)
        t.cuda.synchronize()

    def store_interior(self, U, gi):
        t = self.torch
        outs = [t.zeros(s, dtype=t.float64, device=self.device) for s in self.interior_shapes(gi)]
        amr_store_interior(self.h, gi, U.c, outs)
        t.cuda.synchronize()
        return [o.cpu().numpy() for o in outs]

    def compute_dt(self, U, V=None, parity=0):
        amr_compute_dt(self.h, U.c, (V or U).c, parity, self.dt0)

    def fill(self, level, mode, U, Up=None):
        amr_fill_ghosts_prolong(self.h, level, mode, U.c, Up.c if Up is not None else None)

    def advance(self, Uin, Uout, cycle=0, band=0, subset=None, parity=0):
        """Single-level style: parity 0 reads Uin and writes Uout."""
        amr_advance_patches(self.h, -1 if subset else cycle, subset, band, Uin.c, Uout.c, parity, self.dt0, self.ws)

    def coarse_step(self, Ua, Ub, parity, mode=0):
        return amr_coarse_step(self.h, Ua.c, Ub.c, parity, self.dt0, self.ws, mode)

    def graph_capture(self, Ua, Ub, parity, mode=0):
        amr_graph_capture(self.h, Ua.c, Ub.c, parity, self.dt0, self.ws, mode)

    def graph_launch(self, parity):
        return amr_graph_launch(self.h, parity)

    def autotune(self, Ua, Ub, parity, reps=3):
        return amr_autotune(self.h, Ua.c, Ub.c, parity, self.dt0, self.ws, reps)

    def set_launch_config(self, tile_policy, zchunk, launch_mode, update_zchunk=None):
        amr_set_launch_config(self.h, tile_policy, zchunk, launch_mode)
        if update_zchunk is not None:
            amr_set_update_zchunk(self.h, update_zchunk)

    def current(self, Ua, Ub, parity, level):
        return Ub if (parity >> level) & 1 else Ua

    def set_schedule(self, schedule):
        amr_set_schedule(self.h, schedule)

    def flags(self, level, U, Up, theta):
        """Refinement flags of `level` (uint8 tensor in the flag layout)."""
        t = self.torch
        f = t.zeros(max(amr_level_cells(self.h, level), 1), dtype=t.uint8, device=self.device)
        amr_flag_cells(self.h, level, U.c, Up.c if Up is not None else None, theta, f)
        return f

    def regrid(self, level, U, Up, theta, efficiency=0.7, buffer=1, max_box=16):
        """Grid list of the next iteration with level+1 re-clustered (lo/hi
        trimmed to ndim entries)."""
        g = amr_regrid(self.h, level, U.c, Up.c if Up is not None else None, theta, efficiency, buffer, max_box)
        return [(l, tuple(lo[:self.ndim]), tuple(hi[:self.ndim])) for (l, lo, hi) in g]

    def overlap_from(self, old, old_states):
        """(O)verlap of every level, coarse to fine, from hierarchy `old`
        (old_states[l]: the State holding level l's current data) into a new
        State of this hierarchy, which is returned."""
        U = self.new_state()
        for l in range(self.nlevels):
            amr_overlap(self.h, l, U.c, U.c if l > 0 else None, old.h, old_states[l].c)
        return U

    def error_flags(self):
        return amr_get_error_flags(self.h)
