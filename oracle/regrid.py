"""Regridding of one level (test infrastructure only): refinement flags, flag
buffer, proper-nesting mask and Berger-Rigoutsos clustering.

The paper's mesh is adaptive: each level has successive iterations of grids,
and the fluid variables move from the previous iteration to the current one
(Sec. 2; the (O)verlap of the level cycle, Sec. 4).  It gives no refinement
criterion and no clustering rule; the readings taken here are:

* flag: level-l cell c is flagged when, along some active axis d,
  |rho(c + e_d) - rho(c - e_d)| > theta * (rho(c + e_d) + rho(c - e_d)),
  neighbours read after a fill of level l (copy + prolongation above level 0);
* buffer: the flags grow by `nbuf` cells in every direction (periodic), then
  are limited to the nestable region;
* nesting: a new level-(l+1) box B (in level-l cells) is admissible when B
  grown by buf = g/R + 1 cells lies in the union of level-l interiors
  (periodic images included), the rule hierarchy validation checks; the
  grids of level l+2 are kept, so the cells of each of them grown by buf
  level-(l+1) cells, coarsened to level l, are added to the flags;
* clustering (Berger & Rigoutsos 1991): shrink the box to its flags; accept
  it when flags >= eff * volume, every extent <= maxbox and it is admissible
  (a one-cell box is always accepted); otherwise cut it, in this order of
  preference: at a hole of the signature (zero flag count across the box),
  axes by decreasing extent (ties: lower axis), the hole nearest the middle
  (ties: the lower); else at the strongest sign change of the signature's
  second difference (largest jump; ties: nearer the middle, longer axis,
  lower axis), cutting between the two cells where it changes; else halve
  the longest axis (ties: lower axis; low half floor(n/2) cells).  Boxes are
  emitted depth first, low part before high part.

Everything here works on dense boolean masks over the level's whole index
space, indexed [x, y(, z)].
"""

from __future__ import annotations

import numpy as np

from . import oracle as O


def level_extent(ndim, N0, level, R=2):
    return tuple(int(N0[a]) * R ** level for a in range(ndim))


def _roll_all(mask, r, op):
    """Grow (op = np.logical_or) or erode (np.logical_and) a periodic mask by
    the cube [-r, r]^ndim, one axis at a time."""
    out = mask.copy()
    for a in range(mask.ndim):
        acc = out.copy()
        for s in range(1, r + 1):
            acc = op(acc, np.roll(out, s, axis=a))
            acc = op(acc, np.roll(out, -s, axis=a))
        out = acc
    return out


def flags(ndim, N0, nlev, g, grids, cons, level, theta):
    """Flag mask of level `level` (shape level_extent, indexed [x, y(, z)])."""
    banded = O.amr_fill(ndim, N0, nlev, g, grids, cons, level, full=level > 0)
    ext = level_extent(ndim, N0, level)
    mask = np.zeros(ext, dtype=bool)
    gz = g if ndim == 3 else 0
    for gi, (l, lo, hi) in enumerate(grids):
        if l != level:
            continue
        rho = banded[gi][0]  # (nz + 2gz, ny + 2g, nx + 2g)
        n = [hi[a] - lo[a] for a in range(ndim)]
        nz = n[2] if ndim == 3 else 1
        core = (slice(gz, gz + nz), slice(g, g + n[1]), slice(g, g + n[0]))
        f = np.zeros((nz, n[1], n[0]), dtype=bool)
        for d in range(ndim):
            ax = 2 - d  # array axis of spatial axis d
            up = list(core)
            dn = list(core)
            up[ax] = slice(core[ax].start + 1, core[ax].stop + 1)
            dn[ax] = slice(core[ax].start - 1, core[ax].stop - 1)
            rp, rm = rho[tuple(up)], rho[tuple(dn)]
            f |= np.abs(rp - rm) > theta * (rp + rm)
        fx = np.transpose(f, (2, 1, 0))  # [x, y, z]
        if ndim == 2:
            fx = fx[:, :, 0]
        sl = tuple(slice(lo[a], hi[a]) for a in range(ndim))
        mask[sl] = fx
    return mask


def nestable(ndim, N0, g, grids, level, R=2):
    """Cells c of level `level` whose cube c + [-buf, buf]^ndim lies in the
    union of the level's interiors (periodic), buf = g / R + 1."""
    ext = level_extent(ndim, N0, level)
    cov = np.zeros(ext, dtype=bool)
    for (l, lo, hi) in grids:
        if l == level:
            cov[tuple(slice(lo[a], hi[a]) for a in range(ndim))] = True
    return _roll_all(cov, g // R + 1, np.logical_and)


def forced(ndim, N0, g, grids, level, R=2):
    """Level-`level` cells under each level-(level+2) grid grown by buf
    level-(level+1) cells (periodic)."""
    ext = level_extent(ndim, N0, level)
    out = np.zeros(ext, dtype=bool)
    buf = g // R + 1
    for (l, lo, hi) in grids:
        if l != level + 2:
            continue
        idx = []
        for a in range(ndim):
            a0 = lo[a] // R - buf  # level l+1 cells
            a1 = hi[a] // R + buf
            c0 = a0 // R  # floor
            c1 = -((-a1) // R)  # ceil
            idx.append(np.arange(c0, c1) % ext[a])
        out[np.ix_(*idx)] = True
    return out


def _signatures(sub):
    nd = sub.ndim
    return [sub.sum(axis=tuple(b for b in range(nd) if b != a)).astype(np.int64) for a in range(nd)]


def _choose_cut(sub, lo, ext):
    nd = sub.ndim
    sig = _signatures(sub)
    by_len = sorted(range(nd), key=lambda a: (-ext[a], a))
    # 1. holes
    for a in by_len:
        zeros = [i for i in range(ext[a]) if sig[a][i] == 0]
        if zeros:
            mid = ext[a] / 2.0
            i = min(zeros, key=lambda i: (abs(i + 0.5 - mid), i))
            return a, lo[a] + i
    # 2. inflection: sign change of the second difference
    best, best_key = None, None
    for a in range(nd):
        n = ext[a]
        if n < 4:
            continue
        s = sig[a]
        lap = {i: int(s[i - 1] - 2 * s[i] + s[i + 1]) for i in range(1, n - 1)}
        mid = n / 2.0
        for i in range(2, n - 1):
            x, y = lap[i - 1], lap[i]
            if (x < 0 < y) or (y < 0 < x):
                key = (abs(y - x), -abs(i - mid), n, -a)
                if best_key is None or key > best_key:
                    best_key, best = key, (a, lo[a] + i)
    if best is not None:
        return best
    # 3. halve the longest axis
    a = by_len[0]
    return a, lo[a] + ext[a] // 2


def cluster(mask, admissible, eff=0.7, maxbox=16):
    """Berger-Rigoutsos boxes [(lo, hi)] covering the True cells of `mask`;
    `admissible` is the nestable mask."""
    nd = mask.ndim
    out = []
    stack = [(tuple(0 for _ in range(nd)), tuple(mask.shape))]
    while stack:
        lo, hi = stack.pop()
        sub = mask[tuple(slice(lo[a], hi[a]) for a in range(nd))]
        if not sub.any():
            continue
        sig = _signatures(sub)
        nlo, nhi = [], []
        for a in range(nd):
            nzr = np.nonzero(sig[a])[0]
            nlo.append(lo[a] + int(nzr[0]))
            nhi.append(lo[a] + int(nzr[-1]) + 1)
        lo, hi = tuple(nlo), tuple(nhi)
        sl = tuple(slice(lo[a], hi[a]) for a in range(nd))
        sub = mask[sl]
        ext = [hi[a] - lo[a] for a in range(nd)]
        vol = int(np.prod(ext))
        count = int(sub.sum())
        if vol == 1 or (float(count) >= eff * float(vol) and max(ext) <= maxbox and bool(admissible[sl].all())):
            out.append((lo, hi))
            continue
        a, c = _choose_cut(sub, lo, ext)
        hi_low = list(hi)
        hi_low[a] = c
        lo_high = list(lo)
        lo_high[a] = c
        stack.append((tuple(lo_high), hi))   # popped second
        stack.append((lo, tuple(hi_low)))    # popped first
    return out


def regrid_level(ndim, N0, nlev, g, grids, cons, level, theta, nbuf=1, eff=0.7, maxbox=16, R=2):
    """New grid list with level+1 re-clustered from the flags of `level`:
    levels <= level and >= level + 2 keep their grids (and order); the new
    level-(level+1) boxes follow the former."""
    if not 0 <= level <= nlev - 2:
        raise ValueError("level must be in [0, nlev - 2]")
    f = flags(ndim, N0, nlev, g, grids, cons, level, theta)
    adm = nestable(ndim, N0, g, grids, level, R)
    f = _roll_all(f, nbuf, np.logical_or) & adm
    frc = forced(ndim, N0, g, grids, level, R)
    if np.any(frc & ~adm):
        raise ValueError("a level-(l+2) grid is not nestable in level l")
    f |= frc
    boxes = cluster(f, adm, eff, maxbox)
    keep_lo = [gr for gr in grids if gr[0] <= level]
    keep_hi = [gr for gr in grids if gr[0] >= level + 2]
    new = [(level + 1, tuple(R * x for x in lo), tuple(R * x for x in hi)) for (lo, hi) in boxes]
    return keep_lo + new + keep_hi, f
