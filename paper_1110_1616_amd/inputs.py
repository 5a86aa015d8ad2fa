"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only draws random numbers and samples analytic fields; it holds
none of the scheme's arithmetic (no conserved variables, no fluxes, no
averaging of data between levels).  Every field is produced in float64 in the
"interior layout":

* cells  : shape (nz, ny, nx), x fastest
* Bx face: (nz, ny, nx+1), By face: (nz, ny+1, nx), Bz face: (nz+1, ny, nx)
* in 2D nz = 1 and Bz is a cell array (1, ny, nx)

Recipe for the smooth random fields (the paper's workloads are unspecified
magnetised flows; these stand in for them):

* mode sum f(x) = sum_{m<8} cos(2 pi k_m . x + phi_m), k_m integer in
  [-4, 4]^ndim (k != 0), phi_m uniform in [0, 2 pi);
* rho = 1 + 0.1 f (optionally times 4 on 0.25 <= x < 0.75), p = 1;
* v = curl Psi (analytic, independent modes, random 3-vector amplitudes),
  rescaled to a target rms |v|;
* B = discrete curl of a vector potential A (independent modes, random unit
  3-vector amplitudes) sampled at edge centres, so the face field is
  divergence-free up to rounding; rescaled to a target rms of the
  face-averaged field.  A is sampled at wrapped positions so that the face at
  index n equals the face at index 0 bit for bit on periodic domains.
"""

from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def _modes(rng, ndim, nmodes=8, kmax=4):
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=ndim)
        if np.any(k != 0):
            ks.append(k)
    k3 = np.zeros((nmodes, 3))
    k3[:, :ndim] = np.array(ks, dtype=np.float64)
    phi = rng.uniform(0.0, TWO_PI, size=nmodes)
    return k3, phi


def _unit3(rng, n):
    a = rng.normal(size=(n, 3))
    return a / np.linalg.norm(a, axis=1, keepdims=True)


def _grid(xs, ys, zs):
    z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")
    return x, y, z


def _phase(k3, phi, x, y, z):
    return TWO_PI * (k3[0] * x + k3[1] * y + k3[2] * z) + phi


class _Field:
    """Random smooth fields on the unit periodic box."""

    def __init__(self, rng, ndim):
        self.ndim = ndim
        self.k_rho, self.phi_rho = _modes(rng, ndim)
        self.k_psi, self.phi_psi = _modes(rng, ndim)
        self.a_psi = _unit3(rng, 8)
        self.k_a, self.phi_a = _modes(rng, ndim)
        self.a_a = _unit3(rng, 8)

    def f_rho(self, x, y, z):
        out = np.zeros_like(x)
        for m in range(8):
            out += np.cos(_phase(self.k_rho[m], self.phi_rho[m], x, y, z))
        return out

    def curl_psi(self, x, y, z):
        """Analytic curl of Psi = sum_m a_m cos(theta_m): -sum_m sin(theta_m) 2 pi (k_m x a_m)."""
        v = [np.zeros_like(x) for _ in range(3)]
        for m in range(8):
            s = np.sin(_phase(self.k_psi[m], self.phi_psi[m], x, y, z))
            c = np.cross(TWO_PI * self.k_psi[m], self.a_psi[m])
            for a in range(3):
                v[a] -= s * c[a]
        return v

    def pot(self, comp, x, y, z):
        out = np.zeros_like(x)
        for m in range(8):
            out += self.a_a[m, comp] * np.cos(_phase(self.k_a[m], self.phi_a[m], x, y, z))
        return out


def _wrap_pos(n, count, offset, lo=0, h=None):
    """Positions (index + offset) * h of `count` consecutive indices starting
    at lo, with the index wrapped into [0, n) so periodic images coincide."""
    h = 1.0 / n if h is None else h
    idx = (np.arange(lo, lo + count) % n).astype(np.float64)
    return (idx + offset) * h


def curl_faces(ndim, n, pot):
    """Face B from the discrete curl of A sampled at edge centres.

    pot(comp, x, y, z) evaluates component comp of A.  Returns (bx, by, bz) in
    the interior layout.  This is input construction (a discrete curl of a
    sampled potential), not part of the scheme."""
    nx, ny = n[0], n[1]
    dx, dy = 1.0 / nx, 1.0 / ny
    if ndim == 2:
        # A_z at nodes, A_x at y-faces, A_y at x-faces.
        x, y, z = _grid(_wrap_pos(nx, nx + 1, 0.0), _wrap_pos(ny, ny + 1, 0.0), np.zeros(1))
        az = pot(2, x, y, z)[0]
        x, y, z = _grid(_wrap_pos(nx, nx, 0.5), _wrap_pos(ny, ny + 1, 0.0), np.zeros(1))
        ax = pot(0, x, y, z)[0]
        x, y, z = _grid(_wrap_pos(nx, nx + 1, 0.0), _wrap_pos(ny, ny, 0.5), np.zeros(1))
        ay = pot(1, x, y, z)[0]
        bx = (az[1:, :] - az[:-1, :]) / dy
        by = -(az[:, 1:] - az[:, :-1]) / dx
        bz = (ay[:, 1:] - ay[:, :-1]) / dx - (ax[1:, :] - ax[:-1, :]) / dy
        return bx[None], by[None], bz[None]
    nz = n[2]
    dz = 1.0 / nz
    # A_x at x-edges ((i+1/2)dx, j dy, k dz)
    x, y, z = _grid(_wrap_pos(nx, nx, 0.5), _wrap_pos(ny, ny + 1, 0.0), _wrap_pos(nz, nz + 1, 0.0))
    ax = pot(0, x, y, z)
    x, y, z = _grid(_wrap_pos(nx, nx + 1, 0.0), _wrap_pos(ny, ny, 0.5), _wrap_pos(nz, nz + 1, 0.0))
    ay = pot(1, x, y, z)
    x, y, z = _grid(_wrap_pos(nx, nx + 1, 0.0), _wrap_pos(ny, ny + 1, 0.0), _wrap_pos(nz, nz, 0.5))
    az = pot(2, x, y, z)
    bx = (az[:, 1:, :] - az[:, :-1, :]) / dy - (ay[1:, :, :] - ay[:-1, :, :]) / dz
    by = (ax[1:, :, :] - ax[:-1, :, :]) / dz - (az[:, :, 1:] - az[:, :, :-1]) / dx
    bz = (ay[:, :, 1:] - ay[:, :, :-1]) / dx - (ax[:, 1:, :] - ax[:, :-1, :]) / dy
    return bx, by, bz


def _face_mean_sq(ndim, b):
    """Mean over cells of |face-averaged B|^2 (used only to set an amplitude)."""
    bx, by, bz = b
    s = (0.5 * (bx[:, :, 1:] + bx[:, :, :-1])) ** 2 + (0.5 * (by[:, 1:, :] + by[:, :-1, :])) ** 2
    if ndim == 3:
        s = s + (0.5 * (bz[1:] + bz[:-1])) ** 2
    else:
        s = s + bz ** 2
    return float(np.mean(s))


def smooth_mhd(ndim, n, seed, v_rms=0.1, b_rms=0.1, rho_amp=0.1, jump=False, p0=1.0, p_amp=0.0):
    """Smooth seeded MHD state on the unit periodic box; the pressure is p0,
    or p0 (1 + p_amp f) with f a sum of seeded Fourier modes (drawn from a
    stream of its own, so p_amp = 0 reproduces the other fields exactly).

    Returns dict(prim=[rho, vx, vy, vz, p], b=[bx, by, bz], dx=[...]) in the
    interior layout."""
    n = tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    fld = _Field(rng, ndim)
    nx, ny = n[0], n[1]
    nz = n[2] if ndim == 3 else 1
    xs = (np.arange(nx) + 0.5) / nx
    ys = (np.arange(ny) + 0.5) / ny
    zs = (np.arange(nz) + 0.5) / nz if ndim == 3 else np.zeros(1)
    x, y, z = _grid(xs, ys, zs)
    rho = 1.0 + rho_amp * fld.f_rho(x, y, z)
    if jump:
        rho = np.where((x >= 0.25) & (x < 0.75), 4.0 * rho, rho)
    v = fld.curl_psi(x, y, z)
    vr = np.sqrt(np.mean(v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    v = [c * (v_rms / vr) for c in v]
    p = np.full_like(rho, p0)
    if p_amp:
        p = p0 * (1.0 + p_amp * _Field(np.random.default_rng(seed + 7919), ndim).f_rho(x, y, z))
    b = list(curl_faces(ndim, n, fld.pot))
    scale = b_rms / np.sqrt(_face_mean_sq(ndim, b))
    b = [c * scale for c in b]
    dx = [1.0 / nx, 1.0 / ny, 1.0 / nz if ndim == 3 else 1.0]
    return {"prim": [rho, v[0], v[1], v[2], p], "b": b, "dx": dx, "ndim": ndim, "n": n}


def uniform_state(ndim, n, rho=1.0, v=(0.1, -0.05, 0.02), p=1.0, B=(0.3, 0.2, -0.1)):
    """Spatially uniform state (every cell and face equal)."""
    nx, ny = n[0], n[1]
    nz = n[2] if ndim == 3 else 1
    shp = (nz, ny, nx)
    prim = [np.full(shp, float(rho)), np.full(shp, float(v[0])), np.full(shp, float(v[1])),
            np.full(shp, float(v[2])), np.full(shp, float(p))]
    bx = np.full((nz, ny, nx + 1), float(B[0]))
    by = np.full((nz, ny + 1, nx), float(B[1]))
    bz = np.full((nz + 1, ny, nx) if ndim == 3 else shp, float(B[2]))
    dx = [1.0 / nx, 1.0 / ny, 1.0 / nz if ndim == 3 else 1.0]
    return {"prim": prim, "b": [bx, by, bz], "dx": dx, "ndim": ndim, "n": tuple(n)}


def aligned_field_state(n, seed, B0=1.0, p0=0.1, eps=1e-7, amp=0.1):
    """3D state that varies along y only: rho, p, vx, vy are sums of seeded
    Fourier modes in y, vz = 0, and the face field is uniform, (B0, 0, eps)
    with B0^2 well above gamma p.  Faces normal to x then see equal left and
    right states with no transverse field and an Alfven-dominated fast speed
    (the degenerate outer star states of HLLD), and faces normal to z see
    equal states at rest with a vanishing normal field (degenerate inner
    states)."""
    n = tuple(int(v) for v in n)
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    y = (np.arange(ny) + 0.5) / ny

    def modes():
        f = np.zeros(ny)
        for _ in range(4):
            k = int(rng.integers(1, 5))
            f += rng.uniform(0.5, 1.0) * np.cos(2.0 * np.pi * k * y + rng.uniform(0.0, 2.0 * np.pi))
        return f / 4.0

    shp = (nz, ny, nx)

    def col(v):
        return np.ascontiguousarray(np.broadcast_to(v[None, :, None], shp))

    rho = col(1.0 + amp * modes())
    p = col(p0 * (1.0 + amp * modes()))
    vx = col(0.1 * modes())
    vy = col(0.1 * modes())
    vz = np.zeros(shp)
    bx = np.full((nz, ny, nx + 1), float(B0))
    by = np.zeros((nz, ny + 1, nx))
    bz = np.full((nz + 1, ny, nx), float(eps))
    return {"prim": [rho, vx, vy, vz, p], "b": [bx, by, bz], "dx": [1.0 / nx, 1.0 / ny, 1.0 / nz], "ndim": 3,
            "n": n}


def alfven_wave(ndim, N, amp=1e-6, gamma=5.0 / 3.0):
    """Linear Alfven wave on the unit box: B0 parallel to k, |B0| = 1, rho = 1,
    p = 1/gamma (so v_A = 1, omega = |k|); dB = amp e sin(k.x), dv = -dB.
    k = 2 pi (1, 2) with e = z in 2D; k = 2 pi (1, 1, 2) with e = (1,-1,0)/sqrt2
    in 3D, dB from its vector potential (amp/|k|^2)(k x e) cos(k.x)."""
    if ndim == 2:
        kv = np.array([1.0, 2.0, 0.0])
        e = np.array([0.0, 0.0, 1.0])
        n = (N, N)
    else:
        kv = np.array([1.0, 1.0, 2.0])
        e = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
        n = (N, N, N)
    k = TWO_PI * kv
    khat = kv / np.linalg.norm(kv)
    B0 = khat
    nx, ny = n[0], n[1]
    nz = n[2] if ndim == 3 else 1
    xs = (np.arange(nx) + 0.5) / nx
    ys = (np.arange(ny) + 0.5) / ny
    zs = (np.arange(nz) + 0.5) / nz if ndim == 3 else np.zeros(1)
    x, y, z = _grid(xs, ys, zs)
    th = k[0] * x + k[1] * y + k[2] * z
    dB = [amp * e[a] * np.sin(th) for a in range(3)]
    prim = [np.ones_like(x), -dB[0], -dB[1], -dB[2], np.full_like(x, 1.0 / gamma)]
    a_vec = np.cross(k, e) * (amp / np.dot(k, k))

    def pot(comp, xx, yy, zz):
        return a_vec[comp] * np.cos(k[0] * xx + k[1] * yy + k[2] * zz)

    if ndim == 3:
        bx, by, bz = curl_faces(3, n, pot)
        bx = bx + B0[0]
        by = by + B0[1]
        bz = bz + B0[2]
    else:
        bx = np.full((1, ny, nx + 1), B0[0])
        by = np.full((1, ny + 1, nx), B0[1])
        bz = dB[2].copy()
    dx = [1.0 / nx, 1.0 / ny, 1.0 / nz if ndim == 3 else 1.0]
    return {"prim": prim, "b": [bx, by, bz], "dx": dx, "ndim": ndim, "n": n, "omega": float(np.linalg.norm(k))}


def brio_wu(N, ny=4):
    """Brio & Wu (1988) shock tube along x on [0,1] x [0, ny/N): gamma = 2,
    left (rho, p, By) = (1, 1, 1), right (0.125, 0.1, -1), Bx = 0.75, v = 0."""
    nx = N
    xs = (np.arange(nx) + 0.5) / nx
    left = xs < 0.5
    shp = (1, ny, nx)
    rho = np.broadcast_to(np.where(left, 1.0, 0.125), shp).copy()
    p = np.broadcast_to(np.where(left, 1.0, 0.1), shp).copy()
    zero = np.zeros(shp)
    bx = np.full((1, ny, nx + 1), 0.75)
    by = np.broadcast_to(np.where(left, 1.0, -1.0), (1, ny + 1, nx)).copy()
    bz = np.zeros(shp)
    dx = [1.0 / nx, 1.0 / nx, 1.0]
    return {"prim": [rho, zero.copy(), zero.copy(), zero.copy(), p], "b": [bx, by, bz], "dx": dx, "ndim": 2,
            "n": (nx, ny)}


def advected_profile(N, seed=7, v=(0.37, 0.0, 0.0), p=1.0, B=(0.0, 0.0, 0.0), ndim=2, ny=4):
    """Density profile rho(x) = 1 + 0.5 sum of 3 random x-modes, advected at
    constant v, p and B (a contact discontinuity problem along x)."""
    rng = np.random.default_rng(seed)
    nx = N
    xs = (np.arange(nx) + 0.5) / nx
    ks = rng.integers(1, 5, size=3)
    ph = rng.uniform(0.0, TWO_PI, size=3)
    prof = 1.0 + 0.5 * sum(np.cos(TWO_PI * ks[m] * xs + ph[m]) for m in range(3)) / 3.0
    if ndim == 2:
        shp = (1, ny, nx)
        n = (nx, ny)
    else:
        shp = (ny, ny, nx)
        n = (nx, ny, ny)
    rho = np.broadcast_to(prof, shp).copy()
    u = uniform_state(ndim, n, 1.0, v, p, B)
    u["prim"][0] = rho
    u["dx"] = [1.0 / nx, 1.0 / nx, 1.0 / nx if ndim == 3 else 1.0]
    return u


# ---------------------------------------------------------------- hierarchies
def _draw_extent(rng, lo_ext, hi_ext, log_uniform):
    if log_uniform:
        e = float(np.exp(rng.uniform(np.log(lo_ext), np.log(hi_ext))))
        return int(min(hi_ext, max(lo_ext, round(e / 2) * 2)))
    return int(rng.integers(lo_ext // 2, hi_ext // 2 + 1)) * 2


def _partition(rng, length, lo_ext, hi_ext, log_uniform=False):
    """Split `length` cells into consecutive even segments with extents in
    [lo_ext, hi_ext] (seeded, uniform or log-uniform); the last segment
    absorbs the remainder."""
    segs = []
    left = length
    while left > 0:
        if left <= hi_ext:
            if left >= lo_ext or not segs:
                segs.append(left)
            else:
                segs[-1] += left
                if segs[-1] > hi_ext:  # split the last two evenly
                    t = segs.pop()
                    a = (t // 2) // 2 * 2
                    segs += [a, t - a]
            break
        e = _draw_extent(rng, lo_ext, hi_ext, log_uniform)
        if left - e < lo_ext and left - e != 0:
            e = left - lo_ext if left - lo_ext <= hi_ext else e
        segs.append(e)
        left -= e
    return segs


def _tile_box(rng, lo, hi, ndim, lo_ext, hi_ext, log_uniform=False):
    axes = []
    for a in range(ndim):
        segs = _partition(rng, hi[a] - lo[a], lo_ext, hi_ext, log_uniform)
        starts = np.cumsum([0] + segs[:-1]) + lo[a]
        axes.append(list(zip(starts, segs)))
    boxes = []
    if ndim == 2:
        for (y0, ny) in axes[1]:
            for (x0, nx) in axes[0]:
                boxes.append(((int(x0), int(y0)), (int(x0 + nx), int(y0 + ny))))
    else:
        for (z0, nz) in axes[2]:
            for (y0, ny) in axes[1]:
                for (x0, nx) in axes[0]:
                    boxes.append(((int(x0), int(y0), int(z0)), (int(x0 + nx), int(y0 + ny), int(z0 + nz))))
    return boxes


def amr_hierarchy(ndim, N0, nlevels, seed, ext=(8, 32), fill_fraction=0.125, ghost=4, max_boxes=4, ratio=2,
                  log_uniform=False):
    """Seeded nested hierarchy.  Level 0 tiles the periodic domain; each
    level l >= 1 covers about `fill_fraction` of the volume of level l-1 with
    1..max_boxes boxes placed inside the level-(l-1) boxes shrunk by the
    nesting buffer (ghost/R + 1 coarse cells); every box is tiled by grids
    whose extents are even and drawn from [ext[0], ext[1]] (uniformly, or
    log-uniformly when log_uniform).  Returns a list of (level, lo, hi) in
    level-l cell indices."""
    rng = np.random.default_rng(seed)
    N0 = tuple(int(v) for v in N0)[:ndim]
    grids = [(0, lo, hi) for lo, hi in _tile_box(rng, (0,) * ndim, N0, ndim, ext[0], ext[1], log_uniform)]
    parents = [((0,) * ndim, N0)]  # boxes of the previous level (level units)
    buf = ghost // ratio + 1
    for l in range(1, nlevels):
        cover = sum(np.prod([h - lo for lo, h in zip(b[0], b[1])]) for b in parents)
        target = fill_fraction * cover * ratio ** ndim  # cells on level l
        nb = int(rng.integers(1, max_boxes + 1))
        boxes = []
        tries = 0
        while len(boxes) < nb and tries < 1000:
            tries += 1
            vol = target / nb
            side = max(ext[0], int(round(vol ** (1.0 / ndim) / 2)) * 2)
            pb = parents[int(rng.integers(0, len(parents)))]
            # parent box in level-l units, shrunk by the buffer (periodic
            # level 0 needs no shrink across the domain edge)
            lo_p = [pb[0][a] * ratio + (buf * ratio if l > 1 else 0) for a in range(ndim)]
            hi_p = [pb[1][a] * ratio - (buf * ratio if l > 1 else 0) for a in range(ndim)]
            ext_ok = all(hi_p[a] - lo_p[a] >= side for a in range(ndim))
            if not ext_ok:
                side = min(hi_p[a] - lo_p[a] for a in range(ndim)) // 2 * 2
                if side < ext[0]:
                    continue
            lo = []
            for a in range(ndim):
                span = (hi_p[a] - lo_p[a] - side) // 2
                lo.append(lo_p[a] + 2 * int(rng.integers(0, span + 1)))
            hi = [x + side for x in lo]
            # keep boxes apart by the nesting buffer of the next level
            ok = True
            for (blo, bhi) in boxes:
                if all(lo[a] < bhi[a] + 2 * buf and blo[a] < hi[a] + 2 * buf for a in range(ndim)):
                    ok = False
            if ok:
                boxes.append((tuple(lo), tuple(hi)))
        for (blo, bhi) in boxes:
            grids += [(l, lo, hi) for lo, hi in _tile_box(rng, blo, bhi, ndim, ext[0], ext[1], log_uniform)]
        parents = boxes
    return grids


def _edge_mean_factor(k, h_fine, r):
    """Mean of cos(theta0 + m * 2 pi k h_fine) over m = 0..r-1 about the
    centre of the run: cos(theta_mid) * sin(r d/2) / (r sin(d/2))."""
    d = TWO_PI * k * h_fine
    if r == 1 or abs(np.sin(d / 2)) < 1e-300:
        return 1.0
    return np.sin(r * d / 2) / (r * np.sin(d / 2))


def amr_fields(ndim, N0, nlevels, grids, seed, v_rms=0.1, b_rms=0.3, rho_amp=0.1, ratio=2, p_amp=0.0):
    """Per-grid primitive data of a hierarchy, sampled from one set of smooth
    random fields.  Cells take point values at their centres.  The vector
    potential of every level is the mean of the finest level's edge samples
    along each edge (a closed form per Fourier mode), so face B of every
    level is the discrete curl of consistent potentials: a coarse face equals
    the mean of the finest faces on it, up to rounding.  Amplitudes are set
    from level 0.  The pressure is 1, or 1 + p_amp f with f smooth modes of a
    stream of their own.  Returns a list of dict(prim=[...], b=[...]) per
    grid."""
    rng = np.random.default_rng(seed)
    fld = _Field(rng, ndim)
    pfld = _Field(np.random.default_rng(seed + 7919), ndim) if p_amp else None
    N0 = tuple(int(v) for v in N0)[:ndim]
    Lf = nlevels - 1

    def level_pot(l):
        r = ratio ** (Lf - l)
        hf = [1.0 / (N0[a] * ratio ** Lf) for a in range(ndim)] + [1.0] * (3 - ndim)

        def pot(comp, x, y, z):
            out = np.zeros_like(x)
            for m in range(8):
                fac = 1.0
                if comp < ndim:  # averaged along the edge direction
                    fac = _edge_mean_factor(fld.k_a[m][comp], hf[comp], r)
                out += fld.a_a[m, comp] * fac * np.cos(_phase(fld.k_a[m], fld.phi_a[m], x, y, z))
            return out

        return pot

    def sample_grid(l, lo, hi):
        n = [hi[a] - lo[a] for a in range(ndim)]
        Nl = [N0[a] * ratio ** l for a in range(ndim)]
        h = [1.0 / Nl[a] for a in range(ndim)]
        xs = (np.arange(lo[0], hi[0]) + 0.5) * h[0]
        ys = (np.arange(lo[1], hi[1]) + 0.5) * h[1]
        zs = (np.arange(lo[2], hi[2]) + 0.5) * h[2] if ndim == 3 else np.zeros(1)
        x, y, z = _grid(xs, ys, zs)
        rho = 1.0 + rho_amp * fld.f_rho(x, y, z)
        v = fld.curl_psi(x, y, z)
        p = 1.0 + p_amp * pfld.f_rho(x, y, z) if p_amp else np.ones_like(rho)
        pot = level_pot(l)

        def wp(a, count, off):
            return (np.arange(lo[a], lo[a] + count) % Nl[a] + off) * h[a]

        nx, ny = n[0], n[1]
        if ndim == 3:
            nz = n[2]
            x_, y_, z_ = _grid(wp(0, nx, 0.5), wp(1, ny + 1, 0.0), wp(2, nz + 1, 0.0))
            ax = pot(0, x_, y_, z_)
            x_, y_, z_ = _grid(wp(0, nx + 1, 0.0), wp(1, ny, 0.5), wp(2, nz + 1, 0.0))
            ay = pot(1, x_, y_, z_)
            x_, y_, z_ = _grid(wp(0, nx + 1, 0.0), wp(1, ny + 1, 0.0), wp(2, nz, 0.5))
            az = pot(2, x_, y_, z_)
            bx = (az[:, 1:, :] - az[:, :-1, :]) / h[1] - (ay[1:, :, :] - ay[:-1, :, :]) / h[2]
            by = (ax[1:, :, :] - ax[:-1, :, :]) / h[2] - (az[:, :, 1:] - az[:, :, :-1]) / h[0]
            bz = (ay[:, :, 1:] - ay[:, :, :-1]) / h[0] - (ax[:, 1:, :] - ax[:, :-1, :]) / h[1]
        else:
            zero = np.zeros(1)
            x_, y_, z_ = _grid(wp(0, nx + 1, 0.0), wp(1, ny + 1, 0.0), zero)
            az = pot(2, x_, y_, z_)[0]
            x_, y_, z_ = _grid(wp(0, nx, 0.5), wp(1, ny + 1, 0.0), zero)
            ax = pot(0, x_, y_, z_)[0]
            x_, y_, z_ = _grid(wp(0, nx + 1, 0.0), wp(1, ny, 0.5), zero)
            ay = pot(1, x_, y_, z_)[0]
            bx = ((az[1:, :] - az[:-1, :]) / h[1])[None]
            by = (-(az[:, 1:] - az[:, :-1]) / h[0])[None]
            bz = ((ay[:, 1:] - ay[:, :-1]) / h[0] - (ax[1:, :] - ax[:-1, :]) / h[1])[None]
        return rho, v, [bx, by, bz], p

    raw = [sample_grid(l, lo, hi) for (l, lo, hi) in grids]
    # amplitudes from level 0 (which tiles the domain)
    vs, bs, nc = 0.0, 0.0, 0
    for (l, lo, hi), (rho, v, b, _p) in zip(grids, raw):
        if l != 0:
            continue
        vs += float(np.sum(v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
        nc += rho.size
        bs += _face_mean_sq(ndim, b) * rho.size
    vscale = v_rms / np.sqrt(vs / nc)
    bscale = b_rms / np.sqrt(bs / nc)
    out = []
    for (l, lo, hi), (rho, v, b, p) in zip(grids, raw):
        prim = [rho, v[0] * vscale, v[1] * vscale, v[2] * vscale, p]
        out.append({"prim": prim, "b": [c * bscale for c in b]})
    return out


def loss_box(ndim, n, size, seed):
    """Seeded corner of a size^ndim box of cells on the periodic grid n (the
    box may wrap).  Returns (lo, len) tuples over the active axes."""
    rng = np.random.default_rng(seed)
    lo = tuple(int(rng.integers(0, n[a])) for a in range(ndim))
    return lo, (size,) * ndim


def control_directions(shape, count, seed, scale=0.1):
    """`count` seeded directions in (rho, vx, vy, vz): N(0, 1) entries
    times `scale`, each a list of four arrays of `shape`."""
    rng = np.random.default_rng(seed)
    return [[scale * rng.normal(size=shape) for _ in range(4)] for _ in range(count)]


def split_grid_fields(ic, boxes):
    """Interior arrays of each sub-box (lo, hi) of a single-grid state `ic`
    (cells, and the faces on and inside the sub-box)."""
    ndim = ic["ndim"]
    out = []
    for lo, hi in boxes:
        lo3 = tuple(lo) + (0,) * (3 - len(lo))
        hi3 = tuple(hi) + (1,) * (3 - len(hi))
        cs = (slice(lo3[2], hi3[2]), slice(lo3[1], hi3[1]), slice(lo3[0], hi3[0]))
        prim = [np.ascontiguousarray(np.asarray(p).reshape(_cell_shape(ic))[cs]) for p in ic["prim"]]
        b = []
        for a in range(3):
            sl = list(cs)
            if a < ndim:
                sl[2 - a] = slice(cs[2 - a].start, cs[2 - a].stop + 1)
            arr = np.asarray(ic["b"][a])
            if ndim == 2 and a == 2:
                arr = arr.reshape(_cell_shape(ic))
            b.append(np.ascontiguousarray(arr[tuple(sl)]))
        out.append({"prim": prim, "b": b, "dx": ic["dx"], "ndim": ndim, "n": tuple(hi3[a] - lo3[a] for a in range(ndim))})
    return out


def _cell_shape(ic):
    n = tuple(ic["n"]) + (1,) * (3 - len(ic["n"]))
    return (n[2], n[1], n[0])


def smooth_directions(n, count, seed, kmax=2, nmodes=4, scale=0.1):
    """`count` seeded smooth directions in (rho, vx, vy, vz) on the periodic
    grid n (cell centres): per field a sum of `nmodes` Fourier modes with
    integer wavevectors |k_a| <= kmax, N(0, 1) amplitudes and uniform phases,
    rescaled to rms `scale`."""
    rng = np.random.default_rng(seed)
    ndim = len(n)
    ax = [(np.arange(n[a]) + 0.5) / n[a] for a in range(ndim)]
    if ndim == 3:
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    else:
        Y, X = np.meshgrid(ax[1], ax[0], indexing="ij")
        Y, X = Y[None], X[None]
        Z = np.zeros_like(X)
    out = []
    for _ in range(count):
        d = []
        for _q in range(4):
            f = np.zeros_like(X)
            for _m in range(nmodes):
                k = rng.integers(-kmax, kmax + 1, size=3)
                if ndim == 2:
                    k[2] = 0
                if not np.any(k):
                    k[0] = 1
                f += rng.normal() * np.sin(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + rng.uniform(0, 2 * np.pi))
            f *= scale / np.sqrt(np.mean(f * f))
            d.append(f)
        out.append(d)
    return out


def deep_hierarchy(N0=200, seed=5, p_amp=0.0):
    """The deep-hierarchy workload: 3D, 6 levels, R = 2, each level covering
    12.5% of its parent (so every level holds about N0^3 cells), grids with
    log-uniform even extents in [8, 48], band 4.  N0 = 100 is its 1/8-volume
    subvolume.  Returns (grids, fields)."""
    grids = amr_hierarchy(3, (N0,) * 3, 6, seed=seed, ext=(8, 48), log_uniform=True)
    fields = amr_fields(3, (N0,) * 3, 6, grids, seed=seed, b_rms=0.3, p_amp=p_amp)
    return grids, fields
