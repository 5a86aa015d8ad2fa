"""Pins of the oracle's pointwise pieces against closed forms and textbook
special cases (CPU only)."""

import itertools

import numpy as np
import pytest

import oracle as O

GAMMA = 5.0 / 3.0


def rand_prim(rng, bn=None):
    W = np.array([rng.uniform(0.3, 2.0), *rng.normal(0, 0.5, 3), rng.uniform(0.2, 2.0), *rng.normal(0, 0.7, 3)])
    if bn is not None:
        W[5] = bn
    return W


def test_cons_prim_round_trip():
    rng = np.random.default_rng(11)
    for _ in range(200):
        W = rand_prim(rng)
        U = O.prim_to_cons(W, GAMMA)
        W2 = O.cons_to_prim(U, GAMMA)
        U2 = O.prim_to_cons(W2, GAMMA)
        assert np.max(np.abs(W2 - W) / (np.abs(W) + 1.0)) < 1e-14
        assert np.max(np.abs(U2 - U) / (np.abs(U) + 1.0)) < 1e-14


def test_cons_known_values():
    # rho=2, v=(1,0,0), p=3, B=(0,2,0): E = 3/(2/3) + 0.5*2*1 + 0.5*4 = 4.5 + 1 + 2
    U = O.prim_to_cons([2.0, 1.0, 0.0, 0.0, 3.0, 0.0, 2.0, 0.0], GAMMA)
    assert U[4] == pytest.approx(7.5, rel=1e-15)
    assert U[1] == 2.0


def test_minmod_table():
    # All sign/order cases, brute force over a small value set.
    vals = [-3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 3.0]
    for a, b in itertools.product(vals, vals):
        m = O.minmod(a, b)
        if a * b <= 0:
            assert m == 0.0
        else:
            assert abs(m) == min(abs(a), abs(b))
            assert np.sign(m) == np.sign(a)


def wave_speeds(W, d, gamma):
    """Textbook ideal-MHD characteristic speeds along d (Jeffrey & Taniuti):
    u, u +- c_a, u +- c_s, u +- c_f."""
    rho, p = W[0], W[4]
    B = W[5:8]
    a2 = gamma * p / rho
    b2 = np.dot(B, B) / rho
    bn2 = B[d] ** 2 / rho
    disc = np.sqrt((a2 + b2) ** 2 - 4 * a2 * bn2)
    cf = np.sqrt(0.5 * (a2 + b2 + disc))
    cs = np.sqrt(max(0.5 * (a2 + b2 - disc), 0.0))
    ca = np.sqrt(bn2)
    u = W[1 + d]
    return np.sort([u - cf, u - ca, u - cs, u, u + cs, u + ca, u + cf])


@pytest.mark.parametrize("d", [0, 1, 2])
def test_flux_jacobian_eigenvalues(d):
    """The flux Jacobian dF_d/dU (normal B held fixed) must have the seven MHD
    wave speeds as eigenvalues: pins phys_flux and the variable maps."""
    rng = np.random.default_rng(100 + d)
    for _ in range(20):
        W = rand_prim(rng)
        U0 = O.prim_to_cons(W, GAMMA)
        idx = [s for s in range(8) if s != 5 + d]
        J = np.zeros((7, 7))
        for c, s in enumerate(idx):
            h = 1e-6 * max(1.0, abs(U0[s]))
            Up, Um = U0.copy(), U0.copy()
            Up[s] += h
            Um[s] -= h
            Fp = O.phys_flux(O.cons_to_prim(Up, GAMMA), d, GAMMA)
            Fm = O.phys_flux(O.cons_to_prim(Um, GAMMA), d, GAMMA)
            J[:, c] = ((Fp - Fm) / (2 * h))[idx]
        ev = np.sort(np.linalg.eigvals(J).real)
        np.testing.assert_allclose(ev, wave_speeds(W, d, GAMMA), atol=2e-6)


def test_fast_speed_limits():
    g = GAMMA
    # no field: sound speed
    assert O.fast_speed(1.3, 0.7, 0.0, 0.0, g) == pytest.approx(np.sqrt(g * 0.7 / 1.3), rel=1e-14)
    # field normal to the direction: sqrt(cs^2 + ca^2)
    cs2, ca2 = g * 0.7 / 1.3, 0.5 ** 2 / 1.3
    assert O.fast_speed(1.3, 0.7, 0.25, 0.0, g) == pytest.approx(np.sqrt(cs2 + ca2), rel=1e-14)
    # field along the direction: max(cs, ca)
    for B in (0.2, 2.0):
        assert O.fast_speed(1.3, 0.7, B * B, B, g) == pytest.approx(np.sqrt(max(cs2, B * B / 1.3)), rel=1e-13)


# ------------------------------------------------------------------- HLLD
def rot_flux(W, gamma):
    """Physical flux of a rotated state (n = x frame) via the lab-frame oracle
    flux in direction 0, reordered to the 7 HLLD components."""
    F = O.phys_flux(W, 0, gamma)
    return np.array([F[0], F[1], F[2], F[3], F[4], F[6], F[7]])


def test_hlld_consistency():
    rng = np.random.default_rng(5)
    for _ in range(200):
        W = rand_prim(rng)
        F, _ = O.hlld(W, W, GAMMA)
        np.testing.assert_allclose(F, rot_flux(W, GAMMA), rtol=1e-13, atol=1e-13)


def hllc_textbook(L, R, gamma, SL, SR):
    """HLLC of Toro (2009) Sec. 10.4 for the Euler equations (3 velocity
    components), with given outer speeds."""

    def cons(W):
        r, u, v, w, p = W
        return np.array([r, r * u, r * v, r * w, p / (gamma - 1) + 0.5 * r * (u * u + v * v + w * w)])

    def flux(W):
        r, u, v, w, p = W
        U = cons(W)
        return np.array([r * u, r * u * u + p, r * u * v, r * u * w, (U[4] + p) * u])

    rL, uL, vL, wL, pL = L
    rR, uR, vR, wR, pR = R
    Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) / (rL * (SL - uL) - rR * (SR - uR))

    def ustar(W, S):
        r, u, v, w, p = W
        E = cons(W)[4]
        f = r * (S - u) / (S - Ss)
        return f * np.array([1.0, Ss, v, w, E / r + (Ss - u) * (Ss + p / (r * (S - u)))])

    if SL >= 0:
        return flux(L)
    if Ss >= 0:
        return flux(L) + SL * (ustar(L, SL) - cons(L))
    if SR >= 0:
        return flux(R) + SR * (ustar(R, SR) - cons(R))
    return flux(R)


def test_hlld_reduces_to_hllc_without_field():
    rng = np.random.default_rng(6)
    for _ in range(300):
        L = rand_prim(rng)
        R = rand_prim(rng)
        L[5:] = 0.0
        R[5:] = 0.0
        F, info = O.hlld(L, R, GAMMA)
        cL = np.sqrt(GAMMA * L[4] / L[0])
        cR = np.sqrt(GAMMA * R[4] / R[0])
        SL = min(L[1], R[1]) - max(cL, cR)
        SR = max(L[1], R[1]) + max(cL, cR)
        ref = hllc_textbook(L[:5], R[:5], GAMMA, SL, SR)
        np.testing.assert_allclose(F[:5], ref, rtol=1e-12, atol=1e-12)
        assert F[5] == 0.0 and F[6] == 0.0


@pytest.mark.parametrize("u", [0.3, -0.4])
def test_hlld_isolated_contact_exact(u):
    """A pure contact (density jump only, same u, p, B, with B_n != 0) is
    resolved exactly: the flux is the physical flux of the upwind state."""
    L = np.array([1.0, u, 0.1, -0.2, 0.8, 0.6, 0.3, 0.4])
    R = L.copy()
    R[0] = 0.25
    F, info = O.hlld(L, R, GAMMA)
    up = L if u > 0 else R
    np.testing.assert_allclose(F, rot_flux(up, GAMMA), rtol=1e-12, atol=1e-13)


def test_hlld_isolated_rotational_exact():
    """An isolated rotational (Alfven) discontinuity moving at the Alfven speed
    relative to the flow is resolved exactly by HLLD."""
    rho, p, Bn, u = 1.0, 1.0, 0.8, 0.05
    ca = Bn / np.sqrt(rho)
    # Left state; right state rotates the tangential field by 90 degrees with
    # the velocity jump dv_t = -dB_t/sqrt(rho) of a wave moving at u + ca
    # (sign(Bn) > 0 convention: v_t - B_t/sqrt(rho) is invariant across it).
    BtL = np.array([0.5, 0.0])
    BtR = np.array([0.0, 0.5])
    vtL = np.array([0.1, -0.1])
    vtR = vtL - (BtR - BtL) / np.sqrt(rho)
    L = np.array([rho, u, *vtL, p, Bn, *BtL])
    R = np.array([rho, u, *vtR, p, Bn, *BtR])
    F, info = O.hlld(L, R, GAMMA)
    # The discontinuity moves right at u + ca > 0, so the interface sees L.
    assert u + ca > 0
    np.testing.assert_allclose(F, rot_flux(L, GAMMA), rtol=1e-11, atol=1e-12)


def test_hlld_mirror_symmetry():
    rng = np.random.default_rng(7)
    for _ in range(300):
        L = rand_prim(rng)
        R = rand_prim(rng, bn=L[5])
        F, _ = O.hlld(L, R, GAMMA)

        def mirror(W):
            M = W.copy()
            M[1] = -M[1]
            M[5] = -M[5]
            return M

        Fm, _ = O.hlld(mirror(R), mirror(L), GAMMA)
        sgn = np.array([-1, 1, -1, -1, -1, -1, -1.0])
        np.testing.assert_allclose(Fm, sgn * F, rtol=1e-11, atol=1e-12)


def test_hlld_continuity_across_regions():
    """Sweeping the flow speed moves every wave through the interface; the
    flux must stay continuous (no jump at region changes)."""
    base_L = np.array([1.0, 0.0, 0.2, -0.1, 1.0, 0.7, 0.4, 0.1])
    base_R = np.array([0.5, 0.0, -0.1, 0.2, 0.6, 0.7, -0.3, 0.2])
    us = np.linspace(-3.0, 3.0, 6001)
    Fs = []
    regions = set()
    for u in us:
        L = base_L.copy()
        R = base_R.copy()
        L[1] += u
        R[1] += u
        F, info = O.hlld(L, R, GAMMA)
        regions.add(info[0])
        Fs.append(F)
    Fs = np.array(Fs)
    jumps = np.max(np.abs(np.diff(Fs, axis=0)), axis=0)
    assert regions == {0, 1, 2, 3, 4, 5}
    # step in u is 1e-3; a continuous flux changes by O(1e-3) per step
    assert np.all(jumps < 2e-2)


def test_hlld_degenerate_paths_finite():
    # B_n = 0 (double-star degenerate) and B_t = 0 with Bn^2 = rho (S-u)^2 type cases
    L = np.array([1.0, 0.1, 0.0, 0.0, 1.0, 0.0, 0.5, 0.0])
    R = np.array([0.3, -0.1, 0.0, 0.0, 0.4, 0.0, -0.5, 0.0])
    F, info = O.hlld(L, R, GAMMA)
    # with B_n = 0 the Alfven waves merge with the contact: only F*_L / F*_R remain
    assert info[0] in (1, 4) and np.all(np.isfinite(F))
    L = np.array([1.0, 0.0, 0.0, 0.0, 1.0, 1.0, 0.0, 0.0])
    F, info = O.hlld(L, L, GAMMA)
    assert np.all(np.isfinite(F))
    np.testing.assert_allclose(F, rot_flux(L, GAMMA), atol=1e-14)
