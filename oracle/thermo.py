"""Thermodynamics of the (rescaled) Carnahan-Starling EOS, in high precision.

TEST INFRASTRUCTURE ONLY (part of the oracle).

* ``cs_pressure``       Eq. 29 and its K-rescaled form Eq. 30.
* ``critical_point``    the exact critical point of Eq. 29: dp/drho = d2p/drho2 = 0, solved
                        for (rho_c, T_c) from that definition with mpmath.  The rounded
                        constants printed under Eq. 29 (a = 0.4963 R^2 Tc^2/pc,
                        b = 0.18727 R Tc/pc) are only consistent with it to ~1e-4.
* ``maxwell``           equal-area coexistence densities, Eq. 19: p0(rho_g) = p0(rho_l) = p_c
                        and integral_{rho_g}^{rho_l} (p_c - p0) / rho^2 drho = 0.
* ``mechanical``        the mechanical stability condition Eq. 18 with psi of Eq. 7:
                        integral (p_c - p0) psi' / psi^(1+eps) drho = 0.
* ``eps_from_A`` etc.   the parameter maps eps = -2a/b with Table 1's (a, b) and Eq. 32.
* ``ss_psi`` etc.       the effective density of Eq. 33 and the pressure Eq. 7 implies for it,
                        p0 = rho/3 + G psi^2 / 2, with its Maxwell (Eq. 19) and mechanical
                        (Eq. 18) coexistence densities.

The root finding and quadrature are library routines (mpmath.findroot, mpmath.quad);
the bracketing and bisection on p_c are written out.
"""
from __future__ import annotations

from functools import lru_cache

import mpmath as mp

mp.mp.dps = 25


def cs_pressure(rho, T, a=1.0, b=4.0, R=1.0, K=1.0):
    """K * (rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2), eta = b rho / 4."""
    rho = mp.mpf(rho)
    eta = mp.mpf(b) * rho / 4
    return mp.mpf(K) * (rho * R * T * (1 + eta + eta**2 - eta**3) / (1 - eta) ** 3
                        - mp.mpf(a) * rho**2)


def cs_dpdrho(rho, T, a=1.0, b=4.0, R=1.0, K=1.0):
    """d p / d rho of Eq. 30, from d(rho Z)/d rho = Z + eta Z'(eta) with
    Z = (1 + eta + eta^2 - eta^3)/(1 - eta)^3 and Z' = (4 + 4 eta - 2 eta^2)/(1 - eta)^4
    (pinned against numerical differentiation in the tests)."""
    rho = mp.mpf(rho)
    eta = mp.mpf(b) * rho / 4
    Z = (1 + eta + eta**2 - eta**3) / (1 - eta) ** 3
    dZ = (4 + 4 * eta - 2 * eta**2) / (1 - eta) ** 4
    return mp.mpf(K) * (R * T * (Z + eta * dZ) - 2 * mp.mpf(a) * rho)


@lru_cache(maxsize=None)
def critical_point(a=1.0, b=4.0, R=1.0):
    """(rho_c, T_c, p_c) with dp/drho = 0 and d2p/drho2 = 0 (Eq. 29)."""
    def eqs(rho, T):
        f = lambda r: cs_pressure(r, T, a, b, R)
        return [mp.diff(f, rho, 1), mp.diff(f, rho, 2)]
    # Starting guess from the rounded constants printed under Eq. 29: their ratio gives
    # a / b = (0.4963 / 0.18727) R T_c.
    Tc0 = 0.18727 / 0.4963 * a / (b * R)
    rc, Tc = mp.findroot(eqs, (mp.mpf(0.13) * 4 / b, mp.mpf(Tc0)))
    pc = cs_pressure(rc, Tc, a, b, R)
    return float(rc), float(Tc), float(pc)


def temperature(T_over_Tc, a=1.0, b=4.0, R=1.0) -> float:
    return float(mp.mpf(T_over_Tc) * mp.mpf(critical_point(a, b, R)[1]))


def _spinodals(dp, rho_max):
    """Local maximum (gas side) and local minimum (liquid side) of p(rho): sign changes of
    dp/drho on a grid, refined by bisection."""
    grid = [rho_max * k / 400 for k in range(1, 400)]
    roots = []
    prev = dp(grid[0])
    for r0, r1 in zip(grid[:-1], grid[1:]):
        cur = dp(r1)
        if prev > 0 and cur < 0:
            roots.append(_bisect_increasing(lambda r: -dp(r), r0, r1))
        elif prev < 0 and cur > 0:
            roots.append(_bisect_increasing(dp, r0, r1))
        prev = cur
    if len(roots) != 2:
        raise ValueError("no two-phase region (T >= T_c?)")
    return roots[0], roots[1]


def _bisect_increasing(fn, lo, hi, iters=110):
    """Root of an increasing function on [lo, hi] by plain bisection."""
    for _ in range(iters):
        mid = (lo + hi) / 2
        if fn(mid) < 0:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2


def _coexistence(p, dp, weight, rho_max, tol=mp.mpf("1e-17")):
    """Bisection on p_c for integral_{rho_g}^{rho_l} (p_c - p(rho)) weight(rho) drho = 0."""
    s1, s2 = _spinodals(dp, rho_max)
    # Stay off the spinodal pressures, where a branch root becomes a double root.
    lo = max(p(s2), mp.mpf(0)) * (1 + mp.mpf("1e-12")) + mp.mpf("1e-300")
    hi = p(s1) * (1 - mp.mpf("1e-12"))

    def roots(pc):
        # p rises monotonically on (0, s1) and on (s2, rho_max); bracket, then bisect.
        g = _bisect_increasing(lambda r: p(r) - pc, mp.mpf(0), s1)
        k, r_hi = 1, s2 + (rho_max - s2) / 2
        while p(r_hi) < pc:
            k += 1
            r_hi = s2 + (rho_max - s2) * (1 - mp.mpf(2) ** -k)
        l = _bisect_increasing(lambda r: p(r) - pc, s2, r_hi)
        return g, l

    def integral(pc):
        g, l = roots(pc)
        return mp.quad(lambda r: (pc - p(r)) * weight(r), [g, s1, s2, l]), g, l

    I_lo = integral(lo)[0]
    I_hi = integral(hi)[0]
    if I_lo * I_hi > 0:
        raise ValueError("coexistence pressure not bracketed")
    for _ in range(200):
        mid = (lo + hi) / 2
        I_mid, g, l = integral(mid)
        if I_mid == 0 or (hi - lo) < tol * hi:
            break
        if (I_mid > 0) == (I_hi > 0):
            hi, I_hi = mid, I_mid
        else:
            lo, I_lo = mid, I_mid
    return float(g), float(l), float(mid)


@lru_cache(maxsize=None)
def maxwell(T_over_Tc, a=1.0, b=4.0, R=1.0, K=1.0):
    """(rho_g, rho_l, p_c) from the Maxwell equal-area rule, Eq. 19."""
    T = mp.mpf(T_over_Tc) * mp.mpf(critical_point(a, b, R)[1])
    p = lambda r: cs_pressure(r, T, a, b, R, K)
    dp = lambda r: cs_dpdrho(r, T, a, b, R, K)
    return _coexistence(p, dp, lambda r: 1 / r**2, mp.mpf(4) / b)


@lru_cache(maxsize=None)
def mechanical(T_over_Tc, eps, a=1.0, b=4.0, R=1.0, K=1.0, G=-1.0):
    """(rho_g, rho_l, p_c) from the mechanical stability condition, Eq. 18, with
    psi = sqrt(2 (p0 - rho/3) / G) (Eq. 7)."""
    T = mp.mpf(T_over_Tc) * mp.mpf(critical_point(a, b, R)[1])
    p = lambda r: cs_pressure(r, T, a, b, R, K)
    dp = lambda r: cs_dpdrho(r, T, a, b, R, K)
    psi = lambda r: mp.sqrt(2 * (p(r) - r / 3) / G)
    # psi psi' = (p0' - 1/3) / G
    w = lambda r: (dp(r) - mp.mpf(1) / 3) / (G * psi(r)) / psi(r) ** (1 + mp.mpf(eps))
    # The psi radicand rho/3 - p0 turns negative on the steep liquid branch (eta -> 1);
    # the liquid search must stop before it.
    rad = lambda r: r / 3 - p(r)
    k, r_hi = 1, mp.mpf(2) / b
    while rad(r_hi) > 0:
        k += 1
        r_hi = mp.mpf(4) / b * (1 - mp.mpf(2) ** -k)
    rho_max = _bisect_increasing(lambda r: -rad(r), mp.mpf(2) / b, r_hi)
    return _coexistence(p, dp, w, rho_max)


def chemical_potential(rho, T, a=1.0, b=4.0, R=1.0, K=1.0):
    """mu(rho) of the Carnahan-Starling fluid up to a constant, from its Helmholtz free energy
    per volume rho R T (ln rho - 1) + rho R T (4 eta - 3 eta^2) / (1 - eta)^2 - a rho^2.
    Used only to pin the Maxwell solver: equal mu and equal p at coexistence."""
    rho = mp.mpf(rho)
    fv = lambda r: K * (r * R * T * (mp.log(r) - 1)
                        + r * R * T * (4 * (b * r / 4) - 3 * (b * r / 4) ** 2)
                        / (1 - b * r / 4) ** 2 - a * r**2)
    return mp.diff(fv, rho)


# ---- Eq. 33 (Sbragaglia-Shan effective density) ---------------------------------------

def ss_psi(rho, eps):
    """psi = exp(-1/rho) for eps = 0, (rho / (1 + rho))^(1/eps) otherwise (Eq. 33)."""
    rho = mp.mpf(rho)
    if eps == 0:
        return mp.exp(-1 / rho)
    return (rho / (1 + rho)) ** (1 / mp.mpf(eps))


def ss_dpsi(rho, eps):
    """d psi / d rho of Eq. 33: psi / rho^2 (eps = 0), psi / (eps rho (1 + rho)) otherwise."""
    rho = mp.mpf(rho)
    if eps == 0:
        return ss_psi(rho, eps) / rho**2
    return ss_psi(rho, eps) / (mp.mpf(eps) * rho * (1 + rho))


def ss_pressure(rho, eps, G):
    """The pressure Eq. 7 implies for psi of Eq. 33: rho/3 + G psi^2 / 2."""
    return mp.mpf(rho) / 3 + mp.mpf(G) * ss_psi(rho, eps) ** 2 / 2


def _ss_rho_max(eps, G):
    # psi -> 1, p0 -> rho/3 + G/2 as rho -> infinity: the loop lies well below rho = -3G.
    return mp.mpf(-6) * G + 4


@lru_cache(maxsize=None)
def ss_maxwell(eps, G):
    """(rho_g, rho_l, p_c) of the Maxwell rule (Eq. 19) for the pressure implied by Eq. 33."""
    p = lambda r: ss_pressure(r, eps, G)
    dp = lambda r: mp.mpf(1) / 3 + G * ss_psi(r, eps) * ss_dpsi(r, eps)
    return _coexistence(p, dp, lambda r: 1 / r**2, _ss_rho_max(eps, G))


@lru_cache(maxsize=None)
def ss_mechanical(eps_mech, eps, G):
    """(rho_g, rho_l, p_c) of Eq. 18 with exponent eps_mech for psi of Eq. 33 (exponent eps)."""
    p = lambda r: ss_pressure(r, eps, G)
    dp = lambda r: mp.mpf(1) / 3 + G * ss_psi(r, eps) * ss_dpsi(r, eps)
    w = lambda r: ss_dpsi(r, eps) / ss_psi(r, eps) ** (1 + mp.mpf(eps_mech))
    return _coexistence(p, dp, w, _ss_rho_max(eps, G))


# ---- parameter maps ------------------------------------------------------------------

def eps_from_table1(a_coef, b_coef):
    """eps = -2 a / b (text under Eq. 18) with (a, b) of Table 1."""
    return -2.0 * a_coef / b_coef


def eps_from_A(A):
    """Kupershtokh hybrid model: Table 1 gives (a, b) = (3A, 3)."""
    return eps_from_table1(3.0 * A, 3.0)


def eps_from_sigma(sigma, G=-1.0, alpha=0.0, beta=3.0, dt=1.0):
    """Eq. 32: eps = -2 (alpha + 24 dt G sigma) / beta, with Table 1's effective-density
    (alpha, beta) = (0, 3) for Li's model."""
    return -2.0 * (alpha + 24.0 * dt * G * sigma) / beta
