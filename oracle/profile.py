"""Oracle of the warm-start initial state (TEST INFRASTRUCTURE ONLY: called by the tests, never
by the library or its binding).

A radial profile gives log rho at r_k = r0 + k dr, k = 0..63, r the distance from the lattice
centre (nx/2, ny/2).  The initial density is the piecewise-linear interpolant in r of that
profile, shifted radially by s (rho(r - s)), held at the first value below r0 and at the last
beyond r0 + 63 dr, and the populations are the rest equilibria f_q = w_q rho (Eq. 2 with
u = 0).  In a periodic box the total mass fixes the equilibrium, so the shift is the one whose
density sum equals the mass of the state the warm start replaces: found here by plain
bisection, written out with numpy in FP64.
"""
from __future__ import annotations

import numpy as np

POINTS = 64
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def radii(r0, dr):
    return r0 + dr * np.arange(POINTS)


def density(nx, ny, log_profile, r0, dr, shift=0.0):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2)
    # np.interp holds the end values outside [r_0, r_63]
    return np.exp(np.interp(r - shift, radii(r0, dr), np.asarray(log_profile, dtype=np.float64)))


def populations(nx, ny, log_profile, r0, dr, shift=0.0):
    """f[9][ny][nx] of the rest equilibrium of the profile density."""
    return W[:, None, None] * density(nx, ny, log_profile, r0, dr, shift)[None]


def mass_matched_shift(nx, ny, log_profile, r0, dr, mass, rtol=1e-13):
    """The shift within +- half the lattice diagonal whose density sum equals `mass`, or None."""
    span = 0.5 * np.hypot(nx, ny)
    lo, hi = -span, span

    def excess(s):
        return density(nx, ny, log_profile, r0, dr, s).sum() - mass
    f_lo, f_hi = excess(lo), excess(hi)
    if not (f_lo < 0 < f_hi or f_hi < 0 < f_lo):
        return None
    mid = 0.5 * (lo + hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f_mid = excess(mid)
        if abs(f_mid) <= rtol * mass:
            break
        if (f_mid < 0) == (f_lo < 0):
            lo, f_lo = mid, f_mid
        else:
            hi = mid
    return mid


def rest_populations(params, rho):
    """f = f^eq(rho, u) with u = -F / (2 rho): the density at physical rest (the fluid velocity
    v = u + F / (2 rho) of Sec. 3 is zero), F the interaction force of rho (Eq. 6, psi of
    Eq. 7) as the oracle's stepper computes it."""
    import oracle
    rho = np.asarray(rho, dtype=np.float64)
    fl = oracle.fields(params, oracle.init_feq(rho))
    return oracle.init_feq(rho, -fl["Fx"] / (2 * rho), -fl["Fy"] / (2 * rho))
