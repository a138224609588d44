"""Batched parameter sweeps of static droplets (the sweeps over tau and T/Tc of Sec. 4, as one
job on one GPU): members drawn by `inputs.batch_draw`, initialised from a tanh profile or from
a predicted radial profile (expanded on the device), advanced by the library's batched sweep until the per-step change
of the velocity field falls below a tolerance.

Physics of every member (the droplet workloads): Guo forcing with Li's term, sigma = 0.125
(eps = 2, Eq. 32), A = 0, Carnahan-Starling EOS rescaled by K = 1/49, BGK or MRT
(s_rho = s_j = 1, s_e = s_eps = s_q = 1.1, s_nu = 1/tau).
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs

PHYSICS = dict(scheme="GUO_LI", sigma=0.125, A=0.0, K=1 / 49, s=(1.0, 1.1, 1.1, 1.0, 1.1))
PROFILE_POINTS = 64


def members_from_draw(draw, K=None):
    out = []
    for d in draw:
        m = dict(PHYSICS, nx=d.n, ny=d.n, T_over_Tc=d.T_over_Tc, tau=d.tau,
                 collision="MRT" if d.mrt else "BGK", R=d.R)
        if K is not None:
            m["K"] = K
        out.append(m)
    return out


def coexistence(lbm, m):
    """Maxwell densities (gas, liquid) of a member, from the library's EOS helper."""
    return lbm.eos_maxwell(lbm.make_eos(m["T_over_Tc"], K=m["K"]))


def tanh_density(lbm, m, W=5.0):
    g, l = coexistence(lbm, m)
    return inputs.droplet(m["nx"], m["ny"], m["R"], W, l, g)


def profile_radii(R):
    """Radii of the 64-point radial profile: r_k = 2 R k / 63."""
    return 2.0 * R * np.arange(PROFILE_POINTS) / (PROFILE_POINTS - 1)


def radial_profile(m, rho):
    """log rho of a field sampled at the 64 profile radii along the +x axis from the centre
    (linear interpolation between nodes)."""
    nx, ny = m["nx"], m["ny"]
    cx, cy = nx // 2, ny // 2
    line = rho[cy, :]
    xs = cx + profile_radii(m["R"])
    xs = np.minimum(xs, nx - 1)
    return np.log(np.interp(xs, np.arange(nx), line))


class WarmStart:
    """A predicted radial profile (64 values of log rho at the profile radii), stretched on the
    device to carry `mass`; `fallback` (a density array) is used if the library rejects it."""

    def __init__(self, log_profile, mass, fallback):
        self.log_profile = np.asarray(log_profile, dtype=np.float64)
        self.mass = float(mass)
        self.fallback = fallback


def run_batch(lbm, members, inits, tol=1e-9, check_every=100, max_steps=400_000, tx=128,
              segment=None, tol_rho=0.0):
    """Advance all members to equilibrium (velocity change per step < tol and, if tol_rho > 0,
    relative change per step of the probe densities < tol_rho).  inits[i] is a density array
    or a WarmStart; either starts at physical rest (v = 0).  Returns wall seconds, steps, statuses and the batch (its `fallbacks`
    counts warm starts that fell back)."""
    b = lbm.Batch(members, tx=tx)
    b.fallbacks = 0
    for i, init in enumerate(inits):
        if isinstance(init, WarmStart):
            try:
                b.init_profile(i, init.log_profile, members[i]["R"], init.mass)
            except lbm.LBMError:
                b.fallbacks += 1
                b.init_rest(i, init.fallback)
        else:
            b.init_rest(i, init)
        if segment is not None:
            b.set_segment(i, segment(members[i]))
    b.sync()
    t0 = time.perf_counter()
    steps, status = b.run(tol, check_every=check_every, max_steps=max_steps, tol_rho=tol_rho)
    b.sync()
    return time.perf_counter() - t0, steps, status, b
