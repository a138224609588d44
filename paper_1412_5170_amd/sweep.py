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


PROFILE_SPACING = 2.0
PROFILE_CENTRE = 23.5  # fractional index of the interface radius


def profile_radii(R):
    """Radii of the 64-point radial profile around the interface radius R:
    r_k = R + (k - 23.5) h, h = 2 lattice units, from 47 nodes inside to 79 outside (the
    interface keeps its width in lattice units whatever R is, so the same network serves every
    droplet size).  The vapour side reaches further: at T/Tc = 0.5 and K = 1/49 the vapour 47
    nodes out is still 10 % above its plateau, 79 nodes out within 0.1 %."""
    return R + PROFILE_SPACING * (np.arange(PROFILE_POINTS) - PROFILE_CENTRE)


def radial_profile(m, rho):
    """log rho of a field sampled at the 64 profile radii along the +x axis from the centre
    (linear interpolation between nodes; radii below 0 mirror, radii past the last node along
    the axis take its value)."""
    nx = m["nx"]
    cx, cy = nx // 2, m["ny"] // 2
    line = rho[cy, :]
    xs = cx + np.abs(profile_radii(m["R"]))
    xs = np.minimum(xs, nx - 1)
    return np.log(np.interp(xs, np.arange(nx), line))


class WarmStart:
    """A predicted radial profile (64 values of log rho at the profile radii of a member),
    shifted on the device to carry `mass`; `fallback` (a density array) is used if the library
    rejects it."""

    def __init__(self, log_profile, R, mass, fallback):
        self.log_profile = np.asarray(log_profile, dtype=np.float64)
        self.r0 = float(profile_radii(R)[0])
        self.dr = PROFILE_SPACING
        self.mass = float(mass)
        self.fallback = fallback


def run_to_equilibrium(b, tol, tol_rho=0.0, check_every=100, max_steps=400_000,
                       chunk=50_000, report=None):
    """`lbm_batch_run` in chunks of `chunk` steps: lattices stopped by the chunk's step cap are
    re-activated for the next chunk (their step counts keep counting), so a long run reports
    progress between chunks.  Returns the steps and statuses of the last chunk."""
    n = len(b.members)
    cap = min(chunk, max_steps)
    final = [b.lbm.LBM_ESTATE] * n      # lattices never active keep LBM_ESTATE
    t0 = time.perf_counter()
    while True:
        steps, status = b.run(tol, check_every=check_every, max_steps=cap, tol_rho=tol_rho)
        for i in range(n):
            if status[i] != b.lbm.LBM_ESTATE:   # active in this chunk
                final[i] = status[i]
        capped = [i for i in range(n) if status[i] == b.lbm.LBM_ENOTCONVERGED]
        if report is not None:
            done = sum(s == 0 for s in final)
            report(f"sweep: {cap} steps cap, {done}/{n} converged, {len(capped)} running, "
                   f"{time.perf_counter() - t0:.1f} s")
        if not capped or cap >= max_steps:
            return steps, final
        for i in capped:
            b.set_active(i, 1)
        cap = min(cap + chunk, max_steps)


def run_batch(lbm, members, inits, tol=1e-9, check_every=100, max_steps=400_000, tx=256,
              segment=None, tol_rho=0.0, chunk=None, report=None, flags=None):
    """Advance all members to equilibrium (velocity change per step < tol and, if tol_rho > 0,
    relative change per step of the probe densities < tol_rho).  inits[i] is a density array
    or a WarmStart; either starts at physical rest (v = 0).  Returns wall seconds, steps,
    statuses and the batch (its `fallbacks` counts warm starts that fell back)."""
    b = lbm.Batch(members, tx=tx) if flags is None else lbm.Batch(members, tx=tx, flags=flags)
    b.lbm = lbm
    b.fallbacks = 0
    for i, init in enumerate(inits):
        if isinstance(init, WarmStart):
            try:
                b.init_profile(i, init.log_profile, init.r0, init.dr, init.mass)
            except lbm.LBMError:
                b.fallbacks += 1
                b.init_rest(i, init.fallback)
        else:
            b.init_rest(i, init)
        if segment is not None:
            b.set_segment(i, segment(members[i]))
    b.sync()
    t0 = time.perf_counter()
    if chunk is None:
        steps, status = b.run(tol, check_every=check_every, max_steps=max_steps,
                              tol_rho=tol_rho)
    else:
        steps, status = run_to_equilibrium(b, tol, tol_rho, check_every, max_steps, chunk,
                                           report)
    b.sync()
    return time.perf_counter() - t0, steps, status, b


def main(argv=None):
    """Time to equilibrium of the batched droplet sweep (64 lattices drawn by seed)."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--levels", type=int, default=57, help="sizes 128 + 16 k, k < levels")
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--tol-rho", type=float, default=2e-9)
    ap.add_argument("--check-every", type=int, default=500)
    ap.add_argument("--max-steps", type=int, default=1_000_000)
    ap.add_argument("--chunk", type=int, default=20_000)
    ap.add_argument("--tx", type=int, default=256, help="strip width of the batch tiles")
    ap.add_argument("--flags", type=int, default=None, help="batch launch flags")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    from . import lbm

    def say(m):
        print(m, flush=True)
        sys.stdout.flush()

    members = members_from_draw(inputs.batch_draw(a.seed, count=a.count, n_levels=a.levels))
    inits = [tanh_density(lbm, m) for m in members]
    wall, steps, status, b = run_batch(lbm, members, inits, tol=a.tol, tol_rho=a.tol_rho,
                                       check_every=a.check_every, max_steps=a.max_steps,
                                       chunk=a.chunk, report=say, tx=a.tx, flags=a.flags)
    lu = sum(m["nx"] * m["ny"] * s for m, s in zip(members, steps))
    res = {"wall_s": round(wall, 2), "lattice_updates": int(lu),
           "glups": round(lu / wall / 1e9, 2), "converged": int(sum(s == 0 for s in status)),
           "count": len(members), "max_steps": int(max(steps)),
           "nodes": int(sum(m["nx"] * m["ny"] for m in members)),
           "members": [{"n": m["nx"], "T_over_Tc": round(m["T_over_Tc"], 4),
                        "tau": round(m["tau"], 4), "collision": m["collision"],
                        "steps": int(st), "status": int(ss)}
                       for m, st, ss in zip(members, steps, status)]}
    say(json.dumps({k: v for k, v in res.items() if k != "members"}))
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh)


if __name__ == "__main__":
    main()
