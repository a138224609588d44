"""Shared set-up for the GPU parity tests: one workload description drives both the oracle
and the HIP path, from the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle as O
from oracle import thermo as TH
from paper_1412_5170_amd import inputs

MRT_RATES = (1.0, 1.1, 1.1, 1.0, 1.1)          # s_rho, s_e, s_eps, s_j, s_q of the droplet configs


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def workload(name, **over):
    wl = dict(inputs.WORKLOADS[name])
    wl.update(over)
    return wl


def oracle_params(wl):
    tau = wl["tau"]
    s5 = wl.get("s5", MRT_RATES)
    s = (s5[0], s5[1], s5[2], s5[3], s5[4], s5[3], s5[4], 1 / tau, 1 / tau)
    return O.Params(nx=wl["nx"], ny=wl["ny"], T=TH.temperature(wl["T_over_Tc"]), tau=tau,
                    scheme=getattr(O, wl["scheme"]), collision=getattr(O, wl["collision"]),
                    K=wl["K"], A=wl["A"], sigma=wl["sigma"], s=s)


def gpu_lattice(L, wl, precision, tile=None, layout=1):
    eos = L.make_eos(wl["T_over_Tc"], K=wl["K"])
    force = L.make_force(wl["scheme"], A=wl["A"], sigma=wl["sigma"])
    coll = L.make_collision(wl["collision"], s=wl.get("s5", MRT_RATES))
    return L.Lattice(wl["nx"], wl["ny"], eos, force, coll, wl["tau"], precision=precision,
                     tile=tile, layout=layout)


def initial_density(wl):
    g, l, _ = TH.maxwell(wl["T_over_Tc"])
    return inputs.initial_density(wl, l, g)


def errors(rho_g, u_g, fl):
    """Max pointwise relative error in rho; norm-wise max |v_gpu - v_ref| / max |v_ref|."""
    rho_o = fl["rho"]
    e_rho = float(np.max(np.abs(rho_g - rho_o) / rho_o))
    dv = max(np.abs(u_g[..., 0] - fl["vx"]).max(), np.abs(u_g[..., 1] - fl["vy"]).max())
    vref = max(np.abs(fl["vx"]).max(), np.abs(fl["vy"]).max())
    return e_rho, float(dv / vref)
