"""Equilibrium parity: after 10,000 (flat slab, EDM) and 20,000 (512 x 512 Li droplet) steps
the GPU state (FP32 populations, default mixed arithmetic) matches the FP64 oracle within 1e-4
relative in rho everywhere and in the coexistence (probe) densities.  The slab's oracle runs
here; the droplet's comes from tests/golden/droplet_512_li_20k.npz, written by
tests/golden/make_droplet_equilibria.py, which calls only oracle/."""
import os

import numpy as np
import pytest

import oracle as O
from lbm_cases import gpu_lattice, initial_density, oracle_params, say, workload

pytestmark = pytest.mark.gpu

TOL = 1e-4
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "droplet_512_li_20k.npz")


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1412_5170_amd import lbm
    return lbm


def test_flat_interface_10k_steps(L):
    wl = workload("slab_4x256_edm")
    say("[equilibrium] slab 4x256 EDM T/Tc 0.8, 10000 steps")
    rho0 = initial_density(wl)
    p = oracle_params(wl)
    fl = O.fields(p, O.step(p, O.init_feq(rho0), 10_000))
    lat = gpu_lattice(L, wl, L.LBM_PREC_MIXED)
    lat.init(rho0)
    lat.step(10_000)
    rho, v = lat.read()
    e = np.max(np.abs(rho - fl["rho"]) / fl["rho"])
    rl, rg = rho[wl["ny"] // 2, 0], rho[0, 0]
    ol, og = fl["rho"][wl["ny"] // 2, 0], fl["rho"][0, 0]
    say(f"    max rel rho {e:.2e}; rho_l {rl:.8f} vs {ol:.8f}; rho_g {rg:.8f} vs {og:.8f}")
    assert e < TOL
    assert abs(rl - ol) / ol < TOL and abs(rg - og) / og < TOL
    # the flat interface has no tangential velocity (exact zero in the oracle)
    assert np.max(np.abs(v[..., 0])) < 1e-6


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden file not generated")
@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_li_droplet_20k_steps(L, tau):
    g = np.load(GOLDEN)
    steps, stride = int(g["steps"]), int(g["stride"])
    wl = workload("droplet_512_li", tau=tau)
    say(f"[equilibrium] droplet 512 Li tau {tau}, {steps} steps")
    lat = gpu_lattice(L, wl, L.LBM_PREC_MIXED)
    lat.init(initial_density(wl))
    lat.step(steps)
    rho, v = lat.read()
    key = f"tau{tau}"
    ref = g[key + "_rho"]
    e = np.max(np.abs(rho[::stride, ::stride] - ref) / ref)
    rc, ro = rho[wl["ny"] // 2, wl["nx"] // 2], rho[0, 0]
    oc, oo = float(g[key + "_rho_centre"]), float(g[key + "_rho_corner"])
    say(f"    max rel rho (sampled) {e:.2e}; centre {rc:.8f} vs {oc:.8f}; corner {ro:.8f} vs "
        f"{oo:.8f}")
    assert e < TOL
    assert abs(rc - oc) / oc < TOL and abs(ro - oo) / oo < TOL
