"""Degenerate lattice shapes: a single node, one-node-wide columns and rows (a flat interface
across the long side, so every neighbour across the short side is the node itself), and
lattices narrower than one stencil, in every kernel, against the FP64 oracle and against each
other bit for bit, after an even and an odd number of steps."""
import numpy as np
import pytest

import oracle as O
from lbm_cases import errors, gpu_lattice, oracle_params, say
from oracle import thermo as TH

pytestmark = pytest.mark.gpu

TOL = 1e-5
SHAPES = [(1, 1), (1, 40), (40, 1), (2, 7), (7, 2), (1, 1000), (1000, 1)]
PHYSICS = [dict(T_over_Tc=0.8, K=1.0, A=-0.26, sigma=0.0, scheme="EDM", collision="BGK", tau=1.0),
           dict(T_over_Tc=0.6, K=1 / 49, A=0.0, sigma=0.125, scheme="GUO_LI", collision="MRT",
                tau=0.8)]


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_5170_amd import lbm
    return lbm


def _rho0(nx, ny, ttc):
    """Liquid in the middle half of the longer side between Maxwell densities (tanh, width 5);
    a single node or a square gets the mean density."""
    g, l, _ = TH.maxwell(ttc)
    n = max(nx, ny)
    if nx == ny:
        return np.full((ny, nx), (l + g) / 2)
    r = np.arange(n) + 0.5
    prof = (l + g) / 2 - (l - g) / 2 * np.tanh(2 * (np.abs(r - n / 2) - n / 4) / 5.0)
    return np.tile(prof[:, None], (1, nx)) if ny > nx else np.tile(prof[None, :], (ny, 1))


@pytest.mark.parametrize("phys", range(len(PHYSICS)))
@pytest.mark.parametrize("shape", SHAPES)
def test_degenerate_shapes(L, shape, phys):
    nx, ny = shape
    wl = dict(PHYSICS[phys], nx=nx, ny=ny)
    rho0 = _rho0(nx, ny, wl["T_over_Tc"])
    p = oracle_params(wl)
    for steps in (10, 11):
        fl = O.fields(p, O.step(p, O.init_feq(rho0), steps))
        pops = {}
        for name, kernel, tx, ty in (("two-step", L.LBM_KERNEL_SWEEP2, 256, 16),
                                     ("one-step", L.LBM_KERNEL_SWEEP, 64, 4),
                                     ("two-pass", L.LBM_KERNEL_TWO_PASS, 64, 4)):
            lat = gpu_lattice(L, wl, L.LBM_PREC_MIXED)
            lat.set_launch(kernel, tx, ty, 0)
            lat.init(rho0)
            lat.step(steps)
            rho_g, u_g = lat.read()
            if max(np.abs(fl["vx"]).max(), np.abs(fl["vy"]).max()) > 0:
                e_rho, e_v = errors(rho_g, u_g, fl)
            else:   # a uniform lattice stays exactly at rest
                e_rho = float(np.max(np.abs(rho_g - fl["rho"]) / fl["rho"]))
                e_v = float(np.abs(u_g).max())
            say(f"[degenerate] {nx}x{ny} {wl['scheme']}/{wl['collision']} {name} {steps} steps: "
                f"rho {e_rho:.2e} v {e_v:.2e}")
            assert e_rho < TOL and e_v < TOL
            pops[name] = lat.populations()
        assert np.array_equal(pops["two-step"], pops["one-step"])
        assert np.array_equal(pops["two-step"], pops["two-pass"])
