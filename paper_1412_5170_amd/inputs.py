"""Seeded synthetic inputs: initial density fields and parameter draws.

This module holds no arithmetic of the method (no EOS, no equilibrium, no force): the
coexistence densities a field is built from are arguments, supplied by whoever builds the
workload.  Both the HIP path and the oracle take their inputs from here.

Initial conditions (the paper states none, so these are readings):
  * slab: rho_in for y0 <= y < y1, rho_out elsewhere, a sharp step (flat interfaces of
    Sec. 4.2.1, 4.2.2);
  * droplet/bubble: rho(r) = (rho_in + rho_out)/2 - (rho_in - rho_out)/2 tanh(2 (r - R)/W),
    r measured from node (cx, cy), default (nx/2, ny/2) in 0-based node coordinates
    (static bubble of Sec. 4.2.1, 4.3.2, 4.4.2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def slab(nx: int, ny: int, y0: int, y1: int, rho_in: float, rho_out: float) -> np.ndarray:
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    return np.where((y >= y0) & (y < y1), rho_in, rho_out).astype(np.float64)


def droplet(nx: int, ny: int, R: float, W: float, rho_in: float, rho_out: float,
            cx: float | None = None, cy: float | None = None) -> np.ndarray:
    cx = nx / 2 if cx is None else cx
    cy = ny / 2 if cy is None else cy
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return (rho_in + rho_out) / 2 - (rho_in - rho_out) / 2 * np.tanh(2 * (r - R) / W)


def random_populations(seed: int, nx: int, ny: int, rho_lo: float, rho_hi: float,
                       spread: float = 0.1) -> np.ndarray:
    """Positive, non-equilibrium populations f[9, ny, nx]: a node density drawn in
    [rho_lo, rho_hi) shared out 4:1:1:1:1:1/4:1/4:1/4:1/4 (rest : axis : diagonal), each
    population perturbed by a relative uniform draw in [-spread, spread)."""
    rng = np.random.default_rng(seed)
    share = np.array([4, 1, 1, 1, 1, 0.25, 0.25, 0.25, 0.25])
    share = share / share.sum()
    rho = rng.uniform(rho_lo, rho_hi, size=(ny, nx))
    f = share[:, None, None] * rho[None] * (1 + spread * rng.uniform(-1, 1, size=(9, ny, nx)))
    return np.ascontiguousarray(f)


@dataclass
class BatchMember:
    n: int            # square lattice side
    R: float          # droplet radius
    tau: float
    T_over_Tc: float
    mrt: bool


def batch_draw(seed: int, count: int = 64, n_min: int = 128, n_step: int = 16,
               n_levels: int = 57, tau_range=(0.6, 1.5), ttc_range=(0.5, 0.9),
               radius_frac: float = 0.25) -> list[BatchMember]:
    """Independent droplet lattices for a batched sweep: side n = n_min + n_step * U{0..n_levels-1}
    (128..1024 by default), R = radius_frac * n, tau ~ U(tau_range), T/Tc ~ U(ttc_range),
    BGK or MRT with probability 1/2 each."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(n_min + n_step * rng.integers(0, n_levels))
        out.append(BatchMember(n=n, R=radius_frac * n, tau=float(rng.uniform(*tau_range)),
                               T_over_Tc=float(rng.uniform(*ttc_range)),
                               mrt=bool(rng.integers(0, 2))))
    return out


# Named workloads (physics as stated for each; coexistence densities supplied at build time).
WORKLOADS = {
    "slab_4x256_edm": dict(nx=4, ny=256, init="slab", y0=64, y1=192, T_over_Tc=0.8, K=1.0,
                           A=-0.26, sigma=0.0, scheme="EDM", collision="BGK", tau=1.0),
    "droplet_512_li": dict(nx=512, ny=512, init="droplet", R=80.0, W=5.0, T_over_Tc=0.6,
                           K=1 / 49, A=0.0, sigma=0.125, scheme="GUO_LI", collision="BGK",
                           tau=1.0),
    "droplet_4096_mrt": dict(nx=4096, ny=4096, init="droplet", R=600.0, W=5.0, T_over_Tc=0.5,
                             K=1 / 49, A=0.0, sigma=0.125, scheme="GUO_LI", collision="MRT",
                             tau=1.0, s=(1.0, 1.1, 1.1, 1.0, 1.1, 1.0, 1.1, 1.0, 1.0)),
}


def initial_density(wl: dict, rho_l: float, rho_g: float) -> np.ndarray:
    if wl["init"] == "slab":
        return slab(wl["nx"], wl["ny"], wl["y0"], wl["y1"], rho_l, rho_g)
    return droplet(wl["nx"], wl["ny"], wl["R"], wl["W"], rho_l, rho_g)
