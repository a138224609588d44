"""Pins for the Eq. 33 effective density (Sbragaglia-Shan) in the oracle: closed forms, the
derivative, brute force of the whole step on tiny lattices, and the property Sec. 4.3.1 states
for it -- the mechanical stability condition (Eq. 18) then coincides with the Maxwell rule
(Eq. 19) -- which holds only when Eq. 18's exponent equals Eq. 33's."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import bruteforce as BF
from oracle import thermo as TH
from paper_1412_5170_amd import inputs

# (eps, G) with a van der Waals loop in p0 = rho/3 + G psi^2 / 2
CASES = [(1.0, -3.0), (0.0, -4.0), (0.5, -6.0)]


def test_ss_psi_closed_forms():
    assert float(TH.ss_psi(1.0, 0)) == pytest.approx(math.exp(-1.0), rel=1e-15)
    assert float(TH.ss_psi(0.5, 0)) == pytest.approx(math.exp(-2.0), rel=1e-15)
    assert float(TH.ss_psi(1.0, 1.0)) == pytest.approx(0.5, rel=1e-15)
    assert float(TH.ss_psi(3.0, 2.0)) == pytest.approx(math.sqrt(0.75), rel=1e-15)
    assert float(TH.ss_psi(1.0, 0.5)) == pytest.approx(0.25, rel=1e-15)


@pytest.mark.parametrize("eps", [0.0, 0.5, 1.0, 2.0])
def test_ss_dpsi_is_the_derivative(eps):
    for r in (0.03, 0.4, 2.5):
        num = mp.diff(lambda x: TH.ss_psi(x, eps), mp.mpf(r))
        assert float(TH.ss_dpsi(r, eps)) == pytest.approx(float(num), rel=1e-12)


@pytest.mark.parametrize("eps,G", CASES)
def test_mechanical_equals_maxwell_for_eq33(eps, G):
    """Sec. 4.3.1: with psi of Eq. 33 the two coexistence rules are one and the same."""
    g1, l1, p1 = TH.ss_maxwell(eps, G)
    g2, l2, p2 = TH.ss_mechanical(eps, eps, G)
    assert l1 / g1 > 5  # a genuine two-phase state
    assert g2 == pytest.approx(g1, rel=1e-12) and l2 == pytest.approx(l1, rel=1e-12)
    assert p2 == pytest.approx(p1, rel=1e-12)
    # equal pressures on both branches
    assert float(TH.ss_pressure(g1, eps, G)) == pytest.approx(p1, rel=1e-12)
    assert float(TH.ss_pressure(l1, eps, G)) == pytest.approx(p1, rel=1e-12)


@pytest.mark.parametrize("eps,G", CASES[:2])
def test_mismatched_exponent_breaks_consistency(eps, G):
    """Control: Eq. 18 with another exponent gives other densities (the identity is not an
    artefact of the solver)."""
    g1, l1, _ = TH.ss_maxwell(eps, G)
    g2, l2, _ = TH.ss_mechanical(eps + 0.5, eps, G)
    assert abs(g2 - g1) / g1 > 1e-2


@pytest.mark.parametrize("scheme,coll", [("GUO", "BGK"), ("EDM", "BGK"), ("SC", "BGK"),
                                         ("GUO", "MRT")])
@pytest.mark.parametrize("eps", [0.0, 1.0])
def test_bruteforce_step_eq33(oracle, scheme, coll, eps):
    O = oracle
    nx, ny = 4, 3
    G = -3.0 if eps else -4.0
    f = inputs.random_populations(5, nx, ny, 0.05, 1.5, 0.08)
    rates = (1.0, 1.1, 1.2, 1.0, 1.3, 1.0, 1.3, 1 / 0.8, 1 / 0.8)
    p = O.Params(nx=nx, ny=ny, T=1.0, tau=0.8, G=G, A=-eps / 2, scheme=getattr(O, scheme),
                 collision=getattr(O, coll), s=rates, psi_kind=1, psi_eps=eps)
    a = O.step(p, f, 1)
    b = BF.step(f, nx, ny, 1.0, 0.8, scheme, coll, G=G, A=-eps / 2, s=rates, ss_eps=eps)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


def test_oracle_psi_eq33(oracle):
    O = oracle
    p = O.Params(nx=1, ny=1, T=1.0, G=-3.0, psi_kind=1, psi_eps=1.0)
    assert O.psi(p, 1.0) == pytest.approx(0.5, rel=1e-15)
    p0 = O.Params(nx=1, ny=1, T=1.0, G=-4.0, psi_kind=1, psi_eps=0.0)
    assert O.psi(p0, 0.5) == pytest.approx(math.exp(-2.0), rel=1e-15)
