"""Host-side logic of the batched sweep and the warm start (no GPU), and the oracle of the
warm-start initial state (radial profile to lattice, mass matching) pinned to geometry."""
import math

import numpy as np
import pytest

from oracle import profile as oprof
from paper_1412_5170_amd import inputs, sweep, warmstart


def _member(n=160, R=40.0):
    return dict(sweep.PHYSICS, nx=n, ny=n, R=R, T_over_Tc=0.6, tau=1.0, collision="BGK")


def test_profile_radii_span_the_interface():
    """Uniform radii with the interface radius between points 23 and 24, from 47 nodes inside
    it to 79 outside (the vapour side reaches its plateau further out)."""
    r = sweep.profile_radii(40.0)
    assert len(r) == sweep.PROFILE_POINTS == oprof.POINTS == 64
    assert np.allclose(np.diff(r), sweep.PROFILE_SPACING)
    assert (r[23] + r[24]) / 2 == pytest.approx(40.0)
    assert r[0] == pytest.approx(40.0 - 47.0) and r[-1] == pytest.approx(40.0 + 79.0)
    assert np.array_equal(r, oprof.radii(r[0], sweep.PROFILE_SPACING))


def test_profile_round_trip():
    """A smooth radial profile expanded to the lattice and sampled back along +x is itself."""
    m = _member()
    r = sweep.profile_radii(m["R"])
    prof = np.log(0.2 + 0.19 * np.tanh((38.0 - r) / 6.0))
    rho = oprof.density(m["nx"], m["ny"], prof, r[0], sweep.PROFILE_SPACING)
    back = sweep.radial_profile(m, rho)
    # two linear interpolations (profile to lattice, lattice to profile) of a steep log profile
    assert np.max(np.abs(back - prof)) < 2e-2
    assert np.median(np.abs(back - prof)) < 1e-3


def test_profile_is_rest_equilibrium():
    prof = np.log(np.linspace(0.3, 0.01, 64))
    f = oprof.populations(40, 30, prof, 2.0, 0.25)
    rho = oprof.density(40, 30, prof, 2.0, 0.25)
    assert np.allclose(f.sum(axis=0), rho, rtol=1e-15)
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
    assert np.abs(np.tensordot(ex, f, 1)).max() < 1e-17
    assert np.abs(np.tensordot(ey, f, 1)).max() < 1e-17


def test_profile_ends_are_held():
    """Nodes inside the first radius take the first value, nodes beyond the last the last."""
    prof = np.log(np.linspace(0.4, 0.02, 64))
    rho = oprof.density(64, 64, prof, 5.0, 0.25, shift=2.0)   # radii 7 .. 22.75 after the shift
    assert math.isclose(rho[32, 32], 0.4, rel_tol=1e-15)
    assert math.isclose(rho[0, 0], 0.02, rel_tol=1e-15)


def test_mass_match_disk_closed_form():
    """A sharp disk (rho_l inside radius a, rho_g outside) holds about
    rho_g N + (rho_l - rho_g) pi a^2: the matched shift follows that area law."""
    n = 256
    r = sweep.profile_radii(60.0)
    rl, rg = 0.4, 0.01
    prof = np.log(np.where(r < 60.0, rl, rg))
    for a in (50.0, 60.0, 75.0):
        mass = rg * n * n + (rl - rg) * math.pi * a * a
        s = oprof.mass_matched_shift(n, n, prof, r[0], sweep.PROFILE_SPACING, mass)
        assert s is not None
        assert abs((60.0 + s) - a) < 0.6  # lattice count of a disk vs its area, step width


def test_mass_match_is_exact_and_monotone():
    m = _member()
    r = sweep.profile_radii(m["R"])
    h = sweep.PROFILE_SPACING
    prof = np.log(0.2 + 0.19 * np.tanh((40.0 - r) / 4.0))
    d = lambda s: oprof.density(m["nx"], m["ny"], prof, r[0], h, s).sum()
    base = d(0.0)
    for target in (0.9 * base, base, 1.2 * base):
        s = oprof.mass_matched_shift(m["nx"], m["ny"], prof, r[0], h, target)
        assert s is not None
        assert abs(d(s) - target) <= 1e-12 * target
    # moving a droplet's interface outwards (dense inside) raises its mass
    assert d(2.0) > base > d(-2.0)


def test_mass_match_unreachable_is_none():
    prof = np.log(np.full(64, 0.1))  # uniform: no shift changes the mass
    assert oprof.mass_matched_shift(160, 160, prof, 10.0, 1.5, 2.0 * 0.1 * 160 * 160) is None


def test_features_span_unit_box():
    ms = warmstart.draw_training(3, 256)
    X = np.stack([warmstart.features(m) for m in ms])
    assert X.shape == (256, 4) and X.dtype == np.float32
    assert np.all(np.abs(X) <= 1.0 + 1e-6)
    # the curvature feature stays bounded for the largest droplets of the sweep
    big = dict(ms[0], R=256.0)
    assert -1.0 <= warmstart.features(big)[2] <= 0.0
    assert all(warmstart.K_RANGE[0] <= m["K"] <= warmstart.K_RANGE[1] for m in ms)


def test_batch_draw_seeded_and_in_range():
    a = inputs.batch_draw(5, count=64)
    b = inputs.batch_draw(5, count=64)
    assert a == b
    for d in a:
        assert 128 <= d.n <= 128 + 16 * 56 and (d.n - 128) % 16 == 0
        assert 0.5 <= d.T_over_Tc <= 0.9 and 0.6 <= d.tau <= 1.5
        assert math.isclose(d.R, d.n / 4) or d.R <= d.n / 2


def test_rest_populations_have_zero_fluid_velocity():
    """The rest state keeps the density and makes v = u + F/(2 rho) vanish, while F itself is
    far from zero across the interface (a sign slip would leave v = -F / rho)."""
    import oracle
    from oracle import thermo as TH
    nx = ny = 48
    g, l, _ = TH.maxwell(0.7)
    rho = inputs.droplet(nx, ny, 12.0, 5.0, l, g)
    p = oracle.Params(nx=nx, ny=ny, T=0.7 * TH.critical_point()[1], K=1 / 49,
                      scheme=oracle.GUO_LI, sigma=0.125, tau=1.0)
    f = oprof.rest_populations(p, rho)
    fl = oracle.fields(p, f)
    assert np.allclose(fl["rho"], rho, rtol=1e-14, atol=0)
    F = np.hypot(fl["Fx"], fl["Fy"]) / (2 * rho)
    assert F.max() > 1e-4
    assert np.abs(fl["vx"]).max() < 1e-15 and np.abs(fl["vy"]).max() < 1e-15


def test_time_to_accuracy_is_the_last_entry_into_the_band():
    h = [(100, 1.2), (200, 1.00005), (300, 1.0003), (400, 1.00002), (500, 0.99999)]
    assert warmstart.time_to_accuracy(h, 1.0, 1e-4) == 400
    assert warmstart.time_to_accuracy(h, 1.0, 1e-3) == 200
    assert warmstart.time_to_accuracy(h, 1.0, 1e-6) == 500  # never inside: the last step
