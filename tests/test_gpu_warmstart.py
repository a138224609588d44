"""Warm-start initial states on the device (lbm_batch_init_rest, lbm_batch_init_profile)
against the oracle of the rest state, the profile expansion and the mass matching; error
paths; the bound on the gain (a lattice started at rest from its own equilibrium density needs
far fewer steps than the tanh start and reaches the same density ratio, and so, to a lesser
degree, does the mass-matched radial profile of that equilibrium); and the gain of the trained
network itself on lattices of the batched sweep's distribution, against the tanh start and
against a constant profile."""
import oracle
from oracle import thermo as TH
import numpy as np
import pytest

from lbm_cases import say
from oracle import profile as oprof
from paper_1412_5170_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1412_5170_amd import lbm
    return lbm


def _member(nx, ny, **kw):
    m = dict(nx=nx, ny=ny, T_over_Tc=0.7, K=1 / 49, scheme="GUO_LI", sigma=0.125,
             collision="BGK", tau=1.0)
    m.update(kw)
    return m


def _oracle_params(m):
    return oracle.Params(nx=m["nx"], ny=m["ny"], T=m["T_over_Tc"] * TH.critical_point()[1],
                         K=m["K"], scheme=oracle.GUO_LI, sigma=m["sigma"], tau=m["tau"])


H = 1.5  # profile spacing


def _profile(R, inner=0.35, outer=0.02, width=4.0):
    r = R + H * (np.arange(64) - 31.5)
    return np.log(outer + (inner - outer) * 0.5 * (1 - np.tanh((r - R) / width)))


@pytest.mark.parametrize("nx,ny,R,shift", [(130, 96, 30.0, 0.0), (64, 200, 20.0, 3.7),
                                           (5, 3, 1.0, 0.0)])
def test_profile_init_matches_oracle(L, nx, ny, R, shift):
    say(f"profile init {nx}x{ny} R={R} shift={shift}")
    m = _member(nx, ny)
    prof = _profile(R)
    r0 = R - 31.5 * H
    b = L.Batch([m])
    mass = oprof.density(nx, ny, prof, r0, H, shift).sum() if shift else 0.0
    s = b.init_profile(0, prof, r0, H, mass)
    if not shift:
        assert s == 0.0
    else:
        assert abs(s - shift) < 1e-9
    f = b.populations(0).astype(np.float64)
    rho_ref = oprof.density(nx, ny, prof, r0, H, s)
    ref = oprof.rest_populations(_oracle_params(m), rho_ref)
    # FP32 storage, and a force from the FP32-rounded rest populations
    assert np.max(np.abs(f - ref) / ref) < 1e-6
    rho, v = b.read(0)
    assert np.max(np.abs(rho - rho_ref) / rho_ref) < 1e-6
    assert np.max(np.abs(v)) < 1e-6
    st = b.stats()[0]
    if mass:
        assert abs(st["mass"] - mass) / mass < 1e-6
    assert b.steps(0) == 0


def test_profile_init_errors(L):
    b = L.Batch([_member(64, 64)])
    flat = np.log(np.full(64, 0.1))
    with pytest.raises(L.LBMError) as e:
        b.init_profile(0, flat, 0.0, H, 2 * 0.1 * 64 * 64)  # no shift changes a uniform mass
    assert e.value.code == L.LBM_EINVAL
    bad = _profile(16.0)
    bad[5] = np.nan
    with pytest.raises(L.LBMError) as e:
        b.init_profile(0, bad, 0.0, H)
    assert e.value.code == L.LBM_EINVAL
    dense = np.log(np.full(64, 1.2))  # above the packing limit 4/b = 1
    with pytest.raises(L.LBMError) as e:
        b.init_profile(0, dense, 0.0, H)
    assert e.value.code == L.LBM_EUNSTABLE
    with pytest.raises(L.LBMError) as e:
        b.init_profile(0, _profile(16.0), 0.0, 0.0)  # spacing must be positive
    assert e.value.code == L.LBM_EINVAL
    assert b.stats()[0]["step"] == 0  # a rejected profile leaves the lattice uninitialised


def test_rest_state_matches_oracle(L):
    m = _member(96, 80)
    g, l, _ = TH.maxwell(0.7)
    rho0 = inputs.droplet(96, 80, 20.0, 5.0, l, g)
    b = L.Batch([m])
    b.init_rest(0, rho0)
    f = b.populations(0).astype(np.float64)
    ref = oprof.rest_populations(_oracle_params(m), rho0)
    assert np.max(np.abs(f - ref) / ref) < 1e-6
    rho, v = b.read(0)
    assert np.max(np.abs(v)) < 1e-6


def test_equilibrium_profile_start_gain(L):
    """The bound on any learned start.  From the droplet's own equilibrium density at physical
    rest: at most half the steps of the tanh start, same density ratio.  From the mass-matched
    radial profile of that equilibrium (64 samples along +x, centred on the interface): fewer
    steps, same ratio."""
    from paper_1412_5170_amd import sweep
    m = dict(sweep.PHYSICS, nx=128, ny=128, T_over_Tc=0.7, tau=1.0, collision="BGK", R=32.0)
    plain = sweep.tanh_density(L, m)
    run = dict(tol=1e-9, tol_rho=2e-9, check_every=500, max_steps=200_000)
    w0, s0, st0, b0 = sweep.run_batch(L, [m], [plain], **run)
    assert st0 == [0]
    rho0, _ = b0.read(0)
    ratio0 = rho0[64, 64] / rho0[0, 0]
    w1, s1, st1, b1 = sweep.run_batch(L, [m], [rho0], **run)
    rho1, _ = b1.read(0)
    ratio1 = rho1[64, 64] / rho1[0, 0]
    prof = sweep.radial_profile(m, rho0)
    w2, s2, st2, b2 = sweep.run_batch(L, [m], [sweep.WarmStart(prof, m["R"], plain.sum(), plain)],
                                      **run)
    rho2, _ = b2.read(0)
    ratio2 = rho2[64, 64] / rho2[0, 0]
    say(f"warm start gain: steps tanh {s0[0]}, exact rest {s1[0]}, profile {s2[0]}; "
        f"ratio {ratio0:.8g} / {ratio1:.8g} / {ratio2:.8g}")
    assert st1 == [0] and st2 == [0] and b2.fallbacks == 0
    assert s1[0] <= s0[0] // 2
    assert s2[0] < s0[0]
    assert abs(ratio1 - ratio0) / ratio0 < 1e-4
    assert abs(ratio2 - ratio0) / ratio0 < 1e-4


def test_trained_network_gain(L):
    """The committed network (weights-only file) as the initial state of eight lattices drawn
    like the batched sweep (sizes 128^2-320^2, R = n/4, tau in [0.6, 1.5], T/Tc in [0.5, 0.9],
    BGK or MRT, Guo + Li, K = 1/49), against the plain tanh start and against a constant
    profile (the network's mean output, the same for every lattice, mass-matched the same way).
    Each start runs under a stopping rule 4x tighter than the sweep's, recording the probe
    density ratio every 500 steps; the converged ratio of a lattice is the mean of the tanh and
    learned end points, and a start's cost is the lattice updates until its ratio stays within
    1e-4 of it.  The network must reach that band with at most 0.6x the tanh start's updates,
    and the constant profile must not do as well as the network."""
    from paper_1412_5170_amd import sweep, warmstart as WS
    members = sweep.members_from_draw(inputs.batch_draw(5, count=8, n_levels=13))
    sur = WS.load_surrogate(L)
    rule = dict(tol=2.5e-10, tol_rho=5e-10, check_every=500, max_steps=1_500_000)
    starts = {"tanh": WS._start(L, sur, members, "tanh"),
              "learned": WS._start(L, sur, members, "learned")}
    assert all(isinstance(w, sweep.WarmStart) for w in starts["learned"])
    const = []
    for m, w in zip(members, starts["learned"]):
        const.append(sweep.WarmStart(sur.mean.astype(np.float64), m["R"], w.mass, w.fallback))
    starts["constant"] = const
    hist, fin = {}, {}
    for mode, inits in starts.items():
        hist[mode], fin[mode] = WS.trajectories(L, members, inits, label=mode, **rule)
    ref = [(a + b) / 2 for a, b in zip(fin["tanh"], fin["learned"])]
    spread = max(abs(a - b) / r for a, b, r in zip(fin["tanh"], fin["learned"], ref))
    cost = {}
    for mode in starts:
        steps = [WS.time_to_accuracy(h, r, 1e-4) for h, r in zip(hist[mode], ref)]
        cost[mode] = sum(m["nx"] * m["ny"] * st for m, st in zip(members, steps))
        say(f"trained network gain: {mode} steps {steps}, {cost[mode] / 1e9:.2f} G updates")
    say(f"    learned / tanh {cost['learned'] / cost['tanh']:.3f}, constant / tanh "
        f"{cost['constant'] / cost['tanh']:.3f}; end-point spread {spread:.1e}")
    assert spread < 1e-4
    assert cost["learned"] <= 0.6 * cost["tanh"]
    assert cost["constant"] > cost["learned"]
