"""The paper's numerical claims (Sec. 4), reproduced by batched runs on the GPU and checked
against what the paper states or prints (tests/golden/paper_tables.json holds the printed
table values).  The paper gives neither step counts, initial states nor boundary conditions,
so the printed values pin loosely; its qualitative statements pin strictly."""
import json
import os

import numpy as np
import pytest

from lbm_cases import say

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1412_5170_amd import lbm
    return lbm


@pytest.fixture(scope="module")
def S():
    from paper_1412_5170_amd import studies
    return studies


def test_tau_dependence_of_force_schemes(L, S):
    """Sec. 4.2.1 / Fig. 2 (Table 2: A = -0.26, K = 1): on a flat interface the SC gas density
    grows with tau, EDM and Guo do not move, and SC equals EDM at tau = 1."""
    say("[studies] tau sweep")
    res = S.tau_sweep(L, taus=(0.8, 1.0, 1.5))
    by = {(r["scheme"], r["tau"]): r for r in res}
    for r in res:
        assert r["status"] == 0, r
    sc = [by[("SC", t)]["rho_g"] for t in (0.8, 1.0, 1.5)]
    assert sc[0] < sc[1] < sc[2] and sc[2] / sc[0] > 1.5
    for scheme in ("EDM", "GUO"):
        g = np.array([by[(scheme, t)]["rho_g"] for t in (0.8, 1.0, 1.5)])
        assert np.ptp(g) / g.mean() < 1e-4, (scheme, g)
    assert by[("SC", 1.0)]["rho_g"] == pytest.approx(by[("EDM", 1.0)]["rho_g"], rel=1e-5)


def test_guo_follows_the_mechanical_solution(L, S):
    """Sec. 4.2.2 / Fig. 5 (eps = 0.52, A = -0.26): Guo's gas density sits on the mechanical
    solution (Eq. 18), EDM's does not; Sec. 4.3.1 / Fig. 6 (eps = 1.68): at T/Tc = 0.6 Li's
    model is closer to it than the modified Kupershtokh model; Table 6: the latter's gas
    densities at K = 1 and K = 0.1."""
    say("[studies] coexistence subset")
    members = [S.slab_member(0.9, "EDM", A=-0.26, eps=0.52),
               S.slab_member(0.9, "GUO", A=-0.26, eps=0.52),
               S.slab_member(0.6, "GUO", A=-0.84, eps=1.68),
               S.slab_member(0.6, "GUO_LI", sigma=0.105, eps=1.68),
               S.slab_member(0.6, "GUO", A=-1.0, K=0.1, eps=2.0)]
    res = S.run(L, members)
    for r in res:
        assert r["status"] == 0, r
        e, f = S._eos(L, r), S._force(L, r)
        r["mech_g"], _ = L.coexistence(e, f, "mechanical", r["eps"])
    edm, guo, kup, li, kup01 = res
    assert abs(guo["rho_g"] - guo["mech_g"]) / guo["mech_g"] < 1e-3
    assert abs(edm["rho_g"] - edm["mech_g"]) > 20 * abs(guo["rho_g"] - guo["mech_g"])
    assert abs(li["rho_g"] - li["mech_g"]) < abs(kup["rho_g"] - kup["mech_g"])
    t6 = GOLDEN["table6"]
    assert kup["rho_g"] == pytest.approx(t6["simulation_K1_eps1.68"], rel=0.03)
    assert kup01["rho_g"] == pytest.approx(t6["simulation_K0.1_eps2"], rel=0.03)


def test_bubble_tables_4_and_5(L, S):
    """Tables 4 and 5 (100 x 100 box, bubble of radius 23, T = 0.6 Tc): gas density and peak
    spurious velocity of the modified Kupershtokh and Li models against the printed values."""
    say("[studies] bubbles, Tables 4 and 5")
    members = [dict(S.bubble_member("GUO", A=-0.84, tau=t), table=4) for t in (0.8, 1.0, 1.5)]
    members += [dict(S.bubble_member("GUO_LI", sigma=0.105, tau=t), table=5) for t in (0.8, 1.0)]
    res = S.run(L, members, tol=1e-9, tol_rho=1e-9, check_every=500, max_steps=300_000)
    gold = {(4, r["tau"]): r for r in GOLDEN["table4"]}
    gold.update({(5, r["tau"]): r for r in GOLDEN["table5"]})
    for r in res:
        assert r["status"] == 0, r
        g = gold[(r["table"], r["tau"])]
        say(f"    table {r['table']} tau {r['tau']}: rho_g {r['rho_g']:.6f} (paper "
            f"{g['rho_g']}), Us {r['us_max']:.4f} ({g['us_max']}), rho_l {r['rho_l']:.5f} "
            f"({g['rho_l']})")
        assert r["rho_g"] == pytest.approx(g["rho_g"], rel=0.06)
        assert r["us_max"] == pytest.approx(g["us_max"], rel=0.15)
        assert r["rho_l"] == pytest.approx(g["rho_l"], rel=0.006)
    # Table 4's trend: the gas density falls from tau = 0.8 to tau = 1 (0.0047 -> 0.0043)
    assert res[0]["rho_g"] > res[1]["rho_g"]
    # Table 5's trend: Li's gas density rises with tau
    assert res[3]["rho_g"] < res[4]["rho_g"]


def test_bubble_table_7_mrt(L, S):
    """Table 7 (Sec. 4.4.2: the Table 4 bubble under MRT, tau_nu = 0.7, 1, 1.5) with the EOS scale
    and the free rates the text leaves out taken as K = 0.5 and s_e = s_eps = s_q = 1: gas
    density, peak spurious velocity and liquid density against the printed values, and the
    section's claims that MRT shrinks tau's effect on the gas density and the spurious velocities
    against BGK at the same parameters."""
    say("[studies] bubbles, Table 7")
    mrt = [dict(S.bubble_member("GUO", A=-0.84, K=S.TABLE7_K, tau=t, collision="MRT"),
                s=S.TABLE7_RATES) for t in (0.7, 1.0, 1.5)]
    bgk = [S.bubble_member("GUO", A=-0.84, K=S.TABLE7_K, tau=t) for t in (0.7, 1.0, 1.5)]
    res = S.run(L, mrt + bgk, tol=1e-9, tol_rho=1e-9, check_every=500, max_steps=300_000)
    for r in res:
        assert r["status"] == 0, r
    m, b = res[:3], res[3:]
    for r, g in zip(m, GOLDEN["table7"]):
        say(f"    table 7 tau {r['tau']}: rho_g {r['rho_g']:.6f} (paper {g['rho_g']}), Us "
            f"{r['us_max']:.4f} ({g['us_max']}), rho_l {r['rho_l']:.5f} ({g['rho_l']})")
        assert r["rho_g"] == pytest.approx(g["rho_g"], rel=0.05)
        assert r["us_max"] == pytest.approx(g["us_max"], rel=0.15)
        assert r["rho_l"] == pytest.approx(g["rho_l"], rel=0.006)
    # the gas density falls with tau_nu, as printed, over less than half BGK's range
    gm, gb = [r["rho_g"] for r in m], [r["rho_g"] for r in b]
    assert gm[0] > gm[1] > gm[2]
    assert gm[0] - gm[2] < 0.5 * (gb[0] - gb[2])
    # smaller spurious velocities away from tau = 1, where the two collisions coincide
    assert m[0]["us_max"] < 0.5 * b[0]["us_max"] and m[2]["us_max"] < 0.75 * b[2]["us_max"]
    assert m[1]["rho_g"] == pytest.approx(b[1]["rho_g"], rel=1e-6)


def test_eq33_flat_interface_is_thermodynamically_consistent(L, S):
    """Sec. 4.3.1: with psi of Eq. 33 and A = -eps/2 (Eq. 18 identical to Eq. 19) a flat
    interface settles at the Maxwell densities of the implied EOS, up to the higher-order
    pressure-tensor error, which grows as the interface thins; tau does not enter."""
    say("[studies] eq33")
    res = S.eq33(L, cases=((1.0, -2.6), (1.0, -2.8)))
    dev = {}
    for r in res:
        assert r["status"] == 0, r
        dg = abs(r["rho_g"] - r["maxwell_g"]) / r["maxwell_g"]
        dl = abs(r["rho_l"] - r["maxwell_l"]) / r["maxwell_l"]
        say(f"    G {r['G']} tau {r['tau']}: rho_g {r['rho_g']:.5f} (Maxwell "
            f"{r['maxwell_g']:.5f}), rho_l {r['rho_l']:.4f} ({r['maxwell_l']:.4f})")
        dev[(r["G"], r["tau"])] = (r["rho_g"], dg, dl)
    assert dev[(-2.6, 1.0)][1] < 0.01 and dev[(-2.6, 1.0)][2] < 0.002
    assert dev[(-2.8, 1.0)][1] > dev[(-2.6, 1.0)][1]
    for G in (-2.6, -2.8):
        assert dev[(G, 1.0)][0] == pytest.approx(dev[(G, 0.8)][0], rel=1e-4)
