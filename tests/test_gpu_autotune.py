"""Autotuner: trials leave the simulation exactly where it was, the chosen launch is one of
the candidates, the JSON-lines cache is written and reused, and a tuned run is bitwise equal
to an untuned one (every launch shape computes the same bits)."""
import json

import numpy as np
import pytest

from lbm_cases import say
from oracle import thermo as TH
from paper_1412_5170_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1412_5170_amd import lbm
    return lbm


def _lattice(L, nx, ny):
    lat = L.Lattice(nx, ny, L.make_eos(0.6, K=1 / 49), L.make_force("GUO_LI", sigma=0.125),
                    L.make_collision("MRT"), 0.9)
    g, l, _ = TH.maxwell(0.6)
    lat.init(inputs.droplet(nx, ny, min(nx, ny) / 4, 5.0, l, g))
    return lat


def test_single_autotune_restores_state_and_caches(L, tmp_path):
    say("autotune single 256x130")
    cache = tmp_path / "tune.jsonl"
    a, b = _lattice(L, 256, 130), _lattice(L, 256, 130)
    a.step(10)
    b.step(10)
    before = a.populations()
    ms = a.autotune(str(cache), trial_steps=4)
    assert ms > 0
    assert np.array_equal(a.populations(), before)
    assert a.stats()["step"] == 10
    k, tx, ty, fl = a.get_launch()
    assert ((k == L.LBM_KERNEL_SWEEP and tx in (64, 128, 256, 512) and ty in (4, 8, 16, 32, 64))
            or (k == L.LBM_KERNEL_SWEEP2 and tx in (64, 128, 256) and ty in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32)))
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert "256x130" in rec["key"] and rec["value"] == f"{k} {tx} {ty} {fl}"
    a.step(10)
    b.step(10)
    assert np.array_equal(a.populations(), b.populations())
    # a second handle of the same problem takes the cached choice without trials
    c = _lattice(L, 256, 130)
    assert c.autotune(str(cache), trial_steps=4) == -1.0
    assert c.get_launch() == (k, tx, ty, fl)
    assert len(cache.read_text().splitlines()) == 1


def test_autotune_planes_beyond_4gib_times_two_pass_shapes(L):
    """A planes-layout lattice beyond 4 GiB per population buffer runs only the two-pass step:
    the autotuner times two-pass shapes there and keeps one of them, and the step count is
    left as it was."""
    import torch
    n = 10944  # 9 x 4 x 10944^2 B = 4.31 GB per buffer
    say(f"autotune planes {n}x{n}")
    lat = L.Lattice(n, n, L.make_eos(0.6, K=1 / 49), L.make_force("GUO_LI", sigma=0.125),
                    L.make_collision("MRT"), 0.9, layout=L.LBM_LAYOUT_PLANES)
    assert lat.get_launch()[0] == L.LBM_KERNEL_TWO_PASS
    g, l, _ = TH.maxwell(0.6)
    rho0 = np.full((n, n), l)  # uniform: stays uniform, no interface to resolve
    lat.init(rho0)
    del rho0
    lat.step(2)
    assert lat.autotune(None, trial_steps=2) > 0
    k, tx, ty, fl = lat.get_launch()
    assert k == L.LBM_KERNEL_TWO_PASS and tx in (64, 128, 256) and ty in (2, 4, 8)
    assert fl == L.LBM_LAUNCH_XCD_ORDER
    assert lat.stats()["step"] == 2
    del lat
    torch.cuda.empty_cache()


def test_batch_autotune_restores_state(L, tmp_path):
    say("autotune batch")
    members = [dict(nx=n, ny=n, T_over_Tc=0.7, K=1 / 49, scheme="GUO_LI", sigma=0.125,
                    collision=c, tau=1.0) for n, c in ((96, "BGK"), (160, "MRT"), (200, "BGK"))]

    def make():
        bt = L.Batch(members)
        for i, m in enumerate(members):
            g, l, _ = TH.maxwell(m["T_over_Tc"])
            bt.init(i, inputs.droplet(m["nx"], m["ny"], m["nx"] / 4, 5.0, l, g))
        return bt

    a, b = make(), make()
    a.step(10)
    b.step(10)
    a.set_active(1, 0)
    b.set_active(1, 0)
    before = [a.populations(i) for i in range(3)]
    cache = tmp_path / "batch.jsonl"
    ms = a.autotune(str(cache), trial_steps=4)
    assert ms > 0
    for i in range(3):
        assert np.array_equal(a.populations(i), before[i])
    assert [a.steps(i) for i in range(3)] == [10, 10, 10]
    a.step(10)
    b.step(10)
    assert [a.steps(i) for i in range(3)] == [20, 10, 20]  # lattice 1 stayed inactive
    for i in range(3):
        assert np.array_equal(a.populations(i), b.populations(i))
    assert make().autotune(str(cache), trial_steps=4) == -1.0


def test_kernel_timing_folds_long_runs(L):
    """Kernel timing over more timed units than one fold (1024): the sweep is timed per
    lbm_step call (1100 calls of 2 steps), the two-pass step per step (1100 steps); every step
    is counted once, the sums are positive, reading resets them, and timing does not change
    the state."""
    say("[timing] 96x80, 1100 sweep calls of 2 steps, 1100 two-pass steps")
    lat = _lattice(L, 96, 80)
    ref = _lattice(L, 96, 80)
    lat.timing_enable(True)
    lat.timing()
    for _ in range(1100):
        lat.step(2)
    a, b, steps = lat.timing()
    assert steps == 2200 and b > 0 and a >= 0
    assert lat.timing()[2] == 0
    lat.set_launch(L.LBM_KERNEL_TWO_PASS, 128, 2, L.LBM_LAUNCH_XCD_ORDER)
    lat.step(1100)
    a2, b2, steps2 = lat.timing()
    lat.timing_enable(False)
    assert steps2 == 1100 and a2 > 0 and b2 > 0
    ref.step(3300)
    assert np.array_equal(lat.populations(), ref.populations())
