"""Checkpoint and restart: a run saved and reloaded continues bitwise as the uninterrupted
run; a checkpoint does not load into a lattice of another size or other parameters.  The
batch's plain tanh start matches the same field set at rest from the host."""
import numpy as np
import pytest

from lbm_cases import gpu_lattice, initial_density, say, workload
from paper_1412_5170_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1412_5170_amd import lbm
    return lbm


def test_save_load_continues_bitwise(L, tmp_path):
    wl = workload("droplet_512_li", nx=200, ny=150, R=40.0)
    say("[checkpoint] 200x150 Li droplet")
    a, b = gpu_lattice(L, wl, L.LBM_PREC_MIXED), gpu_lattice(L, wl, L.LBM_PREC_MIXED)
    a.init(initial_density(wl))
    a.step(50)
    path = tmp_path / "run.ckpt"
    a.save(str(path))
    b.load(str(path))
    assert b.stats()["step"] == 50
    a.step(60)
    b.step(60)
    assert np.array_equal(a.populations(), b.populations())
    other = gpu_lattice(L, workload("droplet_512_li", nx=100, ny=150, R=30.0), L.LBM_PREC_MIXED)
    with pytest.raises(L.LBMError):
        other.load(str(path))
    hotter = gpu_lattice(L, dict(wl, T_over_Tc=0.7), L.LBM_PREC_MIXED)
    with pytest.raises(L.LBMError):
        hotter.load(str(path))


def test_batch_tanh_start_matches_host_field(L):
    from paper_1412_5170_amd import sweep
    m = dict(sweep.PHYSICS, nx=144, ny=128, T_over_Tc=0.65, tau=0.9, collision="MRT", R=36.0)
    b1, b2 = L.Batch([m]), L.Batch([m])
    b1.init_tanh(0, m["R"], 5.0, droplet=True)
    b2.init_rest(0, sweep.tanh_density(L, m))
    f1, f2 = b1.populations(0), b2.populations(0)
    assert np.max(np.abs(f1.astype(np.float64) - f2) / f2) < 1e-6
    bub = L.Batch([m])
    bub.init_tanh(0, m["R"], 5.0, droplet=False)
    rho, _ = bub.read(0)
    assert rho[64, 72] < 0.05 < rho[0, 0]  # gas inside, liquid outside
