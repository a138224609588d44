"""lbm_stats_noalloc -- lbm_stats without allocating, its reduction in the library's fixed device
array -- against lbm_stats on the same states: two calls in a row through the C ABI, the first on
a lattice whose reduction fills the array's 2048 partial blocks, the second on a smaller one."""
import ctypes

import pytest

from lbm_cases import gpu_lattice, initial_density, say, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1412_5170_amd import lbm
    return lbm


def test_noalloc_stats_equal_lbm_stats(L):
    for nx, ny, steps in ((1000, 700, 40), (200, 77, 30)):
        say(f"[no-alloc stats] {nx}x{ny}, {steps} steps")
        wl = workload("droplet_4096_mrt", nx=nx, ny=ny, R=min(nx, ny) / 4, T_over_Tc=0.6)
        lat = gpu_lattice(L, wl, L.LBM_PREC_MIXED)
        lat.init(initial_density(wl))
        lat.step(steps)
        s = L.lbm_stats_t()
        assert L.lbm_stats_noalloc(lat.h, ctypes.byref(s)) == L.LBM_OK, L.lbm_last_error(lat.h)
        got = s.as_dict()
        ref = lat.stats(track_dv=False)
        say(f"    mass {got['mass']:.15e} / {ref['mass']:.15e}, us_max {got['us_max']:.6e}")
        assert got == ref
        assert got["step"] == steps and got["nonfinite"] == 0 and got["dv_max"] == 0.0
