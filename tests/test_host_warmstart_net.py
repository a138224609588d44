"""The committed warm-start network (weights-only file and its manifest), checked on the CPU:
it loads without unpickling, matches its manifest, and -- evaluated by the oracle's FP64
network on lattices of the batched sweep's draw -- predicts radial profiles that are
valid densities with a liquid core near the Maxwell liquid density and a vapour outside near
the Maxwell gas density of each lattice's temperature (Eq. 19)."""
import hashlib
import json

import numpy as np

from oracle import mlp
from oracle import thermo as TH
from paper_1412_5170_amd import inputs, sweep, warmstart as WS


def test_network_file_and_manifest():
    d = np.load(WS.NET_PATH, allow_pickle=False)
    assert sorted(d.files) == ["mean", "params", "std"]
    n = sum(i * o + o for i, o in zip(WS.DIMS[:-1], WS.DIMS[1:]))
    assert d["params"].shape == (n,) and d["params"].dtype == np.float32
    assert d["mean"].shape == (WS.DIMS[-1],) and d["std"].shape == (WS.DIMS[-1],)
    assert np.all(np.isfinite(d["params"])) and np.all(d["std"] > 0)
    man = json.load(open(WS.NET_MANIFEST))
    assert man["sha256_16"] == hashlib.sha256(open(WS.NET_PATH, "rb").read()).hexdigest()[:16]
    assert man["network"]["dims"] == WS.DIMS
    assert man["training_draw"]["count"] == 2000
    assert man["generation"][0]["converged"] == man["generation"][0]["members"]
    draw = WS.draw_training(man["training_draw"]["seed"], man["training_draw"]["count"])
    assert min(m["nx"] for m in draw) >= 96 and max(m["nx"] for m in draw) <= 384
    # the droplets of the sweep's largest sizes, so that large radii are not extrapolated
    large = WS.draw_training(man["large_draw"]["seed"], man["large_draw"]["count"], n_min=512,
                             n_levels=33)
    assert min(m["nx"] for m in large) >= 512 and max(m["nx"] for m in large) <= 1024
    assert man["generation"][1]["members"] == len(large)
    # and droplets of the upper sizes at the sweep's own K, the value the sweep is run at
    at_k = WS.draw_training(man["sweep_k_draw"]["seed"], man["sweep_k_draw"]["count"], n_min=384,
                            n_levels=41, K=sweep.PHYSICS["K"])
    assert min(m["nx"] for m in at_k) >= 384 and max(m["nx"] for m in at_k) <= 1024
    assert all(m["K"] == sweep.PHYSICS["K"] for m in at_k)
    assert man["generation"][2]["members"] == len(at_k)
    # and cold droplets at that K, where the densities change fastest with T/Tc
    cold = WS.draw_training(man["cold_draw"]["seed"], man["cold_draw"]["count"], n_min=384,
                            n_levels=41, K=sweep.PHYSICS["K"], ttc_range=(0.5, 0.65))
    assert all(0.5 <= m["T_over_Tc"] <= 0.65 and m["K"] == sweep.PHYSICS["K"] for m in cold)
    assert man["generation"][3]["members"] == len(cold)
    assert man["generation"][0]["tol"] == man["training_draw"]["stopping_rule"]["tol_velocity_per_step"]


def test_predicted_profiles_are_physical():
    d = np.load(WS.NET_PATH, allow_pickle=False)
    members = sweep.members_from_draw(inputs.batch_draw(0))[:12]  # sizes 128..1008, T/Tc 0.5..0.9
    X = np.stack([WS.features(m) for m in members]).astype(np.float64)
    y = mlp.forward(d["params"], WS.DIMS, X)[-1] * d["std"] + d["mean"]
    rho = np.exp(y)
    assert np.all(np.isfinite(rho)) and np.all(rho > 0) and np.all(rho < 1.0)  # 4/b = 1
    for m, r in zip(members, rho):
        g, l, _ = TH.maxwell(m["T_over_Tc"])
        # radii r_k = R + 2 (k - 23.5): k = 0 is 47 nodes inside the interface, k = 63 is 79
        # nodes out.  In a closed periodic box the droplet's Laplace pressure and the finite mass
        # move both bulk densities off the flat-interface values: the liquid's by a few per cent,
        # the vapour's by up to about 2x on small, cold droplets (ratio ~725).
        assert 0.93 < r[0] / l < 1.05, (m, r[0], l)
        assert 0.9 < r[-1] / g < 2.0, (m, r[-1], g)
        assert np.all(np.diff(r[16:32]) < 0)  # the interface falls monotonically outwards
