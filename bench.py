"""Benchmark of the pseudo-potential D2Q9 LBM time step on one MI355X.

Workload (default): the 4096 x 4096 periodic static droplet, radius 600, tanh interface of
width 5 from the Maxwell coexistence densities at T/Tc = 0.5 (ratio ~725), MRT collision
(s_rho = s_j = 1, s_e = s_eps = s_q = 1.1, s_nu = 1/tau, tau = 1), Guo forcing with Li's
modified force term (sigma = 0.125), Carnahan-Starling EOS rescaled by K = 1/49.
A step is one full time step (density/psi pass + fused force/collide/stream pass); the FP64
observables reduction runs every --stats-every steps inside the timed region, as a production
run would.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line: MLUPS, HBM roofline of the dominant (fused) kernel measured with HIP
events on the lattice's stream, and the FP64 oracle's MLUPS on the host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, public spec
FUSED_BYTES_PER_NODE = 76      # 9 FP32 populations read + 9 written + psi read once
PSI_BYTES_PER_NODE = 40        # 9 FP32 populations read + psi written
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="droplet_4096_mrt")
    ap.add_argument("--precision", default="f64", choices=["f32", "f64"])
    ap.add_argument("--tile", default=None, help="tx,ty of the fused pass")
    ap.add_argument("--stats-every", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="do not record per-kernel HIP events (for profiler runs)")
    return ap.parse_args()


def cpu_baseline(wl, budget_s):
    """The FP64 oracle on a bounded sample of the same physics: a 512 x 512 cut of the
    workload (droplet radius scaled with the side), as many steps as fit the budget."""
    import oracle as O
    from oracle import thermo as TH
    from paper_1412_5170_amd import inputs

    n = 512
    scale = n / wl["nx"]
    sample = dict(wl, nx=n, ny=n, R=wl.get("R", 0) * scale if wl["init"] == "droplet" else 0)
    if wl["init"] == "slab":
        sample = dict(wl)
        n = None
    g, l, _ = TH.maxwell(wl["T_over_Tc"])
    rho0 = inputs.initial_density(sample, l, g)
    tau = wl["tau"]
    s = wl.get("s", (1.0,) * 9)
    s = (s[0], s[1], s[2], s[3], s[4], s[5], s[6], 1 / tau, 1 / tau)
    p = O.Params(nx=sample["nx"], ny=sample["ny"], T=TH.temperature(wl["T_over_Tc"]), tau=tau,
                 scheme=getattr(O, wl["scheme"]), collision=getattr(O, wl["collision"]),
                 K=wl["K"], A=wl["A"], sigma=wl["sigma"], s=s)
    f = O.init_feq(rho0)
    t0 = time.perf_counter()
    f = O.step(p, f, 2)                      # calibrate
    per = (time.perf_counter() - t0) / 2
    steps = max(2, int(budget_s / per))
    t0 = time.perf_counter()
    O.step(p, f, steps)
    dt = time.perf_counter() - t0
    nodes = sample["nx"] * sample["ny"]
    return {"value": round(nodes * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"{sample['nx']}x{sample['ny']} cut of the workload (same physics), "
                      f"{steps} FP64 steps, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design note, not code)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1412_5170_amd import inputs, lbm

    wl = dict(inputs.WORKLOADS[args.workload])
    eos = lbm.make_eos(wl["T_over_Tc"], K=wl["K"])
    g, l = lbm.eos_maxwell(eos)
    rho0 = inputs.initial_density(wl, l, g)
    s = wl.get("s", (1.0, 1.1, 1.1, 1.0, 1.1))
    lat = lbm.Lattice(wl["nx"], wl["ny"], eos, lbm.make_force(wl["scheme"], A=wl["A"],
                                                            sigma=wl["sigma"]),
                      lbm.make_collision(wl["collision"], s=s[:5]), wl["tau"],
                      precision=lbm.LBM_PREC_F64 if args.precision == "f64" else lbm.LBM_PREC_F32,
                      tile=tuple(int(v) for v in args.tile.split(",")) if args.tile else None)
    lat.init(rho0)
    del rho0
    nodes = wl["nx"] * wl["ny"]
    print(f"bench: {args.workload} {wl['nx']}x{wl['ny']} {args.precision}, warmup {args.warmup}",
          file=sys.stderr, flush=True)
    lat.step(args.warmup)
    st0 = lat.stats()
    torch.cuda.synchronize()

    if not args.no_timing:
        lat.timing_enable(True)
        lat.timing()                                  # reset
    done = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < args.steps:
        k = min(args.stats_every, args.steps - done)
        lat.step(k)
        done += k
        if args.stats_every and done % args.stats_every == 0:
            st = lat.stats()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    psi_ms = fused_ms = None
    if not args.no_timing:
        psi_ms, fused_ms, nt = lat.timing()
        lat.timing_enable(False)
    st = lat.stats()
    print(f"bench: {args.steps} steps in {elapsed:.3f} s; mass drift "
          f"{(st['mass'] - st0['mass']) / st0['mass']:.2e}; us_max {st['us_max']:.3e}; "
          f"ratio {st['ratio']:.2f}", file=sys.stderr, flush=True)

    mlups = nodes * args.steps / elapsed / 1e6
    roof = None
    if fused_ms is not None:
        avg_fused_s = fused_ms / 1e3 / nt
        avg_psi_s = psi_ms / 1e3 / nt
        achieved = FUSED_BYTES_PER_NODE * nodes / avg_fused_s / 1e9
        traffic = None
        if os.path.exists(PROFILE_TRAFFIC):
            t = json.load(open(PROFILE_TRAFFIC))
            if t.get("workload") == args.workload and t.get("precision") == args.precision:
                traffic = t.get("fused_bytes_per_launch")
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "fused_kernel", "avg_us": round(avg_fused_s * 1e6, 2),
                "psi_pass": {"avg_us": round(avg_psi_s * 1e6, 2),
                             "achieved": round(PSI_BYTES_PER_NODE * nodes / avg_psi_s / 1e9, 1)}}
    out = {
        "metric": "MLUPS", "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "f32" else "f64 (f32 storage)",
        "data": "synthetic",
        "config": {"workload": args.workload, "nx": wl["nx"], "ny": wl["ny"],
                   "collision": wl["collision"], "scheme": wl["scheme"],
                   "T_over_Tc": wl["T_over_Tc"], "K": wl["K"], "tau": wl["tau"],
                   "stats_every": args.stats_every, "parallelism": "single GPU"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        del lat
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
