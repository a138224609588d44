"""Benchmark of the pseudo-potential D2Q9 LBM time step on one MI355X.

Workload (default): the 4096 x 4096 periodic static droplet, radius 600, tanh interface of
width 5 from the Maxwell coexistence densities at T/Tc = 0.5 (ratio ~725), MRT collision
(s_rho = s_j = 1, s_e = s_eps = s_q = 1.1, s_nu = 1/tau, tau = 1), Guo forcing with Li's
modified force term (sigma = 0.125), Carnahan-Starling EOS rescaled by K = 1/49.
A step is one full time step (psi from the populations, force, forcing, collision, streaming)
and the FP64 observables reduction runs every --stats-every steps inside the timed region, as a
production run would.  Inputs are resident in HBM before timing starts.  By default the library's
default launch runs: the two-step sweep (two time steps per pass over HBM, 64-lane strips of 58
output columns over 16-row segments); --kernel sweep runs the one-step sweep (512-column strips,
8-row segments, two rows of loads in flight, XCD-ordered tiles), --kernel two_pass the
density/psi pass and the fused pass; --autotune lets the library's autotuner pick (timed
trials on the initial state, which it restores, before the warm-up), --launch sets the shape.

Prints ONE JSON line: MLUPS, the roofline of the dominant kernel measured with HIP events on the
lattice's stream (the two-step sweep against the vector ALU peak -- algorithmic flops per launch
/ average launch time -- with its HBM figures and its VALU issue rate alongside; the one-step
kernels against HBM), the same for the alternative kernel, and the FP64 oracle's MLUPS on the
host cores (cpu_baseline).

--copy-probe instead times the library's plain copy kernel on a buffer the size of one
population buffer (the scale reference for the HBM counters).
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
SWEEP_BYTES_PER_NODE = 72      # one-pass step: 9 FP32 populations read + 9 written
# Floating-point operations of one node's update on this workload's path (C-S EOS, MRT with Guo
# and Li, mixed precision), counted in the compiled update: 2 per FMA, 1 per add, multiply,
# reciprocal or square root; conversions, moves and lane shifts count 0.
FLOPS_PER_NODE_STEP = 236
# Vector ALU peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz, for
# FP64 and unpacked FP32 alike; and the VALU issue peak, 1024 SIMDs x 16 lanes x 2.4 GHz.
ALU_PEAK_TFLOPS = 78.6
VALU_LANE_OPS_PEAK = 1024 * 16 * 2.4e9
FUSED_BYTES_PER_NODE = 76      # two-pass, pass 2: 9 populations read + 9 written + psi read
PSI_BYTES_PER_NODE = 40        # two-pass, pass 1: 9 populations read + psi written
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="droplet_4096_mrt")
    ap.add_argument("--precision", default="mixed", choices=["f32", "f64", "mixed"])
    ap.add_argument("--kernel", default="sweep2", choices=["sweep2", "sweep", "two_pass"],
                    help="sweep2: two steps per launch (the library's default); sweep: one step")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the sweep's launch with the library's autotuner first")
    ap.add_argument("--launch", default=None,
                    help="tx,ty[,flags] of the kernel (default: the library's choice)")
    ap.add_argument("--layout", default="rows", choices=["rows", "planes"])
    ap.add_argument("--alt-steps", type=int, default=200,
                    help="steps of the two-pass variant timed beside the main result (0: skip)")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--stats-every", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true",
                    help="do not record per-kernel HIP events (for profiler runs)")
    return ap.parse_args()


def kernel_source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_1412_5170_amd", "csrc", "lbm_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def cpu_baseline(wl, budget_s):
    """The FP64 oracle on a bounded sample of the same physics: a 512 x 512 cut of the
    workload (droplet radius scaled with the side), as many steps as fit the budget."""
    import oracle as O
    from oracle import thermo as TH
    from paper_1412_5170_amd import inputs

    if wl["init"] == "droplet" and wl["nx"] > 512:
        sample = dict(wl, nx=512, ny=512, R=wl["R"] * 512 / wl["nx"])
    else:
        sample = dict(wl)
    g, l, _ = TH.maxwell(wl["T_over_Tc"])
    rho0 = inputs.initial_density(sample, l, g)
    tau = wl["tau"]
    s = wl.get("s", (1.0, 1.1, 1.1, 1.0, 1.1))
    s = (s[0], s[1], s[2], s[3], s[4], s[3], s[4], 1 / tau, 1 / tau)
    p = O.Params(nx=sample["nx"], ny=sample["ny"], T=TH.temperature(wl["T_over_Tc"]), tau=tau,
                 scheme=getattr(O, wl["scheme"]), collision=getattr(O, wl["collision"]),
                 K=wl["K"], A=wl["A"], sigma=wl["sigma"], s=s)
    f = O.init_feq(rho0)
    f = O.step(p, f, 1)                      # warm-up (thread start, first touch)
    # chunks of growing length until the budget is spent: no estimate from a first step
    steps, chunk = 0, 4
    t0 = time.perf_counter()
    while True:
        f = O.step(p, f, chunk)
        steps += chunk
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
        chunk = min(2 * chunk, 256)
    nodes = sample["nx"] * sample["ny"]
    return {"value": round(nodes * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"{sample['nx']}x{sample['ny']} lattice of the workload's physics (droplet "
                      f"radius scaled with the side), {steps} FP64 steps, {dt:.1f} s"}


PRECISIONS = {"f32": 0, "f64": 1, "mixed": 2}
DTYPE = {"f32": "f32", "f64": "f64 (f32 storage)", "mixed": "f32+f64 mixed (f32 storage)"}


def make_lattice(lbm, wl, args, kernel):
    eos = lbm.make_eos(wl["T_over_Tc"], K=wl["K"])
    s = wl.get("s", (1.0, 1.1, 1.1, 1.0, 1.1))
    lat = lbm.Lattice(wl["nx"], wl["ny"], eos,
                      lbm.make_force(wl["scheme"], A=wl["A"], sigma=wl["sigma"]),
                      lbm.make_collision(wl["collision"], s=s[:5]), wl["tau"],
                      precision=PRECISIONS[args.precision],
                      layout=lbm.LBM_LAYOUT_ROWS if args.layout == "rows" else lbm.LBM_LAYOUT_PLANES)
    k, tx, ty, fl = lat.get_launch()  # the library's default: the two-step sweep
    if kernel == "two_pass":
        k, tx, ty, fl = lbm.LBM_KERNEL_TWO_PASS, 128, 8, lbm.LBM_LAUNCH_XCD_ORDER
    if kernel == "sweep":  # the one-step sweep's default shape on this lattice
        k, tx, ty, fl = lbm.LBM_KERNEL_SWEEP, 512, 8, lbm.LBM_LAUNCH_XCD_ORDER
    if args.launch and kernel == args.kernel:
        v = [int(t) for t in args.launch.split(",")]
        tx, ty = v[0], v[1]
        fl = v[2] if len(v) > 2 else fl
    lat.set_launch({"sweep": lbm.LBM_KERNEL_SWEEP, "sweep2": lbm.LBM_KERNEL_SWEEP2,
                    "two_pass": lbm.LBM_KERNEL_TWO_PASS}[kernel], tx, ty, fl)
    return lat


def timed(lat, steps, stats_every, torch, timing=True):
    """Run `steps` steps (the observables reduction every `stats_every`); returns wall seconds
    and the library's per-kernel event totals."""
    if timing:
        lat.timing_enable(True)
        lat.timing()                                  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(stats_every or steps, steps - done)
        lat.step(k)
        done += k
        if stats_every and done % stats_every == 0:
            lat.stats()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ev = None
    if timing:
        ev = lat.timing()
        lat.timing_enable(False)
    return elapsed, ev


def copy_probe(args):
    import torch

    from paper_1412_5170_amd import inputs, lbm
    wl = inputs.WORKLOADS[args.workload]
    n = 9 * wl["nx"] * wl["ny"]
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        lbm.check(lbm.lbm_copy_f32(dst.data_ptr(), src.data_ptr(), n, stream))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, args.steps)
    for _ in range(reps):
        lbm.check(lbm.lbm_copy_f32(dst.data_ptr(), src.data_ptr(), n, stream))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_probe": {"bytes_read": 4 * n, "bytes_written": 4 * n,
                                     "us": round(dt * 1e6, 2),
                                     "GBps": round(8 * n / dt / 1e9, 1)}}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: pplbm runs on one GPU; --gpus {args.gpus} is not supported (the "
              "y-slab decomposition across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args)
        return

    import torch

    from paper_1412_5170_amd import inputs, lbm

    wl = dict(inputs.WORKLOADS[args.workload])
    g, l = lbm.eos_maxwell(lbm.make_eos(wl["T_over_Tc"], K=wl["K"]))
    rho0 = inputs.initial_density(wl, l, g)
    nodes = wl["nx"] * wl["ny"]
    timing = not args.no_timing

    lat = make_lattice(lbm, wl, args, args.kernel)
    lat.init(rho0)
    tuned_ms = None
    if args.kernel != "two_pass" and not args.launch and args.autotune:
        # the library's autotuner (timed trials on this state, restored afterwards), before
        # the warm-up and outside the timed region
        tuned_ms = lat.autotune(None, trial_steps=50)
    launch = lat.get_launch()
    print(f"bench: {args.workload} {wl['nx']}x{wl['ny']} {args.precision} {args.kernel} "
          f"launch {launch}, warmup {args.warmup}", file=sys.stderr, flush=True)
    lat.step(args.warmup)
    st0 = lat.stats()
    elapsed, ev = timed(lat, args.steps, args.stats_every, torch, timing)
    st = lat.stats()
    print(f"bench: {args.steps} steps in {elapsed:.3f} s; mass drift "
          f"{(st['mass'] - st0['mass']) / st0['mass']:.2e}; us_max {st['us_max']:.3e}; "
          f"ratio {st['ratio']:.2f}", file=sys.stderr, flush=True)
    del lat

    def roofline(kernel, ev, launch):
        psi_ms, main_ms, nt = ev
        steps_per_launch = 2 if kernel == "sweep2" else 1  # the two-step sweep: 2 per launch
        avg = main_ms / 1e3 / (nt / steps_per_launch)     # per launch of the main kernel
        per_node = FUSED_BYTES_PER_NODE if kernel == "two_pass" else SWEEP_BYTES_PER_NODE
        achieved = per_node * nodes / avg / 1e9
        r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
             "kernel": {"sweep": "sweep_kernel", "sweep2": "sweep2_kernel",
                        "two_pass": "fused_kernel"}[kernel],
             "bytes_per_node": per_node, "steps_per_launch": steps_per_launch,
             "avg_us": round(avg * 1e6, 2)}
        if kernel == "sweep2":
            # Two steps per pass over HBM: the kernel is bound by vector ALU issue, not HBM.
            tflops = FLOPS_PER_NODE_STEP * steps_per_launch * nodes / avg / 1e12
            hbm = {k: r[k] for k in ("achieved", "peak", "unit", "frac", "bytes_per_node")}
            r.update(bound="alu", achieved=round(tflops, 2), peak=ALU_PEAK_TFLOPS,
                     unit="TFLOP/s", frac=round(tflops / ALU_PEAK_TFLOPS, 4),
                     flops_per_node_step=FLOPS_PER_NODE_STEP, hbm=hbm)
        if kernel == "two_pass":
            pavg = psi_ms / 1e3 / nt
            r["psi_pass"] = {"kernel": "psi_kernel", "avg_us": round(pavg * 1e6, 2),
                             "achieved": round(PSI_BYTES_PER_NODE * nodes / pavg / 1e9, 1)}
        if os.path.exists(PROFILE_TRAFFIC):
            t = json.load(open(PROFILE_TRAFFIC))
            key = f"{args.workload}/{kernel}/{args.precision}/{args.layout}"
            # Counters are only valid for the kernel source and launch they were taken on.
            if (key in t and t[key]["kernel_sha256_16"] == kernel_source_hash()
                    and list(t[key].get("launch", [])) == list(launch)):
                r["traffic"] = t[key]["bytes_per_launch"]
                r["traffic_over_algorithmic"] = round(t[key]["bytes_per_launch"] /
                                                      (per_node * nodes), 4)
                if "valu_insts_per_launch" in t[key]:  # wave instructions (SQ_INSTS_VALU)
                    lane_ops = 64 * t[key]["valu_insts_per_launch"] / avg
                    r["valu_issue"] = {"achieved": round(lane_ops / 1e12, 2),
                                       "peak": round(VALU_LANE_OPS_PEAK / 1e12, 2),
                                       "unit": "T lane-instructions/s",
                                       "frac": round(lane_ops / VALU_LANE_OPS_PEAK, 4)}
        return r

    mlups = nodes * args.steps / elapsed / 1e6
    out = {
        "metric": "MLUPS", "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "nx": wl["nx"], "ny": wl["ny"],
                   "collision": wl["collision"], "scheme": wl["scheme"],
                   "T_over_Tc": wl["T_over_Tc"], "K": wl["K"], "tau": wl["tau"],
                   "kernel": args.kernel, "launch": list(launch),
                   "autotuned": tuned_ms is not None, "layout": args.layout,
                   "stats_every": args.stats_every, "parallelism": "single GPU"},
        "roofline": roofline(args.kernel, ev, launch) if ev else None,
    }
    if out["roofline"] is not None:
        # The whole job's rate at the method's minimum of 72 B per lattice update (one read
        # and one write of the nine FP32 populations): the HBM rate a one-step kernel would
        # need for the same throughput.
        gbs = mlups * SWEEP_BYTES_PER_NODE / 1e3
        out["roofline"]["algorithmic_fraction"] = {
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "basis": "whole-job MLUPS x 72 B per lattice update"}
    alt = "sweep" if args.kernel == "sweep2" else ("two_pass" if args.kernel == "sweep" else "sweep")
    if timing and args.alt_steps:
        lat = make_lattice(lbm, wl, args, alt)
        alt_launch = lat.get_launch()
        lat.init(rho0)
        lat.step(args.warmup)
        el2, ev2 = timed(lat, args.alt_steps, args.stats_every, torch, True)
        del lat
        out["alternative"] = {"kernel": alt, "MLUPS": round(nodes * args.alt_steps / el2 / 1e6, 1),
                              "roofline": roofline(alt, ev2, alt_launch)}
    del rho0
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
