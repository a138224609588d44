"""Benchmark of the pseudo-potential D2Q9 LBM on one MI355X.

Main leg (the JSON line's `value`): MLUPS of the 4096 x 4096 periodic static droplet, radius
600, tanh interface of width 5 from the Maxwell coexistence densities at T/Tc = 0.5 (ratio
~725), MRT collision (s_rho = s_j = 1, s_e = s_eps = s_q = 1.1, s_nu = 1/tau, tau = 1), Guo
forcing with Li's modified force term (sigma = 0.125), Carnahan-Starling EOS rescaled by
K = 1/49.  A step is one full time step (psi from the populations, force, forcing, collision,
streaming); the FP64 observables reduction runs every --stats-every steps inside the timed
region, as a production run would.  Inputs are resident in HBM before timing starts.  Before
the W warm-up steps the lattice steps for --settle-seconds of wall time, so that the timed
steps do not run on a GPU still raising its clocks.  By default the library's default launch
runs (the two-step sweep); --kernel sweep / two_pass select the one-step sweep or the
two-pass step, --autotune lets the library's autotuner pick, --launch sets the shape.

`roofline` is the dominant kernel's HBM rate: algorithmic bytes per launch (72 B per node and
time step: nine FP32 populations read and nine written, two time steps per launch of the
two-step sweep) over the kernel's average launch time from HIP events on the lattice's stream,
against 8 TB/s (two steps per launch can pass 1: each launch reads and writes the populations
once for two steps); the real traffic (rocprofv3 counters of the same source and launch), the
HBM bandwidth it draws and the VALU issue rate stand beside it.

Further legs (each can be switched off): the same for the alternative kernel; `small_configs`,
the 4 x 256 EDM slab (microseconds per step, as a lone lattice and replayed from a hipGraph as a
one-member batch) and the 512 x 512 Li droplet at tau 0.6 and 1.0 (MLUPS); `batch`, the
64-lattice droplet draw of the batched sweep (sizes 128^2-1024^2) stepped a fixed number of
steps (GLUPS); `sweep`, that draw run to equilibrium from tanh starts (max |v| change per step
< 1e-9 and probe densities changing < 2e-9 per step, checked every 500 steps): wall time and
steps; `warm_start`, the same draw started from the learned network's profiles vs tanh, each
lattice stepped exactly as far as the recorded equal-accuracy budgets say (density ratio within
1e-4 of the converged one), wall time of both and the ratio errors reached; and `cpu_baseline`,
the FP64 oracle on the host cores (one thread and all threads).

--copy-probe instead times the library's plain copy kernel on a buffer the size of one
population buffer (the scale reference for the HBM counters).
"""
from __future__ import annotations

import argparse
import contextlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, public spec
SWEEP_BYTES_PER_NODE = 72      # one-pass step: 9 FP32 populations read + 9 written
# VALU issue peak: 1024 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second (one wave64
# instruction per SIMD every four cycles; FP64 and unpacked FP32 issue alike).
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
    ap.add_argument("--precision", default="mixed", choices=["f64", "mixed"])
    ap.add_argument("--kernel", default="sweep2", choices=["sweep2", "sweep", "two_pass"],
                    help="sweep2: two steps per launch (the library's default); sweep: one step")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the sweep's launch with the library's autotuner first")
    ap.add_argument("--launch", default=None,
                    help="tx,ty[,flags] of the kernel (default: the library's choice)")
    ap.add_argument("--layout", default="rows", choices=["rows", "planes"])
    ap.add_argument("--alt-steps", type=int, default=200,
                    help="steps of the alternative kernel (the one-step sweep beside the two-step "
                         "one) timed beside the main result (0: skip)")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--stats-every", type=int, default=100)
    ap.add_argument("--settle-seconds", type=float, default=2.0,
                    help="wall seconds of stepping before the warm-up steps (GPU clocks)")
    ap.add_argument("--batch-steps", type=int, default=2000,
                    help="steps of the 64-lattice batch leg (0: skip)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the time-to-equilibrium legs (sweep and warm start)")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the warm-start leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small-workload leg (4 x 256 slab, 512 x 512 droplet)")
    ap.add_argument("--no-timing", action="store_true",
                    help="do not record per-kernel HIP events (for profiler runs)")
    return ap.parse_args()


def kernel_source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_1412_5170_amd", "csrc", "lbm_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def _oracle_run(O, p, f, steps):
    """Wall seconds of `steps` oracle steps (after one untimed step: thread start, first
    touch)."""
    f = O.step(p, f, 1)
    t0 = time.perf_counter()
    O.step(p, f, steps)
    return time.perf_counter() - t0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl):
    """The FP64 oracle (plain C, OpenMP over rows) on bounded samples of the benchmark's
    workloads, on all of the host's threads and on one: the 4096^2 MRT droplet itself for 20
    steps (all threads; `value`), a 256^2 cut of its physics on one thread, and the 512^2 BGK
    Guo + Li droplet at T/Tc = 0.6, K = 1/49 (radius 80) for 200 steps on all threads and 20 on
    one.  MLUPS = nodes x steps / wall seconds; the oracle moves 144 B per lattice update in
    FP64."""
    import oracle as O
    from oracle import thermo as TH
    from paper_1412_5170_amd import inputs

    def params(w):
        tau = w["tau"]
        s = w.get("s", (1.0, 1.1, 1.1, 1.0, 1.1))
        s = (s[0], s[1], s[2], s[3], s[4], s[3], s[4], 1 / tau, 1 / tau)
        return O.Params(nx=w["nx"], ny=w["ny"], T=TH.temperature(w["T_over_Tc"]), tau=tau,
                        scheme=getattr(O, w["scheme"]), collision=getattr(O, w["collision"]),
                        K=w["K"], A=w["A"], sigma=w["sigma"], s=s)

    def state(w):
        g, l, _ = TH.maxwell(w["T_over_Tc"])
        return O.init_feq(inputs.initial_density(w, l, g))

    all_threads = O.threads()
    c2 = dict(inputs.WORKLOADS["droplet_512_li"])
    cut = dict(wl, nx=256, ny=256, R=wl["R"] * 256 / wl["nx"])
    runs = []
    for name, w, steps, threads in ((f"{wl['nx']}x{wl['ny']} (the main leg's workload)", wl, 20,
                                     all_threads),
                                    ("256x256 cut of the main leg's physics", cut, 60, 1),
                                    ("512x512 Guo + Li BGK droplet", c2, 200, all_threads),
                                    ("512x512 Guo + Li BGK droplet", c2, 20, 1)):
        O.set_threads(threads)
        dt = _oracle_run(O, params(w), state(w), steps)
        runs.append({"lattice": name, "threads": threads, "steps": steps,
                     "seconds": round(dt, 2),
                     "MLUPS": round(w["nx"] * w["ny"] * steps / dt / 1e6, 3)})
    O.set_threads(all_threads)
    main = runs[0]
    return {"value": main["MLUPS"], "unit": "MLUPS", "cores": all_threads, "kind": "oracle",
            "sample": f"{main['lattice']}, {main['steps']} FP64 steps in {main['seconds']} s on "
                      f"{all_threads} threads",
            "cpu": cpu_model(), "nproc": os.cpu_count(), "runs": runs}


PRECISIONS = {"f64": 1, "mixed": 2}
DTYPE = {"f64": "f64 (f32 storage)", "mixed": "f32+f64 mixed (f32 storage)"}


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


def settle(lat, seconds, torch):
    """Step for `seconds` of wall time (chunks of 100 steps) before the warm-up, so that the
    timed steps run at the clocks a long job runs at.  Returns the steps taken."""
    if seconds <= 0:
        return 0
    torch.cuda.synchronize()
    t0, n = time.perf_counter(), 0
    while time.perf_counter() - t0 < seconds:
        lat.step(100)
        torch.cuda.synchronize()
        n += 100
    return n


def roofline(kernel, ev, launch, nodes, args):
    """HBM roofline of one launch of `kernel`: algorithmic bytes per launch over the average
    launch time (HIP events around the timed region's launches), against 8 TB/s; the real
    traffic and the VALU issue rate (from the committed counters of the same source and launch)
    beside it."""
    psi_ms, main_ms, nt = ev
    steps_per_launch = 2 if kernel == "sweep2" else 1  # the two-step sweep: 2 per launch
    avg = main_ms / 1e3 / (nt / steps_per_launch)     # per launch of the main kernel
    per_node = FUSED_BYTES_PER_NODE if kernel == "two_pass" else SWEEP_BYTES_PER_NODE
    algo_bytes = per_node * steps_per_launch * nodes  # per launch
    achieved = algo_bytes / avg / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
         "kernel": {"sweep": "sweep_kernel", "sweep2": "sweep2_kernel",
                    "two_pass": "fused_kernel"}[kernel],
         "bytes_per_node_step": per_node, "steps_per_launch": steps_per_launch,
         "algorithmic_bytes_per_launch": algo_bytes, "launches": int(nt // steps_per_launch),
         "avg_us": round(avg * 1e6, 2)}
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
            r["traffic_over_algorithmic"] = round(t[key]["bytes_per_launch"] / algo_bytes, 4)
            # the same against one read and one write of the populations per launch
            r["traffic_over_one_pass"] = round(t[key]["bytes_per_launch"] / (72 * nodes), 4)
            # the HBM bandwidth actually drawn: measured bytes over the same launch time
            r["traffic_achieved"] = round(t[key]["bytes_per_launch"] / avg / 1e9, 1)
            r["traffic_frac"] = round(t[key]["bytes_per_launch"] / avg / 1e9 / HBM_PEAK_GBS, 4)
            if "valu_insts_per_launch" in t[key]:  # wave instructions (SQ_INSTS_VALU)
                lane_ops = 64 * t[key]["valu_insts_per_launch"] / avg
                r["valu_issue"] = {"achieved": round(lane_ops / 1e12, 2),
                                   "peak": round(VALU_LANE_OPS_PEAK / 1e12, 2),
                                   "unit": "T lane-instructions/s",
                                   "frac": round(lane_ops / VALU_LANE_OPS_PEAK, 4)}
    return r


def say(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def batch_leg(lbm, steps):
    """The 64-lattice droplet draw of the batched sweep (seed 0: sizes 128^2-1024^2, R = n/4,
    tau in [0.6, 1.5], T/Tc in [0.5, 0.9], BGK or MRT; Guo + Li, K = 1/49) from its tanh
    starts, stepped `steps` steps with every lattice active (after one untimed block that also
    captures the graph)."""
    from paper_1412_5170_amd import inputs, sweep
    members = sweep.members_from_draw(inputs.batch_draw(0))
    b = lbm.Batch(members)
    for i, m in enumerate(members):
        b.init_rest(i, sweep.tanh_density(lbm, m))
    b.step(steps)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    dt = time.perf_counter() - t0
    nodes = sum(m["nx"] * m["ny"] for m in members)
    del b
    extra = {}
    if os.path.exists(PROFILE_TRAFFIC):
        t = json.load(open(PROFILE_TRAFFIC)).get("batch64/batch2/mixed")
        if t and t["kernel_sha256_16"] == kernel_source_hash() and t["nodes"] == nodes:
            per_launch = 2 * dt / steps  # two steps per launch
            lane_ops = 64 * t["valu_insts_per_launch"] / per_launch
            extra = {"traffic_per_launch": t["bytes_per_launch"],
                     "traffic_over_one_pass": round(t["bytes_per_launch"] / (72 * nodes), 4),
                     "valu_issue": {"achieved": round(lane_ops / 1e12, 2),
                                    "peak": round(VALU_LANE_OPS_PEAK / 1e12, 2),
                                    "unit": "T lane-instructions/s",
                                    "frac": round(lane_ops / VALU_LANE_OPS_PEAK, 4)}}
    return {**extra, "lattices": len(members), "nodes": nodes, "steps": steps,
            "seconds": round(dt, 4), "us_per_step": round(dt / steps * 1e6, 2),
            "GLUPS": round(nodes * steps / dt / 1e9, 2),
            "hbm_algorithmic": {"achieved": round(72 * nodes * steps / dt / 1e9, 1),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(72 * nodes * steps / dt / 1e9 / HBM_PEAK_GBS, 4)}}


def small_configs_leg(lbm, args, torch):
    """The two small workloads, bound by launch latency or cache-resident, so no roofline: the
    4 x 256 flat slab (EDM, BGK, tau = 1, T/Tc = 0.8, K = 1, A = -0.26; liquid rows 64-191 at
    the Maxwell densities) for 10 000 steps, as a lone lattice (one launch per two steps) and as
    a one-member batch (blocks of 100 steps replayed from a captured hipGraph): microseconds per
    step; the 512 x 512 Li droplet (Guo + Li, BGK, T/Tc = 0.6, K = 1/49, R = 80) at tau = 0.6 and
    1.0 for 20 000 steps: MLUPS.  Each after an untimed block of the same launches."""
    from paper_1412_5170_amd import inputs

    def lattice(wl):  # the library's default launch on each lattice
        eos = lbm.make_eos(wl["T_over_Tc"], K=wl["K"])
        g, l = lbm.eos_maxwell(eos)
        rho0 = inputs.initial_density(wl, l, g)
        lat = lbm.Lattice(wl["nx"], wl["ny"], eos,
                          lbm.make_force(wl["scheme"], A=wl["A"], sigma=wl["sigma"]),
                          lbm.make_collision(wl["collision"]), wl["tau"],
                          precision=PRECISIONS[args.precision])
        lat.init(rho0)
        return lat, rho0

    def wall(run, n):
        run(n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(n)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    slab = dict(inputs.WORKLOADS["slab_4x256_edm"])
    n1 = 10_000
    lat, rho0 = lattice(slab)
    t_lone = wall(lat.step, n1)
    del lat
    b = lbm.Batch([dict(slab)])
    b.init(0, rho0)

    def batch_run(n):
        for _ in range(n // 100):
            b.step(100)
        b.sync()

    t_graph = wall(batch_run, n1)
    del b
    out = {"slab_4x256_edm": {"steps": n1, "lone_us_per_step": round(t_lone / n1 * 1e6, 3),
                               "graph_us_per_step": round(t_graph / n1 * 1e6, 3)}}
    n2 = 20_000
    for tau in (0.6, 1.0):
        wl = dict(inputs.WORKLOADS["droplet_512_li"], tau=tau)
        lat, _ = lattice(wl)
        dt = wall(lat.step, n2)
        del lat
        out[f"droplet_512_li_tau{tau}"] = {"steps": n2, "us_per_step": round(dt / n2 * 1e6, 3),
                                           "MLUPS": round(wl["nx"] * wl["ny"] * n2 / dt / 1e6, 1)}
    return out


def sweep_leg(lbm):
    """Time to equilibrium of the 64-lattice draw from tanh starts (the batched sweep's own
    stopping rule)."""
    from paper_1412_5170_amd import inputs, sweep
    members = sweep.members_from_draw(inputs.batch_draw(0))
    inits = [sweep.tanh_density(lbm, m) for m in members]
    wall, steps, status, b = sweep.run_batch(lbm, members, inits, tol=1e-9, tol_rho=2e-9,
                                             check_every=500, max_steps=1_000_000,
                                             chunk=100_000, report=say)
    del b
    lu = sum(m["nx"] * m["ny"] * st for m, st in zip(members, steps))
    return {"wall_s": round(wall, 2), "lattice_updates": int(lu),
            "GLUPS": round(lu / wall / 1e9, 2), "converged": int(sum(s == 0 for s in status)),
            "lattices": len(members), "max_steps": int(max(steps)),
            "rule": "max |v(t) - v(t-500)| / 500 < 1e-9 and probe densities changing < 2e-9 "
                    "per step, checked every 500 steps"}


def warm_start_leg(lbm):
    """The learned warm start against tanh starts on the 64-lattice draw at equal accuracy:
    each lattice steps exactly its recorded budget (the first step from which its density
    ratio stays within 1e-4 of the converged ratio, from trajectories under a 4x tighter rule),
    and the ratios reached are measured against the recorded converged ratios."""
    from paper_1412_5170_amd import inputs, sweep, warmstart as WS
    if not os.path.exists(WS.EQUAL_ACCURACY_PATH):
        return {"skipped": "no equal-accuracy record"}
    rec = json.load(open(WS.EQUAL_ACCURACY_PATH))
    if rec.get("net_sha256_16") != WS.net_digest():
        return {"skipped": "the equal-accuracy record belongs to another network"}
    members = sweep.members_from_draw(inputs.batch_draw(rec["seed"], count=rec["count"],
                                                        n_levels=rec["levels"]))
    sur = WS.load_surrogate(lbm)
    ref = rec["reference_ratio"]
    out = {"eps": rec["eps"], "lattices": len(members), "net_sha256_16": rec["net_sha256_16"]}
    for mode in ("tanh", "learned"):
        inits = WS._start(lbm, sur, members, mode)
        wall, lu, ratios, fb = WS.budgeted(lbm, members, inits, rec["budgets"][mode],
                                           rec["check_every"], mode)
        err = [abs(x - r) / r for x, r in zip(ratios, ref)]
        out[mode] = {"wall_s": round(wall, 2), "lattice_updates": int(lu),
                     "ratio_err_max": float(max(err)), "fallbacks": fb}
        say(f"warm start {mode}: {wall:.1f} s, ratio error max {max(err):.2e}")
    out["speedup_wall"] = round(out["tanh"]["wall_s"] / out["learned"]["wall_s"], 3)
    out["speedup_updates"] = round(out["tanh"]["lattice_updates"] /
                                   out["learned"]["lattice_updates"], 3)
    return out


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
    say(f"{args.workload} {wl['nx']}x{wl['ny']} {args.precision} {args.kernel} launch {launch}, "
        f"settle {args.settle_seconds} s, warmup {args.warmup}")
    # The settle steps advance the workload itself: the timed steps run on its developed state
    # (the first ~160 steps after the tanh start run up to 20 % slower per launch) and at the
    # clocks of a sustained run.
    settled = settle(lat, args.settle_seconds, torch)
    lat.step(args.warmup)
    st0 = lat.stats()
    elapsed, ev = timed(lat, args.steps, args.stats_every, torch, timing)
    st = lat.stats()
    say(f"{args.steps} steps in {elapsed:.4f} s; mass drift "
        f"{(st['mass'] - st0['mass']) / st0['mass']:.2e}; us_max {st['us_max']:.3e}; "
        f"ratio {st['ratio']:.2f}")
    del lat

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
                   "stats_every": args.stats_every, "settle_seconds": args.settle_seconds,
                   "settle_steps": settled, "parallelism": "single GPU"},
        "roofline": roofline(args.kernel, ev, launch, nodes, args) if ev else None,
    }
    if out["roofline"] is not None:
        # The whole job's rate at the method's minimum of 72 B per lattice update, observables
        # and launch gaps included.
        gbs = mlups * SWEEP_BYTES_PER_NODE / 1e3
        out["roofline"]["whole_job"] = {
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
                              "roofline": roofline(alt, ev2, alt_launch, nodes, args)}
    del rho0
    torch.cuda.empty_cache()
    if not args.no_small:
        out["small_configs"] = small_configs_leg(lbm, args, torch)
        say(f"small configs: {json.dumps(out['small_configs'])}")
    if args.batch_steps:
        out["batch"] = batch_leg(lbm, args.batch_steps)
        say(f"batch: {out['batch']['GLUPS']} GLUPS, {out['batch']['us_per_step']} us per step")
    # the library's Python helpers report progress on stdout; the JSON line stays alone there
    with contextlib.redirect_stdout(sys.stderr):
        if not args.no_sweep:
            out["sweep"] = sweep_leg(lbm)
            say(f"sweep to equilibrium: {out['sweep']['wall_s']} s")
        if not args.no_warm_start:
            out["warm_start"] = warm_start_leg(lbm)
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
