"""Learned warm start for the batched droplet sweep.

A small network (4 -> 128 -> 128 -> 128 -> 64, tanh, FP32, the library's own GPU forward,
backward and Adam kernels) maps a droplet's (T/Tc, tau, R, K) to its equilibrium radial density
profile: log rho at 64 radii around the initial radius, r_k = R + 2 (k - 23.5), from 47 nodes
inside the interface to 79 outside.  It is trained on equilibria that the batched sweep itself
produces from plain tanh initial states.
At run time its profile is expanded on the device, shifted radially so that its total mass
equals that of the tanh state it replaces (in a periodic box the mass fixes the equilibrium),
and set at physical rest (f = f^eq(rho, -F/(2 rho))); the tanh state is the fallback when a
prediction is not a valid density.  Both runs stop on the same tolerances (velocity change and
probe-density change per step); a longer, tighter run from the tanh state gives the converged
density ratio that the two are measured against.

    python -m paper_1412_5170_amd.warmstart --out results.json
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

from . import inputs, sweep

DIMS = [4, 128, 128, 128, 64]
K_RANGE = (1 / 49, 1 / 10)
_HERE = os.path.dirname(os.path.abspath(__file__))
# The trained network (weights only: params, mean, std) and the record of its training draw.
NET_PATH = os.path.join(_HERE, "warmstart_net.npz")
NET_MANIFEST = os.path.join(_HERE, "warmstart_net.json")
# Per-member step budgets of the 64-lattice sweep at equal density-ratio accuracy (written by
# `--equal-accuracy --record`), with the converged ratios they were measured against.
EQUAL_ACCURACY_PATH = os.path.join(_HERE, "warmstart_equal_accuracy.json")


def say(*a):
    print(*a, flush=True)


def features(m):
    """(T/Tc, tau, R, K) scaled to about [-1, 1]: R through the curvature (48/R - 1, which
    stays bounded for large droplets), K on a log scale."""
    return np.array([(m["T_over_Tc"] - 0.7) / 0.2,
                     (m["tau"] - 1.05) / 0.45,
                     48.0 / m["R"] - 1.0,
                     (math.log(m["K"]) - 0.5 * math.log(K_RANGE[0] * K_RANGE[1]))
                     / (0.5 * math.log(K_RANGE[1] / K_RANGE[0]))], dtype=np.float32)


def draw_training(seed, count, n_min=96, n_step=16, n_levels=19, K=None, ttc_range=(0.5, 0.9)):
    """Training droplets drawn like the sweep, with K log-uniform in K_RANGE (or every member
    at the given K)."""
    draw = inputs.batch_draw(seed, count=count, n_min=n_min, n_step=n_step, n_levels=n_levels,
                             ttc_range=ttc_range)
    rng = np.random.default_rng(seed + 7919)
    ms = sweep.members_from_draw(draw)
    for m in ms:
        m["K"] = float(K) if K is not None else float(
            math.exp(rng.uniform(math.log(K_RANGE[0]), math.log(K_RANGE[1]))))
    return ms


def equilibria(lbm, members, tol, check_every=500, max_steps=400_000, batch_size=64,
               tol_rho=0.0):
    """Run members to equilibrium from tanh states, in batches of similar size; returns the
    radial log-density profiles, steps and statuses (in the members' order)."""
    order = sorted(range(len(members)), key=lambda i: members[i]["nx"] * members[i]["ny"])
    prof = np.full((len(members), sweep.PROFILE_POINTS), np.nan, dtype=np.float32)
    steps = np.zeros(len(members), dtype=np.int64)
    status = np.zeros(len(members), dtype=np.int64)
    t0 = time.perf_counter()
    for c in range(0, len(order), batch_size):
        idx = order[c:c + batch_size]
        ms = [members[i] for i in idx]
        dens = [sweep.tanh_density(lbm, m) for m in ms]
        wall, st, stat, b = sweep.run_batch(
            lbm, ms, dens, tol=tol, check_every=check_every, max_steps=max_steps,
            tol_rho=tol_rho, chunk=20_000,
            report=lambda t, c=c: say(f"warmstart: equilibria from {c}: {t}"))
        for j, i in enumerate(idx):
            steps[i], status[i] = st[j], stat[j]
            if stat[j] == 0:
                rho, _ = b.read(j)
                prof[i] = sweep.radial_profile(ms[j], rho)
        del b
        say(f"warmstart: equilibria {c + len(idx)}/{len(members)} (batch {wall:.1f} s, "
            f"max steps {max(st)}, total {time.perf_counter() - t0:.1f} s)")
    return prof, steps, status


class Surrogate:
    """The network plus the output standardisation learned from its training set."""

    def __init__(self, lbm, seed=0):
        self.lbm = lbm
        self.net = lbm.MLP(DIMS, seed=seed)
        self.mean = np.zeros(DIMS[-1], dtype=np.float32)
        self.std = np.ones(DIMS[-1], dtype=np.float32)

    def fit(self, X, Y, steps=6000, lr=1e-3, batch=256, seed=0, val_frac=0.1):
        import torch
        rng = np.random.default_rng(seed)
        perm = rng.permutation(len(X))
        nval = max(1, int(val_frac * len(X)))
        val, tr = perm[:nval], perm[nval:]
        self.mean = Y[tr].mean(axis=0).astype(np.float32)
        self.std = (Y[tr].std(axis=0) + 1e-6).astype(np.float32)
        Xt = torch.from_numpy(X[tr]).cuda()
        Yt = torch.from_numpy(((Y[tr] - self.mean) / self.std).astype(np.float32)).cuda()
        loss = None
        for k in range(steps):
            sel = torch.from_numpy(rng.integers(0, len(tr), size=min(batch, len(tr)))).cuda()
            rate = lr * (0.5 * (1 + math.cos(math.pi * k / steps)) * 0.99 + 0.01)
            loss = self.net.train_step(Xt[sel].contiguous(), Yt[sel].contiguous(), rate)
            if k % 1000 == 0:
                say(f"warmstart: train step {k}/{steps} loss {loss:.3e}")
        pred = self.predict_log(X[val])
        val_rmse = float(np.sqrt(np.mean((pred - Y[val]) ** 2)))
        return {"train_loss_std_units": loss, "val_rmse_log_rho": val_rmse, "n_train": len(tr),
                "n_val": int(nval)}

    def predict_log(self, X):
        import torch
        y = self.net.forward(torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda())
        return y.cpu().numpy() * self.std + self.mean

    def warm_start(self, lbm, m):
        """The learned initial state of member m: its predicted profile, to be shifted on the
        device to the mass of the tanh state it replaces (in a periodic box the mass fixes the
        equilibrium), with that tanh state as the fallback."""
        plain = sweep.tanh_density(lbm, m)
        prof = self.predict_log(features(m)[None])[0]
        if not np.all(np.isfinite(prof)):
            return plain
        return sweep.WarmStart(prof, m["R"], plain.sum(), plain)


def net_digest(path=NET_PATH):
    """Short hash of a saved network file (ties results to the weights they came from)."""
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def load_surrogate(lbm, path=NET_PATH):
    """The trained network from a weights-only file (no pickled objects)."""
    d = np.load(path, allow_pickle=False)
    sur = Surrogate(lbm, seed=0)
    sur.net.set_params(d["params"])
    sur.mean, sur.std = d["mean"].astype(np.float32), d["std"].astype(np.float32)
    return sur


def _start(lbm, sur, members, mode):
    if mode == "learned":
        return [sur.warm_start(lbm, m) for m in members]
    return [sweep.tanh_density(lbm, m) for m in members]


def _batch(lbm, members, inits):
    b = lbm.Batch(members)
    fallback = 0
    for i, init in enumerate(inits):
        if isinstance(init, sweep.WarmStart):
            try:
                b.init_profile(i, init.log_profile, init.r0, init.dr, init.mass)
                continue
            except lbm.LBMError:
                fallback += 1
                init = init.fallback
        b.init_rest(i, init)
    b.sync()
    return b, fallback


def trajectories(lbm, members, inits, tol, tol_rho, check_every, max_steps, label):
    """Run every member until it meets the stopping rule (as lbm_batch_run: velocity change and
    probe-density change per step below tol, tol_rho), recording the probe density ratio at
    every check.  Returns per-member lists of (step, ratio) and the final ratios."""
    b, _ = _batch(lbm, members, inits)
    n = len(members)
    hist = [[] for _ in range(n)]
    prev = b.stats(track_dv=True)
    active = [True] * n
    t0, last = time.perf_counter(), time.perf_counter()
    while any(active):
        b.step(check_every)
        st = b.stats(track_dv=True)
        for i in range(n):
            if not active[i]:
                continue
            a, c = st[i]["rho_probe_a"], st[i]["rho_probe_b"]
            hist[i].append((st[i]["step"], a / c))
            dr = max(abs(a - prev[i]["rho_probe_a"]) / a,
                     abs(c - prev[i]["rho_probe_b"]) / c) / check_every
            done = st[i]["nonfinite"] or (st[i]["dv_max"] / check_every < tol and dr < tol_rho)
            if done or st[i]["step"] >= max_steps:
                active[i] = False
                b.set_active(i, 0)
        prev = st
        if time.perf_counter() - last > 20:
            last = time.perf_counter()
            say(f"warmstart {label}: {sum(active)} running, step {max(h[-1][0] for h in hist)}, "
                f"{last - t0:.0f} s")
    del b
    return hist, [h[-1][1] for h in hist]


def time_to_accuracy(hist, ref, eps):
    """First recorded step from which |ratio - ref| / ref stays below eps to the end."""
    for k in range(len(hist)):
        if all(abs(r - ref) / ref < eps for _, r in hist[k:]):
            return hist[k][0]
    return hist[-1][0]


def budgeted(lbm, members, inits, budgets, check_every, label):
    """Timed run in which member i stops after budgets[i] steps (a multiple of check_every)."""
    b, fallback = _batch(lbm, members, inits)
    n = len(members)
    active = [True] * n
    steps = 0
    t0 = time.perf_counter()
    while any(active):
        b.step(check_every)
        steps += check_every
        for i in range(n):
            if active[i] and steps >= budgets[i]:
                active[i] = False
                b.set_active(i, 0)
    b.sync()
    wall = time.perf_counter() - t0
    ratios = []
    for i, m in enumerate(members):
        rho, _ = b.read(i)
        ratios.append(float(rho[m["ny"] // 2, m["nx"] // 2] / rho[0, 0]))
    del b
    lu = sum(m["nx"] * m["ny"] * bb for m, bb in zip(members, budgets))
    say(f"warmstart {label}: budgeted run {wall:.1f} s, {lu / 1e9:.0f} G lattice updates")
    return wall, lu, ratios, fallback


def equal_accuracy(lbm, sur, members, eps=1e-4, tol=2.5e-10, tol_rho=5e-10, check_every=500,
                   max_steps=1_500_000):
    """Wall time to the same density-ratio accuracy: trajectories from both starts under a
    stopping rule 4x tighter than the sweep's give the converged ratio (their mean; their
    difference bounds its uncertainty) and, per member and start, the first step from which the
    ratio stays within eps of it; then each start runs timed with exactly those per-member
    step budgets."""
    res = {"eps": eps}
    hist, fin = {}, {}
    for mode in ("tanh", "learned"):
        hist[mode], fin[mode] = trajectories(lbm, members, _start(lbm, sur, members, mode), tol,
                                             tol_rho, check_every, max_steps, mode)
    ref = [(a + b) / 2 for a, b in zip(fin["tanh"], fin["learned"])]
    res["reference_spread_max"] = float(max(abs(a - b) / r for a, b, r in
                                            zip(fin["tanh"], fin["learned"], ref)))
    res["reference_ratio"] = [float(r) for r in ref]
    for mode in ("tanh", "learned"):
        budgets = [time_to_accuracy(h, r, eps) for h, r in zip(hist[mode], ref)]
        wall, lu, ratios, fb = budgeted(lbm, members, _start(lbm, sur, members, mode), budgets,
                                        check_every, mode)
        err = [abs(x - r) / r for x, r in zip(ratios, ref)]
        res[mode] = {"wall_s": round(wall, 3), "lattice_updates": int(lu),
                     "steps": [int(x) for x in budgets], "ratio_err_max": float(max(err)),
                     "ratio_err_median": float(np.median(err)), "fallbacks": fb}
    res["speedup_wall"] = res["tanh"]["wall_s"] / res["learned"]["wall_s"]
    res["speedup_updates"] = res["tanh"]["lattice_updates"] / res["learned"]["lattice_updates"]
    return res


def evaluate(lbm, sur, members, tol, tol_rho, check_every=500, max_steps=1_500_000,
             chunk=20_000, reference=True):
    """Plain (tanh) and warm-started runs of the same members from physical rest, same
    tolerances; wall time, lattice updates and the density ratio each reaches.  With
    `reference`, a third, untimed run from the tanh state with both tolerances 4x tighter over
    4x longer check windows gives the converged ratio that both are measured against."""
    res = {}
    modes = ("tanh", "learned") + (("reference",) if reference else ())
    for mode in modes:
        if mode == "learned":
            inits = [sur.warm_start(lbm, m) for m in members]
        else:
            inits = [sweep.tanh_density(lbm, m) for m in members]
        fallback = sum(not isinstance(x, sweep.WarmStart) for x in inits) if mode == "learned" else 0
        k = 4 if mode == "reference" else 1
        wall, steps, status, b = sweep.run_batch(
            lbm, members, inits, tol=tol / k, tol_rho=tol_rho / k, check_every=check_every * k,
            max_steps=max_steps, chunk=chunk, report=lambda t: say(f"warmstart {mode}: {t}"))
        fallback += b.fallbacks
        ratios = []
        for i, m in enumerate(members):
            rho, _ = b.read(i)
            ratios.append(float(rho[m["ny"] // 2, m["nx"] // 2] / rho[0, 0]))
        del b
        lu = sum(m["nx"] * m["ny"] * st for m, st in zip(members, steps))
        res[mode] = {"wall_s": round(wall, 3), "steps": [int(x) for x in steps],
                     "status": [int(x) for x in status], "ratio": ratios,
                     "lattice_updates": int(lu), "fallbacks": fallback}
        say(f"warmstart: {mode}: {wall:.2f} s, {lu / 1e9:.1f} G lattice updates, "
            f"max steps {max(steps)}, not converged {sum(int(x != 0) for x in status)}")
    rt, rl = np.array(res["tanh"]["ratio"]), np.array(res["learned"]["ratio"])
    res["ratio_rel_diff_max"] = float(np.max(np.abs(rl - rt) / rt))
    if reference:
        rr = np.array(res["reference"]["ratio"])
        et, el = np.abs(rt - rr) / rr, np.abs(rl - rr) / rr
        res["ratio_err_tanh_max"] = float(et.max())
        res["ratio_err_learned_max"] = float(el.max())
        res["ratio_err_tanh_median"] = float(np.median(et))
        res["ratio_err_learned_median"] = float(np.median(el))
    res["speedup_wall"] = res["tanh"]["wall_s"] / res["learned"]["wall_s"]
    res["speedup_updates"] = res["tanh"]["lattice_updates"] / res["learned"]["lattice_updates"]
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-count", type=int, default=2000)
    ap.add_argument("--train-tol", type=float, default=1e-9)
    ap.add_argument("--train-tol-rho", type=float, default=2e-9)
    ap.add_argument("--train-levels", type=int, default=19, help="sizes 96 + 16 k, k < levels")
    ap.add_argument("--train-steps", type=int, default=100000)
    ap.add_argument("--train-seed", type=int, default=0,
                    help="seed of the validation split and the minibatch draws")
    ap.add_argument("--train-large-count", type=int, default=64,
                    help="extra training droplets of sizes 512 + 16 k, k < 33 (the sweep's largest)")
    ap.add_argument("--train-sweep-k-count", type=int, default=0,
                    help="extra training droplets of sizes 384 + 16 k, k < 41, all at the sweep's "
                         "own K (seed 3)")
    ap.add_argument("--train-cold-count", type=int, default=0,
                    help="extra training droplets of sizes 384 + 16 k, k < 41, at the sweep's own "
                         "K and T/Tc in [0.5, 0.65], where the densities change fastest (seed 4)")
    ap.add_argument("--eval-seed", type=int, default=0)
    ap.add_argument("--eval-count", type=int, default=64)
    ap.add_argument("--eval-levels", type=int, default=57, help="sizes 128 + 16 k, k < levels")
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--tol-rho", type=float, default=2e-9,
                    help="per-step relative change of the probe densities at convergence")
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--data", default=None, help="npz of (X, Y) to reuse instead of generating")
    ap.add_argument("--save-net", default=None, help="npz to write the trained network to")
    ap.add_argument("--load-net", default=None, help="npz of a trained network (skip training)")
    ap.add_argument("--no-eval", action="store_true")
    ap.add_argument("--equal-accuracy", action="store_true",
                    help="time both starts to the same density-ratio accuracy (eps 1e-4)")
    ap.add_argument("--record", default=None,
                    help="with --equal-accuracy: write the per-member budgets and converged "
                         "ratios (the benchmark's warm-start leg replays them)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    from . import lbm

    out = {"dims": DIMS}
    sur = Surrogate(lbm, seed=0)
    if a.load_net:
        sur = load_surrogate(lbm, a.load_net)
        out["training"] = {"loaded": a.load_net, "net_sha256_16": net_digest(a.load_net)}
    else:
        sets, out["generation"] = [], []
        if a.data:
            d = np.load(a.data)
            sets.append((d["X"], d["Y"]))
        draws = [] if a.data else [draw_training(1, a.train_count, n_levels=a.train_levels)]
        if a.train_large_count > 0:
            draws.append(draw_training(2, a.train_large_count, n_min=512, n_levels=33))
        if a.train_sweep_k_count > 0:
            draws.append(draw_training(3, a.train_sweep_k_count, n_min=384, n_levels=41,
                                       K=sweep.PHYSICS["K"]))
        if a.train_cold_count > 0:
            draws.append(draw_training(4, a.train_cold_count, n_min=384, n_levels=41,
                                       K=sweep.PHYSICS["K"], ttc_range=(0.5, 0.65)))
        for tr in draws:
            t0 = time.perf_counter()
            prof, steps, status = equilibria(lbm, tr, a.train_tol, tol_rho=a.train_tol_rho)
            ok = status == 0
            sets.append((np.stack([features(m) for m in tr])[ok], prof[ok]))
            out["generation"].append({"members": len(tr), "converged": int(ok.sum()),
                                      "sizes": [min(m["nx"] for m in tr), max(m["nx"] for m in tr)],
                                      "wall_s": round(time.perf_counter() - t0, 1),
                                      "tol": a.train_tol, "lattice_updates": int(sum(
                                          m["nx"] * m["ny"] * st for m, st in zip(tr, steps)))})
        X = np.concatenate([x for x, _ in sets])
        Y = np.concatenate([y for _, y in sets])
        if a.out and draws:
            np.savez(a.out.replace(".json", "") + "_data.npz", X=X, Y=Y)
        t0 = time.perf_counter()
        out["training"] = sur.fit(X, Y, steps=a.train_steps, seed=a.train_seed)
        out["training"]["wall_s"] = round(time.perf_counter() - t0, 1)
        if a.save_net:
            np.savez(a.save_net, params=sur.net.get_params(), mean=sur.mean, std=sur.std)
    say(json.dumps(out))
    if a.equal_accuracy:
        ev = sweep.members_from_draw(inputs.batch_draw(a.eval_seed, count=a.eval_count,
                                                       n_levels=a.eval_levels))
        out["equal_accuracy"] = equal_accuracy(lbm, sur, ev)
        e = out["equal_accuracy"]
        if a.record:
            rec = {"eps": e["eps"], "seed": a.eval_seed, "count": a.eval_count,
                   "levels": a.eval_levels, "check_every": 500,
                   "net_sha256_16": net_digest(a.load_net) if a.load_net else None,
                   "reference_ratio": e["reference_ratio"],
                   "reference_spread_max": e["reference_spread_max"],
                   "budgets": {m: e[m]["steps"] for m in ("tanh", "learned")},
                   "measured": {m: {k: e[m][k] for k in ("wall_s", "lattice_updates",
                                                         "ratio_err_max")}
                                for m in ("tanh", "learned")},
                   "members": [{k: m[k] for k in ("nx", "T_over_Tc", "tau", "collision")}
                               for m in ev]}
            with open(a.record, "w") as fh:
                json.dump(rec, fh, indent=1)
        say(json.dumps({k: e[k] for k in ("eps", "reference_spread_max", "speedup_wall",
                                          "speedup_updates")}
                       | {m: {k: e[m][k] for k in ("wall_s", "lattice_updates", "ratio_err_max",
                                                   "ratio_err_median")}
                          for m in ("tanh", "learned")}))
    elif not a.no_eval:
        ev = sweep.members_from_draw(inputs.batch_draw(a.eval_seed, count=a.eval_count,
                                                       n_levels=a.eval_levels))
        out["evaluation"] = evaluate(lbm, sur, ev, a.tol, a.tol_rho,
                                     reference=not a.no_reference)
        out["evaluation"]["members"] = [{k: m[k] for k in ("nx", "T_over_Tc", "tau", "collision")}
                                        for m in ev]
        e = out["evaluation"]
        say(json.dumps({k: e[k] for k in ("speedup_wall", "speedup_updates",
                                          "ratio_rel_diff_max", "ratio_err_tanh_max",
                                          "ratio_err_learned_max", "ratio_err_tanh_median",
                                          "ratio_err_learned_median") if k in e}
                       | {"tanh_wall_s": e["tanh"]["wall_s"],
                          "learned_wall_s": e["learned"]["wall_s"]}))
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(out, fh)


if __name__ == "__main__":
    main(sys.argv[1:])
