#!/usr/bin/env python3
"""Benchmark of the tree-gravity hot path on one MI355X.

One step = one pass of the whole path over the workload: half kick, drift,
tree build (cube, Morton keys, radix sort, gather, octree, groups), moments,
group walk with P2P/P2M sums for every star, FP64 direct SMBH <-> star and
SMBH <-> SMBH forces, half kick.  Default workload: Dehnen gamma = 1.5 cusp,
N = 1 048 576 equal-mass stars, SMBH binary 2 x 0.005 at separation 0.01,
eps = 1e-3, theta = 0.5, leaf 8, group 64.  Inputs are seeded synthetic
draws of that model, resident in HBM before timing starts.

Prints ONE JSON line.  value = interactions/s (P2P pairs + particle-cell
pairs per second of whole-step wall time) of the mixed-precision path; the
FP64 path, forces/s, the mixed-vs-FP64 error, the walk kernel's roofline and
the CPU oracle baseline are reported beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle-cell interactions/s + forces/s at N=1M, theta=0.5; "
          "mixed vs FP64 force err")
PEAK_FP64 = 78.6      # TFLOP/s, MI355X vector FP64
PEAK_FP32 = 157.3     # TFLOP/s, MI355X vector FP32 (published, packed)
PEAK_FP32_UNPACKED = 78.6
FLOPS_P2P = 19
FLOPS_P2M = 58


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1048576)
    ap.add_argument("--leaf", type=int, default=8)
    ap.add_argument("--group", type=int, default=64)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--dt", type=float, default=1e-5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    return ap.parse_args()


class Step:
    """Device state and one full step through the C ABI."""

    def __init__(self, w, precision, leaf, group, waves, dt):
        import torch
        from paper_1507_01009_amd import binding as B
        self.B = B
        self.w = w
        self.dt = dt
        self.ctx = B.Context(w.n, leaf_size=leaf, group_size=group, precision=precision,
                             waves_per_cu=waves)
        dev = "cuda"
        f64 = torch.float64
        self.pos = torch.from_numpy(w.pos.copy()).to(dev)
        self.vel = torch.from_numpy(w.vel.copy()).to(dev)
        self.mass = torch.from_numpy(w.mass.copy()).to(dev)
        self.eps_s = torch.full((w.n,), w.eps, dtype=f64, device=dev)
        self.acc = torch.zeros((w.n, 3), dtype=f64, device=dev)
        self.pot = torch.zeros(w.n, dtype=f64, device=dev)
        self.bpos = torch.from_numpy(w.bh_pos.copy()).to(dev)
        self.bvel = torch.from_numpy(w.bh_vel.copy()).to(dev)
        self.bm = torch.from_numpy(w.bh_mass.copy()).to(dev)
        self.be = torch.from_numpy(w.bh_eps.copy()).to(dev)
        self.bacc = torch.zeros((w.bh_mass.shape[0], 3), dtype=f64, device=dev)
        self.bpot = torch.zeros(w.bh_mass.shape[0], dtype=f64, device=dev)
        self.forces()

    def forces(self):
        c, w = self.ctx, self.w
        c.build_tree(self.pos)
        c.compute_moments(self.mass)
        c.tree_forces(w.eps, w.theta, self.acc, self.pot)
        if self.bm.shape[0]:
            c.direct_fp64(self.bpos, self.bm, self.be, self.pos, self.eps_s, self.acc,
                          self.pot, accumulate=True)
            c.direct_fp64(self.pos, self.mass, self.eps_s, self.bpos, self.be, self.bacc,
                          self.bpot)
            c.direct_fp64(self.bpos, self.bm, self.be, self.bpos, self.be, self.bacc,
                          self.bpot, self_pairs=True, accumulate=True)

    def step(self):
        c, dt = self.ctx, self.dt
        c.kick(self.vel, self.acc, dt)
        c.kick(self.bvel, self.bacc, dt)
        c.drift(self.pos, self.vel, dt)
        c.drift(self.bpos, self.bvel, dt)
        self.forces()
        c.kick(self.vel, self.acc, dt)
        c.kick(self.bvel, self.bacc, dt)


def time_path(st, steps, warmup):
    import torch
    for _ in range(warmup):
        st.step()
    st.ctx.sync()
    st.ctx.reset_counts()
    st.ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    walk_ms, n_walks = st.ctx.get_profile()
    st.ctx.set_profiling(False)
    cnt = st.ctx.get_cumulative_counts()
    st.ctx.sync()
    assert n_walks == steps and cnt["n_groups"] > 0
    sec = t1 - t0
    inter = cnt["n_p2p"] + cnt["n_p2m"]
    flops = FLOPS_P2P * cnt["n_p2p"] + FLOPS_P2M * cnt["n_p2m"]
    return {
        "ms_per_step": 1e3 * sec / steps,
        "interactions_per_s": inter / sec,
        "particle_cell_per_s": cnt["n_p2m"] / sec,
        "p2p_per_s": cnt["n_p2p"] / sec,
        "forces_per_s": cnt["n_targets"] / sec,
        "interactions_per_step": inter / steps,
        "walk_ms_avg": walk_ms / n_walks,
        "walk_tflops": flops / steps / (walk_ms / n_walks * 1e-3) / 1e12,
        "flops_per_walk": flops / steps,
    }


def graph_ms(st, steps):
    """Same step captured once into a HIP graph and replayed."""
    import torch
    s = torch.cuda.Stream()
    st.ctx.set_stream(s)
    with torch.cuda.stream(s):
        st.step()
        s.synchronize()
        st.ctx.graph_begin()
        st.step()
        g = st.ctx.graph_end()
        g.launch(s)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch(s)
        s.synchronize()
        t1 = time.perf_counter()
    st.ctx.sync()
    st.ctx.set_stream(torch.cuda.current_stream())
    return 1e3 * (t1 - t0) / steps


def traffic_for(kernel_file, workload):
    """HBM bytes per walk launch from the committed rocprofv3 counter summary,
    only if the kernel source is unchanged since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "walk_counters_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = open(os.path.join(ROOT, "paper_1507_01009_amd", "csrc", kernel_file), "rb").read()
    if kv.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, leaf, group, seconds):
    """The oracle (plain C, all host threads) on a bounded sample of the same
    step: full tree build, then the walk + evaluation of random groups until
    `seconds` of work, extrapolated to all groups."""
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    tree = oracle.build_tree(w.pos, None, leaf)
    spos, smass = oracle.sorted_arrays(tree, w.pos, w.mass)
    mom = oracle.moments(tree, spos, smass)
    g = oracle.groups(tree, group)
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(1234)
    order = rng.permutation(g.shape[0])
    done, inter, t_walk = 0, 0, 0.0
    chunk = max(64, 4 * threads)
    while done < order.size and t_walk < seconds:
        sel = np.sort(order[done:done + chunk])
        t1 = time.perf_counter()
        ev = oracle.tree_forces(w.pos, w.mass, w.eps, w.theta, leaf, group,
                                sel_groups=sel, tree=tree)
        t_walk += time.perf_counter() - t1
        inter += ev.n_p2p + ev.n_p2m
        done += sel.size
        chunk = min(chunk * 2, 4096)
    frac = done / g.shape[0]
    t_step = t_build + t_walk / frac
    return {"value": (inter / frac) / t_step, "unit": "interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": "full oracle tree build (%.1f s) + walk/evaluation of %d of %d groups "
                      "(random, %.1f s), extrapolated to the whole step" % (
                          t_build, done, g.shape[0], t_walk),
            "step_seconds_est": t_step}


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: this build runs on exactly one GPU (requested %d); "
              "multi-GPU sharding is design-only" % max(a.gpus, world), file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1507_01009_amd import binding as B, ics
    torch.cuda.set_device(0)
    log("bench: generating workload N=%d" % a.n)
    w = ics.cusp_c3(n=a.n)
    res = {}
    paths = ["mixed", "fp64"] if a.only == "both" else [a.only]
    accs = {}
    for name in paths:
        prec = B.TG_MIXED if name == "mixed" else B.TG_FP64
        log("bench: %s path" % name)
        st = Step(w, prec, a.leaf, a.group, a.waves, a.dt)
        st.ctx.sync()
        accs[name] = st.acc.cpu().numpy().copy()
        r = time_path(st, a.steps, a.warmup)
        r["graph_ms_per_step"] = graph_ms(st, max(3, a.steps // 2))
        res[name] = r
        log("bench: %s %.3f ms/step, %.3g interactions/s, walk %.3f ms (%.2f TFLOP/s)" % (
            name, r["ms_per_step"], r["interactions_per_s"], r["walk_ms_avg"],
            r["walk_tflops"]))
        del st
        torch.cuda.empty_cache()
    err = None
    if "mixed" in accs and "fp64" in accs:
        e = np.linalg.norm(accs["mixed"] - accs["fp64"], axis=1) / np.linalg.norm(accs["fp64"], axis=1)
        err = {"mixed_vs_fp64": {"p50": float(np.median(e)), "p90": float(np.percentile(e, 90)),
                                 "p99": float(np.percentile(e, 99)),
                                 "p999": float(np.percentile(e, 99.9)), "max": float(e.max())}}
    head = res["mixed"] if "mixed" in res else res["fp64"]
    head_name = "mixed" if "mixed" in res else "fp64"
    peak = PEAK_FP32 if head_name == "mixed" else PEAK_FP64
    roof = {"bound": "alu", "achieved": head["walk_tflops"], "peak": peak, "unit": "TFLOP/s",
            "frac": head["walk_tflops"] / peak,
            "traffic": traffic_for("k_walk.hip", "cusp1m"),
            "kernel": "k_walk_forces<%s>" % ("true" if head_name == "mixed" else "false"),
            "avg_launch_ms": head["walk_ms_avg"], "flops_per_launch": head["flops_per_walk"],
            "flops_per_interaction": {"p2p": FLOPS_P2P, "p2m": FLOPS_P2M},
            "peak_note": "published FP32 vector peak; the build disables packed FP32, "
                         "whose unpacked rate is %.1f TFLOP/s" % PEAK_FP32_UNPACKED
                         if head_name == "mixed" else "FP64 vector peak"}
    out = {
        "metric": METRIC, "value": head["interactions_per_s"], "unit": "interactions/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-walk/f64-state" if head_name == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "n_smbh": int(w.bh_mass.shape[0]),
                   "theta": w.theta, "eps": w.eps, "leaf_size": a.leaf,
                   "group_size": a.group, "precision": head_name, "dt": a.dt},
        "forces_per_s": head["forces_per_s"],
        "particle_cell_interactions_per_s": head["particle_cell_per_s"],
        "p2p_interactions_per_s": head["p2p_per_s"],
        "interactions_per_step": head["interactions_per_step"],
        "graph_ms_per_step": head["graph_ms_per_step"],
        "paths": res, "error": err, "roofline": roof,
    }
    if a.copy_mib:
        src = torch.ones(a.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * src.numel() * 4
        del src, dst
    if not a.no_cpu:
        log("bench: CPU oracle baseline (~%.0f s)" % a.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(w, a.leaf, a.group, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
