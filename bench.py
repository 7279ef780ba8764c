#!/usr/bin/env python3
"""Benchmark of the tree-gravity hot path on one MI355X.

One step = one native kick-drift-kick call (tg_step_kdk): half kick, drift,
tree build (cube, Morton keys, radix sort, gather, octree, groups), moments,
group walk with P2P/P2M sums for every star (FP64 SMBH terms added per
star), FP64 direct SMBH <- star and SMBH <-> SMBH forces, half kick.
Default workload: Dehnen gamma = 1.5 cusp, N = 1 048 576 equal-mass stars,
SMBH binary 2 x 0.005 at separation 0.01, eps = 1e-3, theta = 0.5, leaf 8,
group 64.  Inputs are seeded synthetic draws of that model, resident in HBM
before timing starts.

Prints ONE JSON line.  value = interactions/s (P2P pairs + particle-cell
pairs per second of whole-step wall time) of the mixed-precision path; the
FP64 path, forces/s, the errors (mixed vs FP64, both vs the direct sum), the
walk kernel's roofline and the CPU oracle baseline are reported beside it,
plus measurements selected by --extras (default all, none with --no-extra):
the relative opening test (alpha = 1e-3) and the spline softening on the
same step, the chain coupling on the same workload, the hybrid step with
one chain, a KDK energy check, block steps and batched realisations.
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
FLOPS_P2M = 54


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
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--extras", default="relative,spline,chain,hybrid,kdk,blocksteps,batch",
                    help="comma list of the extra measurements to run")
    ap.add_argument("--only", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    return ap.parse_args()


def percentiles(e):
    import numpy as np
    return {"p50": float(np.median(e)), "p90": float(np.percentile(e, 90)),
            "p99": float(np.percentile(e, 99)), "p999": float(np.percentile(e, 99.9)),
            "max": float(e.max())}


class DevState:
    """A workload resident in HBM and its tg_system view (native steps)."""

    def __init__(self, ctx, w):
        import numpy as np
        import torch
        f64 = dict(dtype=torch.float64, device="cuda")
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
        self.w = w
        self.pos, self.vel, self.mass = t(w.pos), t(w.vel), t(w.mass)
        self.acc = torch.zeros((w.n, 3), **f64)
        self.pot = torch.zeros(w.n, **f64)
        nb = w.bh_mass.shape[0]
        self.nb = nb
        self.bpos, self.bvel = t(w.bh_pos.reshape(-1, 3)), t(w.bh_vel.reshape(-1, 3))
        self.bm, self.be = t(w.bh_mass), t(w.bh_eps)
        self.bacc = torch.zeros((max(nb, 1), 3), **f64)
        self.bpot = torch.zeros(max(nb, 1), **f64)
        S = w.sys_off.shape[0] - 1
        bseg = np.zeros(S + 1, np.int64)
        for s in range(S):
            bseg[s + 1] = bseg[s] + int((w.bh_sys == s).sum())
        self.bseg = bseg
        self.sys = self.view(ctx, 0, w.n, 0, nb, w.sys_off if S > 1 else None,
                             bseg if nb else None)

    def view(self, ctx, lo, hi, blo, bhi, sys_off=None, bseg=None):
        """tg_system over stars [lo, hi) and SMBHs [blo, bhi) (slices)."""
        w = self.w
        nb = bhi - blo
        return ctx.make_system(
            self.pos[lo:hi], self.vel[lo:hi], self.acc[lo:hi], self.mass[lo:hi], w.eps,
            w.theta, pot=self.pot[lo:hi], sys_off=sys_off,
            bh_pos=self.bpos[blo:bhi] if nb else None,
            bh_vel=self.bvel[blo:bhi] if nb else None,
            bh_acc=self.bacc[blo:bhi] if nb else None,
            bh_mass=self.bm[blo:bhi] if nb else None,
            bh_eps=self.be[blo:bhi] if nb else None,
            bh_pot=self.bpot[blo:bhi] if nb else None, bh_seg=bseg)

    def energy(self):
        """Kinetic + potential energy of stars and SMBHs (pot includes G)."""
        m, v, p = self.mass.cpu().numpy(), self.vel.cpu().numpy(), self.pot.cpu().numpy()
        e = 0.5 * (m * (v * v).sum(1)).sum() + 0.5 * (m * p).sum()
        if self.nb:
            bm = self.bm.cpu().numpy()
            bv = self.bvel.cpu().numpy()[:self.nb]
            bp = self.bpot.cpu().numpy()[:self.nb]
            e += 0.5 * (bm * (bv * bv).sum(1)).sum() + 0.5 * (bm * bp).sum()
        return float(e)


class Step:
    """The benchmark step: one native kick-drift-kick call (tg_step_kdk)."""

    def __init__(self, w, precision, leaf, group, waves, dt):
        from paper_1507_01009_amd import binding as B
        self.w = w
        self.dt = dt
        self.ctx = B.Context(w.n, leaf_size=leaf, group_size=group, precision=precision,
                             waves_per_cu=waves)
        self.d = DevState(self.ctx, w)
        self.ctx.forces(self.d.sys)
        self.acc = self.d.acc

    def step(self):
        self.ctx.step_kdk(self.d.sys, self.dt)


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


def graph_ms(ctx, step, steps):
    """The same step captured once into a HIP graph and replayed."""
    import torch
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    ctx.set_stream(s)
    with torch.cuda.stream(s):
        step()
        s.synchronize()
        ctx.graph_begin()
        step()
        g = ctx.graph_end()
        g.launch(s)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch(s)
        s.synchronize()
        t1 = time.perf_counter()
    ctx.sync()
    ctx.set_stream(torch.cuda.current_stream())
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


def direct_errors(w, accs, n_samples=4096, softening="plummer"):
    """Per-percentile error of each path against the oracle's exact direct
    sum (stars and SMBHs, long double accumulation) on seeded sample
    targets: the reference the reported error percentiles rest on."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(99)
    tg = np.sort(rng.choice(w.n, min(n_samples, w.n), replace=False))
    ref, _ = oracle.direct(w.pos, w.mass, w.eps, tg, xpos=w.bh_pos, xmass=w.bh_mass,
                           xeps=w.bh_eps, softening=softening)
    out = {}
    for name, a in accs.items():
        e = np.linalg.norm(a[tg] - ref, axis=1) / np.linalg.norm(ref, axis=1)
        out[name + "_vs_direct_sum"] = percentiles(e)
    out["direct_sum_samples"] = int(tg.size)
    out["direct_sum_reference"] = (
        "oracle long-double direct sum over all stars and SMBHs, %d seeded targets, "
        "%d host threads" % (tg.size, oracle.max_threads()))
    return out


def direct_errors_gpu(w, accs, n_samples=65536, softening="plummer"):
    """Per-percentile error of each path against the FP64 direct sum (stars
    and SMBHs, compensated, tg_direct_fp64, itself parity-tested against the
    oracle) on seeded sample targets.  A target's own pair adds no force."""
    import numpy as np
    import torch
    from paper_1507_01009_amd import binding as B
    rng = np.random.default_rng(98)
    tg = np.sort(rng.choice(w.n, min(n_samples, w.n), replace=False))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    ctx = B.Context(w.n)
    ctx.set_softening(softening)
    pos, m = dev(w.pos), dev(w.mass)
    seps = torch.full((w.n,), w.eps, dtype=torch.float64, device="cuda")
    tpos = dev(w.pos[tg])
    teps = torch.full((tg.size,), w.eps, dtype=torch.float64, device="cuda")
    acc = torch.zeros((tg.size, 3), dtype=torch.float64, device="cuda")
    ctx.direct_fp64(pos, m, seps, tpos, teps, acc)
    if w.bh_mass.shape[0]:
        ctx.direct_fp64(dev(w.bh_pos.reshape(-1, 3)), dev(w.bh_mass), dev(w.bh_eps), tpos, teps,
                        acc, accumulate=True)
    ctx.sync()
    ref = acc.cpu().numpy()
    ctx.close()
    out = {}
    for name, a in accs.items():
        e = np.linalg.norm(a[tg] - ref, axis=1) / np.linalg.norm(ref, axis=1)
        out[name + "_vs_direct_sum_fp64_gpu"] = percentiles(e)
    out["direct_sum_fp64_gpu_samples"] = int(tg.size)
    out["direct_sum_fp64_gpu_reference"] = (
        "tg_direct_fp64 (compensated FP64 on the GPU) on %d seeded targets; its parity "
        "with the oracle's long-double sum at all 1M sources is a GPU test" % tg.size)
    return out


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
    oracle.moments(tree, spos, smass)
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
    # the same walk on one thread, a smaller random sample
    oracle.set_threads(1)
    sel = np.sort(order[:256])
    t1 = time.perf_counter()
    ev = oracle.tree_forces(w.pos, w.mass, w.eps, w.theta, leaf, group, sel_groups=sel,
                            tree=tree)
    t_one = time.perf_counter() - t1
    oracle.set_threads(threads)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": (inter / frac) / t_step, "unit": "interactions/s", "cores": threads,
            "kind": "oracle",
            "sample": "full oracle tree build (%.1f s) + walk/evaluation of %d of %d groups "
                      "(random, %.1f s), extrapolated to the whole step" % (
                          t_build, done, g.shape[0], t_walk),
            "step_seconds_est": t_step, "build_seconds": t_build,
            "walk_interactions_per_s": inter / t_walk,
            "walk_interactions_per_s_1thread": (ev.n_p2p + ev.n_p2m) / t_one,
            "sample_1thread": "256 random groups on one thread (%.1f s)" % t_one,
            "host_cpu": model, "host_nproc": os.cpu_count()}


# ---------------------------------------------------------------- extras
def extra_relative_mac(w, a, alpha=1e-3, steps=10):
    """The paper's own opening test on the same workload and step: the
    relative criterion with tolerance alpha (the runs' 1e-3), old
    accelerations from the previous evaluation (the first from the opening
    angle).  Returns the timing and the forces at the initial positions."""
    from paper_1507_01009_amd import binding as B
    st = Step(w, B.TG_MIXED, a.leaf, a.group, a.waves, a.dt)
    st.ctx.set_mac(True, alpha)
    st.ctx.forces(st.d.sys)
    st.ctx.sync()
    acc = st.acc.cpu().numpy().copy()
    r = time_path(st, steps, 2)
    r["alpha"] = alpha
    st.ctx.close()
    return r, acc


def extra_spline(w, a, steps=10):
    """The tree's other softening (Sec. 2): the cubic spline, h = eps, on the
    same workload and step, mixed precision; the FP64 path evaluated once for
    the precision error; both against the FP64 spline direct sum."""
    import numpy as np
    from paper_1507_01009_amd import binding as B
    accs = {}
    for name, prec in (("fp64", B.TG_FP64), ("mixed", B.TG_MIXED)):
        st = Step(w, prec, a.leaf, a.group, a.waves, a.dt)
        st.ctx.set_softening("spline")
        st.ctx.forces(st.d.sys)
        st.ctx.sync()
        accs["spline_" + name] = st.acc.cpu().numpy().copy()
        if name == "mixed":
            r = time_path(st, steps, 2)
            for k in ("walk_tflops", "flops_per_walk"):   # Plummer flop counts
                r.pop(k)
        st.ctx.close()
        del st
    e = (np.linalg.norm(accs["spline_mixed"] - accs["spline_fp64"], axis=1) /
         np.linalg.norm(accs["spline_fp64"], axis=1))
    r["error"] = {"mixed_vs_fp64": percentiles(e)}
    if not a.no_cpu:
        r["error"].update(direct_errors(w, accs, 1024, softening="spline"))
    r["error"].update(direct_errors_gpu(w, accs, softening="spline"))
    r["softening"] = "cubic spline, h = eps"
    return r


def extra_chain(w, reps=50):
    """Chain coupling on the same workload: both SMBHs and the 30 stars
    nearest to their centre form the chain (the stars stay as excluded
    ghosts), r_crit = 0.01, gamma_crit = 1e-4.  Times the perturber
    selection alone, the whole coupling (selection, star terms, member
    forces, the chain particle with Eq. 3) and the host AR-chain over ten
    tree steps of 1e-5 with the perturbers gathered on the GPU."""
    import numpy as np
    import torch
    from paper_1507_01009_amd import binding as B
    r = np.linalg.norm(w.pos, axis=1)
    ghosts = np.sort(np.argsort(r)[:30])
    mpos = np.concatenate([w.bh_pos.reshape(-1, 3), w.pos[ghosts]])
    mmass = np.concatenate([w.bh_mass, w.mass[ghosts]])
    M, S = 0.0, np.zeros(3)
    for i in range(mmass.size):
        M += mmass[i]
        S += mmass[i] * mpos[i]
    excl = np.zeros(w.n, np.uint8)
    excl[ghosts] = 1
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    f64 = dict(dtype=torch.float64, device="cuda")
    ctx = B.Context(w.n)
    pos, mass, dm, dmm, dex = t(w.pos), t(w.mass), t(mpos), t(mmass), t(excl)
    idx = torch.zeros(8192, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    ch = ctx.make_chain(pos, mass, dm, dmm, S / M, M, 0.01, 1e-4, idx, cnt, exclude=dex)
    acc, pot = torch.zeros((w.n, 3), **f64), torch.zeros(w.n, **f64)
    com, macc = torch.zeros(3, **f64), torch.zeros((mmass.size, 3), **f64)
    out = {"members": int(mmass.size)}
    for name, fn in (("perturbers", lambda: ctx.perturbers(ch)),
                     ("chain_forces", lambda: ctx.chain_forces(ch, acc, com, macc, pot=pot))):
        fn()
        ctx.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        out[name + "_us"] = 1e3 * e0.elapsed_time(e1) / reps
    ctx.sync()
    out["n_perturbers"] = int(cnt.cpu().numpy()[0])
    # selection: position, mass, exclusion flag read, 1-byte flag written,
    # then the flags read again by the compaction
    out["select_bytes_per_star"] = 24 + 8 + 1 + 1 + 1
    out["select_GBps_whole_call"] = w.n * 35 / (out["perturbers_us"] * 1e-6) / 1e9
    # one chain step on the host: the perturbers relative to the chain
    # particle (GPU gather), then the AR-chain over one tree step
    npert = min(out["n_perturbers"], idx.shape[0])
    mvel = np.concatenate([w.bh_vel.reshape(-1, 3), w.vel[ghosts]])
    V = (mmass[:, None] * mvel).sum(0) / M
    px, pv = torch.zeros((8192, 3), **f64), torch.zeros((8192, 3), **f64)
    pm = torch.zeros(8192, **f64)
    ctx.predict_perturbers(ch, t(w.vel), V, 0.0, px, pv, pm)
    ctx.sync()
    px, pv, pm = (a.cpu().numpy()[:npert] for a in (px, pv, pm))
    chain = B.ARChain(mpos - S / M, mvel - V, mmass)
    t0 = time.perf_counter()
    nsteps = 0
    for _ in range(10):
        nsteps += chain.advance(1e-5, tol=1e-12, px=px, pv=pv, pm=pm)
    out["archain_ms_per_tree_step"] = 1e3 * (time.perf_counter() - t0) / 10
    out["archain_bs_steps_per_tree_step"] = nsteps / 10
    out["archain_energy_error"] = chain.energy_error()
    out["archain_tree_step"] = 1e-5
    ctx.close()
    return out


def extra_chains(n_each=524288, reps=50):
    """Several chains: two Dehnen gamma = 1.5 cusps (N = 524 288 each, scale
    0.2) 1.0 apart, each with an SMBH of 0.01 whose chain holds it and the 20
    nearest stars (excluded ghosts), r_crit = 0.005, gamma_crit = 1e-4.
    Times tg_chains_forces for both chains against two single-chain calls."""
    import numpy as np
    import torch
    from paper_1507_01009_amd import binding as B, ics
    parts, masses, specs, ghosts = [], [], [], []
    for k, (c, seed) in enumerate(((np.array([0.5, 0.0, 0.0]), 31),
                                   (np.array([-0.5, 0.1, 0.0]), 32))):
        p, _, m = ics.dehnen(n_each, 1.5, ics.SEED_BASE + seed)
        p = p * 0.2 + c
        near = np.argsort(np.linalg.norm(p - c, axis=1))[:20]
        ghosts.append(near + k * n_each)
        mpos = np.concatenate([c[None, :], p[near]])
        mmass = np.concatenate([[0.01], m[near]])
        M = mmass.sum()
        specs.append((mpos, mmass, (mmass[:, None] * mpos).sum(0) / M, M))
        parts.append(p)
        masses.append(m)
    pos, mass = np.concatenate(parts), np.concatenate(masses)
    n = pos.shape[0]
    excl = np.zeros(n, np.uint8)
    excl[np.concatenate(ghosts)] = 1
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    f64 = dict(dtype=torch.float64, device="cuda")
    ctx = B.Context(n)
    dpos, dmass, dex = t(pos), t(mass), t(excl)
    keep, chs = [], []
    for mpos, mmass, R, M in specs:
        dm, dmm = t(mpos), t(mmass)
        idx = torch.zeros(8192, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        keep += [dm, dmm, idx, cnt]
        chs.append(ctx.make_chain(dpos, dmass, dm, dmm, R, M, 0.005, 1e-4, idx, cnt,
                                  exclude=dex))
    acc, pot = torch.zeros((n, 3), **f64), torch.zeros(n, **f64)
    com, macc = torch.zeros((2, 3), **f64), torch.zeros((42, 3), **f64)
    out = {"workload": "two_dehnen1.5_cusps_n%d" % n, "chains": 2, "members_per_chain": 21}
    calls = (("chains_forces", lambda: ctx.chains_forces(chs, acc, com, macc, pot=pot)),
             ("two_single_chain_calls",
              lambda: [ctx.chain_forces(chs[k], acc, com[k], macc[21 * k:21 * (k + 1)], pot=pot)
                       for k in range(2)]))
    for name, fn in calls:
        fn()
        ctx.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        out[name + "_us"] = 1e3 * e0.elapsed_time(e1) / reps
    ctx.sync()
    out["n_perturbers"] = [int(keep[4 * k + 3].cpu().numpy()[0]) for k in range(2)]
    ctx.close()
    return out


def extra_hybrid(steps=10, dt=1e-5):
    """The hybrid step on a Dehnen gamma = 1.5 cusp of N = 1 048 576 stars
    with one SMBH of 0.01 at rest at its centre (eps = 1e-3, theta = 0.5,
    mixed path), r_chain0 = 0.01, gamma_crit = 1e-4, gamma_esc = 1.5; per
    step against the plain KDK step of the same system."""
    import numpy as np
    import torch
    from paper_1507_01009_amd import binding as B, ics
    n = 1048576
    pos, vel, m = ics.dehnen(n, 1.5, ics.SEED_BASE + 61)
    w = ics.Workload("cusp_n%d_one_smbh" % n, pos, vel, m, 1e-3, 0.5, np.array([0, n]),
                     np.zeros((1, 3)), np.zeros((1, 3)), np.array([0.01]), np.array([1e-3]),
                     np.zeros(1, np.int32))
    out = {"workload": w.name, "dt": dt, "steps": steps, "precision": "mixed"}
    ctx = B.Context(n, precision=B.TG_MIXED)
    d = DevState(ctx, w)
    ctx.forces(d.sys)
    ctx.step_kdk(d.sys, dt)
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step_kdk(d.sys, dt)
    ctx.sync()
    out["kdk_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / steps
    ctx.close()
    ctx = B.Context(n, precision=B.TG_MIXED)
    d = DevState(ctx, w)
    hy = B.Hybrid(ctx, d.sys, r_chain0=0.01)
    hy.begin()
    hy.step(dt)
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        hy.step(dt)
    ctx.sync()
    out["hybrid_ms_per_step"] = 1e3 * (time.perf_counter() - t0) / steps
    s = hy.state()
    out.update({"members": len(s["members"]), "perturbers": s["n_perturbers"],
                "absorbed": s["absorbed"], "escaped": s["escaped"],
                "archain_energy_error": s["energy_error"],
                "archain_share_of_step_time": s["archain_seconds"] / s["step_seconds"]})
    hy.close()
    ctx.close()
    # block substeps of the same system: 8 levels, dt_max = 2^-6, 32 substeps
    # with r_chain0 = 0.005 (the dense cusp feeds a larger chain past the
    # 256-member limit within a cycle)
    ctx = B.Context(n, precision=B.TG_MIXED)
    d = DevState(ctx, w)
    level = torch.zeros(n, dtype=torch.uint8, device="cuda")
    t4e2 = torch.full((n,), 0.3 ** 4 * w.eps ** 2, dtype=torch.float64, device="cuda")
    idx = torch.zeros(n, dtype=torch.int32, device="cuda")
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    k = torch.zeros(1, dtype=torch.int64, device="cuda")
    blk = ctx.make_blocks(level, t4e2, idx, na, k, 2.0 ** -6, 8)
    hy = B.Hybrid(ctx, d.sys, r_chain0=0.005)
    hy.begin()
    hy.step_block(blk)
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(32):
        hy.step_block(blk)
    ctx.sync()
    out["block_substeps"] = 32
    out["block_r_chain0"] = 0.005
    out["block_ms_per_substep"] = 1e3 * (time.perf_counter() - t0) / 32
    s = hy.state()
    out["block_members"] = len(s["members"])
    out["block_archain_share_of_step_time"] = s["archain_seconds"] / s["step_seconds"]
    out["block_level_histogram"] = np.bincount(level.cpu().numpy(), minlength=8).tolist()
    hy.close()
    ctx.close()
    return out


def extra_kdk_energy(steps=100):
    """Hernquist N = 131 072 + SMBH, dt = 1e-3: both precisions, energy error,
    and the step graph-replayed."""
    import torch
    from paper_1507_01009_amd import binding as B, ics
    w = ics.hernquist_c2()
    out = {"workload": w.name, "steps": steps, "dt": 1e-3}
    for name, prec in (("fp64", B.TG_FP64), ("mixed", B.TG_MIXED)):
        st = Step(w, prec, 8, 64, 0, 1e-3)
        st.ctx.sync()
        e0 = st.d.energy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st.ctx.sync()
        e1 = st.d.energy()
        out[name] = {"ms_per_step": 1e3 * (t1 - t0) / steps,
                     "rel_energy_error": abs(e1 - e0) / abs(e0),
                     # the same step captured once and replayed (after the
                     # energy check; launch overheads leave the timing)
                     "graph_ms_per_step": graph_ms(st.ctx, st.step, steps)}
        st.ctx.close()
    return out


def extra_blocksteps(substeps=1000, n=None, driver=False, rebuild_every=0):
    """Hernquist N = 4 194 304 + SMBH, 8 levels, dt_max = 2^-6, tau = 0.3 for
    the stars (the SMBH takes the smallest step).  Either one captured
    substep, replayed (every decision on the device), or the host driver
    tg_step_blocks, which runs the substeps no star takes part in without
    the tree's launches.  rebuild_every > 1: the tree is rebuilt at substeps
    that are multiples of it and refitted at the others."""
    import numpy as np
    import torch
    from paper_1507_01009_amd import binding as B, ics
    w = ics.hernquist_c4() if n is None else ics.hernquist_c4(n=n)
    nlev, dt_max = 8, 2.0 ** -6
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = B.Context(w.n, precision=B.TG_MIXED, stream=s)
        d = DevState(ctx, w)
        level = torch.zeros(w.n, dtype=torch.uint8, device="cuda")
        t4e2 = torch.full((w.n,), 0.3 ** 4 * w.eps ** 2, dtype=torch.float64, device="cuda")
        idx = torch.zeros(w.n, dtype=torch.int32, device="cuda")
        na = torch.zeros(1, dtype=torch.int32, device="cuda")
        k = torch.zeros(1, dtype=torch.int64, device="cuda")
        blk = ctx.make_blocks(level, t4e2, idx, na, k, dt_max, nlev,
                              rebuild_every=rebuild_every)
        ctx.forces(d.sys)
        ctx.step_block(d.sys, blk)
        ctx.sync()
        fr = []
        if driver:
            ctx.step_blocks(d.sys, blk, 128)      # one full cycle of level 0, untimed
        else:
            ctx.graph_begin()
            ctx.step_block(d.sys, blk)
            g = ctx.graph_end()
            for _ in range(128):                  # one full cycle of level 0, untimed
                g.launch(s)
                s.synchronize()
                fr.append(int(na.item()) / w.n)
        ctx.reset_counts()
        ctx.sync()
        t0 = time.perf_counter()
        if driver:
            n_idle = ctx.step_blocks(d.sys, blk, substeps)
        else:
            for _ in range(substeps):
                g.launch(s)
        s.synchronize()
        t1 = time.perf_counter()
        ctx.sync()
        cnt = ctx.get_cumulative_counts()
        lv = np.bincount(level.cpu().numpy(), minlength=nlev)
        ctx.close()
    sec = t1 - t0
    out = {"workload": w.name, "substeps": substeps, "ms_per_substep": 1e3 * sec / substeps,
           "interactions_per_s": (cnt["n_p2p"] + cnt["n_p2m"]) / sec,
           "forces_per_s": cnt["n_targets"] / sec,
           "interactions_per_force": (cnt["n_p2p"] + cnt["n_p2m"]) / max(cnt["n_targets"], 1),
           "level_histogram": lv.tolist(), "precision": "mixed",
           "rebuild_every": rebuild_every}
    if driver:
        out.update({"driver": "tg_step_blocks", "substeps_without_tree": n_idle})
    else:
        fr = np.array(fr)
        out.update({"graph": True,
                    "active_fraction": {"min": float(fr.min()), "median": float(np.median(fr)),
                                        "max": float(fr.max()), "mean": float(fr.mean())}})
    return out


def extra_batch(steps=20):
    """32 realisations (N log-uniform in [2^14, 2^19], gamma 0.5/1/1.5, one
    SMBH each) in one context: autotuned sizes, one captured KDK step; and
    the same systems stepped one after another."""
    import torch
    from paper_1507_01009_amd import binding as B, ics
    w = ics.batch_c5()
    S = w.sys_off.shape[0] - 1
    ctx = B.Context(w.n, max_systems=S, precision=B.TG_MIXED)
    d = DevState(ctx, w)
    best = ctx.autotune(d.pos, d.mass, w.eps, w.theta, sys_off=w.sys_off,
                        leaf_list=[8, 12, 16], group_list=[48, 64], waves_list=[12, 16],
                        repeats=2)
    best["times"] = [round(float(t), 4) for t in best["times"]]   # per candidate, list order
    ctx.forces(d.sys)
    ctx.reset_counts()
    ms_graph = graph_ms(ctx, lambda: ctx.step_kdk(d.sys, 1e-3), steps)
    cnt = ctx.get_cumulative_counts()
    n_steps = steps + 2                       # eager + first replay + timed replays
    # one system at a time through a single-system context (same sizes)
    nmax = int(max(w.sys_off[1:] - w.sys_off[:-1]))
    one = B.Context(nmax, leaf_size=best["leaf_size"], group_size=best["group_size"],
                    precision=B.TG_MIXED, waves_per_cu=best["waves_per_cu"])
    views = [d.view(one, int(w.sys_off[s]), int(w.sys_off[s + 1]), s, s + 1)
             for s in range(S)]
    for v in views:
        one.forces(v)
    one.sync()
    reps = max(3, steps // 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for v in views:
            one.step_kdk(v, 1e-3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    one.sync()
    ms_sep = 1e3 * (t1 - t0) / reps
    out = {"workload": w.name, "systems": S, "n_total": int(w.n), "autotuned": best,
           "ms_per_step_batched_graph": ms_graph,
           "interactions_per_s_batched": (cnt["n_p2p"] + cnt["n_p2m"]) / n_steps / (ms_graph * 1e-3),
           "ms_per_step_separate_systems": ms_sep,
           "speedup_batched_vs_separate": ms_sep / ms_graph, "precision": "mixed"}
    one.close()
    ctx.close()
    return out


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU (requested %d); sharding a system "
              "across GPUs is not implemented" % max(a.gpus, world), file=sys.stderr)
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
        if "tree" not in res:
            t = st.ctx.tree_arrays()
            res["tree"] = {"n_nodes": int(t["level"].size),
                           "n_leaves": int((t["nchild"] == 0).sum()),
                           "n_groups": int(t["groups"].shape[0])}
        r = time_path(st, a.steps, a.warmup)
        r["graph_ms_per_step"] = graph_ms(st.ctx, st.step, max(3, a.steps // 2))
        res[name] = r
        log("bench: %s %.3f ms/step, %.3g interactions/s, walk %.3f ms (%.2f TFLOP/s)" % (
            name, r["ms_per_step"], r["interactions_per_s"], r["walk_ms_avg"],
            r["walk_tflops"]))
        st.ctx.close()
        del st
        torch.cuda.empty_cache()
    rel = None
    ex = set() if a.no_extra else set(a.extras.split(","))
    if "relative" in ex and "mixed" in paths:
        log("bench: relative opening test, alpha = 1e-3")
        rel, accs["mixed_relative"] = extra_relative_mac(w, a)
        log("bench: relative %.3f ms/step, %.3g interactions/step, walk %.3f ms" % (
            rel["ms_per_step"], rel["interactions_per_step"], rel["walk_ms_avg"]))
        torch.cuda.empty_cache()
    err = {}
    if "mixed" in accs and "fp64" in accs:
        e = np.linalg.norm(accs["mixed"] - accs["fp64"], axis=1) / np.linalg.norm(accs["fp64"], axis=1)
        err["mixed_vs_fp64"] = percentiles(e)
        err["mixed_vs_fp64_reference"] = "the FP64 GPU path on all targets (identical lists)"
    if not a.no_cpu:
        log("bench: errors against the oracle's direct sum (4096 targets)")
        err.update(direct_errors(w, accs))
    err.update(direct_errors_gpu(w, accs))
    tree = res.pop("tree")
    head = res["mixed"] if "mixed" in res else res["fp64"]
    head_name = "mixed" if "mixed" in res else "fp64"
    peak = PEAK_FP32 if head_name == "mixed" else PEAK_FP64
    roof = {"bound": "alu", "achieved": head["walk_tflops"], "peak": peak, "unit": "TFLOP/s",
            "frac": head["walk_tflops"] / peak,
            "traffic": traffic_for("k_walk.hip", "cusp1m"),
            "kernel": "k_walk_forces<%s, false, false>" % ("true" if head_name == "mixed" else "false"),
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
                   "group_size": a.group, "precision": head_name, "dt": a.dt,
                   "tree": tree},
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
    if rel is not None:
        out["relative_mac"] = rel
    if "spline" in ex:
        log("bench: spline softening (same workload)")
        out["spline"] = extra_spline(w, a)
        log("bench: spline %.3f ms/step" % out["spline"]["ms_per_step"])
        torch.cuda.empty_cache()
    if "chain" in ex:
        log("bench: chain coupling (same workload)")
        out["chain"] = extra_chain(w)
        log("bench: several chains (two cusps, 1M stars)")
        out["chains"] = extra_chains()
        torch.cuda.empty_cache()
    if "hybrid" in ex:
        log("bench: hybrid step (1M cusp, one SMBH)")
        out["hybrid"] = extra_hybrid()
        torch.cuda.empty_cache()
    if "kdk" in ex:
        log("bench: KDK energy check (Hernquist 131k)")
        out["kdk_energy"] = extra_kdk_energy()
        torch.cuda.empty_cache()
    if "blocksteps" in ex:
        log("bench: block steps (Hernquist 4M)")
        out["blocksteps"] = extra_blocksteps()
        log("block steps, host driver")
        out["blocksteps_driver"] = extra_blocksteps(driver=True)
        log("block steps, host driver, rebuild every 128 substeps and refit between")
        out["blocksteps_driver_refit"] = extra_blocksteps(driver=True, rebuild_every=128)
        torch.cuda.empty_cache()
    if "batch" in ex:
        log("bench: batch of 32 realisations")
        out["batch"] = extra_batch()
        torch.cuda.empty_cache()
    if not a.no_cpu:
        log("bench: CPU oracle baseline (~%.0f s)" % a.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(w, a.leaf, a.group, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
