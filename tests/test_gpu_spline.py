"""GPU parity of the cubic-spline softening (tg_set_softening) against the
oracle's spline evaluation on identical inputs, through the C ABI.

Bar as for Plummer softening: interaction counts equal to the oracle's (the
lists do not depend on the softening), FP64 forces and potentials max
relative error <= 1e-12, mixed precision median <= 1e-5 and p99 <= 1e-4;
SMBH terms, direct sums and whole steps in FP64 to the same bars as their
Plummer tests.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import steps as osteps
from paper_1507_01009_amd import ics
from gpu_helpers import gpu_run, rel_err, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _work(name):
    if name == "plummer4096":
        w = ics.plummer_c1()
        return w.pos, w.mass, w.eps
    if name == "plummer_wide":                 # every pair inside the kernel
        p, _, m = ics.plummer(3000, 41)
        return p, m, 2.0
    if name == "hernquist32k":
        p, _, m = ics.dehnen(32768, 1.0, ics.SEED_BASE + 22)
        return p, m, 0.01
    if name == "cusp65k":
        p, _, m = ics.dehnen(65536, 1.5, ics.SEED_BASE + 23)
        return p, m, 1e-3
    if name == "clustered":                    # duplicates: pairs at r = 0
        rng = np.random.default_rng(5)
        base = rng.normal(size=(300, 3))
        p = np.concatenate([base, np.repeat(base[:5], 40, axis=0),
                            rng.normal(size=(900, 3)) * 1e-7])
        return p, np.full(p.shape[0], 1.0 / p.shape[0]), 1e-3
    raise KeyError(name)


@pytest.mark.parametrize("name,nl,ng,every", [
    ("plummer4096", 8, 64, 1), ("plummer_wide", 8, 64, 1), ("hernquist32k", 8, 64, 1),
    ("hernquist32k", 16, 97, 3), ("cusp65k", 8, 128, 1), ("clustered", 4, 16, 1),
    ("cusp65k", 12, 100, 7)])
def test_forces_fp64(name, nl, ng, every):
    say("spline fp64", name, nl, ng, every)
    pos, m, eps = _work(name)
    active = None if every == 1 else np.arange(1, pos.shape[0], every)
    g = gpu_run(pos, m, eps, 0.5, nl, ng, active=active, softening="spline")
    ev = oracle.tree_forces(pos, m, eps, 0.5, nl, ng, active=active, softening="spline")
    rows = np.arange(pos.shape[0]) if active is None else active
    e = rel_err(g["acc"][rows], ev.acc[rows])
    ep = np.abs(g["pot"][rows] - ev.pot[rows]) / np.abs(ev.pot[rows])
    say("  max rel acc %.3g pot %.3g" % (e.max(), ep.max()))
    assert e.max() <= FP64_TOL and ep.max() <= FP64_TOL
    c = g["counts"]
    assert (c["n_p2p"], c["n_p2m"], c["n_targets"]) == (ev.n_p2p, ev.n_p2m, ev.n_targets)


@pytest.mark.parametrize("name", ["hernquist32k", "cusp65k", "plummer_wide"])
def test_forces_mixed_precision(name):
    say("spline mixed", name)
    pos, m, eps = _work(name)
    g = gpu_run(pos, m, eps, 0.5, 8, 64, precision=1, softening="spline")
    ev = oracle.tree_forces(pos, m, eps, 0.5, 8, 64, softening="spline")
    e = rel_err(g["acc"], ev.acc)
    say("  mixed p50 %.3g p99 %.3g" % (np.median(e), np.percentile(e, 99)))
    assert np.median(e) <= 1e-5 and np.percentile(e, 99) <= 1e-4
    assert g["counts"]["n_p2p"] == ev.n_p2p and g["counts"]["n_p2m"] == ev.n_p2m


def test_relative_test_with_spline():
    say("spline relative")
    pos, m, eps = _work("hernquist32k")
    aold = oracle.tree_forces(pos, m, eps, 0.5).acc
    g = gpu_run(pos, m, eps, 0.5, 8, 64, alpha=1e-3, acc_old=aold, softening="spline")
    ev = oracle.tree_forces(pos, m, eps, 0.5, 8, 64, alpha=1e-3, acc_old=aold,
                            softening="spline")
    assert rel_err(g["acc"], ev.acc).max() <= FP64_TOL
    assert (g["counts"]["n_p2p"], g["counts"]["n_p2m"]) == (ev.n_p2p, ev.n_p2m)


def test_setting_back_to_plummer_restores_it():
    say("spline then plummer")
    from paper_1507_01009_amd import binding as B
    pos, m, eps = _work("plummer4096")
    ctx = B.Context(pos.shape[0])
    a = gpu_run(pos, m, eps, 0.5, ctx=ctx, softening="spline")
    b = gpu_run(pos, m, eps, 0.5, ctx=ctx)                   # helper restored Plummer
    ref = oracle.tree_forces(pos, m, eps, 0.5)
    assert rel_err(b["acc"], ref.acc).max() <= FP64_TOL
    assert rel_err(a["acc"], ref.acc).max() > 1e-6           # the spline differs
    with pytest.raises(B.TGError) as e:
        ctx.set_softening(7)
    assert e.value.status == -1


def test_full_size_cusp_sampled():
    """N = 1 048 576 Dehnen gamma = 1.5 with the SMBH binary's softening, the
    whole-tree GPU walk in FP64 against the oracle on sampled groups."""
    say("spline cusp1m")
    w = ics.cusp_c3()
    pos, m, eps = w.pos, w.mass, w.eps
    g = gpu_run(pos, m, eps, 0.5, 8, 64, softening="spline")
    t = oracle.build_tree(pos, None, 8)
    groups = oracle.groups(t, 64)
    rng = np.random.default_rng(19)
    rg = np.linalg.norm(pos[t.perm[groups[:, 0]].astype(np.int64)], axis=1)
    sel = np.unique(np.r_[rng.choice(groups.shape[0], 150, replace=False), np.argsort(rg)[:16]])
    ev = oracle.tree_forces(pos, m, eps, 0.5, 8, 64, sel_groups=sel, tree=t,
                            softening="spline")
    rows = np.nonzero(~np.isnan(ev.pot))[0]
    e = rel_err(g["acc"][rows], ev.acc[rows])
    say("  fp64 max %.3g over %d targets" % (e.max(), rows.size))
    assert e.max() <= FP64_TOL


def test_direct_fp64_pairs():
    say("spline direct")
    import torch
    from paper_1507_01009_amd import binding as B
    rng = np.random.default_rng(8)
    sp = rng.normal(size=(5000, 3)) * 0.05
    sm = rng.uniform(0.5, 1.5, 5000) / 5000
    se = rng.choice([0.0, 0.01, 0.03], 5000)
    tp = rng.normal(size=(7, 3)) * 0.05
    te = np.array([0.0, 0.02, 0.0, 0.05, 0.01, 0.0, 0.001])
    ctx = B.Context(5000)
    ctx.set_softening("spline")
    acc = torch.zeros((7, 3), dtype=torch.float64, device="cuda")
    pot = torch.zeros(7, dtype=torch.float64, device="cuda")
    ctx.direct_fp64(to_dev(sp), to_dev(sm), to_dev(se), to_dev(tp), to_dev(te), acc, pot)
    ctx.sync()
    ra, rp = oracle.direct_pairs(sp, sm, se, tp, te, softening="spline")
    assert rel_err(acc.cpu().numpy(), ra).max() <= 1e-13
    assert np.max(np.abs(pot.cpu().numpy() - rp) / np.abs(rp)) <= 1e-13


def test_kdk_steps_with_smbh():
    say("spline kdk")
    from paper_1507_01009_amd import binding as B
    from test_gpu_steps import Dev, ostate
    w = ics.hernquist_c2(n=32768)
    dt = 1e-3
    ctx = B.Context(w.n)
    ctx.set_softening("spline")
    d = Dev(ctx, w)
    ctx.forces(d.sys)
    for _ in range(3):
        ctx.step_kdk(d.sys, dt)
    ctx.sync()
    h = d.host()
    st = ostate(w)
    st.softening = "spline"
    osteps.forces(st)
    for _ in range(3):
        osteps.kdk_step(st, dt)
    assert np.max(np.abs(h["pos"] - st.pos)) <= 1e-13 * np.abs(st.pos).max()
    assert np.max(np.abs(h["vel"] - st.vel)) <= 1e-12 * np.abs(st.vel).max()
    assert rel_err(h["acc"], st.acc).max() <= 1e-11
    assert rel_err(h["bacc"], st.bh_acc).max() <= 1e-12
