"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: integer structures (cube, keys, permutation, nodes, groups, interaction
lists, interaction counts) bit-exact; FP64 forces max relative error <= 1e-12;
mixed precision median <= 1e-5 and 99th percentile <= 1e-4, all against the
oracle tree on identical inputs.
"""
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_1507_01009_amd import ics
from gpu_helpers import (gpu_run, rel_err, oracle_lists, gpu_lists_by_group,
                         mac_margin, to_dev)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def _w(name):
    if name == "plummer4096":
        w = ics.plummer_c1()
        return w.pos, w.mass, w.eps
    if name == "hernquist32k":
        p, _, m = ics.dehnen(32768, 1.0, ics.SEED_BASE + 22)
        return p, m, 0.01
    if name == "hernquist131k":
        w = ics.hernquist_c2()
        return w.pos, w.mass, w.eps
    if name == "cusp1m":
        w = ics.cusp_c3()
        return w.pos, w.mass, w.eps
    if name == "clustered":
        rng = np.random.default_rng(5)
        base = rng.normal(size=(300, 3))
        p = np.concatenate([base, np.repeat(base[:5], 40, axis=0), rng.normal(size=(900, 3)) * 1e-7])
        return p, np.full(p.shape[0], 1.0 / p.shape[0]), 1e-3
    if name == "coincident":
        # 1500 particles on one point (a level-21 leaf of 1500, walked with
        # the unpacked prefix sums) inside a Plummer sphere
        p, _, _ = ics.plummer(3000, 17)
        dup = np.repeat(np.array([[0.01, -0.02, 0.03]]), 1500, axis=0)
        p = np.concatenate([p, dup])
        return p, np.full(p.shape[0], 1.0 / p.shape[0]), 0.01
    raise KeyError(name)


def _tree_equal(t_or, g, groups_or=None):
    assert np.array_equal(g["cube"], t_or.cube)
    assert np.array_equal(g["skeys"], t_or.skeys)
    assert np.array_equal(g["perm"], t_or.perm)
    for k in ("level", "first", "count", "child", "nchild", "parent"):
        assert np.array_equal(g[k], getattr(t_or, k)), k
    if groups_or is not None:
        assert np.array_equal(g["groups"], groups_or)


@pytest.mark.parametrize("name,nl,ng", [("plummer4096", 8, 64), ("plummer4096", 1, 1),
                                        ("plummer4096", 16, 48), ("hernquist131k", 8, 64),
                                        ("clustered", 4, 16), ("hernquist32k", 8, 128),
                                        ("coincident", 8, 64)])
def test_tree_and_groups_bit_exact(name, nl, ng):
    say("tree", name, nl, ng)
    pos, m, eps = _w(name)
    g = gpu_run(pos, m, eps, 0.5, nl, ng)
    t = oracle.build_tree(pos, None, nl)
    _tree_equal(t, g["tree"], oracle.groups(t, ng))


@pytest.mark.parametrize("n", [1, 2, 3, 65, 2049])
def test_small_and_ragged_sizes(n):
    say("small", n)
    pos, _, m = ics.plummer(n, 100 + n)
    g = gpu_run(pos, m, 0.01, 0.5, 8, 64, lists=True)
    ev = oracle.tree_forces(pos, m, 0.01, 0.5, 8, 64)
    _tree_equal(ev.tree, g["tree"], ev.groups)
    if n > 1:
        assert rel_err(g["acc"], ev.acc).max() <= FP64_TOL
        assert np.max(np.abs(g["pot"] - ev.pot) / np.abs(ev.pot)) <= FP64_TOL
    else:
        assert np.all(g["acc"] == 0.0) and np.all(g["pot"] == 0.0)
    assert g["counts"]["n_p2p"] == ev.n_p2p and g["counts"]["n_p2m"] == ev.n_p2m


def test_moments_match_plain_definition():
    say("moments")
    pos, m, eps = _w("hernquist32k")
    m = m * np.random.default_rng(2).uniform(0.5, 1.5, m.shape)
    g = gpu_run(pos, m, eps, 0.5, 8, 64)["tree"]
    t = oracle.build_tree(pos, None, 8)
    sp, sm = oracle.sorted_arrays(t, pos, m)
    mom = oracle.moments(t, sp, sm)
    leaf = t.nchild == 0
    # leaves: the same sums in the same order -> bit-exact
    assert np.array_equal(g["mom"][leaf, 0], mom[leaf, 0])
    assert np.array_equal(g["com"][leaf, :3], mom[leaf, 1:4])
    assert np.array_equal(g["mom"][leaf, 1:7], mom[leaf, 4:10])
    # internal nodes: parallel-axis combination, rounding-level differences
    size = t.cube[0, 3] * 2.0 ** -t.level.astype(float)
    assert np.all(np.abs(g["mom"][:, 0] - mom[:, 0]) <= 1e-14 * mom[:, 0])
    assert np.all(np.abs(g["com"][:, :3] - mom[:, 1:4]) <= 1e-14 * (np.abs(mom[:, 1:4]) + size[:, None]))
    scale = np.abs(mom[:, 4:7]).max(1, keepdims=True) + 1e-300
    assert np.all(np.abs(g["mom"][:, 1:7] - mom[:, 4:10]) <= 1e-12 * scale)
    assert np.array_equal(g["com"][:, 3], size * size)


def _check_lists(pos, m, eps, theta, nl, ng, active=None):
    g = gpu_run(pos, m, eps, theta, nl, ng, active=active, lists=True)
    ev = oracle.tree_forces(pos, m, eps, theta, nl, ng, active=active)
    ol = oracle_lists(ev, theta)
    gl = gpu_lists_by_group(*g["lists"])
    assert sorted(gl) == sorted(ol)
    flips = 0
    for k, (om, op) in ol.items():
        gm, gp = gl[k]
        if np.array_equal(gm, om) and np.array_equal(gp, op):
            continue
        # a decision may only differ where it sits on the threshold within
        # the rounding of the centre of mass (internal nodes are combined
        # from children on the GPU, summed from particles in the oracle)
        diff = set(np.setxor1d(gm, om)) | set(np.setxor1d(gp, op))
        for v in diff:
            anc = v
            while anc != 0xFFFFFFFF:
                if mac_margin(ev.tree, ev.mom, ev.box[k], anc, theta) < 1e-12:
                    break
                anc = ev.tree.parent[anc]
            assert anc != 0xFFFFFFFF, (k, v)
        flips += 1
    assert flips <= max(1, len(ol) // 10000)
    return g, ev, flips


@pytest.mark.parametrize("name,theta,nl,ng,every", [
    ("plummer4096", 0.5, 8, 64, 1), ("plummer4096", 0.3, 8, 32, 3),
    ("plummer4096", 0.0, 8, 64, 7), ("hernquist32k", 0.5, 8, 64, 1),
    ("clustered", 0.55, 4, 16, 2), ("hernquist32k", 0.5, 8, 128, 1),
    ("hernquist32k", 0.5, 12, 100, 3), ("coincident", 0.5, 8, 64, 1)])
def test_interaction_lists_match(name, theta, nl, ng, every):
    say("lists", name, theta)
    pos, m, eps = _w(name)
    active = None if every == 1 else np.arange(0, pos.shape[0], every)
    _check_lists(pos, m, eps, theta, nl, ng, active)


@pytest.mark.parametrize("name,nl,ng,every", [("plummer4096", 8, 64, 1),
                                              ("plummer4096", 4, 20, 5),
                                              ("hernquist131k", 8, 64, 1),
                                              ("clustered", 4, 16, 1),
                                              ("hernquist32k", 8, 128, 1),
                                              ("hernquist32k", 16, 97, 2),
                                              ("coincident", 8, 64, 1),
                                              ("coincident", 4, 128, 3)])
def test_forces_fp64(name, nl, ng, every):
    say("fp64", name)
    pos, m, eps = _w(name)
    active = None if every == 1 else np.arange(1, pos.shape[0], every)
    g = gpu_run(pos, m, eps, 0.5, nl, ng, active=active)
    ev = oracle.tree_forces(pos, m, eps, 0.5, nl, ng, active=active)
    rows = np.arange(pos.shape[0]) if active is None else active
    e = rel_err(g["acc"][rows], ev.acc[rows])
    ep = np.abs(g["pot"][rows] - ev.pot[rows]) / np.abs(ev.pot[rows])
    say("  max rel acc %.3g pot %.3g" % (e.max(), ep.max()))
    assert e.max() <= FP64_TOL and ep.max() <= FP64_TOL
    if active is not None:
        untouched = np.setdiff1d(np.arange(pos.shape[0]), rows)
        assert np.all(np.isnan(g["acc"][untouched]))
    c = g["counts"]
    assert (c["n_p2p"], c["n_p2m"], c["n_targets"]) == (ev.n_p2p, ev.n_p2m, ev.n_targets)


@pytest.mark.parametrize("name,ng", [("plummer4096", 64), ("hernquist131k", 64),
                                     ("hernquist131k", 128)])
def test_forces_mixed_precision(name, ng):
    say("mixed", name, ng)
    pos, m, eps = _w(name)
    g = gpu_run(pos, m, eps, 0.5, 8, ng, precision=1)
    ev = oracle.tree_forces(pos, m, eps, 0.5, 8, ng)
    e = rel_err(g["acc"], ev.acc)
    say("  mixed p50 %.3g p99 %.3g max %.3g" % tuple(np.percentile(e, [50, 99, 100])))
    assert np.median(e) <= 1e-5 and np.percentile(e, 99) <= 1e-4
    ep = np.abs(g["pot"] - ev.pot) / np.abs(ev.pot)
    assert np.median(ep) <= 1e-5 and np.percentile(ep, 99) <= 1e-4
    assert g["counts"]["n_p2p"] == ev.n_p2p and g["counts"]["n_p2m"] == ev.n_p2m


def test_batch_of_systems():
    say("batch")
    parts = [ics.plummer(3000, 1)[0], ics.dehnen(9000, 0.5, 2)[0], np.zeros((0, 3)),
             ics.dehnen(2500, 1.5, 3)[0], ics.plummer(7, 4)[0]]
    pos = np.concatenate(parts)
    off = np.r_[0, np.cumsum([p.shape[0] for p in parts])]
    m = np.full(pos.shape[0], 1e-4)
    act = np.arange(0, pos.shape[0], 2)
    g = gpu_run(pos, m, 0.01, 0.5, 8, 32, active=act, sys_off=off)
    ev = oracle.tree_forces(pos, m, 0.01, 0.5, 8, 32, active=act, sys_off=off)
    _tree_equal(ev.tree, g["tree"], ev.groups)
    e = rel_err(g["acc"][act], ev.acc[act])
    assert e.max() <= FP64_TOL
    assert g["counts"]["n_p2p"] == ev.n_p2p and g["counts"]["n_p2m"] == ev.n_p2m


def test_full_size_cusp_sampled():
    """N = 1 048 576 Dehnen gamma = 1.5, theta = 0.5, both precisions.

    Whole arrays: cube, keys, permutation, nodes and groups bit-exact.  The
    oracle walks and evaluates a sample of groups (random plus the densest
    centre); the GPU values for their targets must meet the bar."""
    say("cusp1m")
    pos, m, eps = _w("cusp1m")
    g64 = gpu_run(pos, m, eps, 0.5, 8, 64)
    t = oracle.build_tree(pos, None, 8)
    groups = oracle.groups(t, 64)
    _tree_equal(t, g64["tree"], groups)
    rng = np.random.default_rng(7)
    r = np.linalg.norm(pos[t.perm[groups[:, 0]].astype(np.int64)], axis=1)
    sel = np.unique(np.r_[rng.choice(groups.shape[0], 240, replace=False), np.argsort(r)[:16]])
    ev = oracle.tree_forces(pos, m, eps, 0.5, 8, 64, sel_groups=sel, tree=t)
    rows = np.nonzero(~np.isnan(ev.pot))[0]
    e64 = rel_err(g64["acc"][rows], ev.acc[rows])
    say("  fp64 max %.3g over %d targets" % (e64.max(), rows.size))
    assert e64.max() <= FP64_TOL
    g32 = gpu_run(pos, m, eps, 0.5, 8, 64, precision=1)
    e32 = rel_err(g32["acc"][rows], ev.acc[rows])
    say("  mixed p50 %.3g p99 %.3g" % (np.median(e32), np.percentile(e32, 99)))
    assert np.median(e32) <= 1e-5 and np.percentile(e32, 99) <= 1e-4
    # interaction totals are integers: identical on both GPU paths
    assert g64["counts"] == g32["counts"]


# ---------------------------------------------------- FP64 direct forces
def test_direct_fp64_smbh_pairs():
    say("direct")
    import torch
    from paper_1507_01009_amd import binding as B
    w = ics.cusp_c3(n=200000)
    ctx = B.Context(w.n)
    sp, sm, se = to_dev(w.bh_pos), to_dev(w.bh_mass), to_dev(w.bh_eps)
    tp, te = to_dev(w.pos), to_dev(np.full(w.n, w.eps))
    tm = to_dev(w.mass)
    acc = torch.zeros((w.n, 3), dtype=torch.float64, device="cuda")
    pot = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    ctx.direct_fp64(sp, sm, se, tp, te, acc, pot)                   # stars <- BHs
    bacc = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    bpot = torch.zeros(2, dtype=torch.float64, device="cuda")
    ctx.direct_fp64(tp, tm, te, sp, se, bacc, bpot)                 # BHs <- stars
    ctx.direct_fp64(sp, sm, se, sp, se, bacc, bpot, self_pairs=True, accumulate=True)
    ctx.sync()
    ra, rp = oracle.direct_pairs(w.bh_pos, w.bh_mass, w.bh_eps, w.pos, w.eps)
    assert rel_err(acc.cpu().numpy(), ra).max() <= 1e-13
    ba, bp = oracle.direct_pairs(w.pos, w.mass, w.eps, w.bh_pos, w.bh_eps)
    oracle.direct_pairs(w.bh_pos, w.bh_mass, w.bh_eps, w.bh_pos, w.bh_eps,
                        self_pairs=True, acc=ba, pot=bp)
    # compensated GPU sum vs plain oracle sum: bound by the oracle's rounding
    d = np.linalg.norm(w.pos[None, :, :] - w.bh_pos[:, None, :], axis=2)
    scale = (w.mass[None, :] / (d ** 2 + w.eps ** 2)).sum(1)
    assert np.all(np.linalg.norm(bacc.cpu().numpy() - ba, axis=1) <= 1e-12 * scale)
    assert np.allclose(bpot.cpu().numpy(), bp, rtol=1e-12, atol=0)


def test_direct_fp64_segments():
    say("direct segments")
    import torch
    from paper_1507_01009_amd import binding as B
    w = ics.batch_c5(S=4, nmin=2000, nmax=9000)
    ctx = B.Context(w.n, max_systems=4)
    tp, te = to_dev(w.pos), to_dev(np.full(w.n, w.eps))
    acc = torch.zeros((w.n, 3), dtype=torch.float64, device="cuda")
    bseg = np.arange(5)
    bpos = w.bh_pos + np.arange(4)[:, None] * 0.1
    ctx.direct_fp64(to_dev(bpos), to_dev(w.bh_mass), to_dev(w.bh_eps), tp, te, acc,
                    src_seg=bseg, tgt_seg=w.sys_off)
    ctx.sync()
    a = acc.cpu().numpy()
    for s in range(4):
        sl = slice(w.sys_off[s], w.sys_off[s + 1])
        ra, _ = oracle.direct_pairs(bpos[s:s + 1], w.bh_mass[s:s + 1], w.bh_eps[s:s + 1],
                                    w.pos[sl], w.eps)
        assert rel_err(a[sl], ra).max() <= 1e-13


# ---------------------------------------------------- leapfrog and levels
def test_kick_drift_levels_bit_exact():
    say("integrator")
    import torch
    from paper_1507_01009_amd import binding as B
    rng = np.random.default_rng(9)
    n = 50000
    vel = rng.normal(size=(n, 3))
    acc = rng.normal(size=(n, 3)) * 10.0 ** rng.uniform(-2, 4, (n, 1))
    pos = rng.normal(size=(n, 3))
    level = rng.integers(0, 8, n).astype(np.uint8)
    idx = np.sort(rng.choice(n, 12345, replace=False)).astype(np.int32)
    t4e2 = np.full(n, 0.3 ** 4 * 0.01 ** 2)
    ctx = B.Context(n)
    dv, da, dp, dl = to_dev(vel), to_dev(acc), to_dev(pos), to_dev(level)
    didx, dna = to_dev(idx), to_dev(np.array([idx.size], np.int32))
    k = to_dev(np.array([6], np.int64))
    ctx.kick(dv, da, 2.0 ** -6, didx, dna, dl)
    ctx.drift(dp, dv, 2.0 ** -13)
    ctx.levels(da, to_dev(t4e2), dl, 2.0 ** -6, 8, k, didx, dna)
    out_idx = torch.zeros(n, dtype=torch.int32, device="cuda")
    out_n = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.active_set(dl, 8, k, out_idx, out_n, k_add=2)
    ctx.sync()
    v2, p2, l2 = vel.copy(), pos.copy(), level.copy()
    oracle.kick(v2, acc, 2.0 ** -6, idx=idx, level=level)
    oracle.drift(p2, v2, 2.0 ** -13)
    oracle.levels(acc, t4e2, l2, 2.0 ** -6, 8, 6, idx=idx)
    assert np.array_equal(dv.cpu().numpy(), v2)
    assert np.array_equal(dp.cpu().numpy(), p2)
    assert np.array_equal(dl.cpu().numpy(), l2)
    ref = oracle.active_at(l2, 8, 8)
    assert int(out_n.item()) == ref.size
    assert np.array_equal(out_idx.cpu().numpy()[:ref.size], ref)


def test_kdk_step_matches_oracle():
    """One KDK step (kick, drift, rebuild, forces, kick) on the Plummer
    sphere: positions bit-exact, velocities to the force tolerance."""
    say("kdk")
    import torch
    from paper_1507_01009_amd import binding as B
    w = ics.plummer_c1()
    dt = 1e-3
    ctx = B.Context(w.n)
    dp, dv, dm = to_dev(w.pos), to_dev(w.vel), to_dev(w.mass)
    acc = torch.zeros((w.n, 3), dtype=torch.float64, device="cuda")
    ctx.build_tree(dp); ctx.compute_moments(dm); ctx.tree_forces(w.eps, 0.5, acc)
    ctx.kick(dv, acc, dt); ctx.drift(dp, dv, dt)
    ctx.build_tree(dp); ctx.compute_moments(dm); ctx.tree_forces(w.eps, 0.5, acc)
    ctx.kick(dv, acc, dt)
    ctx.sync()
    a0 = oracle.tree_forces(w.pos, w.mass, w.eps, 0.5, 8, 64).acc
    v, x = w.vel.copy(), w.pos.copy()
    oracle.kick(v, a0, dt)
    oracle.drift(x, v, dt)
    gx = dp.cpu().numpy()
    # drift from velocities that carry the force rounding: tiny differences
    assert np.max(np.abs(gx - x)) <= 1e-15 * (1 + np.abs(x).max())
    a1 = oracle.tree_forces(gx, w.mass, w.eps, 0.5, 8, 64).acc
    assert rel_err(acc.cpu().numpy(), a1).max() <= FP64_TOL


# ---------------------------------------------------- graphs / runtime
def test_graph_replay_equals_eager():
    say("graph")
    import torch
    from paper_1507_01009_amd import binding as B
    pos, m, eps = _w("hernquist32k")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = B.Context(pos.shape[0], stream=s)
        dp, dm = to_dev(pos), to_dev(m)
        acc_e = torch.zeros((pos.shape[0], 3), dtype=torch.float64, device="cuda")
        acc_g = torch.zeros_like(acc_e)
        ctx.build_tree(dp); ctx.compute_moments(dm); ctx.tree_forces(eps, 0.5, acc_e)
        ctx.sync()
        ctx.graph_begin()
        ctx.build_tree(dp); ctx.compute_moments(dm); ctx.tree_forces(eps, 0.5, acc_g)
        graph = ctx.graph_end()
        for rep in range(3):
            acc_g.zero_()
            graph.launch(s)
            s.synchronize()
            assert torch.equal(acc_g, acc_e), rep
            ctx.build_tree(dp); ctx.compute_moments(dm); ctx.tree_forces(eps, 0.5, acc_e)
            ctx.sync()
        # a graph replays kernels on its context's buffers: once the context
        # is closed, launching it is refused on the host (nothing runs)
        ctx.close()
        with pytest.raises(B.TGError):
            graph.launch(s)


def test_deterministic_bitwise():
    say("determinism")
    pos, m, eps = _w("hernquist32k")
    a = gpu_run(pos, m, eps, 0.5, 8, 64)["acc"]
    b = gpu_run(pos, m, eps, 0.5, 8, 64, waves_per_cu=3)["acc"]
    assert np.array_equal(a, b)


def test_error_paths():
    say("errors")
    import torch
    from paper_1507_01009_amd import binding as B
    pos, m, eps = _w("plummer4096")
    ctx = B.Context(pos.shape[0])
    dp, dm = to_dev(pos), to_dev(m)
    acc = torch.zeros((pos.shape[0], 3), dtype=torch.float64, device="cuda")
    with pytest.raises(B.TGError) as e:
        ctx.build_tree(to_dev(np.zeros((pos.shape[0] + 1, 3))))
    assert e.value.status == -1
    with pytest.raises(B.TGError) as e:
        ctx.compute_moments(dm)
    assert e.value.status == -5
    ctx.build_tree(dp)
    ctx.compute_moments(dm)
    for bad_eps, bad_theta in ((0.0, 0.5), (-1.0, 0.5), (0.01, 0.58), (0.01, -0.1)):
        with pytest.raises(B.TGError) as e:
            ctx.tree_forces(bad_eps, bad_theta, acc)
        assert e.value.status == -1
    bad = pos.copy()
    bad[17, 1] = np.nan
    ctx.build_tree(to_dev(bad))
    with pytest.raises(B.TGError) as e:
        ctx.sync()
    assert e.value.status == -6
    ctx.build_tree(dp)
    mm = m.copy()
    mm[5] = -1.0
    ctx.compute_moments(to_dev(mm))
    with pytest.raises(B.TGError) as e:
        ctx.sync()
    assert e.value.status == -6
    small = B.Context(pos.shape[0], max_nodes=100)
    small.build_tree(dp)
    with pytest.raises(B.TGError) as e:
        small.sync()
    assert e.value.status == -4
    tiny = B.Context(pos.shape[0], frontier_cap=64)
    tiny.build_tree(dp); tiny.compute_moments(dm); tiny.tree_forces(eps, 0.5, acc)
    with pytest.raises(B.TGError) as e:
        tiny.sync()
    assert e.value.status == -4


def test_empty_input():
    say("empty")
    import torch
    from paper_1507_01009_amd import binding as B
    ctx = B.Context(16)
    dp = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    dm = torch.zeros(0, dtype=torch.float64, device="cuda")
    acc = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    ctx.build_tree(dp)
    ctx.compute_moments(dm)
    ctx.tree_forces(0.01, 0.5, acc)
    ctx.sync()
    assert ctx.get_tree().n_nodes == 0


def test_direct_fp64_at_1m_sources_against_oracle():
    """The compensated FP64 direct sum over all 1 048 576 stars of the cusp
    plus its two SMBHs, on 4096 seeded targets, against the oracle's
    long-double direct sum: max relative error <= 1e-12."""
    say("direct 1M sources")
    import torch
    from paper_1507_01009_amd import binding as B
    w = ics.cusp_c3()
    rng = np.random.default_rng(98)
    tg = np.sort(rng.choice(w.n, 4096, replace=False))
    ctx = B.Context(w.n)
    tpos = to_dev(w.pos[tg])
    teps = to_dev(np.full(tg.size, w.eps))
    acc = torch.zeros((tg.size, 3), dtype=torch.float64, device="cuda")
    ctx.direct_fp64(to_dev(w.pos), to_dev(w.mass), to_dev(np.full(w.n, w.eps)), tpos, teps, acc)
    ctx.direct_fp64(to_dev(w.bh_pos), to_dev(w.bh_mass), to_dev(w.bh_eps), tpos, teps, acc,
                    accumulate=True)
    ctx.sync()
    ref, _ = oracle.direct(w.pos, w.mass, w.eps, tg, xpos=w.bh_pos, xmass=w.bh_mass,
                           xeps=w.bh_eps)
    e = rel_err(acc.cpu().numpy(), ref)
    say("  max rel %.3g" % e.max())
    assert e.max() <= 1e-12
    ctx.close()


def test_running_counts_add_up_over_walks():
    """The force walk's counts are summed per workgroup after each walk: the
    last walk's equal the oracle's, the running totals add them up over
    walks, an evaluation with no active star adds nothing and reports zero,
    and a reset clears the totals."""
    import torch
    pos, m, eps = _w("hernquist32k")
    ev = oracle.tree_forces(pos, m, eps, 0.5, 8, 64)
    g = gpu_run(pos, m, eps, 0.5, 8, 64)
    ctx = g["ctx"]
    one = (ev.n_p2p, ev.n_p2m, ev.n_targets)
    assert (g["counts"]["n_p2p"], g["counts"]["n_p2m"], g["counts"]["n_targets"]) == one
    acc = torch.zeros((pos.shape[0], 3), dtype=torch.float64, device="cuda")
    ctx.reset_counts()
    for k in range(3):
        ctx.tree_forces(eps, 0.5, acc)
    ctx.sync()
    c = ctx.get_cumulative_counts()
    assert (c["n_p2p"], c["n_p2m"], c["n_targets"]) == tuple(3 * v for v in one)
    # nothing active: the walk is skipped on the device
    didx = to_dev(np.zeros(1, np.int32))
    dna = to_dev(np.zeros(1, np.int32))
    ctx.tree_forces(eps, 0.5, acc, None, didx, dna)
    ctx.sync()
    last, run = ctx.get_counts(), ctx.get_cumulative_counts()
    assert (last["n_p2p"], last["n_p2m"], last["n_targets"]) == (0, 0, 0)
    assert (run["n_p2p"], run["n_p2m"], run["n_targets"]) == tuple(3 * v for v in one)
    ctx.reset_counts()
    ctx.sync()
    z = ctx.get_cumulative_counts()
    assert (z["n_p2p"], z["n_p2m"], z["n_targets"], z["n_groups"]) == (0, 0, 0, 0)
