"""Pins for the oracle's refitted tree (between full builds the order,
nodes and groups stay; moments and opening sizes follow the particles).

Independent references: on unmoved particles the refit is the build; after
a drift every node's particles lie in the cube of side s' about the cell
centre (brute force); theta = 0 still gives the direct sum; no accepted cell
holds a target of its group; the force error against the direct sum stays
that of a fresh build.
"""
import numpy as np

import oracle
from paper_1507_01009_amd import ics


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def _drifted(n, seed, dt):
    pos, vel, m = ics.dehnen(n, 1.0, seed)
    return pos, pos + vel * dt, m


def test_refit_of_unmoved_particles_is_the_build():
    pos, _, m = ics.plummer(3000, 21)
    t = oracle.build_tree(pos, None, 8)
    sp, _ = oracle.sorted_arrays(t, pos, m)
    side = oracle.refit_sides(t, sp)
    s = t.cube[t.sys, 3] * 2.0 ** -t.level.astype(float)
    assert np.all(side >= s) and np.mean(side == s) > 0.99
    a = oracle.tree_forces(pos, m, 0.01, 0.5, tree=t)
    b = oracle.tree_forces(pos, m, 0.01, 0.5, tree=t, refit=True)
    assert _rel(b.acc, a.acc).max() < 1e-12


def test_drifted_particles_stay_inside_the_refitted_cubes():
    p0, p1, m = _drifted(4000, 22, 0.05)
    t = oracle.build_tree(p0, None, 8)
    sp, _ = oracle.sorted_arrays(t, p1, m)
    side = oracle.refit_sides(t, sp)
    s = t.cube[t.sys, 3] * 2.0 ** -t.level.astype(float)
    assert np.mean(side > s) > 0.2           # the drift moved particles out of cells
    L = t.cube[0, 3]
    lo = t.cube[0, :3]
    for v in range(t.nn):
        # the cell centre from the cell's integer coordinates (plain geometry)
        q = np.floor((p0[t.perm[t.first[v]]] - lo) * (2.0 ** 21 / L)).clip(0, 2 ** 21 - 1)
        i = np.floor(q / 2.0 ** (21 - int(t.level[v])))
        g = lo + (i + 0.5) * s[v]
        x = sp[t.first[v]:t.first[v] + t.count[v]]
        assert np.all(np.abs(x - g) <= 0.5 * side[v] * (1 + 1e-12)), v


def test_refitted_walk_at_theta_zero_is_the_direct_sum():
    p0, p1, m = _drifted(1500, 23, 0.1)
    t = oracle.build_tree(p0, None, 8)
    ev = oracle.tree_forces(p1, m, 0.01, 0.0, 8, 32, tree=t, refit=True)
    a, _ = oracle.direct(p1, m, 0.01)
    assert ev.n_p2m == 0 and _rel(ev.acc, a).max() < 1e-12


def test_refitted_walk_never_accepts_a_cell_holding_a_target():
    p0, p1, m = _drifted(3000, 24, 0.2)
    t = oracle.build_tree(p0, None, 8)
    act = np.arange(0, 3000, 2)
    ev = oracle.tree_forces(p1, m, 0.01, 0.57, 8, 32, active=act, tree=t, refit=True)
    L = oracle.walk_lists(ev.tree, ev.mom, ev.groups, ev.box, ev.sel, 0.57, side=ev.side)
    sact = oracle.active_mask(3000, act)[t.perm.astype(np.int64)]
    for k, (p2m, p2p) in zip(ev.sel, L):
        cover = np.zeros(3000, np.int32)
        for v in np.concatenate([p2m, p2p]).astype(np.int64):
            cover[t.first[v]:t.first[v] + t.count[v]] += 1
        assert np.all(cover == 1)
        tg = np.nonzero(sact[ev.groups[k, 0]:ev.groups[k, 0] + ev.groups[k, 1]])[0]
        tg += ev.groups[k, 0]
        for v in p2m.astype(np.int64):
            assert not np.any((tg >= t.first[v]) & (tg < t.first[v] + t.count[v]))


def test_refitted_error_is_that_of_a_fresh_build():
    p0, p1, m = _drifted(4000, 25, 0.02)
    t = oracle.build_tree(p0, None, 8)
    ref, _ = oracle.direct(p1, m, 1e-3)
    fresh = oracle.tree_forces(p1, m, 1e-3, 0.5)
    refit = oracle.tree_forces(p1, m, 1e-3, 0.5, tree=t, refit=True)
    ef, er = _rel(fresh.acc, ref), _rel(refit.acc, ref)
    assert np.percentile(er, 99) < 1.5 * np.percentile(ef, 99)
    assert np.median(er) < 1.5 * np.median(ef)


def test_block_steps_rebuild_on_the_period_and_refit_between():
    from oracle import steps as osteps
    w = ics.hernquist_c4(n=4096)
    st = osteps.State(w.pos.copy(), w.vel.copy(), w.mass.copy(), w.eps, w.theta,
                      w.sys_off.copy(), w.bh_pos.reshape(-1, 3).copy(),
                      w.bh_vel.reshape(-1, 3).copy(), w.bh_mass.copy(), w.bh_eps.copy(),
                      np.array([0, 1], np.int64))
    osteps.forces(st)
    level = np.zeros(4096, np.uint8)
    t4 = np.full(4096, 0.3 ** 4 * w.eps ** 2)
    k, builds = 0, []
    for _ in range(24):
        before = st.tree
        k, act = osteps.block_substep(st, level, t4, k, 0.25, 6, rebuild_every=4)
        if st.tree is not before:
            builds.append(k)
        if act.size == 0:
            assert st.tree is before
    assert builds and all(b % 4 == 0 for b in builds)
