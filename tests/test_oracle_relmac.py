"""Pins for the oracle's relative opening test (the paper's tree runs use a
relative "Gadget" criterion with an error tolerance, Sec. 3, run set-up; the
rule itself is Springel 2005, MNRAS 364, 1105, Sec. 3.1, taken per group).

Independent references: the cell cubes must contain their particles and tile
their parents (geometry of the octree); alpha = 0 opens every cell, so the
walk is the direct sum; a hand-built two-cluster system where the flip of the
decision sits exactly at the closed-form threshold alpha* = G M s^2 /
(|a| d^4), and where only the 20 % separation rule decides; the force error
against the direct sum falls with alpha.
"""
import numpy as np
import pytest

import oracle
from paper_1507_01009_amd import ics


def _rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def test_cell_cubes_hold_their_particles_and_tile_their_parents():
    pos = ics.dehnen(3000, 1.0, 33)[0]
    t = oracle.build_tree(pos, None, 6)
    sp, sm = oracle.sorted_arrays(t, pos, np.full(3000, 1.0 / 3000))
    mom = oracle.moments(t, sp, sm)
    rel = oracle.rel_records(t, mom, G=1.0)
    lo, hi = rel[:, 0:3], rel[:, 4:7]
    g = 0.5 * (lo + hi)
    s = t.cube[t.sys, 3] * 2.0 ** -t.level.astype(float)
    # the enlarged cube is 1.2 cell sides wide
    assert np.allclose(hi - lo, 1.2 * s[:, None], rtol=1e-12, atol=0)
    tol = 1e-12 * t.cube[0, 3]
    for v in range(t.nn):
        x = sp[t.first[v]:t.first[v] + t.count[v]]
        assert np.all(x >= g[v] - 0.5 * s[v] - tol) and np.all(x <= g[v] + 0.5 * s[v] + tol), v
        if t.nchild[v]:
            for c in range(t.child[v], t.child[v] + t.nchild[v]):
                off = (g[c] - g[v]) / (0.25 * s[v])
                assert np.allclose(np.abs(off), 1.0, atol=1e-9), (v, c)
    # P = G M s^2 with M the cell mass
    assert np.allclose(rel[:, 3], mom[:, 0] * s * s, rtol=1e-15, atol=0)


def test_alpha_zero_opens_everything_and_gives_the_direct_sum():
    pos, _, m = ics.plummer(1500, 8)
    aold = oracle.tree_forces(pos, m, 0.01, 0.5).acc
    ev = oracle.tree_forces(pos, m, 0.01, 0.5, 8, 32, alpha=0.0, acc_old=aold)
    a, p = oracle.direct(pos, m, 0.01)
    assert ev.n_p2m == 0
    assert ev.n_p2p == 1500 * 1499
    assert _rel(ev.acc, a).max() < 1e-12
    assert np.max(np.abs(ev.pot - p) / np.abs(p)) < 1e-12


def _two_clusters(target):
    """Anchor at the origin and a target in octant 0 of the unit cube; eight
    equal masses on the corners of the 1/64 cube at the far corner.  With
    n_L = 4 the cluster forms one node on each of levels 1..6 (side 2^-l,
    centre of mass 127/128 on every axis), split into single particles on
    level 7."""
    b = 1.0 / 64.0
    corners = np.array([[1 - b + b * i, 1 - b + b * j, 1 - b + b * k]
                        for i in (0, 1) for j in (0, 1) for k in (0, 1)])
    pos = np.vstack([[0.0, 0.0, 0.0], target, corners])
    m = np.full(10, 0.125)
    return pos, m


def _accepted(pos, m, alpha, aold, active):
    ev = oracle.tree_forces(pos, m, 1e-4, 0.5, 4, 4, active=active, alpha=alpha,
                            acc_old=aold)
    sel = ev.sel
    L = oracle.walk_lists(ev.tree, ev.mom, ev.groups, ev.box, sel, 0.5,
                          rel=ev.rel, arel=ev.arel)
    cells = np.concatenate([p2m for p2m, _ in L]).astype(np.int64)
    return ev, cells


@pytest.mark.parametrize("a_target", [1.0, 3.0])
def test_flip_sits_at_the_closed_form_threshold(a_target):
    pos, m = _two_clusters([0.1, 0.2, 0.05])
    aold = np.zeros((10, 3))
    aold[1] = [0.0, a_target, 0.0]
    M = 8 * 0.125
    c = 127.0 / 128.0
    box = pos[1]
    d4 = np.sum((c - box) ** 2) ** 2
    for lev in range(1, 7):
        s = 2.0 ** -lev
        astar = M * s * s / (a_target * d4)
        ev, cells = _accepted(pos, m, astar * (1 + 1e-9), aold, [1])
        assert ev.tree.level[cells].tolist() == [lev], (lev, "above")
        ev, cells = _accepted(pos, m, astar * (1 - 1e-9), aold, [1])
        # below the level-6 threshold the single corners (level 7, side
        # 1/128) are accepted as cells of their own
        expect = [lev + 1] if lev < 6 else [7] * 8
        assert ev.tree.level[cells].tolist() == expect, (lev, "below")
    # below every threshold the eight corners are summed one by one
    ev, cells = _accepted(pos, m, 1e-9, aold, [1])
    assert cells.size == 0 and ev.n_p2p == 9


def test_smallest_old_acceleration_of_the_group_decides():
    pos, m = _two_clusters([0.1, 0.2, 0.05])
    aold = np.zeros((10, 3))
    aold[0] = [0.5, 0.0, 0.0]     # anchor: half the target's |a|
    aold[1] = [0.0, 1.0, 0.0]
    c = 127.0 / 128.0
    d4 = np.sum((c - np.max(pos[:2], 0)) ** 2) ** 2   # group box of both
    astar = 1.0 * 0.25 / (0.5 * d4)                   # level 1, |a| = 0.5
    ev, cells = _accepted(pos, m, astar * (1 + 1e-9), aold, [0, 1])
    assert ev.tree.level[cells].tolist() == [1]
    ev, cells = _accepted(pos, m, astar * (1 - 1e-9), aold, [0, 1])
    assert ev.tree.level[cells].tolist() == [2]


@pytest.mark.parametrize("target,level", [([0.46, 0.46, 0.46], 2),
                                          ([0.44, 0.46, 0.46], 1),
                                          ([0.46, 0.44, 0.46], 1),
                                          ([0.46, 0.46, 0.44], 1)])
def test_separation_rule_alone(target, level):
    # level-1 cluster cell: centre 0.75, enlarged half width 0.3 -> [0.45,
    # 1.05] on every axis; with a huge alpha only that rule decides
    pos, m = _two_clusters(target)
    aold = np.zeros((10, 3))
    aold[1] = [1.0, 0.0, 0.0]
    ev, cells = _accepted(pos, m, 1e30, aold, [1])
    assert ev.tree.level[cells].tolist() == [level]


def test_walk_covers_every_particle_once_and_skips_own_cells():
    pos, _, m = ics.dehnen(3000, 1.0, 21)
    act = np.arange(0, 3000, 3)
    aold = oracle.tree_forces(pos, m, 0.01, 0.5).acc
    ev = oracle.tree_forces(pos, m, 0.01, 0.5, 8, 32, active=act, alpha=1e-3,
                            acc_old=aold)
    L = oracle.walk_lists(ev.tree, ev.mom, ev.groups, ev.box, ev.sel, 0.5,
                          rel=ev.rel, arel=ev.arel)
    t = ev.tree
    sact = oracle.active_mask(3000, act)[t.perm.astype(np.int64)]
    for k, (p2m, p2p) in zip(ev.sel, L):
        cover = np.zeros(3000, np.int32)
        for v in np.concatenate([p2m, p2p]).astype(np.int64):
            cover[t.first[v]:t.first[v] + t.count[v]] += 1
        assert np.all(cover == 1)
        assert np.all(t.nchild[p2p.astype(np.int64)] == 0)
        tg = np.nonzero(sact[ev.groups[k, 0]:ev.groups[k, 0] + ev.groups[k, 1]])[0]
        tg += ev.groups[k, 0]
        for v in p2m.astype(np.int64):
            assert not np.any((tg >= t.first[v]) & (tg < t.first[v] + t.count[v]))


def test_error_falls_with_alpha():
    pos, _, m = ics.dehnen(4000, 1.0, 5)
    eps = 1e-3
    a_ref, _ = oracle.direct(pos, m, eps)
    aold = oracle.tree_forces(pos, m, eps, 0.5).acc
    med, work = [], []
    for alpha in (1e-2, 1e-3, 1e-4):
        ev = oracle.tree_forces(pos, m, eps, 0.5, 8, 64, alpha=alpha, acc_old=aold)
        e = _rel(ev.acc, a_ref)
        med.append(np.median(e))
        work.append(ev.n_p2p + ev.n_p2m)
        if alpha == 1e-3:
            assert np.percentile(e, 99) < 1e-3
    assert med[0] > med[1] > med[2]
    assert work[0] < work[1] < work[2]
