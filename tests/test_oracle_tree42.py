"""Pins for the oracle's 42-level keys, sort and octree (two key words).

Independent references: the Morton key built from Python integers bit by
bit, numpy's lexicographic sort, a recursive geometric subdivision on the
42-bit integer cell coordinates, and the 21-level tree, which the 42-level
one must reproduce wherever 21 levels resolve every leaf (the first 21
digits of a 42-bit key are the 21-bit key: 2^42 / L is 2^21 / L scaled by
a power of two, so the quantised coordinates agree in their top bits).
On an untruncated cusp, where 21 levels leave the centre in over-full
leaves, 42 levels resolve it.
"""
from collections import deque

import numpy as np
import pytest

import oracle
from paper_1507_01009_amd import ics

NB = 42


def _q42(pos, lo, L):
    t = pos - lo[None, :]
    u = t * (2.0 ** NB / L)
    q = np.floor(u)
    q = np.where(q <= 0, 0, q)
    return np.minimum(q.astype(np.int64), 2 ** NB - 1)


def _key_words(q):
    """(hi, lo) words of the interleaved 126-bit key, from Python integers."""
    hi = np.zeros(q.shape[0], np.uint64)
    lo = np.zeros(q.shape[0], np.uint64)
    for i in range(q.shape[0]):
        k = 0
        for j in range(NB - 1, -1, -1):
            k = (k << 3) | (((int(q[i, 0]) >> j) & 1) << 2) | (((int(q[i, 1]) >> j) & 1) << 1) \
                | ((int(q[i, 2]) >> j) & 1)
        hi[i] = np.uint64(k >> 63)
        lo[i] = np.uint64(k & ((1 << 63) - 1))
    return hi, lo


def _geometric_tree(q, nleaf):
    out = []
    dq = deque([(0, np.arange(q.shape[0]), np.zeros(3, np.int64))])
    while dq:
        lev, mem, corner = dq.popleft()
        rec = {"level": lev, "members": set(mem.tolist()), "children": []}
        out.append(rec)
        if len(mem) > nleaf and lev < NB:
            half = 2 ** (NB - lev - 1)
            side = (q[mem] - corner[None, :]) >= half
            for o in range(8):
                b = np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1], bool)
                sel = mem[np.all(side == b[None, :], axis=1)]
                if sel.size:
                    rec["children"].append(len(out) + len(dq))
                    dq.append((lev + 1, sel, corner + half * b.astype(np.int64)))
    return out


def _deep_cluster(n, seed):
    """A wide sphere with a tight clump at a point: 21 levels cannot split
    the clump, 42 can."""
    return ics.clump_in_halo(n, seed)


@pytest.mark.parametrize("seed,nleaf", [(1, 1), (2, 4), (3, 8)])
def test_keys_sort_and_tree_match_geometry_at_42_levels(seed, nleaf):
    pos = _deep_cluster(160, seed)
    t = oracle.build_tree(pos, None, nleaf, 42)
    lo = pos.min(0)
    L = float((pos.max(0) - lo).max())
    assert np.array_equal(t.cube[0], np.r_[lo, L])
    q = _q42(pos, lo, L)
    hi, klo = _key_words(q)
    assert np.array_equal(t.keys, hi) and np.array_equal(t.keys_lo, klo)
    ref_perm = np.lexsort((np.arange(pos.shape[0]), klo, hi))
    assert np.array_equal(t.perm.astype(np.int64), ref_perm)
    ref = _geometric_tree(q, nleaf)
    assert t.nn == len(ref)
    for v, r in enumerate(ref):
        assert t.level[v] == r["level"]
        assert set(t.perm[t.first[v]:t.first[v] + t.count[v]].tolist()) == r["members"]
        assert t.nchild[v] == len(r["children"])
        if r["children"]:
            assert list(range(t.child[v], t.child[v] + t.nchild[v])) == r["children"]
    assert t.level.max() > 21


def test_first_word_is_the_21_level_key_and_trees_agree_when_resolved():
    pos, _, _ = ics.plummer(4000, 11)
    t21 = oracle.build_tree(pos, None, 8)
    t42 = oracle.build_tree(pos, None, 8, 42)
    assert np.array_equal(t42.keys, t21.keys)
    # 21 levels resolve this sample (no over-full leaf), so the trees agree
    assert not np.any((t21.nchild == 0) & (t21.count > 8))
    for f in ("perm", "level", "first", "count", "child", "nchild", "parent"):
        assert np.array_equal(getattr(t42, f), getattr(t21, f)), f
    # a deep clump: the first words still equal the 21-level keys
    pos = _deep_cluster(3000, 5)
    assert np.array_equal(oracle.build_tree(pos, None, 8, 42).keys,
                          oracle.build_tree(pos, None, 8).keys)


def test_untruncated_cusp_is_resolved_at_42_levels():
    """A Dehnen gamma = 1.5 sample without the 0.99 mass truncation reaches
    r ~ 1e5 at N = 40 000; with 21 levels its centre sits in over-full
    leaves, with 42 levels every leaf holds at most n_L."""
    pos, _, m = ics.dehnen(40000, 1.5, ics.SEED_BASE + 77, mass_fraction=1.0 - 1e-9)
    r = np.linalg.norm(pos, axis=1)
    assert r.max() > 1e4
    t21 = oracle.build_tree(pos, None, 8)
    t42 = oracle.build_tree(pos, None, 8, 42)
    full21 = (t21.nchild == 0) & (t21.count > 8)
    assert full21.any() and t21.count[full21].sum() > 50
    assert not np.any((t42.nchild == 0) & (t42.count > 8))
    assert t42.level.max() > 21
    # structure invariants: children partition the parent, counts decrease
    inner = np.nonzero(t42.nchild > 0)[0]
    for v in inner[:2000]:
        c0, nc = int(t42.child[v]), int(t42.nchild[v])
        assert t42.first[c0] == t42.first[v]
        assert t42.count[c0:c0 + nc].sum() == t42.count[v]
        assert np.all(t42.level[c0:c0 + nc] == t42.level[v] + 1)
        assert np.all(t42.parent[c0:c0 + nc] == v)
    # the forces of the deep tree at theta = 0 are the direct sum
    sel = np.arange(0, 40000, 97)
    ev = oracle.tree_forces(pos, m, 1e-3, 0.0, 8, 64, active=sel, levels=42)
    a, _ = oracle.direct(pos, m, 1e-3, sel)
    e = np.linalg.norm(ev.acc[sel] - a, axis=1) / np.linalg.norm(a, axis=1)
    assert e.max() < 1e-12
