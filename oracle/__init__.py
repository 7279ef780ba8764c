"""Plain CPU oracle for the softened Barnes-Hut tree-gravity path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never does.  The arithmetic
lives in ``bh_oracle.c`` (plain C, double precision, no FMA contraction);
this module only marshals numpy arrays through ctypes.  It imports nothing
from the HIP package.

Every function follows a passage of the paper (Karl et al., rVINE):
multipole expansion about a group's centre of mass with direct near-field
sums (Sec. 1 and the integration-regions list of Sec. 2), Plummer softening
(Sec. 3), forces only for active particles and the leapfrog/block-step driver
(Sec. 2, the hybrid time-step recipe; Sec. 3 for the tau values).  Readings
where the paper is silent are marked in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall"]

MAX_LEVEL = 21


def build_sanitized(path: str) -> str:
    """Compile bh_oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer
    into ``path`` (for the CPU test that runs the oracle under them; load it
    through TG_ORACLE_LIB with the ASan runtime preloaded)."""
    subprocess.check_call(["gcc", *_CFLAGS, "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-o", path, _SRC, "-lm"])
    return path


def build(force: bool = True) -> str:
    """Compile bh_oracle.c into liboracle.so next to it (gcc)."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("TG_ORACLE_LIB")   # a sanitized build (tests)
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        L = C.CDLL(path)
        P = C.c_void_p
        i64, i32, f64 = C.c_int64, C.c_int32, C.c_double
        sig = {
            "or_max_threads": (C.c_int, []),
            "or_set_threads": (None, [C.c_int]),
            "or_cube": (None, [P, P, i32, P]),
            "or_keys": (None, [P, P, i32, P, P]),
            "or_sort": (C.c_int, [P, P, i32, P]),
            "or_build": (i64, [P, P, i32, i32, i64, P, P, P, P, P, P, P]),
            "or_keys42": (None, [P, P, i32, P, P, P]),
            "or_sort42": (C.c_int, [P, P, P, i32, P]),
            "or_build42": (i64, [P, P, P, i32, i32, i64, P, P, P, P, P, P, P]),
            "or_moments": (None, [P, P, i64, P, P, P]),
            "or_groups": (i64, [i64, P, P, P, P, P, P, i32, i64, P]),
            "or_group_boxes": (None, [P, P, i64, P, P, P]),
            "or_rel_records": (None, [i64, P, P, P, P, P, P, f64, P, P]),
            "or_refit_sides": (None, [i64, P, P, P, P, P, P, P, P]),
            "or_walk_lists": (C.c_int, [i64, P, P, P, P, P, P, P, P, P, i64, f64,
                                        P, P, P, P, P, P, P]),
            "or_tree_forces": (C.c_int, [i64, P, P, P, P, P, P, P, P, P, P, P, i64,
                                         P, P, P, f64, f64, P, P, P, f64, P, P, P, i32]),
            "or_direct": (None, [P, P, P, i32, P, P, i64, f64, P, P, P, i64, f64,
                                 P, P, i32]),
            "or_direct_pairs": (None, [P, P, P, i64, P, P, i64, C.c_int, f64,
                                       C.c_int, P, P, i32]),
            "or_kick": (None, [P, P, P, i64, P, f64]),
            "or_drift": (None, [P, P, i64, f64]),
            "or_levels": (None, [P, P, P, i64, f64, i32, i64, P]),
            "or_levels_v": (None, [P, P, P, P, P, i64, f64, i32, i64, P]),
            "or_active_at": (i64, [P, i64, i32, i64, P]),
            "or_p2m_single": (None, [P, P, f64, f64, P, i32]),
            "or_p2p_single": (None, [P, f64, P, f64, f64, P, i32]),
            "or_spline": (None, [f64, f64, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def max_threads() -> int:
    return int(lib().or_max_threads())


def _offsets(n, sys_off):
    if sys_off is None:
        return np.array([0, n], dtype=np.int64)
    off = _c(sys_off, np.int64)
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) >= 0)
    return off


@dataclass
class Tree:
    """Octree over the sorted keys of one or more systems."""
    off: np.ndarray      # int64 [S+1]
    cube: np.ndarray     # float64 [S, 4]: lo x, y, z, side L
    keys: np.ndarray     # uint64 [N], original order
    perm: np.ndarray     # uint32 [N], sorted rank -> original index
    skeys: np.ndarray    # uint64 [N], sorted
    level: np.ndarray    # uint8 [nn]
    first: np.ndarray    # uint32 [nn]
    count: np.ndarray    # uint32 [nn]
    child: np.ndarray    # uint32 [nn] first child id (0 for leaves)
    nchild: np.ndarray   # uint8 [nn]
    sys: np.ndarray      # int32 [nn]
    parent: np.ndarray   # uint32 [nn] (0xffffffff for roots)
    leaf_size: int
    levels: int = MAX_LEVEL          # 21, or 42 with two key words
    keys_lo: np.ndarray = None       # 42 levels: uint64 [N] last 21 digits, original order
    skeys_lo: np.ndarray = None      # 42 levels: the same, sorted

    @property
    def nn(self) -> int:
        return int(self.level.shape[0])

    def prefix(self) -> np.ndarray:
        """Key prefix of every node: key >> 3 * (21 - level) (21 levels)."""
        assert self.levels == MAX_LEVEL
        sh = (3 * (MAX_LEVEL - self.level.astype(np.uint64))).astype(np.uint64)
        return self.skeys[self.first.astype(np.int64)] >> sh


def cube_keys(pos, sys_off=None):
    """Bounding cube per system and Morton keys (original order)."""
    pos = _c(pos, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    off = _offsets(n, sys_off)
    S = off.shape[0] - 1
    cube = np.zeros((S, 4), np.float64)
    keys = np.zeros(n, np.uint64)
    lib().or_cube(_p(pos), _p(off), S, _p(cube))
    lib().or_keys(_p(pos), _p(off), S, _p(cube), _p(keys))
    return off, cube, keys


def build_tree(pos, sys_off=None, leaf_size: int = 8, levels: int = MAX_LEVEL) -> Tree:
    """Cube -> keys -> stable sort -> breadth-first octree (21 or 42 levels)."""
    pos = _c(pos, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    if levels == 42:
        return _build_tree42(pos, sys_off, leaf_size)
    assert levels == MAX_LEVEL
    off, cube, keys = cube_keys(pos, off_or_none(sys_off, n))
    S = off.shape[0] - 1
    perm = np.zeros(n, np.uint32)
    if lib().or_sort(_p(keys), _p(off), S, _p(perm)) != 0:
        raise MemoryError("oracle sort")
    skeys = keys[perm.astype(np.int64)] if n else keys.copy()
    cap = 4 * n + S + 64
    while True:
        level = np.zeros(cap, np.uint8)
        first = np.zeros(cap, np.uint32)
        count = np.zeros(cap, np.uint32)
        child = np.zeros(cap, np.uint32)
        nchild = np.zeros(cap, np.uint8)
        sysid = np.zeros(cap, np.int32)
        parent = np.zeros(cap, np.uint32)
        nn = lib().or_build(_p(skeys), _p(off), S, int(leaf_size), cap,
                            _p(level), _p(first), _p(count), _p(child),
                            _p(nchild), _p(sysid), _p(parent))
        if nn >= 0:
            break
        cap *= 2
    return Tree(off, cube, keys, perm, skeys, level[:nn].copy(),
                first[:nn].copy(), count[:nn].copy(), child[:nn].copy(),
                nchild[:nn].copy(), sysid[:nn].copy(), parent[:nn].copy(),
                int(leaf_size))


def _build_tree42(pos, sys_off, leaf_size):
    n = pos.shape[0]
    off = _offsets(n, off_or_none(sys_off, n))
    S = off.shape[0] - 1
    cube = np.zeros((S, 4), np.float64)
    lib().or_cube(_p(pos), _p(off), S, _p(cube))
    khi = np.zeros(n, np.uint64)
    klo = np.zeros(n, np.uint64)
    lib().or_keys42(_p(pos), _p(off), S, _p(cube), _p(khi), _p(klo))
    perm = np.zeros(n, np.uint32)
    if lib().or_sort42(_p(khi), _p(klo), _p(off), S, _p(perm)) != 0:
        raise MemoryError("oracle sort")
    p = perm.astype(np.int64)
    skhi = khi[p] if n else khi.copy()
    sklo = klo[p] if n else klo.copy()
    cap = 4 * n + S + 64
    while True:
        level = np.zeros(cap, np.uint8)
        first = np.zeros(cap, np.uint32)
        count = np.zeros(cap, np.uint32)
        child = np.zeros(cap, np.uint32)
        nchild = np.zeros(cap, np.uint8)
        sysid = np.zeros(cap, np.int32)
        parent = np.zeros(cap, np.uint32)
        nn = lib().or_build42(_p(skhi), _p(sklo), _p(off), S, int(leaf_size), cap,
                              _p(level), _p(first), _p(count), _p(child),
                              _p(nchild), _p(sysid), _p(parent))
        if nn >= 0:
            break
        cap *= 2
    return Tree(off, cube, khi, perm, skhi, level[:nn].copy(), first[:nn].copy(),
                count[:nn].copy(), child[:nn].copy(), nchild[:nn].copy(), sysid[:nn].copy(),
                parent[:nn].copy(), int(leaf_size), 42, klo, sklo)


def off_or_none(sys_off, n):
    return None if sys_off is None else _offsets(n, sys_off)


def sorted_arrays(tree: Tree, pos, mass):
    p = tree.perm.astype(np.int64)
    spos = np.ascontiguousarray(_c(pos, np.float64).reshape(-1, 3)[p])
    smass = np.ascontiguousarray(_c(mass, np.float64)[p])
    return spos, smass


def moments(tree: Tree, spos, smass) -> np.ndarray:
    """[nn, 10]: M, com x, y, z, Sxx, Syy, Szz, Sxy, Sxz, Syz."""
    mom = np.zeros((tree.nn, 10), np.float64)
    lib().or_moments(_p(_c(spos, np.float64)), _p(_c(smass, np.float64)),
                     tree.nn, _p(tree.first), _p(tree.count), _p(mom))
    return mom


def groups(tree: Tree, group_size: int) -> np.ndarray:
    """[ng, 4] uint32: first, count, node, system (ordered by first)."""
    cap = tree.count.shape[0] + int(tree.off[-1]) + 16
    g = np.zeros((cap, 4), np.uint32)
    ng = lib().or_groups(tree.nn, _p(tree.level), _p(tree.first),
                         _p(tree.count), _p(tree.child), _p(tree.nchild),
                         _p(tree.sys), int(group_size), cap, _p(g))
    if ng < 0:
        raise MemoryError("oracle groups")
    return g[:ng].copy()


def group_boxes(spos, sactive, g):
    box = np.zeros((g.shape[0], 6), np.float64)
    nact = np.zeros(g.shape[0], np.int32)
    lib().or_group_boxes(_p(_c(spos, np.float64)), _p(_c(sactive, np.uint8)),
                         g.shape[0], _p(_c(g, np.uint32)), _p(box), _p(nact))
    return box, nact


def active_mask(n, active=None):
    """uint8 mask in ORIGINAL order from an index list (None = all)."""
    m = np.zeros(n, np.uint8)
    if active is None:
        m[:] = 1
    else:
        m[np.asarray(active, np.int64)] = 1
    return m


def rel_records(tree: Tree, mom, G=1.0, side=None) -> np.ndarray:
    """[nn, 8] per cell: the 1.2x cube {lo x, y, z, P = (G M) s^2, hi x, y, z, 0}
    of the relative opening test (s = side[v] for a refitted tree)."""
    rel = np.zeros((tree.nn, 8), np.float64)
    side = None if side is None else _c(side, np.float64)
    lib().or_rel_records(tree.nn, _p(tree.level), _p(tree.first), _p(tree.sys),
                         _p(tree.skeys), _p(tree.cube), _p(_c(mom, np.float64)),
                         float(G), _p(side), _p(rel))
    return rel


def refit_sides(tree: Tree, spos) -> np.ndarray:
    """[nn] opening size of every cell of a refitted tree (see or_refit_sides)."""
    side = np.zeros(tree.nn, np.float64)
    lib().or_refit_sides(tree.nn, _p(tree.level), _p(tree.first), _p(tree.count),
                         _p(tree.sys), _p(tree.skeys), _p(tree.cube),
                         _p(_c(spos, np.float64)), _p(side))
    return side


def group_arel(tree: Tree, g, sactive, acc_old, alpha: float) -> np.ndarray:
    """Per group: (alpha alpha) * min over its active targets of |a_old|^2,
    |a|^2 = (ax ax + ay ay) + az az (acc_old in original order; 0 for a
    group without active targets)."""
    n = tree.perm.shape[0]
    out = np.zeros(g.shape[0], np.float64)
    if n == 0 or g.shape[0] == 0:
        return out
    a = _c(acc_old, np.float64).reshape(-1, 3)[tree.perm.astype(np.int64)]
    a2 = (a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1]) + a[:, 2] * a[:, 2]
    a2 = np.where(np.asarray(sactive, bool), a2, np.inf)
    m = np.minimum.reduceat(a2, g[:, 0].astype(np.int64))
    aa = float(alpha) * float(alpha)
    return aa * np.where(np.isfinite(m), m, 0.0)


def walk_lists(tree: Tree, mom, g, box, sel, theta: float, rel=None, arel=None, side=None):
    """Sorted P2M and P2P node-id lists for each selected group (relative
    opening test when rel / arel are given, see :func:`rel_records`)."""
    sel = _c(sel, np.int32)
    ns = sel.shape[0]
    np2m = np.zeros(ns, np.int64)
    np2p = np.zeros(ns, np.int64)
    rel = None if rel is None else _c(rel, np.float64)
    arel = None if arel is None else _c(arel, np.float64)
    side = None if side is None else _c(side, np.float64)
    args = (tree.nn, _p(tree.level), _p(tree.child), _p(tree.nchild),
            _p(tree.sys), _p(_c(mom, np.float64)), _p(tree.cube),
            _p(_c(g, np.uint32)), _p(_c(box, np.float64)), _p(sel), ns,
            float(theta), _p(side), _p(rel), _p(arel), _p(np2m), _p(np2p))
    if lib().or_walk_lists(*args, None, None) != 0:
        raise MemoryError("oracle walk")
    sizes = np.stack([np2m, np2p], 1).reshape(-1)
    lofs = np.zeros(sizes.shape[0], np.int64)
    if sizes.shape[0]:
        lofs[1:] = np.cumsum(sizes)[:-1]
    ids = np.zeros(int(sizes.sum()), np.uint32)
    if lib().or_walk_lists(*args, _p(lofs), _p(ids)) != 0:
        raise MemoryError("oracle walk")
    out = []
    for t in range(ns):
        a, b = lofs[2 * t], lofs[2 * t + 1]
        out.append((ids[a:a + np2m[t]].copy(), ids[b:b + np2p[t]].copy()))
    return out


@dataclass
class Evaluation:
    tree: Tree
    mom: np.ndarray
    groups: np.ndarray
    box: np.ndarray
    nact: np.ndarray
    sel: np.ndarray          # selected (evaluated) group indices
    acc: np.ndarray          # [N, 3] original order (NaN where not evaluated)
    pot: np.ndarray          # [N]
    n_p2p: int
    n_p2m: int
    n_targets: int
    rel: np.ndarray = None   # relative test: cell records and per-group A
    arel: np.ndarray = None
    side: np.ndarray = None  # refitted tree: opening size per cell


SOFTENINGS = {"plummer": 0, "spline": 1}


def _soft(softening):
    try:
        return SOFTENINGS[softening]
    except KeyError:
        raise ValueError("softening must be 'plummer' or 'spline'") from None


def spline_psi(r, h):
    """Cubic-spline softening (support 2h): psi, psi_1, psi_2, psi_3 at r,
    psi_{k+1} = -(1/r) d psi_k / dr, Newtonian 1/r, 1/r^3, 3/r^5, 15/r^7
    beyond 2h."""
    out = np.zeros(4)
    lib().or_spline(float(r), float(h), _p(out))
    return out


def tree_forces(pos, mass, eps, theta, leaf_size=8, group_size=64, active=None,
                sys_off=None, G=1.0, sel_groups=None, tree=None, alpha=None,
                acc_old=None, refit=False, softening="plummer", levels=MAX_LEVEL):
    """Build, moments, groups, walk and evaluation, all in the oracle.

    ``active``: original indices of the targets (None = all).  ``sel_groups``:
    evaluate only these group indices (None = every group with a target).
    With ``alpha`` (and ``acc_old``, [N, 3] original order) the walk uses the
    relative opening test instead of theta.  ``refit``: ``tree`` is an earlier
    build kept as it is (order, nodes, groups) for the current positions, the
    cells opened by their refitted sizes (:func:`refit_sides`).
    ``softening``: "plummer" (eps) or "spline" (cubic spline, h = eps).
    Returns an :class:`Evaluation`; acc/pot are NaN for rows not evaluated.
    """
    pos = _c(pos, np.float64).reshape(-1, 3)
    n = pos.shape[0]
    if tree is None:
        tree = build_tree(pos, sys_off, leaf_size, levels)
    if tree.levels != MAX_LEVEL and (alpha is not None or refit):
        raise ValueError("the relative test and refit take 21-level trees")
    spos, smass = sorted_arrays(tree, pos, mass)
    mom = moments(tree, spos, smass)
    g = groups(tree, group_size)
    sact = active_mask(n, active)[tree.perm.astype(np.int64)]
    box, nact = group_boxes(spos, sact, g)
    if sel_groups is None:
        sel = np.nonzero(nact > 0)[0].astype(np.int32)
    else:
        sel = _c(sel_groups, np.int32)
        sel = sel[nact[sel] > 0]
    side = refit_sides(tree, spos) if refit else None
    rel = arel = None
    if alpha is not None:
        rel = rel_records(tree, mom, G, side)
        arel = group_arel(tree, g, sact, acc_old, alpha)
    sacc = np.full((n, 3), np.nan)
    spot = np.full(n, np.nan)
    counts = np.zeros(3, np.int64)
    rc = lib().or_tree_forces(
        tree.nn, _p(tree.level), _p(tree.first), _p(tree.count),
        _p(tree.child), _p(tree.nchild), _p(tree.sys), _p(mom), _p(tree.cube),
        _p(g), _p(box), _p(sel), sel.shape[0], _p(spos), _p(smass), _p(sact),
        float(eps), float(theta), _p(side), _p(rel), _p(arel), float(G), _p(sacc),
        _p(spot), _p(counts), _soft(softening))
    if rc != 0:
        raise MemoryError("oracle tree forces")
    acc = np.full((n, 3), np.nan)
    pot = np.full(n, np.nan)
    p = tree.perm.astype(np.int64)
    acc[p] = sacc
    pot[p] = spot
    return Evaluation(tree, mom, g, box, nact, sel, acc, pot, int(counts[0]),
                      int(counts[1]), int(counts[2]), rel, arel, side)


def direct(pos, mass, eps, targets=None, sys_off=None, xpos=None, xmass=None,
           xeps=None, G=1.0, softening="plummer"):
    """Exact softened direct sum (long double) for the listed targets.

    Sources: every other particle of the target's own system (softening eps)
    plus optional external masses (pair softening max(eps, xeps)).
    """
    pos = _c(pos, np.float64).reshape(-1, 3)
    mass = _c(mass, np.float64)
    n = pos.shape[0]
    off = _offsets(n, sys_off)
    tgt = np.arange(n, dtype=np.int64) if targets is None else _c(targets, np.int64)
    sysof = (np.searchsorted(off, tgt, side="right") - 1).astype(np.int32)
    if xpos is None:
        xpos = np.zeros((0, 3)); xmass = np.zeros(0); xeps = np.zeros(0)
    xpos = _c(xpos, np.float64).reshape(-1, 3)
    xmass = _c(xmass, np.float64)
    xeps = _c(np.broadcast_to(xeps, xmass.shape), np.float64)
    acc = np.zeros((tgt.shape[0], 3))
    pot = np.zeros(tgt.shape[0])
    lib().or_direct(_p(pos), _p(mass), _p(off), off.shape[0] - 1, _p(sysof),
                    _p(tgt), tgt.shape[0], float(eps), _p(xpos), _p(xmass),
                    _p(xeps), xmass.shape[0], float(G), _p(acc), _p(pot),
                    _soft(softening))
    return acc, pot


def direct_pairs(spos, sm, seps, tpos, teps, self_pairs=False, G=1.0,
                 acc=None, pot=None, softening="plummer"):
    """Double-precision pair forces, pair softening max(eps_i, eps_j)."""
    spos = _c(spos, np.float64).reshape(-1, 3)
    sm = _c(sm, np.float64)
    seps = _c(np.broadcast_to(seps, sm.shape), np.float64)
    tpos = _c(tpos, np.float64).reshape(-1, 3)
    teps = _c(np.broadcast_to(teps, (tpos.shape[0],)), np.float64)
    accumulate = acc is not None
    if acc is None:
        acc = np.zeros((tpos.shape[0], 3))
        pot = np.zeros(tpos.shape[0])
    lib().or_direct_pairs(_p(spos), _p(sm), _p(seps), sm.shape[0], _p(tpos),
                          _p(teps), tpos.shape[0], int(bool(self_pairs)),
                          float(G), int(accumulate), _p(acc), _p(pot), _soft(softening))
    return acc, pot


def kick(vel, acc, dt, idx=None, level=None):
    """In place: v += a * h, h = dt/2, or (dt * 2^-level)/2 per particle."""
    assert vel.dtype == np.float64 and vel.flags.c_contiguous
    acc = _c(acc, np.float64)
    n = vel.shape[0] if idx is None else len(idx)
    idx = None if idx is None else _c(idx, np.int32)
    level = None if level is None else _c(level, np.uint8)
    lib().or_kick(_p(vel), _p(acc), _p(idx), n, _p(level), float(dt))


def drift(pos, vel, dt):
    assert pos.dtype == np.float64 and pos.flags.c_contiguous
    lib().or_drift(_p(pos), _p(_c(vel, np.float64)), pos.shape[0], float(dt))


def levels(acc, tau4eps2, level, dt_max, nlev, k, idx=None, vel=None, tau2eps2v=None):
    """In place: new block levels for the listed (active) particles; with vel
    and tau2eps2v = tau_vel^2 eps^2 also the velocity criterion."""
    assert level.dtype == np.uint8 and level.flags.c_contiguous
    acc = _c(acc, np.float64)
    n = acc.shape[0] if idx is None else len(idx)
    idx = None if idx is None else _c(idx, np.int32)
    if vel is None:
        lib().or_levels(_p(acc), _p(_c(tau4eps2, np.float64)), _p(idx), n,
                        float(dt_max), int(nlev), int(k), _p(level))
    else:
        lib().or_levels_v(_p(acc), _p(_c(vel, np.float64)), _p(_c(tau4eps2, np.float64)),
                          _p(_c(tau2eps2v, np.float64)), _p(idx), n, float(dt_max),
                          int(nlev), int(k), _p(level))


def active_at(level, nlev, k):
    level = _c(level, np.uint8)
    idx = np.zeros(level.shape[0], np.int32)
    m = lib().or_active_at(_p(level), level.shape[0], int(nlev), int(k), _p(idx))
    return idx[:m].copy()


def p2m_single(cell, x, eps, G=1.0, softening="plummer"):
    """One multipole term: cell = [M, c(3), S(6)] -> (acc[3], phi)."""
    out = np.zeros(4)
    lib().or_p2m_single(_p(_c(cell, np.float64)), _p(_c(x, np.float64)),
                        float(eps), float(G), _p(out), _soft(softening))
    return out[:3].copy(), float(out[3])


def p2p_single(src, m, x, eps, G=1.0, softening="plummer"):
    """One softened particle term -> (acc[3], phi)."""
    out = np.zeros(4)
    lib().or_p2p_single(_p(_c(src, np.float64)), float(m), _p(_c(x, np.float64)),
                        float(eps), float(G), _p(out), _soft(softening))
    return out[:3].copy(), float(out[3])
