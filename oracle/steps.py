"""Plain CPU oracle of whole steps (TEST INFRASTRUCTURE ONLY).

Composes the oracle's primitives in the order of the paper's hybrid step
(Sec. 2, steps (1), (6), (7)), read as kick-drift-kick:

* forces: tree forces on the listed stars (opening angle, or with ``alpha``
  the relative test against the stars' current accelerations) plus the FP64
  softened (Plummer, or the cubic spline) force of the
  SMBHs of the star's system (pair softening max(eps_star, eps_bh)); every
  SMBH feels all stars of its system and the other SMBHs (Sec. 2, the
  perturber / chain force-correction paragraph).
* KDK step: v += a dt/2 (stars, SMBHs), x += v dt, forces, v += a dt/2.
* Frozen stars (ghost chain members, Sec. 2) are never kicked, drifted or
  active; they stay sources of the tree forces.
* block substep (power-of-two levels, smallest step dt_min):
  closing half kicks of the stars active at k (not at k = 0) with their old
  level, new levels at k, opening half kicks with the new level, SMBH half
  kicks of dt_min/2 (SMBHs always on the smallest step), drift of all by
  dt_min, k += 1, forces for the stars active at the new k.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle


@dataclass
class State:
    pos: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    eps: float
    theta: float
    sys_off: np.ndarray
    bh_pos: np.ndarray
    bh_vel: np.ndarray
    bh_mass: np.ndarray
    bh_eps: np.ndarray
    bh_seg: np.ndarray
    leaf_size: int = 8
    group_size: int = 64
    alpha: float = None      # relative opening test (None: opening angle theta)
    frozen: np.ndarray = None  # bool [n]: stars held still (ghost chain members)
    tree: object = None        # the last tree built (refitted between builds)
    softening: str = "plummer"  # or "spline" (cubic spline, h = eps)
    acc: np.ndarray = field(default=None)
    pot: np.ndarray = field(default=None)
    bh_acc: np.ndarray = field(default=None)
    bh_pot: np.ndarray = field(default=None)

    def __post_init__(self):
        n, nb = self.pos.shape[0], self.bh_mass.shape[0]
        if self.acc is None:
            self.acc = np.zeros((n, 3))
            self.pot = np.zeros(n)
        if self.bh_acc is None:
            self.bh_acc = np.zeros((nb, 3))
            self.bh_pot = np.zeros(nb)


def forces(st: State, active=None, k=None, rebuild_every=0):
    """Tree + SMBH forces for the listed stars; SMBH forces for all SMBHs.
    With a rebuild period (block steps, substep k) the tree is rebuilt when k
    is a multiple of it or none was built yet, and refitted otherwise (READING
    of Sec. 2 step 7, which updates the tree structure when needed without a
    rule).  No tree work when the list is empty.  ``st.softening`` applies to
    every pair, the SMBH ones included."""
    n = st.pos.shape[0]
    S = st.sys_off.shape[0] - 1
    rows = np.arange(n) if active is None else np.asarray(active, np.int64)
    if rows.size:
        rel = {} if st.alpha is None else {"alpha": st.alpha, "acc_old": st.acc.copy()}
        refit = (rebuild_every > 1 and k is not None and st.tree is not None
                 and k % rebuild_every != 0)
        ev = oracle.tree_forces(st.pos, st.mass, st.eps, st.theta, st.leaf_size,
                                st.group_size, active=active, sys_off=st.sys_off,
                                tree=st.tree if refit else None, refit=refit,
                                softening=st.softening, **rel)
        if not refit:
            st.tree = ev.tree
        st.acc[rows] = ev.acc[rows]
        st.pot[rows] = ev.pot[rows]
    else:
        ev = None
    for s in range(S):
        b0, b1 = int(st.bh_seg[s]), int(st.bh_seg[s + 1])
        if b1 == b0:
            continue
        lo, hi = int(st.sys_off[s]), int(st.sys_off[s + 1])
        r = rows[(rows >= lo) & (rows < hi)]
        if r.size:
            a, p = oracle.direct_pairs(st.bh_pos[b0:b1], st.bh_mass[b0:b1],
                                       st.bh_eps[b0:b1], st.pos[r], st.eps,
                                       softening=st.softening)
            st.acc[r] += a
            st.pot[r] += p
        a, p = oracle.direct_pairs(st.pos[lo:hi], st.mass[lo:hi], st.eps,
                                   st.bh_pos[b0:b1], st.bh_eps[b0:b1],
                                   softening=st.softening)
        oracle.direct_pairs(st.bh_pos[b0:b1], st.bh_mass[b0:b1], st.bh_eps[b0:b1],
                            st.bh_pos[b0:b1], st.bh_eps[b0:b1], self_pairs=True,
                            acc=a, pot=p, softening=st.softening)
        st.bh_acc[b0:b1] = a
        st.bh_pot[b0:b1] = p
    return ev


def _moving(st: State):
    """Indices of the stars that move (all unless some are frozen)."""
    if st.frozen is None:
        return None
    return np.nonzero(~np.asarray(st.frozen, bool))[0]


def _kick_stars(st: State, dt, idx=None, level=None):
    mv = _moving(st)
    if mv is not None:
        idx = mv if idx is None else np.asarray(idx)[~np.asarray(st.frozen, bool)[idx]]
    oracle.kick(st.vel, st.acc, dt, idx=idx, level=level)


def _drift_stars(st: State, dt):
    mv = _moving(st)
    if mv is None:
        oracle.drift(st.pos, st.vel, dt)
        return
    p = np.ascontiguousarray(st.pos[mv])
    oracle.drift(p, np.ascontiguousarray(st.vel[mv]), dt)
    st.pos[mv] = p


def kdk_step(st: State, dt: float):
    _kick_stars(st, dt)
    if st.bh_mass.size:
        oracle.kick(st.bh_vel, st.bh_acc, dt)
    _drift_stars(st, dt)
    if st.bh_mass.size:
        oracle.drift(st.bh_pos, st.bh_vel, dt)
    forces(st)
    _kick_stars(st, dt)
    if st.bh_mass.size:
        oracle.kick(st.bh_vel, st.bh_acc, dt)


def dkd_step(st: State, dt: float):
    """Drift-kick-drift (Sec. 2, step 6): x += v dt/2, forces, v += a dt,
    x += v dt/2 (stars and SMBHs)."""
    _drift_stars(st, 0.5 * dt)
    if st.bh_mass.size:
        oracle.drift(st.bh_pos, st.bh_vel, 0.5 * dt)
    forces(st)
    _kick_stars(st, 2.0 * dt)                      # kick() applies half its dt
    if st.bh_mass.size:
        oracle.kick(st.bh_vel, st.bh_acc, 2.0 * dt)
    _drift_stars(st, 0.5 * dt)
    if st.bh_mass.size:
        oracle.drift(st.bh_pos, st.bh_vel, 0.5 * dt)


def _active(st: State, level, nlev, k):
    act = oracle.active_at(level, nlev, k)
    if st.frozen is not None:
        act = act[~np.asarray(st.frozen, bool)[act]]
    return act


def block_substep(st: State, level: np.ndarray, tau4eps2: np.ndarray, k: int,
                  dt_max: float, nlev: int, tau2eps2v=None, rebuild_every=0):
    """One substep at counter k; returns k + 1 and the new active set.  With
    tau2eps2v the levels also take the velocity criterion; with a rebuild
    period the tree is refitted between rebuilds."""
    dt_min = dt_max * 2.0 ** -(nlev - 1)
    act = _active(st, level, nlev, k)
    if k > 0:
        oracle.kick(st.vel, st.acc, dt_max, idx=act, level=level)
        if st.bh_mass.size:
            oracle.kick(st.bh_vel, st.bh_acc, dt_min)
    if tau2eps2v is None:
        oracle.levels(st.acc, tau4eps2, level, dt_max, nlev, k, idx=act)
    else:
        oracle.levels(st.acc, tau4eps2, level, dt_max, nlev, k, idx=act, vel=st.vel,
                      tau2eps2v=tau2eps2v)
    oracle.kick(st.vel, st.acc, dt_max, idx=act, level=level)
    if st.bh_mass.size:
        oracle.kick(st.bh_vel, st.bh_acc, dt_min)
    _drift_stars(st, dt_min)
    if st.bh_mass.size:
        oracle.drift(st.bh_pos, st.bh_vel, dt_min)
    k += 1
    act = _active(st, level, nlev, k)
    forces(st, act, k, rebuild_every)
    return k, act
